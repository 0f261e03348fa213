"""The CPU oracle against its pins (closed forms, brute force, invariants,
the paper's regrouped formula, finite differences)."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests import pins


@pytest.mark.parametrize("name", sorted(pins.ALL_PINS))
def test_pin(name):
    ok, detail = pins.ALL_PINS[name]()
    assert ok, f"{name}: {detail}"


def test_layout_matches_oracle_screening():
    for sysm in (synth.config(1), synth.cluster_batch(4, n_max=20)):
        lay = synth.make_layout(sysm)
        pa, pb = O.screened_pairs(sysm.pos, sysm.r_cut, sysm.sys_off)
        assert np.array_equal(pa, lay.pair_a) and np.array_equal(pb, lay.pair_b)


def test_generated_inputs_symmetric():
    inp = synth.make_inputs(synth.config(1))
    blk = O.Blocks(inp)
    Vd = blk.dense_V()
    C3 = blk.dense_C()
    assert np.array_equal(blk.D, blk.D.T)
    assert np.array_equal(Vd, Vd.T)
    assert np.array_equal(C3, C3.transpose(0, 2, 1))


def test_rows_match_eigen_on_config1_sample():
    inp = synth.make_inputs(synth.config(1))
    K = O.k_eigen(inp)
    rows = np.arange(0, 192, 23)
    assert pins.rel(O.k_rows(inp, rows), K[rows]) < 1e-12


def test_batch_systems_independent():
    """K of a batch member equals K of the same cluster built alone."""
    b = synth.cluster_batch(3, n_min=2, n_max=4)
    inp = synth.make_inputs(b)
    for s in range(b.n_systems):
        alone = synth.water_cluster((b.sys_off[s + 1] - b.sys_off[s]) // 3, seed=s)
        K1 = O.k_eigen(inp, s)
        K2 = O.k_eigen(synth.make_inputs(alone))
        assert pins.rel(K1, K2) < 1e-13
