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


def golden_inputs(name):
    """Inputs of a hand-worked fixture in tests/golden (layout from synth)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        g = json.load(fh)
    sysm = synth.System(np.array(g["species"]), np.array(g["positions"]), g["r_cut"], 0,
                        basis_table=np.array(g["basis_table"]), aux_table=np.array(g["aux_table"]))
    lay = synth.make_layout(sysm)
    inp = synth.Inputs(sysm, lay, np.array(g["C"]), np.array(g["V"]), np.array(g["D"]))
    return inp, g


def test_hand_worked_two_atom_case():
    inp, g = golden_inputs("two_atom_hand.json")
    assert len(inp.C) == len(g["C"]) and len(inp.V) == len(g["V"])
    Kx = np.array(g["K"]).reshape(2, 2)
    K4, e_k, e_direct = O.k_4index(inp)
    assert np.abs(K4 - Kx).max() < 1e-12
    assert np.abs(O.k_eigen(inp) - Kx).max() < 1e-12
    assert np.abs(O.k_full_rows(inp) - Kx).max() < 1e-12
    assert abs(e_k - g["E_x"]) < 1e-12 and abs(e_direct - g["E_x"]) < 1e-12
    assert abs(O.exchange_energy(Kx, inp.D.reshape(2, 2)) - g["E_x"]) < 1e-12


def test_periodic_rows_of_atom_subsets():
    """The periodic row route on a few atoms (what the GPU tests sample on large
    boxes) gives the same rows as the whole cell, in any atom order, and with
    the image table built by an earlier call."""
    inp = synth.make_inputs(pins._tiny_periodic(23))
    pb = O.PBlocks(inp)
    X = O.x_periodic(inp)
    for atoms in ([3], [4, 1], [0, 2, 3]):
        rows = np.concatenate([np.arange(pb.bo[a], pb.bo[a + 1]) for a in atoms])
        Xr = O.x_atom_rows_periodic(inp, atoms, pb)
        assert pins.rel(Xr, X[rows]) < 1e-13
