"""libexx on the CPU: loads, exports every declared symbol, host-only plans,
argument errors (no compute call needs a GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import exx_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "exx.h")).read()
    return sorted(set(re.findall(r"^(?:int|int64_t|const char\*)\s+(\w+)\(", src, re.M)))


def test_library_exports_all_declared_symbols():
    import paper_2403_10343_amd as m
    L = m.lib()
    names = _declared()
    assert "build_K" in names and "exchange_energy" in names and "exchange_backward" in names
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("cfg", [1, 2])
def test_host_plan_layout_matches_oracle(cfg):
    from paper_2403_10343_amd import Plan
    sysm = synth.config(cfg)
    p = Plan.for_system(sysm, host_only=True)
    pa, pb, co, vo = p.pairs()
    oa, ob = O.screened_pairs(sysm.pos, sysm.r_cut, sysm.sys_off)
    assert np.array_equal(pa, oa) and np.array_equal(pb, ob)
    lay = synth.make_layout(sysm)
    assert np.array_equal(co, lay.c_off) and np.array_equal(vo, lay.v_off)
    ptr, nb = p.neighbors()
    assert ptr[-1] == 2 * len(pa) - sysm.n_atoms


def test_batch_pairs_never_cross_systems():
    from paper_2403_10343_amd import Plan
    b = synth.cluster_batch(4, n_min=2, n_max=6)
    p = Plan.for_system(b, host_only=True)
    pa, pb, _, _ = p.pairs()
    sys_of = np.searchsorted(b.sys_off, np.arange(b.n_atoms), side="right") - 1
    assert np.array_equal(sys_of[pa], sys_of[pb])


def test_errors_are_codes_not_aborts():
    from paper_2403_10343_amd import ExxError, Plan
    sysm = synth.config(1)
    with pytest.raises(ExxError) as e:
        Plan(sysm.species, sysm.pos, synth.N_BASIS, synth.N_AUX, -1.0, host_only=True)
    assert e.value.code == -1
    with pytest.raises(ExxError) as e:
        Plan(sysm.species, sysm.pos, [20, 5], synth.N_AUX, 6.0, host_only=True)
    assert e.value.code == -5
    with pytest.raises(ExxError):
        Plan(sysm.species, sysm.pos, synth.N_BASIS, synth.N_AUX, 6.0, sys_atom_off=[0, 30], host_only=True)
    p = Plan.for_system(sysm, host_only=True)
    import paper_2403_10343_amd._lib as L
    rc = L.lib().build_K(p._h, None, None, None, 0, None, None, None)
    assert rc == L.EXX_ESTATE
    rc = L.lib().build_K(None, None, None, None, 0, None, None, None)
    assert rc == L.EXX_EINVAL
    assert L.lib().exx_last_error()
