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
    # the spin and two-Coulomb-matrix entry points: same codes, checked before any device work
    assert L.lib().build_K_spin(p._h, None, None, None, 0, None, None, None) == L.EXX_ESTATE
    assert L.lib().build_K_spin(None, None, None, None, 0, None, None, None) == L.EXX_EINVAL
    assert L.lib().build_K_two_kernels(p._h, None, None, None, None, 0, None, None, None) == L.EXX_ESTATE
    assert L.lib().build_K_two_kernels(None, None, None, None, None, 0, None, None, None) == L.EXX_EINVAL
    assert b"build_K_two_kernels" in L.lib().exx_last_error()


def test_mixed_split_flop_accounting():
    """Host-only plan: the FP32 share of the V-stage and T2 flops is all of
    them at split 0, none beyond the cutoff, and grows as the split shrinks."""
    import paper_2403_10343_amd as exx
    sysm = synth.ice_box(2, 2, 1, seed=0)
    p = exx.Plan.for_system(sysm, host_only=True)
    full = [p.flops(i) for i in range(5)]
    prev = -1
    for r in (7.0, 5.0, 4.0, 3.0, 1.0, 0.0):
        p.set_mixed_split(r)
        f32 = [p.flops(20 + i) for i in range(5)]
        assert f32[0] == f32[1] == f32[4] == 0
        assert 0 <= f32[2] <= full[2] and 0 <= f32[3] <= full[3]
        assert f32[2] + f32[3] >= prev
        prev = f32[2] + f32[3]
        alg, issued = p.stage_flops(mixed=True)
        assert sum(alg) == sum(full)
    assert f32[2] == full[2] and f32[3] == full[3]
    p.set_mixed_split(7.0)
    assert p.flops(22) == 0 and p.flops(23) == 0
    with pytest.raises(exx.ExxError):
        p.set_mixed_split(-1.0)


def test_tuning_choices_validated_on_host_plan():
    import paper_2403_10343_amd as exx
    p = exx.Plan.for_system(synth.water_cluster(2, seed=0), host_only=True)
    assert {k: v[0] for k, v in p.tuning().items()} == {"E k-chunk": 16, "T2 columns x waves": "8x4",
                                                         "Y k-chunk": 16}
    p.set_tuning([1, 2, 1])
    assert {k: v[0] for k, v in p.tuning().items()} == {"E k-chunk": 32, "T2 columns x waves": "8x8",
                                                         "Y k-chunk": 32}
    with pytest.raises(exx.ExxError):
        p.set_tuning([0, 3, 0])
    with pytest.raises(exx.ExxError):
        p.set_tuning([2, 0, 0])


def test_periodic_host_plan_layout_matches_generator():
    """Periodic host plans: canonical pairs, their lattice images and block
    offsets equal the generator's and the oracle's screening; a cutoff not below
    half the cell width is EXX_EINVAL; a budget that would chunk a periodic plan
    is EXX_EUNSUPPORTED."""
    from paper_2403_10343_amd import ExxError, Plan
    lat = np.array([[3.0, 0.0, 0.0], [0.4, 3.2, 0.0], [0.2, -0.3, 3.4]])
    pos = np.array([[0.2, 0.3, 0.1], [2.6, 0.5, 0.4], [1.3, 2.9, 3.0], [1.5, 1.6, 1.7], [0.5, 2.8, 3.2]])
    tiny = synth.System(np.array([0, 1, 1, 0, 1]), pos, 1.45, 3, lattice=lat)
    for sysm in (tiny, synth.ice_box_periodic(2, 2, 2, seed=0, r_cut=6.0)):
        p = Plan.for_system(sysm, host_only=True)
        lay = synth.make_layout(sysm)
        pa, pb, co, vo = p.pairs()
        assert np.array_equal(pa, lay.pair_a) and np.array_equal(pb, lay.pair_b)
        assert np.array_equal(p.pair_images(), lay.pair_img)
        assert np.array_equal(co, lay.c_off) and np.array_equal(vo, lay.v_off)
        mine = [(int(a), int(b), tuple(int(x) for x in n)) for a, b, n in zip(pa, pb, p.pair_images())]
        assert mine == O.periodic_pairs(sysm.pos, sysm.lattice, sysm.r_cut)
    assert (np.abs(Plan.for_system(tiny, host_only=True).pair_images()).sum(1) > 1).any()
    with pytest.raises(ExxError) as e:
        Plan(tiny.species, tiny.pos, synth.N_BASIS, synth.N_AUX, 1.6, host_only=True, lattice=lat)
    assert e.value.code == -1
    # periodic plans chunk like clusters; a budget below one group's E atoms is EXX_ENOMEM
    big = synth.ice_box_periodic(2, 2, 2, seed=0, r_cut=6.0)
    stored = Plan.for_system(big, host_only=True).info["intermediate_bytes_stored"]
    p = Plan.for_system(big, host_only=True, ws_budget_bytes=stored // 2)
    assert p.info["n_chunks"] >= 2 and p.info["intermediate_bytes"] <= stored // 2
    with pytest.raises(ExxError) as e:
        Plan.for_system(big, host_only=True, ws_budget_bytes=1 << 20)
    assert e.value.code == -2


def test_workspace_budget_chunks_on_host_plan():
    """A budget below the stored E, H' and Y splits the plan into chunks that
    each fit; no budget (or a large one) keeps one chunk; a budget below one
    V-stage group's needs is EXX_ENOMEM."""
    from paper_2403_10343_amd import ExxError, Plan
    sysm = synth.ice_box(2, 2, 2, seed=0)
    full = Plan.for_system(sysm, host_only=True)
    stored = full.info["intermediate_bytes_stored"]
    assert full.info["n_chunks"] == 1 and full.info["intermediate_bytes"] == stored
    assert Plan.for_system(sysm, host_only=True, ws_budget_bytes=2 * stored).info["n_chunks"] == 1
    prev = 1
    for frac in (2, 3, 5):
        p = Plan.for_system(sysm, host_only=True, ws_budget_bytes=stored // frac)
        assert p.info["n_chunks"] >= prev and p.info["n_chunks"] >= 2
        assert p.info["intermediate_bytes"] <= stored // frac
        assert p.info["intermediate_bytes_stored"] == stored
        prev = p.info["n_chunks"]
    with pytest.raises(ExxError) as e:
        Plan.for_system(sysm, host_only=True, ws_budget_bytes=4096)
    assert e.value.code == -2


def test_binding_rejects_arrays_before_the_library():
    """Arrays of the wrong type, device, layout or size raise EXX_EINVAL in the
    binding (they never reach a kernel)."""
    import torch
    from paper_2403_10343_amd import ExxError, Plan
    sysm = synth.water_cluster(2, seed=0)
    inp = synth.make_inputs(sysm)
    p = Plan.for_system(sysm, host_only=True)
    C, V, D = (torch.from_numpy(a) for a in (inp.C, inp.V, inp.D))
    K = torch.empty(p.info["d_size"], dtype=torch.float64)
    for args in ((C, V, D, K), (C.float(), V, D, K), (C, V[:-1], D, K), (C.numpy(), V, D, K)):
        with pytest.raises(ExxError) as e:
            p.build_K(*args)
        assert e.value.code == -1
    with pytest.raises(ExxError):
        p.exchange_backward(C, V, D, 1.0, dC=torch.empty_like(C))


def test_new_entry_points_reject_before_the_library():
    """The spin backward, block norms, strain derivative and Bloch-sum bindings
    reject host (CPU) arrays with EXX_EINVAL; on a host-only plan the library
    itself answers EXX_ESTATE for the screening threshold, and EXX_EINVAL for
    bad k-points or a bad threshold, without touching a device."""
    import ctypes
    import torch
    from paper_2403_10343_amd import ExxError, Plan, lib
    sysm = synth.water_cluster(2, seed=0)
    inp = synth.make_inputs(sysm)
    p = Plan.for_system(sysm, host_only=True)
    C, V, D = (torch.from_numpy(a) for a in (inp.C, inp.V, inp.D))
    calls = (lambda: p.exchange_backward_spin(C, V, torch.cat([D, D]), 1.0, dC=torch.empty_like(C)),
             lambda: p.block_norms(C, V, D),
             lambda: p.strain_derivative(C, V, C, V),
             lambda: p.bloch_sum(D, [(0.1, 0.2, 0.3)]),
             lambda: p.density_from_k(torch.zeros(p.info["d_size"], dtype=torch.complex128), [(0, 0, 0)]))
    for f in calls:
        with pytest.raises(ExxError) as e:
            f()
        assert e.value.code == -1
    with pytest.raises(ExxError) as e:
        p.bloch_sum(D, np.zeros((0, 3)))
    assert e.value.code == -1
    with pytest.raises(ExxError) as e:
        p.set_screening(1e-3)
    assert e.value.code == -4
    L = lib()
    assert L.exx_set_screening(None, 0.0) == -1
    k = np.array([np.nan, 0.0, 0.0])
    assert L.exx_bloch_sum(p._h, ctypes.c_void_p(1), 1, k.ctypes.data, ctypes.c_void_p(1), None) == -4
    assert L.exx_density_from_k(None, 1, k.ctypes.data, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1


def test_tile_cache_file(tmp_path):
    """The tile cache: entries stored and read back by key, other entries kept,
    a missing or corrupt file reads as empty; keys separate precisions, plan
    shapes and chunking."""
    from paper_2403_10343_amd import Plan
    from paper_2403_10343_amd._lib import load_tune_cache, store_tune_cache
    path = str(tmp_path / "tiles.json")
    assert load_tune_cache(path) == {}
    store_tune_cache(path, "a", {"choices": [0, 2, 1], "ms": [1.0] * 9})
    store_tune_cache(path, "b", {"choices": [1, 0, 0], "ms": [2.0] * 9})
    c = load_tune_cache(path)
    assert c["a"]["choices"] == [0, 2, 1] and c["b"]["choices"] == [1, 0, 0]
    (tmp_path / "bad.json").write_text("{not json")
    assert load_tune_cache(str(tmp_path / "bad.json")) == {}
    s1, s2 = synth.water_cluster(2, seed=0), synth.water_cluster(3, seed=0)
    p1, p2 = Plan.for_system(s1, host_only=True), Plan.for_system(s2, host_only=True)
    assert p1.tune_key("gfx950") == Plan.for_system(s1, host_only=True).tune_key("gfx950")
    assert p1.tune_key("gfx950") != p2.tune_key("gfx950")
    assert p1.tune_key("gfx950", 0) != p1.tune_key("gfx950", 1)
    big = synth.ice_box(2, 2, 2, seed=0)
    st = Plan.for_system(big, host_only=True).info["intermediate_bytes_stored"]
    assert (Plan.for_system(big, host_only=True).tune_key("gfx950")
            != Plan.for_system(big, host_only=True, ws_budget_bytes=st // 2).tune_key("gfx950"))


def test_backward_reuse_entry_points_on_host():
    """The workspace generation starts at 0 on a new plan; the reuse backward
    answers like exchange_backward (EXX_EINVAL for a NULL plan, EXX_ESTATE for a
    host-only plan) and reports that nothing was reused."""
    import ctypes
    from paper_2403_10343_amd import Plan, lib
    sysm = synth.water_cluster(2, seed=0)
    p = Plan.for_system(sysm, host_only=True)
    assert p.build_id() == 0
    L = lib()
    x = ctypes.c_uint64(7)
    assert L.exx_plan_build_id(None, ctypes.byref(x)) == -1
    assert L.exx_plan_build_id(p._h, None) == -1
    one = ctypes.c_void_p(1)
    r = ctypes.c_int(5)
    assert L.exchange_backward_reuse(None, 1, one, one, one, None, one, 0, one, None, None, None, 1.5, 8.0,
                                     ctypes.byref(r), None) == -1
    assert r.value == 0
    r.value = 5
    assert L.exchange_backward_reuse(p._h, 0, one, one, one, None, one, 0, one, None, None, None, 1.5, 8.0,
                                     ctypes.byref(r), None) == -4
    assert r.value == 0


def test_spin_backward_reuse_entry_point_on_host():
    import ctypes
    from paper_2403_10343_amd import Plan, lib
    p = Plan.for_system(synth.water_cluster(2, seed=0), host_only=True)
    one = ctypes.c_void_p(1)
    r = ctypes.c_int(5)
    L = lib()
    assert L.exchange_backward_spin_reuse(None, 1, one, one, one, None, one, 0, one, None, None, None, 1.5, 8.0,
                                          ctypes.byref(r), None) == -1
    assert r.value == 0
    r.value = 5
    assert L.exchange_backward_spin_reuse(p._h, 0, one, one, one, None, one, 0, one, None, None, None, 1.5, 8.0,
                                          ctypes.byref(r), None) == -4
    assert r.value == 0
