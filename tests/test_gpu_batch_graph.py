"""Batched clusters and HIP-graph replay of build_K."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import device_inputs, relmax, run_build, system_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def test_graph_replays_match_eager(exx):
    sysm = synth.water_cluster(6, 4)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K_eager, E_eager = run_build(plan, inp, torch)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    Ex = torch.empty(1, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.graph_build(C, V, D, K, Ex, stream=s.cuda_stream)
    for rep in range(4):
        K.fill_(float("nan"))
        Ex.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.graph_launch(stream=s.cuda_stream)
        torch.cuda.synchronize()
        assert np.array_equal(K.cpu().numpy(), K_eager), rep
        assert Ex.item() == E_eager[0]
        # eager work between replays
        run_build(plan, inp, torch)


def test_graph_requires_created_stream(exx):
    sysm = synth.water_cluster(1, 4)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    with pytest.raises(exx.ExxError):
        plan.graph_build(C, V, D, K, None, stream=0)
    with pytest.raises(exx.ExxError):
        plan.graph_launch(stream=torch.cuda.current_stream().cuda_stream)


def test_batch_members_equal_standalone_builds(exx):
    """Every cluster of an uneven batch, built in one batched graph, equals
    bit for bit the standalone build of the same inputs, and the oracle."""
    b = synth.cluster_batch(8, n_min=2, n_max=24)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    Ex = torch.empty(b.n_systems, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.graph_build(C, V, D, K, Ex, stream=s.cuda_stream)
    plan.graph_launch(stream=s.cuda_stream)
    torch.cuda.synchronize()
    Kb, Eb = K.cpu().numpy(), Ex.cpu().numpy()
    lay = inp.layout
    for c in range(b.n_systems):
        lo, hi = int(b.sys_off[c]), int(b.sys_off[c + 1])
        alone = synth.System(b.species[lo:hi], b.pos[lo:hi], b.r_cut, seed=c)
        la = synth.make_layout(alone)
        p0 = int(np.searchsorted(lay.pair_a, lo))
        p1 = int(np.searchsorted(lay.pair_a, hi))
        ia = synth.Inputs(alone, la, inp.C[lay.c_off[p0]:lay.c_off[p1]].copy(),
                          inp.V[lay.v_off[p0]:lay.v_off[p1]].copy(),
                          system_block(inp.D, lay, c).ravel().copy())
        Ka, Ea = run_build(exx.Plan.for_system(alone), ia, torch)
        assert np.array_equal(system_block(Kb, lay, c), system_block(Ka, la, 0)), c
        assert Eb[c] == Ea[0]
        if c < 3:
            assert relmax(system_block(Kb, lay, c), O.k_eigen(inp, c)) < 1e-10


def test_full_batch_of_64_clusters_sampled(exx):
    """The 64-cluster batch (8..128 molecules each) at full size: energies are
    finite, K blocks exactly symmetric, two small members against the oracle."""
    b = synth.cluster_batch()
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    K, Ex = run_build(plan, inp, torch)
    sizes = np.diff(b.sys_off)
    for c in np.argsort(sizes)[:2]:
        Kc = system_block(K, inp.layout, int(c))
        assert relmax(Kc, O.k_eigen(inp, int(c))) < 1e-10
    for c in range(b.n_systems):
        Kc = system_block(K, inp.layout, c)
        assert np.array_equal(Kc, Kc.T)
    assert np.all(np.isfinite(Ex))


def test_every_tile_variant_and_the_autotuner(exx):
    """All 12 combinations of the tuned tile shapes give K equal to the oracle
    (and to each other up to rounding); the autotuner picks one of them and
    leaves a correct K behind."""
    import itertools
    b = synth.cluster_batch(4, n_min=3, n_max=16)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    ref = [O.k_eigen(inp, s) for s in range(b.n_systems)]
    base = None
    for ch in itertools.product((0, 1), (0, 1, 2), (0, 1)):
        plan.set_tuning(ch)
        print("tile choices", ch, flush=True)
        K, _ = run_build(plan, inp, torch)
        for s in range(b.n_systems):
            assert relmax(system_block(K, inp.layout, s), ref[s]) < 1e-10
        if base is None:
            base = K
        assert relmax(K, base) < 1e-12
    C, V, D = device_inputs(inp, torch)
    Kt = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    plan.autotune(C, V, D, Kt)
    torch.cuda.synchronize()
    tun = plan.tuning()
    assert set(tun) == {"E k-chunk", "T2 columns x waves", "Y k-chunk"}
    for name, (val, ms) in tun.items():
        assert len(ms) == (3 if name.startswith("T2") else 2)
        assert all(t > 0 for t in ms.values()) and val == min(ms, key=ms.get)
    assert relmax(Kt.cpu().numpy(), base) < 1e-12
    K2, _ = run_build(plan, inp, torch)
    assert np.array_equal(K2, Kt.cpu().numpy())


def test_autotuner_tile_cache(exx, tmp_path, monkeypatch):
    """A tile cache file (EXX_TUNE_CACHE): the first autotune times the variants and
    stores the choice; a second plan of the same shape takes it without timing and
    builds the same K bit for bit."""
    from paper_2403_10343_amd._lib import load_tune_cache
    path = str(tmp_path / "tiles.json")
    monkeypatch.setenv("EXX_TUNE_CACHE", path)
    sysm = synth.ice_box(2, 2, 1, seed=3)
    inp = synth.make_inputs(sysm)
    C, V, D = device_inputs(inp, torch)
    p1 = exx.Plan.for_system(sysm)
    K1 = torch.empty_like(D)
    p1.autotune(C, V, D, K1)
    t1 = p1.tuning()
    assert all(len(ms) > 0 for _, ms in t1.values())
    assert len(load_tune_cache(path)) == 1
    p2 = exx.Plan.for_system(sysm)
    K2 = torch.empty_like(D)
    p2.autotune(C, V, D, K2)
    t2 = p2.tuning()
    assert {k: v[0] for k, v in t2.items()} == {k: v[0] for k, v in t1.items()}
    assert all(len(ms) == 0 for _, ms in t2.values())
    K3 = torch.empty_like(D)
    p1.build_K(C, V, D, K3)
    torch.cuda.synchronize()
    assert torch.equal(K2, K3)
