"""Maximum-norm estimates (binary64, per canonical pair) and the screening of
V blocks by them, through the C ABI, against the oracle: the norms bit for
bit, the screening flags bit for bit (both sides form the same binary64
products), and the screened K against the oracle's K of V with the flagged
blocks set to zero."""
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


def _eps_at(est, q):
    """A threshold between two consecutive estimates near quantile q (no ties)."""
    s = np.unique(est)
    k = min(max(int(q * len(s)), 1), len(s) - 1)
    return 0.5 * (s[k - 1] + s[k])


def _screened(exx, plan, inp, eps, precision=0):
    plan.set_screening(eps)
    K, Ex = run_build(plan, inp, torch, precision)
    flags = plan.screened_pairs().cpu().numpy().astype(bool)
    plan.set_screening(0.0)
    return K, Ex, flags


@pytest.mark.parametrize("which", ["cluster", "batch", "periodic"])
def test_block_norms_equal_oracle(exx, which):
    sysm = {"cluster": lambda: synth.config(1), "batch": lambda: synth.cluster_batch(4, n_min=6, n_max=30),
            "periodic": lambda: synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)}[which]()
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    got = plan.block_norms(C, V, D).cpu().numpy()
    assert np.array_equal(got, O.block_max_norms(inp))


def test_screened_cluster_matches_oracle(exx):
    """24-atom cluster: with eps at the 30 % point of the estimates the flags
    equal the oracle's and K, E_x equal the oracle's exchange of the screened V;
    eps = 0 afterwards, and eps below every estimate, give the unscreened build
    bit for bit."""
    sysm = synth.config(1)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K0, E0 = run_build(plan, inp, torch)
    est = O.screening_estimates(inp, O.block_max_norms(inp))
    eps = _eps_at(est, 0.3)
    K, Ex, flags = _screened(exx, plan, inp, eps)
    want = est < eps
    print(f"eps {eps:.4g}: {flags.sum()} of {len(flags)} pairs screened, rel change {relmax(K, K0):.2e}", flush=True)
    assert np.array_equal(flags, want) and 0 < flags.sum() < len(flags)
    scr = O.screened_coulomb(inp, want)
    n = int(inp.layout.sys_nbas[0])
    Ko = O.k_eigen(scr)
    assert relmax(K.reshape(n, n), Ko) < 1e-10
    Eo = O.exchange_energy(Ko, inp.D.reshape(n, n))
    assert abs(Ex[0] - Eo) < 1e-10 * abs(Eo)
    K1, E1 = run_build(plan, inp, torch)               # screening off again
    assert np.array_equal(K1, K0) and np.array_equal(E1, E0)
    K2, E2, f2 = _screened(exx, plan, inp, 0.5 * est.min())
    assert not f2.any() and np.array_equal(K2, K0) and np.array_equal(E2, E0)


def test_screened_batch_and_periodic_match_oracle(exx):
    b = synth.cluster_batch(4, n_min=6, n_max=30)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    est = O.screening_estimates(inp, O.block_max_norms(inp))
    eps = _eps_at(est, 0.25)
    K, Ex, flags = _screened(exx, plan, inp, eps)
    assert np.array_equal(flags, est < eps)
    scr = O.screened_coulomb(inp, flags)
    for s in range(b.n_systems):
        assert relmax(system_block(K, inp.layout, s), O.k_eigen(scr, s)) < 1e-10
    cell = synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)
    inp = synth.make_inputs(cell)
    plan = exx.Plan.for_system(cell)
    est = O.screening_estimates(inp, O.block_max_norms(inp))
    eps = _eps_at(est, 0.3)
    K, Ex, flags = _screened(exx, plan, inp, eps)
    assert np.array_equal(flags, est < eps) and flags.any()
    scr = O.screened_coulomb(inp, flags)
    n = int(inp.layout.sys_nbas[0])
    Xo = O.x_periodic(scr)
    assert relmax(K.reshape(n, n), Xo) < 1e-10
    Eo = O.periodic_energy(Xo, inp.D.reshape(n, n))
    assert abs(Ex[0] - Eo) < 1e-10 * abs(Eo)


def test_screened_768_box_rows_mixed_chunks_and_graph(exx):
    """768-atom box at the 20 % point: flags equal the oracle's, sampled rows
    equal the oracle's rows of the screened V; the screened mixed build stays
    within the mixed bar of the screened FP64 build; a chunked plan gives the
    same screened K; a graph captured with screening on replays the eager build."""
    sysm = synth.config(2)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    est = O.screening_estimates(inp, O.block_max_norms(inp))
    eps = _eps_at(est, 0.2)
    K0, E0 = run_build(plan, inp, torch)
    K, Ex, flags = _screened(exx, plan, inp, eps)
    assert np.array_equal(flags, est < eps)
    n = int(inp.layout.sys_nbas[0])
    print(f"768 box, eps {eps:.4g}: {flags.mean():.1%} of pairs screened, max|dK| {np.abs(K - K0).max():.2e}, "
          f"dE/atom {abs(Ex[0] - E0[0]) / sysm.n_atoms:.2e}", flush=True)
    scr = O.screened_coulomb(inp, flags)
    blk = O.Blocks(scr)
    Kg = K.reshape(n, n)
    for a in (301, 302):
        rows = np.arange(blk.bo[a], blk.bo[a + 1])
        Xr = O.k_atom_rows(scr, [a], blk=blk)
        assert np.abs(Kg[rows] - Xr).max() < 1e-10 * np.abs(Xr).max()
    Km, Em, fm = _screened(exx, plan, inp, eps, exx.PREC_MIXED)
    assert np.array_equal(fm, flags)
    assert np.abs(Km - K).max() <= 1e-5 and abs(Em[0] - Ex[0]) / sysm.n_atoms <= 1e-6
    part = exx.Plan.for_system(sysm, ws_budget_bytes=plan.info["intermediate_bytes_stored"] // 4)
    assert part.info["n_chunks"] >= 3
    Kc, Ec, fc = _screened(exx, part, inp, eps)
    assert np.array_equal(fc, flags) and relmax(Kc, K) < 1e-12
    C, V, D = device_inputs(inp, torch)
    Kd = torch.empty_like(D)
    Ed = torch.empty(1, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    plan.set_screening(eps)
    plan.graph_build(C, V, D, Kd, Ed, stream=s.cuda_stream)
    plan.set_screening(0.0)
    for _ in range(2):
        Kd.fill_(3.0)
        torch.cuda.synchronize()
        plan.graph_launch(stream=s.cuda_stream)
        torch.cuda.synchronize()
        assert np.array_equal(Kd.cpu().numpy(), K) and Ed.item() == Ex[0]


def test_screened_spin_and_two_kernels(exx):
    """Spin builds screen both spins with one flag per pair (the D norm over both
    spins), two-kernel builds each Coulomb matrix by its own estimates; each K
    equals the oracle's exchange of the screened V."""
    sysm = synth.water_cluster(8, 5)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    n = int(inp.layout.sys_nbas[0])
    dev = "cuda:0"
    C, V, D = device_inputs(inp, torch)
    Ds = synth.spin_densities(inp)
    both = O.with_density(inp, np.maximum(np.abs(Ds[0]), np.abs(Ds[1])))
    est = O.screening_estimates(inp, O.block_max_norms(both))
    eps = _eps_at(est, 0.3)
    plan.set_screening(eps)
    K2 = torch.empty(2 * n * n, dtype=torch.float64, device=dev)
    plan.build_K_spin(C, V, torch.from_numpy(Ds.reshape(-1)).to(dev), K2)
    flags = plan.screened_pairs().cpu().numpy().astype(bool)
    assert np.array_equal(flags, est < eps) and flags.any()
    Ko = O.k_spin(O.screened_coulomb(inp, flags), list(Ds))
    Kg = K2.cpu().numpy().reshape(2, n, n)
    for s in range(2):
        assert relmax(Kg[s], Ko[s]) < 1e-10
    V2 = synth.short_range_V(inp)
    Kt = torch.empty(2 * n * n, dtype=torch.float64, device=dev)
    plan.build_K_two_kernels(C, V, torch.from_numpy(V2).to(dev), D, Kt)
    f2 = plan.screened_pairs().cpu().numpy().astype(bool)
    plan.set_screening(0.0)
    Kt = Kt.cpu().numpy().reshape(2, n, n)
    for a, Vx in enumerate((inp.V, V2)):
        ia = O.with_coulomb(inp, Vx)
        fa = O.screening_estimates(ia, O.block_max_norms(ia)) < eps
        if a == 1:
            assert np.array_equal(f2, fa)
        assert relmax(Kt[a], O.k_eigen(O.screened_coulomb(ia, fa))) < 1e-10


def test_screening_errors(exx):
    sysm = synth.water_cluster(2, 3)
    plan = exx.Plan.for_system(sysm)
    with pytest.raises(exx.ExxError) as e:            # no screened build yet
        plan.screened_pairs()
    assert e.value.code == -4
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(exx.ExxError) as e:
            plan.set_screening(bad)
        assert e.value.code == -1
