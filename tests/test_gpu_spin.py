"""Collinear spin (build_K_spin) against the CPU oracle, and against the
one-density build on each spin's density matrix."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import device_inputs, relmax, system_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_K = 1e-10
TOL_E = 1e-10


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def spin_build(plan, inp, Ds):
    dev = "cuda:0"
    C, V, _ = device_inputs(inp, torch)
    D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to(dev)
    n = plan.info["d_size"]
    K2 = torch.empty(2 * n, dtype=torch.float64, device=dev)
    Ex = torch.empty(plan.n_systems, dtype=torch.float64, device=dev)
    plan.build_K_spin(C, V, D2, K2, Ex)
    torch.cuda.synchronize()
    return K2.cpu().numpy().reshape(2, n), Ex.cpu().numpy()


def one_density_build(plan, inp, D):
    dev = "cuda:0"
    C, V, _ = device_inputs(inp, torch)
    Dd = torch.from_numpy(np.ascontiguousarray(D)).to(dev)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
    plan.build_K(C, V, Dd, K)
    torch.cuda.synchronize()
    return K.cpu().numpy()


@pytest.mark.parametrize("n_mol,seed", [(1, 3), (2, 4), (8, 5)])
def test_spin_clusters_match_oracle(exx, n_mol, seed):
    sysm = synth.water_cluster(n_mol, seed)
    print("spin cluster", n_mol, flush=True)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(sysm)
    K2, Ex = spin_build(plan, inp, Ds)
    Ko = O.k_spin(inp, Ds)
    for s in range(2):
        Kg = system_block(K2[s], inp.layout, 0)
        assert relmax(Kg, Ko[s]) < TOL_K
        assert np.array_equal(Kg, Kg.T)
    n = Ko[0].shape[0]
    Eo = O.spin_exchange_energy(Ko, [x.reshape(n, n) for x in Ds])
    assert abs(Ex[0] - Eo) < TOL_E * abs(Eo)


def test_spin_config1_4index(exx):
    inp = synth.make_inputs(synth.config(1))
    Ds = synth.spin_densities(inp, polarization=0.7)
    K2, Ex = spin_build(exx.Plan.for_system(inp.system), inp, Ds)
    Ko = O.k_spin(inp, Ds, route="4index")
    for s in range(2):
        assert relmax(system_block(K2[s], inp.layout, 0), Ko[s]) < TOL_K
    n = Ko[0].shape[0]
    Eo = O.spin_exchange_energy(Ko, [x.reshape(n, n) for x in Ds])
    assert abs(Ex[0] - Eo) < TOL_E * abs(Eo)


def test_spin_uneven_batch(exx):
    """A plan over several clusters of different sizes: every cluster's K^s
    and E_x against the oracle."""
    sysm = synth.cluster_batch(4, batch_seed=7, n_min=2, n_max=12)
    print("spin batch", sysm.n_systems, flush=True)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    K2, Ex = spin_build(exx.Plan.for_system(sysm), inp, Ds)
    for c in range(sysm.n_systems):
        Ko = O.k_spin(inp, Ds, s=c)
        for s in range(2):
            assert relmax(system_block(K2[s], inp.layout, c), Ko[s]) < TOL_K
        Db = [system_block(x, inp.layout, c) for x in Ds]
        Eo = O.spin_exchange_energy(Ko, Db)
        assert abs(Ex[c] - Eo) < TOL_E * abs(Eo)


def test_spin_equals_one_density_builds_768(exx):
    """On the 768-atom box: K^s of the two-spin build equals build_K on D^s
    bit for bit (the shared V-stage pass keeps every sum in the same order),
    and with D^0 = D^1 = D/2 the spin E_x is the one-density E_x of D."""
    sysm = synth.config(2)
    print("spin 768 atoms", flush=True)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    Ds = synth.spin_densities(inp)
    K2, Ex = spin_build(plan, inp, Ds)
    for s in range(2):
        assert np.array_equal(K2[s], one_density_build(plan, inp, Ds[s]))
    half = np.stack([0.5 * inp.D, 0.5 * inp.D])
    Kh, Eh = spin_build(plan, inp, half)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    E1 = torch.empty(1, dtype=torch.float64, device="cuda:0")
    plan.build_K(C, V, D, K, E1)
    torch.cuda.synchronize()
    assert np.array_equal(Kh[0], 0.5 * K.cpu().numpy())
    assert abs(Eh[0] - E1.item()) <= 1e-13 * abs(E1.item())


def test_spin_mixed_and_fp32(exx):
    """Mixed and all-FP32 spin builds on the 768-atom box: each K^s equals the
    one-density build_K of D^s in the same precision bit for bit, and the mixed
    K^s and E_x are within the mixed bar of the FP64 spin build."""
    sysm = synth.config(2)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(sysm)
    dev = "cuda:0"
    C, V, _ = device_inputs(inp, torch)
    D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to(dev)
    n = plan.info["d_size"]
    K64, E64 = spin_build(plan, inp, Ds)
    for prec in (exx.PREC_MIXED, exx.PREC_FP32):
        K2 = torch.empty(2 * n, dtype=torch.float64, device=dev)
        Ex = torch.empty(1, dtype=torch.float64, device=dev)
        plan.build_K_spin(C, V, D2, K2, Ex, precision=prec)
        torch.cuda.synchronize()
        Km = K2.cpu().numpy().reshape(2, n)
        for s in range(2):
            K1 = torch.empty(n, dtype=torch.float64, device=dev)
            plan.build_K(C, V, torch.from_numpy(np.ascontiguousarray(Ds[s])).to(dev), K1, precision=prec)
            torch.cuda.synchronize()
            assert np.array_equal(Km[s], K1.cpu().numpy())
        if prec == exx.PREC_MIXED:
            dK, dE = np.abs(Km - K64).max(), abs(Ex.item() - E64[0]) / sysm.n_atoms
            print(f"mixed spin: max|dK| {dK:.2e}, |dE|/atom {dE:.2e}", flush=True)
            assert dK <= 1e-5 and dE <= 1e-6
    with pytest.raises(exx.ExxError) as e:
        plan.build_K_spin(C, V, D2, torch.empty(2 * n, dtype=torch.float64, device=dev), precision=exx.PREC_BF16X3)
    assert e.value.code == -5


def _spin_grads(plan, inp, Ds, gE=1.0, K=None):
    dev = "cuda:0"
    C, V, _ = device_inputs(inp, torch)
    D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to(dev)
    dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D2)
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device=dev)
    plan.exchange_backward_spin(C, V, D2, gE, dC=dC, dV=dV, dD=dD, forces=F, K=K)
    torch.cuda.synchronize()
    return {"dC": dC.cpu().numpy(), "dV": dV.cpu().numpy(), "dD": dD.cpu().numpy().reshape(2, -1),
            "F": F.cpu().numpy().reshape(-1, 3)}


@pytest.mark.parametrize("n_mol,seed", [(2, 4), (8, 5)])
def test_spin_backward_matches_oracle(exx, n_mol, seed):
    """dE/dC, dE/dV, dE/dD^s and forces of the spin energy against the oracle's
    spin gradients (pinned by central differences of the spin energy)."""
    sysm = synth.water_cluster(n_mol, seed)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(sysm)
    g = _spin_grads(plan, inp, Ds)
    go = O.spin_gradients(inp, Ds)
    print(f"spin backward, {n_mol} waters: dC {relmax(g['dC'], go['dC']):.1e}, dV {relmax(g['dV'], go['dV']):.1e}",
          flush=True)
    assert relmax(g["dC"], go["dC"]) < 1e-10 and relmax(g["dV"], go["dV"]) < 1e-10
    for s in range(2):
        assert relmax(system_block(g["dD"][s], inp.layout, 0), go["dD"][s]) < 1e-10
    assert relmax(g["F"], O.forces(inp, go)) < 1e-10


def test_spin_backward_identities(exx):
    """768-atom box, in a chunked plan too: K^s passed in gives dD^s = -K^s
    exactly; equal spins D/2, D/2 give the one-density gradients of D; the spin
    gradients are twice the one-density gradients of D^0 plus those of D^1
    (each spin's term is twice a one-density energy)."""
    sysm = synth.config(2)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(sysm)
    K2, _ = spin_build(plan, inp, Ds)
    g = _spin_grads(plan, inp, Ds)
    gk = _spin_grads(plan, inp, Ds, K=torch.from_numpy(K2.reshape(-1)).to("cuda:0"))
    assert np.array_equal(gk["dD"], -K2)
    assert relmax(gk["dD"], g["dD"]) < 1e-12
    assert relmax(gk["dC"], g["dC"]) < 1e-12 and np.array_equal(gk["dV"], g["dV"])

    def one(D, gE):
        C, V, Dd = device_inputs(O.with_density(inp, D), torch)
        dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(Dd)
        F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0")
        plan.exchange_backward(C, V, Dd, gE, dC=dC, dV=dV, dD=dD, forces=F)
        torch.cuda.synchronize()
        return {"dC": dC.cpu().numpy(), "dV": dV.cpu().numpy(), "dD": dD.cpu().numpy(),
                "F": F.cpu().numpy().reshape(-1, 3)}

    g0, g1 = one(Ds[0], 2.0), one(Ds[1], 2.0)
    for k in ("dC", "dV", "F"):
        assert relmax(g[k], g0[k] + g1[k]) < 1e-12, k
    assert np.array_equal(g["dD"][0], g0["dD"]) and np.array_equal(g["dD"][1], g1["dD"])
    half = np.stack([0.5 * inp.D, 0.5 * inp.D])
    gh, gd = _spin_grads(plan, inp, half), one(inp.D, 1.0)
    for k in ("dC", "dV", "F"):
        assert relmax(gh[k], gd[k]) < 1e-12, k
    part = exx.Plan.for_system(sysm, ws_budget_bytes=plan.info["intermediate_bytes_stored"] // 4)
    gp = _spin_grads(part, inp, Ds)
    for k in ("dC", "dV", "dD", "F"):
        assert relmax(gp[k], g[k]) < 1e-12, k


def test_spin_backward_periodic(exx):
    """Periodic cell: equal spins give the one-density gradients of D, and
    unequal spins twice the sum of the one-density gradients of each spin."""
    cell = synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)
    inp = synth.make_inputs(cell)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(cell)
    g = _spin_grads(plan, inp, Ds)

    def one(D, gE):
        C, V, Dd = device_inputs(O.with_density(inp, D), torch)
        dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(Dd)
        F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0")
        plan.exchange_backward(C, V, Dd, gE, dC=dC, dV=dV, dD=dD, forces=F)
        torch.cuda.synchronize()
        return {"dC": dC.cpu().numpy(), "dV": dV.cpu().numpy(), "dD": dD.cpu().numpy(),
                "F": F.cpu().numpy().reshape(-1, 3)}

    g0, g1 = one(Ds[0], 2.0), one(Ds[1], 2.0)
    for k in ("dC", "dV", "F"):
        assert relmax(g[k], g0[k] + g1[k]) < 1e-12, k
    half = np.stack([0.5 * inp.D, 0.5 * inp.D])
    gh, gd = _spin_grads(plan, inp, half), one(inp.D, 1.0)
    for k in ("dC", "dV", "F"):
        assert relmax(gh[k], gd[k]) < 1e-12, k
    with pytest.raises(exx.ExxError) as e:
        C, V, _ = device_inputs(inp, torch)
        D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to("cuda:0")
        plan.exchange_backward_spin(C, V, D2, 1.0, dC=torch.empty_like(C), precision=exx.PREC_MIXED)
    assert e.value.code == -5


def test_spin_autograd(exx):
    """torch.autograd through the spin energy: the gradients of a weighted sum
    of the per-system energies of a batch equal exchange_backward_spin's."""
    b = synth.cluster_batch(3, n_min=6, n_max=18)
    inp = synth.make_inputs(b)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(b)
    C, V, _ = device_inputs(inp, torch)
    D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to("cuda:0")
    C.requires_grad_(True)
    D2.requires_grad_(True)
    w = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda:0")
    E = exx.spin_exchange_energy(plan, C, V, D2)
    (w * E).sum().backward()
    dC, dD = torch.empty_like(C), torch.empty_like(D2)
    plan.exchange_backward_spin(C.detach(), V, D2.detach(), w, dC=dC, dD=dD)
    torch.cuda.synchronize()
    assert relmax(C.grad.cpu().numpy(), dC.cpu().numpy()) < 1e-12
    assert relmax(D2.grad.cpu().numpy(), dD.cpu().numpy()) < 1e-12


def test_spin_backward_reuses_forward_intermediates(exx):
    """After a binary64 build_K_spin, exchange_backward_spin_reuse takes E^s and
    H'^s from the workspace: dD and dV equal the recomputing spin backward's bit
    for bit, dC and the forces to rounding; after another build, or after a
    one-density build, it recomputes (bit for bit the plain spin backward)."""
    dev = "cuda:0"
    sysm = synth.water_cluster(8, 5)
    inp = synth.make_inputs(sysm)
    Ds = synth.spin_densities(inp)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    D2 = torch.from_numpy(np.ascontiguousarray(Ds.reshape(-1))).to(dev)
    n = plan.info["d_size"]
    K2 = torch.empty(2 * n, dtype=torch.float64, device=dev)

    def grads(build_id=None):
        dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D2)
        F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device=dev)
        used = plan.exchange_backward_spin(C, V, D2, 0.6, dC=dC, dV=dV, dD=dD, forces=F, K=K2, build_id=build_id)
        torch.cuda.synchronize()
        return used, {k: x.cpu().numpy() for k, x in (("dC", dC), ("dV", dV), ("dD", dD), ("F", F))}

    plan.build_K_spin(C, V, D2, K2)
    _, ref = grads()
    plan.build_K_spin(C, V, D2, K2)
    used, g = grads(plan.build_id())
    print("spin reuse after an FP64 spin build:", used, flush=True)
    assert used
    assert np.array_equal(g["dD"], ref["dD"]) and np.array_equal(g["dV"], ref["dV"])
    assert relmax(g["dC"], ref["dC"]) < 1e-12 and relmax(g["F"], ref["F"]) < 1e-12
    go = O.spin_gradients(inp, Ds)
    assert relmax(g["dC"], 0.6 * go["dC"]) < 1e-10 and relmax(g["dV"], 0.6 * go["dV"]) < 1e-10
    plan.build_K_spin(C, V, D2, K2)
    bid = plan.build_id()
    plan.build_K(C, V, D, torch.empty(n, dtype=torch.float64, device=dev))
    used, g2 = grads(bid)
    assert not used and all(np.array_equal(g2[k], ref[k]) for k in ref)
    used, _ = grads(plan.build_id())                  # a one-density build is not a spin build
    assert not used
