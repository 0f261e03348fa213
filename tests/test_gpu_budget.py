"""Workspace-bounded plans (the C.D intermediates recomputed per chunk of aux
atoms instead of stored), the masked density matrix, per-system gradient
weights and the precision slots, through the C ABI."""
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


def grads(plan, inp, gE=1.0, K=None):
    C, V, D = device_inputs(inp, torch)
    dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D)
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0")
    plan.exchange_backward(C, V, D, gE, dC=dC, dV=dV, dD=dD, forces=F, K=K)
    torch.cuda.synchronize()
    return {k: x.cpu().numpy() for k, x in (("dC", dC), ("dV", dV), ("dD", dD), ("F", F))}


@pytest.mark.parametrize("which", ["ice192", "ice768"])
def test_chunked_plan_equals_stored(exx, which):
    """A budget a quarter of the stored intermediates forces several chunks; K,
    E_x and every gradient agree with the unbounded plan (dV bit for bit: the
    same blocks in the same order; K and E_x up to the order in which the
    chunks' parts of the final sum are added; dC up to the unbounded plan's
    reuse of its forward V stage, whose G term is taken twice and once
    subtracted)."""
    sysm = synth.ice_box(2, 2, 2, seed=3) if which == "ice192" else synth.config(2)
    inp = synth.make_inputs(sysm)
    full = exx.Plan.for_system(sysm)
    stored = full.info["intermediate_bytes_stored"]
    budget = stored // (3 if which == "ice192" else 4)
    part = exx.Plan.for_system(sysm, ws_budget_bytes=budget)
    nch = part.info["n_chunks"]
    print(f"{which}: stored {stored / 1e9:.3f} GB, budget {budget / 1e9:.3f} GB, {nch} chunks, "
          f"held {part.info['intermediate_bytes'] / 1e9:.3f} GB", flush=True)
    assert full.info["n_chunks"] == 1 and nch >= 3
    assert part.info["intermediate_bytes"] <= budget
    K1, E1 = run_build(full, inp, torch)
    K2, E2 = run_build(part, inp, torch)
    assert relmax(K2, K1) < 1e-12 and abs(E2[0] - E1[0]) < 1e-12 * abs(E1[0])
    assert np.array_equal(K2, K2.reshape(int(inp.layout.sys_nbas[0]), -1).T.ravel())
    for prec in (exx.PREC_MIXED, exx.PREC_FP32):
        Km1, Em1 = run_build(full, inp, torch, prec)
        Km2, Em2 = run_build(part, inp, torch, prec)
        assert relmax(Km2, Km1) < 1e-12 and abs(Em2[0] - Em1[0]) < 1e-12 * abs(Em1[0])
    g1, g2 = grads(full, inp), grads(part, inp)
    assert relmax(g2["dC"], g1["dC"]) < 1e-12 and np.array_equal(g1["dV"], g2["dV"])
    assert relmax(g2["dD"], g1["dD"]) < 1e-12
    assert relmax(g2["F"], g1["F"]) < 1e-12


def test_chunked_batch_and_forward_K(exx):
    b = synth.cluster_batch(5, n_min=6, n_max=30)
    inp = synth.make_inputs(b)
    full = exx.Plan.for_system(b)
    part = exx.Plan.for_system(b, ws_budget_bytes=full.info["intermediate_bytes_stored"] // 5)
    assert part.info["n_chunks"] >= 3
    K1, E1 = run_build(full, inp, torch)
    K2, E2 = run_build(part, inp, torch)
    assert relmax(K2, K1) < 1e-12 and relmax(E2, E1) < 1e-12
    C, V, D = device_inputs(inp, torch)
    K = torch.from_numpy(K2).to("cuda:0")
    g1 = grads(full, inp, 0.5)
    g2 = grads(part, inp, 0.5, K=K)
    assert np.array_equal(g2["dD"], -0.25 * K2)
    assert relmax(g2["dC"], g1["dC"]) < 1e-12 and np.array_equal(g1["dV"], g2["dV"])
    for s in range(b.n_systems):
        Ko = O.k_eigen(inp, s)
        assert relmax(system_block(K2, inp.layout, s), Ko) < 1e-10


def test_budget_errors(exx):
    sysm = synth.ice_box(2, 2, 1, seed=3)
    with pytest.raises(exx.ExxError) as e:
        exx.Plan.for_system(sysm, ws_budget_bytes=1000)
    assert e.value.code == -2


def test_chunked_spin_and_two_kernels(exx):
    """Collinear-spin and two-Coulomb-matrix builds on a chunked plan (FP64 and
    mixed) equal those of the unbounded plan, and so does the spin backward."""
    sysm = synth.ice_box(2, 2, 2, seed=3)
    inp = synth.make_inputs(sysm)
    full = exx.Plan.for_system(sysm)
    part = exx.Plan.for_system(sysm, ws_budget_bytes=full.info["intermediate_bytes_stored"] // 3)
    assert part.info["n_chunks"] >= 3
    C, V, D = device_inputs(inp, torch)
    Ds = torch.from_numpy(synth.spin_densities(inp).reshape(-1)).to("cuda:0")
    V2 = torch.from_numpy(synth.short_range_V(inp)).to("cuda:0")
    n = full.info["d_size"]
    for prec in (exx.PREC_FP64, exx.PREC_MIXED):
        out = []
        for plan in (full, part):
            Ks = torch.empty(2 * n, dtype=torch.float64, device="cuda:0")
            Es = torch.empty(1, dtype=torch.float64, device="cuda:0")
            plan.build_K_spin(C, V, Ds, Ks, Es, precision=prec)
            Kt = torch.empty(2 * n, dtype=torch.float64, device="cuda:0")
            Et = torch.empty(2, dtype=torch.float64, device="cuda:0")
            plan.build_K_two_kernels(C, V, V2, D, Kt, Et, precision=prec)
            torch.cuda.synchronize()
            out.append([x.cpu().numpy() for x in (Ks, Es, Kt, Et)])
        for a, b in zip(*out):
            assert relmax(b, a) < 1e-12
    g = []
    for plan in (full, part):
        dC, dV = torch.empty_like(C), torch.empty_like(V)
        plan.exchange_backward_spin(C, V, Ds, 1.0, dC=dC, dV=dV)
        torch.cuda.synchronize()
        g.append((dC.cpu().numpy(), dV.cpu().numpy()))
    assert relmax(g[1][0], g[0][0]) < 1e-12 and np.array_equal(g[1][1], g[0][1])


def test_density_beyond_cutoff_is_ignored(exx):
    """D entries of atom pairs beyond r_cut do not change K or E_x (the build
    contracts D restricted to the screened pair blocks)."""
    sysm = synth.ice_box(2, 2, 1, seed=5)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K1, E1 = run_build(plan, inp, torch)
    n = int(inp.layout.sys_nbas[0])
    blk = O.Blocks(inp)
    mask = np.zeros((blk.nat, blk.nat), bool)
    mask[blk.pa, blk.pb] = mask[blk.pb, blk.pa] = True
    atom = np.repeat(np.arange(blk.nat), blk.nb)
    off = ~mask[atom][:, atom]
    assert off.any()
    rng = np.random.default_rng(11)
    noise = rng.normal(size=(n, n))
    noise = noise + noise.T
    D2 = inp.D.reshape(n, n) + np.where(off, noise, 0.0)
    inp2 = synth.Inputs(sysm, inp.layout, inp.C, inp.V, D2.ravel())
    K2, E2 = run_build(plan, inp2, torch)
    assert np.array_equal(K1, K2) and np.array_equal(E1, E2)
    # the standalone energy entry point also sums over the pair blocks only
    Kd = torch.from_numpy(K1).to("cuda:0")
    Ex = torch.empty(1, dtype=torch.float64, device="cuda:0")
    plan.exchange_energy(Kd, torch.from_numpy(inp2.D).to("cuda:0"), Ex)
    assert Ex.item() == E1[0]
    # gradients ignore it too
    g1, g2 = grads(plan, inp), grads(plan, inp2)
    for k in ("dC", "dV", "dD", "F"):
        assert np.array_equal(g1[k], g2[k]), k


def test_exchange_energy_entry_point(exx):
    """exchange_energy (C ABI) on an oracle K: E_x = -1/4 sum K D per system."""
    b = synth.cluster_batch(3, n_min=3, n_max=9)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    Ks = np.zeros(inp.layout.d_size)
    Eo = []
    for s in range(b.n_systems):
        Ko = O.k_eigen(inp, s)
        o, n = int(inp.layout.sys_bas_off[s]), int(inp.layout.sys_nbas[s])
        Ks[o:o + n * n] = Ko.ravel()
        Eo.append(O.exchange_energy(Ko, O.Blocks(inp, s).D))
    Ex = torch.empty(b.n_systems, dtype=torch.float64, device="cuda:0")
    plan.exchange_energy(torch.from_numpy(Ks).to("cuda:0"), torch.from_numpy(inp.D).to("cuda:0"), Ex)
    assert relmax(Ex.cpu().numpy(), np.array(Eo)) < 1e-13


def test_per_system_upstream_gradients(exx):
    """exchange_backward with one dL/dE_x per system, and the autograd.Function
    on a weighted loss over a batch: each system's gradients are its own oracle
    gradients times its weight."""
    b = synth.cluster_batch(4, n_min=2, n_max=6)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    w = np.array([0.5, -2.0, 1.25, 3.0])
    C, V, D = (x.clone().requires_grad_(True) for x in device_inputs(inp, torch))
    E = exx.exchange_energy(plan, C, V, D)
    (E * torch.from_numpy(w).to("cuda:0")).sum().backward()
    dC, dV, dD = (x.grad.cpu().numpy() for x in (C, V, D))
    g = grads(plan, inp, torch.from_numpy(w).to("cuda:0"))
    assert relmax(dC, g["dC"]) < 1e-14 and relmax(dV, g["dV"]) < 1e-14
    lay = inp.layout
    for s in range(b.n_systems):
        go = O.gradients(inp, s)
        sel = np.zeros(lay.n_pairs, bool)
        sel[go["blk"].pidx] = True
        cm = np.concatenate([np.arange(lay.c_off[p], lay.c_off[p + 1]) for p in np.nonzero(sel)[0]])
        vm = np.concatenate([np.arange(lay.v_off[p], lay.v_off[p + 1]) for p in np.nonzero(sel)[0]])
        assert relmax(dC[cm], w[s] * go["dC"][cm]) < 1e-10
        assert relmax(dV[vm], w[s] * go["dV"][vm]) < 1e-10
        assert relmax(system_block(dD, lay, s), w[s] * go["dD"]) < 1e-10


def test_precision_slots(exx):
    """EXX_PREC_FP32 is the mixed build at split 0 (bit for bit), whatever split
    the plan holds; EXX_PREC_BF16X3 is reserved."""
    b = synth.cluster_batch(3, n_min=4, n_max=12)
    inp = synth.make_inputs(b)
    plan = exx.Plan.for_system(b)
    K32, E32 = run_build(plan, inp, torch, exx.PREC_FP32)
    plan.set_mixed_split(0.0)
    Km, Em = run_build(plan, inp, torch, exx.PREC_MIXED)
    assert np.array_equal(K32, Km) and np.array_equal(E32, Em)
    plan.set_mixed_split(5.0)
    K32b, _ = run_build(plan, inp, torch, exx.PREC_FP32)
    assert np.array_equal(K32, K32b)
    with pytest.raises(exx.ExxError) as e:
        run_build(plan, inp, torch, exx.PREC_BF16X3)
    assert e.value.code == -5


def test_binding_rejects_wrong_arrays(exx):
    sysm = synth.water_cluster(2, seed=1)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    bad = [(C.float(), V, D, K), (C, V[:-1], D, K), (C, V, D.cpu(), K), (C, V, D, K[::2]),
           (C, V, D, torch.empty(plan.info["d_size"] + 1, dtype=torch.float64, device="cuda:0"))]
    for args in bad:
        with pytest.raises(exx.ExxError) as e:
            plan.build_K(*args)
        assert e.value.code == -1
    with pytest.raises(exx.ExxError):
        plan.build_K_spin(C, V, D, torch.empty(2 * plan.info["d_size"], dtype=torch.float64, device="cuda:0"))
