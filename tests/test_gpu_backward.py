"""exchange_backward (FP64) against the CPU oracle, finite differences and
identities that hold at any size."""
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


def backward(plan, inp, gE=1.0, want=("dC", "dV", "dD", "F")):
    dev = "cuda:0"
    C, V, D = device_inputs(inp, torch)
    out = {}
    dC = torch.empty_like(C) if "dC" in want else None
    dV = torch.empty_like(V) if "dV" in want else None
    dD = torch.empty_like(D) if "dD" in want else None
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device=dev) if "F" in want else None
    plan.exchange_backward(C, V, D, gE, dC=dC, dV=dV, dD=dD, forces=F)
    torch.cuda.synchronize()
    for k, x in (("dC", dC), ("dV", dV), ("dD", dD), ("F", F)):
        if x is not None:
            out[k] = x.cpu().numpy()
    if "F" in out:
        out["F"] = out["F"].reshape(-1, 3)
    return out


@pytest.mark.parametrize("n_mol,seed", [(1, 1), (2, 2), (8, 0)])
def test_gradients_match_oracle(exx, n_mol, seed):
    sysm = synth.water_cluster(n_mol, seed)
    print("backward cluster", n_mol, flush=True)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    g = backward(plan, inp)
    go = O.gradients(inp)
    assert relmax(g["dC"], go["dC"]) < 1e-10
    assert relmax(g["dV"], go["dV"]) < 1e-10
    assert relmax(system_block(g["dD"], inp.layout, 0), go["dD"]) < 1e-10
    Fo = O.forces(inp, go)
    assert relmax(g["F"], Fo) < 1e-10


@pytest.mark.parametrize("tables", [([16, 3], [64, 7]), ([1, 2], [1, 5])])
def test_gradients_other_species_shapes(exx, tables):
    nb, na = tables
    base = synth.water_cluster(3, seed=21)
    sysm = synth.System(base.species, base.pos, 6.0, seed=21,
                        basis_table=np.array(nb), aux_table=np.array(na))
    print("backward species tables", tables, flush=True)
    inp = synth.make_inputs(sysm)
    g = backward(exx.Plan.for_system(sysm), inp)
    go = O.gradients(inp)
    assert relmax(g["dC"], go["dC"]) < 1e-10
    assert relmax(g["dV"], go["dV"]) < 1e-10
    assert relmax(system_block(g["dD"], inp.layout, 0), go["dD"]) < 1e-10
    assert relmax(g["F"], O.forces(inp, go)) < 1e-10


def test_partial_outputs_and_scaling(exx):
    sysm = synth.water_cluster(2, 5)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    full = backward(plan, inp, gE=1.0)
    part = backward(plan, inp, gE=-2.5, want=("dC",))
    assert relmax(part["dC"], -2.5 * full["dC"]) < 1e-13
    only_f = backward(plan, inp, gE=1.0, want=("F",))
    assert relmax(only_f["F"], full["F"]) < 1e-13
    only_v = backward(plan, inp, gE=1.0, want=("dV",))
    assert np.array_equal(only_v["dV"], full["dV"])


def test_forces_central_differences(exx):
    """-dE/dR by central differences (1e-4 A) of the GPU FP64 energy, pair
    lists frozen at the reference geometry, D held fixed."""
    sysm = synth.water_cluster(3, 11)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    F = backward(plan, inp, want=("F",))["F"]
    rng = np.random.default_rng(3)
    h = 1e-4
    for _ in range(6):
        A, x = int(rng.integers(0, sysm.n_atoms)), int(rng.integers(0, 3))
        es = []
        for sgn in (+1, -1):
            pos = sysm.pos.copy()
            pos[A, x] += sgn * h
            s2 = synth.System(sysm.species, pos, sysm.r_cut, sysm.seed)
            i2 = synth.make_inputs(s2, inp.layout)
            i2.D[:] = inp.D
            _, Ex = run_build(plan, i2, torch)
            es.append(Ex[0])
        fd = -(es[0] - es[1]) / (2 * h)
        assert abs(fd - F[A, x]) < 1e-6 * max(1.0, abs(F[A, x])), (A, x, fd, F[A, x])


def test_identities_on_768_atom_box(exx):
    """Euler identities (E is quadratic in C and D, linear in V), force and
    torque balance, and dE/dD = -K/2 at full size."""
    inp = synth.make_inputs(synth.config(4))
    sysm = inp.system
    plan = exx.Plan.for_system(sysm)
    K, Ex = run_build(plan, inp, torch)
    g = backward(plan, inp)
    E = Ex[0]
    assert abs(g["dC"] @ inp.C - 2 * E) < 1e-10 * abs(E)
    assert abs(g["dV"] @ inp.V - E) < 1e-10 * abs(E)
    assert abs(g["dD"] @ inp.D - 2 * E) < 1e-10 * abs(E)
    assert np.array_equal(g["dD"], -0.5 * K)
    F = g["F"]
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-10 * scale * sysm.n_atoms
    assert np.abs(np.cross(sysm.pos, F).sum(0)).max() < 1e-10 * scale * sysm.n_atoms * 30


def test_autograd_function(exx):
    sysm = synth.water_cluster(2, 8)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    C.requires_grad_(True)
    V.requires_grad_(True)
    D.requires_grad_(True)
    Ex = exx.exchange_energy(plan, C, V, D)
    (3.0 * Ex.sum()).backward()
    go = O.gradients(inp)
    assert relmax(C.grad.cpu().numpy(), 3.0 * go["dC"]) < 1e-10
    assert relmax(V.grad.cpu().numpy(), 3.0 * go["dV"]) < 1e-10
    assert relmax(system_block(D.grad.cpu().numpy(), inp.layout, 0), 3.0 * go["dD"]) < 1e-10
    F = exx.exchange_forces(plan, C.detach(), V.detach(), D.detach()).cpu().numpy()
    assert relmax(F, O.forces(inp, go)) < 1e-10


def test_backward_with_forward_K(exx):
    """Passing the forward K: dE/dD is exactly -gE K / 2 and the other
    gradients agree with the self-contained backward (and the oracle)."""
    sysm = synth.water_cluster(4, 6)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    plan.build_K(C, V, D, K)
    ref = backward(plan, inp, gE=0.7)
    dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D)
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0")
    plan.exchange_backward(C, V, D, 0.7, dC=dC, dV=dV, dD=dD, forces=F, K=K)
    torch.cuda.synchronize()
    assert np.array_equal(dD.cpu().numpy(), -0.35 * K.cpu().numpy())
    assert relmax(dC.cpu().numpy(), ref["dC"]) < 1e-12
    assert np.array_equal(dV.cpu().numpy(), ref["dV"])
    assert relmax(F.cpu().numpy().reshape(-1, 3), ref["F"]) < 1e-12
    go = O.gradients(inp)
    assert relmax(dC.cpu().numpy(), 0.7 * go["dC"]) < 1e-10


def test_autograd_mixed_forward(exx):
    """Mixed-precision forward, binary64 backward: dC and dV match the oracle at
    the FP64 bar; dD = -K/2 of the mixed K, within the mixed-path bar."""
    sysm = synth.water_cluster(8, 4)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)   # default split distance
    C, V, D = (x.clone().requires_grad_(True) for x in device_inputs(inp, torch))
    E = exx.exchange_energy(plan, C, V, D, precision=exx.PREC_MIXED)
    E.sum().backward()
    go = O.gradients(inp)
    assert relmax(C.grad.cpu().numpy(), go["dC"]) < 1e-10
    assert relmax(V.grad.cpu().numpy(), go["dV"]) < 1e-10
    dD = system_block(D.grad.cpu().numpy(), inp.layout, 0)
    assert np.abs(dD - go["dD"]).max() <= 0.5e-5
    assert abs(E.item() - go["E"]) / sysm.n_atoms <= 1e-6


def _moved(inp, A, axis, h, c_decay=1.5, v_2s2=8.0):
    """Inputs with atom A moved by h along axis and the pair lists frozen: the
    blocks of every pair (A, B) rescaled by the generator's distance model
    (C ~ exp(-r / c_decay), V ~ exp(-r^2 / v_2s2); D held fixed)."""
    lay = inp.layout
    pos = inp.system.pos.copy()
    pos[A, axis] += h
    C, V = inp.C.copy(), inp.V.copy()
    for p in np.nonzero((lay.pair_a == A) ^ (lay.pair_b == A))[0]:
        a, b = int(lay.pair_a[p]), int(lay.pair_b[p])
        r0 = float(np.linalg.norm(inp.system.pos[a] - inp.system.pos[b]))
        r1 = float(np.linalg.norm(pos[a] - pos[b]))
        C[lay.c_off[p]:lay.c_off[p + 1]] *= np.exp(-(r1 - r0) / c_decay)
        V[lay.v_off[p]:lay.v_off[p + 1]] *= np.exp(-(r1 * r1 - r0 * r0) / v_2s2)
    return synth.Inputs(inp.system, lay, C, V, inp.D)


def test_forces_fd_on_24_atoms_of_the_768_box(exx):
    """Forces on a 24-atom subset (8 molecules around the box centre) of the
    768-atom box: central differences (h = 1e-4 A) of the GPU FP64 E_x with the
    pair lists frozen, on six coordinates; and the same 8 molecules cut out as
    a cluster against the oracle's FP64 gradient and forces."""
    inp = synth.make_inputs(synth.config(4))
    sysm = inp.system
    plan = exx.Plan.for_system(sysm)
    g = backward(plan, inp, want=("F",))
    F = g["F"]
    centre = sysm.pos.mean(0)
    o_atoms = np.nonzero(sysm.species == synth.O)[0]
    near = o_atoms[np.argsort(np.linalg.norm(sysm.pos[o_atoms] - centre, axis=1), kind="stable")[:8]]
    subset = np.sort(np.concatenate([near, near + 1, near + 2]))
    assert len(subset) == 24
    h = 1e-4
    picks = [(subset[0], 0), (subset[4], 1), (subset[8], 2), (subset[13], 0), (subset[17], 1), (subset[23], 2)]
    for A, ax in picks:
        es = [run_build(plan, _moved(inp, int(A), ax, s * h), torch)[1][0] for s in (1, -1)]
        fd = -(es[0] - es[1]) / (2 * h)
        print(f"atom {A} axis {ax}: FD {fd:.9f}  analytic {F[A, ax]:.9f}", flush=True)
        assert abs(fd - F[A, ax]) < 1e-6 * np.abs(F).max() + 1e-5, (A, ax, fd, F[A, ax])
    # the 8 molecules as a standalone cluster: GPU gradients against the oracle's
    cut = synth.System(sysm.species[subset], sysm.pos[subset], sysm.r_cut, seed=sysm.seed,
                       labels=sysm.labels[subset], name="ice768_cut24")
    ci = synth.make_inputs(cut)
    cp = exx.Plan.for_system(cut)
    gc = backward(cp, ci)
    go = O.gradients(ci)
    assert relmax(gc["dC"], go["dC"]) < 1e-10 and relmax(gc["dV"], go["dV"]) < 1e-10
    assert relmax(gc["F"], O.forces(ci, go)) < 1e-10


def _grads(plan, C, V, D, gE, K, build_id=None, want=("dC", "dV", "dD", "F")):
    dC = torch.empty_like(C) if "dC" in want else None
    dV = torch.empty_like(V) if "dV" in want else None
    dD = torch.empty_like(D) if "dD" in want else None
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0") if "F" in want else None
    used = plan.exchange_backward(C, V, D, gE, dC=dC, dV=dV, dD=dD, forces=F, K=K, build_id=build_id)
    torch.cuda.synchronize()
    return used, {k: x.cpu().numpy() for k, x in (("dC", dC), ("dV", dV), ("dD", dD), ("F", F)) if x is not None}


def test_backward_reuses_forward_intermediates(exx):
    """After a binary64 build_K, exchange_backward_reuse takes E and H' from the
    workspace: dD and dV equal the recomputing backward's bit for bit (E is the
    same), dC and the forces to rounding (H' gets its G term back to once by a
    pass of its own).  Once any call has written the workspace since, or after
    a mixed or screened build, it recomputes and equals exchange_backward bit
    for bit."""
    sysm = synth.water_cluster(8, 3)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    plan.build_K(C, V, D, K)
    used, ref = _grads(plan, C, V, D, 0.7, K)
    assert used is None
    plan.build_K(C, V, D, K)
    bid = plan.build_id()
    used, g = _grads(plan, C, V, D, 0.7, K, bid)
    print("reuse after an FP64 build:", used, flush=True)
    assert used
    assert np.array_equal(g["dD"], ref["dD"]) and np.array_equal(g["dV"], ref["dV"])
    assert relmax(g["dC"], ref["dC"]) < 1e-12 and relmax(g["F"], ref["F"]) < 1e-12
    go = O.gradients(inp)
    assert relmax(g["dC"], 0.7 * go["dC"]) < 1e-10 and relmax(g["dV"], 0.7 * go["dV"]) < 1e-10
    used, g2 = _grads(plan, C, V, D, 0.7, K, bid)      # the backward itself moved the generation on
    assert not used and all(np.array_equal(g2[k], ref[k]) for k in ref)
    plan.build_K(C, V, D, K)
    bid = plan.build_id()
    K2 = torch.empty_like(K)
    plan.build_K(C, V, 0.5 * D, K2)                   # another build in between
    used, g3 = _grads(plan, C, V, D, 0.7, K, bid)
    assert not used and all(np.array_equal(g3[k], ref[k]) for k in ref)
    plan.build_K(C, V, D, K2, precision=exx.PREC_MIXED)
    used, _ = _grads(plan, C, V, D, 0.7, K, plan.build_id())
    assert not used
    plan.set_screening(1e-300)
    plan.build_K(C, V, D, K2)
    plan.set_screening(0.0)
    used, _ = _grads(plan, C, V, D, 0.7, K, plan.build_id())
    assert not used
    plan.build_K(C, V, D, K2)
    used, g4 = _grads(plan, C, V, D, 0.7, K, plan.build_id(), want=("dV",))
    assert used and np.array_equal(g4["dV"], ref["dV"])


def test_backward_reuse_batch_periodic_and_chunked(exx):
    """Per-system upstream gradients on a batch and a periodic cell: the reuse
    backward agrees with the recomputing one to rounding; a chunked plan does not
    reuse and gives the same gradients."""
    dev = "cuda:0"
    for name, sysm in (("batch", synth.cluster_batch(4, n_min=6, n_max=30)),
                       ("periodic", synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4))):
        inp = synth.make_inputs(sysm)
        plan = exx.Plan.for_system(sysm)
        C, V, D = device_inputs(inp, torch)
        K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
        gE = torch.linspace(0.5, 1.5, plan.n_systems, dtype=torch.float64, device=dev)
        plan.build_K(C, V, D, K)
        _, ref = _grads(plan, C, V, D, gE, K)
        plan.build_K(C, V, D, K)
        used, g = _grads(plan, C, V, D, gE, K, plan.build_id())
        print(name, "reused:", used, flush=True)
        assert used
        assert np.array_equal(g["dD"], ref["dD"]) and np.array_equal(g["dV"], ref["dV"])
        assert relmax(g["dC"], ref["dC"]) < 1e-12 and relmax(g["F"], ref["F"]) < 1e-12
    sysm = synth.ice_box(2, 2, 2, seed=3)
    inp = synth.make_inputs(sysm)
    whole = exx.Plan.for_system(sysm)
    part = exx.Plan.for_system(sysm, ws_budget_bytes=whole.info["intermediate_bytes_stored"] // 3)
    assert part.info["n_chunks"] >= 3
    C, V, D = device_inputs(inp, torch)
    K = torch.empty(part.info["d_size"], dtype=torch.float64, device=dev)
    whole.build_K(C, V, D, K)
    _, ref = _grads(whole, C, V, D, 1.0, K)
    part.build_K(C, V, D, K)
    used, g = _grads(part, C, V, D, 1.0, K, part.build_id())
    assert not used
    assert relmax(g["dC"], ref["dC"]) < 1e-12 and relmax(g["dV"], ref["dV"]) < 1e-12
