"""Periodic systems (lattice images, the pattern-folded X of the real-space
exchange) on the GPU against the periodic oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import device_inputs, relmax, run_build

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def _tiny(seed, species=(0, 1, 1, 0, 1)):
    lat = np.array([[3.0, 0.0, 0.0], [0.4, 3.2, 0.0], [0.2, -0.3, 3.4]])
    pos = np.array([[0.2, 0.3, 0.1], [2.6, 0.5, 0.4], [1.3, 2.9, 3.0], [1.5, 1.6, 1.7], [0.5, 2.8, 3.2]])
    return synth.System(np.array(species), pos, 1.45, seed, lattice=lat)


def _check_full(exx, sysm, tol=TOL):
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    assert np.array_equal(plan.pair_images(), inp.layout.pair_img)
    K, Ex = run_build(plan, inp, torch)
    n = int(inp.layout.sys_nbas[0])
    Kg = K.reshape(n, n)
    Xo = O.x_periodic(inp)
    Eo = O.periodic_energy(Xo, inp.D.reshape(n, n))
    print(f"{sysm.name}: rel {relmax(Kg, Xo):.2e}, E {Ex[0]:.10e} vs {Eo:.10e}", flush=True)
    assert relmax(Kg, Xo) < tol
    assert abs(Ex[0] - Eo) < tol * abs(Eo)
    assert np.array_equal(Kg, Kg.T)
    return plan, inp, K, Ex


@pytest.mark.parametrize("seed", [1, 2])
def test_tiny_skewed_cell_matches_oracle(exx, seed):
    """A skewed cell with water species whose atoms pair with images across
    faces, edges and corners: the whole folded X and E_x."""
    _check_full(exx, _tiny(seed))


def test_one_cell_ice_matches_oracle(exx):
    """One diamond-like cell of 8 waters, r_cut 3.4 A (below half the 7.16 A
    edge): the whole folded X and E_x."""
    _check_full(exx, synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4))


def test_vacuum_box_equals_cluster(exx):
    """A cluster in a cell far wider than its reach: the periodic build gives
    the cluster build's K on the pair pattern and the same E_x."""
    cl = synth.water_cluster(8, seed=6)
    vb = synth.System(cl.species, cl.pos, cl.r_cut, cl.seed, lattice=np.diag([60.0, 61.0, 62.0]), name="vacuum")
    ic, iv = synth.make_inputs(cl), synth.make_inputs(vb)
    Kc, Ec = run_build(exx.Plan.for_system(cl), ic, torch)
    Kv, Ev = run_build(exx.Plan.for_system(vb), iv, torch)
    n = int(ic.layout.sys_nbas[0])
    blk = O.Blocks(ic)
    mask = np.zeros((blk.nat, blk.nat), bool)
    mask[blk.pa, blk.pb] = mask[blk.pb, blk.pa] = True
    atom = np.repeat(np.arange(blk.nat), blk.nb)
    M = mask[atom][:, atom]
    assert relmax(Kv.reshape(n, n), np.where(M, Kc.reshape(n, n), 0.0)) < 1e-12
    assert np.all(Kv.reshape(n, n)[~M] == 0.0)
    assert abs(Ev[0] - Ec[0]) < 1e-12 * abs(Ec[0])


def test_supercell_is_extensive(exx):
    """E_x per cell of a 2x1x1 and a 1x2x1 supercell is twice the cell's."""
    cell = synth.ice_box_periodic(1, 1, 1, seed=7, r_cut=3.4)
    _, Ec = run_build(exx.Plan.for_system(cell), synth.make_inputs(cell), torch)
    for mult in ([2, 1, 1], [1, 2, 1]):
        sup = synth.supercell(cell, mult)
        _, Es = run_build(exx.Plan.for_system(sup), synth.make_inputs(sup), torch)
        assert abs(Es[0] - 2 * Ec[0]) < 1e-12 * abs(Ec[0]), (mult, Es[0], 2 * Ec[0])


def test_2x2x2_box_sampled_rows_and_mixed(exx):
    """64 waters, r_cut 6 A: rows of an O and an H atom against the oracle;
    the mixed build (default split) within the mixed bar of the FP64 build;
    the FP64 build bitwise run to run; graph replays equal the eager build."""
    sysm = synth.ice_box_periodic(2, 2, 2, seed=8, r_cut=6.0)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K, Ex = run_build(plan, inp, torch)
    K2, Ex2 = run_build(plan, inp, torch)
    assert np.array_equal(K, K2) and np.array_equal(Ex, Ex2)
    n = int(inp.layout.sys_nbas[0])
    Kg = K.reshape(n, n)
    pb = O.PBlocks(inp)
    for a in (30, 31):
        rows = np.arange(pb.bo[a], pb.bo[a + 1])
        Xr = O.x_atom_rows_periodic(inp, [a], pb)
        print(f"atom {a}: rel {np.abs(Kg[rows] - Xr).max() / np.abs(Xr).max():.2e}", flush=True)
        assert np.abs(Kg[rows] - Xr).max() < TOL * np.abs(Xr).max()
    Km, Em = run_build(plan, inp, torch, exx.PREC_MIXED)
    dK, dE = np.abs(Km - K).max(), abs(Em[0] - Ex[0]) / sysm.n_atoms
    print(f"mixed: max|dK| {dK:.2e}, |dE|/atom {dE:.2e}", flush=True)
    assert dK <= 1e-5 and dE <= 1e-6
    C, V, D = device_inputs(inp, torch)
    Kd = torch.empty_like(D)
    Ed = torch.empty(1, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    plan.graph_build(C, V, D, Kd, Ed, stream=s.cuda_stream)
    for _ in range(2):
        Kd.fill_(3.0)
        torch.cuda.synchronize()
        plan.graph_launch(stream=s.cuda_stream)
        torch.cuda.synchronize()
        assert np.array_equal(Kd.cpu().numpy(), K) and Ed.item() == Ex[0]


def _grads(plan, inp, gE=1.0, K=None):
    C, V, D = device_inputs(inp, torch)
    dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D)
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device="cuda:0")
    plan.exchange_backward(C, V, D, gE, dC=dC, dV=dV, dD=dD, forces=F, K=K)
    torch.cuda.synchronize()
    return {k: x.cpu().numpy() for k, x in (("dC", dC), ("dV", dV), ("dD", dD), ("F", F.view(-1, 3)))}


def test_periodic_gradients_against_oracle_differences(exx):
    """Skewed tiny cell: dE/dC, dE/dV and dE/dD entries against central
    differences of the oracle's periodic E_x (E is quadratic in C and D and
    linear in V, so the differences are exact up to rounding)."""
    sysm = _tiny(5)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    g = _grads(plan, inp)
    n = int(inp.layout.sys_nbas[0])
    rng = np.random.default_rng(3)

    def energy(C=None, V=None, D=None):
        i2 = synth.Inputs(sysm, inp.layout, inp.C if C is None else C, inp.V if V is None else V,
                          inp.D if D is None else D)
        return O.periodic_energy(O.x_periodic(i2), i2.D.reshape(n, n))

    h = 1e-3
    for name, arr in (("dC", inp.C), ("dV", inp.V)):
        for idx in rng.choice(len(arr), 4, replace=False):
            e = []
            for sgn in (1, -1):
                x = arr.copy()
                x[idx] += sgn * h
                e.append(energy(**{name[1]: x}))
            fd = (e[0] - e[1]) / (2 * h)
            print(f"{name}[{idx}]: FD {fd:.10f}  GPU {g[name][idx]:.10f}", flush=True)
            assert abs(fd - g[name][idx]) < 1e-7 * max(1.0, abs(fd))
    # dD on the pattern: a symmetric perturbation of (a, b) and (b, a) gives dD_ab + dD_ba
    nz = np.nonzero(inp.D)[0]
    for idx in rng.choice(nz, 3, replace=False):
        a, b = divmod(int(idx), n)
        e = []
        for sgn in (1, -1):
            x = inp.D.copy()
            x[a * n + b] += sgn * h
            if a != b:
                x[b * n + a] += sgn * h
            e.append(energy(D=x))
        fd = (e[0] - e[1]) / (2 * h)
        an = g["dD"][a * n + b] + (g["dD"][b * n + a] if a != b else 0.0)
        assert abs(fd - an) < 1e-7 * max(1.0, abs(fd)), (a, b, fd, an)


def _moved_periodic(inp, A, axis, h, c_decay=1.5, v_2s2=8.0):
    """Atom A moved by h along axis, pair lists frozen: the blocks of every pair
    involving A rescaled by the generator's distance model at the pair's image."""
    sysm, lay = inp.system, inp.layout
    pos = sysm.pos.copy()
    pos[A, axis] += h
    C, V = inp.C.copy(), inp.V.copy()
    for p in np.nonzero((lay.pair_a == A) ^ (lay.pair_b == A))[0]:
        a, b = int(lay.pair_a[p]), int(lay.pair_b[p])
        sh = synth.water.image_shift(sysm.lattice, lay.pair_img[p])
        r0 = float(np.linalg.norm(sysm.pos[a] - (sysm.pos[b] + sh)))
        r1 = float(np.linalg.norm(pos[a] - (pos[b] + sh)))
        C[lay.c_off[p]:lay.c_off[p + 1]] *= np.exp(-(r1 - r0) / c_decay)
        V[lay.v_off[p]:lay.v_off[p + 1]] *= np.exp(-(r1 * r1 - r0 * r0) / v_2s2)
    return synth.Inputs(sysm, lay, C, V, inp.D)


def test_periodic_backward_identities_and_forces(exx):
    """64 waters, r_cut 6 A: Euler identities (E quadratic in C and D, linear
    in V), dE/dD = -K/2, zero net force, and forces against central
    differences of the GPU E_x (h = 1e-4 A, lists frozen) on four coordinates
    of atoms whose pairs cross the cell faces."""
    sysm = synth.ice_box_periodic(2, 2, 2, seed=9, r_cut=6.0)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K, Ex = run_build(plan, inp, torch)
    g = _grads(plan, inp)
    E = Ex[0]
    assert abs(g["dC"] @ inp.C - 2 * E) < 1e-10 * abs(E)
    assert abs(g["dV"] @ inp.V - E) < 1e-10 * abs(E)
    assert abs(g["dD"] @ inp.D - 2 * E) < 1e-10 * abs(E)
    assert np.array_equal(g["dD"], -0.5 * K)
    F = g["F"]
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max() * sysm.n_atoms
    crossing = np.unique(np.concatenate([inp.layout.pair_a[np.abs(inp.layout.pair_img).sum(1) > 0],
                                         inp.layout.pair_b[np.abs(inp.layout.pair_img).sum(1) > 0]]))
    h = 1e-4
    for A, ax in ((int(crossing[0]), 0), (int(crossing[5]), 1), (int(crossing[-1]), 2), (int(crossing[len(crossing) // 2]), 0)):
        es = [run_build(plan, _moved_periodic(inp, A, ax, s * h), torch)[1][0] for s in (1, -1)]
        fd = -(es[0] - es[1]) / (2 * h)
        print(f"atom {A} axis {ax}: FD {fd:.9f}  analytic {F[A, ax]:.9f}", flush=True)
        assert abs(fd - F[A, ax]) < 1e-6 * np.abs(F).max() + 1e-5


def test_periodic_gradients_vacuum_and_supercell(exx):
    """The cluster's gradients from a cell far wider than its reach; a 2x1x1
    supercell's dC and dV repeat the cell's on every copy of a block (each copy
    of a pair block carries the cell's gradient)."""
    cl = synth.water_cluster(4, seed=10)
    vb = synth.System(cl.species, cl.pos, cl.r_cut, cl.seed, lattice=np.diag([60.0, 61.0, 62.0]))
    ic, iv = synth.make_inputs(cl), synth.make_inputs(vb)
    gc, gv = _grads(exx.Plan.for_system(cl), ic), _grads(exx.Plan.for_system(vb), iv)
    for k in ("dC", "dV", "F"):
        assert relmax(gv[k], gc[k]) < 1e-12, k
    cell = synth.ice_box_periodic(1, 1, 1, seed=11, r_cut=3.4)
    sup = synth.supercell(cell, [2, 1, 1])
    ic, isu = synth.make_inputs(cell), synth.make_inputs(sup)
    g1, g2 = _grads(exx.Plan.for_system(cell), ic), _grads(exx.Plan.for_system(sup), isu)
    l1, l2 = ic.layout, isu.layout
    nat = cell.n_atoms
    for p in range(l2.n_pairs):
        a, b = int(l2.pair_a[p]), int(l2.pair_b[p])
        a0, b0 = a % nat, b % nat
        # the cell pair with the same atoms and relative image (in cells of the cell lattice)
        n_cell = sup.cell_index[b] - sup.cell_index[a] + sup.cell_mult * l2.pair_img[p]
        if a0 <= b0:
            q = [i for i in range(l1.n_pairs) if l1.pair_a[i] == a0 and l1.pair_b[i] == b0
                 and np.array_equal(l1.pair_img[i], n_cell)]
            flip = False
        else:
            q = [i for i in range(l1.n_pairs) if l1.pair_a[i] == b0 and l1.pair_b[i] == a0
                 and np.array_equal(l1.pair_img[i], -n_cell)]
            flip = True
        assert len(q) == 1
        if flip:
            continue   # stored in the other orientation in the cell: compared through its mirror pair
        q = q[0]
        assert relmax(g2["dC"][l2.c_off[p]:l2.c_off[p + 1]], g1["dC"][l1.c_off[q]:l1.c_off[q + 1]]) < 1e-12
        assert relmax(g2["dV"][l2.v_off[p]:l2.v_off[p + 1]], g1["dV"][l1.v_off[q]:l1.v_off[q + 1]]) < 1e-12


def test_periodic_spin_and_two_kernels(exx):
    """Collinear spin and two Coulomb matrices on periodic cells: each X^s and X^a
    against the periodic oracle with D^s or V^a (a skewed 5-atom cell and one ice
    cell), the spin E_x = -1/2 sum_s <X^s, D^s> and E_x per Coulomb matrix; on a
    2x2x2-cell box every result bitwise equal to build_K with that D or V."""
    dev = "cuda:0"
    for sysm in (_tiny(1), synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)):
        inp = synth.make_inputs(sysm)
        plan = exx.Plan.for_system(sysm)
        n = int(inp.layout.sys_nbas[0])
        ds = n * n
        C, V, D = device_inputs(inp, torch)
        Ds = synth.spin_densities(inp)
        K2 = torch.empty(2 * ds, dtype=torch.float64, device=dev)
        Ex = torch.empty(1, dtype=torch.float64, device=dev)
        plan.build_K_spin(C, V, torch.from_numpy(Ds.reshape(-1)).to(dev), K2, Ex)
        torch.cuda.synchronize()
        Kg = K2.cpu().numpy()
        Es = 0.0
        for s in range(2):
            Xo = O.x_periodic(O.with_density(inp, Ds[s]))
            print(f"{sysm.name} spin {s}: rel {relmax(Kg[s * ds:(s + 1) * ds].reshape(n, n), Xo):.2e}", flush=True)
            assert relmax(Kg[s * ds:(s + 1) * ds].reshape(n, n), Xo) < TOL
            Es += 2.0 * O.periodic_energy(Xo, Ds[s].reshape(n, n))
        assert abs(float(Ex.item()) - Es) < TOL * abs(Es)
        V2 = synth.short_range_V(inp)
        E2 = torch.empty(2, dtype=torch.float64, device=dev)
        plan.build_K_two_kernels(C, V, torch.from_numpy(V2).to(dev), D, K2, E2)
        torch.cuda.synchronize()
        Kg, Eg = K2.cpu().numpy(), E2.cpu().numpy()
        for a, Va in enumerate((inp.V, V2)):
            Xo = O.x_periodic(O.with_coulomb(inp, Va))
            assert relmax(Kg[a * ds:(a + 1) * ds].reshape(n, n), Xo) < TOL
            Eo = O.periodic_energy(Xo, inp.D.reshape(n, n))
            assert abs(Eg[a] - Eo) < TOL * abs(Eo)
    sysm = synth.ice_box_periodic(2, 2, 2, seed=9, r_cut=6.0)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    ds = int(inp.layout.d_size)
    C, V, D = device_inputs(inp, torch)
    Ds = torch.from_numpy(synth.spin_densities(inp).reshape(-1)).to(dev)
    V2 = torch.from_numpy(synth.short_range_V(inp)).to(dev)
    K2 = torch.empty(2 * ds, dtype=torch.float64, device=dev)
    K1 = torch.empty(ds, dtype=torch.float64, device=dev)
    plan.build_K_spin(C, V, Ds, K2)
    for s in range(2):
        plan.build_K(C, V, Ds[s * ds:(s + 1) * ds].contiguous(), K1)
        assert torch.equal(K1, K2[s * ds:(s + 1) * ds])
    plan.build_K_two_kernels(C, V, V2, D, K2)
    for a, Va in enumerate((V, V2)):
        plan.build_K(C, Va, D, K1)
        assert torch.equal(K1, K2[a * ds:(a + 1) * ds])


@pytest.mark.parametrize("which", ["cell", "box"])
def test_periodic_chunked_plan_equals_stored(exx, which):
    """A workspace budget half the stored intermediates splits a periodic plan
    into chunks of V-stage groups; per chunk the pattern contraction keeps the
    terms of the chunk's aux atoms.  K, E_x (FP64, mixed, FP32), every
    gradient (dV bit for bit) and the spin build agree with the unbounded plan."""
    sysm = (synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4) if which == "cell"
            else synth.ice_box_periodic(2, 2, 2, seed=8, r_cut=6.0))
    inp = synth.make_inputs(sysm)
    full = exx.Plan.for_system(sysm)
    stored = full.info["intermediate_bytes_stored"]
    part = exx.Plan.for_system(sysm, ws_budget_bytes=stored // 2)
    nch = part.info["n_chunks"]
    print(f"{which}: stored {stored / 1e9:.3f} GB, {nch} chunks, held {part.info['intermediate_bytes'] / 1e9:.3f} GB",
          flush=True)
    assert full.info["n_chunks"] == 1 and nch >= 3
    assert part.info["intermediate_bytes"] <= stored // 2
    K1, E1 = run_build(full, inp, torch)
    K2, E2 = run_build(part, inp, torch)
    n = int(inp.layout.sys_nbas[0])
    print(f"{which}: rel {relmax(K2, K1):.2e}", flush=True)
    assert relmax(K2, K1) < 1e-12 and abs(E2[0] - E1[0]) < 1e-12 * abs(E1[0])
    assert np.array_equal(K2.reshape(n, n), K2.reshape(n, n).T)
    if which == "cell":
        assert relmax(K2.reshape(n, n), O.x_periodic(inp)) < TOL
    for prec in (exx.PREC_MIXED, exx.PREC_FP32):
        Km1, Em1 = run_build(full, inp, torch, prec)
        Km2, Em2 = run_build(part, inp, torch, prec)
        assert relmax(Km2, Km1) < 1e-12 and abs(Em2[0] - Em1[0]) < 1e-12 * abs(Em1[0])
    g1, g2 = _grads(full, inp), _grads(part, inp)
    assert relmax(g2["dC"], g1["dC"]) < 1e-12 and np.array_equal(g1["dV"], g2["dV"])
    assert relmax(g2["dD"], g1["dD"]) < 1e-12 and relmax(g2["F"], g1["F"]) < 1e-12
    C, V, D = device_inputs(inp, torch)
    Ds = torch.from_numpy(synth.spin_densities(inp).reshape(-1)).to("cuda:0")
    Kf, Kp = (torch.empty(2 * n * n, dtype=torch.float64, device="cuda:0") for _ in range(2))
    full.build_K_spin(C, V, Ds, Kf)
    part.build_K_spin(C, V, Ds, Kp)
    torch.cuda.synchronize()
    assert relmax(Kp.cpu().numpy(), Kf.cpu().numpy()) < 1e-12


def test_periodic_unsupported_calls(exx):
    sysm = synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)
    with pytest.raises(exx.ExxError) as e:   # a budget below one V-stage group's E atoms
        exx.Plan.for_system(sysm, ws_budget_bytes=1 << 20)
    assert e.value.code == -2
    with pytest.raises(exx.ExxError) as e:   # cutoff not below half the cell width
        exx.Plan(sysm.species, sysm.pos, sysm.basis_table, sysm.aux_table, 3.7, lattice=sysm.lattice)
    assert e.value.code == -1


def test_config5_full_size(exx):
    """The periodic 3072-atom ice box (1024 waters, r_cut 8 A), in the launch
    configuration the benchmark times: the FP64 build is exactly symmetric and
    bitwise reproducible, matches the oracle on the rows of one H atom, and the
    mixed build stays within the mixed bar of it."""
    import time
    t0 = time.time()
    sysm = synth.config(5)
    inp = synth.make_inputs(sysm)
    print(f"config 5 inputs: {time.time() - t0:.1f} s, {inp.layout.n_pairs} pairs", flush=True)
    plan = exx.Plan.for_system(sysm)
    print(f"plan: {time.time() - t0:.1f} s, {plan.info['flops_fp64'] / 1e12:.2f} TFLOP per build, "
          f"workspace {plan.info['workspace_bytes'] / 1e9:.1f} GB", flush=True)
    assert np.array_equal(plan.pair_images(), inp.layout.pair_img)
    C, V, D = device_inputs(inp, torch)
    K = torch.empty_like(D)
    Ex = torch.empty(1, dtype=torch.float64, device="cuda:0")
    plan.autotune(C, V, D, K)
    plan.build_K(C, V, D, K, Ex)
    torch.cuda.synchronize()
    K1, E1 = K.clone(), Ex.item()
    plan.build_K(C, V, D, K, Ex)
    torch.cuda.synchronize()
    assert torch.equal(K, K1) and Ex.item() == E1
    n = int(inp.layout.sys_nbas[0])
    Km = K1.view(n, n)
    assert torch.equal(Km, Km.T)
    print(f"builds: {time.time() - t0:.1f} s, E_x per atom {E1 / sysm.n_atoms:.6f}", flush=True)
    pb = O.PBlocks(inp)
    rows = np.arange(pb.bo[1], pb.bo[2])
    Xr = O.x_atom_rows_periodic(inp, [1], pb)
    Kr = Km[torch.as_tensor(rows, device="cuda:0")].cpu().numpy()
    rel = np.abs(Kr - Xr).max() / np.abs(Xr).max()
    print(f"oracle rows of atom 1: rel {rel:.2e} ({time.time() - t0:.1f} s)", flush=True)
    assert rel < TOL
    plan.build_K(C, V, D, K, Ex, precision=exx.PREC_MIXED)
    torch.cuda.synchronize()
    dK = (K - K1).abs().max().item()
    dE = abs(Ex.item() - E1) / sysm.n_atoms
    print(f"mixed: max|dK| {dK:.2e}, |dE|/atom {dE:.2e}", flush=True)
    assert dK <= 1e-5 and dE <= 1e-6
