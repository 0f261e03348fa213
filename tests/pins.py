"""Independent checks ("pins") of the CPU oracle.

Each pin compares the oracle with something other than itself: a closed form
for a special input, brute force on a tiny input, an algebraic invariant of
the definition, the paper's own regrouped formula, or finite differences.
Inputs are built dense-first here and packed into the library layout by this
module's own packer, so a mistake in the oracle's unpacking also shows up.

Every pin returns (ok, detail) so the mutation tests can reuse them.
"""
from __future__ import annotations

import math

import numpy as np

import synth
from oracle import exx_oracle as O

TOL = 1e-12


def rel(a, b):
    cplx = np.iscomplexobj(a) or np.iscomplexobj(b)
    a, b = np.asarray(a, complex if cplx else float), np.asarray(b, complex if cplx else float)
    s = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / s)


# ----------------------------------------------------------------------------
# dense-first random problems packed into the layout


def _offsets(sysm):
    nb = sysm.nbas().astype(int)
    na = sysm.naux().astype(int)
    return nb, na, np.concatenate([[0], np.cumsum(nb)]), np.concatenate([[0], np.cumsum(na)])


def random_problem(sysm, seed, d_rank1=None):
    """Dense C3, V, D with the RI-LVL structure, plus the packed Inputs.

    Off-site V blocks are generic (not symmetric); D is symmetric unless a
    rank-1 pair (v, w) is requested, in which case D = v w^T."""
    rng = np.random.default_rng(seed)
    lay = synth.make_layout(sysm)
    nb, na, bo, ao = _offsets(sysm)
    n, naux = bo[-1], ao[-1]
    C3 = np.zeros((naux, n, n))
    Vd = np.zeros((naux, naux))
    C = np.empty(int(lay.c_off[-1]))
    V = np.empty(int(lay.v_off[-1]))
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
        ma, mb = slice(ao[a], ao[a + 1]), slice(ao[b], ao[b + 1])
        if a == b:
            x = rng.normal(size=(na[a], nb[a], nb[a]))
            x = x + x.transpose(0, 2, 1)
            C3[ma, ia, ia] = x
            C[lay.c_off[p]:lay.c_off[p + 1]] = x.ravel()
            v = rng.normal(size=(na[a], na[a]))
            v = v + v.T
            Vd[ma, ma] = v
        else:
            x = rng.normal(size=(na[a] + na[b], nb[a], nb[b]))
            C3[ma, ia, ib] = x[:na[a]]
            C3[ma, ib, ia] = x[:na[a]].transpose(0, 2, 1)
            C3[mb, ia, ib] = x[na[a]:]
            C3[mb, ib, ia] = x[na[a]:].transpose(0, 2, 1)
            C[lay.c_off[p]:lay.c_off[p + 1]] = x.ravel()
            v = rng.normal(size=(na[a], na[b]))
            Vd[ma, mb] = v
            Vd[mb, ma] = v.T
        V[lay.v_off[p]:lay.v_off[p + 1]] = v.ravel()
    if d_rank1 is None:
        Dd = rng.normal(size=(n, n))
        Dd = Dd + Dd.T
    else:
        v, w = d_rank1
        Dd = np.outer(v, w)
    inp = synth.Inputs(sysm, lay, C, V, Dd.ravel().copy())
    return inp, C3, Vd, Dd


# ----------------------------------------------------------------------------
# pins


def pin_rank1_closed_form(route="4index", seed=1):
    """D = v w^T  =>  K = U V W^T with U[:, mu] = C^mu v, W[:, nu] = C^nu w;
    for w = v:  E_x = -1/4 q^T V q with q_mu = v^T C^mu v."""
    sysm = synth.water_cluster(2, seed)
    nb, *_ = _offsets(sysm)
    rng = np.random.default_rng(seed + 100)
    n = int(nb.sum())
    v, w = rng.normal(size=n), rng.normal(size=n)
    inp, C3, Vd, _ = random_problem(sysm, seed, d_rank1=(v, w))
    U = np.einsum("mij,j->im", C3, v)
    W = np.einsum("mij,j->im", C3, w)
    K_closed = U @ Vd @ W.T
    K = _route(inp, route)
    ok1 = rel(K, K_closed) < TOL
    inp2, C3, Vd, Dd = random_problem(sysm, seed, d_rank1=(v, v))
    q = np.einsum("i,mij,j->m", v, C3, v)
    E_closed = -0.25 * q @ Vd @ q
    E = O.exchange_energy(_route(inp2, route), Dd)
    ok2 = abs(E - E_closed) <= TOL * abs(E_closed)
    return ok1 and ok2, f"K rel {rel(K, K_closed):.2e}  E {E:.6e} vs {E_closed:.6e}"


def _route(inp, route):
    if route == "4index":
        return O.k_4index(inp)[0]
    if route == "eigen":
        return O.k_eigen(inp)
    if route == "rows":
        return O.k_full_rows(inp)
    if route == "block":
        blk = O.Blocks(inp)
        return O.k_atom_rows(inp, range(blk.nat), blk=blk)
    raise ValueError(route)


def pin_brute_force(seed=2, n_entries=12):
    """K_ik by explicit loops over j, l, mu, nu on a two-hydrogen system."""
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.7]])
    sysm = synth.System(np.array([synth.H, synth.H]), pos, 6.0, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    K = O.k_4index(inp)[0]
    Kr = O.k_full_rows(inp)
    rng = np.random.default_rng(seed)
    n, naux = Dd.shape[0], Vd.shape[0]
    worst = 0.0
    for _ in range(n_entries):
        i, k = (int(x) for x in rng.integers(0, n, 2))
        s = 0.0
        for j in range(n):
            for l in range(n):
                for mu in range(naux):
                    cij = C3[mu, i, j]
                    if cij == 0.0:
                        continue
                    for nu in range(naux):
                        s += cij * Vd[mu, nu] * C3[nu, k, l] * Dd[j, l]
        worst = max(worst, abs(K[i, k] - s) / max(abs(s), 1e-12), abs(Kr[i, k] - s) / max(abs(s), 1e-12))
    return worst < 1e-12, f"worst rel {worst:.2e}"


def pin_invariants(route="4index", seed=3):
    """K = K^T for symmetric D; K linear in D; D = 0 gives K = 0."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    K1 = _route(inp, route)
    sym = rel(K1, K1.T)
    rng = np.random.default_rng(seed)
    D2 = rng.normal(size=Dd.shape)
    D2 = D2 + D2.T
    a, b = 0.7, -1.3
    inp2 = synth.Inputs(sysm, inp.layout, inp.C, inp.V, D2.ravel().copy())
    inp3 = synth.Inputs(sysm, inp.layout, inp.C, inp.V, (a * Dd + b * D2).ravel())
    K2, K3 = _route(inp2, route), _route(inp3, route)
    lin = rel(K3, a * K1 + b * K2)
    inp0 = synth.Inputs(sysm, inp.layout, inp.C, inp.V, np.zeros_like(inp.D))
    zero = float(np.abs(_route(inp0, route)).max())
    ok = sym < TOL and lin < TOL and zero == 0.0
    return ok, f"sym {sym:.1e} lin {lin:.1e} zero {zero}"


def pin_permutation(route="rows", seed=4):
    """Reordering the atoms permutes K the same way (generator keyed by label)."""
    sysm = synth.water_cluster(3, seed)
    inp = synth.make_inputs(sysm)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(sysm.n_atoms)
    sp = synth.permuted(sysm, perm)
    inp_p = synth.make_inputs(sp)
    K = _route(inp, route)
    Kp = _route(inp_p, route)
    nb = sysm.nbas()
    bo = np.concatenate([[0], np.cumsum(nb)])
    bidx = np.concatenate([np.arange(bo[a], bo[a + 1]) for a in perm])
    r = rel(Kp, K[np.ix_(bidx, bidx)])
    return r < TOL, f"perm rel {r:.1e}"


def pin_energy_direct(seed=5):
    """E_x from K equals E_x contracted directly from (ij|kl) with D (x) D."""
    sysm = synth.water_cluster(2, seed)
    inp, *_ = random_problem(sysm, seed)
    K, e1, e2 = O.k_4index(inp)
    return abs(e1 - e2) <= TOL * abs(e1), f"{e1:.12e} vs {e2:.12e}"


def pin_routes_agree(seed=6):
    """The 4-index, eigen, row and block routes give the same K."""
    sysm = synth.water_cluster(2, seed)
    inp, *_ = random_problem(sysm, seed)
    K4 = O.k_4index(inp)[0]
    r1, r2, r3 = rel(K4, O.k_eigen(inp)), rel(K4, O.k_full_rows(inp)), rel(K4, _route(inp, "block"))
    return max(r1, r2, r3) < TOL, f"eigen {r1:.1e} rows {r2:.1e} block {r3:.1e}"


def pin_block_route(seed=16):
    """The block route (the CPU baseline's) on its own: the rank-1 closed form,
    the invariants, and a three-molecule cluster with atoms of uneven
    neighbourhoods against the 4-index route."""
    ok1, m1 = pin_rank1_closed_form(route="block", seed=seed)
    ok2, m2 = pin_invariants(route="block", seed=seed + 1)
    sysm = synth.water_cluster(3, seed)
    sysm.r_cut = 3.2
    inp, *_ = random_problem(sysm, seed)
    r = rel(_route(inp, "block"), O.k_4index(inp)[0])
    return ok1 and ok2 and r < TOL, f"{m1}; {m2}; cut 3.2 A vs 4-index {r:.1e}"


def paper_regrouped_X(C3, Vd, Dd, aux_atom, bas_atom):
    """The paper's pair-grouped exchange with intermediates E, F, G, H at R = 0
    (Eq. ri_lvl_exchange_matrix with Eq. temp, Sec. "Description of the
    real-space formalism"), with on-site coefficient blocks counted once by
    halving them in the row-owned part M (the paper is silent on this)."""
    naux, n, _ = C3.shape
    own = aux_atom[:, None] == bas_atom[None, :]            # mu on atom of i
    M = C3 * own[:, :, None]                                 # rows of C^mu on A(mu)
    onsite = own[:, :, None] & own[:, None, :]
    M = np.where(onsite, 0.5 * C3, M)
    # E^nu_{jk} = sum_l C^nu_{jl} D_{kl}, nu on the atom of j
    E = np.einsum("njl,kl->njk", M, Dd)
    # F^nu_{ik} = sum_{mu on A(i)} C^mu_{ik} V_{mu nu}
    F = np.einsum("mik,mn->nik", M, Vd)
    # G^nu_{il} = sum_{mu on A(i)} E^mu_{il} V_{mu nu}
    G = np.einsum("mil,mn->nil", E, Vd)
    # H^nu_{il} = sum_k F^nu_{ki} D_{kl}
    H = np.einsum("nki,kl->nil", F, Dd)
    # X_ij = sum_{k, nu on A(j)} F^nu_ik E^nu_jk + sum_{l, nu on A(l)} (2G + H)^nu_il C^nu_lj
    X = np.einsum("nik,njk->ij", F, E) + np.einsum("nil,nlj->ij", 2.0 * G + H, M)
    return X


def pin_paper_regrouping(seed=7):
    """The symmetric part of the paper's regrouped X equals K."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    nb, na, *_ = _offsets(sysm)
    aux_atom = np.repeat(np.arange(sysm.n_atoms), na)
    bas_atom = np.repeat(np.arange(sysm.n_atoms), nb)
    X = paper_regrouped_X(C3, Vd, Dd, aux_atom, bas_atom)
    K = O.k_4index(inp)[0]
    r = rel(0.5 * (X + X.T), K)
    return r < TOL, f"sym(X) vs K rel {r:.1e}"


# ----------------------------------------------------------------------------
# gradient pins


def _grads(seed):
    sysm = synth.water_cluster(2, seed)
    inp = synth.make_inputs(sysm)
    return sysm, inp, O.gradients(inp)


def pin_euler(seed=8):
    """E is homogeneous of degree 2 in C and D and degree 1 in V."""
    sysm, inp, g = _grads(seed)
    E = g["E"]
    Dd = g["blk"].D
    eC = float(g["dC"] @ inp.C) / (2 * E) - 1
    eV = float(g["dV"] @ inp.V) / E - 1
    eD = float(np.sum(g["dD"] * Dd)) / (2 * E) - 1
    ok = max(abs(eC), abs(eV), abs(eD)) < 1e-12
    return ok, f"C {eC:.1e} V {eV:.1e} D {eD:.1e}"


def _energy(inp):
    return O.exchange_energy(O.k_eigen(inp), O.Blocks(inp).D)


def pin_fd_params(seed=9, h=1e-4, n_entries=6):
    """Central differences of E_x in stored C, V entries and symmetric D pairs."""
    sysm, inp, g = _grads(seed)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for arr_name in ("C", "V"):
        arr = getattr(inp, arr_name)
        grad = g["d" + arr_name]
        for idx in rng.integers(0, arr.size, n_entries):
            a0 = arr[idx]
            arr[idx] = a0 + h
            ep = _energy(inp)
            arr[idx] = a0 - h
            em = _energy(inp)
            arr[idx] = a0
            fd = (ep - em) / (2 * h)
            worst = max(worst, abs(fd - grad[idx]) / max(abs(grad[idx]), 1e-3))
    n = int(math.isqrt(inp.D.size))
    Dm = inp.D.reshape(n, n)
    for _ in range(n_entries):
        i, k = (int(x) for x in rng.integers(0, n, 2))
        d0 = Dm[i, k]
        for s in (+1, -1):
            Dm[i, k] = d0 + s * h
            Dm[k, i] = d0 + s * h
            if s > 0:
                ep = _energy(inp)
            else:
                em = _energy(inp)
        Dm[i, k] = d0
        Dm[k, i] = d0
        fd = (ep - em) / (2 * h)
        an = g["dD"][i, k] * (1 if i == k else 2)
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    return worst < 1e-6, f"worst rel {worst:.1e}"


def pin_dD_is_minus_half_K(seed=10):
    """dE/dD = -1/2 K, checked by central differences along a random symmetric direction."""
    sysm, inp, g = _grads(seed)
    n = int(math.isqrt(inp.D.size))
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(n, n))
    Z = Z + Z.T
    D0 = inp.D.copy()
    h = 1e-5
    inp.D[:] = (D0.reshape(n, n) + h * Z).ravel()
    ep = _energy(inp)
    inp.D[:] = (D0.reshape(n, n) - h * Z).ravel()
    em = _energy(inp)
    inp.D[:] = D0
    fd = (ep - em) / (2 * h)
    an = float(np.sum(-0.5 * g["K"] * Z))
    return abs(fd - an) < 1e-7 * abs(an), f"fd {fd:.10e} an {an:.10e}"


def pin_force_invariants(seed=11):
    """Forces from distance-only dependence: sum F = 0, sum R x F = 0."""
    sysm, inp, g = _grads(seed)
    F = O.forces(inp, g)
    scale = np.abs(F).max()
    t = np.abs(F.sum(0)).max() / scale
    tq = np.abs(np.cross(sysm.pos, F).sum(0)).max() / scale
    return max(t, tq) < 1e-12, f"sumF {t:.1e} torque {tq:.1e}"


def inputs_at(sysm, layout, D_fixed, pos):
    s2 = synth.System(sysm.species, pos, sysm.r_cut, sysm.seed, labels=sysm.labels)
    inp = synth.make_inputs(s2, layout)
    inp.D[:] = D_fixed
    return inp


def pin_fd_forces(seed=12, h=1e-4, n_checks=4):
    """Central differences (step 1e-4 A) of E_x in atom positions; pair lists
    frozen at the reference geometry, D held fixed."""
    sysm, inp, g = _grads(seed)
    F = O.forces(inp, g)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(n_checks):
        A, x = int(rng.integers(0, sysm.n_atoms)), int(rng.integers(0, 3))
        pp, pm = sysm.pos.copy(), sysm.pos.copy()
        pp[A, x] += h
        pm[A, x] -= h
        ep = _energy(inputs_at(sysm, inp.layout, inp.D, pp))
        em = _energy(inputs_at(sysm, inp.layout, inp.D, pm))
        fd = -(ep - em) / (2 * h)
        worst = max(worst, abs(fd - F[A, x]) / max(abs(F[A, x]), 1e-2))
    return worst < 1e-6, f"worst rel {worst:.1e}"


def pin_screening(seed=13):
    """Pair screening equals an explicit loop over all atom pairs."""
    ok = True
    for sysm in (synth.config(1), synth.cluster_batch(3, n_min=8, n_max=30)):
        pa, pb = O.screened_pairs(sysm.pos, sysm.r_cut, sysm.sys_off)
        got = set(zip(pa.tolist(), pb.tolist()))
        want = set()
        rc2 = sysm.r_cut * sysm.r_cut
        for s in range(sysm.n_systems):
            lo, hi = int(sysm.sys_off[s]), int(sysm.sys_off[s + 1])
            for a in range(lo, hi):
                for b in range(a, hi):
                    dx, dy, dz = (float(sysm.pos[a, c] - sysm.pos[b, c]) for c in range(3))
                    if (dx * dx + dy * dy) + dz * dz <= rc2:
                        want.add((a, b))
        ok = ok and got == want and len(want) < (sysm.n_atoms * (sysm.n_atoms + 1)) // 2
    return ok, "screened pair sets equal"


def pin_spin(seed=14):
    """Collinear spin: with D^0 = D^1 = D/2 each K^s is K(D)/2 and the spin
    energy equals the closed-shell E_x of D; for unequal spins K^0 + K^1 =
    K(D^0 + D^1) (linearity in D) and the energy is -1/2 sum_s <K^s, D^s>
    evaluated from the 4-index tensor, without K."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    K, e_cs, _ = O.k_4index(inp)
    half = [0.5 * inp.D, 0.5 * inp.D]
    Kh = O.k_spin(inp, half, route="4index")
    n = Dd.shape[0]
    e_half = O.spin_exchange_energy(Kh, [x.reshape(n, n) for x in half])
    rng = np.random.default_rng(seed)
    S = rng.normal(size=(n, n))
    S = (S + S.T) * (np.abs(Dd) > 0)
    D0 = 0.5 * (Dd + 0.4 * S)
    D1 = Dd - D0
    Ku = O.k_spin(inp, [D0.ravel(), D1.ravel()], route="eigen")
    B = np.einsum("aij,ab->bij", C3, Vd)                 # sum_mu C^mu_ij V_{mu nu}
    e_direct = sum(-0.5 * float(np.einsum("aij,akl,ik,jl->", C3, B, Dx, Dx, optimize=True))
                   for Dx in (D0, D1))
    e_spin = O.spin_exchange_energy(Ku, [D0, D1])
    r = max(rel(Kh[0], 0.5 * K), rel(Kh[1], 0.5 * K), rel(Ku[0] + Ku[1], K))
    ok = r < TOL and abs(e_half - e_cs) <= TOL * abs(e_cs) and abs(e_spin - e_direct) <= TOL * abs(e_direct)
    return ok, f"K {r:.1e}, E(D/2, D/2) {e_half:.12e} vs {e_cs:.12e}, E {e_spin:.12e} vs {e_direct:.12e}"


def pin_spin_gradients(seed=21, h=1e-4, n_entries=4):
    """Collinear-spin gradients against central differences of the spin energy
    -1/2 sum_s <K(D^s), D^s> (evaluated from the 4-index tensor) in stored C and
    V entries and in symmetric entry pairs of D^0 and of D^1 (unequal spins)."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    n = Dd.shape[0]
    rng = np.random.default_rng(seed)
    S = rng.normal(size=(n, n))
    D0 = 0.5 * (Dd + 0.4 * (S + S.T))
    D1 = Dd - D0
    Ds = [D0.ravel().copy(), D1.ravel().copy()]
    g = O.spin_gradients(inp, Ds)

    def energy():
        Ks = O.k_spin(inp, Ds, route="4index")
        return O.spin_exchange_energy(Ks, [x.reshape(n, n) for x in Ds])

    worst = 0.0
    for arr_name in ("C", "V"):
        arr = getattr(inp, arr_name)
        for idx in rng.integers(0, arr.size, n_entries):
            a0 = arr[idx]
            arr[idx] = a0 + h
            ep = energy()
            arr[idx] = a0 - h
            em = energy()
            arr[idx] = a0
            an = g["d" + arr_name][idx]
            worst = max(worst, abs((ep - em) / (2 * h) - an) / max(abs(an), 1e-3))
    for sp in (0, 1):
        Dm = Ds[sp].reshape(n, n)
        for _ in range(n_entries):
            i, k = (int(x) for x in rng.integers(0, n, 2))
            d0 = Dm[i, k]
            Dm[i, k] = Dm[k, i] = d0 + h
            ep = energy()
            Dm[i, k] = Dm[k, i] = d0 - h
            em = energy()
            Dm[i, k] = Dm[k, i] = d0
            an = g["dD"][sp][i, k] * (1 if i == k else 2)
            worst = max(worst, abs((ep - em) / (2 * h) - an) / max(abs(an), 1e-3))
    e_ok = abs(g["E"] - energy()) <= TOL * abs(g["E"])
    return worst < 1e-6 and e_ok, f"worst rel {worst:.1e}, energy {e_ok}"


def pin_two_kernels(seed=15):
    """Two Coulomb matrices: the second K against brute force over dense
    arrays (C V2 C contracted with D by einsum), the first unchanged, and
    K(V) + K(V2) = K(V + V2)."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    inp2, _, Vd2, _ = random_problem(sysm, seed + 100)     # same layout, another V
    K1, K2 = O.k_two_kernels(inp, inp2.V, route="4index")
    Kb = np.einsum("aij,ab,bkl,jl->ik", C3, Vd2, C3, Dd, optimize=True)
    Ks = O.k_two_kernels(inp, inp.V + inp2.V, route="eigen")[1]
    r = max(rel(K2, Kb), rel(K1, O.k_4index(inp)[0]), rel(K1 + K2, Ks))
    return r < TOL, f"{r:.1e}"


def _signed_problem(sysm, seed, cmag, vmag, dmag):
    """A random_problem whose entries are random signs times a magnitude that is
    constant per block: cmag[p], vmag[p] per canonical pair, dmag[A, B] (symmetric)
    per atom pair of D."""
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    nb, na, bo, ao = _offsets(sysm)
    lay = inp.layout
    C3, Vd, Dd = np.sign(C3), np.sign(Vd), np.sign(Dd)
    C, V = np.sign(inp.C), np.sign(inp.V)
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
        ma, mb = slice(ao[a], ao[a + 1]), slice(ao[b], ao[b + 1])
        for m in ((ma,) if a == b else (ma, mb)):
            C3[m, ia, ib] *= cmag[p]
            if a != b:
                C3[m, ib, ia] *= cmag[p]
        C[lay.c_off[p]:lay.c_off[p + 1]] *= cmag[p]
        Vd[ma, mb] *= vmag[p]
        if a != b:
            Vd[mb, ma] *= vmag[p]
        V[lay.v_off[p]:lay.v_off[p + 1]] *= vmag[p]
    atom = np.repeat(np.arange(sysm.n_atoms), nb)
    Dd = Dd * dmag[atom][:, atom]
    return synth.Inputs(sysm, lay, C, V, Dd.ravel().copy()), C3, Vd, Dd


def _term_maxima(sysm, lay, C3, Vd, Dd):
    """Per canonical pair (P, Q): the largest |C^mu_ij V_mu,nu C^nu_kl D_jl| over mu
    on P, nu on Q and the reverse, by brute force over the dense arrays (D on the
    screened atom pairs only, as the exchange contracts it)."""
    nb, na, bo, ao = _offsets(sysm)
    near = np.zeros((sysm.n_atoms, sysm.n_atoms), bool)
    for a, b in zip(lay.pair_a, lay.pair_b):
        near[a, b] = near[b, a] = True
    atom = np.repeat(np.arange(sysm.n_atoms), nb)
    Dm = np.where(near[atom][:, atom], np.abs(Dd), 0.0)
    amax = np.abs(C3).max(axis=1)                   # [mu, j]: max over i of |C^mu_ij|
    out = np.zeros(lay.n_pairs)
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        for P, Q in ((a, b), (b, a)):
            mP, mQ = slice(ao[P], ao[P + 1]), slice(ao[Q], ao[Q + 1])
            x = np.max(amax[mP][:, :, None] * Dm[None], axis=1)          # [mu, l]
            t = np.max(x[:, None, :] * amax[mQ][None, :, :], axis=2)     # [mu, nu]
            out[p] = max(out[p], float(np.max(np.abs(Vd[mP, mQ]) * t)))
    return out, near


def pin_norm_estimates(seed=20):
    """Maximum-norm estimates and screening.  (i) The per-pair maxima of C, V
    and D equal maxima over the dense arrays' blocks.  (ii) Every term C^mu_ij
    V_mu,nu C^nu_kl D_jl with mu on P and nu on Q (or the reverse) is at most
    the estimate of (P, Q), by brute force.  (iii) The estimate is attained
    when the blocks have constant magnitudes and either D or C is uniform (all
    atoms neighbours): then the largest term is max|V_PQ| tau_P tau_Q times the
    largest D entry reachable, exactly.  (iv) The screened V is zero exactly on
    the flagged pairs' dense blocks, and K of the screened V plus K of the V of
    only the flagged blocks is K (linearity)."""
    sysm = synth.water_cluster(2, seed)
    inp, C3, Vd, Dd = random_problem(sysm, seed)
    nb, na, bo, ao = _offsets(sysm)
    lay = inp.layout
    nrm = O.block_max_norms(inp)
    bad = 0
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
        mu = np.r_[ao[a]:ao[a + 1], ao[b]:ao[b + 1]] if a != b else np.r_[ao[a]:ao[a + 1]]
        want = [np.abs(C3[mu][:, ia, ib]).max(), np.abs(Vd[ao[a]:ao[a + 1], ao[b]:ao[b + 1]]).max(),
                max(np.abs(Dd[ia, ib]).max(), np.abs(Dd[ib, ia]).max())]
        bad += int(not np.array_equal(nrm[p], want))
    est = O.screening_estimates(inp, nrm)
    tmax, near = _term_maxima(sysm, lay, C3, Vd, Dd)
    worst = float(np.max(tmax / est))
    # constant-magnitude blocks: the estimate is attained
    rng = np.random.default_rng(seed + 1)
    nat, npr = sysm.n_atoms, lay.n_pairs
    sym = lambda m: np.triu(m) + np.triu(m, 1).T
    cases = ((rng.uniform(0.5, 2.0, npr), rng.uniform(0.5, 2.0, npr), np.ones((nat, nat))),
             (np.ones(npr), rng.uniform(0.5, 2.0, npr), sym(rng.uniform(0.5, 2.0, (nat, nat)))))
    tight = 0.0
    for cm, vm, dm in cases:
        ci, c3, vd, dd = _signed_problem(sysm, seed, cm, vm, dm)
        e = O.screening_estimates(ci, O.block_max_norms(ci))
        t, _ = _term_maxima(sysm, lay, c3, vd, dd)
        tight = max(tight, float(np.max(np.abs(t / e - 1.0))))
    flags = est < np.quantile(est, 0.4)
    scr = O.screened_coulomb(inp, flags)
    Vs = O.Blocks(scr).dense_V()
    blk_ok = True
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        ma, mb = slice(ao[a], ao[a + 1]), slice(ao[b], ao[b + 1])
        want = 0.0 * Vd[ma, mb] if flags[p] else Vd[ma, mb]
        blk_ok = blk_ok and np.array_equal(Vs[ma, mb], want) and np.array_equal(Vs[mb, ma], want.T)
    only = O.with_coulomb(inp, inp.V - scr.V)
    r = rel(O.k_eigen(scr) + O.k_eigen(only), O.k_eigen(inp))
    ok = (bad == 0 and worst <= 1.0 + 1e-12 and tight < 1e-12 and near.all()
          and 0 < flags.sum() < len(flags) and blk_ok and r < TOL)
    return ok, (f"norm mismatches {bad}, worst term / estimate {worst:.3f}, attained to {tight:.1e}, "
                f"blocks {blk_ok}, linearity {r:.1e}")


def _tiny_periodic(seed):
    lat = np.array([[3.0, 0.0, 0.0], [0.4, 3.2, 0.0], [0.2, -0.3, 3.4]])
    pos = np.array([[0.2, 0.3, 0.1], [2.6, 0.5, 0.4], [1.3, 2.9, 3.0], [1.5, 1.6, 1.7], [0.5, 2.8, 3.2]])
    return synth.System(np.array([0, 1, 1, 0, 1]), pos, 1.45, seed, lattice=lat,
                        basis_table=np.array([2, 1]), aux_table=np.array([3, 2]))


def pin_bloch(seed=22):
    """Bloch sums on a skewed cell whose pairs cross faces, edges and corners:
    (i) K(k) of the pair-block route equals the sum over Cartesian lattice
    vectors R = n L of e^{i k_c.R} X(R), k_c = k B with B = 2 pi inv(L)^T, over
    the pairs of the oracle's own periodic search; (ii) K(0) = X, K(k) is
    Hermitian and K(-k) = conj K(k); (iii) on a full 3x3x3 Gamma-centred grid
    density_from_k inverts D(k) = sum_R e^{-i k.R} D(R) exactly, also with a term
    at a second image of one pair added (the grid's phases are orthogonal);
    (iv) -1/4 (1/N_k) sum_k <K(k), D(k)> equals E_x of the folded matrices."""
    sysm = _tiny_periodic(seed)
    inp = synth.make_inputs(sysm)
    X = O.x_periodic(inp)
    n = X.shape[0]
    D = inp.D.reshape(n, n)
    lat = sysm.lattice
    Bm = 2 * np.pi * np.linalg.inv(lat).T
    nb, _, bo, _ = _offsets(sysm)
    pairs = O.periodic_pairs(sysm.pos, lat, sysm.r_cut)
    kpts = np.array([(0.25, -0.1, 0.4), (0.5, 0.5, 0.0), (-0.3, 0.2, 0.1)])
    Kk = O.bloch_sum(inp, X, kpts)
    worst = 0.0
    for k, K1 in zip(kpts, Kk):
        kc = k @ Bm
        K2 = np.zeros((n, n), dtype=complex)
        for a, b, nn in pairs:
            ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
            ph = np.exp(1j * float(kc @ (np.asarray(nn) @ lat)))
            K2[ia, ib] += ph * X[ia, ib]
            if a != b:
                K2[ib, ia] += np.conj(ph) * X[ib, ia]
        worst = max(worst, rel(K1, K2), rel(K1, K1.conj().T))
    K0 = O.bloch_sum(inp, X, [(0.0, 0.0, 0.0)])[0]
    Km = O.bloch_sum(inp, X, -kpts)
    worst = max(worst, rel(K0, X), max(rel(a, b.conj()) for a, b in zip(Km, Kk)))
    grid = np.array([(i / 3, j / 3, l / 3) for i in range(3) for j in range(3) for l in range(3)])
    rng = np.random.default_rng(seed)
    lay = inp.layout
    q = next(p for p in range(lay.n_pairs) if lay.pair_a[p] != lay.pair_b[p])
    a, b = int(lay.pair_a[q]), int(lay.pair_b[q])
    Z = rng.normal(size=(nb[a], nb[b]))
    n2 = np.asarray(lay.pair_img[q]) + np.array([1, 0, 0])
    Dk = []
    for k in grid:
        Dq = np.zeros((n, n), dtype=complex)
        for pa, pb, nn in zip(lay.pair_a, lay.pair_b, lay.pair_img):
            ia, ib = slice(bo[pa], bo[pa + 1]), slice(bo[pb], bo[pb + 1])
            ph = np.exp(-2j * np.pi * float(k @ nn))
            Dq[ia, ib] = ph * D[ia, ib]
            Dq[ib, ia] = np.conj(ph) * D[ib, ia]
        ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
        ph2 = np.exp(-2j * np.pi * float(k @ n2))
        Dq[ia, ib] += ph2 * Z
        Dq[ib, ia] += np.conj(ph2) * Z.T
        Dk.append(Dq)
    Dback = O.density_from_k(inp, Dk, grid)
    r_inv = rel(Dback, D)
    Kg = O.bloch_sum(inp, X, grid)
    e_k = -0.25 * np.real(sum(np.sum(K * Dq) for K, Dq in zip(Kg, Dk))) / len(grid)
    e_r = O.periodic_energy(X, D)
    ok = worst < TOL and r_inv < TOL and abs(e_k - e_r) <= TOL * abs(e_r)
    return ok, f"K(k) routes {worst:.1e}, D round trip {r_inv:.1e}, E {e_k:.12e} vs {e_r:.12e}"


def pin_periodic_unfolded(seed=17):
    """Periodic route against an explicit cluster of the home cell and its
    images (copied blocks, 4-index route), on a skewed cell whose atoms pair
    with images across faces, edges and corners."""
    sysm = _tiny_periodic(seed)
    inp = synth.make_inputs(sysm)
    imgs = np.abs(inp.layout.pair_img).sum(1)
    Xp, Xu = O.x_periodic(inp), O.x_unfolded(inp)
    r = rel(Xp, Xu)
    n = Xp.shape[0]
    e = abs(O.periodic_energy(Xp, inp.D.reshape(n, n)) - O.periodic_energy(Xu, inp.D.reshape(n, n)))
    ok = r < TOL and (imgs > 1).any() and e <= TOL * abs(O.periodic_energy(Xu, inp.D.reshape(n, n)))
    return ok, f"rel {r:.1e}, pairs with images {(imgs > 0).sum()} of {len(imgs)}"


def pin_periodic_vacuum(seed=18):
    """A cluster in a cell far larger than its reach: the periodic route gives
    the cluster's K on the pair pattern (and the same E_x)."""
    cl = synth.water_cluster(3, seed)
    vb = synth.System(cl.species, cl.pos, cl.r_cut, cl.seed, lattice=np.diag([60.0, 61.0, 62.0]))
    iv, ic = synth.make_inputs(vb), synth.make_inputs(cl)
    Xv, Kc = O.x_periodic(iv), O.k_4index(ic)[0]
    blk = O.Blocks(ic)
    mask = np.zeros((blk.nat, blk.nat), bool)
    mask[blk.pa, blk.pb] = mask[blk.pb, blk.pa] = True
    atom = np.repeat(np.arange(blk.nat), blk.nb)
    M = mask[atom][:, atom]
    r = rel(Xv, np.where(M, Kc, 0.0))
    Ev, Ec = O.periodic_energy(Xv, blk.D), O.exchange_energy(Kc, blk.D)
    return r < TOL and abs(Ev - Ec) <= TOL * abs(Ec), f"rel {r:.1e}, E {Ev:.10e} vs {Ec:.10e}"


def pin_periodic_supercell(seed=19):
    """E_x per cell is extensive: a 2x1x1 and a 1x1x2 supercell (copies keep
    their values) give twice the cell's E_x."""
    cell = synth.ice_box_periodic(1, 1, 1, seed, r_cut=3.4)
    ic = synth.make_inputs(cell)
    n = int(ic.layout.sys_nbas[0])
    Ec = O.periodic_energy(O.x_periodic(ic), ic.D.reshape(n, n))
    worst = 0.0
    for mult in ([2, 1, 1], [1, 1, 2]):
        sup = synth.supercell(cell, mult)
        isup = synth.make_inputs(sup)
        Es = O.periodic_energy(O.x_periodic(isup), isup.D.reshape(2 * n, 2 * n))
        worst = max(worst, abs(Es - 2 * Ec) / abs(Ec))
    return worst < TOL, f"E cell {Ec:.10e}, worst rel deviation of E(super)/2 {worst:.1e}"


ALL_PINS = {
    "block_route": pin_block_route,
    "screening": pin_screening,
    "rank1_4index": lambda: pin_rank1_closed_form("4index"),
    "rank1_rows": lambda: pin_rank1_closed_form("rows"),
    "brute_force": pin_brute_force,
    "invariants_4index": lambda: pin_invariants("4index"),
    "invariants_rows": lambda: pin_invariants("rows"),
    "invariants_eigen": lambda: pin_invariants("eigen"),
    "permutation_rows": lambda: pin_permutation("rows"),
    "permutation_4index": lambda: pin_permutation("4index"),
    "energy_direct": pin_energy_direct,
    "routes_agree": pin_routes_agree,
    "paper_regrouping": pin_paper_regrouping,
    "euler": pin_euler,
    "fd_params": pin_fd_params,
    "dD_minus_half_K": pin_dD_is_minus_half_K,
    "force_invariants": pin_force_invariants,
    "fd_forces": pin_fd_forces,
    "spin": pin_spin,
    "two_kernels": pin_two_kernels,
    "periodic_unfolded": pin_periodic_unfolded,
    "periodic_vacuum": pin_periodic_vacuum,
    "periodic_supercell": pin_periodic_supercell,
    "norm_estimates": pin_norm_estimates,
    "spin_gradients": pin_spin_gradients,
    "bloch": pin_bloch,
}
