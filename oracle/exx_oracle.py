"""Plain FP64 CPU oracle for the RI-LVL real-space exchange matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this module; only the tests, the package's smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the GPU library: it reads the inputs
written by the seeded generator (``synth``) and recomputes everything,
including the atom-pair screening, on its own.

What is computed (non-periodic case, i.e. only the lattice vector R = 0 of the
paper's real-space exchange equation, Sec. "Description of the real-space
formalism", Eq. (realspace_exchange)):

    K_ik = sum_{j,l} sum_{mu,nu} C^mu_ij V_{mu nu} C^nu_kl D_jl
    E_x  = -1/4 sum_{i,k} K_ik D_ik

with the RI-LVL pair restriction (same section): C^mu_ij = 0 unless the
auxiliary function mu sits on the atom of i or on the atom of j.  C^mu is
symmetric in (i, j) (it expands the product phi_i phi_j).  The paper does not
write E_x; the energy convention is the usual exchange energy for a
closed-shell density matrix scaled as stated above.

Routes (three independent evaluations of the same definition):

* ``k_4index``  forms the 4-index tensor (ij|kl) = sum C V C in i-slabs and
  contracts it with D; it also returns E_x contracted directly from (ij|kl).
* ``k_eigen``   uses D = sum_m lambda_m v_m v_m^T, so that
  K = sum_m lambda_m U_m V U_m^T with U_m[:, mu] = C^mu v_m.
* ``k_rows``    evaluates whole rows K[i, :] from the definition with the
  structural zeros of C and V skipped; usable at any system size.
* ``k_atom_rows`` (the block route) evaluates the same rows for all basis
  functions of one atom at once, so that every step is a matrix product over
  structural blocks; it is the route the CPU baseline times.

Collinear spin (``k_spin``, ``spin_exchange_energy``): the spin index of
Eq. (realspace_exchange) only selects the density matrix, so each spin's K^s
is the definition above with D^s.  The paper does not write the spin energy
either; the reading used is E_x = -1/2 sum_s sum_ik K^s_ik D^s_ik, which for
D^0 = D^1 = D/2 is the closed-shell E_x above.

Two Coulomb kernels (``k_two_kernels``): one exchange matrix per Coulomb
matrix, K^a = sum C V^a C D, each by the same definition (Sec.
"Introduction" motivates computing both in one call).

Gradients (``gradients``) follow from E_x being quadratic in C and D and
linear in V:  dE/dD = -1/2 K,  dE/dC^mu = -1/2 sum_nu V_{mu nu} D C^nu D,
dE/dV_{mu nu} = -1/4 tr(C^mu D C^nu D); per stored layout entry the mirrored
copies are summed (off-site C and V blocks are each stored once for both
orientations).  Forces use the synthetic analytic dependence of C and V on
the atom positions (C ~ exp(-r/1.5), V ~ exp(-r^2/8)), with D held fixed.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ----------------------------------------------------------------------------
# screening and index bookkeeping (independent of the generator's own code)


def screened_pairs(pos, r_cut, sys_off):
    """Atom pairs (A <= B, same system) with squared distance <= r_cut^2.

    The squared distance is (dx*dx + dy*dy) + dz*dz in float64.  Returned in
    lexicographic order, which is the storage order of the C and V blocks."""
    out_a, out_b = [], []
    rc2 = r_cut * r_cut
    for s in range(len(sys_off) - 1):
        lo, hi = int(sys_off[s]), int(sys_off[s + 1])
        P = pos[lo:hi]
        dx = P[:, None, 0] - P[None, :, 0]
        dy = P[:, None, 1] - P[None, :, 1]
        dz = P[:, None, 2] - P[None, :, 2]
        r2 = (dx * dx + dy * dy) + dz * dz
        a, b = np.nonzero(np.triu(r2 <= rc2))
        out_a.append(a + lo)
        out_b.append(b + lo)
    return np.concatenate(out_a).astype(np.int32), np.concatenate(out_b).astype(np.int32)


class Blocks:
    """Read access to the C / V / D inputs of one system (atoms lo..hi-1)."""

    def __init__(self, inputs, s=0):
        sysm, lay = inputs.system, inputs.layout
        self.lo, self.hi = int(sysm.sys_off[s]), int(sysm.sys_off[s + 1])
        self.nat = self.hi - self.lo
        sp = sysm.species[self.lo:self.hi]
        self.nb = sysm.basis_table[sp].astype(np.int64)   # species tables: input metadata
        self.na = sysm.aux_table[sp].astype(np.int64)
        self.bo = np.concatenate([[0], np.cumsum(self.nb)])
        self.ao = np.concatenate([[0], np.cumsum(self.na)])
        self.n, self.naux = int(self.bo[-1]), int(self.ao[-1])
        self.pos = sysm.pos[self.lo:self.hi]
        self.r_cut = sysm.r_cut
        pa, pb = screened_pairs(sysm.pos, sysm.r_cut, sysm.sys_off)
        if not (np.array_equal(pa, lay.pair_a) and np.array_equal(pb, lay.pair_b)):
            raise ValueError("input layout does not match the oracle's screening")
        sel = (pa >= self.lo) & (pa < self.hi)
        self.pidx = np.nonzero(sel)[0]
        self.pa, self.pb = pa[sel] - self.lo, pb[sel] - self.lo
        self.C, self.V = inputs.C, inputs.V
        self.c_off, self.v_off = lay.c_off, lay.v_off
        d0 = int(lay.sys_bas_off[s])
        self.D = inputs.D[d0:d0 + self.n * self.n].reshape(self.n, self.n)
        self.pair_of = {}
        for q, (a, b) in enumerate(zip(self.pa, self.pb)):
            self.pair_of[(int(a), int(b))] = q
        self.nbrs = [[] for _ in range(self.nat)]
        for a, b in zip(self.pa, self.pb):
            self.nbrs[a].append(int(b))
            if a != b:
                self.nbrs[b].append(int(a))
        for lst in self.nbrs:
            lst.sort()

    def c_block(self, q):
        p = self.pidx[q]
        a, b = self.pa[q], self.pb[q]
        blk = self.C[self.c_off[p]:self.c_off[p + 1]]
        if a == b:
            return blk.reshape(self.na[a], self.nb[a], self.nb[a])
        return blk.reshape(self.na[a] + self.na[b], self.nb[a], self.nb[b])

    def v_block(self, q):
        p = self.pidx[q]
        a, b = self.pa[q], self.pb[q]
        return self.V[self.v_off[p]:self.v_off[p + 1]].reshape(self.na[a], self.na[b])

    # dense forms (small systems only)
    def dense_C(self):
        """C3[mu, i, j] over the whole system (n_aux x n x n)."""
        C3 = np.zeros((self.naux, self.n, self.n))
        for q, (a, b) in enumerate(zip(self.pa, self.pb)):
            blk = self.c_block(q)
            ia, ib = slice(self.bo[a], self.bo[a + 1]), slice(self.bo[b], self.bo[b + 1])
            if a == b:
                C3[self.ao[a]:self.ao[a + 1], ia, ia] = blk
                continue
            for owner, part in ((a, blk[:self.na[a]]), (b, blk[self.na[a]:])):
                mu = slice(self.ao[owner], self.ao[owner + 1])
                C3[mu, ia, ib] = part
                C3[mu, ib, ia] = part.transpose(0, 2, 1)
        return C3

    def dense_V(self):
        Vd = np.zeros((self.naux, self.naux))
        for q, (a, b) in enumerate(zip(self.pa, self.pb)):
            blk = self.v_block(q)
            ma, mb = slice(self.ao[a], self.ao[a + 1]), slice(self.ao[b], self.ao[b + 1])
            Vd[ma, mb] = blk
            if a != b:
                Vd[mb, ma] = blk.T
        return Vd


def exchange_energy(K, D):
    """E_x = -1/4 sum_ik K_ik D_ik."""
    return -0.25 * float(np.sum(K * D))


# ----------------------------------------------------------------------------
# route 1: the 4-index tensor


def k_4index(inputs, s=0, slab=8):
    """K from (ij|kl) = sum_{mu nu} C^mu_ij V_{mu nu} C^nu_kl, in i-slabs.

    Returns (K, E_from_K, E_direct) where E_direct contracts (ij|kl) with
    D_ik D_jl without forming K (k summed first, then j and l)."""
    blk = Blocks(inputs, s)
    n = blk.n
    B = blk.dense_C().reshape(blk.naux, n * n)       # B[mu, (k,l)]
    VB = blk.dense_V() @ B                            # (V B)[mu, (k,l)]
    D = blk.D
    K = np.zeros((n, n))
    e_direct = 0.0
    for i0 in range(0, n, slab):
        i1 = min(n, i0 + slab)
        rows = B.reshape(blk.naux, n, n)[:, i0:i1, :].reshape(blk.naux, -1)
        eri = (rows.T @ VB).reshape(i1 - i0, n, n, n)  # (ij|kl), i in slab
        K[i0:i1] = np.einsum("ijkl,jl->ik", eri, D, optimize=True)
        t = np.einsum("ijkl,ik->ijl", eri, D[i0:i1], optimize=True)
        e_direct += float(np.sum(t * D[None, :, :]))
    return K, exchange_energy(K, D), -0.25 * e_direct


# ----------------------------------------------------------------------------
# route 2: eigen-decomposition of D


def k_eigen(inputs, s=0):
    blk = Blocks(inputs, s)
    n = blk.n
    lam, vec = np.linalg.eigh(blk.D)
    C3 = blk.dense_C()
    U = (C3.reshape(-1, n) @ vec).reshape(blk.naux, n, n)      # U[mu, i, m]
    W = (blk.dense_V() @ U.reshape(blk.naux, -1)).reshape(blk.naux, n, n)
    Ul = U * lam[None, None, :]
    K = np.einsum("aim,akm->ik", Ul, W, optimize=True)
    return K


# ----------------------------------------------------------------------------
# route 3: rows of K from the definition, structural zeros skipped


def k_rows(inputs, rows, s=0, blk=None):
    """K[rows, :] for rows given as basis indices local to system s.

    For row i:  u^mu = C^mu[i, :];  t^mu = D u^mu;  y^nu = sum_mu V_{nu mu} t^mu;
    K[i, k] = sum_nu sum_l C^nu_kl y^nu_l."""
    if blk is None:
        blk = Blocks(inputs, s)
    atom_of = np.repeat(np.arange(blk.nat), blk.nb)
    D = blk.D
    out = np.zeros((len(rows), blk.n))
    for r, i in enumerate(rows):
        I = int(atom_of[i])
        ii = i - blk.bo[I]
        # u^mu restricted to the aux functions whose C^mu has a nonzero row i
        mu_idx, u_rows = [], []
        for J in blk.nbrs[I]:
            a, b = (I, J) if I <= J else (J, I)
            cb = blk.c_block(blk.pair_of[(a, b)])
            if I == J:
                u = np.zeros((blk.na[I], blk.n))
                u[:, blk.bo[I]:blk.bo[I + 1]] = cb[:, ii, :]
                mu_idx.append(np.arange(blk.ao[I], blk.ao[I + 1]))
                u_rows.append(u)
                continue
            if I < J:   # block rows: basis of I, cols: basis of J
                rowpart = cb[:, ii, :]                     # [m, j in J]
            else:       # block rows: basis of J, cols: basis of I
                rowpart = cb[:, :, ii]
            na_a = blk.na[a]
            for owner, part in ((a, rowpart[:na_a]), (b, rowpart[na_a:])):
                u = np.zeros((blk.na[owner], blk.n))
                u[:, blk.bo[J]:blk.bo[J + 1]] = part
                mu_idx.append(np.arange(blk.ao[owner], blk.ao[owner + 1]))
                u_rows.append(u)
        mu_idx = np.concatenate(mu_idx)
        Ufull = np.concatenate(u_rows)
        # several blocks contribute to the same mu (mu on I appears for every J)
        uniq, inv = np.unique(mu_idx, return_inverse=True)
        Um = np.zeros((len(uniq), blk.n))
        np.add.at(Um, inv, Ufull)
        t = Um @ D                                         # t^mu (D symmetric)
        # y^nu for every nu coupled by V to some mu in uniq
        aux_atom = np.repeat(np.arange(blk.nat), blk.na)
        mu_atoms = np.unique(aux_atom[uniq])
        y = {}
        for P in mu_atoms:
            selP = aux_atom[uniq] == P
            tP = t[selP]
            locP = uniq[selP] - blk.ao[P]
            for Q in blk.nbrs[P]:
                a, b = (P, Q) if P <= Q else (Q, P)
                vb = blk.v_block(blk.pair_of[(a, b)])
                VPQ = vb if P <= Q else vb.T                 # [mu on P, nu on Q]
                contrib = VPQ[locP].T @ tP                   # [nu on Q, n]
                y[Q] = y.get(Q, 0.0) + contrib
        # K[i, k] = sum_nu (C^nu y^nu)[k]
        Ki = np.zeros(blk.n)
        for Q, yQ in y.items():
            for J in blk.nbrs[Q]:
                a, b = (Q, J) if Q <= J else (J, Q)
                cb = blk.c_block(blk.pair_of[(a, b)])
                sq, sj = slice(blk.bo[Q], blk.bo[Q + 1]), slice(blk.bo[J], blk.bo[J + 1])
                if Q == J:
                    Ki[sq] += np.einsum("nkl,nl->k", cb, yQ[:, sq])
                    continue
                part = cb[:blk.na[a]] if Q == a else cb[blk.na[a]:]
                if Q < J:   # part[nu, k in Q, l in J]
                    Ki[sq] += np.einsum("nkl,nl->k", part, yQ[:, sj])
                    Ki[sj] += np.einsum("nkl,nk->l", part, yQ[:, sq])
                else:       # part[nu, k in J, l in Q]
                    Ki[sj] += np.einsum("nkl,nl->k", part, yQ[:, sq])
                    Ki[sq] += np.einsum("nkl,nk->l", part, yQ[:, sj])
        out[r] = Ki
    return out


def _c_row_parts(blk, I, J):
    """Parts of C^mu restricted to rows on atom I and columns on atom J, for
    every mu whose C^mu has such a block: a list of (aux atom P, array
    [n_aux(P), n_basis(I), n_basis(J)])."""
    a, b = (I, J) if I <= J else (J, I)
    cb = blk.c_block(blk.pair_of[(a, b)])
    if I == J:
        return [(I, cb)]
    na_a = blk.na[a]
    out = []
    for owner, part in ((a, cb[:na_a]), (b, cb[na_a:])):
        out.append((owner, part if I < J else part.transpose(0, 2, 1)))
    return out


def k_atom_rows(inputs, atoms, s=0, blk=None):
    """K[rows of the given atoms, :] of system s (rows in the order of atoms).

    The definition K_ik = sum_mu sum_nu V_{mu nu} (C^mu D C^nu)_ik taken for
    all rows i of one atom I at once, each step a matrix product over
    structural blocks only:
      U^mu[i, j]  = C^mu_ij        (mu on I or on a neighbour of I; j near I)
      T^mu        = U^mu D         (on the columns the C^nu below can reach)
      Y^nu        = sum_mu V_{nu mu} T^mu      (nu on a neighbour Q of mu's atom)
      K[i, k]     = sum_nu sum_l C^nu_kl Y^nu[i, l]."""
    if blk is None:
        blk = Blocks(inputs, s)
    D = blk.D
    cols_of = lambda atoms_: np.concatenate([np.arange(blk.bo[J], blk.bo[J + 1]) for J in atoms_])
    c1 = [cols_of(blk.nbrs[A]) for A in range(blk.nat)]                       # basis of N[A]
    n2 = [sorted(set(L for J in blk.nbrs[A] for L in blk.nbrs[J])) for A in range(blk.nat)]
    c2 = [cols_of(x) for x in n2]                                              # basis of N2[A]
    out = []
    for I in atoms:
        I = int(I)
        bI = int(blk.nb[I])
        loc1 = {}
        c = 0
        for J in blk.nbrs[I]:
            loc1[J] = c
            c += blk.nb[J]
        U = {}
        for J in blk.nbrs[I]:
            for P, part in _c_row_parts(blk, I, J):
                if P not in U:
                    U[P] = np.zeros((blk.na[P], bI, len(c1[I])))
                U[P][:, :, loc1[J]:loc1[J] + blk.nb[J]] += part
        Y = {}
        DI = D[c1[I]]
        for P, UP in U.items():
            pos2 = {int(x): k for k, x in enumerate(c2[P])}
            TP = (UP.reshape(-1, len(c1[I])) @ DI[:, c2[P]]).reshape(blk.na[P], bI, len(c2[P]))
            for Q in blk.nbrs[P]:
                idx = np.array([pos2[int(x)] for x in c1[Q]])
                a, b = (P, Q) if P <= Q else (Q, P)
                vb = blk.v_block(blk.pair_of[(a, b)])
                VPQ = vb if P <= Q else vb.T                   # [mu on P, nu on Q]
                contrib = (VPQ.T @ TP[:, :, idx].reshape(blk.na[P], -1)).reshape(blk.na[Q], bI, len(idx))
                if Q in Y:
                    Y[Q] += contrib
                else:
                    Y[Q] = contrib
        KI = np.zeros((bI, blk.n))
        for Q, YQ in Y.items():
            pos = {}
            c = 0
            for J in blk.nbrs[Q]:
                pos[J] = c
                c += blk.nb[J]
            for J in blk.nbrs[Q]:
                # C^nu (nu on Q) on rows of Q and columns of J, and its mirror
                for P, part in _c_row_parts(blk, Q, J):
                    if P != Q:
                        continue
                    sq, sj = slice(blk.bo[Q], blk.bo[Q + 1]), slice(blk.bo[J], blk.bo[J + 1])
                    yJ = YQ[:, :, pos[J]:pos[J] + blk.nb[J]]          # [nu, i, l on J]
                    KI[:, sq] += np.einsum("nkl,nil->ik", part, yJ, optimize=True)
                    if J != Q:
                        yQ = YQ[:, :, pos[Q]:pos[Q] + blk.nb[Q]]      # [nu, i, l on Q]
                        KI[:, sj] += np.einsum("nkl,nik->il", part, yQ, optimize=True)
        out.append(KI)
    return np.concatenate(out) if out else np.zeros((0, blk.n))


def k_full_rows(inputs, s=0):
    """The whole K of system s via the row route (moderate sizes only)."""
    blk = Blocks(inputs, s)
    return k_rows(inputs, np.arange(blk.n), s, blk)


# ----------------------------------------------------------------------------
# collinear spin


def with_density(inputs, D):
    """A shallow copy of ``inputs`` whose (flat) density matrix is D."""
    out = copy.copy(inputs)
    out.D = np.asarray(D, dtype=np.float64)
    return out


def k_spin(inputs, D_spin, s=0, route="eigen"):
    """[K^0, K^1] of system s: the definition evaluated once per spin density
    matrix (D_spin: two flat arrays in the layout of inputs.D)."""
    f = {"eigen": k_eigen, "rows": k_full_rows, "4index": lambda i, s: k_4index(i, s)[0]}[route]
    return [f(with_density(inputs, D), s) for D in D_spin]


def with_coulomb(inputs, V):
    """A shallow copy of ``inputs`` whose (flat, pair-block) Coulomb matrix is V."""
    out = copy.copy(inputs)
    out.V = np.asarray(V, dtype=np.float64)
    return out


def k_two_kernels(inputs, V2, s=0, route="eigen"):
    """[K(V), K(V2)] of system s for a second Coulomb matrix V2 in the layout of inputs.V."""
    f = {"eigen": k_eigen, "rows": k_full_rows, "4index": lambda i, s: k_4index(i, s)[0]}[route]
    return [f(inputs, s), f(with_coulomb(inputs, V2), s)]


def spin_exchange_energy(K_spin, D_spin):
    """E_x = -1/2 sum_s sum_ik K^s_ik D^s_ik (K^s and D^s dense, one system)."""
    return -0.5 * sum(float(np.sum(K * D)) for K, D in zip(K_spin, D_spin))


# ----------------------------------------------------------------------------
# maximum-norm estimates and screening (Sec. "Evaluation of the EXX matrix in
# real space": whether a product of temporaries is formed is decided from
# estimates of the maximum norms of the arrays involved, e.g. D and C)


def block_max_norms(inputs):
    """Per canonical pair p = (A, B): [max|C block|, max|V block|, max|D|] with
    the C and V blocks as stored (C: every aux function of A and of B, rows on
    A, columns on B; V: aux of A by aux of B) and D over both the (A, B) and
    the (B, A) blocks of the pair's system.  Maxima of absolute values are
    exact in any order."""
    sysm, lay = inputs.system, inputs.layout
    nb = sysm.basis_table[sysm.species].astype(np.int64)
    sys_of = np.zeros(sysm.n_atoms, dtype=np.int64)
    bo = np.zeros(sysm.n_atoms, dtype=np.int64)
    for s in range(sysm.n_systems):
        lo, hi = int(sysm.sys_off[s]), int(sysm.sys_off[s + 1])
        sys_of[lo:hi] = s
        bo[lo:hi] = np.concatenate([[0], np.cumsum(nb[lo:hi])[:-1]])
    out = np.zeros((lay.n_pairs, 3))
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        out[p, 0] = np.abs(inputs.C[lay.c_off[p]:lay.c_off[p + 1]]).max()
        out[p, 1] = np.abs(inputs.V[lay.v_off[p]:lay.v_off[p + 1]]).max()
        s = sys_of[a]
        n = int(lay.sys_nbas[s])
        Ds = inputs.D[lay.sys_bas_off[s]:lay.sys_bas_off[s] + n * n].reshape(n, n)
        ia, ib = slice(bo[a], bo[a] + nb[a]), slice(bo[b], bo[b] + nb[b])
        out[p, 2] = max(np.abs(Ds[ia, ib]).max(), np.abs(Ds[ib, ia]).max())
    return out


def screening_estimates(inputs, norms):
    """The maximum-norm estimate of the terms C^mu_ij V_{mu nu} C^nu_kl D_jl that
    run through the V block of each canonical pair (P, Q) (mu on P, nu on Q):

        est_PQ = ((max|V_PQ| * tau_P) * tau_Q) * min(sigma_P, sigma_Q)

    tau_A = the largest max|C| of a pair block with A (it bounds every C^mu with
    mu on A); rho_A = the largest max|D| of a pair with A; sigma_A = the largest
    rho_J over the neighbours J of A (j of C^mu_ij with mu on P lies on an atom of
    N[P], l on an atom of N[Q]).  Every such term has modulus at most est_PQ."""
    lay = inputs.layout
    nat = inputs.system.n_atoms
    tau = np.zeros(nat)
    rho = np.zeros(nat)
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        for x in (a, b):
            tau[x] = max(tau[x], norms[p, 0])
            rho[x] = max(rho[x], norms[p, 2])
    sigma = np.zeros(nat)
    for a, b in zip(lay.pair_a, lay.pair_b):
        sigma[a] = max(sigma[a], rho[b])
        sigma[b] = max(sigma[b], rho[a])
    est = np.empty(lay.n_pairs)
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        est[p] = ((norms[p, 1] * tau[a]) * tau[b]) * min(sigma[a], sigma[b])
    return est


def screened_coulomb(inputs, flags):
    """A copy of ``inputs`` with the V blocks of the flagged pairs set to zero:
    the result of a build that skips every product through those blocks."""
    V = inputs.V.copy()
    lay = inputs.layout
    for p in np.nonzero(flags)[0]:
        V[lay.v_off[p]:lay.v_off[p + 1]] = 0.0
    return with_coulomb(inputs, V)


# ----------------------------------------------------------------------------
# gradients and forces (dense; small systems)


def gradients(inputs, s=0):
    """dE/dC, dE/dV (stored layouts, entries of system s only), dE/dD (dense).

    Returns dict with 'E', 'K', 'dC' (flat, layout of C), 'dV', 'dD',
    'sC' and 'sV' (per stored pair q of the system: <dE/dblock, block>)."""
    blk = Blocks(inputs, s)
    n = blk.n
    C3 = blk.dense_C()
    Vd = blk.dense_V()
    D = blk.D
    DCD = np.einsum("ab,mbc,cd->mad", D, C3, D, optimize=True)     # D C^nu D
    G = -0.5 * (Vd @ DCD.reshape(blk.naux, -1)).reshape(blk.naux, n, n)
    Q = np.einsum("mab,bc->mac", C3, D, optimize=True)              # C^mu D
    tau = Q.reshape(blk.naux, -1) @ Q.transpose(0, 2, 1).reshape(blk.naux, -1).T
    lam, vec = np.linalg.eigh(D)
    K = k_eigen(inputs, s)
    E = exchange_energy(K, D)
    dC = np.zeros_like(inputs.C)
    dV = np.zeros_like(inputs.V)
    sC = np.zeros(len(blk.pa))
    sV = np.zeros(len(blk.pa))
    for q, (a, b) in enumerate(zip(blk.pa, blk.pb)):
        p = blk.pidx[q]
        ia, ib = slice(blk.bo[a], blk.bo[a + 1]), slice(blk.bo[b], blk.bo[b + 1])
        ma, mb = slice(blk.ao[a], blk.ao[a + 1]), slice(blk.ao[b], blk.ao[b + 1])
        if a == b:
            g = G[ma, ia, ia]
            vg = -0.25 * tau[ma, ma]
        else:
            g = np.concatenate([G[ma, ia, ib], G[mb, ia, ib]]) * 2.0
            vg = -0.5 * tau[ma, mb]
        dC[blk.c_off[p]:blk.c_off[p + 1]] = g.ravel()
        dV[blk.v_off[p]:blk.v_off[p + 1]] = vg.ravel()
        sC[q] = float(np.sum(g * blk.c_block(q)))
        sV[q] = float(np.sum(vg * blk.v_block(q)))
    return dict(E=E, K=K, dC=dC, dV=dV, dD=-0.5 * K, sC=sC, sV=sV, blk=blk)


def spin_gradients(inputs, D_spin, s=0):
    """Gradients of the collinear-spin E_x = -1/2 sum_s sum_ik K^s_ik D^s_ik.

    Each spin's term is twice the one-density energy -1/4 <K(D^s), D^s>, so dC,
    dV, sC and sV are twice the sums over the spins of the one-density
    gradients, and dE/dD^s = -K^s (twice the one-density -1/2 K(D^s))."""
    parts = [gradients(with_density(inputs, D), s) for D in D_spin]
    out = {k: 2.0 * (parts[0][k] + parts[1][k]) for k in ("E", "dC", "dV", "sC", "sV")}
    out["K"] = [p["K"] for p in parts]
    out["dD"] = [2.0 * p["dD"] for p in parts]
    out["blk"] = parts[0]["blk"]
    return out


def forces(inputs, grads, c_decay=1.5, v_2s2=8.0):
    """-dE/dR_A through C_AB ~ exp(-r/c_decay) and V_AB ~ exp(-r^2/v_2s2).

    On-site blocks do not depend on positions; D is held fixed."""
    blk = grads["blk"]
    F = np.zeros((blk.nat, 3))
    for q, (a, b) in enumerate(zip(blk.pa, blk.pb)):
        if a == b:
            continue
        d = blk.pos[a] - blk.pos[b]
        r = math.sqrt(float(d @ d))
        # dE/dR_a = sC * (-1/c_decay) d/r + sV * (-2/v_2s2) d
        g = grads["sC"][q] * (-1.0 / c_decay) * d / r + grads["sV"][q] * (-2.0 / v_2s2) * d
        F[a] -= g
        F[b] += g
    return F


# ----------------------------------------------------------------------------
# periodic systems (lattice vectors R != 0 of Eq. (realspace_exchange))
#
# Atoms of the home cell carry functions phi(r - R_A); their images in cell n
# are phi(r - R_A - n.L).  The real-space exchange matrix X_ik(n) couples a
# function i in the home cell with a function k in cell n; by translation
# symmetry every block depends on relative images only, so the C, V and D
# blocks of a pair of home-cell atoms (A, B) serve every pair of their images
# with the same relative image.  With the cutoff below half the cell width a
# pair of atoms has at most one image within the cutoff, and X is returned on
# that pattern: the dense home-cell block (A, B) holds X_AB(n_AB) for the image
# n_AB of B within the cutoff of A (zero if there is none).  D is given the same
# way.  E_x = -1/4 sum over those blocks of X o D, the energy per cell.


def _shift(lat, n):
    return np.array([(n[0] * lat[0, c] + n[1] * lat[1, c]) + n[2] * lat[2, c] for c in range(3)])


def periodic_pairs(pos, lat, r_cut):
    """Canonical pairs (A <= B) with the image n of B within r_cut of A, in
    lexicographic order of (A, B): squared distance ((x_B + s_x) - x_A)^2 + ...
    summed as (dx*dx + dy*dy) + dz*dz, s the image shift."""
    rc2 = r_cut * r_cut
    imgs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    shifts = [_shift(lat, n) for n in imgs]
    out = []
    for a in range(len(pos)):
        found = {}
        for n, sft in zip(imgs, shifts):
            b = np.arange(a, len(pos))
            dx = (pos[b, 0] + sft[0]) - pos[a, 0]
            dy = (pos[b, 1] + sft[1]) - pos[a, 1]
            dz = (pos[b, 2] + sft[2]) - pos[a, 2]
            for bb in b[(dx * dx + dy * dy) + dz * dz <= rc2]:
                if bb == a and n != (0, 0, 0):
                    continue
                found[int(bb)] = n
        out.extend((a, b, found[b]) for b in sorted(found))
    return out


class PBlocks:
    """Read access to the C / V / D inputs of a periodic system, blocks keyed
    by atom pairs and relative lattice images."""

    def __init__(self, inputs):
        sysm, lay = inputs.system, inputs.layout
        self.lat = sysm.lattice
        self.nat = sysm.n_atoms
        self.nb = sysm.basis_table[sysm.species].astype(np.int64)
        self.na = sysm.aux_table[sysm.species].astype(np.int64)
        self.bo = np.concatenate([[0], np.cumsum(self.nb)])
        self.n = int(self.bo[-1])
        pairs = periodic_pairs(sysm.pos, self.lat, sysm.r_cut)
        mine = [(int(a), int(b), tuple(int(x) for x in n)) for a, b, n in zip(lay.pair_a, lay.pair_b, lay.pair_img)]
        if mine != pairs:
            raise ValueError("input layout does not match the oracle's periodic screening")
        self.C, self.V = inputs.C, inputs.V
        self.c_off, self.v_off = lay.c_off, lay.v_off
        self.D = inputs.D[:self.n * self.n].reshape(self.n, self.n)
        self.pair = {}                                  # (A, B, n) -> canonical index, A <= B
        self.nbrs = [[] for _ in range(self.nat)]       # entries (B, n): B + n within r_cut of A
        for q, (a, b, n) in enumerate(pairs):
            self.pair[(a, b, n)] = q
            self.nbrs[a].append((b, n))
            if a != b:
                self.nbrs[b].append((a, tuple(-x for x in n)))
        for lst in self.nbrs:
            lst.sort()
        self.img_of = [dict(lst) for lst in self.nbrs]  # B -> its image within r_cut of A

    def _canon(self, A, B, n):
        """(canonical pair index, whether (A, B) is stored as (B, A))."""
        if A < B or (A == B and n == (0, 0, 0)):
            return self.pair.get((A, B, n)), False
        return self.pair.get((B, A, tuple(-x for x in n))), True

    def c_rows(self, I, J, m):
        """C^mu restricted to rows on I (home cell) and columns on J + m, for
        every mu with such a block: list of ((aux atom, image), [a, b_I, b_J])."""
        q, flip = self._canon(I, J, m)
        if q is None:
            return []
        blk = self.C[self.c_off[q]:self.c_off[q + 1]]
        if I == J:
            return [((I, (0, 0, 0)), blk.reshape(self.na[I], self.nb[I], self.nb[I]))]
        if not flip:    # pair (I, J + m): rows aux of I, then aux of J + m
            blk = blk.reshape(self.na[I] + self.na[J], self.nb[I], self.nb[J])
            return [((I, (0, 0, 0)), blk[:self.na[I]]), ((J, m), blk[self.na[I]:])]
        # stored as (J, I - m): aux of J first; translated by m it is the pair (J + m, I)
        blk = blk.reshape(self.na[J] + self.na[I], self.nb[J], self.nb[I])
        return [((J, m), blk[:self.na[J]].transpose(0, 2, 1)), ((I, (0, 0, 0)), blk[self.na[J]:].transpose(0, 2, 1))]

    def v(self, P, p, Q, q):
        """V_{mu nu}, mu on P + p, nu on Q + q (None beyond the cutoff)."""
        r = tuple(b - a for a, b in zip(p, q))
        k, flip = self._canon(P, Q, r)
        if k is None:
            return None
        blk = self.V[self.v_off[k]:self.v_off[k + 1]]
        return blk.reshape(self.na[Q], self.na[P]).T if flip else blk.reshape(self.na[P], self.na[Q])

    def d(self, J, m, L, b):
        """D between J + m and L + b (zeros beyond the cutoff)."""
        r = tuple(y - x for x, y in zip(m, b))
        if self.img_of[J].get(L) != r:
            return np.zeros((self.nb[J], self.nb[L]))
        return self.D[self.bo[J]:self.bo[J + 1], self.bo[L]:self.bo[L + 1]]

    def entries(self, A, a):
        """The neighbour entries of atom A placed at image a: (B, a + n)."""
        return [(B, tuple(x + y for x, y in zip(a, n))) for B, n in self.nbrs[A]]


def _add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def _sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def x_atom_rows_periodic(inputs, atoms, pb=None):
    """Rows of the folded X (see above) for all basis functions of the given
    home-cell atoms: the definition X_ik(n) = sum_mu sum_nu V_{mu nu}
    (C^mu D C^nu)_{i, k(n)} over all images, taken atom by atom as in
    k_atom_rows with every atom labelled by its image, and kept on the pattern."""
    if pb is None:
        pb = PBlocks(inputs)
    zero = (0, 0, 0)
    nat = pb.nat
    # image of B within r_cut of A as a dense table (codes; -1: none), for the D blocks
    code = lambda n: (n[0] + 8) + 16 * (n[1] + 8) + 256 * (n[2] + 8)
    if not hasattr(pb, "_img_tab"):
        tab = np.full((nat, nat), -1, dtype=np.int64)
        for A in range(nat):
            for B, n in pb.nbrs[A]:
                tab[A, B] = code(n)
        pb._img_tab = tab
    tab = pb._img_tab

    def d_rows_cols(rows, cols):
        """D between the row entries (J, m) and column entries (L, b): the folded
        D block of (J, L) where n_JL = b - m, zero elsewhere."""
        rj = np.array([J for J, _ in rows])
        rm = np.array([code(m) for _, m in rows])
        cl = np.array([L for L, _ in cols])
        cb = np.array([code(b) for _, b in cols])
        ok = (tab[np.ix_(rj, cl)] >= 0) & (tab[np.ix_(rj, cl)] + rm[:, None] - code(zero) == cb[None, :])
        rb = np.concatenate([np.arange(pb.bo[J], pb.bo[J + 1]) for J in rj])
        cbas = np.concatenate([np.arange(pb.bo[L], pb.bo[L + 1]) for L in cl])
        okb = np.repeat(np.repeat(ok, pb.nb[rj], axis=0), pb.nb[cl], axis=1)
        return np.where(okb, pb.D[np.ix_(rb, cbas)], 0.0)

    out = []
    for I in atoms:
        I = int(I)
        bI = int(pb.nb[I])
        ent1 = pb.entries(I, zero)                               # N[I]
        loc1, c = {}, 0
        for e in ent1:
            loc1[e] = c
            c += pb.nb[e[0]]
        n1 = c
        U = {}
        for (J, m) in ent1:
            for key, part in pb.c_rows(I, J, m):
                if key not in U:
                    U[key] = np.zeros((pb.na[key[0]], bI, n1))
                U[key][:, :, loc1[(J, m)]:loc1[(J, m)] + pb.nb[J]] += part
        Y = {}
        for (P, p), UP in U.items():
            nq = pb.entries(P, p)                                # the nu atoms Q + q coupled to P + p
            cols = sorted({e for (Q, q) in nq for e in pb.entries(Q, q)})   # their neighbourhoods
            loc2, c = {}, 0
            for e in cols:
                loc2[e] = c
                c += pb.nb[e[0]]
            TP = (UP.reshape(-1, n1) @ d_rows_cols(ent1, cols)).reshape(pb.na[P], bI, c)
            for (Q, q) in nq:
                VPQ = pb.v(P, p, Q, q)
                ents = pb.entries(Q, q)
                idx = np.concatenate([np.arange(loc2[e], loc2[e] + pb.nb[e[0]]) for e in ents])
                contrib = (VPQ.T @ TP[:, :, idx].reshape(pb.na[P], -1)).reshape(pb.na[Q], bI, len(idx))
                if (Q, q) in Y:
                    Y[(Q, q)] += contrib
                else:
                    Y[(Q, q)] = contrib
        XI = np.zeros((bI, pb.n))
        pattern = dict(ent1)                                     # B -> the image kept for row atom I
        for (Q, q), YQ in Y.items():
            ents = pb.entries(Q, q)
            on_q = pattern.get(Q) == q
            if not on_q and not any(pattern.get(J) == b for J, b in ents):
                continue
            pos, c = {}, 0
            for e in ents:
                pos[e] = c
                c += pb.nb[e[0]]
            for (J, b) in ents:
                mirror = (J, b) != (Q, q) and pattern.get(J) == b
                if not (on_q or mirror):
                    continue
                # C^nu (nu on Q + q) on rows of Q + q and columns of J + b, and its mirror
                for key, part in pb.c_rows(Q, J, _sub(b, q)):
                    if key != (Q, zero):
                        continue
                    if on_q:
                        yJ = YQ[:, :, pos[(J, b)]:pos[(J, b)] + pb.nb[J]]
                        XI[:, pb.bo[Q]:pb.bo[Q + 1]] += np.einsum("nkl,nil->ik", part, yJ, optimize=True)
                    if mirror:
                        yQ = YQ[:, :, pos[(Q, q)]:pos[(Q, q)] + pb.nb[Q]]
                        XI[:, pb.bo[J]:pb.bo[J + 1]] += np.einsum("nkl,nik->il", part, yQ, optimize=True)
        out.append(XI)
    return np.concatenate(out) if out else np.zeros((0, pb.n))


def x_periodic(inputs):
    """The folded X of the whole home cell (moderate sizes only)."""
    pb = PBlocks(inputs)
    return x_atom_rows_periodic(inputs, range(pb.nat), pb)


def x_unfolded(inputs, reach=2.0):
    """The folded X by a second, independent route: an explicit cluster of the
    home cell's atoms and of every image within reach * r_cut of a home atom,
    with each pair block copied from its home-cell pair at the same relative
    image, evaluated with the 4-index route; rows of home atoms, kept on the
    pattern.  (A pattern entry X_AB(n) involves only atoms within two cutoffs
    of A, so reach 2 is exact.)  Small systems only."""
    sysm, lay = inputs.system, inputs.layout
    pb = PBlocks(inputs)
    lat = sysm.lattice
    reach_r = reach * sysm.r_cut
    cands = []
    rng3 = range(-3, 4)
    for a in range(pb.nat):
        for n in ((i, j, k) for i in rng3 for j in rng3 for k in rng3):
            p = sysm.pos[a] + _shift(lat, n)
            dmin = np.sqrt(((sysm.pos - p) ** 2).sum(1)).min()
            if n == (0, 0, 0) or dmin <= reach_r + 1e-9:
                cands.append((a, n))
    cands.sort(key=lambda x: (x[1] != (0, 0, 0), x[1], x[0]))   # home cell first, in atom order
    species = np.array([sysm.species[a] for a, _ in cands])
    pos = np.array([sysm.pos[a] + _shift(lat, n) for a, n in cands])
    import synth
    ext = synth.System(species, pos, sysm.r_cut, sysm.seed, basis_table=sysm.basis_table,
                       aux_table=sysm.aux_table, name="unfolded")
    el = synth.make_layout(ext)
    C = np.empty(int(el.c_off[-1]))
    V = np.empty(int(el.v_off[-1]))
    nbx = sysm.basis_table[species].astype(np.int64)
    box = np.concatenate([[0], np.cumsum(nbx)])
    nx = int(box[-1])
    Dx = np.zeros((nx, nx))
    for q, (A2, B2) in enumerate(zip(el.pair_a, el.pair_b)):
        (A, a), (B, b) = cands[A2], cands[B2]
        r = _sub(b, a)
        if A2 == B2:
            blk = pb.c_rows(A, A, (0, 0, 0))[0][1]
            C[el.c_off[q]:el.c_off[q + 1]] = blk.ravel()
        else:
            parts = dict(pb.c_rows(A, B, r))
            C[el.c_off[q]:el.c_off[q + 1]] = np.concatenate([parts[(A, (0, 0, 0))], parts[(B, r)]]).ravel()
        V[el.v_off[q]:el.v_off[q + 1]] = pb.v(A, (0, 0, 0), B, r).ravel()
        blkD = pb.d(A, (0, 0, 0), B, r)
        Dx[box[A2]:box[A2 + 1], box[B2]:box[B2 + 1]] = blkD
        Dx[box[B2]:box[B2 + 1], box[A2]:box[A2 + 1]] = blkD.T
    ei = synth.Inputs(ext, el, C, V, Dx.ravel())
    Kx = k_4index(ei)[0]
    X = np.zeros((pb.n, pb.n))
    for i2, (A, a) in enumerate(cands):
        if a != (0, 0, 0):
            continue
        for j2, (B, b) in enumerate(cands):
            if pb.img_of[A].get(B) == b:
                X[pb.bo[A]:pb.bo[A + 1], pb.bo[B]:pb.bo[B + 1]] = Kx[box[i2]:box[i2 + 1], box[j2]:box[j2 + 1]]
    return X


# ----------------------------------------------------------------------------
# k-point Bloch sums (Eq. fock_operator_k, Eq. realspace_dm).  k-points are in
# fractional reciprocal coordinates: for the lattice vector R = n L, k.R = 2 pi k.n.


def _pair_blocks(inputs):
    """(A, B, n_AB, rows of A, rows of B) for every canonical pair of a one-system plan."""
    sysm, lay = inputs.system, inputs.layout
    nb = sysm.basis_table[sysm.species].astype(np.int64)
    bo = np.concatenate([[0], np.cumsum(nb)])
    img = lay.pair_img if lay.pair_img is not None else np.zeros((lay.n_pairs, 3), np.int64)
    for p, (a, b) in enumerate(zip(lay.pair_a, lay.pair_b)):
        yield int(a), int(b), np.asarray(img[p], dtype=np.int64), slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])


def bloch_sum(inputs, X, kpts):
    """K(k) = sum_R e^{i k.R} X(R) from the folded real-space X (dense, one system):
    every pair (A, B) has the single image n_AB inside the cutoff, so block (A, B)
    of K(k) is e^{2 pi i k.n_AB} X_AB and block (B, A) takes the conjugate phase;
    zero outside the pair blocks."""
    n = X.shape[0]
    out = []
    for k in np.asarray(kpts, dtype=np.float64).reshape(-1, 3):
        Kk = np.zeros((n, n), dtype=complex)
        for a, b, nab, ia, ib in _pair_blocks(inputs):
            ph = np.exp(2j * np.pi * float(np.dot(k, nab)))
            Kk[ia, ib] = ph * X[ia, ib]
            Kk[ib, ia] = np.conj(ph) * X[ib, ia]
        out.append(Kk)
    return out


def density_from_k(inputs, Dk, kpts):
    """The folded real-space density matrix from D(k) on a k-grid:
    D_AB(n_AB) = Re (1 / N_k) sum_k e^{2 pi i k.n_AB} D_AB(k) (block (B, A) with the
    conjugate phase), zero outside the pair blocks."""
    kp = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
    n = Dk[0].shape[0]
    D = np.zeros((n, n))
    for a, b, nab, ia, ib in _pair_blocks(inputs):
        ph = np.exp(2j * np.pi * (kp @ nab))
        D[ia, ib] = np.real(sum(ph[q] * Dk[q][ia, ib] for q in range(len(kp)))) / len(kp)
        D[ib, ia] = np.real(sum(np.conj(ph[q]) * Dk[q][ib, ia] for q in range(len(kp)))) / len(kp)
    return D


def periodic_energy(X, D):
    """E_x per cell: -1/4 sum over the pattern blocks of X o D (D is zero off the pattern)."""
    return -0.25 * float(np.sum(X * D))
