"""Seeded synthetic water / ice systems and their RI-LVL inputs C, V, D.

This module only produces inputs: atom positions, species, and the three
arrays the exchange build consumes (RI coefficients C, the screened auxiliary
Coulomb matrix V, the density matrix D), in the block layouts the library's
boundary documents.  It contains none of the exchange arithmetic; both the
CPU oracle and the GPU path read what it writes.

Recipe (the paper's workloads are FHI-aims water/ice with "light" species,
8 basis functions per atom on average; here the species counts and value
distributions are synthetic stand-ins):

* species O: 14 basis / 40 auxiliary functions; H: 5 basis / 15 auxiliary.
* O sites: a jittered 2.8 A half-integer cubic grid (clusters) or a jittered
  diamond-like lattice with 3.1 A O-O nearest-neighbour distance (ice boxes).
  Jitter is uniform in [-0.15, 0.15] A per coordinate.
* each O carries two H at 0.96 A with a 104.5 degree H-O-H angle, oriented by
  a uniformly random unit quaternion.
* atom order is molecule by molecule: O, H, H.
* one inclusive cutoff r <= r_cut on atom-pair distance decides which C, V and
  D blocks exist (all other blocks are structurally zero).
* C block of pair (A, B), A != B: N(0,1) * exp(-r_AB / 1.5), aux of A first,
  then aux of B; on-site blocks: N(0,1), symmetric in the two basis indices.
* D block (A, B): N(0,1) * exp(-r_AB / 2.0), D symmetric, on-site block
  symmetric N(0,1).
* V block (A, B) = exp(-r_AB^2 / 8) * (L_s(A) L_s(B)^T), L_s an n_aux(s) x 40
  matrix of N(0,1)/sqrt(40) entries per species (SPD by the Schur product
  theorem before screening).

Random numbers come from per-block keyed streams (seed, kind, label_a,
label_b), so values follow atoms under any permutation of the atom order.
Periodic systems add the pair's lattice image (in cells of the generating
lattice) to the key when it is not zero, so a cluster in a large box has the
cluster's values and a supercell repeats its cell's values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# species table: index -> (name, n_basis, n_aux)
SPECIES_NAMES = ("O", "H")
N_BASIS = np.array([14, 5], dtype=np.int32)
N_AUX = np.array([40, 15], dtype=np.int32)
O, H = 0, 1

C_DECAY = 1.5          # A, C ~ exp(-r / C_DECAY)
D_DECAY = 2.0          # A, D ~ exp(-r / D_DECAY)
V_GAUSS_2S2 = 8.0      # A^2, V ~ exp(-r^2 / V_GAUSS_2S2)  (2 * 2.0^2)
V_SR_2S2 = 2.0         # A^2, the second (shorter-range) Coulomb matrix: exp(-r^2 / V_SR_2S2)
L_RANK = 40            # inner dimension of the per-species V factors

_KIND_GEOM, _KIND_C, _KIND_D, _KIND_V, _KIND_BATCH, _KIND_SPIN = 1, 2, 3, 4, 5, 6
SPIN_POLARIZATION = 0.3   # weight m of the spin-difference matrix S in D^0, D^1 = (D +- m S) / 2

OH_BOND = 0.96
HOH_ANGLE = math.radians(104.5)
JITTER = 0.15


@dataclass
class System:
    """A set of atoms, possibly several independent clusters (a batch)."""
    species: np.ndarray            # (n_atoms,) int32
    pos: np.ndarray                # (n_atoms, 3) float64, Angstrom
    r_cut: float
    seed: int
    labels: np.ndarray = None      # (n_atoms,) int64, persistent ids for RNG keys
    sys_off: np.ndarray = None     # (n_systems + 1,) int32 atom offsets
    name: str = ""
    basis_table: np.ndarray = None  # per-species basis counts (default N_BASIS)
    aux_table: np.ndarray = None    # per-species aux counts (default N_AUX)
    lattice: np.ndarray = None      # (3, 3) lattice vectors (rows, A) of a periodic system, or None
    cell_index: np.ndarray = None   # (n_atoms, 3) int: copy of the generating cell an atom sits in
    cell_mult: np.ndarray = None    # (3,) int: cells of the generating lattice per lattice vector

    def __post_init__(self):
        self.species = np.ascontiguousarray(self.species, dtype=np.int32)
        self.pos = np.ascontiguousarray(self.pos, dtype=np.float64)
        n = len(self.species)
        if self.labels is None:
            self.labels = np.arange(n, dtype=np.int64)
        self.labels = np.ascontiguousarray(self.labels, dtype=np.int64)
        if self.sys_off is None:
            self.sys_off = np.array([0, n], dtype=np.int32)
        self.sys_off = np.ascontiguousarray(self.sys_off, dtype=np.int32)
        self.basis_table = np.ascontiguousarray(N_BASIS if self.basis_table is None else self.basis_table,
                                                dtype=np.int32)
        self.aux_table = np.ascontiguousarray(N_AUX if self.aux_table is None else self.aux_table,
                                              dtype=np.int32)
        if self.lattice is not None:
            self.lattice = np.ascontiguousarray(self.lattice, dtype=np.float64).reshape(3, 3)
            if self.cell_index is None:
                self.cell_index = np.zeros((n, 3), dtype=np.int64)
            if self.cell_mult is None:
                self.cell_mult = np.ones(3, dtype=np.int64)
            self.cell_index = np.ascontiguousarray(self.cell_index, dtype=np.int64).reshape(n, 3)
            self.cell_mult = np.asarray(self.cell_mult, dtype=np.int64).reshape(3)

    @property
    def periodic(self):
        return self.lattice is not None

    @property
    def n_atoms(self):
        return len(self.species)

    @property
    def n_systems(self):
        return len(self.sys_off) - 1

    def nbas(self):
        return self.basis_table[self.species]

    def naux(self):
        return self.aux_table[self.species]


@dataclass
class Layout:
    """Block layout of C and V (canonical pairs) and of dense D/K per system."""
    pair_a: np.ndarray             # (n_pairs,) int32, A <= B, lexicographic
    pair_b: np.ndarray
    c_off: np.ndarray              # (n_pairs + 1,) int64
    v_off: np.ndarray              # (n_pairs + 1,) int64
    bas_off: np.ndarray            # (n_atoms,) basis offset within its system
    sys_bas_off: np.ndarray        # (n_systems + 1,) int64, offsets of dense blocks in D/K
    sys_nbas: np.ndarray           # (n_systems,) int64
    pair_img: np.ndarray = None    # (n_pairs, 3) int: lattice image n of B in pair (A, B + n)

    @property
    def n_pairs(self):
        return len(self.pair_a)

    @property
    def d_size(self):
        return int(self.sys_bas_off[-1])


@dataclass
class Inputs:
    system: System
    layout: Layout
    C: np.ndarray                  # flat float64, pair blocks
    V: np.ndarray                  # flat float64, pair blocks
    D: np.ndarray                  # flat float64, dense per system (concatenated)
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# geometry

def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _waters_from_oxygens(o_pos, rng):
    """Jitter O sites, add two H per O; atom order O, H, H per molecule."""
    n = len(o_pos)
    o = o_pos + rng.uniform(-JITTER, JITTER, size=(n, 3))
    half = 0.5 * HOH_ANGLE
    h1_local = OH_BOND * np.array([math.sin(half), 0.0, math.cos(half)])
    h2_local = OH_BOND * np.array([-math.sin(half), 0.0, math.cos(half)])
    pos = np.empty((3 * n, 3))
    for m in range(n):
        R = _random_rotation(rng)
        pos[3 * m] = o[m]
        pos[3 * m + 1] = o[m] + R @ h1_local
        pos[3 * m + 2] = o[m] + R @ h2_local
    species = np.tile(np.array([O, H, H], dtype=np.int32), n)
    return species, pos


def cubic_cluster_sites(n_mol, spacing=2.8):
    """The n_mol sites of a half-integer cubic grid nearest its centre.

    Ties in distance are broken lexicographically by (x, y, z)."""
    m = int(math.ceil(n_mol ** (1.0 / 3.0))) // 2 + 2
    g = np.arange(-m, m) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * spacing
    r2 = np.round((sites ** 2).sum(1), 9)
    order = np.lexsort((sites[:, 2], sites[:, 1], sites[:, 0], r2))
    return sites[order[:n_mol]]


def water_cluster(n_mol, seed, r_cut=6.0, spacing=2.8):
    """Non-periodic water cluster on a jittered cubic grid."""
    rng = _rng(seed, _KIND_GEOM)
    species, pos = _waters_from_oxygens(cubic_cluster_sites(n_mol, spacing), rng)
    return System(species, pos, r_cut, seed, name=f"water_cluster_{n_mol}")


ICE_NN = 3.1


def diamond_sites(nx, ny, nz, nn=ICE_NN):
    """O sites of a diamond-like lattice, nearest-neighbour distance nn."""
    a = 4.0 * nn / math.sqrt(3.0)
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])
    sites = []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                for b in basis:
                    sites.append((np.array([ix, iy, iz]) + b) * a)
    return np.array(sites), a


def ice_box(nx, ny, nz, seed, r_cut=6.0):
    """Open (non-periodic) ice-like box of 8*nx*ny*nz water molecules."""
    rng = _rng(seed, _KIND_GEOM)
    sites, _ = diamond_sites(nx, ny, nz)
    species, pos = _waters_from_oxygens(sites, rng)
    return System(species, pos, r_cut, seed, name=f"ice_box_{nx}x{ny}x{nz}")


def ice_box_periodic(nx, ny, nz, seed, r_cut=8.0):
    """Periodic ice-like box of 8*nx*ny*nz water molecules: the sites and
    jitter of ice_box, with the box edges as lattice vectors."""
    sysm = ice_box(nx, ny, nz, seed, r_cut)
    a = 4.0 * ICE_NN / math.sqrt(3.0)
    return System(sysm.species, sysm.pos, r_cut, seed, name=f"ice_box_periodic_{nx}x{ny}x{nz}",
                  lattice=np.diag([nx * a, ny * a, nz * a]))


def supercell(system, mult):
    """The periodic system repeated mult[0] x mult[1] x mult[2] times: copies
    keep their atom labels and record the copy they sit in, so every pair block
    of the supercell carries the values of the same pair of the cell."""
    mult = np.asarray(mult, dtype=np.int64)
    lat = system.lattice
    species, pos, labels, cells = [], [], [], []
    for i in range(mult[0]):
        for j in range(mult[1]):
            for k in range(mult[2]):
                c = np.array([i, j, k])
                species.append(system.species)
                pos.append(system.pos + image_shift(lat, c))
                labels.append(system.labels)
                cells.append(np.tile(c, (system.n_atoms, 1)))
    return System(np.concatenate(species), np.concatenate(pos), system.r_cut, system.seed,
                  labels=np.concatenate(labels), name=system.name + "_super",
                  basis_table=system.basis_table, aux_table=system.aux_table,
                  lattice=lat * mult[:, None], cell_index=np.concatenate(cells), cell_mult=mult)


def cluster_batch(n_clusters=64, batch_seed=123, n_min=8, n_max=128, r_cut=6.0):
    """Independent water clusters of uneven sizes, concatenated as one batch.

    Cluster c has n_c ~ U{n_min..n_max} molecules (drawn from the batch
    seed) and uses seed c for its geometry and values."""
    rng = _rng(batch_seed, _KIND_BATCH)
    sizes = rng.integers(n_min, n_max + 1, size=n_clusters)
    species, pos, labels, off = [], [], [], [0]
    for c, n in enumerate(sizes):
        s = water_cluster(int(n), seed=c, r_cut=r_cut)
        species.append(s.species)
        # keep clusters far apart; pairs never cross systems anyway
        pos.append(s.pos + np.array([1000.0 * c, 0.0, 0.0]))
        labels.append(np.arange(s.n_atoms, dtype=np.int64))  # keys also carry seed c
        off.append(off[-1] + s.n_atoms)
    sysm = System(np.concatenate(species), np.concatenate(pos), r_cut, batch_seed,
                  labels=np.concatenate(labels), sys_off=np.array(off, dtype=np.int32),
                  name=f"cluster_batch_{n_clusters}")
    sysm.cluster_seeds = list(range(n_clusters))
    return sysm


def permuted(system, perm):
    """The same system with atoms reordered (labels follow the atoms)."""
    perm = np.asarray(perm)
    assert system.n_systems == 1
    return System(system.species[perm], system.pos[perm], system.r_cut, system.seed,
                  labels=system.labels[perm], name=system.name + "_perm",
                  basis_table=system.basis_table, aux_table=system.aux_table)


# ----------------------------------------------------------------------------
# block layout

def image_shift(lattice, n):
    """n[0] a_0 + n[1] a_1 + n[2] a_2 per component, summed in that order."""
    a = lattice
    return np.array([(n[0] * a[0, c] + n[1] * a[1, c]) + n[2] * a[2, c] for c in range(3)])


def half_width(lattice):
    """Half the smallest distance between opposite faces of the cell."""
    a = lattice
    vol = abs(float(np.linalg.det(a)))
    return 0.5 * min(vol / float(np.linalg.norm(np.cross(a[(i + 1) % 3], a[(i + 2) % 3]))) for i in range(3))


IMAGES = [np.array((i, j, k)) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]


def canonical_pairs(system):
    """All (A, B), A <= B, same system, |R_A - R_B|^2 <= r_cut^2, lexicographic.

    The squared distance is formed as dx*dx + dy*dy + dz*dz in float64,
    left to right, without fused multiply-add.  Periodic systems: B is taken
    at the one lattice image R_B + n (n in {-1, 0, 1}^3, d = (R_B + shift) -
    R_A) within the cutoff, which is unique because the cutoff is below half
    the cell width; returns (pair_a, pair_b, pair_img)."""
    pa, pb = [], []
    rc2 = system.r_cut * system.r_cut
    if system.periodic:
        if system.r_cut >= half_width(system.lattice):
            raise ValueError("r_cut must be below half the cell width")
        shifts = [image_shift(system.lattice, n) for n in IMAGES]
        P = system.pos
        out_b, out_n = [], []
        for a in range(system.n_atoms):
            Pb = P[a:]
            bs, ns = [], []
            for k, sh in enumerate(shifts):
                dx = (Pb[:, 0] + sh[0]) - P[a, 0]
                dy = (Pb[:, 1] + sh[1]) - P[a, 1]
                dz = (Pb[:, 2] + sh[2]) - P[a, 2]
                hit = np.nonzero((dx * dx + dy * dy) + dz * dz <= rc2)[0]
                if IMAGES[k].any():
                    hit = hit[hit > 0]          # an atom is never paired with its own image
                bs.append(hit + a)
                ns.append(np.full(len(hit), k))
            b = np.concatenate(bs)
            k = np.concatenate(ns)
            order = np.argsort(b, kind="stable")
            pa.append(np.full(len(b), a, dtype=np.int32))
            out_b.append(b[order].astype(np.int32))
            out_n.append(np.array(IMAGES)[k[order]])
        return np.concatenate(pa), np.concatenate(out_b), np.concatenate(out_n).astype(np.int64).reshape(-1, 3)
    for s in range(system.n_systems):
        lo, hi = int(system.sys_off[s]), int(system.sys_off[s + 1])
        P = system.pos[lo:hi]
        for a in range(hi - lo):
            d = P[a:] - P[a]
            dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
            r2 = (dx * dx + dy * dy) + dz * dz
            idx = np.nonzero(r2 <= rc2)[0]
            pa.append(np.full(len(idx), lo + a, dtype=np.int32))
            pb.append((lo + a + idx).astype(np.int32))
    return np.concatenate(pa), np.concatenate(pb)


def make_layout(system):
    if system.periodic:
        pa, pb, pimg = canonical_pairs(system)
    else:
        pa, pb = canonical_pairs(system)
        pimg = np.zeros((len(pa), 3), dtype=np.int64)
    nb, na = system.nbas().astype(np.int64), system.naux().astype(np.int64)
    csz = np.where(pa == pb, na[pa] * nb[pa] * nb[pa], (na[pa] + na[pb]) * nb[pa] * nb[pb])
    vsz = na[pa] * na[pb]
    c_off = np.concatenate([[0], np.cumsum(csz)]).astype(np.int64)
    v_off = np.concatenate([[0], np.cumsum(vsz)]).astype(np.int64)
    bas_off = np.zeros(system.n_atoms, dtype=np.int64)
    sys_nbas = np.zeros(system.n_systems, dtype=np.int64)
    for s in range(system.n_systems):
        lo, hi = int(system.sys_off[s]), int(system.sys_off[s + 1])
        bas_off[lo:hi] = np.concatenate([[0], np.cumsum(nb[lo:hi])[:-1]])
        sys_nbas[s] = nb[lo:hi].sum()
    sys_bas_off = np.concatenate([[0], np.cumsum(sys_nbas ** 2)]).astype(np.int64)
    return Layout(pa, pb, c_off, v_off, bas_off, sys_bas_off, sys_nbas, pimg)


# ----------------------------------------------------------------------------
# values

def _sym_upper(x):
    """Mirror the upper triangle (incl. diagonal) of the last two axes."""
    u = np.triu(x)
    return u + np.swapaxes(np.triu(x, 1), -1, -2)


def v_factors(seed, aux_table=N_AUX):
    rng = _rng(seed, _KIND_V)
    return [rng.normal(size=(int(aux_table[s]), L_RANK)) / math.sqrt(L_RANK)
            for s in range(len(aux_table))]


def _pair_geometry(system, layout, p):
    """Separation vector R_A - (R_B + shift) of canonical pair p (shift: the
    pair's lattice image for periodic systems) and the RNG image key: None for
    clusters, else the image in units of the generating cell, so that a
    supercell repeats its cell's values."""
    A, B = int(layout.pair_a[p]), int(layout.pair_b[p])
    if not system.periodic:
        return system.pos[A] - system.pos[B], None
    n = layout.pair_img[p]
    d = system.pos[A] - (system.pos[B] + image_shift(system.lattice, n))
    key = system.cell_index[B] - system.cell_index[A] + system.cell_mult * n
    return d, np.asarray(key, dtype=np.int64)


def make_inputs(system, layout=None, zero_D=False):
    """Generate C, V, D for a system in the library's block layouts.

    Periodic systems: the blocks of pair (A, B) belong to B's lattice image
    within the cutoff, and D holds, in its dense (A, B) block, D_AB at that
    image (the only one inside the cutoff)."""
    if layout is None:
        layout = make_layout(system)
    sp, lab, pos = system.species, system.labels, system.pos
    nb, na = system.basis_table, system.aux_table
    C = np.empty(int(layout.c_off[-1]))
    V = np.empty(int(layout.v_off[-1]))
    D = np.zeros(layout.d_size)
    L = v_factors(system.seed, na)
    seeds = getattr(system, "cluster_seeds", None)
    atom_sys = np.zeros(system.n_atoms, dtype=np.int64)
    for s in range(system.n_systems):
        atom_sys[system.sys_off[s]:system.sys_off[s + 1]] = s
    for p in range(layout.n_pairs):
        A, B = int(layout.pair_a[p]), int(layout.pair_b[p])
        sA, sB = int(sp[A]), int(sp[B])
        seed = system.seed if seeds is None else seeds[atom_sys[A]]
        Ls = L if seeds is None else v_factors(seed, na)
        d, key = _pair_geometry(system, layout, p)
        r = math.sqrt(float(d @ d))
        c0, c1 = int(layout.c_off[p]), int(layout.c_off[p + 1])
        v0, v1 = int(layout.v_off[p]), int(layout.v_off[p + 1])
        so = int(layout.sys_bas_off[atom_sys[A]])
        n_s = int(layout.sys_nbas[atom_sys[A]])
        ia, ib = int(layout.bas_off[A]), int(layout.bas_off[B])
        if A == B:
            rng_c = _rng(seed, _KIND_C, lab[A], lab[A])
            blk = _sym_upper(rng_c.normal(size=(na[sA], nb[sA], nb[sA])))
            C[c0:c1] = blk.ravel()
            V[v0:v1] = (Ls[sA] @ Ls[sA].T).ravel()
            rng_d = _rng(seed, _KIND_D, lab[A], lab[A])
            dblk = _sym_upper(rng_d.normal(size=(nb[sA], nb[sA])))
        else:
            # generate in label orientation (lower label first), then map
            flip = lab[A] > lab[B] or (lab[A] == lab[B] and tuple(key) < (0, 0, 0))
            la, lb = (lab[B], lab[A]) if flip else (lab[A], lab[B])
            s1, s2 = (sB, sA) if flip else (sA, sB)
            img = [] if key is None or not key.any() else [int(x) + 8 for x in (-key if flip else key)]
            rng_c = _rng(seed, _KIND_C, la, lb, *img)
            blk = rng_c.normal(size=(na[s1] + na[s2], nb[s1], nb[s2])) * math.exp(-r / C_DECAY)
            if flip:  # label order (B, A) -> index order (A, B)
                blk = np.concatenate([blk[na[s1]:], blk[:na[s1]]], axis=0).transpose(0, 2, 1)
            C[c0:c1] = np.ascontiguousarray(blk).ravel()
            V[v0:v1] = (math.exp(-r * r / V_GAUSS_2S2) * (Ls[sA] @ Ls[sB].T)).ravel()
            rng_d = _rng(seed, _KIND_D, la, lb, *img)
            dblk = rng_d.normal(size=(nb[s1], nb[s2])) * math.exp(-r / D_DECAY)
            if flip:
                dblk = dblk.T
        if not zero_D:
            Dm = D[so:so + n_s * n_s].reshape(n_s, n_s)
            Dm[ia:ia + nb[sA], ib:ib + nb[sB]] = dblk
            Dm[ib:ib + nb[sB], ia:ia + nb[sA]] = dblk.T
    return Inputs(system, layout, C, V, D)


def short_range_V(inputs, two_s2=V_SR_2S2):
    """A second, shorter-range Coulomb matrix in the layout of inputs.V:
    block (A, B) = exp(-r_AB^2 / two_s2) * (L_s(A) L_s(B)^T) with the same
    per-species factors L as V (SPD before screening, like V)."""
    system, layout = inputs.system, inputs.layout
    sp, pos = system.species, system.pos
    na = system.aux_table
    seeds = getattr(system, "cluster_seeds", None)
    atom_sys = np.zeros(system.n_atoms, dtype=np.int64)
    for s in range(system.n_systems):
        atom_sys[system.sys_off[s]:system.sys_off[s + 1]] = s
    L = v_factors(system.seed, na)
    V2 = np.empty(int(layout.v_off[-1]))
    for p in range(layout.n_pairs):
        A, B = int(layout.pair_a[p]), int(layout.pair_b[p])
        sA, sB = int(sp[A]), int(sp[B])
        Ls = L if seeds is None else v_factors(seeds[atom_sys[A]], na)
        d, _ = _pair_geometry(system, layout, p)
        r2 = float(d @ d)
        w = 1.0 if A == B else math.exp(-r2 / two_s2)
        V2[int(layout.v_off[p]):int(layout.v_off[p + 1])] = (w * (Ls[sA] @ Ls[sB].T)).ravel()
    return V2


def spin_densities(inputs, polarization=SPIN_POLARIZATION):
    """Two collinear-spin density matrices, shape (2, d_size):
    D^0 = (D + m S) / 2 and D^1 = (D - m S) / 2 with m = polarization.

    S, a spin-difference (magnetisation-like) matrix, follows the D recipe:
    the same block pattern, symmetry and exp(-r / 2.0) decay, drawn from its
    own keyed streams, so D^0 + D^1 = D exactly (up to one rounding)."""
    system, layout = inputs.system, inputs.layout
    sp, lab, pos = system.species, system.labels, system.pos
    nb = system.basis_table
    seeds = getattr(system, "cluster_seeds", None)
    atom_sys = np.zeros(system.n_atoms, dtype=np.int64)
    for s in range(system.n_systems):
        atom_sys[system.sys_off[s]:system.sys_off[s + 1]] = s
    S = np.zeros(layout.d_size)
    for p in range(layout.n_pairs):
        A, B = int(layout.pair_a[p]), int(layout.pair_b[p])
        sA, sB = int(sp[A]), int(sp[B])
        seed = system.seed if seeds is None else seeds[atom_sys[A]]
        so = int(layout.sys_bas_off[atom_sys[A]])
        n_s = int(layout.sys_nbas[atom_sys[A]])
        ia, ib = int(layout.bas_off[A]), int(layout.bas_off[B])
        if A == B:
            blk = _sym_upper(_rng(seed, _KIND_SPIN, lab[A], lab[A]).normal(size=(nb[sA], nb[sA])))
        else:
            d, key = _pair_geometry(system, layout, p)
            r = math.sqrt(float(d @ d))
            flip = lab[A] > lab[B] or (lab[A] == lab[B] and key is not None and tuple(key) < (0, 0, 0))
            la, lb = (lab[B], lab[A]) if flip else (lab[A], lab[B])
            s1, s2 = (sB, sA) if flip else (sA, sB)
            img = [] if key is None or not key.any() else [int(x) + 8 for x in (-key if flip else key)]
            blk = _rng(seed, _KIND_SPIN, la, lb, *img).normal(size=(nb[s1], nb[s2])) * math.exp(-r / D_DECAY)
            if flip:
                blk = blk.T
        Sm = S[so:so + n_s * n_s].reshape(n_s, n_s)
        Sm[ia:ia + nb[sA], ib:ib + nb[sB]] = blk
        Sm[ib:ib + nb[sB], ia:ia + nb[sA]] = blk.T
    m = float(polarization)
    return np.stack([0.5 * (inputs.D + m * S), 0.5 * (inputs.D - m * S)])


# ----------------------------------------------------------------------------
# the five workloads

def config(n, seed=0):
    """Workload n (1-based) at full size.

    1: 8-molecule cluster (24 atoms), r_cut 6 A.
    2: 256-molecule open ice box (768 atoms), r_cut 6 A.
    3: batch of 64 clusters of 8..128 molecules, r_cut 6 A.
    4: the 768-atom box again (differentiation workload).
    5: 1024-molecule periodic ice box (3072 atoms, 57.3 x 28.6 x 28.6 A
       cell), r_cut 8 A."""
    if n == 1:
        return water_cluster(8, seed)
    if n in (2, 4):
        return ice_box(4, 4, 2, seed)
    if n == 3:
        return cluster_batch()
    if n == 5:
        return ice_box_periodic(8, 4, 4, seed, r_cut=8.0)
    raise ValueError(n)
