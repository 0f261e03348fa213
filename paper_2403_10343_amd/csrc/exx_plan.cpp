// Host-side bookkeeping of an exchange plan: validation, canonical pairs,
// second neighbourhoods, column maps, workspace layout and the task lists of
// every kernel (the atom-pair / atom-quartet block lists of the build).
//
// The lists mirror the grouping of the pair-restricted exchange sum by atom
// pairs (Sec. "Description of the real-space formalism", Eq.
// ri_lvl_exchange_matrix): every task is keyed by the auxiliary atom P that
// owns the row-owned coefficient block T_P, and by output tiles.
#include "exx_internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

namespace exx {

int describe_system(const int32_t n_atoms, const int32_t n_species, const int32_t* species,
                    const double* positions, const int32_t* n_basis, const int32_t* n_aux,
                    double r_cut, int32_t n_systems, const int32_t* sys_atom_off,
                    const double* lattice, HostPlan& hp, std::string& err) {
  if (n_atoms <= 0 || n_species <= 0 || !species || !positions || !n_basis || !n_aux) {
    err = "exx_system: null array or non-positive count";
    return -1;
  }
  if (!(r_cut > 0) || !std::isfinite(r_cut)) { err = "exx_system: r_cut must be positive"; return -1; }
  if (n_systems < 1 || (n_systems > 1 && !sys_atom_off)) { err = "exx_system: bad n_systems / sys_atom_off"; return -1; }
  for (int s = 0; s < n_species; ++s) {
    if (n_basis[s] < 1 || n_aux[s] < 1) { err = "exx_system: species with no functions"; return -1; }
    if (n_basis[s] > NB_MAX || n_aux[s] > NA_MAX) {
      err = "exx_system: species exceeds the supported per-atom sizes (basis <= 16, aux <= 64)";
      return -5;
    }
  }
  hp.n_atoms = n_atoms;
  hp.n_sys = n_systems;
  hp.mixed[0].split = 5.0;
  hp.mixed[1].split = 0.0;
  hp.r_cut = r_cut;
  hp.species.assign(species, species + n_atoms);
  hp.pos.assign(positions, positions + 3 * (size_t)n_atoms);
  for (double x : hp.pos) if (!std::isfinite(x)) { err = "exx_system: non-finite position"; return -1; }
  hp.sys_atom_off.resize(n_systems + 1);
  if (sys_atom_off) {
    for (int s = 0; s <= n_systems; ++s) hp.sys_atom_off[s] = sys_atom_off[s];
  } else {
    hp.sys_atom_off[0] = 0;
    hp.sys_atom_off[1] = n_atoms;
  }
  if (hp.sys_atom_off[0] != 0 || hp.sys_atom_off[n_systems] != n_atoms) {
    err = "exx_system: sys_atom_off must start at 0 and end at n_atoms";
    return -1;
  }
  for (int s = 0; s < n_systems; ++s)
    if (hp.sys_atom_off[s + 1] <= hp.sys_atom_off[s]) { err = "exx_system: empty or decreasing system"; return -1; }
  hp.nb.resize(n_atoms);
  hp.na.resize(n_atoms);
  hp.atom_sys.resize(n_atoms);
  hp.bo.resize(n_atoms);
  hp.sys_n.assign(n_systems, 0);
  hp.sys_d_off.assign(n_systems + 1, 0);
  for (int s = 0; s < n_systems; ++s) {
    int64_t off = 0;
    for (int a = hp.sys_atom_off[s]; a < hp.sys_atom_off[s + 1]; ++a) {
      int sp = species[a];
      if (sp < 0 || sp >= n_species) { err = "exx_system: species index out of range"; return -1; }
      hp.nb[a] = n_basis[sp];
      hp.na[a] = n_aux[sp];
      hp.atom_sys[a] = s;
      hp.bo[a] = (int)off;
      off += n_basis[sp];
    }
    if (off > (int64_t)1 << 30) { err = "exx_system: system too large"; return -1; }
    hp.sys_n[s] = off;
    hp.sys_d_off[s + 1] = hp.sys_d_off[s] + off * off;
    hp.n_basis_max = std::max(hp.n_basis_max, off);
  }
  hp.d_size = hp.sys_d_off[n_systems];
  hp.periodic = lattice != nullptr;
  if (hp.periodic) {
    if (n_systems != 1) { err = "exx_system: a periodic plan holds one system"; return -5; }
    for (int i = 0; i < 9; ++i) {
      if (!std::isfinite(lattice[i])) { err = "exx_system: non-finite lattice vector"; return -1; }
      hp.lat[i] = lattice[i];
    }
    // the cutoff must be below half the distance between opposite cell faces, so that an
    // atom pair has at most one image within it
    const double* a = hp.lat;
    const double vol = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                                 a[2] * (a[3] * a[7] - a[4] * a[6]));
    double hw = 1e300;
    for (int i = 0; i < 3; ++i) {
      const double* u = a + 3 * ((i + 1) % 3);
      const double* v = a + 3 * ((i + 2) % 3);
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
      hw = std::min(hw, 0.5 * vol / std::sqrt(cx * cx + cy * cy + cz * cz));
    }
    if (!(vol > 0) || !(r_cut < hw)) {
      err = "exx_system: r_cut must be below half the cell width (" + std::to_string(hw) + " A)";
      return -1;
    }
    // image components of N2 entries stay within [-8, 8) when the positions lie within two
    // cell widths of the home cell
    if (hp.n_atoms > 0 && hp.n_atoms * (int64_t)hp.n_atoms > (int64_t)1 << 31) {
      err = "exx_system: periodic plans hold at most 46340 atoms";
      return -5;
    }
  }
  return 0;
}

#pragma clang fp contract(off)
void host_neighbors(HostPlan& hp) {
  const double rc2 = hp.r_cut * hp.r_cut;
  hp.nbr_ptr.assign(hp.n_atoms + 1, 0);
  hp.nbr_atom.clear();
  for (int s = 0; s < hp.n_sys; ++s) {
    const int lo = hp.sys_atom_off[s], hi = hp.sys_atom_off[s + 1];
    for (int a = lo; a < hi; ++a) {
      const double* pa = &hp.pos[3 * (size_t)a];
      for (int b = lo; b < hi; ++b) {
        const double* pb = &hp.pos[3 * (size_t)b];
        volatile double dx = pa[0] - pb[0], dy = pa[1] - pb[1], dz = pa[2] - pb[2];
        volatile double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        volatile double r2 = (xx + yy);
        r2 = r2 + zz;
        if (r2 <= rc2) hp.nbr_atom.push_back(b);
      }
      hp.nbr_ptr[a + 1] = (int)hp.nbr_atom.size();
    }
  }
}

namespace {

int64_t ceil_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

void tile_kflags(const HostPlan& hp, const std::vector<KEnt>& krow, const std::vector<KEnt>& ccol, int klen,
                 std::vector<uint8_t>& out) {
  const size_t base = out.size();
  out.resize(base + (klen + 15) / 16, 0);
  const int NA = hp.n_atoms;
  if (hp.periodic) {
    for (const KEnt& r : krow) {
      int bits = 0;   // quarters holding a column at the image of a neighbour of r
      for (const KEnt& c : ccol) {
        const int n = hp.pimg[(size_t)r.atom * NA + c.atom];
        if (n >= 0 && img_add(n, r.img) == c.img)
          for (int q = c.beg / 16; q <= (c.beg + c.len - 1) / 16; ++q) bits |= 1 << q;
      }
      if (bits)
        for (int g = r.beg / 16; g <= (r.beg + r.len - 1) / 16; ++g) out[base + g] |= (uint8_t)bits;
    }
    return;
  }
  // clusters: D_JL is nonzero for J in N[L]; mark the neighbours of every column atom with
  // the column's quarter bits, then read them off for the k-side atoms
  static thread_local std::vector<uint8_t> qbits;
  static thread_local std::vector<int> touched;
  if ((int)qbits.size() < NA) qbits.assign(NA, 0);
  touched.clear();
  for (const KEnt& c : ccol) {
    int bits = 0;
    for (int q = c.beg / 16; q <= (c.beg + c.len - 1) / 16; ++q) bits |= 1 << q;
    for (int k = hp.nbr_ptr[c.atom]; k < hp.nbr_ptr[c.atom + 1]; ++k) {
      const int j = hp.nbr_atom[k];
      if (!qbits[j]) touched.push_back(j);
      qbits[j] |= (uint8_t)bits;
    }
  }
  for (const KEnt& r : krow) {
    const int bits = qbits[r.atom];
    if (bits)
      for (int g = r.beg / 16; g <= (r.beg + r.len - 1) / 16; ++g) out[base + g] |= (uint8_t)bits;
  }
  for (int j : touched) qbits[j] = 0;
}

// issued MFMA flops of the E (or gradient) GEMM on one column tile with flags f
// (ceil(klen / 16) bytes) over an output of s_P rows: 16 x 16 x 16 blocks, skipped where D
// is structurally zero or the 16 rows lie past s_P
int64_t kflag_issued(const uint8_t* f, int klen, int sP) {
  int64_t n = 0;
  for (int g = 0; g < (klen + 15) / 16; ++g) n += __builtin_popcount(f[g]);
  return n * ((sP + 15) / 16) * 2LL * 16 * 16 * 16;
}

int derive_lists(HostPlan& hp, std::string& err) {
  const int NA = hp.n_atoms;
  const auto& np = hp.nbr_ptr;
  const auto& nat = hp.nbr_atom;
  const int64_t nn = np[NA];
  // every atom must be its own neighbour
  for (int a = 0; a < NA; ++a) {
    if (!std::binary_search(nat.begin() + np[a], nat.begin() + np[a + 1], a)) {
      err = "neighbour list lost an atom's self pair";
      return -3;
    }
  }
  // ---- canonical pairs (A <= B, lexicographic) and pair id of every entry
  hp.nbr_pair.assign(nn, -1);
  hp.nbr_owner.assign(nn, 0);
  hp.pair_a.clear();
  hp.pair_b.clear();
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k) {
      hp.nbr_owner[k] = a;
      if (nat[k] >= a) {
        hp.nbr_pair[k] = (int)hp.pair_a.size();
        hp.pair_a.push_back(a);
        hp.pair_b.push_back(nat[k]);
      }
    }
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k)
      if (nat[k] < a) {
        int b = nat[k];
        auto it = std::lower_bound(nat.begin() + np[b], nat.begin() + np[b + 1], a);
        if (it == nat.begin() + np[b + 1] || *it != a) { err = "neighbour list not symmetric"; return -3; }
        hp.nbr_pair[k] = hp.nbr_pair[it - nat.begin()];
      }
  const int64_t npairs = (int64_t)hp.pair_a.size();
  hp.c_off.assign(npairs + 1, 0);
  hp.v_off.assign(npairs + 1, 0);
  for (int64_t p = 0; p < npairs; ++p) {
    int a = hp.pair_a[p], b = hp.pair_b[p];
    int64_t cs = (a == b) ? (int64_t)hp.na[a] * hp.nb[a] * hp.nb[a]
                          : (int64_t)(hp.na[a] + hp.na[b]) * hp.nb[a] * hp.nb[b];
    hp.c_off[p + 1] = hp.c_off[p] + cs;
    hp.v_off[p + 1] = hp.v_off[p] + (int64_t)hp.na[a] * hp.na[b];
  }
  // ---- local columns of T_P
  hp.nbr_lcol.assign(nn, 0);
  hp.n_loc.assign(NA, 0);
  for (int a = 0; a < NA; ++a) {
    int c = 0;
    for (int k = np[a]; k < np[a + 1]; ++k) { hp.nbr_lcol[k] = c; c += hp.nb[nat[k]]; }
    hp.n_loc[a] = c;
  }
  // ---- N2
  hp.n2_ptr.assign(NA + 1, 0);
  hp.n2_atom.clear();
  hp.m_loc.assign(NA, 0);
  std::vector<int> stamp(NA, -1);
  std::vector<int> tmp;
  for (int a = 0; a < NA; ++a) {
    tmp.clear();
    for (int k = np[a]; k < np[a + 1]; ++k) {
      int j = nat[k];
      for (int k2 = np[j]; k2 < np[j + 1]; ++k2) {
        int l = nat[k2];
        if (stamp[l] != a) { stamp[l] = a; tmp.push_back(l); }
      }
    }
    std::sort(tmp.begin(), tmp.end());
    int m = 0;
    for (int l : tmp) { hp.n2_atom.push_back(l); m += hp.nb[l]; }
    hp.n2_ptr[a + 1] = (int)hp.n2_atom.size();
    hp.m_loc[a] = m;
  }
  // ---- per-atom maps over the basis of its system, column -> system basis
  hp.map_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) hp.map_off[a + 1] = hp.map_off[a] + hp.sys_n[hp.atom_sys[a]];
  hp.map1.assign(hp.map_off[NA], -1);
  hp.map2.assign(hp.map_off[NA], -1);
  hp.col1g_off.assign(NA + 1, 0);
  hp.col2g_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) {
    hp.col1g_off[a + 1] = hp.col1g_off[a] + hp.n_loc[a];
    hp.col2g_off[a + 1] = hp.col2g_off[a] + hp.m_loc[a];
  }
  hp.col1g.assign(hp.col1g_off[NA], 0);
  hp.col2g.assign(hp.col2g_off[NA], 0);
  for (int a = 0; a < NA; ++a) {
    int c = 0;
    for (int k = np[a]; k < np[a + 1]; ++k) {
      int j = nat[k];
      for (int x = 0; x < hp.nb[j]; ++x, ++c) {
        hp.map1[hp.map_off[a] + hp.bo[j] + x] = c;
        hp.col1g[hp.col1g_off[a] + c] = hp.bo[j] + x;
      }
    }
    c = 0;
    for (int k = hp.n2_ptr[a]; k < hp.n2_ptr[a + 1]; ++k) {
      int l = hp.n2_atom[k];
      for (int x = 0; x < hp.nb[l]; ++x, ++c) {
        hp.map2[hp.map_off[a] + hp.bo[l] + x] = c;
        hp.col2g[hp.col2g_off[a] + c] = hp.bo[l] + x;
      }
    }
  }
  // ---- workspace layout
  hp.t_off.assign(NA + 1, 0);
  hp.e_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) {
    int64_t s = (int64_t)hp.na[a] * hp.nb[a];
    hp.t_off[a + 1] = hp.t_off[a] + ceil_to(s * hp.n_loc[a], 2);
    hp.e_off[a + 1] = hp.e_off[a] + ceil_to(s * hp.m_loc[a], 2);
  }
  hp.t_total = hp.t_off[NA];
  hp.e_total = hp.e_off[NA];
  for (auto& f : hp.flops) f = 0;
  for (auto& f : hp.issued) f = 0;
  // ---- block-sparse "rows of P times D" tasks.  E_P = T_P D takes the
  // columns of N[P] as k and produces the columns of N2[P]; the gradient
  // product G_P = H_P D takes N2[P] as k and produces N[P].  Output column
  // tiles of 32; the k-range of a tile is the list of runs of input atoms J
  // with some tile atom in N[J] (D is zero elsewhere).
  int stampv = 0;
  std::vector<int> stamp2(NA, -1), stamp3(NA, -1), colcnt(NA, 0);
  auto rowd_lists = [&](bool grad, std::vector<EItem>& items, std::vector<int>& run_ptr,
                        std::vector<int>& klens, std::vector<Run>& runs, std::vector<uint8_t>& kflag,
                        std::vector<int64_t>& kflag_off, int64_t& issued) {
    items.clear();
    run_ptr.assign(1, 0);
    klens.clear();
    runs.clear();
    kflag.clear();
    kflag_off.assign(1, 0);
    std::vector<KEnt> krow, ccol;
    for (int a = 0; a < NA; ++a) {
      const int sP = hp.na[a] * hp.nb[a];
      // input atoms (k side) and output atoms (column side) with local offsets
      const int* in_b = grad ? &hp.n2_atom[hp.n2_ptr[a]] : &nat[np[a]];
      const int n_in = grad ? hp.n2_ptr[a + 1] - hp.n2_ptr[a] : np[a + 1] - np[a];
      const int* out_b = grad ? &nat[np[a]] : &hp.n2_atom[hp.n2_ptr[a]];
      const int n_out = grad ? np[a + 1] - np[a] : hp.n2_ptr[a + 1] - hp.n2_ptr[a];
      const int mOut = grad ? hp.n_loc[a] : hp.m_loc[a];
      for (int c0 = 0; c0 < mOut; c0 += E_TILE) {
        ++stampv;
        const int c1 = std::min(mOut, c0 + E_TILE);
        int c = 0;
        ccol.clear();
        krow.clear();
        for (int k = 0; k < n_out; ++k) {
          const int l = out_b[k];
          if (c < c1 && c + hp.nb[l] > c0) {
            stamp2[l] = stampv;
            // input atoms J with this tile atom in N[J], i.e. the neighbours of l
            for (int k2 = np[l]; k2 < np[l + 1]; ++k2) stamp3[nat[k2]] = stampv;
            const int b0 = std::max(c, c0), b1 = std::min(c + hp.nb[l], c1);
            ccol.push_back(KEnt{l, 0, b0 - c0, b1 - b0});
          }
          c += hp.nb[l];
          if (c >= c1) break;
        }
        const int ct = (int)klens.size();
        int klen = 0, lcol = 0, prevJ = -2;
        Run cur{-1, -1, 0, 0};
        for (int k = 0; k < n_in; ++k) {
          const int j = in_b[k];
          const bool rel = stamp3[j] == stampv;   // some tile atom in N[j]
          if (rel) {
            if (cur.len > 0 && j == prevJ + 1) {
              cur.len += hp.nb[j];
            } else {
              if (cur.len > 0) runs.push_back(cur);
              cur = Run{lcol, hp.bo[j], hp.nb[j], 0};
            }
            prevJ = j;
            krow.push_back(KEnt{j, 0, klen, hp.nb[j]});
            klen += hp.nb[j];
          } else {
            prevJ = -2;
          }
          lcol += hp.nb[j];
        }
        if (cur.len > 0) runs.push_back(cur);
        run_ptr.push_back((int)runs.size());
        klens.push_back(klen);
        tile_kflags(hp, krow, ccol, klen, kflag);
        kflag_off.push_back((int64_t)kflag.size());
        issued += kflag_issued(kflag.data() + kflag_off[ct], klen, sP);
        for (int r0 = 0; r0 < sP; r0 += E_TILE) items.push_back(EItem{a, r0, c0, ct});
      }
    }
  };
  for (int a = 0; a < NA; ++a) {
    const int sP = hp.na[a] * hp.nb[a];
    int64_t kk = 0;   // structural flops: sum_J b_J sum_{L in N[J]} b_L
    for (int k = np[a]; k < np[a + 1]; ++k) {
      int j = nat[k];
      int64_t sl = 0;
      for (int k2 = np[j]; k2 < np[j + 1]; ++k2) sl += hp.nb[nat[k2]];
      kk += (int64_t)hp.nb[j] * sl;
    }
    hp.flops[1] += 2 * (int64_t)sP * kk;
  }
  rowd_lists(false, hp.e_items, hp.ct_run_ptr, hp.ct_klen, hp.runs, hp.ct_kflag, hp.ct_kflag_off, hp.issued[1]);
  int64_t gd_issued = 0;
  rowd_lists(true, hp.gd_items, hp.gd_run_ptr, hp.gd_klen, hp.gd_runs, hp.gd_kflag, hp.gd_kflag_off, gd_issued);
  // ---- H tasks: atom groups (runs of consecutive, nearby atoms of one
  // system; one wavefront per 16-wide aux tile of each atom) x 16-wide tiles
  // of the group's second-neighbourhood columns.  Q-lists (V (x) D part) and
  // X-lists (G part) carry the pair id of every group atom with Q / X.
  for (int a = 0; a < NA; ++a) {
    const int aP = hp.na[a], bP = hp.nb[a];
    for (int k = np[a]; k < np[a + 1]; ++k) {
      int q = nat[k];
      hp.flops[2] += 2LL * aP * hp.na[q] * hp.nb[q] * hp.n_loc[q];   // F = V T
      hp.flops[2] += 2LL * aP * bP * hp.nb[q] * hp.n_loc[q];          // D contraction
      hp.flops[2] += 2LL * aP * hp.na[q] * bP * hp.nb[q];             // G part
    }
  }
  hp.grp_first.clear();
  hp.grp_unit_ptr.assign(1, 0);
  hp.grp_units.clear();
  hp.grp_col_ptr.assign(1, 0);
  hp.grp_cols.clear();
  hp.g_tiles.clear();
  hp.gq.clear();
  hp.gx.clear();
  hp.h_waves = 1;
  {
    const double gr2 = GROUP_RADIUS * GROUP_RADIUS;
    int a = 0;
    while (a < NA) {
      const int s = hp.atom_sys[a];
      int n = 1, units = (hp.na[a] + 15) / 16;
      while (a + n < NA && n < GROUP_ATOMS && hp.atom_sys[a + n] == s) {
        const int b = a + n;
        const int u = (hp.na[b] + 15) / 16;
        double dx = hp.pos[3 * a] - hp.pos[3 * b], dy = hp.pos[3 * a + 1] - hp.pos[3 * b + 1],
               dz = hp.pos[3 * a + 2] - hp.pos[3 * b + 2];
        if (units + u > GROUP_WAVES || dx * dx + dy * dy + dz * dz > gr2) break;
        units += u;
        ++n;
      }
      const int g = (int)hp.grp_first.size();
      hp.grp_first.push_back(a);
      for (int t = 0; t < n; ++t)
        for (int mu0 = 0; mu0 < hp.na[a + t]; mu0 += 16) hp.grp_units.push_back(Unit{a + t, mu0, t, 0});
      hp.grp_unit_ptr.push_back((int)hp.grp_units.size());
      hp.h_waves = std::max(hp.h_waves, units);
      // union of N2 over the group, as system basis columns
      ++stampv;
      std::vector<int> atoms;
      for (int t = 0; t < n; ++t)
        for (int k = hp.n2_ptr[a + t]; k < hp.n2_ptr[a + t + 1]; ++k) {
          int l = hp.n2_atom[k];
          if (stamp2[l] != stampv) { stamp2[l] = stampv; atoms.push_back(l); }
        }
      std::sort(atoms.begin(), atoms.end());
      const int col0 = (int)hp.grp_cols.size();
      std::vector<int> col_atom;
      for (int l : atoms)
        for (int x = 0; x < hp.nb[l]; ++x) { hp.grp_cols.push_back(hp.bo[l] + x); col_atom.push_back(l); }
      hp.grp_col_ptr.push_back((int)hp.grp_cols.size());
      const int ncol = (int)col_atom.size();
      // neighbours of the group (union of N[P]) with the pair id per group slot
      std::vector<int> nbrs;
      ++stampv;
      for (int t = 0; t < n; ++t)
        for (int k = np[a + t]; k < np[a + t + 1]; ++k)
          if (stamp2[nat[k]] != stampv) { stamp2[nat[k]] = stampv; nbrs.push_back(nat[k]); }
      std::sort(nbrs.begin(), nbrs.end());
      // the list entry of every neighbour (pair ids per group slot), formed once per group
      std::vector<Slot4> nbr_slots(nbrs.size());
      for (size_t i = 0; i < nbrs.size(); ++i) {
        const int q = nbrs[i];
        Slot4 e{q, -1, -1, -1};
        int* sl = &e.p0;
        for (int t = 0; t < n; ++t) {
          auto it = std::lower_bound(nat.begin() + np[a + t], nat.begin() + np[a + t + 1], q);
          if (it != nat.begin() + np[a + t + 1] && *it == q) sl[t] = hp.nbr_pair[it - nat.begin()];
        }
        nbr_slots[i] = e;
      }
      for (int c0 = 0; c0 < ncol; c0 += H_COLS) {
        const int c1 = std::min(ncol, c0 + H_COLS);
        ++stampv;
        for (int c = c0; c < c1; ++c) {
          const int l = col_atom[c];
          int ncl = 1;   // tile columns on l (consecutive)
          while (c + ncl < c1 && col_atom[c + ncl] == l) ++ncl;
          stamp2[l] = stampv;
          for (int k2 = np[l]; k2 < np[l + 1]; ++k2) {   // Q with l in N[Q]
            const int q = nat[k2];
            if (stamp3[q] != stampv) { stamp3[q] = stampv; colcnt[q] = 0; }
            colcnt[q] += ncl;                              // tile columns present in N[q]
          }
          c += ncl - 1;
        }
        GTile tl{};
        tl.grp = g;
        tl.col_beg = col0 + c0;
        tl.ncols = c1 - c0;
        tl.q_beg = (int)hp.gq.size();
        tl.x_beg = (int)hp.gx.size();
        for (size_t i = 0; i < nbrs.size(); ++i) {
          const int q = nbrs[i];
          if (stamp3[q] == stampv) hp.gq.push_back(nbr_slots[i]);   // a tile column in N[q]
          if (stamp2[q] == stampv) hp.gx.push_back(nbr_slots[i]);
        }
        tl.q_end = (int)hp.gq.size();
        tl.x_end = (int)hp.gx.size();
        for (int e = tl.q_beg; e < tl.q_end; ++e) {
          const int q = hp.gq[e].atom;
          const int* sl = &hp.gq[e].p0;
          const int cq = colcnt[q];   // tile columns present in N[Q]
          for (int t = 0; t < n; ++t)
            if (sl[t] >= 0)
              hp.issued[2] += 2048LL * ((hp.na[a + t] + 15) / 16) * cq *
                              (((hp.na[q] + 3) / 4) + ((hp.nb[q] + 3) / 4));
        }
        for (int e = tl.x_beg; e < tl.x_end; ++e) {
          const int x = hp.gx[e].atom;
          const int* sl = &hp.gx[e].p0;
          int cx = 0;
          for (int c = c0; c < c1; ++c) cx += (col_atom[c] == x);
          for (int t = 0; t < n; ++t)
            if (sl[t] >= 0) hp.issued[2] += 2048LL * ((hp.na[a + t] + 15) / 16) * cx * ((hp.na[x] + 3) / 4);
        }
        hp.g_tiles.push_back(tl);
      }
      a += n;
    }
  }
  // ---- T2 tasks: every canonical pair, oriented (bit 0) so that the atom
  // with fewer 16-wide aux tiles is the row side P (less MFMA padding)
  hp.t2_items.resize(npairs);
  for (int64_t p = 0; p < npairs; ++p) {
    int a = hp.pair_a[p], b = hp.pair_b[p];
    auto cost = [&](int x, int y) {
      return (int64_t)((hp.na[x] + 15) / 16) * (((hp.na[y] + 3) / 4) + 4) * hp.n_loc[y];
    };
    const bool flip = cost(b, a) < cost(a, b);
    if (flip) std::swap(a, b);
    hp.t2_items[p] = (int)(2 * p + (flip ? 1 : 0));
    hp.flops[3] += 2LL * hp.na[a] * hp.na[b] * hp.nb[b] * hp.n_loc[b] + 2LL * hp.na[a] * hp.nb[a] * hp.nb[b] * hp.n_loc[b];
    hp.issued[3] += 2048LL * cost(a, b);
  }
  hp.t2col_off.assign(npairs + 1, 0);
  hp.t2col.clear();
  for (int64_t p = 0; p < npairs; ++p) {
    const int item = hp.t2_items[p];
    const int a = (item & 1) ? hp.pair_b[p] : hp.pair_a[p], b = (item & 1) ? hp.pair_a[p] : hp.pair_b[p];
    for (int l = 0; l < hp.n_loc[b]; ++l)
      hp.t2col.push_back(hp.map2[hp.map_off[a] + hp.col1g[hp.col1g_off[b] + l]]);
    hp.t2col_off[p + 1] = (int64_t)hp.t2col.size();
  }
  // shape classes: aux tiles of 16 of the row atom, nu steps of 4 (rounded up
  // to a compiled size) of the column atom; inside a class the items of one column atom Q
  // are consecutive, so the workgroups of one XCD (consecutive items) share T_Q in its L2
  {
    auto ns_class = [](int ns) { return ns <= 4 ? 4 : ns <= 8 ? 8 : ns <= 10 ? 10 : ns <= 12 ? 12 : 16; };
    auto key = [&](int item) {
      const int p = item >> 1;
      const bool flip = item & 1;
      const int a = flip ? hp.pair_b[p] : hp.pair_a[p], b = flip ? hp.pair_a[p] : hp.pair_b[p];
      return ((hp.na[a] + 15) / 16) * 64 + ns_class((hp.na[b] + 3) / 4);
    };
    auto col_atom = [&](int item) { return (item & 1) ? hp.pair_a[item >> 1] : hp.pair_b[item >> 1]; };
    std::stable_sort(hp.t2_items.begin(), hp.t2_items.end(), [&](int x, int y) {
      return key(x) != key(y) ? key(x) < key(y) : col_atom(x) < col_atom(y);
    });
    hp.t2_classes.clear();
    for (int i = 0; i < (int)hp.t2_items.size(); ++i) {
      const int k = key(hp.t2_items[i]);
      if (hp.t2_classes.empty() || hp.t2_classes.back().nt * 64 + hp.t2_classes.back().ns != k)
        hp.t2_classes.push_back(T2Class{k / 64, k % 64, i, i, 0});
      hp.t2_classes.back().end = i + 1;
    }
  }
  // ---- dV tasks: canonical pairs grouped by shape (aux tiles of 16 of P and
  // Q, basis steps of 4 of Q and P); stable order inside a class
  {
    auto key = [&](int p) {
      const int a = hp.pair_a[p], b = hp.pair_b[p];
      return (((hp.na[a] + 15) / 16) * 8 + (hp.na[b] + 15) / 16) * 64 + ((hp.nb[b] + 3) / 4) * 8 + (hp.nb[a] + 3) / 4;
    };
    hp.dv_items.resize(npairs);
    for (int64_t p = 0; p < npairs; ++p) hp.dv_items[p] = (int)p;
    // pairs of one second atom Q consecutive inside a class (T_Q shared in an XCD's L2)
    std::stable_sort(hp.dv_items.begin(), hp.dv_items.end(), [&](int x, int y) {
      return key(x) != key(y) ? key(x) < key(y) : hp.pair_b[x] < hp.pair_b[y];
    });
    hp.dv_classes.clear();
    for (int i = 0; i < (int)hp.dv_items.size(); ++i) {
      const int k = key(hp.dv_items[i]);
      if (hp.dv_classes.empty() || i == 0 || key(hp.dv_items[i - 1]) != k)
        hp.dv_classes.push_back(DVClass{k / 512, (k / 64) % 8, (k / 8) % 8, k % 8, i, i});
      hp.dv_classes.back().end = i + 1;
    }
  }
  hp.dvcol_off.assign(npairs + 1, 0);
  hp.dvcol.clear();
  hp.dv_cp.assign(npairs, 0);
  hp.dv_cq.assign(npairs, 0);
  for (int64_t p = 0; p < npairs; ++p) {
    const int a = hp.pair_a[p], b = hp.pair_b[p];
    for (int l = 0; l < hp.n_loc[b]; ++l) hp.dvcol.push_back(hp.map2[hp.map_off[a] + hp.col1g[hp.col1g_off[b] + l]]);
    hp.dvcol_off[p + 1] = (int64_t)hp.dvcol.size();
    hp.dv_cp[p] = hp.map2[hp.map_off[a] + hp.bo[b]];
    hp.dv_cq[p] = hp.map2[hp.map_off[b] + hp.bo[a]];
  }
  // ---- final tasks: 32 x 32 tile pairs (upper triangle) with their P-lists
  hp.f_items.clear();
  hp.f_plist.clear();
  std::vector<std::pair<int64_t, int>> fcost;
  std::vector<FItem> fit;
  for (int s = 0; s < hp.n_sys; ++s) {
    const int lo = hp.sys_atom_off[s], hi = hp.sys_atom_off[s + 1];
    const int nt = (int)((hp.sys_n[s] + 31) / 32);
    std::vector<std::vector<int>> lists((size_t)nt * nt);
    std::vector<int> t1, t2;
    for (int a = lo; a < hi; ++a) {
      const int64_t sP = (int64_t)hp.na[a] * hp.nb[a];
      hp.flops[4] += 2LL * hp.n_loc[a] * sP * hp.m_loc[a];
      t1.clear();
      t2.clear();
      for (int k = np[a]; k < np[a + 1]; ++k) {
        int j = nat[k];
        for (int t = hp.bo[j] / 32; t <= (hp.bo[j] + hp.nb[j] - 1) / 32; ++t) t1.push_back(t);
      }
      for (int k = hp.n2_ptr[a]; k < hp.n2_ptr[a + 1]; ++k) {
        int l = hp.n2_atom[k];
        for (int t = hp.bo[l] / 32; t <= (hp.bo[l] + hp.nb[l] - 1) / 32; ++t) t2.push_back(t);
      }
      std::sort(t1.begin(), t1.end());
      t1.erase(std::unique(t1.begin(), t1.end()), t1.end());
      std::sort(t2.begin(), t2.end());
      t2.erase(std::unique(t2.begin(), t2.end()), t2.end());
      for (int x : t1)
        for (int y : t2) {
          int i = std::min(x, y), l = std::max(x, y);
          auto& v = lists[(size_t)i * nt + l];
          if (v.empty() || v.back() != a) v.push_back(a);
        }
    }
    for (int i = 0; i < nt; ++i)
      for (int l = i; l < nt; ++l) {
        auto& v = lists[(size_t)i * nt + l];
        if (v.empty()) continue;
        FItem f{};
        f.sys = s;
        f.gI0 = 32 * i;
        f.gL0 = 32 * l;
        f.pbeg = (int)hp.f_plist.size();
        int64_t cost = 0;
        for (int a : v) { hp.f_plist.push_back(a); cost += (int64_t)hp.na[a] * hp.nb[a]; }
        f.pend = (int)hp.f_plist.size();

        fcost.push_back({cost, (int)fit.size()});
        fit.push_back(f);
      }
  }
  std::stable_sort(fcost.begin(), fcost.end(), [](auto& x, auto& y) { return x.first > y.first; });
  for (auto& c : fcost) hp.f_items.push_back(fit[c.second]);
  // ---- Y_P = T_P^T H'_P tiles (64 x 64), P-major for L2 locality
  hp.y_off.assign(NA + 1, 0);
  hp.y_tiles.clear();
  for (int a = 0; a < NA; ++a) {
    hp.y_off[a + 1] = hp.y_off[a] + ceil_to((int64_t)hp.n_loc[a] * hp.m_loc[a], 2);
    for (int n0 = 0; n0 < hp.m_loc[a]; n0 += 64)
      for (int m0 = 0; m0 < hp.n_loc[a]; m0 += 64) hp.y_tiles.push_back(YTile{a, m0, n0, 0});
  }
  hp.y_total = hp.y_off[NA];
  hp.issued[4] = 0;
  for (const auto& t : hp.y_tiles) hp.issued[4] += 2LL * 64 * 64 * ceil_to((int64_t)hp.na[t.P] * hp.nb[t.P], 16);
  // ---- energy chunks: runs of at most EN_PAIRS canonical pairs of one system
  hp.en_sys.clear();
  hp.en_pbeg.clear();
  hp.en_pend.clear();
  for (int64_t p = 0; p < npairs;) {
    const int s = hp.atom_sys[hp.pair_a[p]];
    int64_t q = p + 1;
    while (q < npairs && q - p < EN_PAIRS && hp.atom_sys[hp.pair_a[q]] == s) ++q;
    hp.en_sys.push_back(s);
    hp.en_pbeg.push_back((int)p);
    hp.en_pend.push_back((int)q);
    p = q;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Mixed precision: the V-stage Q- and X-lists and the T2 pairs are split by
// atom-pair distance.  Pairs at or beyond the split (their V block, C blocks
// and D blocks all decay with distance) go to the binary32 kernels, the rest
// stay binary64.  The V stage runs the near lists as the storing launch (every
// tile, so every H' entry is written) and the far lists as an accumulating
// launch (tiles with no far pair dropped).
void derive_mixed_lists(HostPlan& hp, int set) {
  MixedSet& m = hp.mixed[set];
  const int NA = hp.n_atoms;
  const int64_t npairs = (int64_t)hp.pair_a.size();
  const std::vector<int>& np = hp.nbr_ptr;
  const std::vector<int>& nat = hp.nbr_atom;
  const double s2 = m.split * m.split;
  std::vector<char> far(npairs, 0);
  for (int64_t p = 0; p < npairs; ++p) {
    const double* pa = &hp.pos[3 * (size_t)hp.pair_a[p]];
    double pb[3] = {hp.pos[3 * (size_t)hp.pair_b[p]], hp.pos[3 * (size_t)hp.pair_b[p] + 1],
                    hp.pos[3 * (size_t)hp.pair_b[p] + 2]};
    if (hp.periodic) {
      double sh[3];
      image_shift(hp.lat, hp.pair_img[p], sh);
      for (int c = 0; c < 3; ++c) pb[c] += sh[c];
    }
    volatile double dx = pa[0] - pb[0], dy = pa[1] - pb[1], dz = pa[2] - pb[2];
    volatile double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    volatile double r2 = (xx + yy);
    r2 = r2 + zz;
    far[p] = (m.split <= 0.0) || (r2 >= s2);
  }
  for (int i = 0; i < 5; ++i) m.flops32[i] = m.issued32[i] = m.issued64[i] = 0;
  // algorithmic binary32 flops of the V stage (ordered pairs) and T2
  for (int a = 0; a < NA; ++a) {
    const int aP = hp.na[a], bP = hp.nb[a];
    for (int k = np[a]; k < np[a + 1]; ++k) {
      const int q = nat[k];
      if (!far[hp.nbr_pair[k]]) continue;
      m.flops32[2] += 2LL * aP * hp.na[q] * hp.nb[q] * hp.n_loc[q] + 2LL * aP * bP * hp.nb[q] * hp.n_loc[q] +
                      2LL * aP * hp.na[q] * bP * hp.nb[q];
    }
  }
  // atom of a basis column of a system
  auto col_atom = [&](int s, int col) {
    const int lo = hp.sys_atom_off[s], hi = hp.sys_atom_off[s + 1];
    int l = lo, h = hi - 1;
    while (l < h) {
      const int mm = (l + h + 1) / 2;
      if (hp.bo[mm] <= col) l = mm; else h = mm - 1;
    }
    return l;
  };
  m.tiles_near.clear();
  m.tiles_far.clear();
  m.far_src.clear();
  m.q_near.clear();
  m.x_near.clear();
  m.q_far.clear();
  m.x_far.clear();
  std::vector<int> catom;
  for (size_t ti = 0; ti < hp.g_tiles.size(); ++ti) {
    const GTile& t = hp.g_tiles[ti];
    const int a = hp.grp_first[t.grp];
    const int s = hp.atom_sys[a];
    catom.resize(t.ncols);
    for (int c = 0; c < t.ncols; ++c) catom[c] = col_atom(s, hp.grp_cols[t.col_beg + c]);
    GTile tn = t, tf = t;
    tn.q_beg = (int)m.q_near.size();
    tf.q_beg = (int)m.q_far.size();
    tn.x_beg = (int)m.x_near.size();
    tf.x_beg = (int)m.x_far.size();
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<Slot4>& src = pass == 0 ? hp.gq : hp.gx;
      const int e0 = pass == 0 ? t.q_beg : t.x_beg, e1 = pass == 0 ? t.q_end : t.x_end;
      for (int e = e0; e < e1; ++e) {
        const Slot4& x = src[e];
        const int q = x.atom;
        int cnt = 0;   // tile columns this entry touches: in N[Q] (Q part) or on X (G part)
        for (int c = 0; c < t.ncols; ++c)
          cnt += pass == 0 ? std::binary_search(nat.begin() + np[q], nat.begin() + np[q + 1], catom[c])
                           : (catom[c] == q);
        // MFMAs per column and aux tile: F chain + D chain (the binary32 kernel
        // always runs all four D steps) or the G chain
        const int per = pass == 0 ? ((hp.na[q] + 3) / 4) + ((hp.nb[q] + 3) / 4) : (hp.na[q] + 3) / 4;
        const int per32 = pass == 0 ? ((hp.na[q] + 3) / 4) + 4 : per;
        Slot4 n4 = x, f4 = x;   // keeps the entry's image and E columns (periodic plans)
        n4.p0 = n4.p1 = n4.p2 = f4.p0 = f4.p1 = f4.p2 = -1;
        const int* sl = &x.p0;
        int* sn = &n4.p0;
        int* sf = &f4.p0;
        bool anyn = false, anyf = false;
        for (int k = 0; k < GROUP_ATOMS; ++k) {
          if (sl[k] < 0) continue;
          const int64_t fl = 2048LL * ((hp.na[a + k] + 15) / 16) * cnt;
          if (far[sl[k]]) { sf[k] = sl[k]; anyf = true; m.issued32[2] += fl * per32; }
          else { sn[k] = sl[k]; anyn = true; m.issued64[2] += fl * per; }
        }
        if (anyn) (pass == 0 ? m.q_near : m.x_near).push_back(n4);
        if (anyf) (pass == 0 ? m.q_far : m.x_far).push_back(f4);
      }
    }
    tn.q_end = (int)m.q_near.size();
    tf.q_end = (int)m.q_far.size();
    tn.x_end = (int)m.x_near.size();
    tf.x_end = (int)m.x_far.size();
    m.tiles_near.push_back(tn);
    if (tf.q_end > tf.q_beg || tf.x_end > tf.x_beg) {
      m.tiles_far.push_back(tf);
      m.far_src.push_back((int)ti);
    }
  }
  // T2: the full list's order (shape classes) kept inside each precision
  m.t2_items.clear();
  m.t2_classes.clear();
  for (int prec = 0; prec < 2; ++prec) {
    for (const T2Class& c : hp.t2_classes) {
      const int beg = (int)m.t2_items.size();
      for (int i = c.beg; i < c.end; ++i) {
        const int item = hp.t2_items[i];
        const int p = item >> 1;
        if (far[p] != (prec == 1)) continue;
        m.t2_items.push_back(item);
        const bool flip = item & 1;
        const int x = flip ? hp.pair_b[p] : hp.pair_a[p], y = flip ? hp.pair_a[p] : hp.pair_b[p];
        const int64_t iss = 2048LL * ((hp.na[x] + 15) / 16) * (((hp.na[y] + 3) / 4) + 4) * hp.n_loc[y];
        if (prec == 1) {
          m.flops32[3] += 2LL * hp.na[x] * hp.na[y] * hp.nb[y] * hp.n_loc[y] +
                          2LL * hp.na[x] * hp.nb[x] * hp.nb[y] * hp.n_loc[y];
          m.issued32[3] += iss;
        } else {
          m.issued64[3] += iss;
        }
      }
      const int end = (int)m.t2_items.size();
      if (end > beg) m.t2_classes.push_back(T2Class{c.nt, c.ns, beg, end, prec});
    }
  }
  // per chunk: the items whose row atom the chunk owns, class by class
  m.chunk_t2_items.assign(hp.chunks.size(), {});
  m.chunk_t2_classes.assign(hp.chunks.size(), {});
  for (size_t ci = 0; ci < hp.chunks.size(); ++ci) {
    const ChunkHost& ch = hp.chunks[ci];
    auto& items = m.chunk_t2_items[ci];
    auto& cls = m.chunk_t2_classes[ci];
    for (const T2Class& c : m.t2_classes) {
      const int beg = (int)items.size();
      for (int i = c.beg; i < c.end; ++i) {
        const int item = m.t2_items[i], p = item >> 1;
        const int row = (item & 1) ? hp.pair_b[p] : hp.pair_a[p];
        if (row >= ch.a0 && row < ch.a1) items.push_back(item);
      }
      if ((int)items.size() > beg) cls.push_back(T2Class{c.nt, c.ns, beg, (int)items.size(), c.prec});
    }
  }
  for (int i : {0, 1, 4}) m.issued64[i] = hp.issued[i];
  m.ready = true;
}

// ---------------------------------------------------------------------------
// Workspace-bounded plans.  A chunk owns whole V-stage groups, i.e. a range
// [a0, a1) of consecutive aux atoms P: their H'_P (V stage) and Y_P (final
// product) are formed in the chunk, and their T2 blocks (row atom P) and dV
// pairs (first atom P) are computed there.  The V stage's G part reads E_X of
// the neighbours X of P and the dV pairs read E_Q, so each chunk computes E for
// its atoms and their neighbours: E of an atom near a chunk boundary is
// recomputed by every chunk that needs it.
// The X' terms of a chunk of a periodic plan: the pattern tiles keep their entries
// whose P is one of the chunk's aux atoms (tiles left without entries are dropped, the
// shape classes formed again), and the per-pair gather keeps its terms of those P.
// X' is linear in the terms over P, so the chunks' parts add up to the whole.
static void chunk_pattern_lists(const HostPlan& hp, ChunkHost& ch) {
  auto own = [&](int P) { return P >= ch.a0 && P < ch.a1; };
  for (const PTClass& c : hp.pt_classes) {
    const int tb = (int)ch.pt_tiles.size();
    for (int i = c.beg; i < c.end; ++i) {
      PTile t = hp.pt_tiles[i];
      const int eb = (int)ch.pt_ent.size();
      for (int e = t.e_beg; e < t.e_end; ++e)
        if (own(hp.pt_ent[e].P)) ch.pt_ent.push_back(hp.pt_ent[e]);
      if ((int)ch.pt_ent.size() == eb) continue;
      t.e_beg = eb;
      t.e_end = (int)ch.pt_ent.size();
      ch.pt_tiles.push_back(t);
    }
    if ((int)ch.pt_tiles.size() > tb) ch.pt_classes.push_back(PTClass{c.ta, c.tb, tb, (int)ch.pt_tiles.size()});
  }
  const size_t npairs = hp.pg_beg.size();
  ch.pg_beg.assign(npairs, 0);
  ch.pg_mid.assign(npairs, 0);
  ch.pg_end.assign(npairs, 0);
  for (int p : hp.pg_pairs) {
    ch.pg_beg[p] = (int)ch.pg_ent.size();
    for (int i = hp.pg_beg[p]; i < hp.pg_mid[p]; ++i)
      if (own(hp.pg_ent[i].P)) ch.pg_ent.push_back(hp.pg_ent[i]);
    ch.pg_mid[p] = (int)ch.pg_ent.size();
    for (int i = hp.pg_mid[p]; i < hp.pg_end[p]; ++i)
      if (own(hp.pg_ent[i].P)) ch.pg_ent.push_back(hp.pg_ent[i]);
    ch.pg_end[p] = (int)ch.pg_ent.size();
    if (ch.pg_end[p] > ch.pg_beg[p]) ch.pg_pairs.push_back(p);
  }
}

int derive_chunks(HostPlan& hp, int64_t budget, std::string& err) {
  const int NA = hp.n_atoms;
  hp.chunks.clear();
  hp.ws_budget = budget;
  const int64_t stored = (int64_t)sizeof(double) * (2 * hp.e_total + hp.y_total);
  hp.inter_stored = stored;
  hp.ws_total = 2 * hp.e_total + hp.y_total;
  if (budget <= 0 || stored <= budget) return 0;
  const auto& np = hp.nbr_ptr;
  const auto& nat = hp.nbr_atom;
  auto esz = [&](int a) { return hp.e_off[a + 1] - hp.e_off[a]; };
  auto ysz = [&](int a) { return hp.y_off[a + 1] - hp.y_off[a]; };
  const int NG = (int)hp.grp_first.size();
  auto grp_end = [&](int g) { return g + 1 < NG ? hp.grp_first[g + 1] : NA; };
  std::vector<int> stamp(NA, -1);
  std::vector<std::pair<int, int>> ranges;   // groups [g0, g1)
  int g = 0;
  while (g < NG) {
    const int tag = (int)ranges.size();
    int64_t e_d = 0, hy_d = 0;   // doubles: E of the E atoms, H' + Y of the owned atoms
    int g1 = g;
    while (g1 < NG) {
      int64_t de = 0, dhy = 0;
      std::vector<int> added;
      for (int a = hp.grp_first[g1]; a < grp_end(g1); ++a) {
        dhy += esz(a) + ysz(a);
        for (int k = np[a]; k < np[a + 1]; ++k)
          if (stamp[nat[k]] != tag) { stamp[nat[k]] = tag; added.push_back(nat[k]); de += esz(nat[k]); }
      }
      if ((int64_t)sizeof(double) * (e_d + de + hy_d + dhy) > budget && g1 > g) {
        for (int x : added) stamp[x] = -1;   // not taken: undo
        break;
      }
      if ((int64_t)sizeof(double) * (e_d + de + hy_d + dhy) > budget) {
        err = "exx_plan_create: ws_budget_bytes is smaller than the workspace of one V-stage group (" +
              std::to_string((int64_t)sizeof(double) * (e_d + de + hy_d + dhy)) + " bytes)";
        hp.chunks.clear();
        return -2;
      }
      e_d += de;
      hy_d += dhy;
      ++g1;
    }
    ranges.push_back({g, g1});
    g = g1;
  }
  hp.ws_total = 0;
  std::vector<char> in_e(NA);
  for (const auto& r : ranges) {
    ChunkHost ch;
    ch.g0 = r.first;
    ch.g1 = r.second;
    ch.a0 = hp.grp_first[ch.g0];
    ch.a1 = grp_end(ch.g1 - 1);
    std::fill(in_e.begin(), in_e.end(), 0);
    for (int a = ch.a0; a < ch.a1; ++a)
      for (int k = np[a]; k < np[a + 1]; ++k) in_e[nat[k]] = 1;
    ch.e_off.assign(NA + 1, 0);
    ch.h_off.assign(NA + 1, 0);
    ch.y_off.assign(NA + 1, 0);
    for (int a = 0; a < NA; ++a) {
      if (in_e[a]) { ch.e_off[a] = ch.e_total; ch.e_total += esz(a); }
      if (a >= ch.a0 && a < ch.a1) {
        ch.h_off[a] = ch.h_total; ch.h_total += esz(a);
        ch.y_off[a] = ch.y_total; ch.y_total += ysz(a);
      }
    }
    for (const EItem& it : hp.e_items)
      if (in_e[it.P]) ch.e_items.push_back(it);
    // ranges of the lists kept in group / atom order
    ch.gt_beg = (int)(std::lower_bound(hp.g_tiles.begin(), hp.g_tiles.end(), ch.g0,
                                       [](const GTile& t, int x) { return t.grp < x; }) - hp.g_tiles.begin());
    ch.gt_end = (int)(std::lower_bound(hp.g_tiles.begin(), hp.g_tiles.end(), ch.g1,
                                       [](const GTile& t, int x) { return t.grp < x; }) - hp.g_tiles.begin());
    auto atom_range = [&](const auto& v, int& b, int& e) {
      b = (int)(std::lower_bound(v.begin(), v.end(), ch.a0, [](const auto& t, int x) { return t.P < x; }) - v.begin());
      e = (int)(std::lower_bound(v.begin(), v.end(), ch.a1, [](const auto& t, int x) { return t.P < x; }) - v.begin());
    };
    atom_range(hp.y_tiles, ch.y_beg, ch.y_end);
    atom_range(hp.gd_items, ch.gd_beg, ch.gd_end);
    // T2 items with their row atom in the chunk, class by class
    for (const T2Class& c : hp.t2_classes) {
      const int beg = (int)ch.t2_items.size();
      for (int i = c.beg; i < c.end; ++i) {
        const int item = hp.t2_items[i], p = item >> 1;
        const int row = (item & 1) ? hp.pair_b[p] : hp.pair_a[p];
        if (row >= ch.a0 && row < ch.a1) ch.t2_items.push_back(item);
      }
      if ((int)ch.t2_items.size() > beg) ch.t2_classes.push_back(T2Class{c.nt, c.ns, beg, (int)ch.t2_items.size(), 0});
    }
    for (const DVClass& c : hp.dv_classes) {
      const int beg = (int)ch.dv_items.size();
      for (int i = c.beg; i < c.end; ++i)
        if (hp.pair_a[hp.dv_items[i]] >= ch.a0 && hp.pair_a[hp.dv_items[i]] < ch.a1) ch.dv_items.push_back(hp.dv_items[i]);
      if ((int)ch.dv_items.size() > beg) {
        DVClass d = c;
        d.beg = beg;
        d.end = (int)ch.dv_items.size();
        ch.dv_classes.push_back(d);
      }
    }
    // gather tiles: the P-lists restricted to the chunk's atoms
    for (const FItem& f : hp.f_items) {
      FItem x = f;
      x.pbeg = (int)ch.f_plist.size();
      for (int i = f.pbeg; i < f.pend; ++i)
        if (hp.f_plist[i] >= ch.a0 && hp.f_plist[i] < ch.a1) ch.f_plist.push_back(hp.f_plist[i]);
      x.pend = (int)ch.f_plist.size();
      if (x.pend > x.pbeg) ch.f_items.push_back(x);
    }
    if (hp.periodic) chunk_pattern_lists(hp, ch);
    hp.ws_total = std::max(hp.ws_total, ch.e_total + ch.h_total + ch.y_total);
    hp.chunks.push_back(std::move(ch));
  }
  return 0;
}

}  // namespace exx
