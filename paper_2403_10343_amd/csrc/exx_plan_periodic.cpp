// Host-side lists of a periodic plan.  The real-space exchange couples a
// function in the home cell with functions in every cell n (Sec. "Description
// of the real-space formalism", Eq. realspace_exchange with lattice vectors);
// by translation symmetry all blocks are those of home-cell atom pairs at a
// relative image.  With the cutoff below half the cell width an atom pair has
// at most one image within the cutoff, so C, V, D and the returned X keep the
// layouts of a cluster (the dense (A, B) block of D and X holds the pair's
// block at that image), while the intermediates are indexed by image-labelled
// atoms: N[P] holds each neighbour once with its image, N2[P] may hold an atom
// at several images, and every column map below is keyed by (atom, image).
#include "exx_internal.h"

#include <algorithm>
#include <cmath>

namespace exx {

namespace {

int64_t ceil_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t ekey(int atom, int img) { return (int64_t)atom * 4096 + img; }
inline int img_comp(int code, int c) { return (code / (c == 0 ? 1 : c == 1 ? IMG_S : IMG_S * IMG_S)) % IMG_S - IMG_OFF; }

}  // namespace

void image_shift(const double* lat, int code, double* s) {
  const int n0 = img_comp(code, 0), n1 = img_comp(code, 1), n2 = img_comp(code, 2);
  for (int c = 0; c < 3; ++c) {
    volatile double x = n0 * lat[c];
    volatile double y = n1 * lat[3 + c];
    volatile double z = n2 * lat[6 + c];
    volatile double xy = x + y;
    s[c] = xy + z;
  }
}

#pragma clang fp contract(off)
void host_neighbors_periodic(HostPlan& hp) {
  const double rc2 = hp.r_cut * hp.r_cut;
  const int NA = hp.n_atoms;
  hp.nbr_ptr.assign(NA + 1, 0);
  hp.nbr_atom.clear();
  hp.nbr_img.clear();
  double sh[27][3];
  int codes[27];
  for (int t = 0; t < 27; ++t) {
    codes[t] = img_code(t / 9 - 1, (t / 3) % 3 - 1, t % 3 - 1);
    image_shift(hp.lat, codes[t], sh[t]);
  }
  for (int a = 0; a < NA; ++a) {
    const double* pa = &hp.pos[3 * (size_t)a];
    for (int b = 0; b < NA; ++b) {
      const double* pb = &hp.pos[3 * (size_t)b];
      for (int t = 0; t < 27; ++t) {
        if (a == b && codes[t] != IMG0) continue;
        volatile double bx = pb[0] + sh[t][0], by = pb[1] + sh[t][1], bz = pb[2] + sh[t][2];
        volatile double dx = bx - pa[0], dy = by - pa[1], dz = bz - pa[2];
        volatile double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        volatile double r2 = (xx + yy);
        r2 = r2 + zz;
        if (r2 <= rc2) {
          hp.nbr_atom.push_back(b);
          hp.nbr_img.push_back(codes[t]);
          break;   // at most one image within the cutoff
        }
      }
    }
    hp.nbr_ptr[a + 1] = (int)hp.nbr_atom.size();
  }
}

int derive_lists_periodic(HostPlan& hp, std::string& err) {
  const int NA = hp.n_atoms;
  const auto& np = hp.nbr_ptr;
  const auto& nat = hp.nbr_atom;
  const auto& nim = hp.nbr_img;
  const int64_t nn = np[NA];
  if ((int64_t)nim.size() != nn) { err = "periodic neighbour lists without images"; return -3; }
  // image of B within r_cut of A (dense atom table) and the self entries
  hp.pimg.assign((size_t)NA * NA, -1);
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k) hp.pimg[(size_t)a * NA + nat[k]] = nim[k];
  for (int a = 0; a < NA; ++a)
    if (hp.pimg[(size_t)a * NA + a] != IMG0) { err = "neighbour list lost an atom's self pair"; return -3; }
  // ---- canonical pairs (A <= B, lexicographic): the image of B within r_cut of A
  hp.nbr_pair.assign(nn, -1);
  hp.nbr_owner.assign(nn, 0);
  hp.pair_a.clear();
  hp.pair_b.clear();
  hp.pair_img.clear();
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k) {
      hp.nbr_owner[k] = a;
      if (nat[k] >= a) {
        hp.nbr_pair[k] = (int)hp.pair_a.size();
        hp.pair_a.push_back(a);
        hp.pair_b.push_back(nat[k]);
        hp.pair_img.push_back(nim[k]);
      }
    }
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k)
      if (nat[k] < a) {
        const int b = nat[k];
        auto it = std::lower_bound(nat.begin() + np[b], nat.begin() + np[b + 1], a);
        if (it == nat.begin() + np[b + 1] || *it != a || nim[it - nat.begin()] != img_neg(nim[k])) {
          err = "periodic neighbour list not symmetric";
          return -3;
        }
        hp.nbr_pair[k] = hp.nbr_pair[it - nat.begin()];
      }
  const int64_t npairs = (int64_t)hp.pair_a.size();
  hp.c_off.assign(npairs + 1, 0);
  hp.v_off.assign(npairs + 1, 0);
  for (int64_t p = 0; p < npairs; ++p) {
    const int a = hp.pair_a[p], b = hp.pair_b[p];
    const int64_t cs = (a == b) ? (int64_t)hp.na[a] * hp.nb[a] * hp.nb[a]
                                : (int64_t)(hp.na[a] + hp.na[b]) * hp.nb[a] * hp.nb[b];
    hp.c_off[p + 1] = hp.c_off[p] + cs;
    hp.v_off[p + 1] = hp.v_off[p] + (int64_t)hp.na[a] * hp.na[b];
  }
  // ---- T_P columns: the N[P] entries (one per atom)
  hp.nbr_lcol.assign(nn, 0);
  hp.n_loc.assign(NA, 0);
  for (int a = 0; a < NA; ++a) {
    int c = 0;
    for (int k = np[a]; k < np[a + 1]; ++k) { hp.nbr_lcol[k] = c; c += hp.nb[nat[k]]; }
    hp.n_loc[a] = c;
  }
  // ---- N2[P]: (L, m + n_JL) over the entries (J, m) of N[P], sorted by (atom, image)
  hp.n2_ptr.assign(NA + 1, 0);
  hp.n2_atom.clear();
  hp.n2_img.clear();
  hp.m_loc.assign(NA, 0);
  // N2 entry lookup: n2first[P * NA + L] = first entry of atom L in N2[P] (entries sorted by
  // (atom, image), an atom at most a few images), n2loc[entry] = its first E_P column
  std::vector<int> n2first((size_t)NA * NA, -1), n2loc;
  {
    std::vector<int64_t> keys;
    for (int a = 0; a < NA; ++a) {
      keys.clear();
      for (int k = np[a]; k < np[a + 1]; ++k) {
        const int j = nat[k], m = nim[k];
        for (int k2 = np[j]; k2 < np[j + 1]; ++k2) keys.push_back(ekey(nat[k2], img_add(m, nim[k2])));
      }
      std::sort(keys.begin(), keys.end());
      keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
      int c = 0;
      for (int64_t key : keys) {
        const int l = (int)(key / 4096), im = (int)(key % 4096);
        if (n2first[(size_t)a * NA + l] < 0) n2first[(size_t)a * NA + l] = (int)hp.n2_atom.size();
        hp.n2_atom.push_back(l);
        hp.n2_img.push_back(im);
        n2loc.push_back(c);
        c += hp.nb[l];
      }
      hp.n2_ptr[a + 1] = (int)hp.n2_atom.size();
      hp.m_loc[a] = c;
    }
  }
  // first E_P column of atom l at image im in N2[P], or -1
  auto n2col = [&](int P, int l, int im) {
    for (int e = n2first[(size_t)P * NA + l]; e >= 0 && e < hp.n2_ptr[P + 1] && hp.n2_atom[e] == l; ++e)
      if (hp.n2_img[e] == im) return n2loc[e];
    return -1;
  };
  // ---- column tables: T_P column -> dense column and N[P] entry; E_P column -> dense column and image
  hp.map_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) hp.map_off[a + 1] = hp.map_off[a] + hp.sys_n[0];
  hp.map1.assign(hp.map_off[NA], -1);
  hp.map2.clear();
  hp.col1g_off.assign(NA + 1, 0);
  hp.col2g_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) {
    hp.col1g_off[a + 1] = hp.col1g_off[a] + hp.n_loc[a];
    hp.col2g_off[a + 1] = hp.col2g_off[a] + hp.m_loc[a];
  }
  hp.col1g.assign(hp.col1g_off[NA], 0);
  hp.col2g.assign(hp.col2g_off[NA], 0);
  hp.col2img.assign(hp.col2g_off[NA], 0);
  hp.col1img.assign(hp.col1g_off[NA], 0);
  hp.atom_of_col.assign(hp.sys_n[0], 0);
  for (int a = 0; a < NA; ++a)
    for (int x = 0; x < hp.nb[a]; ++x) hp.atom_of_col[hp.bo[a] + x] = a;
  for (int a = 0; a < NA; ++a) {
    int c = 0;
    for (int k = np[a]; k < np[a + 1]; ++k) {
      const int j = nat[k];
      for (int x = 0; x < hp.nb[j]; ++x, ++c) {
        hp.map1[hp.map_off[a] + hp.bo[j] + x] = c;
        hp.col1g[hp.col1g_off[a] + c] = hp.bo[j] + x;
        hp.col1img[hp.col1g_off[a] + c] = nim[k];
      }
    }
    c = 0;
    for (int k = hp.n2_ptr[a]; k < hp.n2_ptr[a + 1]; ++k) {
      const int l = hp.n2_atom[k];
      for (int x = 0; x < hp.nb[l]; ++x, ++c) {
        hp.col2g[hp.col2g_off[a] + c] = hp.bo[l] + x;
        hp.col2img[hp.col2g_off[a] + c] = hp.n2_img[k];
      }
    }
  }
  // separation of every neighbour entry (forces): R_A - (R_J + shift of its image)
  hp.nbr_sep.assign(3 * (size_t)nn, 0.0);
  for (int a = 0; a < NA; ++a)
    for (int k = np[a]; k < np[a + 1]; ++k) {
      double sh[3];
      image_shift(hp.lat, nim[k], sh);
      for (int c = 0; c < 3; ++c) {
        volatile double pj = hp.pos[3 * (size_t)nat[k] + c] + sh[c];
        hp.nbr_sep[3 * (size_t)k + c] = hp.pos[3 * (size_t)a + c] - pj;
      }
    }
  // ---- workspace layout
  hp.t_off.assign(NA + 1, 0);
  hp.e_off.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) {
    const int64_t s = (int64_t)hp.na[a] * hp.nb[a];
    hp.t_off[a + 1] = hp.t_off[a] + ceil_to(s * hp.n_loc[a], 2);
    hp.e_off[a + 1] = hp.e_off[a] + ceil_to(s * hp.m_loc[a], 2);
  }
  hp.t_total = hp.t_off[NA];
  hp.e_total = hp.e_off[NA];
  for (auto& f : hp.flops) f = 0;
  for (auto& f : hp.issued) f = 0;
  // ---- E_P = T_P D: 64-column tiles of the N2 entries; the k-range of a tile is the runs of
  // entries (J, m) of N[P] whose neighbourhood meets the tile (J's row of D at image
  // n_JL = b - m for a tile column (L, b)), runs of consecutive atoms at one image
  hp.e_items.clear();
  hp.ct_run_ptr.assign(1, 0);
  hp.ct_klen.clear();
  hp.runs.clear();
  hp.gd_items.clear();
  hp.gd_run_ptr.assign(1, 0);
  hp.gd_klen.clear();
  hp.gd_runs.clear();
  hp.ct_kflag.clear();
  hp.ct_kflag_off.assign(1, 0);
  hp.gd_kflag.clear();
  hp.gd_kflag_off.assign(1, 0);
  std::vector<KEnt> krow, ccol;
  {
    // an entry (J, m) of N[P] is relevant to a tile column (L, b) if J lies in N[L] at
    // image b + n_LJ = m: mark those J per tile
    std::vector<int> mark(NA, -1);
    int stamp = 0;
    for (int a = 0; a < NA; ++a) {
      const int sP = hp.na[a] * hp.nb[a];
      const int mOut = hp.m_loc[a];
      const int e0 = hp.n2_ptr[a], e1 = hp.n2_ptr[a + 1];
      int kstart = e0, cstart = 0;
      for (int c0 = 0; c0 < mOut; c0 += E_TILE) {
        const int c1 = std::min(mOut, c0 + E_TILE);
        ++stamp;
        while (kstart < e1 && cstart + hp.nb[hp.n2_atom[kstart]] <= c0) { cstart += hp.nb[hp.n2_atom[kstart]]; ++kstart; }
        ccol.clear();
        krow.clear();
        for (int k = kstart, c = cstart; k < e1 && c < c1; c += hp.nb[hp.n2_atom[k]], ++k) {
          const int l = hp.n2_atom[k], b = hp.n2_img[k];
          {
            const int b0 = std::max(c, c0), b1 = std::min(c + hp.nb[l], c1);
            ccol.push_back(KEnt{l, b, b0 - c0, b1 - b0});
          }
          for (int k2 = np[l]; k2 < np[l + 1]; ++k2) {
            const int j = nat[k2];
            if (hp.pimg[(size_t)a * NA + j] == img_add(b, nim[k2])) mark[j] = stamp;
          }
        }
        const int ct = (int)hp.ct_klen.size();
        int klen = 0, lcol = 0, prevJ = -2, prevImg = -1;
        Run cur{-1, -1, 0, 0};
        for (int k = np[a]; k < np[a + 1]; ++k) {
          const int j = nat[k];
          if (mark[j] == stamp) {
            if (cur.len > 0 && j == prevJ + 1 && nim[k] == prevImg) {
              cur.len += hp.nb[j];
            } else {
              if (cur.len > 0) hp.runs.push_back(cur);
              cur = Run{lcol, hp.bo[j], hp.nb[j], nim[k]};
            }
            prevJ = j;
            prevImg = nim[k];
            krow.push_back(KEnt{j, nim[k], klen, hp.nb[j]});
            klen += hp.nb[j];
          } else {
            prevJ = -2;
          }
          lcol += hp.nb[j];
        }
        if (cur.len > 0) hp.runs.push_back(cur);
        hp.ct_run_ptr.push_back((int)hp.runs.size());
        hp.ct_klen.push_back(klen);
        tile_kflags(hp, krow, ccol, klen, hp.ct_kflag);
        hp.ct_kflag_off.push_back((int64_t)hp.ct_kflag.size());
        hp.issued[1] += kflag_issued(hp.ct_kflag.data() + hp.ct_kflag_off[ct], klen, sP);
        for (int r0 = 0; r0 < sP; r0 += E_TILE) hp.e_items.push_back(EItem{a, r0, c0, ct});
      }
    }
  }
  // ---- the gradient product G_P = H_P D: 64-column tiles of the N[P] entries (J, m); its
  // k-range is the runs of N2[P] entries (L, b) with J in N[L] at image m - b (runs of
  // consecutive atoms at one image)
  {
    std::vector<int> mark(hp.n2_atom.size(), -1);
    int stamp = 0;
    int64_t gd_issued = 0;
    for (int a = 0; a < NA; ++a) {
      const int sP = hp.na[a] * hp.nb[a];
      const int nOut = hp.n_loc[a];
      int kstart = np[a], cstart = 0;
      for (int c0 = 0; c0 < nOut; c0 += E_TILE) {
        const int c1 = std::min(nOut, c0 + E_TILE);
        ++stamp;
        while (kstart < np[a + 1] && cstart + hp.nb[nat[kstart]] <= c0) { cstart += hp.nb[nat[kstart]]; ++kstart; }
        ccol.clear();
        krow.clear();
        for (int k = kstart, c = cstart; k < np[a + 1] && c < c1; c += hp.nb[nat[k]], ++k) {
          const int j = nat[k], m = nim[k];
          {
            const int b0 = std::max(c, c0), b1 = std::min(c + hp.nb[j], c1);
            ccol.push_back(KEnt{j, m, b0 - c0, b1 - b0});
          }
          for (int k2 = np[j]; k2 < np[j + 1]; ++k2) {
            const int l = nat[k2], b = img_add(m, nim[k2]);   // L = nat[k2] at image m + n_JL
            for (int e = n2first[(size_t)a * NA + l]; e >= 0 && e < hp.n2_ptr[a + 1] && hp.n2_atom[e] == l; ++e)
              if (hp.n2_img[e] == b) mark[e] = stamp;
          }
        }
        const int ct = (int)hp.gd_klen.size();
        int klen = 0, lcol = 0, prevL = -2, prevImg = -1;
        Run cur{-1, -1, 0, 0};
        for (int e = hp.n2_ptr[a]; e < hp.n2_ptr[a + 1]; ++e) {
          const int l = hp.n2_atom[e], b = hp.n2_img[e];
          if (mark[e] == stamp) {
            if (cur.len > 0 && l == prevL + 1 && b == prevImg) {
              cur.len += hp.nb[l];
            } else {
              if (cur.len > 0) hp.gd_runs.push_back(cur);
              cur = Run{lcol, hp.bo[l], hp.nb[l], b};
            }
            prevL = l;
            prevImg = b;
            krow.push_back(KEnt{l, b, klen, hp.nb[l]});
            klen += hp.nb[l];
          } else {
            prevL = -2;
          }
          lcol += hp.nb[l];
        }
        if (cur.len > 0) hp.gd_runs.push_back(cur);
        hp.gd_run_ptr.push_back((int)hp.gd_runs.size());
        hp.gd_klen.push_back(klen);
        tile_kflags(hp, krow, ccol, klen, hp.gd_kflag);
        hp.gd_kflag_off.push_back((int64_t)hp.gd_kflag.size());
        for (int r0 = 0; r0 < sP; r0 += E_TILE) {
          hp.gd_items.push_back(EItem{a, r0, c0, ct});
          gd_issued += 2LL * E_TILE * E_TILE * ceil_to(klen, 16);
        }
      }
    }
  }
  for (int a = 0; a < NA; ++a) {
    const int64_t sP = (int64_t)hp.na[a] * hp.nb[a];
    int64_t kk = 0;
    for (int k = np[a]; k < np[a + 1]; ++k) {
      const int j = nat[k];
      int64_t sl = 0;
      for (int k2 = np[j]; k2 < np[j + 1]; ++k2) sl += hp.nb[nat[k2]];
      kk += (int64_t)hp.nb[j] * sl;
    }
    hp.flops[1] += 2 * sP * kk;
    for (int k = np[a]; k < np[a + 1]; ++k) {
      const int q = nat[k];
      hp.flops[2] += 2LL * hp.na[a] * hp.na[q] * hp.nb[q] * hp.n_loc[q];
      hp.flops[2] += 2LL * hp.na[a] * hp.nb[a] * hp.nb[q] * hp.n_loc[q];
      hp.flops[2] += 2LL * hp.na[a] * hp.na[q] * hp.nb[a] * hp.nb[q];
    }
  }
  // ---- V-stage groups (up to three consecutive atoms within GROUP_RADIUS at image 0) x
  // H_COLS-column tiles of the union of their N2 entries.  Q-lists: neighbour entries
  // (Q, q) of the group whose neighbourhood meets the tile; X-lists: entries (X, x) with a
  // tile column on (X, x).  Both carry per slot the pair id of the slot atom with Q.
  hp.grp_first.clear();
  hp.grp_unit_ptr.assign(1, 0);
  hp.grp_units.clear();
  hp.grp_col_ptr.assign(1, 0);
  hp.grp_cols.clear();
  hp.grp_colimg.clear();
  hp.grp_cmap.clear();
  hp.g_tiles.clear();
  hp.gq.clear();
  hp.gx.clear();
  hp.h_waves = 1;
  {
    const double gr2 = GROUP_RADIUS * GROUP_RADIUS;
    std::vector<int> mark(NA, -1), mark_img(NA, 0), qcnt(NA, 0), qsel;
    int stamp = 0;
    int a = 0;
    while (a < NA) {
      int n = 1, units = (hp.na[a] + 15) / 16;
      while (a + n < NA && n < GROUP_ATOMS) {
        const int b = a + n;
        const int u = (hp.na[b] + 15) / 16;
        const double dx = hp.pos[3 * a] - hp.pos[3 * b], dy = hp.pos[3 * a + 1] - hp.pos[3 * b + 1],
                     dz = hp.pos[3 * a + 2] - hp.pos[3 * b + 2];
        if (units + u > GROUP_WAVES || hp.pimg[(size_t)a * NA + b] != IMG0 || dx * dx + dy * dy + dz * dz > gr2) break;
        units += u;
        ++n;
      }
      const int g = (int)hp.grp_first.size();
      hp.grp_first.push_back(a);
      for (int t = 0; t < n; ++t)
        for (int mu0 = 0; mu0 < hp.na[a + t]; mu0 += 16) hp.grp_units.push_back(Unit{a + t, mu0, t, 0});
      hp.grp_unit_ptr.push_back((int)hp.grp_units.size());
      hp.h_waves = std::max(hp.h_waves, units);
      // union of the N2 entries of the group atoms, as (atom, image) columns
      std::vector<int64_t> ents;
      for (int t = 0; t < n; ++t)
        for (int k = hp.n2_ptr[a + t]; k < hp.n2_ptr[a + t + 1]; ++k) ents.push_back(ekey(hp.n2_atom[k], hp.n2_img[k]));
      std::sort(ents.begin(), ents.end());
      ents.erase(std::unique(ents.begin(), ents.end()), ents.end());
      const int col0 = (int)hp.grp_cols.size();
      std::vector<int> col_atom, col_img;
      for (int64_t e : ents) {
        const int l = (int)(e / 4096), im = (int)(e % 4096);
        int cm[GROUP_ATOMS];
        for (int t = 0; t < GROUP_ATOMS; ++t) cm[t] = t < n ? n2col(a + t, l, im) : -1;
        for (int x = 0; x < hp.nb[l]; ++x) {
          hp.grp_cols.push_back(hp.bo[l] + x);
          hp.grp_colimg.push_back(im);
          col_atom.push_back(l);
          col_img.push_back(im);
          for (int t = 0; t < GROUP_ATOMS; ++t) hp.grp_cmap.push_back(cm[t] >= 0 ? cm[t] + x : -1);
        }
      }
      hp.grp_col_ptr.push_back((int)hp.grp_cols.size());
      const int ncol = (int)col_atom.size();
      // neighbour entries (Q, q) of the group, each with its slots (pair id of every group
      // atom with Q at that image) and, for the G part, the E_Q column of each slot atom
      std::vector<int64_t> nbrs;
      for (int t = 0; t < n; ++t)
        for (int k = np[a + t]; k < np[a + t + 1]; ++k) nbrs.push_back(ekey(nat[k], nim[k]));
      std::sort(nbrs.begin(), nbrs.end());
      nbrs.erase(std::unique(nbrs.begin(), nbrs.end()), nbrs.end());
      std::vector<Slot4> slots;
      for (int64_t e : nbrs) {
        const int q = (int)(e / 4096), im = (int)(e % 4096);
        Slot4 sl4{q, -1, -1, -1, im, -1, -1, -1};
        int* sl = &sl4.p0;
        int* ec = &sl4.e0;
        for (int t = 0; t < n; ++t) {
          const int P = a + t;
          if (hp.pimg[(size_t)P * NA + q] != im) continue;
          auto it = std::lower_bound(nat.begin() + np[P], nat.begin() + np[P + 1], q);
          sl[t] = hp.nbr_pair[it - nat.begin()];
          ec[t] = n2col(q, P, hp.pimg[(size_t)q * NA + P]);
        }
        slots.push_back(sl4);
      }
      // group-neighbour index of every atom: one image per atom, since the cell is wider
      // than twice the cutoff plus the group's extent
      for (size_t i = 0; i < slots.size(); ++i) {
        if (i > 0 && slots[i].atom == slots[i - 1].atom) {
          err = "periodic cell too narrow: an atom neighbours one V-stage group at two images";
          return -5;
        }
        mark_img[slots[i].atom] = (int)i;
      }
      for (int c0 = 0; c0 < ncol; c0 += H_COLS) {
        const int c1 = std::min(ncol, c0 + H_COLS);
        GTile tl{};
        tl.grp = g;
        tl.col_beg = col0 + c0;
        tl.ncols = c1 - c0;
        tl.q_beg = (int)hp.gq.size();
        tl.x_beg = (int)hp.gx.size();
        // Q-list: entries (Q, q) with some tile column (L, b) in N[Q + q], i.e. Q in N[L] at
        // image b + n_LQ = q; counted per tile column, listed in slot order
        ++stamp;
        qsel.clear();
        for (int c = c0; c < c1;) {
          const int l = col_atom[c], b = col_img[c];
          int ncl = 1;   // consecutive tile columns on (l, b)
          while (c + ncl < c1 && col_atom[c + ncl] == l && col_img[c + ncl] == b) ++ncl;
          for (int k2 = np[l]; k2 < np[l + 1]; ++k2) {
            const int q = nat[k2];
            const int i = mark_img[q];
            if (i < (int)slots.size() && slots[i].atom == q && slots[i].img == img_add(b, nim[k2])) {
              if (mark[q] != stamp) { mark[q] = stamp; qcnt[q] = 0; qsel.push_back(i); }
              qcnt[q] += ncl;
            }
          }
          c += ncl;
        }
        std::sort(qsel.begin(), qsel.end());
        for (int i : qsel) {
          const Slot4& s4 = slots[i];
          const int q = s4.atom;
          hp.gq.push_back(s4);
          const int cq = qcnt[q];
          const int* sl = &s4.p0;
          for (int t = 0; t < n; ++t)
            if (sl[t] >= 0)
              hp.issued[2] += 2048LL * ((hp.na[a + t] + 15) / 16) * cq * (((hp.na[q] + 3) / 4) + ((hp.nb[q] + 3) / 4));
        }
        // X-list: the group neighbours (X, x) that are tile columns, in slot (atom) order
        for (int c = c0; c < c1;) {
          const int l = col_atom[c], b = col_img[c];
          int ncl = 1;
          while (c + ncl < c1 && col_atom[c + ncl] == l && col_img[c + ncl] == b) ++ncl;
          const int i = mark_img[l];
          if (i < (int)slots.size() && slots[i].atom == l && slots[i].img == b) {
            const Slot4& s4 = slots[i];
            hp.gx.push_back(s4);
            const int* sl = &s4.p0;
            for (int t = 0; t < n; ++t)
              if (sl[t] >= 0) hp.issued[2] += 2048LL * ((hp.na[a + t] + 15) / 16) * ncl * ((hp.na[l] + 3) / 4);
          }
          c += ncl;
        }
        tl.q_end = (int)hp.gq.size();
        tl.x_end = (int)hp.gx.size();
        hp.g_tiles.push_back(tl);
      }
      a += n;
    }
  }
  // ---- T2 pairs: every canonical pair, oriented by cost as for clusters; per pair the E_P
  // column of each column of T_Q: entry (L, n_QL) of N[Q] meets E_P at (L, q + n_QL), q the
  // image of Q within r_cut of P
  hp.t2_items.resize(npairs);
  hp.t2col_off.assign(npairs + 1, 0);
  hp.t2col.clear();
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
    const int q = hp.pimg[(size_t)a * NA + b];
    for (int k = np[b]; k < np[b + 1]; ++k) {
      const int c = n2col(a, nat[k], img_add(q, nim[k]));
      if (c < 0) { err = "periodic T2 column outside N2"; return -3; }
      for (int x = 0; x < hp.nb[nat[k]]; ++x) hp.t2col.push_back(c + x);
    }
    hp.t2col_off[p + 1] = (int64_t)hp.t2col.size();
  }
  {
    auto ns_class = [](int ns) { return ns <= 4 ? 4 : ns <= 8 ? 8 : ns <= 10 ? 10 : ns <= 12 ? 12 : 16; };
    auto key = [&](int item) {
      const int p = item >> 1;
      const bool flip = item & 1;
      const int x = flip ? hp.pair_b[p] : hp.pair_a[p], y = flip ? hp.pair_a[p] : hp.pair_b[p];
      return ((hp.na[x] + 15) / 16) * 64 + ns_class((hp.na[y] + 3) / 4);
    };
    // items of one column atom consecutive inside a class (T_Q shared in an XCD's L2)
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
  // ---- dV pairs: grouped by shape as for clusters; per pair (P, Q) = (pair_a, pair_b) the
  // E_P column of every column of T_Q and the E columns of each other's basis
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
    hp.dvcol_off.assign(npairs + 1, 0);
    hp.dvcol.clear();
    hp.dv_cp.assign(npairs, 0);
    hp.dv_cq.assign(npairs, 0);
    for (int64_t p = 0; p < npairs; ++p) {
      const int a = hp.pair_a[p], b = hp.pair_b[p], q = hp.pair_img[p];
      for (int k = np[b]; k < np[b + 1]; ++k) {
        const int c = n2col(a, nat[k], img_add(q, nim[k]));
        if (c < 0) { err = "periodic dV column outside N2"; return -3; }
        for (int x = 0; x < hp.nb[nat[k]]; ++x) hp.dvcol.push_back(c + x);
      }
      hp.dvcol_off[p + 1] = (int64_t)hp.dvcol.size();
      hp.dv_cp[p] = n2col(a, b, q);
      hp.dv_cq[p] = n2col(b, a, img_neg(q));
    }
  }
  hp.f_items.clear();
  hp.f_plist.clear();
  hp.y_tiles.clear();
  hp.y_off.assign(NA + 1, 0);
  hp.y_total = 0;
  // ---- final contraction on the pattern: per canonical pair (A, B) at image n, the terms
  // X'_AB = sum_P T_P[:, A]^T H'_P[:, (B, a + n)] over the P with A in N[P] at image a, and
  // X'_BA likewise (B in N[P] at image b, H' column (A, b - n)).  They are evaluated by
  // tiles of two V-stage groups (one image for the whole tile, one image per P for each
  // group); the pairs of tiles without such images keep per-pair term lists.
  hp.pg_beg.assign(npairs, 0);
  hp.pg_mid.assign(npairs, 0);
  hp.pg_end.assign(npairs, 0);
  hp.pg_ent.clear();
  hp.pg_pairs.clear();
  hp.pt_tiles.clear();
  hp.pt_ent.clear();
  hp.pt_classes.clear();
  auto lcol_in = [&](int P, int R) {   // first T_P column of R (R in N[P])
    auto jt = std::lower_bound(nat.begin() + np[P], nat.begin() + np[P + 1], R);
    return hp.nbr_lcol[jt - nat.begin()];
  };
  // algorithmic flops: the pair terms, whichever route evaluates them
  for (int64_t p = 0; p < npairs; ++p) {
    const int A = hp.pair_a[p], B = hp.pair_b[p], n = hp.pair_img[p];
    for (int dir = 0; dir < (A == B ? 1 : 2); ++dir) {
      const int R = dir ? B : A, S = dir ? A : B, img_rs = dir ? img_neg(n) : n;
      for (int k = np[R]; k < np[R + 1]; ++k) {
        const int P = nat[k];
        if (n2col(P, S, img_add(hp.pimg[(size_t)P * NA + R], img_rs)) >= 0)
          hp.flops[4] += 2LL * hp.nb[R] * hp.nb[S] * hp.na[P] * hp.nb[P];
      }
    }
  }
  const int NG = (int)hp.grp_first.size();
  std::vector<int> grp_of(NA);
  for (int g = 0; g < NG; ++g)
    for (int a = hp.grp_first[g]; a < (g + 1 < NG ? hp.grp_first[g + 1] : NA); ++a) grp_of[a] = g;
  std::vector<std::pair<int64_t, int>> tp(npairs);
  for (int64_t p = 0; p < npairs; ++p)
    tp[p] = {(int64_t)grp_of[hp.pair_a[p]] * NG + grp_of[hp.pair_b[p]], (int)p};
  std::sort(tp.begin(), tp.end());
  std::vector<PTile> tiles;
  std::vector<int> tile_ta, tile_tb;
  std::vector<int> plist;
  std::vector<int> mark(NA, -1);
  for (size_t i0 = 0; i0 < tp.size();) {
    size_t i1 = i0;
    while (i1 < tp.size() && tp[i1].first == tp[i0].first) ++i1;
    const int ga = (int)(tp[i0].first / NG), gb = (int)(tp[i0].first % NG);
    const int a0 = hp.grp_first[ga], na_ = (ga + 1 < NG ? hp.grp_first[ga + 1] : NA) - a0;
    const int b0 = hp.grp_first[gb], nb_ = (gb + 1 < NG ? hp.grp_first[gb + 1] : NA) - b0;
    const int n = hp.pair_img[tp[i0].second];
    bool ok = true;
    int mask = 0;
    for (size_t i = i0; i < i1; ++i) {
      const int p = tp[i].second;
      ok = ok && hp.pair_img[p] == n;
      mask |= 1 << (3 * (hp.pair_a[p] - a0) + (hp.pair_b[p] - b0));
    }
    if (ga == gb) ok = ok && n == IMG0;
    PTile tl{a0, na_, b0, nb_, (int)hp.pt_ent.size(), 0, mask, 0};
    for (int part = 0; part < 2 && ok; ++part) {
      // part 0: P with a ga atom in N[P]; part 1: P with a gb atom in N[P]
      const int r0 = part ? b0 : a0, nr = part ? nb_ : na_;
      const int o0 = part ? a0 : b0, no = part ? na_ : nb_;
      const int img_ro = part ? img_neg(n) : n;   // image of the other group relative to this one
      plist.clear();
      for (int t = 0; t < nr; ++t)
        for (int k = np[r0 + t]; k < np[r0 + t + 1]; ++k)
          if (mark[nat[k]] != (int)i0 * 2 + part) { mark[nat[k]] = (int)i0 * 2 + part; plist.push_back(nat[k]); }
      std::sort(plist.begin(), plist.end());
      for (int P : plist) {
        int rimg = -1;
        int tc[3] = {-1, -1, -1}, hc[3] = {-1, -1, -1};
        for (int t = 0; t < nr; ++t) {
          const int im = hp.pimg[(size_t)P * NA + r0 + t];
          if (im < 0) continue;
          if (rimg >= 0 && im != rimg) ok = false;
          rimg = im;
          tc[t] = lcol_in(P, r0 + t);
        }
        if (!ok) break;
        bool anyh = false;
        for (int t = 0; t < no; ++t) {
          hc[t] = n2col(P, o0 + t, img_add(rimg, img_ro));
          anyh = anyh || hc[t] >= 0;
        }
        if (!anyh) continue;
        PTEnt e{P, part, {-1, -1, -1}, {-1, -1, -1}};
        for (int t = 0; t < 3; ++t) {
          e.rc[t] = part ? hc[t] : tc[t];
          e.cc[t] = part ? tc[t] : hc[t];
        }
        hp.pt_ent.push_back(e);
      }
    }
    if (!ok) {
      hp.pt_ent.resize(tl.e_beg);
      for (size_t i = i0; i < i1; ++i) hp.pg_pairs.push_back(tp[i].second);
    } else {
      tl.e_end = (int)hp.pt_ent.size();
      int ba = 0, bb = 0;
      for (int t = 0; t < na_; ++t) ba += hp.nb[a0 + t];
      for (int t = 0; t < nb_; ++t) bb += hp.nb[b0 + t];
      tiles.push_back(tl);
      tile_ta.push_back((ba + 15) / 16);
      tile_tb.push_back((bb + 15) / 16);
      for (int e = tl.e_beg; e < tl.e_end; ++e) {
        const int P = hp.pt_ent[e].P;
        hp.issued[4] += 2048LL * tile_ta.back() * tile_tb.back() * ((hp.na[P] * hp.nb[P] + 3) / 4);
      }
    }
    i0 = i1;
  }
  // tiles by class (ta, tb), group-pair order kept inside a class
  for (int ta = 1; ta <= GROUP_ATOMS; ++ta)
    for (int tb = 1; tb <= GROUP_ATOMS; ++tb) {
      const int beg = (int)hp.pt_tiles.size();
      for (size_t i = 0; i < tiles.size(); ++i)
        if (tile_ta[i] == ta && tile_tb[i] == tb) hp.pt_tiles.push_back(tiles[i]);
      if ((int)hp.pt_tiles.size() > beg) hp.pt_classes.push_back(PTClass{ta, tb, beg, (int)hp.pt_tiles.size()});
    }
  std::sort(hp.pg_pairs.begin(), hp.pg_pairs.end());
  for (int p : hp.pg_pairs) {
    const int A = hp.pair_a[p], B = hp.pair_b[p], n = hp.pair_img[p];
    hp.pg_beg[p] = (int)hp.pg_ent.size();
    for (int dir = 0; dir < (A == B ? 1 : 2); ++dir) {
      const int R = dir ? B : A, S = dir ? A : B, img_rs = dir ? img_neg(n) : n;
      for (int k = np[R]; k < np[R + 1]; ++k) {
        const int P = nat[k];
        const int r_img = hp.pimg[(size_t)P * NA + R];   // image of R within r_cut of P
        const int hc = n2col(P, S, img_add(r_img, img_rs));
        if (hc < 0) continue;
        hp.pg_ent.push_back(PGEnt{P, lcol_in(P, R), hc, 0});
        hp.issued[4] += 2048LL * ((hp.na[P] * hp.nb[P] + 3) / 4);
      }
      if (dir == 0) hp.pg_mid[p] = (int)hp.pg_ent.size();
    }
    if (A == B) hp.pg_mid[p] = (int)hp.pg_ent.size();
    hp.pg_end[p] = (int)hp.pg_ent.size();
  }
  // ---- energy chunks: runs of at most EN_PAIRS canonical pairs
  hp.en_sys.clear();
  hp.en_pbeg.clear();
  hp.en_pend.clear();
  for (int64_t p = 0; p < npairs; p += EN_PAIRS) {
    hp.en_sys.push_back(0);
    hp.en_pbeg.push_back((int)p);
    hp.en_pend.push_back((int)std::min<int64_t>(npairs, p + EN_PAIRS));
  }
  return 0;
}

}  // namespace exx
