// libexx kernels: the block-sparse GEMM E_P = T_P D (and its adjoint), the
// batched GEMM Y_P = T_P^T H'_P and the owner-computes gather of K.

#include "exx_dev.h"

using namespace exx;


// EK: k-chunk per LDS stage (a tuning choice: 16 or 32); the next chunk is loaded into
// registers while the current one is multiplied.  NSP = 2 (collinear spin): the
// products with D (into r.O) and D1 (into O1) in one pass, the A_P tile staged once.
// PER: periodic plans (image check on every D element, see RowD::ocolimg)
template <int EK, int NSP, bool PER>
__global__ __launch_bounds__(256) void k_rowD(const double* __restrict__ D, RowD r, DevPlan d, int n_items,
                                              int n_padded, const double* __restrict__ D1, double* __restrict__ O1) {
  // one LDS stage (the next chunk waits in registers): half the LDS of two stages, so more
  // workgroups are resident per CU
  __shared__ double As[EK][EPITCH];
  __shared__ double Bs[NSP][EK][EPITCH];
  const int w = xcd_task(n_padded);
  if (w >= n_items) return;
  const EItem it = r.items[w];
  const int P = it.P;
  const int sP = d.na[P] * d.nb[P], lda = r.a_ld[P], ldo = r.o_ld[P];
  const int s = d.atom_sys[P];
  const int64_t ns = d.sys_n[s];
  const double* Dsp[NSP];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp) Dsp[sp] = (sp == 0 ? D : D1) + d.sys_d_off[s];
  const double* AP = r.A + r.a_off[P];
  const int t = threadIdx.x;
  const int wv = t >> 6, L = t & 63, lr = L & 15, lk = L >> 4;
  const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
  // staging roles: A (rows of A_P) k = t % EK, rows ma + MS x; B (rows of D) k = t / (256 / EK)... per pass of
  // 16 k rows: k = pass * 16 + (t >> 4), columns nb0 + x
  constexpr int MS = 256 / EK, NA_ = ET / MS, NP = EK / 16;
  const int ka = t % EK, ma = t / EK;
  const int kb = t >> 4, nb0 = (t & 15) * 4;
  int gcn[4];
  int gat[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};   // periodic: atom and image code of the column
  constexpr bool per = PER;
  const int NAt = d.n_atoms;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int n = it.c0 + nb0 + x;
    gcn[x] = n < ldo ? r.ocolg[r.ocolg_off[P] + n] : -1;
    if (per && gcn[x] >= 0) {
      gat[x] = d.atom_of_col[gcn[x]];
      gim[x] = r.ocolimg[r.ocolg_off[P] + n];
    }
  }
  const int klen = r.klen[it.ct];
  const Run* runs = r.runs + r.run_ptr[it.ct];
  int ia = 0, sa = 0;                   // run cursor (run index, its first k) of the A role
  int ib[NP], sb[NP];                    // and of each pass of the B role
#pragma unroll
  for (int pz = 0; pz < NP; ++pz) ib[pz] = sb[pz] = 0;
  double va[NA_], vb[NSP][NP][4];
  auto gload = [&](int k0) {
    const int k1 = k0 + ka;
    const bool oka = k1 < klen;
    if (oka) while (k1 >= sa + runs[ia].len) { sa += runs[ia].len; ++ia; }
    const int lc = oka ? runs[ia].lcol + (k1 - sa) : 0;
#pragma unroll
    for (int x = 0; x < NA_; ++x) {
      const int m = it.r0 + ma + MS * x;
      const bool ok = oka && m < sP;
      const double y = AP[ok ? (size_t)m * lda + lc : 0];
      va[x] = ok ? y : 0.0;
    }
#pragma unroll
    for (int pz = 0; pz < NP; ++pz) {
      const int k2 = k0 + 16 * pz + kb;
      const bool okb = k2 < klen;
      if (okb) while (k2 >= sb[pz] + runs[ib[pz]].len) { sb[pz] += runs[ib[pz]].len; ++ib[pz]; }
      const int gr = okb ? runs[ib[pz]].grow + (k2 - sb[pz]) : 0;
      int jrow = 0, mimg = 0;   // periodic: the row's atom and its image (that of its run)
      if (per && okb) {
        jrow = d.atom_of_col[gr];
        mimg = runs[ib[pz]].img;
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        bool okd = okb && gcn[x] >= 0;
        if (per && okd) {
          const int nJL = d.pimg[(size_t)jrow * NAt + gat[x]];
          okd = nJL >= 0 && nJL + mimg - IMG0 == gim[x];
        }
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp) {
          const double z = Dsp[sp][okd ? (size_t)gr * ns + gcn[x] : 0];
          vb[sp][pz][x] = okd ? z : 0.0;
        }
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int x = 0; x < NA_; ++x) As[ka][ma + MS * x] = va[x];
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
      for (int pz = 0; pz < NP; ++pz)
#pragma unroll
        for (int x = 0; x < 4; ++x) Bs[sp][16 * pz + kb][nb0 + x] = vb[sp][pz][x];
  };
  d4 acc[NSP][2][2];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[sp][x][y] = d4{0, 0, 0, 0};
  gload(0);
  sstore();
  __syncthreads();
  const uint8_t* kf = r.kflag + r.kflag_off[it.ct];
  const int q0 = wn >> 4;   // this wavefront's column quarters q0, q0 + 1
  // and its two 16-row blocks: skipped where they lie past s_P (uniform per wavefront)
  const bool rv0 = it.r0 + wm < sP, rv1 = it.r0 + wm + 16 < sP;
  for (int k0 = 0; k0 < klen; k0 += EK) {
    const bool more = k0 + EK < klen;
    if (more) gload(k0 + EK);
#pragma unroll
    for (int ks = 0; ks < EK; ks += 4) {
      // skip the products of 16 x 16 blocks where D is structurally zero (uniform per wavefront)
      const int f = (k0 + ks < klen) ? (kf[(k0 + ks) >> 4] >> q0) : 0;
      const double a0 = As[ks + lk][wm + lr], a1 = As[ks + lk][wm + 16 + lr];
#pragma unroll
      for (int sp = 0; sp < NSP; ++sp) {
        if (f & 1) {
          const double b0 = Bs[sp][ks + lk][wn + lr];
          if (rv0) acc[sp][0][0] = mfma64(a0, b0, acc[sp][0][0]);
          if (rv1) acc[sp][1][0] = mfma64(a1, b0, acc[sp][1][0]);
        }
        if (f & 2) {
          const double b1 = Bs[sp][ks + lk][wn + 16 + lr];
          if (rv0) acc[sp][0][1] = mfma64(a0, b1, acc[sp][0][1]);
          if (rv1) acc[sp][1][1] = mfma64(a1, b1, acc[sp][1][1]);
        }
      }
    }
    if (more) {   // every wavefront is done with the stage before it is overwritten
      __syncthreads();
      sstore();
      __syncthreads();
    }
  }
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp) {
    double* OP = (sp == 0 ? r.O : O1) + r.o_off[P];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int col = it.c0 + wn + 16 * y + lr;
        if (col >= ldo) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = it.r0 + wm + 16 * x + lk + 4 * v;
          if (row < sP) OP[(size_t)row * ldo + col] = acc[sp][x][y][v];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// stage 4a: Y_P = T_P^T H'_P for every aux atom P (n_P x m_P, K = s_P), a
// batched GEMM with both operands stored k-major.  64 x 64 tile per
// workgroup of four wavefronts (32 x 32 each), k-steps of 16 staged in
// double-buffered LDS with coalesced row loads.


constexpr int YT = 64, YPITCH = YT + 4;

// YK: k-chunk per LDS stage (a tuning choice: 16 or 32)
template <int YK>
__global__ __launch_bounds__(256) void k_Y(DevPlan d, int n_tiles, int n_padded) {
  __shared__ double As[2][YK][YPITCH];
  __shared__ double Bs[2][YK][YPITCH];
  const int ti = xcd_task(n_padded);
  if (ti >= n_tiles) return;
  const YTile yt = d.y_tiles[ti];
  const int P = yt.P;
  const int Kd = d.na[P] * d.nb[P], M = d.n_loc[P], N = d.m_loc[P];
  const double* A = d.T + d.t_off[P];   // A(m, k) = T_P[k * M + m]
  const double* B = d.H + d.h_off[P];   // B(k, n) = H'_P[k * N + n]
  const int t = threadIdx.x;
  const int wv = t >> 6, L = t & 63, lr = L & 15, lk = L >> 4;
  const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
  // global -> LDS staging role: rows kr + 16 pz of the k-chunk, 4 columns
  constexpr int NP = YK / 16;
  const int kr = t >> 4, cc = (t & 15) * 4;
  double ra[NP][4], rb[NP][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int pz = 0; pz < NP; ++pz) {
      const int k = k0 + 16 * pz + kr;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int m = yt.m0 + cc + x, n = yt.n0 + cc + x;
        const bool oa = k < Kd && m < M, ob = k < Kd && n < N;
        const double a = A[oa ? (size_t)k * M + m : 0];
        const double b = B[ob ? (size_t)k * N + n : 0];
        ra[pz][x] = oa ? a : 0.0;
        rb[pz][x] = ob ? b : 0.0;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int pz = 0; pz < NP; ++pz)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        As[buf][16 * pz + kr][cc + x] = ra[pz][x];
        Bs[buf][16 * pz + kr][cc + x] = rb[pz][x];
      }
  };
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0, 0, 0, 0};
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < Kd; k0 += YK) {
    const bool more = k0 + YK < Kd;
    if (more) gload(k0 + YK);
#pragma unroll
    for (int ks = 0; ks < YK; ks += 4) {
      double a0 = As[buf][ks + lk][wm + lr], a1 = As[buf][ks + lk][wm + 16 + lr];
      double b0 = Bs[buf][ks + lk][wn + lr], b1 = Bs[buf][ks + lk][wn + 16 + lr];
      acc[0][0] = mfma64(a0, b0, acc[0][0]);
      acc[0][1] = mfma64(a0, b1, acc[0][1]);
      acc[1][0] = mfma64(a1, b0, acc[1][0]);
      acc[1][1] = mfma64(a1, b1, acc[1][1]);
    }
    if (more) {
      sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  double* Y = d.Y + d.y_off[P];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int n = yt.n0 + wn + 16 * y + lr;
      if (n >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = yt.m0 + wm + 16 * x + lk + 4 * v;
        if (m < M) Y[(size_t)m * N + n] = acc[x][y][v];
      }
    }
}

// ---------------------------------------------------------------------------
// stage 4b: K = T2 + (X + X^T)/2 with X[i, l] = sum_P Y_P[c1_P(i), c2_P(l)]
// (c1: column of T_P, c2: column of H'_P).  One workgroup per 32 x 32 tile
// pair of the upper triangle; the aux atoms of its list are visited in a
// fixed order, two per step (the loads of both issued together, the maps of
// the next two fetched meanwhile).  X[i, l] is gathered with l fastest across threads and
// X[l, i] with i fastest (both coalesced), the two halves are combined in
// LDS, and every element is written together with its mirror.

__global__ __launch_bounds__(256) void k_symreduce(double* __restrict__ K, DevPlan d, int n_items,
                                                   int n_padded) {
  constexpr int PB = 128;                 // aux atoms whose list data are staged per round
  __shared__ int cmap[2][4][32];   // two aux atoms: c1(I rows), c2(I rows), c1(L cols), c2(L cols)
  __shared__ double xa[32][33], xb[32][33];
  __shared__ int64_t s_yoff[PB], s_moff[PB];
  __shared__ int s_n[PB];
  const int w = xcd_task(n_padded);
  if (w >= n_items) return;
  const FItem it = d.f_items[w];
  const int s = it.sys;
  const int64_t ns = d.sys_n[s];
  const int t = threadIdx.x;
  const int ta = t & 31, tb = t >> 5;   // element (tb + 8 r, ta)
  double acc_a[4] = {0, 0, 0, 0}, acc_b[4] = {0, 0, 0, 0};
  // per round of PB aux atoms their list data in LDS; per step two atoms' column maps in LDS
  // (threads < 128 load the next two atoms' maps while the current Y entries are gathered)
  const int which = (t >> 5) & 3, xm = t & 31;
  const int gm = ((which < 2) ? it.gI0 : it.gL0) + xm;
  const int* mbase = (which & 1) ? d.map2 : d.map1;
  for (int p0 = it.pbeg; p0 < it.pend; p0 += PB) {
    const int nb = min(PB, it.pend - p0);
    __syncthreads();
    for (int j = t; j < nb; j += 256) {
      const int P = d.f_plist[p0 + j];
      s_n[j] = d.m_loc[P];
      s_yoff[j] = d.y_off[P];
      s_moff[j] = d.map_off[P];
    }
    __syncthreads();
    auto map_at = [&](int j) { return (t < 128 && j < nb && gm < ns) ? mbase[s_moff[j] + gm] : -1; };
    if (t < 128) {
      cmap[0][which][xm] = map_at(0);
      cmap[1][which][xm] = map_at(1);
    }
    int m2 = map_at(2), m3 = map_at(3);
    __syncthreads();
    // two aux atoms per step: the loads of both are issued together, then added in list order
    for (int j = 0; j < nb; j += 2) {
      double ya[2][4], yb[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool jv = j + u < nb;
        const int nP_ = s_n[jv ? j + u : j];
        const double* Y = d.Y + s_yoff[jv ? j + u : j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = tb + 8 * r;
          // X[i = I0 + ii, l = L0 + ta] = Y_P[c1(i), c2(l)]
          const int c1 = cmap[u][0][ii], c2 = cmap[u][3][ta];
          ya[u][r] = (jv && c1 >= 0 && c2 >= 0) ? Y[(size_t)c1 * nP_ + c2] : 0.0;
          // X[l = L0 + ii, i = I0 + ta] = Y_P[c1(l), c2(i)], stored at (ta, ii)
          const int d1 = cmap[u][2][ii], d2 = cmap[u][1][ta];
          yb[u][r] = (jv && d1 >= 0 && d2 >= 0) ? Y[(size_t)d1 * nP_ + d2] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (j + u < nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ii = tb + 8 * r;
            if (cmap[u][0][ii] >= 0 && cmap[u][3][ta] >= 0) acc_a[r] += ya[u][r];
            if (cmap[u][2][ii] >= 0 && cmap[u][1][ta] >= 0) acc_b[r] += yb[u][r];
          }
        }
      }
      __syncthreads();
      if (t < 128) {
        cmap[0][which][xm] = m2;
        cmap[1][which][xm] = m3;
      }
      m2 = map_at(j + 4);
      m3 = map_at(j + 5);
      __syncthreads();
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    xa[tb + 8 * r][ta] = acc_a[r];
    xb[ta][tb + 8 * r] = acc_b[r];
  }
  __syncthreads();
  double* Ks = K + d.sys_d_off[s];
  const bool diag = it.gI0 == it.gL0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = tb + 8 * r, ll = ta;
    const int i = it.gI0 + ii, l = it.gL0 + ll;
    if (i >= ns || l >= ns) continue;
    if (diag && i > l) continue;
    const double val = Ks[(size_t)i * ns + l] + 0.5 * (xa[ii][ll] + xb[ii][ll]);
    Ks[(size_t)i * ns + l] = val;
    if (i != l) Ks[(size_t)l * ns + i] = val;
  }
}


void launch_rowD(exx_plan plan, const double* D, const RowD& r, int n, hipStream_t st) {
  if (n <= 0) return;
  const int nwgp = (n + 7) / 8 * 8;
  const bool per = r.ocolimg != nullptr;
  if (plan->tune[TUNE_E] == 1) {
    if (per) hipLaunchKernelGGL((k_rowD<32, 1, true>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
    else hipLaunchKernelGGL((k_rowD<32, 1, false>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
  } else {
    if (per) hipLaunchKernelGGL((k_rowD<16, 1, true>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
    else hipLaunchKernelGGL((k_rowD<16, 1, false>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
  }
}

// the two products of a collinear-spin build (clusters): r.O = A D, O1 = A D1
void launch_rowD_spin(exx_plan plan, const double* D, const double* D1, double* O1, const RowD& r, int n,
                      hipStream_t st) {
  if (n <= 0) return;
  const int nwgp = (n + 7) / 8 * 8;
  const bool per = r.ocolimg != nullptr;   // periodic plans: the image check on every D element
#define RDS(EK, PER) hipLaunchKernelGGL((k_rowD<EK, 2, PER>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, D1, O1)
  if (plan->tune[TUNE_E] == 1) { if (per) RDS(32, true); else RDS(32, false); }
  else { if (per) RDS(16, true); else RDS(16, false); }
#undef RDS
}

// ---------------------------------------------------------------------------
// Periodic plans: the final contraction on the pair pattern, per canonical pair
// for the pairs whose group tile has no single image (the rest run in k_ptile
// below).  Per such pair (A, B) (B at its image n within r_cut of A) one workgroup of four
// wavefronts forms X'_AB = sum_P T_P[:, A]^T H'_P[:, (B, a + n)] (P over the
// atoms with A in N[P] at image a) and likewise X'_BA, each term a chain of
// 16x16x4 MFMAs over the s_P rows of P; the terms are dealt to the wavefronts
// in turn and the four partial sums added in a fixed order.  Then, with T2
// already in K, K_AB = K_AB + (X'_AB + X'_BA^T) / 2 and K_BA = K_AB^T (for
// A = B, K_AA + (X' + X'^T) / 2 from its upper triangle).  Each term runs as four
// independent MFMA chains (interleaved k-steps) added in a fixed order.
__global__ __launch_bounds__(256) void k_pgather(double* __restrict__ K, DevPlan d, int n_pairs, int n_padded) {
  __shared__ double red[4][2][4][64];
  __shared__ double xs[2][16][17];
  const int pi = xcd_task(n_padded);
  if (pi >= n_pairs) return;
  const int p = d.pg_pairs[pi];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63, lr = L & 15, lk = L >> 4;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t ns = d.sys_n[0];
  d4 acc[2];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int beg = dir == 0 ? d.pg_beg[p] : d.pg_mid[p], end = dir == 0 ? d.pg_mid[p] : d.pg_end[p];
    const bool ia = lr < (dir == 0 ? bA : bB), kb = lr < (dir == 0 ? bB : bA);
    d4 a4 = d4{0, 0, 0, 0};
    for (int e = beg + wv; e < end; e += 4) {
      const PGEnt pe = d.pg_ent[e];
      const int P = pe.P;
      const int sP = d.na[P] * d.nb[P], nP = d.n_loc[P], mP = d.m_loc[P];
      const double* TP = d.T + d.t_off[P] + pe.tcol + lr;   // A[i][r] = T_P[r][tcol + i]
      const double* HP = d.H + d.h_off[P] + pe.hcol + lr;   // B[r][k] = H'_P[r][hcol + k]
      // four independent chains over k-steps r0 + 4 u (loads of a round issued together)
      d4 c4[4] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}, d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
      for (int r0 = 0; r0 < sP; r0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + 4 * u + lk;
          const bool ok = r < sP;
          const double x = TP[(ok && ia) ? (size_t)r * nP : 0];
          const double y = HP[(ok && kb) ? (size_t)r * mP : 0];
          a[u] = (ok && ia) ? x : 0.0;
          b[u] = (ok && kb) ? y : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) c4[u] = mfma64(a[u], b[u], c4[u]);
      }
      a4 += (c4[0] + c4[1]) + (c4[2] + c4[3]);
    }
    acc[dir] = a4;
  }
#pragma unroll
  for (int dir = 0; dir < 2; ++dir)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv][dir][v][L] = acc[dir][v];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int dir = 0; dir < 2; ++dir)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = red[0][dir][v][L];
        for (int w2 = 1; w2 < 4; ++w2) x += red[w2][dir][v][L];
        xs[dir][lk + 4 * v][lr] = x;
      }
  }
  __syncthreads();
  const int i = threadIdx.x >> 4, k = threadIdx.x & 15;
  if (i < bA && k < bB && (A != B || i <= k)) {
    double* Kp = K + d.sys_d_off[0];
    const size_t ab = (size_t)(d.bo[A] + i) * ns + d.bo[B] + k;
    const double x = 0.5 * (xs[0][i][k] + (A == B ? xs[0][k][i] : xs[1][k][i]));
    const double val = Kp[ab] + x;
    Kp[ab] = val;
    if (A != B || i != k) Kp[(size_t)(d.bo[B] + k) * ns + d.bo[A] + i] = val;
  }
}

// Tiled pattern contraction: one workgroup per tile of two V-stage groups (ga, gb), whose
// TA x TB output tiles of 16 x 16 (the ga basis functions by the gb ones) sit in registers
// of every wavefront.  The tile's entries (P, part) are dealt to the four wavefronts in turn;
// an entry adds, over the s_P rows r of P, R[r][row column]^T C[r][column column] with
// (R, C) = (T_P, H'_P) for part 0 (X'_AB) and (H'_P, T_P) for part 1 (the transpose of
// X'_BA), so the sum is X'_AB + X'_BA^T for every atom pair of the tile.  Each k-round
// covers four k-steps, whose loads are issued one round ahead (across entries too); the
// four wavefront partials are added in a fixed order.  Then K_AB += (X'_AB + X'_BA^T) / 2 on the tile's pattern pairs (upper
// triangle of a diagonal tile), mirrored to K_BA.
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_ptile(double* __restrict__ K, DevPlan d, const PTile* __restrict__ tiles,
                                               int n_tiles, int n_padded) {
  __shared__ double red[4][TA * TB][4][64];
  const int ti = xcd_task(n_padded);
  if (ti >= n_tiles) return;
  const PTile tl = tiles[ti];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63, lr = L & 15, lk = L >> 4;
  // group atom (slot) and local basis index of the lane's output rows and columns
  int rs[TA], rx[TA], cs[TB], cx[TB];
#pragma unroll
  for (int t = 0; t < TA; ++t) {
    int i = 16 * t + lr, sl = -1;
    for (int a = 0; a < tl.na && sl < 0; ++a) {
      const int nbs = d.nb[tl.a0 + a];
      if (i < nbs) sl = a; else i -= nbs;
    }
    rs[t] = sl;
    rx[t] = i;
  }
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    int i = 16 * t + lr, sl = -1;
    for (int a = 0; a < tl.nbt && sl < 0; ++a) {
      const int nbs = d.nb[tl.b0 + a];
      if (i < nbs) sl = a; else i -= nbs;
    }
    cs[t] = sl;
    cx[t] = i;
  }
  d4 acc[TA][TB];
#pragma unroll
  for (int t = 0; t < TA; ++t)
#pragma unroll
    for (int u = 0; u < TB; ++u) acc[t][u] = d4{0, 0, 0, 0};
  // The rounds (16 rows of P) of this wavefront's entries in one stream: the loads of the
  // next round are issued before the MFMAs of the current one.
  struct Src {
    const double *R, *C;
    int rp, cp, sP, r0;
    int rcol[TA], ccol[TB];
    bool rok[TA], cok[TB];
  } ls;
  int e = tl.e_beg + wv;
  auto setup = [&](int ei) {
    const PTEnt pe = d.pt_ent[ei];
    const int P = pe.P;
    const int nP = d.n_loc[P], mP = d.m_loc[P];
    const double* Tm = d.T + d.t_off[P];
    const double* Hm = d.H + d.h_off[P];
    ls.R = pe.part ? Hm : Tm;
    ls.C = pe.part ? Tm : Hm;
    ls.rp = pe.part ? mP : nP;
    ls.cp = pe.part ? nP : mP;
    ls.sP = d.na[P] * d.nb[P];
    ls.r0 = 0;
#pragma unroll
    for (int t = 0; t < TA; ++t) {
      const int c = rs[t] >= 0 ? pe.rc[rs[t]] : -1;
      ls.rok[t] = c >= 0;
      ls.rcol[t] = ls.rok[t] ? c + rx[t] : 0;
    }
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      const int c = cs[t] >= 0 ? pe.cc[cs[t]] : -1;
      ls.cok[t] = c >= 0;
      ls.ccol[t] = ls.cok[t] ? c + cx[t] : 0;
    }
  };
  // loads one round of the entry in ls, then moves ls to the next round (or entry)
  auto load = [&](double (&a)[4][TA], double (&b)[4][TB]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = ls.r0 + 4 * u + lk;
      const bool ok = r < ls.sP;
#pragma unroll
      for (int t = 0; t < TA; ++t) {
        const bool v = ok && ls.rok[t];
        const double x = ls.R[v ? (size_t)r * ls.rp + ls.rcol[t] : 0];
        a[u][t] = v ? x : 0.0;
      }
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        const bool v = ok && ls.cok[t];
        const double x = ls.C[v ? (size_t)r * ls.cp + ls.ccol[t] : 0];
        b[u][t] = v ? x : 0.0;
      }
    }
    ls.r0 += 16;
    if (ls.r0 >= ls.sP) {
      e += 4;
      if (e < tl.e_end) setup(e);
    }
  };
  if (e < tl.e_end) {
    setup(e);
    double a[4][TA], b[4][TB];
    load(a, b);
    bool valid = true;
    while (valid) {
      const bool nvalid = e < tl.e_end;
      double an[4][TA], bn[4][TB];
      if (nvalid) load(an, bn);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < TA; ++t)
#pragma unroll
          for (int v = 0; v < TB; ++v) acc[t][v] = mfma64(a[u][t], b[u][v], acc[t][v]);
      if (nvalid) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int t = 0; t < TA; ++t) a[u][t] = an[u][t];
#pragma unroll
          for (int t = 0; t < TB; ++t) b[u][t] = bn[u][t];
        }
      }
      valid = nvalid;
    }
  }
#pragma unroll
  for (int t = 0; t < TA; ++t)
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wv][t * TB + u][v][L] = acc[t][u][v];
  __syncthreads();
  const int64_t ns = d.sys_n[0];
  double* Kp = K + d.sys_d_off[0];
  const bool diag = tl.a0 == tl.b0;
  for (int idx = threadIdx.x; idx < TA * TB * 256; idx += 256) {
    const int tile = idx >> 8, v = (idx >> 6) & 3, Lx = idx & 63;
    const int i0 = 16 * (tile / TB) + (Lx >> 4) + 4 * v, k0 = 16 * (tile % TB) + (Lx & 15);
    int sa = -1, xa = i0, sb = -1, xb = k0;
    for (int a = 0; a < tl.na && sa < 0; ++a) {
      const int nbs = d.nb[tl.a0 + a];
      if (xa < nbs) sa = a; else xa -= nbs;
    }
    for (int a = 0; a < tl.nbt && sb < 0; ++a) {
      const int nbs = d.nb[tl.b0 + a];
      if (xb < nbs) sb = a; else xb -= nbs;
    }
    if (sa < 0 || sb < 0 || !((tl.mask >> (3 * sa + sb)) & 1)) continue;
    if (diag && (sa > sb || (sa == sb && xa > xb))) continue;
    const double x = 0.5 * (((red[0][tile][v][Lx] + red[1][tile][v][Lx]) + red[2][tile][v][Lx]) + red[3][tile][v][Lx]);
    const int A = tl.a0 + sa, B = tl.b0 + sb;
    const size_t ab = (size_t)(d.bo[A] + xa) * ns + d.bo[B] + xb;
    const double val = Kp[ab] + x;
    Kp[ab] = val;
    if (!(diag && sa == sb && xa == xb)) Kp[(size_t)(d.bo[B] + xb) * ns + d.bo[A] + xa] = val;
  }
}

void launch_pgather(exx_plan plan, double* K, hipStream_t st) {
  const ChunkDev& ch = plan->chunks[plan->cur];
  for (const PTClass& c : ch.pt_classes) {
    const int n = c.end - c.beg, np_ = (n + 7) / 8 * 8;
    const PTile* tl = plan->d.pt_tiles + c.beg;
    switch (c.ta * 4 + c.tb) {
#define PTC(TA, TB) case TA * 4 + TB: hipLaunchKernelGGL((k_ptile<TA, TB>), dim3(np_), dim3(256), 0, st, K, plan->d, tl, n, np_); break;
      PTC(1, 1) PTC(1, 2) PTC(1, 3) PTC(2, 1) PTC(2, 2) PTC(2, 3) PTC(3, 1) PTC(3, 2) PTC(3, 3)
#undef PTC
      default: break;
    }
  }
  const int n = ch.n_pg, np_ = (n + 7) / 8 * 8;
  if (n > 0) hipLaunchKernelGGL(k_pgather, dim3(np_), dim3(256), 0, st, K, plan->d, n, np_);
}

void launch_Y(exx_plan plan, int choice, hipStream_t st) {
  const ChunkDev& ch = plan->chunks[plan->cur];
  const int nY = ch.y_end - ch.y_beg, nYp = (nY + 7) / 8 * 8;
  if (nY <= 0) return;
  if (choice == 1) hipLaunchKernelGGL(k_Y<32>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
  else hipLaunchKernelGGL(k_Y<16>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
}

void launch_symreduce(exx_plan plan, double* K, hipStream_t st) {
  const int nF = plan->chunks[plan->cur].n_f, nFp = (nF + 7) / 8 * 8;
  if (nF <= 0) return;
  hipLaunchKernelGGL(k_symreduce, dim3(nFp), dim3(256), 0, st, K, plan->d, nF, nFp);
}
