// libexx kernel: the V stage of the exchange build (k_H).

#include "exx_dev.h"

using namespace exx;

// ---------------------------------------------------------------------------
// stage 2: H'_P[(mu, j), c] for a group of consecutive atoms (its "units"
// are the 16-wide aux tiles of the group atoms) and H_COLS columns c of the
// group's second neighbourhood.  Four wavefronts per workgroup, each owning
// H_CPW of the columns and looping over all units, so the SIMDs carry equal
// work.  For every Q of the tile's Q-list, T_Q[:, columns] is staged once in
// LDS, then per (unit, column) two chained MFMAs (the first result feeding
// the second as its B operand):
//   F_c[l][mu] = sum_nu T_Q[(nu, l), c] V_PQ[mu, nu]
//   H_c[j][mu] += sum_l D_PQ[j, l] F_c[l][mu]
// G part for columns c on atom X in N[P]:
//   H_c[l][nu] += g sum_mu' E_X[(mu', c), l] V_XP[mu', nu]   (g = 2 forward).
// The chain lengths are compile-time per shape class of Q.


__device__ __forceinline__ int h_class(int ns, int nl) {
  if (ns <= 4 && nl <= 2) return 0;
  if (ns <= 10) return 1;
  return 2;
}

struct HUnits {            // unit table of the group (LDS)
  int P[GROUP_WAVES], mu0[GROUP_WAVES], slot[GROUP_WAVES], a[GROUP_WAVES], b[GROUP_WAVES], bo[GROUP_WAVES];
};

// The V and D operands of one unit and Q, read from their lane-ordered copies: one
// coalesced row per MFMA step (steps past the blocks are zero).  Binary64 reads d.Vr and
// d.Dr (second density matrix: Dr1); binary32 reads the binary32 copies d.Vr32 and d.Dr32,
// whose D rows follow the binary32 accumulator layout (all four k-steps).
template <typename R> struct HOperands;
template <> struct HOperands<double> {
  template <int NS, int NLR, int NSP>
  static __device__ __forceinline__ void load(double (&vb)[NS], double (&da)[NSP][NLR], const DevPlan& d,
                                              const double* Dr1, int pp, int orient, int mu_tile, int aQ, int bQ,
                                              int L) {
    const int nsq = (aQ + 3) >> 2, nlq = (bQ + 3) >> 2;
    const double* vrow = d.Vr + d.vr_off[2 * pp + orient] + (size_t)mu_tile * nsq * 64 + L;
#pragma unroll
    for (int q = 0; q < NS; ++q) vb[q] = q < nsq ? vrow[q * 64] : 0.0;
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp) {
      const double* dr = (sp == 0 ? d.Dr : Dr1) + d.dr_off[2 * pp + orient] + L;
#pragma unroll
      for (int q = 0; q < NLR; ++q) da[sp][q] = q < nlq ? dr[q * 64] : 0.0;
    }
  }
};
template <> struct HOperands<float> {
  template <int NS, int NLR, int NSP>
  static __device__ __forceinline__ void load(float (&vb)[NS], float (&da)[NSP][NLR], const DevPlan& d,
                                              const double*, int pp, int orient, int mu_tile, int aQ, int, int L) {
    static_assert(NSP == 1 && NLR == 4, "binary32: one density matrix, four D steps");
    const int nsq = (aQ + 3) >> 2;
    const float* vrow = d.Vr32 + d.vr_off[2 * pp + orient] + (size_t)mu_tile * nsq * 64 + L;
#pragma unroll
    for (int q = 0; q < NS; ++q) vb[q] = q < nsq ? vrow[q * 64] : 0.f;
    const float* dr = d.Dr32 + (size_t)(2 * pp + orient) * 256 + L;
#pragma unroll
    for (int q = 0; q < 4; ++q) da[0][q] = dr[q * 64];
  }
};

// One Q of a V-stage tile, all H_CPW columns of this wavefront.  The staged T_Q
// rows are read without masks: rows past s_Q (or of lanes past n_b(Q)) hold
// finite values, and they meet zero V (nu >= n_a(Q)) or zero D (l >= n_b(Q))
// operands.  A column missing from N[Q] is staged as zeros.  NSP density
// matrices (collinear spin: two, the second's D operands in Dr1) share F, and
// each has its own D contraction and accumulators.
template <int NS, int NL, int U, int NSP, typename R>
__device__ __forceinline__ void h_q(typename Mf<R>::acc (&Hc)[NSP][U][H_CPW], const R* sT, const HUnits& un,
                                    int nU, const int* qp, int Q, int aQ, int bQ, const int* lc_row, int ncols,
                                    int c0, int lr, int lk, const DevPlan& d, const double* Dr1) {
  typedef typename Mf<R>::acc A4;
  bool anyc = false;
#pragma unroll
  for (int cc = 0; cc < H_CPW; ++cc) anyc = anyc || ((c0 + cc < ncols) && lc_row[c0 + cc] >= 0);
  if (!anyc) return;
  const R* t0 = sT + lr * LDS_PITCH + c0;
  constexpr int NLR = sizeof(R) == sizeof(double) ? NL : 4;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < nU) {
      const int sl = un.slot[u];
      if (qp[sl] >= 0) {
        R vb[NS];
        R da[NSP][NLR];
        HOperands<R>::template load<NS, NLR, NSP>(vb, da, d, Dr1, qp[sl], un.P[u] <= Q ? 0 : 1, un.mu0[u] >> 4,
                                                  aQ, bQ, lk * 16 + lr);
        // the A operands of all columns first (independent LDS reads), then the chains
        R ta[NS][H_CPW];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const R* row = t0 + (q * 4 + lk) * bQ * LDS_PITCH;
#pragma unroll
          for (int cc = 0; cc < H_CPW; ++cc) ta[q][cc] = row[cc];
        }
        A4 F[H_CPW];
#pragma unroll
        for (int cc = 0; cc < H_CPW; ++cc) F[cc] = A4{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
          for (int cc = 0; cc < H_CPW; ++cc) F[cc] = Mf<R>::mma(ta[q][cc], vb[q], F[cc]);
#pragma unroll
        for (int q = 0; q < NLR; ++q)
#pragma unroll
          for (int cc = 0; cc < H_CPW; ++cc)
#pragma unroll
            for (int sp = 0; sp < NSP; ++sp) Hc[sp][u][cc] = Mf<R>::mma(da[sp][q], F[cc][q], Hc[sp][u][cc]);
      }
    }
  }
}


// NSP = 2: the two spin density matrices of a collinear-spin build in one pass (F = V T_Q is
// formed once); H'^0 goes to d.H, H'^1 to hl.H1.  Four wavefronts per SIMD for one density
// matrix (at most 128 VGPRs: measured faster than three with 168 since the V and D operands
// are coalesced rows), two for two (their accumulators double).
template <int U, typename R, int NSP, bool WIDE>
__global__ __launch_bounds__(64 * H_WAVES) __attribute__((amdgpu_waves_per_eu(NSP == 1 ? 4 : 2))) void k_H(
    const double* __restrict__ V, const double* __restrict__ D, DevPlan d, HLists hl, int n_tiles,
    int n_padded, double gscale, int mode) {
  typedef typename Mf<R>::acc A4;
  extern __shared__ double sraw[];
  R* sT = reinterpret_cast<R*>(sraw);
  __shared__ HUnits un;
  __shared__ int qm_atom[HQ_CHUNK], qm_n[HQ_CHUNK], qm_a[HQ_CHUNK], qm_b[HQ_CHUNK], qm_bo[HQ_CHUNK];
  __shared__ int qm_lc[HQ_CHUNK][H_COLS], qm_p[HQ_CHUNK][GROUP_ATOMS];
  __shared__ int64_t qm_toff[HQ_CHUNK];
  const int ti = xcd_task(n_padded);
  if (ti >= n_tiles) return;
  const GTile tl = hl.tiles[ti];
  const int g = tl.grp;
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int lr = L & 15, lk = L >> 4;
  const int u0 = d.grp_unit_ptr[g];
  const int nU = d.grp_unit_ptr[g + 1] - u0;
  if (threadIdx.x < nU) {
    const Unit x = d.grp_units[u0 + threadIdx.x];
    un.P[threadIdx.x] = x.P;
    un.mu0[threadIdx.x] = x.mu0;
    un.slot[threadIdx.x] = x.slot;
    un.a[threadIdx.x] = d.na[x.P];
    un.b[threadIdx.x] = d.nb[x.P];
    un.bo[threadIdx.x] = d.bo[x.P];
  }
  const int* gcol = d.grp_cols + tl.col_beg;
  const int ncols = tl.ncols;
  const int c0 = wv * H_CPW;
  A4 Hc[NSP][U][H_CPW];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int cc = 0; cc < H_CPW; ++cc) Hc[sp][u][cc] = A4{0, 0, 0, 0};
  const int tc = threadIdx.x % H_COLS;
  const int tstep = blockDim.x / H_COLS;
  // LDS: T_Q[:, tile columns]
  // rows read past s_Q stay finite (the G-only pass has no Q loop and no dynamic LDS)
  if (mode != H_G_ADD)
    for (int i = threadIdx.x; i < hl.v_base; i += blockDim.x) sT[i] = (R)0;
  __syncthreads();
  for (int e0 = mode == H_G_ADD ? tl.q_end : tl.q_beg; e0 < tl.q_end; e0 += HQ_CHUNK) {
    const int nchunk = min(HQ_CHUNK, tl.q_end - e0);
    __syncthreads();
    for (int t = threadIdx.x; t < nchunk * H_COLS; t += blockDim.x) {
      const int ei = t / H_COLS, c = t % H_COLS;
      const Slot4 qe = hl.gq[e0 + ei];
      const int Q = qe.atom;
      int lc = (c < ncols) ? d.map1[d.map_off[Q] + gcol[c]] : -1;
      // periodic: the column's atom L at image b lies in N[Q + q] only if n_QL = b - q
      if (d.periodic && lc >= 0 &&
          d.pimg[(size_t)Q * d.n_atoms + d.atom_of_col[gcol[c]]] + qe.img - IMG0 != d.grp_colimg[tl.col_beg + c])
        lc = -1;
      qm_lc[ei][c] = lc;
      if (c == 0) {
        qm_atom[ei] = Q;
        qm_n[ei] = d.n_loc[Q];
        qm_a[ei] = d.na[Q];
        qm_b[ei] = d.nb[Q];
        qm_bo[ei] = d.bo[Q];
        qm_toff[ei] = d.t_off[Q];
        const int pp[3] = {qe.p0, qe.p1, qe.p2};
        // a pair whose V block is screened out takes no part (as if the block were zero)
        for (int k = 0; k < GROUP_ATOMS; ++k) qm_p[ei][k] = (pp[k] >= 0 && d.scr && d.scr[pp[k]]) ? -1 : pp[k];
      }
    }
    __syncthreads();
    for (int ei = 0; ei < nchunk; ++ei) {
      const int Q = qm_atom[ei], aQ = qm_a[ei], bQ = qm_b[ei], nQ = qm_n[ei], sQ = aQ * bQ;
      const int lcq = qm_lc[ei][tc];
      const double* TQ = d.T + qm_toff[ei] + (lcq >= 0 ? lcq : 0);
      for (int r = threadIdx.x / H_COLS; r < sQ; r += tstep)
        sT[r * LDS_PITCH + tc] = (R)(lcq >= 0 ? TQ[(size_t)r * nQ] : 0.0);
      __syncthreads();
      const int nsQ = (aQ + 3) >> 2, nlQ = (bQ + 3) >> 2;
      switch (h_class(nsQ, nlQ)) {
        case 0: h_q<4, 2, U, NSP, R>(Hc, sT, un, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1); break;
        case 1: h_q<10, 4, U, NSP, R>(Hc, sT, un, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1); break;
        default:   // more than 40 aux functions on Q: plans with such a species only
          if constexpr (WIDE) h_q<16, 4, U, NSP, R>(Hc, sT, un, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1);
          break;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // G part (this wavefront's columns)
  for (int e = tl.x_beg; e < tl.x_end; ++e) {
    const Slot4 xe = hl.gx[e];
    const int X = xe.atom;
    const int aX = d.na[X], bX = d.nb[X], mX = d.m_loc[X], boX = d.bo[X];
    const int pp[3] = {xe.p0, xe.p1, xe.p2};
    const int ecol[3] = {xe.e0, xe.e1, xe.e2};   // periodic: E_X column of each slot atom's basis
    const double* EXs[NSP];
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp) EXs[sp] = (sp == 0 ? d.E : hl.E1) + d.e_off[X];
    const int* m2X = d.periodic ? nullptr : d.map2 + d.map_off[X];
#pragma unroll
    for (int cc = 0; cc < H_CPW; ++cc) {
      const int c = c0 + cc;
      const int ic = (c < ncols) ? gcol[c] - boX : -1;
      // periodic: the column must be on X at the image of this entry
      if (ic >= 0 && ic < bX && (!d.periodic || d.grp_colimg[tl.col_beg + c] == xe.img)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u < nU) {
            const int p = pp[un.slot[u]];
            if (p >= 0 && !(d.scr && d.scr[p])) {
              const int P = un.P[u], aP = un.a[u], bP = un.b[u];
              const int muB = un.mu0[u] + lr;
              const bool muv = muB < aP;
              const int colx = lr < bP ? (d.periodic ? ecol[un.slot[u]] + lr : m2X[un.bo[u] + lr]) : 0;
              const size_t xo = colx + (size_t)ic * mX;
              const int nsx = (aX + 3) / 4;
              // V_PX[muB][m2] from the lane-ordered copy (zero outside the block)
              const double* vrx = d.Vr + d.vr_off[2 * p + (P <= X ? 0 : 1)] + (size_t)(un.mu0[u] >> 4) * nsx * 64 + L;
              for (int q = 0; q < nsx; ++q) {
                const int m2 = 4 * q + lk;
                const bool mv = m2 < aX;
                const bool oka = mv && lr < bP, okb = mv && muv;
                const double b = vrx[q * 64];
                const R bv = okb ? (R)(gscale * b) : (R)0;
#pragma unroll
                for (int sp = 0; sp < NSP; ++sp) {
                  const double a = EXs[sp][oka ? xo + (size_t)(m2 * bX) * mX : xo];
                  Hc[sp][u][cc] = Mf<R>::mma(oka ? (R)a : (R)0, bv, Hc[sp][u][cc]);
                }
              }
            }
          }
        }
      }
    }
  }
  // store, or add to H'
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < nU) {
      const int P = un.P[u], aP = un.a[u], bP = un.b[u], mP = d.m_loc[P];
      const int muB = un.mu0[u] + lr;
      const int* m2P = d.periodic ? nullptr : d.map2 + d.map_off[P];
#pragma unroll
      for (int sp = 0; sp < NSP; ++sp) {
        double* HP = (sp == 0 ? d.H : hl.H1) + d.h_off[P];
#pragma unroll
        for (int cc = 0; cc < H_CPW; ++cc) {
          const int c = c0 + cc;
          const int col = (c < ncols) ? (d.periodic ? d.grp_cmap[(size_t)(tl.col_beg + c) * 3 + un.slot[u]]
                                                    : m2P[gcol[c]])
                                      : -1;
          if (col >= 0 && muB < aP) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int j = Mf<R>::row(lk, v);
              if (j < bP) {
                double* h = HP + (size_t)(muB * bP + j) * mP + col;
                *h = mode == H_WRITE ? (double)Hc[sp][u][cc][v] : *h + (double)Hc[sp][u][cc][v];
              }
            }
          }
        }
      }
    }
  }
}


template <typename R, int NSP>
void launch_H_lists(exx_plan plan, const double* V, const double* D, const HLists& hl, int n, double gscale,
                           int mode, hipStream_t st) {
  if (n <= 0) return;
  const HostPlan& hp = plan->hp;
  const int np_ = (n + 7) / 8 * 8;
  const size_t lds = mode == H_G_ADD ? 0 : (sizeof(R) == sizeof(double) ? plan->h_lds : plan->h_lds32);
  const dim3 grid(np_), blk(64 * H_WAVES);
  // the widest shape class (chains of 16 aux steps) is compiled in only where a species needs it
  const bool wide = *std::max_element(hp.na.begin(), hp.na.end()) > 40;
#define KH(UU, W) hipLaunchKernelGGL((k_H<UU, R, NSP, W>), grid, blk, lds, st, V, D, plan->d, hl, n, np_, gscale, mode)
  if (hp.h_waves <= 2) { if (wide) KH(2, true); else KH(2, false); }
  else if (hp.h_waves <= 5) { if (wide) KH(5, true); else KH(5, false); }
  else { if (wide) KH(8, true); else KH(8, false); }
#undef KH
}
template void launch_H_lists<double, 1>(exx_plan, const double*, const double*, const HLists&, int, double, int,
                                        hipStream_t);
template void launch_H_lists<float, 1>(exx_plan, const double*, const double*, const HLists&, int, double, int,
                                       hipStream_t);
template void launch_H_lists<double, 2>(exx_plan, const double*, const double*, const HLists&, int, double, int,
                                        hipStream_t);
