// libexx kernel: dE/dV pair blocks of the backward pass (k_dV).

#include "exx_dev.h"

using namespace exx;

// dE/dV.  tau_{mu nu} = tr(C^mu D C^nu D) = 2 (tA + tB),
//   tA[mu][nu] = sum_{i in P, l in Q} E_P[(mu, i), l] E_Q[(nu, l), i]
//   tB[mu][nu] = sum_{i in P, j in N[Q]} E_P[(mu, i), j] Y[(nu, i), j],
//   Y[(nu, i), j] = sum_{l in Q} D[i, l] T_Q[(nu, l), j].
// Off-site stored entries carry both V_{mu nu} and V_{nu mu}.  Same LDS
// staging as the T2 kernel (columns j of N[Q] in chunks).

// One workgroup of eight wavefronts per canonical pair, one column of each
// 8-column chunk per wavefront; compile-time shape per pair class (aux tiles
// of 16 of P and Q, basis steps of 4 of Q and P); the next chunk is fetched
// into registers while the current one is used from LDS.

template <int NTP, int NTQ, int NLQ, int NIP>
__global__ __launch_bounds__(64 * DV_WAVES) void k_dV(const double* __restrict__ V, const double* __restrict__ D,
                                                     double* __restrict__ dV, DevPlan d, const int* __restrict__ items,
                                                     const double* __restrict__ gE, int n_items, int n_padded, int item_base) {
  extern __shared__ double sm[];
  const int w = xcd_task(n_padded);
  if (w >= n_items) return;
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int lr = L & 15, lk = L >> 4;
  const int p = items[item_base + w];
  const int P = d.pair_a[p], Q = d.pair_b[p];
  const int aP = d.na[P], bP = d.nb[P], aQ = d.na[Q], bQ = d.nb[Q];
  const int sP = aP * bP, sQ = aQ * bQ;
  const int nQ = d.n_loc[Q], mP = d.m_loc[P], mQ = d.m_loc[Q];
  const int s = d.atom_sys[P];
  const int64_t ns = d.sys_n[s];
  const int* colP = d.dvcol + d.dvcol_off[p];   // E_P column of every column of T_Q
  const int cPQ = d.dv_cp[p], cQP = d.dv_cq[p];   // E_P column of Q's basis, E_Q column of P's
  const double* TQ = d.T + d.t_off[Q];
  const double* EP = d.E + d.e_off[P];
  const double* EQ = d.E + d.e_off[Q];
  double* sT = sm;
  double* sE = sm + (size_t)sQ * DV_PITCH;
  // D_PQ fragments: A[i][l] with i = lr, l = 4 q + lk
  double da[NLQ];
  const double* DPQ = D + d.sys_d_off[s] + (size_t)d.bo[P] * ns + d.bo[Q];
#pragma unroll
  for (int q = 0; q < NLQ; ++q) {
    const int l = 4 * q + lk;
    const bool ok = lr < bP && l < bQ;
    const double x = DPQ[ok ? (size_t)lr * ns + l : 0];
    da[q] = ok ? x : 0.0;
  }
  d4 acc[NTP][NTQ];
#pragma unroll
  for (int x = 0; x < NTP; ++x)
#pragma unroll
    for (int y = 0; y < NTQ; ++y) acc[x][y] = d4{0, 0, 0, 0};
  const int tc = threadIdx.x & (DV_COLS - 1), r0 = threadIdx.x / DV_COLS;
  constexpr int RT = (NTQ * 16 * NB_MAX + DV_RSTEP - 1) / DV_RSTEP;
  constexpr int RE = (NTP * 16 * NB_MAX + DV_RSTEP - 1) / DV_RSTEP;
  double pt[RT], pe[RE];
  auto fetch = [&](int l0) {
    const int l = l0 + tc;
    const bool cv = l < nQ;
    const int ce = cv ? colP[l] : 0;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int r = r0 + DV_RSTEP * i;
      const bool ok = cv && r < sQ;
      const double x = TQ[ok ? (size_t)r * nQ + l : 0];
      pt[i] = ok ? x : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RE; ++i) {
      const int r = r0 + DV_RSTEP * i;
      const bool ok = cv && r < sP;
      const double x = EP[ok ? (size_t)r * mP + ce : 0];
      pe[i] = ok ? x : 0.0;
    }
  };
  fetch(0);
  for (int l0 = 0; l0 < nQ; l0 += DV_COLS) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int r = r0 + DV_RSTEP * i;
      if (r < sQ) sT[r * DV_PITCH + tc] = pt[i];
    }
#pragma unroll
    for (int i = 0; i < RE; ++i) {
      const int r = r0 + DV_RSTEP * i;
      if (r < sP) sE[r * DV_PITCH + tc] = pe[i];
    }
    __syncthreads();
    if (l0 + DV_COLS < nQ) fetch(l0 + DV_COLS);
    const int c = wv;
    if (l0 + c < nQ) {
#pragma unroll
      for (int y = 0; y < NTQ; ++y) {
        // Yt[i][nu] = sum_l D[i, l] T_Q[(nu, l), j]
        d4 Yt = d4{0, 0, 0, 0};
        const int nu = 16 * y + lr;
#pragma unroll
        for (int q = 0; q < NLQ; ++q) {
          const int lq = 4 * q + lk;
          const bool ok = nu < aQ && lq < bQ;
          const double b = sT[(ok ? (nu * bQ + lq) * DV_PITCH : 0) + c];
          Yt = mfma64(da[q], ok ? b : 0.0, Yt);
        }
        // tB[mu][nu] += sum_i E_P[(mu, i), j] Yt[i][nu]
#pragma unroll
        for (int x = 0; x < NTP; ++x) {
          const int mu = 16 * x + lr;
#pragma unroll
          for (int v = 0; v < NIP; ++v) {
            const int i = 4 * v + lk;
            const bool ok = mu < aP && i < bP;
            const double a = sE[(ok ? (mu * bP + i) * DV_PITCH : 0) + c];
            acc[x][y] = mfma64(ok ? a : 0.0, Yt[v], acc[x][y]);
          }
        }
      }
    }
  }
  // tA: k = (i, l) flattened, k-steps dealt round-robin to the wavefronts
  {
    const int K2 = bP * bQ, nk = (K2 + 3) >> 2;
    for (int q = wv; q < nk; q += DV_WAVES) {
      const int kf = 4 * q + lk;
      const bool kv = kf < K2;
      const int i = kv ? kf / bQ : 0, l = kv ? kf - i * bQ : 0;
      const int cP = kv ? cPQ + l : 0, cQ = kv ? cQP + i : 0;
#pragma unroll
      for (int y = 0; y < NTQ; ++y) {
        const int nu = 16 * y + lr;
        const bool okb = kv && nu < aQ;
        const double b = EQ[okb ? (size_t)(nu * bQ + l) * mQ + cQ : 0];
#pragma unroll
        for (int x = 0; x < NTP; ++x) {
          const int mu = 16 * x + lr;
          const bool oka = kv && mu < aP;
          const double a = EP[oka ? (size_t)(mu * bP + i) * mP + cP : 0];
          acc[x][y] = mfma64(oka ? a : 0.0, okb ? b : 0.0, acc[x][y]);
        }
      }
    }
  }
  // fixed-order reduction of the wavefront partials, tile by tile
  const double f = -0.5 * gE[s] * (P != Q ? 2.0 : 1.0);
  double* dVp = dV + d.v_off[p];
#pragma unroll
  for (int x = 0; x < NTP; ++x)
#pragma unroll
    for (int y = 0; y < NTQ; ++y) {
      __syncthreads();
      for (int v = 0; v < 4; ++v) sm[(wv * 4 + v) * 64 + L] = acc[x][y][v];
      __syncthreads();
      if (wv == 0) {
        for (int v = 0; v < 4; ++v) {
          double t = sm[v * 64 + L];
          for (int w2 = 1; w2 < DV_WAVES; ++w2) t += sm[(w2 * 4 + v) * 64 + L];
          const int mu = 16 * x + lk + 4 * v, nu = 16 * y + lr;
          if (mu < aP && nu < aQ) dVp[(size_t)mu * aQ + nu] = f * t;
        }
      }
    }
}


template <int NTP, int NTQ>
static void launch_dV_t(exx_plan plan, const DVClass& c, const double* V, const double* D, double* dV, const double* gE,
                        hipStream_t st) {
  const int n = c.end - c.beg, np_ = (n + 7) / 8 * 8;
  DevPlan& d = plan->d;
  const size_t lds = std::max((size_t)2 * plan->h_smax_t2 * DV_PITCH, (size_t)DV_WAVES * 4 * 64) * sizeof(double);
  const dim3 g(np_), b(64 * DV_WAVES);
  const int key = c.nlq * 8 + c.nip;
  // basis steps of 4 of Q and P: 1..4 each
  switch (key) {
#define DVC(NL, NI) case NL * 8 + NI: hipLaunchKernelGGL((k_dV<NTP, NTQ, NL, NI>), g, b, lds, st, V, D, dV, d, d.dv_items, gE, n, np_, c.beg); break;
    DVC(1, 1) DVC(1, 2) DVC(1, 3) DVC(1, 4) DVC(2, 1) DVC(2, 2) DVC(2, 3) DVC(2, 4)
    DVC(3, 1) DVC(3, 2) DVC(3, 3) DVC(3, 4) DVC(4, 1) DVC(4, 2) DVC(4, 3) DVC(4, 4)
#undef DVC
    default: break;
  }
}

void launch_dV(exx_plan plan, const double* V, const double* D, double* dV, const double* gE, hipStream_t st) {
  for (const DVClass& c : plan->chunks[plan->cur].dv_classes) {
    if (c.end <= c.beg) continue;
    const int k = c.ntp * 8 + c.ntq;
    switch (k) {
#define DVT(TP, TQ) case TP * 8 + TQ: launch_dV_t<TP, TQ>(plan, c, V, D, dV, gE, st); break;
      DVT(1, 1) DVT(1, 2) DVT(1, 3) DVT(1, 4) DVT(2, 1) DVT(2, 2) DVT(2, 3) DVT(2, 4)
      DVT(3, 1) DVT(3, 2) DVT(3, 3) DVT(3, 4) DVT(4, 1) DVT(4, 2) DVT(4, 3) DVT(4, 4)
#undef DVT
      default: break;
    }
  }
}
