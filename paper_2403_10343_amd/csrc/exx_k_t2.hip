// libexx kernel: the T2 pair blocks of K (k_T2).

#include "exx_dev.h"

using namespace exx;

// ---------------------------------------------------------------------------
// stage 3: T2[P, Q] = sum_{mu, l} E_P[(mu, i), l] F[mu, k, l],
//          F[mu, k, l] = sum_nu V_PQ[mu, nu] T_Q[(nu, k), l], l over N[Q].
// One workgroup of four wavefronts per canonical pair.  Columns l are
// processed in chunks of T2_COLS: the chunk of T_Q and the matching columns
// of E_P are staged in LDS with coalesced loads; each wavefront takes two
// columns.  Per column, the stage-one accumulator element v is directly the
// stage-two B operand.  The four partial sums are added in a fixed order.


// COLS: columns per staged chunk (a tuning choice: 4 or 8).  NSP = 2 (collinear spin): F is
// formed once per column and contracted with E_P^0 (d.E) and E_P^1 (E1); K^1 sits d_spin
// after K^0.
template <int NT, int NS, typename R, int COLS, int WAVES, int NSP>
__global__ __launch_bounds__(64 * WAVES) void k_T2(const double* __restrict__ V, double* __restrict__ K,
                                            DevPlan d, const int* __restrict__ items, int n_items,
                                            int n_padded, int item_base, const double* __restrict__ E1,
                                            int64_t d_spin) {
  typedef typename Mf<R>::acc A4;
  extern __shared__ double sraw[];
  R* sm = reinterpret_cast<R*>(sraw);
  const int w = xcd_task(n_padded);
  if (w >= n_items) return;
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int lr = L & 15, lk = L >> 4;
  const int p = items[item_base + w] >> 1;
  if (d.scr && d.scr[p]) return;   // V_PQ screened out: the pair adds nothing
  const bool flip = items[item_base + w] & 1;
  const int P = flip ? d.pair_b[p] : d.pair_a[p], Q = flip ? d.pair_a[p] : d.pair_b[p];
  const int aP = d.na[P], bP = d.nb[P], aQ = d.na[Q], bQ = d.nb[Q];
  const int sP = aP * bP, sQ = aQ * bQ;
  const int nQ = d.n_loc[Q], mP = d.m_loc[P];
  const int s = d.atom_sys[P];
  const int64_t ns = d.sys_n[s];
  const double* Vp = V + d.v_off[p];
  const int* t2c = d.t2col + d.t2col_off[p];   // E_P column of every column of T_Q
  const double* TQ = d.T + d.t_off[Q];
  const double* EPs[NSP];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp) EPs[sp] = (sp == 0 ? d.E : E1) + d.e_off[P];
  constexpr int PITCH = COLS + 1, RSTEP = 64 * WAVES / COLS, CPW = COLS / WAVES;
  R* sT = sm;                                  // [sQ][PITCH]
  R* sE = sm + (size_t)sQ * PITCH;             // [NSP][sP][PITCH]
  const size_t espin = (size_t)sP * PITCH;
  // V_PQ in MFMA lane order (written by the V stage's operand repack): coalesced rows
  R va[NT][NS];
  {
    const int ntp = (aP + 15) >> 4, nsq = (aQ + 3) >> 2;
    const double* vr = d.Vr + d.vr_off[2 * p + (flip && P != Q ? 1 : 0)] + L;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < NS; ++q) va[t][q] = (t < ntp && q < nsq) ? (R)vr[(t * nsq + q) * 64] : (R)0;
    (void)Vp;
  }
  const bool kv = lr < bQ, iv = lr < bP;
  // staging role: column tc of the chunk, rows r0, r0 + RSTEP, ...  The next
  // chunk is fetched into registers while the current one is computed from LDS.
  const int tc = threadIdx.x & (COLS - 1);
  const int r0 = threadIdx.x / COLS;
  constexpr int RT = (NS * 4 * NB_MAX + RSTEP - 1) / RSTEP;   // rows of T_Q per thread at most
  constexpr int RE = (NT * 16 * NB_MAX + RSTEP - 1) / RSTEP;  // rows of E_P per thread at most
  R pt[RT], pe[NSP][RE];
  auto fetch = [&](int l0) {
    const int l = l0 + tc;
    const bool cv = l < nQ;
    const int ce = cv ? t2c[l] : 0;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int r = r0 + RSTEP * i;
      const bool ok = cv && r < sQ;
      const double x = TQ[ok ? (size_t)r * nQ + l : 0];
      pt[i] = ok ? (R)x : (R)0;
    }
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
      for (int i = 0; i < RE; ++i) {
        const int r = r0 + RSTEP * i;
        const bool ok = cv && r < sP;
        const double x = EPs[sp][ok ? (size_t)r * mP + ce : 0];
        pe[sp][i] = ok ? (R)x : (R)0;
      }
  };
  A4 acc[NSP];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp) acc[sp] = A4{0, 0, 0, 0};
  fetch(0);
  for (int l0 = 0; l0 < nQ; l0 += COLS) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int r = r0 + RSTEP * i;
      if (r < sQ) sT[r * PITCH + tc] = pt[i];
    }
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
      for (int i = 0; i < RE; ++i) {
        const int r = r0 + RSTEP * i;
        if (r < sP) sE[sp * espin + r * PITCH + tc] = pe[sp][i];
      }
    __syncthreads();
    if (l0 + COLS < nQ) fetch(l0 + COLS);
#pragma unroll
    for (int h = 0; h < CPW; ++h) {
      const int c = wv * CPW + h;
      if (l0 + c < nQ) {
        // straight-line chains: NT aux tiles of P, NS nu steps of Q (compile time)
        R b[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int nu = 4 * q + lk;
          const bool ok = kv && nu < aQ;
          const R t = sT[(ok ? (nu * bQ + lr) * PITCH : 0) + c];
          b[q] = ok ? t : (R)0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          A4 F = A4{0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < NS; ++q) F = Mf<R>::mma(va[t][q], b[q], F);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // element v of F holds aux row mu of P; the E operand uses the same mu as k
            const int mu = 16 * t + Mf<R>::row(lk, v);
            const bool ok = iv && mu < aP;
#pragma unroll
            for (int sp = 0; sp < NSP; ++sp) {
              const R x = sE[sp * espin + (ok ? (mu * bP + lr) * PITCH : 0) + c];
              acc[sp] = Mf<R>::mma(ok ? x : (R)0, F[v], acc[sp]);
            }
          }
        }
      }
    }
  }
  // fixed-order reduction of the wavefront partials (binary64)
  __syncthreads();
  double* red = sraw;
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)
    for (int v = 0; v < 4; ++v) red[((sp * WAVES + wv) * 4 + v) * 64 + L] = (double)acc[sp][v];
  __syncthreads();
  if (wv < NSP) {
    const int sp = wv;   // wavefront sp writes spin sp
    double out[4];
    for (int v = 0; v < 4; ++v) {
      double x = red[((sp * WAVES) * 4 + v) * 64 + L];
      for (int w2 = 1; w2 < WAVES; ++w2) x += red[((sp * WAVES + w2) * 4 + v) * 64 + L];
      out[v] = x;
    }
    double* Ks = K + sp * d_spin + d.sys_d_off[s];
    const int bPo = d.bo[P], bQo = d.bo[Q];
    for (int v = 0; v < 4; ++v) {
      const int i = Mf<R>::row(lk, v), k = lr;
      if (i < bP && k < bQ) {
        // added to K: a chunked build may have gathered other parts of these entries already
        Ks[(size_t)(bPo + i) * ns + bQo + k] += out[v];
        if (P != Q) Ks[(size_t)(bQo + k) * ns + bPo + i] += out[v];
      }
    }
  }
}


template <int NT, typename R, int COLS, int WAVES, int NSP>
static void launch_T2_nt(exx_plan plan, int nsc, const double* V, double* K, const int* items, int beg, int n,
                         hipStream_t st) {
  const int np_ = (n + 7) / 8 * 8;
  DevPlan& d = plan->d;
  const size_t lds = t2_lds_bytes(plan->h_smax_t2, sizeof(R), COLS, WAVES, NSP);
  const dim3 g(np_), b(64 * WAVES);
  const double* E1 = plan->spin_E1;
  const int64_t ds = plan->hp.d_size;
  switch (nsc) {
#define T2NS(NS) case NS: hipLaunchKernelGGL((k_T2<NT, NS, R, COLS, WAVES, NSP>), g, b, lds, st, V, K, d, items, n, np_, beg, E1, ds); break;
    T2NS(4) T2NS(8) T2NS(10) T2NS(12)
#undef T2NS
    default: hipLaunchKernelGGL((k_T2<NT, 16, R, COLS, WAVES, NSP>), g, b, lds, st, V, K, d, items, n, np_, beg, E1, ds); break;
  }
}

template <typename R, int COLS, int WAVES, int NSP>
static void launch_T2_cols(exx_plan plan, const T2Class& c, const double* V, double* K, const int* items, int n,
                           hipStream_t st) {
  switch (c.nt) {
    case 1: launch_T2_nt<1, R, COLS, WAVES, NSP>(plan, c.ns, V, K, items, c.beg, n, st); break;
    case 2: launch_T2_nt<2, R, COLS, WAVES, NSP>(plan, c.ns, V, K, items, c.beg, n, st); break;
    case 3: launch_T2_nt<3, R, COLS, WAVES, NSP>(plan, c.ns, V, K, items, c.beg, n, st); break;
    default: launch_T2_nt<4, R, COLS, WAVES, NSP>(plan, c.ns, V, K, items, c.beg, n, st); break;
  }
}

template <typename R, int NSP>
void launch_T2_class(exx_plan plan, const T2Class& c, const double* V, double* K, const int* items,
                            hipStream_t st) {
  const int n = c.end - c.beg;
  if (n <= 0) return;
  switch (plan->tune[TUNE_T2]) {
    case 0: launch_T2_cols<R, 4, 4, NSP>(plan, c, V, K, items, n, st); break;
    case 1: launch_T2_cols<R, 8, 4, NSP>(plan, c, V, K, items, n, st); break;
    default: launch_T2_cols<R, 8, 8, NSP>(plan, c, V, K, items, n, st); break;
  }
}
template void launch_T2_class<double, 1>(exx_plan, const T2Class&, const double*, double*, const int*, hipStream_t);
template void launch_T2_class<float, 1>(exx_plan, const T2Class&, const double*, double*, const int*, hipStream_t);
template void launch_T2_class<double, 2>(exx_plan, const T2Class&, const double*, double*, const int*, hipStream_t);
