// libexx: RI-LVL exact-exchange build on MI355X (gfx950).
//
// Evaluates K_ik = sum_{jl} sum_{mu nu} C^mu_ij V_{mu nu} C^nu_kl D_jl for
// non-periodic systems (lattice vector R = 0 of Eq. realspace_exchange) and
// E_x = -1/4 sum K_ik D_ik.  Writing C^mu = M^mu + M^mu^T with M^mu the rows
// of C^mu on the atom of mu (on-site block halved), the sum splits into the
// terms of the paper's pair-grouped form (Eq. ri_lvl_exchange_matrix with the
// intermediates of Eq. temp):
//   T2 = sum V M^mu D M^nu^T      (the F*E term)
//   T1 = sum V M^mu D M^nu        (the G term)
//   T3 = sum V M^mu^T D M^nu      (the H term)
//   K  = T2 + T3 + T1 + T1^T.
// The paper's form carries 2G and is symmetrised here: with
// H'_P = sum_Q (V_PQ (x) D_PQ) T_Q + 2 G, the product X = T^T H' equals
// T3 + 2 T1^T and K = T2 + (X + X^T) / 2.
//
// Kernels of a build (all contractions on FP64 MFMA 16x16x4, or FP32 16x16x4 for the
// far pair terms of a mixed build):
//   k_repack     C pair blocks -> row-owned T_P
//   k_rowD       E_P = T_P D over N2[P]              (LDS-tiled GEMM over k-runs)
//   k_vdrepack   V_PQ and D_PQ in MFMA lane order    (coalesced operand rows)
//   k_H          H'_P: F = V T_Q, D contraction, G part (chained MFMAs per Q)
//   k_T2         T2 pair blocks into K               (two chained MFMA stages)
//   k_Y          Y_P = T_P^T H'_P                    (LDS-tiled batched GEMM)
//   k_symreduce  K = T2 + (X + X^T)/2 gathered from Y, owner-computes, atomic-free
//   k_energy_*   E_x per system, fixed-order reduction
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/exx.h"
#include "exx_internal.h"

using namespace exx;

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64: lane L supplies A[L%16][L/16] and B[L/16][L%16];
// accumulator element v of lane L is C[L/16 + 4v][L%16].
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Arithmetic of the pair-term kernels (V stage, T2) by element type R.
// Both 16x16x4 MFMAs take A[L%16][L/16] and B[L/16][L%16]; they differ in
// where the result lands: accumulator element v of lane L is row
// row(L/16, v) of the 16 x 16 result (column L%16).  A chained product uses
// element v as its B operand, i.e. as k-row row(L/16, v).
template <typename R> struct Mf;
template <> struct Mf<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mf<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      return fail(_e == hipErrorOutOfMemory ? EXX_ENOMEM : EXX_EDEVICE,        \
                  std::string(#expr) + ": " + hipGetErrorString(_e));          \
  } while (0)

// ---------------------------------------------------------------------------
// device-side plan

struct DevPlan {
  int n_atoms, n_sys;
  int *nb, *na, *atom_sys, *bo;
  int64_t *sys_n, *sys_d_off;
  int *nbr_ptr, *nbr_atom, *nbr_pair, *nbr_lcol, *nbr_owner;
  int *pair_a, *pair_b;
  int64_t *c_off, *v_off;
  int *n_loc, *m_loc;
  int64_t *map_off, *col1g_off, *col2g_off;
  int *map1, *map2, *col1g, *col2g;
  int64_t *t_off, *e_off;
  EItem* e_items;
  int *ct_run_ptr, *ct_klen;
  Run* runs;
  EItem* gd_items;
  int *gd_run_ptr, *gd_klen;
  Run* gd_runs;
  double* pos;
  int *grp_first, *grp_unit_ptr, *grp_col_ptr, *grp_cols;
  Unit* grp_units;
  GTile* g_tiles;
  Slot4 *gq, *gx;
  int* t2_items;
  GTile *hm_tiles_near, *hm_tiles_far;
  Slot4 *hm_q_near, *hm_x_near, *hm_q_far, *hm_x_far;
  int* t2m_items;
  int* dv_items;
  FItem* f_items;
  int* f_plist;
  int *en_sys, *en_beg, *en_end;
  YTile* y_tiles;
  int64_t* y_off;
  double *T, *E, *H, *Y, *GD, *sC, *sV, *epart;
  // The V-stage operands in MFMA lane order, rebuilt from V and D before every V stage:
  // per canonical pair p and orientation o (0: P = pair_a, Q = pair_b; 1: swapped) at
  // Vr + vr_off[2 p + o], [16-wide aux tile t of P][4-wide aux step q of Q][lane L] =
  // V_PQ[16 t + L % 16][4 q + L / 16], and at Dr + dr_off[2 p + o], [basis step q of Q][lane L] =
  // D_PQ[L % 16][L / 16 + 4 q] (zero outside the blocks).  Each MFMA operand is then one
  // coalesced 512-byte row instead of a gather over 16 rows of V or D.
  int64_t *vr_off, *dr_off;
  double *Vr, *Dr;
};

constexpr int N_STAGE_EV = EXX_N_STAGES + 1;   // stage boundaries, start and end included
constexpr int MAX_PROFILED = 512;

// tunable tile choices (exx_plan_autotune): E GEMM k-chunk {16, 32}; T2 column
// chunk x wavefronts {4 x 4, 8 x 4, 8 x 8}; Y GEMM k-chunk {16, 32}
enum { TUNE_E = 0, TUNE_T2 = 1, TUNE_Y = 2, N_TUNE = 3, N_CAND = 3 };
static const int kTuneCands[N_TUNE] = {2, 3, 2};

// T_Q and nsp E_P column chunks, or the nsp fixed-order reduction buffers
static size_t t2_lds_bytes(int smax, size_t esize, int cols, int waves, int nsp = 1) {
  return std::max((size_t)(1 + nsp) * smax * (cols + 1) * esize, (size_t)nsp * waves * 4 * 64 * sizeof(double));
}

struct exx_plan_s {
  HostPlan hp;
  int tune[N_TUNE] = {0, 1, 0};     // defaults: E 16, T2 8 columns, Y 16
  float tune_ms[N_TUNE][N_CAND] = {};
  bool tuned = false;
  bool host_only = false;
  int device = -1;
  DevPlan d{};
  std::vector<void*> allocs;
  int64_t dev_bytes = 0;
  // optional per-stage timing of build_K (HIP events on the build's stream)
  bool profiling = false;
  std::vector<hipEvent_t> events;   // MAX_PROFILED * N_STAGE_EV, created lazily
  int n_recorded = 0;
  int t2_nt = 4;                    // aux tiles of 16 needed by the largest atom
  size_t h_lds = 0;                 // dynamic LDS bytes of k_H (binary64)
  size_t t2_lds = 0;                // dynamic LDS bytes of k_T2 (binary64)
  size_t h_lds32 = 0, t2_lds32 = 0; // the same for the binary32 kernels
  int h_vbase = 0, h_dbase = 0;     // element offsets of V and D in k_H's LDS
  int h_smax_t2 = 1;                // largest n_aux * n_basis (T2 staging)
  int lds_max = 0;                  // LDS bytes a workgroup may use on the plan's device
  std::vector<void*> mixed_allocs;  // device copies of the mixed-precision lists
  int64_t mixed_bytes = 0;
  bool mixed_uploaded = false;
  hipGraph_t graph = nullptr;       // captured build_K (exx_graph_build)
  hipGraphExec_t graph_exec = nullptr;
  double* dC_scratch = nullptr;     // gradient buffers used when the caller passes NULL
  double* dV_scratch = nullptr;
  double* spin_E1 = nullptr;        // E and H' of the second spin (build_K_spin), allocated on first use
  double* spin_H1 = nullptr;
  double* spin_Dr1 = nullptr;       // lane-ordered D operands of the second spin
  int64_t dr_total = 0;             // doubles of the lane-ordered D operands (DevPlan::Dr)
};

template <typename X>
static int upload(exx_plan_s* p, X*& dst, const std::vector<X>& src, bool mixed = false) {
  dst = nullptr;
  if (src.empty()) return 0;
  size_t bytes = src.size() * sizeof(X);
  HIP_TRY(hipMalloc((void**)&dst, bytes));
  (mixed ? p->mixed_allocs : p->allocs).push_back(dst);
  (mixed ? p->mixed_bytes : p->dev_bytes) += bytes;
  HIP_TRY(hipMemcpy(dst, src.data(), bytes, hipMemcpyHostToDevice));
  return 0;
}

static int alloc_buf(exx_plan_s* p, double*& dst, int64_t n) {
  dst = nullptr;
  if (n <= 0) return 0;
  HIP_TRY(hipMalloc((void**)&dst, n * sizeof(double)));
  p->allocs.push_back(dst);
  p->dev_bytes += n * sizeof(double);
  return 0;
}

// ---------------------------------------------------------------------------
// screening on the device: one workgroup per atom A, all B of its system in
// chunks of 256, ordered compaction by a workgroup prefix sum.

__device__ __forceinline__ bool within_cut(const double* pos, int a, int b, double rc2) {
  double dx = __dsub_rn(pos[3 * a], pos[3 * b]);
  double dy = __dsub_rn(pos[3 * a + 1], pos[3 * b + 1]);
  double dz = __dsub_rn(pos[3 * a + 2], pos[3 * b + 2]);
  double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  return r2 <= rc2;
}

__global__ __launch_bounds__(256) void k_nbr_count(const double* pos, const int* atom_sys,
                                                   const int* sys_atom_off, double rc2, int* count) {
  const int a = blockIdx.x;
  const int s = atom_sys[a];
  const int lo = sys_atom_off[s], hi = sys_atom_off[s + 1];
  __shared__ int part[256];
  int c = 0;
  for (int b = lo + threadIdx.x; b < hi; b += 256) c += within_cut(pos, a, b, rc2) ? 1 : 0;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[a] = part[0];
}

__global__ __launch_bounds__(256) void k_nbr_fill(const double* pos, const int* atom_sys,
                                                  const int* sys_atom_off, double rc2,
                                                  const int* ptr, int* out) {
  const int a = blockIdx.x;
  const int s = atom_sys[a];
  const int lo = sys_atom_off[s], hi = sys_atom_off[s + 1];
  __shared__ int scan[256];
  int base = ptr[a];
  for (int b0 = lo; b0 < hi; b0 += 256) {
    const int b = b0 + threadIdx.x;
    const int f = (b < hi && within_cut(pos, a, b, rc2)) ? 1 : 0;
    scan[threadIdx.x] = f;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {  // inclusive Hillis-Steele scan
      int v = (threadIdx.x >= w) ? scan[threadIdx.x - w] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) out[base + scan[threadIdx.x] - 1] = b;
    base += scan[255];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stage 0: row-owned coefficients T_P from the canonical C pair blocks.
// One workgroup per neighbour entry (P, J): the s_P x n_basis(J) sub-block.

__global__ __launch_bounds__(256) void k_repack(const double* __restrict__ C, DevPlan d) {
  const int k = blockIdx.x;
  const int P = d.nbr_owner[k], J = d.nbr_atom[k], p = d.nbr_pair[k];
  const int aP = d.na[P], bP = d.nb[P], bJ = d.nb[J], aJ = d.na[J];
  const int nP = d.n_loc[P], lc = d.nbr_lcol[k];
  const int sP = aP * bP;
  const double* Cp = C + d.c_off[p];
  double* TP = d.T + d.t_off[P];
  const int nel = sP * bJ;
  for (int e = threadIdx.x; e < nel; e += 256) {
    const int r = e / bJ, j = e - r * bJ;
    const int mu = r / bP, i = r - mu * bP;
    double v;
    if (P < J)
      v = Cp[(size_t)(mu * bP + i) * bJ + j];
    else if (P > J)
      v = Cp[(size_t)((aJ + mu) * bJ + j) * bP + i];
    else
      v = 0.5 * Cp[(size_t)(mu * bP + i) * bP + j];
    TP[(size_t)r * nP + lc + j] = v;
  }
}

// ---------------------------------------------------------------------------
// Workgroups are dealt to the eight XCDs in turn.  Tasks are renumbered so
// that each XCD receives one contiguous range of the (locality-ordered) task
// list: neighbouring tasks share T / E / D blocks in that XCD's L2.  The grid
// is padded to a multiple of eight workgroups.
__device__ __forceinline__ int xcd_task(int n_padded) {
  const int per = n_padded >> 3;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// ---------------------------------------------------------------------------
// stage 1 (and its adjoint): O_P = A_P D restricted to block-sparse D, where
// A_P has s_P rows.  Forward: A = T_P (columns N[P]), O = E_P (columns
// N2[P]).  Gradient: A = H_P (columns N2[P]), O = G_P (columns N[P]).  One
// 32 x 32 output tile per wavefront; k runs over the runs of input atoms J
// whose neighbourhood meets the tile's atoms.

struct RowD {
  const double* A;
  const int64_t* a_off;
  const int* a_ld;
  double* O;
  const int64_t* o_off;
  const int* o_ld;
  const int* ocolg;
  const int64_t* ocolg_off;
  const EItem* items;
  const int* run_ptr;
  const int* klen;
  const Run* runs;
};

// Batched GEMM: 64 x 64 output tile per workgroup of four wavefronts (32 x 32
// each), k in steps of 16 staged through double-buffered LDS.  The k index
// runs over the basis functions of the input atoms listed for the tile's
// column tile (runs of consecutive atoms: column lcol.. of A, row grow.. of D).
constexpr int ET = 64, EPITCH = ET + 4;

// EK: k-chunk per LDS stage (a tuning choice: 16 or 32).  NSP = 2 (collinear spin): the
// products with D (into r.O) and D1 (into O1) in one pass, the A_P tile staged once.
template <int EK, int NSP>
__global__ __launch_bounds__(256) void k_rowD(const double* __restrict__ D, RowD r, DevPlan d, int n_items,
                                              int n_padded, const double* __restrict__ D1, double* __restrict__ O1) {
  __shared__ double As[2][EK][EPITCH];
  __shared__ double Bs[NSP][2][EK][EPITCH];
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
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int n = it.c0 + nb0 + x;
    gcn[x] = n < ldo ? r.ocolg[r.ocolg_off[P] + n] : -1;
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
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const bool okd = okb && gcn[x] >= 0;
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp) {
          const double z = Dsp[sp][okd ? (size_t)gr * ns + gcn[x] : 0];
          vb[sp][pz][x] = okd ? z : 0.0;
        }
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int x = 0; x < NA_; ++x) As[buf][ka][ma + MS * x] = va[x];
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
      for (int pz = 0; pz < NP; ++pz)
#pragma unroll
        for (int x = 0; x < 4; ++x) Bs[sp][buf][16 * pz + kb][nb0 + x] = vb[sp][pz][x];
  };
  d4 acc[NSP][2][2];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[sp][x][y] = d4{0, 0, 0, 0};
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < klen; k0 += EK) {
    const bool more = k0 + EK < klen;
    if (more) gload(k0 + EK);
#pragma unroll
    for (int ks = 0; ks < EK; ks += 4) {
      const double a0 = As[buf][ks + lk][wm + lr], a1 = As[buf][ks + lk][wm + 16 + lr];
#pragma unroll
      for (int sp = 0; sp < NSP; ++sp) {
        const double b0 = Bs[sp][buf][ks + lk][wn + lr], b1 = Bs[sp][buf][ks + lk][wn + 16 + lr];
        acc[sp][0][0] = mfma64(a0, b0, acc[sp][0][0]);
        acc[sp][0][1] = mfma64(a0, b1, acc[sp][0][1]);
        acc[sp][1][0] = mfma64(a1, b0, acc[sp][1][0]);
        acc[sp][1][1] = mfma64(a1, b1, acc[sp][1][1]);
      }
    }
    if (more) {
      sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
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

// V_PQ[mu][nu] (mu on P, nu on Q) from the canonical V block of pair p.
__device__ __forceinline__ double v_elem(const double* Vp, int P, int Q, int aP, int aQ, int mu, int nu) {
  return (P <= Q) ? Vp[mu * aQ + nu] : Vp[nu * aP + mu];
}

// The V-stage operands in MFMA lane order (DevPlan::Vr, Dr), one workgroup per canonical
// pair, both orientations.
// V == nullptr: the D operands only (into Dr)
__global__ __launch_bounds__(256) void k_vdrepack(const double* __restrict__ V, const double* __restrict__ D,
                                                 double* __restrict__ Dr, DevPlan d) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const double* Vp = V ? V + d.v_off[p] : nullptr;
  const int s = d.atom_sys[A];
  const int64_t ns = d.sys_n[s];
  const double* Ds = D + d.sys_d_off[s];
  for (int o = 0; o < (A == B ? 1 : 2); ++o) {
    const int P = o ? B : A, Q = o ? A : B;
    const int aP = d.na[P], aQ = d.na[Q], bP = d.nb[P], bQ = d.nb[Q];
    const int nsq = (aQ + 3) / 4;
    double* vr = d.Vr + d.vr_off[2 * p + o];
    const int nv = V ? (int)(d.vr_off[2 * p + o + 1] - d.vr_off[2 * p + o]) : 0;
    for (int e = threadIdx.x; e < nv; e += 256) {
      const int L = e & 63, tq = e >> 6, q = tq % nsq, t = tq / nsq;
      const int mu = 16 * t + (L & 15), nu = 4 * q + (L >> 4);
      vr[e] = (mu < aP && nu < aQ) ? v_elem(Vp, P, Q, aP, aQ, mu, nu) : 0.0;
    }
    double* dr = Dr + d.dr_off[2 * p + o];
    const int nd = (int)(d.dr_off[2 * p + o + 1] - d.dr_off[2 * p + o]);
    for (int e = threadIdx.x; e < nd; e += 256) {
      const int L = e & 63, q = e >> 6;
      const int j = L & 15, l = (L >> 4) + 4 * q;   // the f64 MFMA A-operand row of lane L, step q
      dr[e] = (j < bP && l < bQ) ? Ds[(size_t)(d.bo[P] + j) * ns + d.bo[Q] + l] : 0.0;
    }
  }
}

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

constexpr int LDS_PITCH = H_COLS + 1;   // doubles per staged row (one pad column: no bank conflicts)
constexpr int H_DPITCH = 17;            // staged D_PQ blocks: [slot][16 rows][17]
constexpr int HQ_CHUNK = 64;            // Q-list entries whose metadata sits in LDS at once
constexpr int H_WAVES = 4;
constexpr int H_CPW = H_COLS / H_WAVES;

__device__ __forceinline__ int h_class(int ns, int nl) {
  if (ns <= 4 && nl <= 2) return 0;
  if (ns <= 10) return 1;
  return 2;
}

struct HUnits {            // unit table of the group (LDS)
  int P[GROUP_WAVES], mu0[GROUP_WAVES], slot[GROUP_WAVES], a[GROUP_WAVES], b[GROUP_WAVES], bo[GROUP_WAVES];
};

// The binary32 kernel stages the V_PQ and D_PQ blocks of the group in LDS
// once per Q; the binary64 kernel reads them per unit from their lane-ordered copies.
template <typename R> struct HStage { static constexpr bool vd = sizeof(R) == sizeof(float); };

// One Q of a V-stage tile, all H_CPW columns of this wavefront.  The staged T_Q
// rows are read without masks: rows past s_Q (or of lanes past n_b(Q)) hold
// finite values, and they meet zero V (nu >= n_a(Q)) or zero D (l >= n_b(Q))
// operands.  A column missing from N[Q] is staged as zeros.
// The binary64 kernel reads the V and D operands from their lane-ordered copies (d.Vr,
// d.Dr); NSP density matrices (collinear spin: two, the second's D operands in Dr1) share F,
// and each has its own D contraction and accumulators.  The binary32 kernel reads them from
// the blocks it staged in LDS (sV, sD).
template <int NS, int NL, int U, int NSP, typename R>
__device__ __forceinline__ void h_q(typename Mf<R>::acc (&Hc)[NSP][U][H_CPW], const R* sT, const R* sV,
                                    const R* sD, const HUnits& un, const int* roff, int nU, const int* qp, int Q,
                                    int aQ, int bQ, const int* lc_row, int ncols, int c0, int lr, int lk,
                                    const DevPlan& d, const double* Dr1) {
  typedef typename Mf<R>::acc A4;
  static_assert(NSP == 1 || !HStage<R>::vd, "the LDS-staged binary32 kernel takes one density matrix");
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
        const int aP = un.a[u], bP = un.b[u];
        const int muB = un.mu0[u] + lr;
        const bool muv = muB < aP;
        R vb[NS];
        R da[NSP][NLR];
        if constexpr (HStage<R>::vd) {
          const bool pqs = un.P[u] <= Q;
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            const int nu = 4 * q + lk;
            const bool ok = muv && nu < aQ;
            // the canonical block as stored: [mu][nu] if P <= Q, else [nu][mu]
            const int vi = pqs ? muB * aQ + nu : nu * aP + muB;
            const R x = sV[ok ? roff[sl] * aQ + vi : 0];
            vb[q] = ok ? x : (R)0;
          }
#pragma unroll
          for (int q = 0; q < NLR; ++q) {
            const int l = Mf<R>::row(lk, q);
            const bool ok = lr < bP && l < bQ;
            const R x = sD[ok ? (sl * 16 + lr) * H_DPITCH + l : 0];
            da[0][q] = ok ? x : (R)0;
          }
        } else {
          // the lane-ordered copies: one coalesced row per MFMA step (steps past the
          // blocks are zero)
          const int pp = qp[sl], orient = un.P[u] <= Q ? 0 : 1;
          const int nsq = (aQ + 3) >> 2, nlq = (bQ + 3) >> 2, L = lk * 16 + lr;
          const double* vrow = d.Vr + d.vr_off[2 * pp + orient] + (size_t)(un.mu0[u] >> 4) * nsq * 64 + L;
#pragma unroll
          for (int q = 0; q < NS; ++q) vb[q] = q < nsq ? (R)vrow[q * 64] : (R)0;
#pragma unroll
          for (int sp = 0; sp < NSP; ++sp) {
            const double* dr = (sp == 0 ? d.Dr : Dr1) + d.dr_off[2 * pp + orient] + L;
#pragma unroll
            for (int q = 0; q < NLR; ++q) da[sp][q] = q < nlq ? (R)dr[q * 64] : (R)0;
          }
        }
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

// Task lists of one k_H launch: tiles and their Q- and X-lists.
struct HLists {
  const GTile* tiles;
  const Slot4 *gq, *gx;
  int v_base, d_base;     // element offsets of the staged V and D blocks in LDS
  // second density matrix (collinear spin): its E and H' workspaces and its lane-ordered
  // D operands
  const double* E1;
  double* H1;
  const double* Dr1;
};

// mode: H_WRITE stores H' = (Q part + G part); H_ADD adds both parts to H';
// H_G_ADD adds the G part only.
enum { H_WRITE = 0, H_ADD = 1, H_G_ADD = 2 };

// NSP = 2: the two spin density matrices of a collinear-spin build in one pass (F = V T_Q is
// formed once); H'^0 goes to d.H, H'^1 to hl.H1.  Four wavefronts per SIMD for one density
// matrix (at most 128 VGPRs: measured faster than three with 168 since the V and D operands
// are coalesced rows), two for two (their accumulators double).
template <int U, typename R, int NSP>
__global__ __launch_bounds__(64 * H_WAVES) __attribute__((amdgpu_waves_per_eu(NSP == 1 ? 4 : 2))) void k_H(
    const double* __restrict__ V, const double* __restrict__ D, DevPlan d, HLists hl, int n_tiles,
    int n_padded, double gscale, int mode) {
  typedef typename Mf<R>::acc A4;
  extern __shared__ double sraw[];
  R* sT = reinterpret_cast<R*>(sraw);
  __shared__ HUnits un;
  __shared__ int qm_atom[HQ_CHUNK], qm_n[HQ_CHUNK], qm_a[HQ_CHUNK], qm_b[HQ_CHUNK], qm_bo[HQ_CHUNK];
  __shared__ int qm_lc[HQ_CHUNK][H_COLS], qm_p[HQ_CHUNK][GROUP_ATOMS];
  __shared__ int64_t qm_toff[HQ_CHUNK], qm_voff[HQ_CHUNK][GROUP_ATOMS];
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
  const int s = d.atom_sys[d.grp_first[g]];
  const int64_t ns = d.sys_n[s];
  const double* Ds = D + d.sys_d_off[s];
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
  // LDS: T_Q[:, tile columns] | V_PQ of the group's atoms, [nu][group aux row] | D_PQ blocks
  R* sV = sT + hl.v_base;
  R* sD = sV + hl.d_base;
  __shared__ int roff[GROUP_ATOMS + 1], sP_[GROUP_ATOMS], sa_[GROUP_ATOMS], sb_[GROUP_ATOMS], sbo_[GROUP_ATOMS];
  if (threadIdx.x == 0) {
    const int a0 = d.grp_first[g];
    const int nsl = d.grp_units[u0 + nU - 1].slot + 1;
    roff[0] = 0;
    for (int t = 0; t < GROUP_ATOMS; ++t) {
      const int P = a0 + t;
      const bool in = t < nsl;
      sP_[t] = in ? P : -1;
      sa_[t] = in ? d.na[P] : 0;
      sb_[t] = in ? d.nb[P] : 0;
      sbo_[t] = in ? d.bo[P] : 0;
      roff[t + 1] = roff[t] + sa_[t];
    }
  }
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
      qm_lc[ei][c] = (c < ncols) ? d.map1[d.map_off[Q] + gcol[c]] : -1;
      if (c == 0) {
        qm_atom[ei] = Q;
        qm_n[ei] = d.n_loc[Q];
        qm_a[ei] = d.na[Q];
        qm_b[ei] = d.nb[Q];
        qm_bo[ei] = d.bo[Q];
        qm_toff[ei] = d.t_off[Q];
        const int pp[3] = {qe.p0, qe.p1, qe.p2};
        for (int k = 0; k < GROUP_ATOMS; ++k) {
          qm_p[ei][k] = pp[k];
          qm_voff[ei][k] = pp[k] >= 0 ? d.v_off[pp[k]] : 0;
        }
      }
    }
    __syncthreads();
    for (int ei = 0; ei < nchunk; ++ei) {
      const int Q = qm_atom[ei], aQ = qm_a[ei], bQ = qm_b[ei], nQ = qm_n[ei], sQ = aQ * bQ;
      const int lcq = qm_lc[ei][tc];
      const double* TQ = d.T + qm_toff[ei] + (lcq >= 0 ? lcq : 0);
      for (int r = threadIdx.x / H_COLS; r < sQ; r += tstep)
        sT[r * LDS_PITCH + tc] = (R)(lcq >= 0 ? TQ[(size_t)r * nQ] : 0.0);
      // V_PQ and D_PQ of every group atom paired with Q (coalesced reads of the
      // canonical V block, transposed into [nu][row])
#pragma unroll
      for (int k = 0; k < GROUP_ATOMS; ++k) {
        if (HStage<R>::vd && qm_p[ei][k] >= 0) {
          const int P = sP_[k], aP = sa_[k], bP = sb_[k];
          // plain copies: the V block as stored, the D block row by row
          const double* Vp = V + qm_voff[ei][k];
          R* dv = sV + roff[k] * aQ;
          for (int i = threadIdx.x; i < aP * aQ; i += blockDim.x) dv[i] = (R)Vp[i];
          const double* DPQ = Ds + (size_t)sbo_[k] * ns + qm_bo[ei];
          for (int i = threadIdx.x; i < bP * 16; i += blockDim.x) {
            const int j = i >> 4, l = i & 15;
            if (l < bQ) sD[(k * 16 + j) * H_DPITCH + l] = (R)DPQ[(size_t)j * ns + l];
          }
          (void)P;
        }
      }
      __syncthreads();
      const int nsQ = (aQ + 3) >> 2, nlQ = (bQ + 3) >> 2;
      switch (h_class(nsQ, nlQ)) {
        case 0: h_q<4, 2, U, NSP, R>(Hc, sT, sV, sD, un, roff, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1); break;
        case 1: h_q<10, 4, U, NSP, R>(Hc, sT, sV, sD, un, roff, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1); break;
        default: h_q<16, 4, U, NSP, R>(Hc, sT, sV, sD, un, roff, nU, qm_p[ei], Q, aQ, bQ, qm_lc[ei], ncols, c0, lr, lk, d, hl.Dr1); break;
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
    const double* EXs[NSP];
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp) EXs[sp] = (sp == 0 ? d.E : hl.E1) + d.e_off[X];
    const int* m2X = d.map2 + d.map_off[X];
#pragma unroll
    for (int cc = 0; cc < H_CPW; ++cc) {
      const int c = c0 + cc;
      const int ic = (c < ncols) ? gcol[c] - boX : -1;
      if (ic >= 0 && ic < bX) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u < nU) {
            const int p = pp[un.slot[u]];
            if (p >= 0) {
              const int P = un.P[u], aP = un.a[u], bP = un.b[u];
              const int muB = un.mu0[u] + lr;
              const bool muv = muB < aP;
              const int colx = lr < bP ? m2X[un.bo[u] + lr] : 0;
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
      const int* m2P = d.map2 + d.map_off[P];
#pragma unroll
      for (int sp = 0; sp < NSP; ++sp) {
        double* HP = (sp == 0 ? d.H : hl.H1) + d.e_off[P];
#pragma unroll
        for (int cc = 0; cc < H_CPW; ++cc) {
          const int c = c0 + cc;
          const int col = (c < ncols) ? m2P[gcol[c]] : -1;
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

// ---------------------------------------------------------------------------
// stage 3: T2[P, Q] = sum_{mu, l} E_P[(mu, i), l] F[mu, k, l],
//          F[mu, k, l] = sum_nu V_PQ[mu, nu] T_Q[(nu, k), l], l over N[Q].
// One workgroup of four wavefronts per canonical pair.  Columns l are
// processed in chunks of T2_COLS: the chunk of T_Q and the matching columns
// of E_P are staged in LDS with coalesced loads; each wavefront takes two
// columns.  Per column, the stage-one accumulator element v is directly the
// stage-two B operand.  The four partial sums are added in a fixed order.

constexpr int T2_COLS = 8;               // column chunk of the backward pair kernel
constexpr int T2_PITCH = T2_COLS + 1;

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
  const bool flip = items[item_base + w] & 1;
  const int P = flip ? d.pair_b[p] : d.pair_a[p], Q = flip ? d.pair_a[p] : d.pair_b[p];
  const int aP = d.na[P], bP = d.nb[P], aQ = d.na[Q], bQ = d.nb[Q];
  const int sP = aP * bP, sQ = aQ * bQ;
  const int nQ = d.n_loc[Q], mP = d.m_loc[P];
  const int s = d.atom_sys[P];
  const int64_t ns = d.sys_n[s];
  const double* Vp = V + d.v_off[p];
  const int* cg = d.col1g + d.col1g_off[Q];
  const int* m2P = d.map2 + d.map_off[P];
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
    const int ce = cv ? m2P[cg[l]] : 0;
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
        Ks[(size_t)(bPo + i) * ns + bQo + k] = out[v];
        if (P != Q) Ks[(size_t)(bQo + k) * ns + bPo + i] = out[v];
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
  const double* B = d.H + d.e_off[P];   // B(k, n) = H'_P[k * N + n]
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
// fixed order.  X[i, l] is gathered with l fastest across threads and
// X[l, i] with i fastest (both coalesced), the two halves are combined in
// LDS, and every element is written together with its mirror.

__global__ __launch_bounds__(256) void k_symreduce(double* __restrict__ K, DevPlan d, int n_items,
                                                   int n_padded) {
  __shared__ int cmap[4][32];      // c1(I rows), c2(I rows), c1(L cols), c2(L cols)
  __shared__ double xa[32][33], xb[32][33];
  const int w = xcd_task(n_padded);
  if (w >= n_items) return;
  const FItem it = d.f_items[w];
  const int s = it.sys;
  const int64_t ns = d.sys_n[s];
  const int t = threadIdx.x;
  const int ta = t & 31, tb = t >> 5;   // element (tb + 8 r, ta)
  double acc_a[4] = {0, 0, 0, 0}, acc_b[4] = {0, 0, 0, 0};
  for (int pi = it.pbeg; pi < it.pend; ++pi) {
    const int P = d.f_plist[pi];
    const int nP_ = d.m_loc[P];
    const double* Y = d.Y + d.y_off[P];
    __syncthreads();
    if (t < 128) {
      const int which = t >> 5, x = t & 31;
      const int g = ((which < 2) ? it.gI0 : it.gL0) + x;
      const int* mp = ((which & 1) ? d.map2 : d.map1) + d.map_off[P];
      cmap[which][x] = g < ns ? mp[g] : -1;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = tb + 8 * r;
      // X[i = I0 + ii, l = L0 + ta] = Y_P[c1(i), c2(l)]
      const int c1 = cmap[0][ii], c2 = cmap[3][ta];
      if (c1 >= 0 && c2 >= 0) acc_a[r] += Y[(size_t)c1 * nP_ + c2];
      // X[l = L0 + ii, i = I0 + ta] = Y_P[c1(l), c2(i)], stored at (ta, ii)
      const int d1 = cmap[2][ii], d2 = cmap[1][ta];
      if (d1 >= 0 && d2 >= 0) acc_b[r] += Y[(size_t)d1 * nP_ + d2];
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

// ---------------------------------------------------------------------------
// energy: per-chunk tree reduction, then per-system ordered sum.  n_spin density
// matrices (and their K) are stored spin_stride apart; the chunk sums run over all.

__global__ __launch_bounds__(256) void k_energy_part(const double* K, const double* D, DevPlan d,
                                                     int n_chunks, int n_spin, int64_t spin_stride) {
  const int c = blockIdx.x;
  if (c >= n_chunks) return;
  const int s = d.en_sys[c];
  const int64_t base = d.sys_d_off[s];
  __shared__ double part[256];
  double acc = 0.0;
  for (int sp = 0; sp < n_spin; ++sp) {
    const double* Ks = K + sp * spin_stride;
    const double* Dsp = D + sp * spin_stride;
    for (int e = d.en_beg[c] + threadIdx.x; e < d.en_end[c]; e += 256) acc += Ks[base + e] * Dsp[base + e];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.epart[c] = part[0];
}

// scale: -1/4 for one (spin-summed) density matrix, -1/2 for the two spin density matrices
__global__ void k_energy_sum(double* Ex, DevPlan d, int n_chunks, double scale) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= d.n_sys) return;
  double acc = 0.0;
  for (int c = 0; c < n_chunks; ++c)
    if (d.en_sys[c] == s) acc += d.epart[c];
  Ex[s] = scale * acc;
}

__global__ void k_zero(double* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// ---------------------------------------------------------------------------
// backward.  dE/dC^mu = -1/2 sum_nu V_{mu nu} D C^nu D.  With the row-owned
// M^mu, the gradient per row-owned entry is -sum_nu V_{mu nu} (D C^nu D) on
// rows of P; writing C^nu = M^nu + M^nu^T gives the rows-of-P blocks
//   G_P = (H_P + Gt_P) D,   H_P = rows of P of D F^mu,  F^mu = sum_nu V M^nu,
// where Gt_P is exactly the G term of the forward V stage taken once.  The
// un-repack maps G_P back to the canonical C layout (the on-site halving
// of the repack appears as a factor 1/2).

__global__ __launch_bounds__(256) void k_unrepack(const double* __restrict__ GD, double* __restrict__ dC,
                                                  DevPlan d, double scale) {
  const int k = blockIdx.x;
  const int P = d.nbr_owner[k], J = d.nbr_atom[k], p = d.nbr_pair[k];
  const int aP = d.na[P], bP = d.nb[P], bJ = d.nb[J], aJ = d.na[J];
  const int nP = d.n_loc[P], lc = d.nbr_lcol[k];
  const int sP = aP * bP;
  double* Cp = dC + d.c_off[p];
  const double* GP = GD + d.t_off[P];
  const int nel = sP * bJ;
  for (int e = threadIdx.x; e < nel; e += 256) {
    const int r = e / bJ, j = e - r * bJ;
    const int mu = r / bP, i = r - mu * bP;
    const double v = scale * GP[(size_t)r * nP + lc + j];
    if (P < J)
      Cp[(size_t)(mu * bP + i) * bJ + j] = v;
    else if (P > J)
      Cp[(size_t)((aJ + mu) * bJ + j) * bP + i] = v;
    else
      Cp[(size_t)(mu * bP + i) * bP + j] = 0.5 * v;
  }
}

// <X, Y> over every canonical pair block (offsets off[p]..off[p+1]),
// fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_block_dot(const double* __restrict__ X, const double* __restrict__ Y,
                                                   const int64_t* __restrict__ off, double* __restrict__ out) {
  const int p = blockIdx.x;
  __shared__ double part[256];
  double acc = 0.0;
  for (int64_t e = off[p] + threadIdx.x; e < off[p + 1]; e += 256) acc += X[e] * Y[e];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = part[0];
}

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
constexpr int DV_WAVES = 8, DV_COLS = 8, DV_PITCH = DV_COLS + 1, DV_RSTEP = 64 * DV_WAVES / DV_COLS;

template <int NTP, int NTQ, int NLQ, int NIP>
__global__ __launch_bounds__(64 * DV_WAVES) void k_dV(const double* __restrict__ V, const double* __restrict__ D,
                                                     double* __restrict__ dV, DevPlan d, const int* __restrict__ items,
                                                     double gE, int n_items, int n_padded, int item_base) {
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
  const int* cg = d.col1g + d.col1g_off[Q];
  const int* m2P = d.map2 + d.map_off[P];
  const int* m2Q = d.map2 + d.map_off[Q];
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
    const int ce = cv ? m2P[cg[l]] : 0;
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
      const int cP = kv ? m2P[d.bo[Q] + l] : 0, cQ = kv ? m2Q[d.bo[P] + i] : 0;
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
  const double f = -0.5 * gE * (P != Q ? 2.0 : 1.0);
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

// forces: -dE/dR_A = -sum_{J in N[A], J != A} [sC (-1/c_decay) d/r + sV (-2/v_2s2) d],
// d = R_A - R_J; sC, sV are the per-pair <gradient, block> sums.
__global__ void k_forces(const double* __restrict__ pos, const double* __restrict__ sC,
                         const double* __restrict__ sV, double* __restrict__ F, DevPlan d,
                         double c_decay, double v_2s2) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= d.n_atoms) return;
  double f0 = 0, f1 = 0, f2 = 0;
  for (int k = d.nbr_ptr[A]; k < d.nbr_ptr[A + 1]; ++k) {
    const int J = d.nbr_atom[k];
    if (J == A) continue;
    const int p = d.nbr_pair[k];
    const double dx = pos[3 * A] - pos[3 * J], dy = pos[3 * A + 1] - pos[3 * J + 1], dz = pos[3 * A + 2] - pos[3 * J + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double gc = sC[p] * (-1.0 / c_decay) / r, gv = sV[p] * (-2.0 / v_2s2);
    f0 -= (gc + gv) * dx;
    f1 -= (gc + gv) * dy;
    f2 -= (gc + gv) * dz;
  }
  F[3 * A] = f0;
  F[3 * A + 1] = f1;
  F[3 * A + 2] = f2;
}

__global__ void k_scaled_copy(double* __restrict__ y, const double* __restrict__ x, int64_t n, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ void k_scale(double* x, int64_t n, double a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= a;
}

// ---------------------------------------------------------------------------
// plan creation

static int device_neighbors(exx_plan_s* pl) {
  HostPlan& hp = pl->hp;
  double* dpos = nullptr;
  int *dsys = nullptr, *doff = nullptr, *dcnt = nullptr, *dptr = nullptr, *dout = nullptr;
  auto cleanup = [&]() {
    hipFree(dpos); hipFree(dsys); hipFree(doff); hipFree(dcnt); hipFree(dptr); hipFree(dout);
  };
  const int NA = hp.n_atoms;
  hipError_t e = hipSuccess;
#define NB_TRY(x) do { e = (x); if (e != hipSuccess) { cleanup(); return fail(EXX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e)); } } while (0)
  NB_TRY(hipMalloc((void**)&dpos, sizeof(double) * 3 * NA));
  NB_TRY(hipMalloc((void**)&dsys, sizeof(int) * NA));
  NB_TRY(hipMalloc((void**)&doff, sizeof(int) * (hp.n_sys + 1)));
  NB_TRY(hipMalloc((void**)&dcnt, sizeof(int) * NA));
  NB_TRY(hipMemcpy(dpos, hp.pos.data(), sizeof(double) * 3 * NA, hipMemcpyHostToDevice));
  NB_TRY(hipMemcpy(dsys, hp.atom_sys.data(), sizeof(int) * NA, hipMemcpyHostToDevice));
  NB_TRY(hipMemcpy(doff, hp.sys_atom_off.data(), sizeof(int) * (hp.n_sys + 1), hipMemcpyHostToDevice));
  const double rc2 = hp.r_cut * hp.r_cut;
  hipLaunchKernelGGL(k_nbr_count, dim3(NA), dim3(256), 0, 0, dpos, dsys, doff, rc2, dcnt);
  NB_TRY(hipGetLastError());
  std::vector<int> cnt(NA);
  NB_TRY(hipMemcpy(cnt.data(), dcnt, sizeof(int) * NA, hipMemcpyDeviceToHost));
  hp.nbr_ptr.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) hp.nbr_ptr[a + 1] = hp.nbr_ptr[a] + cnt[a];
  NB_TRY(hipMalloc((void**)&dptr, sizeof(int) * (NA + 1)));
  NB_TRY(hipMalloc((void**)&dout, sizeof(int) * std::max(1, hp.nbr_ptr[NA])));
  NB_TRY(hipMemcpy(dptr, hp.nbr_ptr.data(), sizeof(int) * (NA + 1), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_nbr_fill, dim3(NA), dim3(256), 0, 0, dpos, dsys, doff, rc2, dptr, dout);
  NB_TRY(hipGetLastError());
  hp.nbr_atom.resize(hp.nbr_ptr[NA]);
  NB_TRY(hipMemcpy(hp.nbr_atom.data(), dout, sizeof(int) * hp.nbr_ptr[NA], hipMemcpyDeviceToHost));
#undef NB_TRY
  cleanup();
  return 0;
}

static int upload_plan(exx_plan_s* pl) {
  HostPlan& hp = pl->hp;
  DevPlan& d = pl->d;
  d.n_atoms = hp.n_atoms;
  d.n_sys = hp.n_sys;
  int rc = 0;
#define UP(field) if ((rc = upload(pl, d.field, hp.field)) != 0) return rc
  UP(nb); UP(na); UP(atom_sys); UP(bo); UP(sys_n); UP(sys_d_off);
  UP(nbr_ptr); UP(nbr_atom); UP(nbr_pair); UP(nbr_lcol); UP(nbr_owner);
  UP(pair_a); UP(pair_b); UP(c_off); UP(v_off); UP(n_loc); UP(m_loc);
  UP(map_off); UP(col1g_off); UP(col2g_off); UP(map1); UP(map2); UP(col1g); UP(col2g);
  UP(t_off); UP(e_off); UP(e_items); UP(ct_run_ptr); UP(ct_klen); UP(runs);
  UP(gd_items); UP(gd_run_ptr); UP(gd_klen); UP(gd_runs); UP(pos);
  UP(grp_first); UP(grp_unit_ptr); UP(grp_col_ptr); UP(grp_cols); UP(grp_units);
  UP(g_tiles); UP(gq); UP(gx); UP(t2_items); UP(dv_items);
  UP(f_items); UP(f_plist); UP(en_sys); UP(en_beg); UP(en_end); UP(y_tiles); UP(y_off);
#undef UP
  if ((rc = alloc_buf(pl, d.T, hp.t_total))) return rc;
  if ((rc = alloc_buf(pl, d.E, hp.e_total))) return rc;
  if ((rc = alloc_buf(pl, d.H, hp.e_total))) return rc;
  if ((rc = alloc_buf(pl, d.Y, hp.y_total))) return rc;
  if ((rc = alloc_buf(pl, d.GD, hp.t_total))) return rc;
  if ((rc = alloc_buf(pl, d.sC, (int64_t)hp.pair_a.size()))) return rc;
  if ((rc = alloc_buf(pl, d.sV, (int64_t)hp.pair_a.size()))) return rc;
  if ((rc = alloc_buf(pl, d.epart, (int64_t)hp.en_sys.size()))) return rc;
  const size_t np = hp.pair_a.size();
  std::vector<int64_t> vro(2 * np + 1, 0), dro(2 * np + 1, 0);
  for (size_t p = 0; p < np; ++p) {
    const int A = hp.pair_a[p], B = hp.pair_b[p];
    const int64_t v0 = (int64_t)((hp.na[A] + 15) / 16) * ((hp.na[B] + 3) / 4) * 64;
    const int64_t v1 = A == B ? 0 : (int64_t)((hp.na[B] + 15) / 16) * ((hp.na[A] + 3) / 4) * 64;
    const int64_t d0 = (int64_t)((hp.nb[B] + 3) / 4) * 64, d1 = A == B ? 0 : (int64_t)((hp.nb[A] + 3) / 4) * 64;
    vro[2 * p + 1] = vro[2 * p] + v0;
    vro[2 * p + 2] = vro[2 * p + 1] + v1;
    dro[2 * p + 1] = dro[2 * p] + d0;
    dro[2 * p + 2] = dro[2 * p + 1] + d1;
  }
  if ((rc = upload(pl, d.vr_off, vro))) return rc;
  if ((rc = upload(pl, d.dr_off, dro))) return rc;
  if ((rc = alloc_buf(pl, d.Vr, std::max<int64_t>(1, vro.back())))) return rc;
  if ((rc = alloc_buf(pl, d.Dr, std::max<int64_t>(1, dro.back())))) return rc;
  pl->dr_total = dro.back();
  return 0;
}

static void release(exx_plan_s* pl) {
  if (pl->graph_exec) hipGraphExecDestroy(pl->graph_exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  pl->graph_exec = nullptr;
  pl->graph = nullptr;
  for (void* p : pl->allocs) hipFree(p);
  pl->allocs.clear();
  for (void* p : pl->mixed_allocs) hipFree(p);
  pl->mixed_allocs.clear();
  for (hipEvent_t e : pl->events) hipEventDestroy(e);
  pl->events.clear();
}

// Record boundary `i` of the current profiled build (no-op when off or full).
static void stage_mark(exx_plan_s* pl, int i, hipStream_t st) {
  if (!pl->profiling || pl->n_recorded >= MAX_PROFILED) return;
  hipEventRecord(pl->events[(size_t)pl->n_recorded * N_STAGE_EV + i], st);
  if (i == N_STAGE_EV - 1) ++pl->n_recorded;
}

extern "C" {

const char* exx_last_error(void) { return g_err.c_str(); }

int exx_plan_create(const exx_system* sys, uint32_t flags, exx_plan* out) {
  g_err.clear();
  if (!out) return fail(EXX_EINVAL, "exx_plan_create: out is NULL");
  *out = nullptr;
  if (!sys) return fail(EXX_EINVAL, "exx_plan_create: sys is NULL");
  exx_plan_s* pl = new (std::nothrow) exx_plan_s();
  if (!pl) return fail(EXX_ENOMEM, "exx_plan_create: host allocation");
  pl->host_only = (flags & EXX_PLAN_HOST_ONLY) != 0;
  std::string err;
  int rc = describe_system(sys->n_atoms, sys->n_species, sys->species, sys->positions, sys->n_basis,
                           sys->n_aux, sys->r_cut, sys->n_systems, sys->sys_atom_off, pl->hp, err);
  if (rc != 0) {
    delete pl;
    return fail(rc, err);
  }
  if (pl->host_only) {
    host_neighbors(pl->hp);
  } else {
    if (hipGetDevice(&pl->device) != hipSuccess) {
      delete pl;
      return fail(EXX_EDEVICE, "exx_plan_create: no HIP device");
    }
    if ((rc = device_neighbors(pl)) != 0) {
      delete pl;
      return rc;
    }
  }
  try {
    rc = derive_lists(pl->hp, err);
  } catch (const std::bad_alloc&) {
    delete pl;
    return fail(EXX_ENOMEM, "exx_plan_create: host allocation in list building");
  }
  if (rc != 0) {
    delete pl;
    return fail(EXX_EDEVICE, err);
  }
  {
    int amax = 1;
    for (int a = 0; a < pl->hp.n_atoms; ++a) amax = std::max(amax, pl->hp.na[a]);
    pl->t2_nt = (amax + 15) / 16;
    int smax = 1;
    for (int a = 0; a < pl->hp.n_atoms; ++a) smax = std::max(smax, pl->hp.na[a] * pl->hp.nb[a]);
    // k_H: T_Q tile | V blocks [nu][aux rows of the group] | D blocks
    int vr_max = 1;
    const HostPlan& hq = pl->hp;
    for (size_t g = 0; g + 1 < hq.grp_unit_ptr.size(); ++g) {
      const int nsl = hq.grp_units[hq.grp_unit_ptr[g + 1] - 1].slot + 1;
      int vr = 0;
      for (int t = 0; t < nsl; ++t) vr += hq.na[hq.grp_first[g] + t];
      vr_max = std::max(vr_max, vr);
    }
    // rows of the staged T_Q read by the chains: up to 4 NS * n_b(Q) + 16 (NS of Q's shape class)
    int h_rows = smax;
    for (int a = 0; a < pl->hp.n_atoms; ++a) {
      const int nsq = (pl->hp.na[a] + 3) / 4, nlq = (pl->hp.nb[a] + 3) / 4;
      const int NS = (nsq <= 4 && nlq <= 2) ? 4 : (nsq <= 10 ? 10 : 16);
      h_rows = std::max(h_rows, 4 * NS * pl->hp.nb[a] + 16);
    }
    pl->h_vbase = h_rows * LDS_PITCH;
    pl->h_dbase = amax * vr_max;
    const size_t h_elems = (size_t)pl->h_vbase + pl->h_dbase + GROUP_ATOMS * 16 * H_DPITCH;
    pl->h_lds = (size_t)pl->h_vbase * sizeof(double);   // the binary64 kernel stages T_Q only
    pl->t2_lds = std::max((size_t)2 * smax * T2_PITCH, (size_t)16 * 64) * sizeof(double);
    pl->h_smax_t2 = smax;
    pl->h_lds32 = h_elems * sizeof(float);
    pl->t2_lds32 = std::max((size_t)2 * smax * T2_PITCH * sizeof(float), (size_t)16 * 64 * sizeof(double));
  }
  if (!pl->host_only) {
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device) != hipSuccess) {
      delete pl;
      return fail(EXX_EDEVICE, "exx_plan_create: cannot query the LDS size");
    }
    pl->lds_max = lds_max;
    if (pl->t2_lds > (size_t)lds_max || pl->h_lds + 8192 > (size_t)lds_max) {   // static LDS of k_H < 8 KB
      delete pl;
      return fail(EXX_EUNSUPPORTED, "exx_plan_create: the largest n_aux * n_basis needs more LDS than a workgroup has");
    }
    if ((rc = upload_plan(pl)) != 0) {
      release(pl);
      delete pl;
      return rc;
    }
  }
  *out = pl;
  return EXX_OK;
}

int exx_plan_destroy(exx_plan plan) {
  if (!plan) return fail(EXX_EINVAL, "exx_plan_destroy: NULL plan");
  release(plan);
  delete plan;
  return EXX_OK;
}

int exx_plan_info(exx_plan plan, exx_info* info) {
  if (!plan || !info) return fail(EXX_EINVAL, "exx_plan_info: NULL argument");
  const HostPlan& hp = plan->hp;
  info->n_atoms = hp.n_atoms;
  info->n_systems = hp.n_sys;
  info->n_pairs = (int64_t)hp.pair_a.size();
  info->c_size = hp.c_off.empty() ? 0 : hp.c_off.back();
  info->v_size = hp.v_off.empty() ? 0 : hp.v_off.back();
  info->d_size = hp.d_size;
  info->n_basis_max = hp.n_basis_max;
  info->workspace_bytes = plan->dev_bytes + plan->mixed_bytes;
  info->flops_fp64 = hp.flops[0] + hp.flops[1] + hp.flops[2] + hp.flops[3] + hp.flops[4];
  return EXX_OK;
}

int exx_plan_pairs(exx_plan plan, int32_t* pair_a, int32_t* pair_b, int64_t* c_off, int64_t* v_off) {
  if (!plan) return fail(EXX_EINVAL, "exx_plan_pairs: NULL plan");
  const HostPlan& hp = plan->hp;
  const size_t n = hp.pair_a.size();
  if (pair_a) std::memcpy(pair_a, hp.pair_a.data(), n * sizeof(int32_t));
  if (pair_b) std::memcpy(pair_b, hp.pair_b.data(), n * sizeof(int32_t));
  if (c_off) std::memcpy(c_off, hp.c_off.data(), (n + 1) * sizeof(int64_t));
  if (v_off) std::memcpy(v_off, hp.v_off.data(), (n + 1) * sizeof(int64_t));
  return EXX_OK;
}

int exx_plan_neighbors(exx_plan plan, int32_t* nbr_ptr, int32_t* nbr_atom) {
  if (!plan || !nbr_ptr) return fail(EXX_EINVAL, "exx_plan_neighbors: NULL argument");
  const HostPlan& hp = plan->hp;
  std::memcpy(nbr_ptr, hp.nbr_ptr.data(), hp.nbr_ptr.size() * sizeof(int32_t));
  if (nbr_atom) std::memcpy(nbr_atom, hp.nbr_atom.data(), hp.nbr_atom.size() * sizeof(int32_t));
  return EXX_OK;
}

int64_t exx_plan_flops(exx_plan plan, int stage) {
  if (!plan) return -1;
  const HostPlan& hp = plan->hp;
  if (stage < 0) return hp.flops[0] + hp.flops[1] + hp.flops[2] + hp.flops[3] + hp.flops[4];
  if (stage >= 10 && stage <= 14) return hp.issued[stage - 10];
  if (stage >= 20 && stage <= 44 && stage % 10 <= 4) {
    if (!plan->hp.mixed_ready) derive_mixed_lists(plan->hp);
    if (stage < 30) return hp.flops32[stage - 20];
    if (stage < 40) return hp.issued32[stage - 30];
    return hp.issued64m[stage - 40];
  }
  if (stage > 4) return -1;
  return hp.flops[stage];
}

static int launch_energy(exx_plan plan, const double* K, const double* D, double* Ex, hipStream_t st,
                         int n_spin = 1) {
  const int nch = (int)plan->hp.en_sys.size();
  hipLaunchKernelGGL(k_energy_part, dim3(nch), dim3(256), 0, st, K, D, plan->d, nch, n_spin, plan->hp.d_size);
  hipLaunchKernelGGL(k_energy_sum, dim3((plan->hp.n_sys + 63) / 64), dim3(64), 0, st, Ex, plan->d, nch,
                     n_spin == 1 ? -0.25 : -0.5);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exx_plan_set_profiling(exx_plan plan, int enable) {
  if (!plan) return fail(EXX_EINVAL, "exx_plan_set_profiling: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_plan_set_profiling: host-only plan");
  if (enable && plan->events.empty()) {
    plan->events.resize((size_t)MAX_PROFILED * N_STAGE_EV);
    for (auto& e : plan->events) HIP_TRY(hipEventCreate(&e));
  }
  plan->profiling = enable != 0;
  plan->n_recorded = 0;
  return EXX_OK;
}

int exx_plan_stage_times(exx_plan plan, double* ms, int64_t* n_builds) {
  if (!plan || !ms || !n_builds) return fail(EXX_EINVAL, "exx_plan_stage_times: NULL argument");
  for (int i = 0; i < EXX_N_STAGES; ++i) ms[i] = 0.0;
  *n_builds = plan->n_recorded;
  for (int b = 0; b < plan->n_recorded; ++b) {
    hipEvent_t* ev = &plan->events[(size_t)b * N_STAGE_EV];
    HIP_TRY(hipEventSynchronize(ev[N_STAGE_EV - 1]));
    for (int i = 0; i < EXX_N_STAGES; ++i) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[i] += t;
    }
  }
  plan->n_recorded = 0;
  return EXX_OK;
}

static RowD rowd_E(exx_plan plan) {
  DevPlan& d = plan->d;
  return RowD{d.T, d.t_off, d.n_loc, d.E, d.e_off, d.m_loc, d.col2g, d.col2g_off,
              d.e_items, d.ct_run_ptr, d.ct_klen, d.runs};
}

static RowD rowd_GD(exx_plan plan) {
  DevPlan& d = plan->d;
  return RowD{d.H, d.e_off, d.m_loc, d.GD, d.t_off, d.n_loc, d.col1g, d.col1g_off,
              d.gd_items, d.gd_run_ptr, d.gd_klen, d.gd_runs};
}

static void launch_rowD(exx_plan plan, const double* D, const RowD& r, int n, hipStream_t st) {
  if (n <= 0) return;
  const int nwgp = (n + 7) / 8 * 8;
  if (plan->tune[TUNE_E] == 1)
    hipLaunchKernelGGL((k_rowD<32, 1>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_rowD<16, 1>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, nullptr, nullptr);
}

// the two products of a collinear-spin build: r.O = A D, O1 = A D1
static void launch_rowD_spin(exx_plan plan, const double* D, const double* D1, double* O1, const RowD& r, int n,
                             hipStream_t st) {
  if (n <= 0) return;
  const int nwgp = (n + 7) / 8 * 8;
  if (plan->tune[TUNE_E] == 1)
    hipLaunchKernelGGL((k_rowD<32, 2>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, D1, O1);
  else
    hipLaunchKernelGGL((k_rowD<16, 2>), dim3(nwgp), dim3(256), 0, st, D, r, plan->d, n, nwgp, D1, O1);
}

// repack C into T_P, then E_P = T_P D (stage mark 1 in between)
static void launch_repack_E(exx_plan plan, const double* C, const double* D, hipStream_t st, bool mark) {
  const HostPlan& hp = plan->hp;
  hipLaunchKernelGGL(k_repack, dim3(hp.nbr_ptr[hp.n_atoms]), dim3(256), 0, st, C, plan->d);
  if (mark) stage_mark(plan, 1, st);
  launch_rowD(plan, D, rowd_E(plan), (int)hp.e_items.size(), st);
}

extern "C++" {
template <typename R, int NSP = 1>
static void launch_H_lists(exx_plan plan, const double* V, const double* D, const HLists& hl, int n, double gscale,
                           int mode, hipStream_t st) {
  if (n <= 0) return;
  const HostPlan& hp = plan->hp;
  const int np_ = (n + 7) / 8 * 8;
  const size_t lds = mode == H_G_ADD ? 0 : (sizeof(R) == sizeof(double) ? plan->h_lds : plan->h_lds32);
  const dim3 grid(np_), blk(64 * H_WAVES);
  if (hp.h_waves <= 2)
    hipLaunchKernelGGL((k_H<2, R, NSP>), grid, blk, lds, st, V, D, plan->d, hl, n, np_, gscale, mode);
  else if (hp.h_waves <= 5)
    hipLaunchKernelGGL((k_H<5, R, NSP>), grid, blk, lds, st, V, D, plan->d, hl, n, np_, gscale, mode);
  else
    hipLaunchKernelGGL((k_H<8, R, NSP>), grid, blk, lds, st, V, D, plan->d, hl, n, np_, gscale, mode);
}
}  // extern "C++"

// V stage over the full lists in binary64
// the lane-ordered V and D operands of the V stage (DevPlan::Vr, Dr) for these V and D
static void launch_vd_operands(exx_plan plan, const double* V, const double* D, hipStream_t st) {
  const unsigned np = (unsigned)plan->hp.pair_a.size();
  if (np) hipLaunchKernelGGL(k_vdrepack, dim3(np), dim3(256), 0, st, V, D, plan->d.Dr, plan->d);
}

static void launch_H(exx_plan plan, const double* V, const double* D, double gscale, int mode, hipStream_t st) {
  const DevPlan& d = plan->d;
  launch_vd_operands(plan, V, D, st);
  launch_H_lists<double>(plan, V, D, HLists{d.g_tiles, d.gq, d.gx, plan->h_vbase, plan->h_dbase},
                         (int)plan->hp.g_tiles.size(), gscale, mode, st);
}

// V stage of the mixed build: near pairs stored in binary64, far pairs added in binary32
static void stage_mark(exx_plan_s* pl, int i, hipStream_t st);
static void launch_H_mixed(exx_plan plan, const double* V, const double* D, hipStream_t st) {
  const DevPlan& d = plan->d;
  const HostPlan& hp = plan->hp;
  launch_vd_operands(plan, V, D, st);
  launch_H_lists<double>(plan, V, D, HLists{d.hm_tiles_near, d.hm_q_near, d.hm_x_near, plan->h_vbase, plan->h_dbase},
                         (int)hp.hm_tiles_near.size(), 2.0, H_WRITE, st);
  stage_mark(plan, 3, st);
  launch_H_lists<float>(plan, V, D, HLists{d.hm_tiles_far, d.hm_q_far, d.hm_x_far, plan->h_vbase, plan->h_dbase},
                        (int)hp.hm_tiles_far.size(), 2.0, H_ADD, st);
}

extern "C++" {
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

template <typename R, int NSP = 1>
static void launch_T2_class(exx_plan plan, const T2Class& c, const double* V, double* K, const int* items,
                            hipStream_t st) {
  const int n = c.end - c.beg;
  if (n <= 0) return;
  switch (plan->tune[TUNE_T2]) {
    case 0: launch_T2_cols<R, 4, 4, NSP>(plan, c, V, K, items, n, st); break;
    case 1: launch_T2_cols<R, 8, 4, NSP>(plan, c, V, K, items, n, st); break;
    default: launch_T2_cols<R, 8, 8, NSP>(plan, c, V, K, items, n, st); break;
  }
}
}  // extern "C++"

// one launch per shape class (aux tiles of P, nu steps of Q) and precision
// (mixed: the classes of one precision only)
// spin: both spin density matrices in one pass (binary64 lists; K holds K^0 then K^1)
static void launch_T2_spin(exx_plan plan, const double* V, double* K, hipStream_t st) {
  for (const T2Class& c : plan->hp.t2_classes) launch_T2_class<double, 2>(plan, c, V, K, plan->d.t2_items, st);
}

static void launch_T2(exx_plan plan, const double* V, double* K, hipStream_t st, bool mixed = false, int prec = 0) {
  const HostPlan& hp = plan->hp;
  const DevPlan& d = plan->d;
  for (const T2Class& c : mixed ? hp.t2m_classes : hp.t2_classes) {
    if (mixed && c.prec != prec) continue;
    if (c.prec) launch_T2_class<float>(plan, c, V, K, d.t2m_items, st);
    else launch_T2_class<double>(plan, c, V, K, mixed ? d.t2m_items : d.t2_items, st);
  }
}

// device copies of the near / far lists for the current split distance
static int prepare_mixed(exx_plan pl) {
  if (pl->mixed_uploaded) return EXX_OK;
  HostPlan& hp = pl->hp;
  if (!hp.mixed_ready) derive_mixed_lists(hp);
  for (void* p : pl->mixed_allocs) hipFree(p);
  pl->mixed_allocs.clear();
  pl->mixed_bytes = 0;
  DevPlan& d = pl->d;
  int rc = 0;
#define UPM(field) if ((rc = upload(pl, d.field, hp.field, true)) != 0) return rc
  UPM(hm_tiles_near); UPM(hm_tiles_far); UPM(hm_q_near); UPM(hm_x_near); UPM(hm_q_far); UPM(hm_x_far);
  UPM(t2m_items);
#undef UPM
  pl->mixed_uploaded = true;
  return EXX_OK;
}

static void launch_final(exx_plan plan, double* K, hipStream_t st) {
  const HostPlan& hp = plan->hp;
  const int nY = (int)hp.y_tiles.size(), nYp = (nY + 7) / 8 * 8;
  if (plan->tune[TUNE_Y] == 1) hipLaunchKernelGGL(k_Y<32>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
  else hipLaunchKernelGGL(k_Y<16>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
  const int nF = (int)hp.f_items.size(), nFp = (nF + 7) / 8 * 8;
  hipLaunchKernelGGL(k_symreduce, dim3(nFp), dim3(256), 0, st, K, plan->d, nF, nFp);
}

extern "C++" {
template <int NTP, int NTQ>
static void launch_dV_t(exx_plan plan, const DVClass& c, const double* V, const double* D, double* dV, double gE,
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
}  // extern "C++"

static void launch_dV(exx_plan plan, const double* V, const double* D, double* dV, double gE, hipStream_t st) {
  for (const DVClass& c : plan->hp.dv_classes) {
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

int build_K(exx_plan plan, const double* C, const double* V, const double* D, int precision,
            double* K, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "build_K: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "build_K: host-only plan");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "build_K: NULL array");
  if (precision != EXX_PREC_FP64 && precision != EXX_PREC_MIXED)
    return fail(EXX_EINVAL, "build_K: unknown precision");
  const bool mixed = precision == EXX_PREC_MIXED;
  if (mixed) {
    const int rcm = prepare_mixed(plan);
    if (rcm != EXX_OK) return rcm;
  }
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, hp.d_size);
  launch_repack_E(plan, C, D, st, true);
  stage_mark(plan, 2, st);
  if (mixed) {
    launch_H_mixed(plan, V, D, st);   // marks boundary 3 between its binary64 and binary32 parts
  } else {
    launch_H(plan, V, D, 2.0, H_WRITE, st);
    stage_mark(plan, 3, st);
  }
  stage_mark(plan, 4, st);
  launch_T2(plan, V, K, st, mixed, 0);
  stage_mark(plan, 5, st);
  if (mixed) launch_T2(plan, V, K, st, true, 1);
  stage_mark(plan, 6, st);
  launch_final(plan, K, st);
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
  int rc = EXX_OK;
  if (Ex) rc = launch_energy(plan, K, D, Ex, st);
  stage_mark(plan, 8, st);
  return rc;
}

// E and H' workspaces of a second result (build_K_spin, build_K_two_kernels), allocated once
static int second_workspace(exx_plan plan) {
  if (plan->spin_E1) return EXX_OK;
  const int64_t ne = std::max<int64_t>(1, plan->hp.e_total);
  HIP_TRY(hipMalloc((void**)&plan->spin_E1, sizeof(double) * ne));
  plan->allocs.push_back(plan->spin_E1);
  HIP_TRY(hipMalloc((void**)&plan->spin_H1, sizeof(double) * ne));
  plan->allocs.push_back(plan->spin_H1);
  plan->dev_bytes += 2 * (int64_t)sizeof(double) * ne;
  const int64_t ndr = std::max<int64_t>(1, plan->dr_total);
  HIP_TRY(hipMalloc((void**)&plan->spin_Dr1, sizeof(double) * ndr));
  plan->allocs.push_back(plan->spin_Dr1);
  plan->dev_bytes += (int64_t)sizeof(double) * ndr;
  return EXX_OK;
}

// Collinear spin: E^s = T D^s for both spins, then one V-stage pass for both (F shared), then
// T2 and the final contraction per spin with E and H' pointed at that spin's workspace.
int build_K_spin(exx_plan plan, const double* C, const double* V, const double* D, int precision, double* K,
                 double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "build_K_spin: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "build_K_spin: host-only plan");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "build_K_spin: NULL array");
  if (precision == EXX_PREC_MIXED)
    return fail(EXX_EUNSUPPORTED, "build_K_spin: only the binary64 build takes two spins");
  if (precision != EXX_PREC_FP64) return fail(EXX_EINVAL, "build_K_spin: unknown precision");
  const HostPlan& hp = plan->hp;
  const int64_t ds = hp.d_size;
  {
    static const int t2c[3][2] = {{4, 4}, {8, 4}, {8, 8}};
    const int* cw = t2c[std::min(std::max(plan->tune[TUNE_T2], 0), 2)];
    if (t2_lds_bytes(plan->h_smax_t2, sizeof(double), cw[0], cw[1], 2) > (size_t)plan->lds_max)
      return fail(EXX_EUNSUPPORTED, "build_K_spin: the largest n_aux * n_basis needs more LDS than a workgroup has "
                                    "for two spins in the T2 tile shape chosen");
  }
  const int rcw = second_workspace(plan);
  if (rcw != EXX_OK) return rcw;
  hipStream_t st = (hipStream_t)stream;
  DevPlan& d = plan->d;
  const int n_e = (int)hp.e_items.size();
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, 2 * ds);
  hipLaunchKernelGGL(k_repack, dim3(hp.nbr_ptr[hp.n_atoms]), dim3(256), 0, st, C, plan->d);
  stage_mark(plan, 1, st);
  launch_rowD_spin(plan, D, D + ds, plan->spin_E1, rowd_E(plan), n_e, st);
  stage_mark(plan, 2, st);
  launch_vd_operands(plan, V, D, st);   // V and D^0 operands
  if (!hp.pair_a.empty())
    hipLaunchKernelGGL(k_vdrepack, dim3((unsigned)hp.pair_a.size()), dim3(256), 0, st, nullptr, D + ds,
                       plan->spin_Dr1, plan->d);   // D^1 operands
  launch_H_lists<double, 2>(plan, V, D,
                            HLists{d.g_tiles, d.gq, d.gx, plan->h_vbase, plan->h_dbase, plan->spin_E1,
                                   plan->spin_H1, plan->spin_Dr1},
                            (int)hp.g_tiles.size(), 2.0, H_WRITE, st);
  stage_mark(plan, 3, st);
  stage_mark(plan, 4, st);
  launch_T2_spin(plan, V, K, st);
  stage_mark(plan, 5, st);
  stage_mark(plan, 6, st);
  double* const H0 = d.H;
  launch_final(plan, K, st);
  d.H = plan->spin_H1;
  launch_final(plan, K + ds, st);
  d.H = H0;
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
  int rc = EXX_OK;
  if (Ex) rc = launch_energy(plan, K, D, Ex, st, 2);
  stage_mark(plan, 8, st);
  return rc;
}

// Two Coulomb matrices: repack and E = T D once, then the V stage, T2 and the final
// contraction per Coulomb matrix (H' of the second in the second workspace).  A V-stage pass
// computing both at once (shared T_Q staging and D operands) measured slower than two passes
// (49.4 against 2 x 22.0 ms at 768 atoms, with the operands then gathered from V and D): the
// V operands, whose loads bound the stage, are not shared, and the doubled accumulators
// halve the occupancy.
int build_K_two_kernels(exx_plan plan, const double* C, const double* V, const double* V2, const double* D,
                        int precision, double* K, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "build_K_two_kernels: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "build_K_two_kernels: host-only plan");
  if (!C || !V || !V2 || !D || !K) return fail(EXX_EINVAL, "build_K_two_kernels: NULL array");
  if (precision == EXX_PREC_MIXED)
    return fail(EXX_EUNSUPPORTED, "build_K_two_kernels: only the binary64 build takes two Coulomb matrices");
  if (precision != EXX_PREC_FP64) return fail(EXX_EINVAL, "build_K_two_kernels: unknown precision");
  const int rcw = second_workspace(plan);
  if (rcw != EXX_OK) return rcw;
  const HostPlan& hp = plan->hp;
  const int64_t ds = hp.d_size;
  hipStream_t st = (hipStream_t)stream;
  DevPlan& d = plan->d;
  double* const H0 = d.H;
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, 2 * ds);
  launch_repack_E(plan, C, D, st, true);
  stage_mark(plan, 2, st);
  // T2 reads the lane-ordered copy of the V operands that the V stage writes: each Coulomb
  // matrix's T2 follows its own V stage
  launch_H(plan, V, D, 2.0, H_WRITE, st);
  launch_T2(plan, V, K, st);
  d.H = plan->spin_H1;
  launch_H(plan, V2, D, 2.0, H_WRITE, st);
  d.H = H0;
  launch_T2(plan, V2, K + ds, st);
  stage_mark(plan, 3, st);
  stage_mark(plan, 4, st);
  stage_mark(plan, 5, st);
  stage_mark(plan, 6, st);
  launch_final(plan, K, st);
  d.H = plan->spin_H1;
  launch_final(plan, K + ds, st);
  d.H = H0;
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
  int rc = EXX_OK;
  if (Ex) rc = launch_energy(plan, K, D, Ex, st);
  if (Ex && rc == EXX_OK) rc = launch_energy(plan, K + ds, D, Ex + hp.n_sys, st);
  stage_mark(plan, 8, st);
  return rc;
}

int exx_graph_build(exx_plan plan, const double* C, const double* V, const double* D, int precision, double* K,
                    double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_graph_build: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_graph_build: host-only plan");
  if (!stream) return fail(EXX_EINVAL, "exx_graph_build: capture needs a created (non-default) stream");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "exx_graph_build: NULL array");
  if (precision != EXX_PREC_FP64 && precision != EXX_PREC_MIXED)
    return fail(EXX_EINVAL, "exx_graph_build: unknown precision");
  if (precision == EXX_PREC_MIXED) {
    const int rcm = prepare_mixed(plan);   // list uploads stay outside the capture
    if (rcm != EXX_OK) return rcm;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->graph_exec) { hipGraphExecDestroy(plan->graph_exec); plan->graph_exec = nullptr; }
  if (plan->graph) { hipGraphDestroy(plan->graph); plan->graph = nullptr; }
  const bool prof = plan->profiling;
  plan->profiling = false;
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = build_K(plan, C, V, D, precision, K, Ex, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  plan->profiling = prof;
  if (rc != EXX_OK) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return fail(EXX_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  plan->graph = g;
  HIP_TRY(hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0));
  return EXX_OK;
}

int exx_graph_launch(exx_plan plan, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_graph_launch: NULL plan");
  if (!plan->graph_exec) return fail(EXX_ESTATE, "exx_graph_launch: no graph built");
  HIP_TRY(hipGraphLaunch(plan->graph_exec, (hipStream_t)stream));
  return EXX_OK;
}

// time `launch` (one stage of a build) `reps` times on `st`; returns the fastest, ms
extern "C++" {
template <typename F>
static int time_stage(hipStream_t st, int reps, F launch, float& best) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  best = 1e30f;
  int rc = EXX_OK;
  for (int r = 0; r < reps && rc == EXX_OK; ++r) {
    hipEventRecord(e0, st);
    launch();
    hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(EXX_EDEVICE, "exx_plan_autotune: stage failed"); break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
}  // extern "C++"

int exx_plan_autotune(exx_plan plan, const double* C, const double* V, const double* D, int precision, double* K,
                      void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_plan_autotune: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_plan_autotune: host-only plan");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "exx_plan_autotune: NULL array");
  if (precision != EXX_PREC_FP64 && precision != EXX_PREC_MIXED)
    return fail(EXX_EINVAL, "exx_plan_autotune: unknown precision");
  hipStream_t st = (hipStream_t)stream;
  const bool mixed = precision == EXX_PREC_MIXED;
  const bool prof = plan->profiling;
  plan->profiling = false;
  // one build fills the workspace the stage kernels read
  int rc = build_K(plan, C, V, D, precision, K, nullptr, stream);
  if (rc == EXX_OK) HIP_TRY(hipStreamSynchronize(st));
  const HostPlan& hp = plan->hp;
  constexpr int REPS = 3;
  for (int stage = 0; stage < N_TUNE && rc == EXX_OK; ++stage) {
    for (int c = 0; c < kTuneCands[stage] && rc == EXX_OK; ++c) {
      plan->tune[stage] = c;
      float ms = 0.f;
      if (stage == TUNE_E) {
        rc = time_stage(st, REPS, [&] { launch_rowD(plan, D, rowd_E(plan), (int)hp.e_items.size(), st); }, ms);
      } else if (stage == TUNE_T2) {
        rc = time_stage(st, REPS, [&] {
          launch_T2(plan, V, K, st, mixed, 0);
          if (mixed) launch_T2(plan, V, K, st, true, 1);
        }, ms);
      } else {
        const int nY = (int)hp.y_tiles.size(), nYp = (nY + 7) / 8 * 8;
        rc = time_stage(st, REPS, [&] {
          if (c == 1) hipLaunchKernelGGL(k_Y<32>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
          else hipLaunchKernelGGL(k_Y<16>, dim3(nYp), dim3(256), 0, st, plan->d, nY, nYp);
        }, ms);
      }
      plan->tune_ms[stage][c] = ms;
    }
    if (rc == EXX_OK) {
      int best = 0;
      for (int c = 1; c < kTuneCands[stage]; ++c)
        if (plan->tune_ms[stage][c] < plan->tune_ms[stage][best]) best = c;
      plan->tune[stage] = best;
    }
  }
  plan->profiling = prof;
  if (rc != EXX_OK) return rc;
  plan->tuned = true;
  // leave a K of the chosen configuration behind
  rc = build_K(plan, C, V, D, precision, K, nullptr, stream);
  if (rc == EXX_OK) HIP_TRY(hipStreamSynchronize(st));
  return rc;
}

int exx_plan_tuning(exx_plan plan, int32_t* choices, float* ms) {
  if (!plan || !choices) return fail(EXX_EINVAL, "exx_plan_tuning: NULL argument");
  for (int i = 0; i < N_TUNE; ++i) {
    choices[i] = plan->tune[i];
    if (ms)
      for (int c = 0; c < N_CAND; ++c)
        ms[i * N_CAND + c] = (plan->tuned && c < kTuneCands[i]) ? plan->tune_ms[i][c] : 0.f;
  }
  return EXX_OK;
}

int exx_plan_set_tuning(exx_plan plan, const int32_t* choices) {
  if (!plan || !choices) return fail(EXX_EINVAL, "exx_plan_set_tuning: NULL argument");
  for (int i = 0; i < N_TUNE; ++i)
    if (choices[i] < 0 || choices[i] >= kTuneCands[i]) return fail(EXX_EINVAL, "exx_plan_set_tuning: choice out of range");
  for (int i = 0; i < N_TUNE; ++i) plan->tune[i] = choices[i];
  return EXX_OK;
}

int exx_plan_set_mixed_split(exx_plan plan, double r_split) {
  if (!plan) return fail(EXX_EINVAL, "exx_plan_set_mixed_split: NULL plan");
  if (!(r_split >= 0.0) || r_split > 1e6) return fail(EXX_EINVAL, "exx_plan_set_mixed_split: r_split must be in [0, 1e6]");
  if (plan->hp.mixed_ready && plan->hp.mixed_split == r_split) return EXX_OK;
  if (plan->graph_exec) { hipGraphExecDestroy(plan->graph_exec); plan->graph_exec = nullptr; }
  if (plan->graph) { hipGraphDestroy(plan->graph); plan->graph = nullptr; }
  plan->hp.mixed_split = r_split;
  plan->hp.mixed_ready = false;
  plan->mixed_uploaded = false;
  derive_mixed_lists(plan->hp);
  if (plan->host_only) return EXX_OK;
  HIP_TRY(hipDeviceSynchronize());   // lists of an earlier split may still be in use
  return prepare_mixed(plan);
}

int exchange_energy(exx_plan plan, const double* K, const double* D, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exchange_energy: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exchange_energy: host-only plan");
  if (!K || !D || !Ex) return fail(EXX_EINVAL, "exchange_energy: NULL array");
  return launch_energy(plan, K, D, Ex, (hipStream_t)stream);
}

int exchange_backward(exx_plan plan, const double* C, const double* V, const double* D, const double* K,
                      double gE, int precision, double* dC, double* dV, double* dD, double* forces,
                      double c_decay, double v_2s2, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exchange_backward: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exchange_backward: host-only plan");
  if (!C || !V || !D) return fail(EXX_EINVAL, "exchange_backward: NULL input array");
  if (precision == EXX_PREC_MIXED)
    return fail(EXX_EUNSUPPORTED, "exchange_backward: only the binary64 backward is implemented");
  if (precision != EXX_PREC_FP64) return fail(EXX_EINVAL, "exchange_backward: unknown precision");
  if (forces && (!(c_decay > 0) || !(v_2s2 > 0))) return fail(EXX_EINVAL, "exchange_backward: decay lengths must be positive");
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  const bool needC = dC || forces, needV = dV || forces;
  if (needC && !dC && !plan->dC_scratch) {
    HIP_TRY(hipMalloc((void**)&plan->dC_scratch, sizeof(double) * std::max<int64_t>(1, hp.c_off.back())));
    plan->allocs.push_back(plan->dC_scratch);
  }
  if (needV && !dV && !plan->dV_scratch) {
    HIP_TRY(hipMalloc((void**)&plan->dV_scratch, sizeof(double) * std::max<int64_t>(1, hp.v_off.back())));
    plan->allocs.push_back(plan->dV_scratch);
  }
  double* dCb = dC ? dC : plan->dC_scratch;
  double* dVb = dV ? dV : plan->dV_scratch;
  launch_repack_E(plan, C, D, st, false);
  if (dD && K) {
    // dE/dD = -1/2 K from the caller's K
    hipLaunchKernelGGL(k_scaled_copy, dim3(1024), dim3(256), 0, st, dD, K, hp.d_size, -0.5 * gE);
    if (needC) launch_H(plan, V, D, 1.0, H_WRITE, st);
  } else if (dD) {
    // dE/dD = -1/2 K: the forward build into dD, then scaled
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, dD, hp.d_size);
    launch_H(plan, V, D, 2.0, H_WRITE, st);
    launch_T2(plan, V, dD, st);
    launch_final(plan, dD, st);
    hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, st, dD, hp.d_size, -0.5 * gE);
    if (needC) launch_H(plan, V, D, -1.0, H_G_ADD, st);   // G term taken once
  } else if (needC) {
    launch_H(plan, V, D, 1.0, H_WRITE, st);
  }
  if (needC) {
    launch_rowD(plan, D, rowd_GD(plan), (int)hp.gd_items.size(), st);
    hipLaunchKernelGGL(k_unrepack, dim3(hp.nbr_ptr[hp.n_atoms]), dim3(256), 0, st, d.GD, dCb, d, -gE);
    if (forces)
      hipLaunchKernelGGL(k_block_dot, dim3((int)hp.pair_a.size()), dim3(256), 0, st, dCb, C, d.c_off, d.sC);
  }
  if (needV) {
    launch_dV(plan, V, D, dVb, gE, st);
    if (forces)
      hipLaunchKernelGGL(k_block_dot, dim3((int)hp.pair_a.size()), dim3(256), 0, st, dVb, V, d.v_off, d.sV);
  }
  if (forces)
    hipLaunchKernelGGL(k_forces, dim3((hp.n_atoms + 127) / 128), dim3(128), 0, st, d.pos, d.sC, d.sV, forces, d,
                       c_decay, v_2s2);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

}  // extern "C"
