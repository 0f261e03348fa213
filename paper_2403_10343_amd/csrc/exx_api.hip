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
#include "exx_dev.h"

#include <mutex>

using namespace exx;

thread_local std::string g_err;

// Partial sums of exchange_energy_noalloc: a fixed array in device memory (one copy per
// GPU, held until the process ends), so that the call allocates nothing.  Host code never
// uses the array's name as an address: its device address is looked up once per device
// at plan creation (hipGetSymbolAddress with that device current) and kept per device.
static __device__ __align__(256) double scratch[EXX_NOALLOC_MAX_CHUNKS];
constexpr int MAX_DEVICES = 64;
static double* g_scratch_dev[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device `dev` (looked up once)
static int scratch_lookup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(EXX_EDEVICE, "libexx: device index beyond the supported 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return EXX_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(EXX_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_dev[dev] = static_cast<double*>(p);
  return EXX_OK;
}

// Device copy of a host list, owned by the plan (or by mixed set m).
template <typename X>
static int upload(exx_plan_s* p, X*& dst, const std::vector<X>& src, MixedDev* m = nullptr) {
  dst = nullptr;
  if (src.empty()) return 0;
  size_t bytes = src.size() * sizeof(X);
  HIP_TRY(hipMalloc((void**)&dst, bytes));
  (m ? m->allocs : p->allocs).push_back(dst);
  (m ? m->bytes : p->dev_bytes) += bytes;
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

// Periodic screening: atom b pairs with a at the one image (of the 27 around the home
// cell, shifts sh[t] computed on the host) within the cutoff; the atom itself only at
// image 0.  Same arithmetic as the host builder: ((x_b + s) - x_a)^2 ... summed (xx + yy) + zz.
__device__ __forceinline__ int periodic_image(const double* pos, const double* sh, const int* codes, int a, int b,
                                              double rc2) {
  for (int t = 0; t < 27; ++t) {
    if (a == b && codes[t] != IMG0) continue;
    const double dx = __dsub_rn(__dadd_rn(pos[3 * b], sh[3 * t]), pos[3 * a]);
    const double dy = __dsub_rn(__dadd_rn(pos[3 * b + 1], sh[3 * t + 1]), pos[3 * a + 1]);
    const double dz = __dsub_rn(__dadd_rn(pos[3 * b + 2], sh[3 * t + 2]), pos[3 * a + 2]);
    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    if (r2 <= rc2) return codes[t];
  }
  return -1;
}

__global__ __launch_bounds__(256) void k_nbr_count_p(const double* pos, const double* sh, const int* codes, int n,
                                                     double rc2, int* count) {
  const int a = blockIdx.x;
  __shared__ int part[256];
  int c = 0;
  for (int b = threadIdx.x; b < n; b += 256) c += periodic_image(pos, sh, codes, a, b, rc2) >= 0 ? 1 : 0;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[a] = part[0];
}

__global__ __launch_bounds__(256) void k_nbr_fill_p(const double* pos, const double* sh, const int* codes, int n,
                                                    double rc2, const int* ptr, int* out, int* out_img) {
  const int a = blockIdx.x;
  __shared__ int scan[256];
  int base = ptr[a];
  for (int b0 = 0; b0 < n; b0 += 256) {
    const int b = b0 + threadIdx.x;
    const int im = b < n ? periodic_image(pos, sh, codes, a, b, rc2) : -1;
    const int f = im >= 0 ? 1 : 0;
    scan[threadIdx.x] = f;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {  // inclusive Hillis-Steele scan
      int v = (threadIdx.x >= w) ? scan[threadIdx.x - w] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) {
      out[base + scan[threadIdx.x] - 1] = b;
      out_img[base + scan[threadIdx.x] - 1] = im;
    }
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


// The V-stage operands in MFMA lane order (DevPlan::Vr, Dr), one workgroup per canonical
// pair, both orientations.
// V == nullptr: the D operands only (into Dr)
__global__ __launch_bounds__(256) void k_vdrepack(const double* __restrict__ V, const double* __restrict__ D,
                                                 double* __restrict__ Dr, DevPlan d, int fp32) {
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
    float* vr32 = fp32 ? d.Vr32 + d.vr_off[2 * p + o] : nullptr;
    const int nv = V ? (int)(d.vr_off[2 * p + o + 1] - d.vr_off[2 * p + o]) : 0;
    for (int e = threadIdx.x; e < nv; e += 256) {
      const int L = e & 63, tq = e >> 6, q = tq % nsq, t = tq / nsq;
      const int mu = 16 * t + (L & 15), nu = 4 * q + (L >> 4);
      const double x = (mu < aP && nu < aQ) ? v_elem(Vp, P, Q, aP, aQ, mu, nu) : 0.0;
      vr[e] = x;
      if (fp32) vr32[e] = (float)x;
    }
    double* dr = Dr + d.dr_off[2 * p + o];
    const int nd = (int)(d.dr_off[2 * p + o + 1] - d.dr_off[2 * p + o]);
    for (int e = threadIdx.x; e < nd; e += 256) {
      const int L = e & 63, q = e >> 6;
      const int j = L & 15, l = (L >> 4) + 4 * q;   // the f64 MFMA A-operand row of lane L, step q
      dr[e] = (j < bP && l < bQ) ? Ds[(size_t)(d.bo[P] + j) * ns + d.bo[Q] + l] : 0.0;
    }
    if (fp32) {
      float* dr32 = d.Dr32 + (size_t)(2 * p + o) * 256;
      for (int e = threadIdx.x; e < 256; e += 256) {
        const int L = e & 63, q = e >> 6;
        const int j = L & 15, l = 4 * (L >> 4) + q;   // binary32 accumulator row 4 (L / 16) + q
        dr32[e] = (j < bP && l < bQ) ? (float)Ds[(size_t)(d.bo[P] + j) * ns + d.bo[Q] + l] : 0.f;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// energy: sum_ik K_ik D_ik over the screened pair blocks (D beyond the cutoff
// counts as zero), per chunk of canonical pairs a workgroup tree reduction,
// then per system an ordered sum of its chunks.  n_spin density matrices (and
// their K) are stored spin_stride apart; the chunk sums run over all.

__global__ __launch_bounds__(256) void k_energy_part(const double* __restrict__ K, const double* __restrict__ D,
                                                     DevPlan d, int n_chunks, int n_spin, int64_t spin_stride,
                                                     double* __restrict__ part_out) {
  const int c = blockIdx.x;
  if (c >= n_chunks) return;
  const int s = d.en_sys[c];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s];
  __shared__ double part[256];
  double acc = 0.0;
  for (int p = d.en_pbeg[c]; p < d.en_pend[c]; ++p) {
    const int A = d.pair_a[p], B = d.pair_b[p];
    const int bA = d.nb[A], bB = d.nb[B];
    const int64_t oA = d.bo[A], oB = d.bo[B];
    for (int sp = 0; sp < n_spin; ++sp) {
      const double* Ks = K + sp * spin_stride + base;
      const double* Ds = D + sp * spin_stride + base;
      for (int e = threadIdx.x; e < bA * bB; e += 256) {
        const int i = e / bB, k = e - i * bB;
        const int64_t x = (oA + i) * ns + oB + k;
        acc += Ks[x] * Ds[x];
        if (A != B) {
          const int64_t y = (oB + k) * ns + oA + i;
          acc += Ks[y] * Ds[y];
        }
      }
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part_out[c] = part[0];
}

// scale: -1/4 for one (spin-summed) density matrix, -1/2 for the two spin density matrices
__global__ void k_energy_sum(double* Ex, DevPlan d, int n_chunks, double scale, const double* __restrict__ part) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= d.n_sys) return;
  double acc = 0.0;
  for (int c = 0; c < n_chunks; ++c)
    if (d.en_sys[c] == s) acc += part[c];
  Ex[s] = scale * acc;
}

// Dm = D on the screened pair blocks (one workgroup per canonical pair, both
// orientations); entries outside them stay zero from the plan's set-up.
__global__ __launch_bounds__(256) void k_dmask(const double* __restrict__ D, double* __restrict__ Dm, DevPlan d) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int s = d.atom_sys[A];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t oA = d.bo[A], oB = d.bo[B];
  for (int e = threadIdx.x; e < bA * bB; e += 256) {
    const int i = e / bB, k = e - i * bB;
    const int64_t x = base + (oA + i) * ns + oB + k, y = base + (oB + k) * ns + oA + i;
    Dm[x] = D[x];
    Dm[y] = D[y];
  }
}

// ---------------------------------------------------------------------------
// maximum-norm estimates (binary64).  Per canonical pair (A, B): max|C| over its stored
// block, max|V| over its block, max|D| over the (A, B) and (B, A) blocks of D (one
// workgroup per pair; maxima are exact in any order).  Then per atom A: tau_A, the largest
// max|C| of a pair with A, and rho_A, the largest max|D| of a pair with A; sigma_A, the
// largest rho_J over J in N[A].  The estimate of the V block of a pair (P, Q),
// ((max|V_PQ| tau_P) tau_Q) min(sigma_P, sigma_Q), bounds every term C^mu_ij V_mu,nu
// C^nu_kl D_jl with mu on P and nu on Q (j lies on an atom of N[P], l on one of N[Q]);
// below the threshold the build skips every product through that block.

// D1 (may be null): a second density matrix (collinear spin) whose blocks enter max|D| too
__global__ __launch_bounds__(256) void k_block_norms(const double* __restrict__ C, const double* __restrict__ V,
                                                     const double* __restrict__ D, DevPlan d,
                                                     double* __restrict__ nrm, const double* __restrict__ D1) {
  __shared__ double red[3][256];
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int s = d.atom_sys[A];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t oA = d.bo[A], oB = d.bo[B];
  double mc = 0.0, mv = 0.0, md = 0.0;
  for (int64_t e = d.c_off[p] + threadIdx.x; e < d.c_off[p + 1]; e += 256) mc = fmax(mc, fabs(C[e]));
  for (int64_t e = d.v_off[p] + threadIdx.x; e < d.v_off[p + 1]; e += 256) mv = fmax(mv, fabs(V[e]));
  for (int e = threadIdx.x; e < bA * bB; e += 256) {
    const int i = e / bB, k = e - i * bB;
    md = fmax(md, fmax(fabs(D[base + (oA + i) * ns + oB + k]), fabs(D[base + (oB + k) * ns + oA + i])));
    if (D1) md = fmax(md, fmax(fabs(D1[base + (oA + i) * ns + oB + k]), fabs(D1[base + (oB + k) * ns + oA + i])));
  }
  red[0][threadIdx.x] = mc;
  red[1][threadIdx.x] = mv;
  red[2][threadIdx.x] = md;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 3; ++j) red[j][threadIdx.x] = fmax(red[j][threadIdx.x], red[j][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) nrm[3 * (int64_t)p + threadIdx.x] = red[threadIdx.x][0];
}

// tau_A, rho_A (pass 0) or sigma_A (pass 1) for every atom; nrm + 3 n_pairs holds tau, rho, sigma
__global__ void k_atom_norms(DevPlan d, double* __restrict__ nrm, int n_pairs, int pass) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= d.n_atoms) return;
  double* at = nrm + 3 * (int64_t)n_pairs;
  if (pass == 0) {
    double t = 0.0, r = 0.0;
    for (int k = d.nbr_ptr[A]; k < d.nbr_ptr[A + 1]; ++k) {
      const int64_t p = d.nbr_pair[k];
      t = fmax(t, nrm[3 * p]);
      r = fmax(r, nrm[3 * p + 2]);
    }
    at[A] = t;
    at[d.n_atoms + A] = r;
  } else {
    double sg = 0.0;
    for (int k = d.nbr_ptr[A]; k < d.nbr_ptr[A + 1]; ++k) sg = fmax(sg, at[d.n_atoms + d.nbr_atom[k]]);
    at[2 * d.n_atoms + A] = sg;
  }
}

__global__ void k_screen(DevPlan d, const double* __restrict__ nrm, int n_pairs, double eps,
                         uint8_t* __restrict__ flags) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const double* tau = nrm + 3 * (int64_t)n_pairs;
  const double* sigma = tau + 2 * d.n_atoms;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const double est = ((nrm[3 * (int64_t)p + 1] * tau[A]) * tau[B]) * fmin(sigma[A], sigma[B]);
  flags[p] = est < eps ? 1 : 0;
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
                                                  DevPlan d, const double* __restrict__ gE, double a) {
  const int k = blockIdx.x;
  const int P = d.nbr_owner[k], J = d.nbr_atom[k], p = d.nbr_pair[k];
  const int aP = d.na[P], bP = d.nb[P], bJ = d.nb[J], aJ = d.na[J];
  const int nP = d.n_loc[P], lc = d.nbr_lcol[k];
  const int sP = aP * bP;
  double* Cp = dC + d.c_off[p];
  const double* GP = GD + d.t_off[P];
  const double scale = a * gE[d.atom_sys[P]];
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
    // separation R_A - R_J (periodic: to J's image within the cutoff)
    const double dx = d.periodic ? d.nbr_sep[3 * (size_t)k] : pos[3 * A] - pos[3 * J];
    const double dy = d.periodic ? d.nbr_sep[3 * (size_t)k + 1] : pos[3 * A + 1] - pos[3 * J + 1];
    const double dz = d.periodic ? d.nbr_sep[3 * (size_t)k + 2] : pos[3 * A + 2] - pos[3 * J + 2];
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

// Strain derivative dE/d(eps_ab) of the energy under a homogeneous deformation x -> (1 + eps) x
// of every position (and of the lattice): sum over canonical pairs of g_a r_b, where r is the
// pair's separation (at its image) and g = dE/dr from the same per-pair sums as the forces.
// Per atom the half sum over its neighbour entries (each pair is seen from both ends with r
// and g negated), then one fixed-order reduction over the atoms.
__global__ void k_strain_part(const double* __restrict__ pos, const double* __restrict__ sC,
                              const double* __restrict__ sV, double* __restrict__ part, DevPlan d,
                              double c_decay, double v_2s2) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= d.n_atoms) return;
  double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = d.nbr_ptr[A]; k < d.nbr_ptr[A + 1]; ++k) {
    const int J = d.nbr_atom[k];
    if (J == A) continue;
    const int p = d.nbr_pair[k];
    double r3[3];
    for (int x = 0; x < 3; ++x) r3[x] = d.periodic ? d.nbr_sep[3 * (size_t)k + x] : pos[3 * A + x] - pos[3 * J + x];
    const double r = sqrt(r3[0] * r3[0] + r3[1] * r3[1] + r3[2] * r3[2]);
    const double f = sC[p] * (-1.0 / c_decay) / r + sV[p] * (-2.0 / v_2s2);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) w[3 * a + b] += (f * r3[a]) * r3[b];
  }
  for (int x = 0; x < 9; ++x) part[9 * (size_t)A + x] = 0.5 * w[x];
}

__global__ __launch_bounds__(256) void k_strain_sum(const double* __restrict__ part, int n_atoms,
                                                    double* __restrict__ out) {
  __shared__ double red[256];
  for (int x = 0; x < 9; ++x) {
    double acc = 0.0;
    for (int A = threadIdx.x; A < n_atoms; A += 256) acc += part[9 * (size_t)A + x];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[x] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Bloch sums.  With the cutoff below half the cell width every pair (A, B) has one image
// n_AB, so K_AB(k) = sum_R e^{i k.R} X_AB(R) keeps one term, e^{2 pi i k.n_AB} X_AB (k in
// fractional reciprocal coordinates), and the (B, A) block takes the conjugate phase.  The
// density matrix in real space, D_AB(R) = (1 / N_k) sum_k D_AB(k) e^{i k.R}, is needed at
// R = n_AB only: the real part of (1 / N_k) sum_k e^{2 pi i k.n_AB} D_AB(k).  One workgroup
// per canonical pair; the k-points (at most KPT_MAX per launch) are kernel arguments.

constexpr int KPT_MAX = 32;
struct KPts { double k[KPT_MAX][3]; int n; };

__device__ __forceinline__ void pair_image(const DevPlan& d, int A, int B, int (&n)[3]) {
  const int code = d.periodic ? d.pimg[(size_t)A * d.n_atoms + B] : IMG0;
  n[0] = code % IMG_S - IMG_OFF;
  n[1] = (code / IMG_S) % IMG_S - IMG_OFF;
  n[2] = code / (IMG_S * IMG_S) - IMG_OFF;
}

// Kk[k0 + q] (complex, interleaved) on the pair blocks from the real folded X
__global__ __launch_bounds__(256) void k_bloch(const double* __restrict__ X, double* __restrict__ Kk, DevPlan d,
                                               KPts kp, int k0) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int s = d.atom_sys[A];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s], dsz = d.sys_d_off[d.n_sys];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t oA = d.bo[A], oB = d.bo[B];
  int n[3];
  pair_image(d, A, B, n);
  for (int q = 0; q < kp.n; ++q) {
    double sn, cs;
    sincospi(2.0 * (kp.k[q][0] * n[0] + kp.k[q][1] * n[1] + kp.k[q][2] * n[2]), &sn, &cs);
    double* Kq = Kk + 2 * (size_t)(k0 + q) * dsz;
    for (int e = threadIdx.x; e < bA * bB; e += 256) {
      const int i = e / bB, j = e - i * bB;
      const int64_t x = base + (oA + i) * ns + oB + j, y = base + (oB + j) * ns + oA + i;
      Kq[2 * x] = cs * X[x];
      Kq[2 * x + 1] = sn * X[x];
      if (A != B) {
        Kq[2 * y] = cs * X[y];
        Kq[2 * y + 1] = -sn * X[y];
      }
    }
  }
}

// D (pair blocks) += sum over the launch's k-points of Re(e^{2 pi i k.n} Dk[k0 + q])
__global__ __launch_bounds__(256) void k_density_k(const double* __restrict__ Dk, double* __restrict__ D, DevPlan d,
                                                   KPts kp, int k0) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int s = d.atom_sys[A];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s], dsz = d.sys_d_off[d.n_sys];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t oA = d.bo[A], oB = d.bo[B];
  int n[3];
  pair_image(d, A, B, n);
  double cs[KPT_MAX], sn[KPT_MAX];
  for (int q = 0; q < kp.n; ++q)
    sincospi(2.0 * (kp.k[q][0] * n[0] + kp.k[q][1] * n[1] + kp.k[q][2] * n[2]), &sn[q], &cs[q]);
  for (int e = threadIdx.x; e < bA * bB; e += 256) {
    const int i = e / bB, j = e - i * bB;
    const int64_t x = base + (oA + i) * ns + oB + j, y = base + (oB + j) * ns + oA + i;
    double ax = D[x], ay = D[y];
    for (int q = 0; q < kp.n; ++q) {
      const double* Dq = Dk + 2 * (size_t)(k0 + q) * dsz;
      ax += cs[q] * Dq[2 * x] - sn[q] * Dq[2 * x + 1];
      if (A != B) ay += cs[q] * Dq[2 * y] + sn[q] * Dq[2 * y + 1];
    }
    D[x] = ax;
    if (A != B) D[y] = ay;
  }
}

// D *= a on the pair blocks
__global__ __launch_bounds__(256) void k_scale_pairs(double* __restrict__ D, DevPlan d, double a) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int s = d.atom_sys[A];
  const int64_t base = d.sys_d_off[s], ns = d.sys_n[s];
  const int bA = d.nb[A], bB = d.nb[B];
  const int64_t oA = d.bo[A], oB = d.bo[B];
  for (int e = threadIdx.x; e < bA * bB; e += 256) {
    const int i = e / bB, j = e - i * bB;
    const int64_t x = base + (oA + i) * ns + oB + j, y = base + (oB + j) * ns + oA + i;
    D[x] *= a;
    if (A != B) D[y] *= a;
  }
}

// y = a gE[s] x over the dense block of every system s (blockIdx.y = s); y == x scales in place
__global__ void k_scaled_copy_sys(double* y, const double* x, const double* __restrict__ gE, DevPlan d, double a) {
  const int s = blockIdx.y;
  const int64_t b = d.sys_d_off[s], n = d.sys_d_off[s + 1] - b;
  const double f = a * gE[s];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[b + i] = f * x[b + i];
}

// ---------------------------------------------------------------------------
// plan creation

static int device_neighbors_periodic(exx_plan_s* pl) {
  HostPlan& hp = pl->hp;
  const int NA = hp.n_atoms;
  double sh[27 * 3];
  int codes[27];
  for (int t = 0; t < 27; ++t) {
    codes[t] = img_code(t / 9 - 1, (t / 3) % 3 - 1, t % 3 - 1);
    image_shift(hp.lat, codes[t], sh + 3 * t);
  }
  double *dpos = nullptr, *dsh = nullptr;
  int *dcodes = nullptr, *dcnt = nullptr, *dptr = nullptr, *dout = nullptr, *dimg = nullptr;
  auto cleanup = [&]() {
    hipFree(dpos); hipFree(dsh); hipFree(dcodes); hipFree(dcnt); hipFree(dptr); hipFree(dout); hipFree(dimg);
  };
  hipError_t e = hipSuccess;
#define NB_TRY(x) do { e = (x); if (e != hipSuccess) { cleanup(); return fail(EXX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e)); } } while (0)
  NB_TRY(hipMalloc((void**)&dpos, sizeof(double) * 3 * NA));
  NB_TRY(hipMalloc((void**)&dsh, sizeof(sh)));
  NB_TRY(hipMalloc((void**)&dcodes, sizeof(codes)));
  NB_TRY(hipMalloc((void**)&dcnt, sizeof(int) * NA));
  NB_TRY(hipMemcpy(dpos, hp.pos.data(), sizeof(double) * 3 * NA, hipMemcpyHostToDevice));
  NB_TRY(hipMemcpy(dsh, sh, sizeof(sh), hipMemcpyHostToDevice));
  NB_TRY(hipMemcpy(dcodes, codes, sizeof(codes), hipMemcpyHostToDevice));
  const double rc2 = hp.r_cut * hp.r_cut;
  hipLaunchKernelGGL(k_nbr_count_p, dim3(NA), dim3(256), 0, 0, dpos, dsh, dcodes, NA, rc2, dcnt);
  NB_TRY(hipGetLastError());
  std::vector<int> cnt(NA);
  NB_TRY(hipMemcpy(cnt.data(), dcnt, sizeof(int) * NA, hipMemcpyDeviceToHost));
  hp.nbr_ptr.assign(NA + 1, 0);
  for (int a = 0; a < NA; ++a) hp.nbr_ptr[a + 1] = hp.nbr_ptr[a] + cnt[a];
  NB_TRY(hipMalloc((void**)&dptr, sizeof(int) * (NA + 1)));
  NB_TRY(hipMalloc((void**)&dout, sizeof(int) * std::max(1, hp.nbr_ptr[NA])));
  NB_TRY(hipMalloc((void**)&dimg, sizeof(int) * std::max(1, hp.nbr_ptr[NA])));
  NB_TRY(hipMemcpy(dptr, hp.nbr_ptr.data(), sizeof(int) * (NA + 1), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_nbr_fill_p, dim3(NA), dim3(256), 0, 0, dpos, dsh, dcodes, NA, rc2, dptr, dout, dimg);
  NB_TRY(hipGetLastError());
  hp.nbr_atom.resize(hp.nbr_ptr[NA]);
  hp.nbr_img.resize(hp.nbr_ptr[NA]);
  NB_TRY(hipMemcpy(hp.nbr_atom.data(), dout, sizeof(int) * hp.nbr_ptr[NA], hipMemcpyDeviceToHost));
  NB_TRY(hipMemcpy(hp.nbr_img.data(), dimg, sizeof(int) * hp.nbr_ptr[NA], hipMemcpyDeviceToHost));
#undef NB_TRY
  cleanup();
  return 0;
}

static int device_neighbors(exx_plan_s* pl) {
  HostPlan& hp = pl->hp;
  if (hp.periodic) return device_neighbors_periodic(pl);
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
  UP(t_off); UP(ct_run_ptr); UP(ct_klen); UP(runs); UP(ct_kflag); UP(ct_kflag_off);
  UP(gd_run_ptr); UP(gd_klen); UP(gd_runs); UP(pos); UP(gd_kflag); UP(gd_kflag_off);
  UP(grp_first); UP(grp_unit_ptr); UP(grp_col_ptr); UP(grp_cols); UP(grp_units);
  UP(gq); UP(gx); UP(en_sys); UP(en_pbeg); UP(en_pend);
  UP(pimg); UP(col2img); UP(col1img); UP(atom_of_col); UP(grp_colimg); UP(grp_cmap); UP(t2col_off); UP(t2col);
  UP(nbr_sep); UP(dvcol_off); UP(dvcol); UP(dv_cp); UP(dv_cq);
  UP(pg_beg); UP(pg_mid); UP(pg_end); UP(pg_ent); UP(pt_tiles); UP(pt_ent); UP(pg_pairs);
#undef UP
  d.periodic = hp.periodic ? 1 : 0;
  if ((rc = upload(pl, pl->g_tiles_all, hp.g_tiles))) return rc;
  if ((rc = upload(pl, pl->y_tiles_all, hp.y_tiles))) return rc;
  if ((rc = upload(pl, pl->gd_items_all, hp.gd_items))) return rc;
  d.g_tiles = pl->g_tiles_all;
  // chunk lists: the global lists for an unbounded plan, else one set per chunk
  if (hp.chunks.empty()) {
    ChunkDev c;
    if ((rc = upload(pl, c.e_items, hp.e_items))) return rc;
    c.n_e = (int)hp.e_items.size();
    c.gt_end = (int)hp.g_tiles.size();
    c.y_end = (int)hp.y_tiles.size();
    c.gd_end = (int)hp.gd_items.size();
    if ((rc = upload(pl, c.t2_items, hp.t2_items))) return rc;
    c.t2_classes = hp.t2_classes;
    if ((rc = upload(pl, c.dv_items, hp.dv_items))) return rc;
    c.dv_classes = hp.dv_classes;
    if ((rc = upload(pl, c.f_items, hp.f_items))) return rc;
    c.n_f = (int)hp.f_items.size();
    if ((rc = upload(pl, c.f_plist, hp.f_plist))) return rc;
    if ((rc = upload(pl, c.e_off, hp.e_off))) return rc;
    c.h_off = c.e_off;   // H'_P and E_P share the layout
    if ((rc = upload(pl, c.y_off, hp.y_off))) return rc;
    c.h_base = hp.e_total;
    c.y_base = 2 * hp.e_total;
    c.pt_tiles = d.pt_tiles;
    c.pt_ent = d.pt_ent;
    c.pt_classes = hp.pt_classes;
    c.pg_beg = d.pg_beg; c.pg_mid = d.pg_mid; c.pg_end = d.pg_end; c.pg_ent = d.pg_ent;
    c.pg_pairs = d.pg_pairs;
    c.n_pg = (int)hp.pg_pairs.size();
    pl->chunks.push_back(std::move(c));
  } else {
    for (const ChunkHost& h : hp.chunks) {
      ChunkDev c;
      if ((rc = upload(pl, c.e_items, h.e_items))) return rc;
      c.n_e = (int)h.e_items.size();
      c.gt_beg = h.gt_beg; c.gt_end = h.gt_end;
      c.y_beg = h.y_beg; c.y_end = h.y_end;
      c.gd_beg = h.gd_beg; c.gd_end = h.gd_end;
      if ((rc = upload(pl, c.t2_items, h.t2_items))) return rc;
      c.t2_classes = h.t2_classes;
      if ((rc = upload(pl, c.dv_items, h.dv_items))) return rc;
      c.dv_classes = h.dv_classes;
      if ((rc = upload(pl, c.f_items, h.f_items))) return rc;
      c.n_f = (int)h.f_items.size();
      if ((rc = upload(pl, c.f_plist, h.f_plist))) return rc;
      if ((rc = upload(pl, c.e_off, h.e_off))) return rc;
      if ((rc = upload(pl, c.h_off, h.h_off))) return rc;
      if ((rc = upload(pl, c.y_off, h.y_off))) return rc;
      c.h_base = h.e_total;
      c.y_base = h.e_total + h.h_total;
      if (hp.periodic) {
        if ((rc = upload(pl, c.pt_tiles, h.pt_tiles))) return rc;
        if ((rc = upload(pl, c.pt_ent, h.pt_ent))) return rc;
        c.pt_classes = h.pt_classes;
        if ((rc = upload(pl, c.pg_beg, h.pg_beg))) return rc;
        if ((rc = upload(pl, c.pg_mid, h.pg_mid))) return rc;
        if ((rc = upload(pl, c.pg_end, h.pg_end))) return rc;
        if ((rc = upload(pl, c.pg_ent, h.pg_ent))) return rc;
        if ((rc = upload(pl, c.pg_pairs, h.pg_pairs))) return rc;
        c.n_pg = (int)h.pg_pairs.size();
      }
      pl->chunks.push_back(std::move(c));
    }
  }
  if ((rc = alloc_buf(pl, d.T, hp.t_total))) return rc;
  if ((rc = alloc_buf(pl, pl->W, hp.ws_total))) return rc;
  if ((rc = alloc_buf(pl, d.GD, hp.t_total))) return rc;
  if ((rc = alloc_buf(pl, d.sC, (int64_t)hp.pair_a.size()))) return rc;
  if ((rc = alloc_buf(pl, d.sV, (int64_t)hp.pair_a.size()))) return rc;
  if ((rc = alloc_buf(pl, d.epart, std::max<int64_t>(1, (int64_t)hp.en_sys.size())))) return rc;
  if ((rc = alloc_buf(pl, d.Dm, std::max<int64_t>(1, hp.d_size)))) return rc;
  HIP_TRY(hipMemset(d.Dm, 0, sizeof(double) * std::max<int64_t>(1, hp.d_size)));
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
  set_chunk(pl, 0);
  return 0;
}

void set_chunk(exx_plan pl, int c) {
  ChunkDev& ch = pl->chunks[c];
  DevPlan& d = pl->d;
  pl->cur = c;
  d.e_items = ch.e_items;
  d.t2_items = ch.t2_items;
  d.dv_items = ch.dv_items;
  d.f_items = ch.f_items;
  d.f_plist = ch.f_plist;
  d.e_off = ch.e_off;
  d.h_off = ch.h_off;
  d.y_off = ch.y_off;
  d.y_tiles = pl->y_tiles_all + ch.y_beg;
  d.gd_items = pl->gd_items_all + ch.gd_beg;
  d.pt_tiles = ch.pt_tiles;
  d.pt_ent = ch.pt_ent;
  d.pg_beg = ch.pg_beg;
  d.pg_mid = ch.pg_mid;
  d.pg_end = ch.pg_end;
  d.pg_ent = ch.pg_ent;
  d.pg_pairs = ch.pg_pairs;
  d.E = pl->W;
  d.H = pl->W ? pl->W + ch.h_base : nullptr;
  d.Y = pl->W ? pl->W + ch.y_base : nullptr;
}

static void free_mixed(MixedDev& m) {
  for (void* p : m.allocs) hipFree(p);
  m = MixedDev{};
}

static void release(exx_plan_s* pl) {
  if (pl->graph_exec) hipGraphExecDestroy(pl->graph_exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  pl->graph_exec = nullptr;
  pl->graph = nullptr;
  for (void* p : pl->allocs) hipFree(p);
  pl->allocs.clear();
  for (MixedDev& m : pl->mdev) free_mixed(m);
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

int exx_plan_create(const exx_system* sys, uint32_t flags, size_t ws_budget_bytes, exx_plan* out) {
  g_err.clear();
  if (!out) return fail(EXX_EINVAL, "exx_plan_create: out is NULL");
  *out = nullptr;
  if (!sys) return fail(EXX_EINVAL, "exx_plan_create: sys is NULL");
  exx_plan_s* pl = new (std::nothrow) exx_plan_s();
  if (!pl) return fail(EXX_ENOMEM, "exx_plan_create: host allocation");
  pl->host_only = (flags & EXX_PLAN_HOST_ONLY) != 0;
  std::string err;
  int rc = describe_system(sys->n_atoms, sys->n_species, sys->species, sys->positions, sys->n_basis,
                           sys->n_aux, sys->r_cut, sys->n_systems, sys->sys_atom_off, sys->lattice, pl->hp, err);
  if (rc != 0) {
    delete pl;
    return fail(rc, err);
  }
  if (pl->host_only) {
    if (pl->hp.periodic) host_neighbors_periodic(pl->hp);
    else host_neighbors(pl->hp);
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
  if (ws_budget_bytes > (size_t)INT64_MAX) ws_budget_bytes = (size_t)INT64_MAX;
  try {
    rc = pl->hp.periodic ? derive_lists_periodic(pl->hp, err) : derive_lists(pl->hp, err);
    if (rc != 0) {
      delete pl;
      return fail(rc == -5 ? EXX_EUNSUPPORTED : EXX_EDEVICE, err);
    }
    rc = derive_chunks(pl->hp, (int64_t)ws_budget_bytes, err);
  } catch (const std::bad_alloc&) {
    delete pl;
    return fail(EXX_ENOMEM, "exx_plan_create: host allocation in list building");
  }
  if (rc != 0) {
    delete pl;
    return fail(rc == -5 ? EXX_EUNSUPPORTED : EXX_ENOMEM, err);
  }
  {
    int amax = 1;
    for (int a = 0; a < pl->hp.n_atoms; ++a) amax = std::max(amax, pl->hp.na[a]);
    pl->t2_nt = (amax + 15) / 16;
    int smax = 1;
    for (int a = 0; a < pl->hp.n_atoms; ++a) smax = std::max(smax, pl->hp.na[a] * pl->hp.nb[a]);
    // k_H: T_Q tile | V blocks [nu][aux rows of the group] | D blocks
    // rows of the staged T_Q read by the chains: up to 4 NS * n_b(Q) + 16 (NS of Q's shape class)
    int h_rows = smax;
    for (int a = 0; a < pl->hp.n_atoms; ++a) {
      const int nsq = (pl->hp.na[a] + 3) / 4, nlq = (pl->hp.nb[a] + 3) / 4;
      const int NS = (nsq <= 4 && nlq <= 2) ? 4 : (nsq <= 10 ? 10 : 16);
      h_rows = std::max(h_rows, 4 * NS * pl->hp.nb[a] + 16);
    }
    pl->h_vbase = h_rows * LDS_PITCH;
    pl->h_lds = (size_t)pl->h_vbase * sizeof(double);   // k_H stages T_Q only
    pl->t2_lds = std::max((size_t)2 * smax * T2_PITCH, (size_t)16 * 64) * sizeof(double);
    pl->h_smax_t2 = smax;
    pl->h_lds32 = (size_t)pl->h_vbase * sizeof(float);
    pl->t2_lds32 = std::max((size_t)2 * smax * T2_PITCH * sizeof(float), (size_t)16 * 64 * sizeof(double));
  }
  if (!pl->host_only) {
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device) != hipSuccess) {
      delete pl;
      return fail(EXX_EDEVICE, "exx_plan_create: cannot query the LDS size");
    }
    pl->lds_max = lds_max;
    if ((rc = scratch_lookup(pl->device)) != EXX_OK) {
      delete pl;
      return rc;
    }
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
  info->workspace_bytes = plan->dev_bytes + plan->mdev[0].bytes + plan->mdev[1].bytes;
  info->flops_fp64 = hp.flops[0] + hp.flops[1] + hp.flops[2] + hp.flops[3] + hp.flops[4];
  info->n_chunks = hp.chunks.empty() ? 1 : (int64_t)hp.chunks.size();
  info->intermediate_bytes = (int64_t)sizeof(double) * hp.ws_total;
  info->intermediate_bytes_stored = hp.inter_stored;
  return EXX_OK;
}

int exx_pair_layout(exx_plan plan, int32_t* pair_a, int32_t* pair_b, int64_t* c_off, int64_t* v_off) {
  if (!plan) return fail(EXX_EINVAL, "exx_pair_layout: NULL plan");
  const HostPlan& hp = plan->hp;
  const size_t n = hp.pair_a.size();
  if (pair_a) std::memcpy(pair_a, hp.pair_a.data(), n * sizeof(int32_t));
  if (pair_b) std::memcpy(pair_b, hp.pair_b.data(), n * sizeof(int32_t));
  if (c_off) std::memcpy(c_off, hp.c_off.data(), (n + 1) * sizeof(int64_t));
  if (v_off) std::memcpy(v_off, hp.v_off.data(), (n + 1) * sizeof(int64_t));
  return EXX_OK;
}

int exx_pair_images(exx_plan plan, int32_t* images) {
  if (!plan || !images) return fail(EXX_EINVAL, "exx_pair_images: NULL argument");
  const HostPlan& hp = plan->hp;
  const size_t n = hp.pair_a.size();
  for (size_t p = 0; p < n; ++p) {
    const int code = hp.periodic ? hp.pair_img[p] : IMG0;
    images[3 * p] = code % IMG_S - IMG_OFF;
    images[3 * p + 1] = (code / IMG_S) % IMG_S - IMG_OFF;
    images[3 * p + 2] = code / (IMG_S * IMG_S) - IMG_OFF;
  }
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
    if (!plan->hp.mixed[0].ready) derive_mixed_lists(plan->hp, 0);
    const MixedSet& m = hp.mixed[0];
    if (stage < 30) return m.flops32[stage - 20];
    if (stage < 40) return m.issued32[stage - 30];
    return m.issued64[stage - 40];
  }
  if (stage > 4) return -1;
  return hp.flops[stage];
}

// E_x of every system; part: device buffer of one double per energy chunk
static int launch_energy(exx_plan plan, const double* K, const double* D, double* Ex, hipStream_t st,
                         int n_spin = 1, double* part = nullptr) {
  const int nch = (int)plan->hp.en_sys.size();
  if (!part) part = plan->d.epart;
  if (nch > 0)
    hipLaunchKernelGGL(k_energy_part, dim3(nch), dim3(256), 0, st, K, D, plan->d, nch, n_spin, plan->hp.d_size, part);
  hipLaunchKernelGGL(k_energy_sum, dim3((plan->hp.n_sys + 63) / 64), dim3(64), 0, st, Ex, plan->d, nch,
                     n_spin == 1 ? -0.25 : -0.5, (const double*)part);
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
              d.e_items, d.ct_run_ptr, d.ct_klen, d.runs, plan->hp.periodic ? d.col2img : nullptr,
              d.ct_kflag, d.ct_kflag_off};
}

static RowD rowd_GD(exx_plan plan) {
  DevPlan& d = plan->d;
  return RowD{d.H, d.h_off, d.m_loc, d.GD, d.t_off, d.n_loc, d.col1g, d.col1g_off,
              d.gd_items, d.gd_run_ptr, d.gd_klen, d.gd_runs, plan->hp.periodic ? d.col1img : nullptr,
              d.gd_kflag, d.gd_kflag_off};
}

static const ChunkDev& cur_chunk(exx_plan plan) { return plan->chunks[plan->cur]; }

// Dm: the caller's D on the screened pair blocks (everything the E = M D
// product and the gradient product read of D)
static void launch_dmask(exx_plan plan, const double* D, double* Dm, hipStream_t st) {
  const unsigned np = (unsigned)plan->hp.pair_a.size();
  if (np) hipLaunchKernelGGL(k_dmask, dim3(np), dim3(256), 0, st, D, Dm, plan->d);
}

static void launch_repack(exx_plan plan, const double* C, hipStream_t st) {
  const HostPlan& hp = plan->hp;
  hipLaunchKernelGGL(k_repack, dim3(hp.nbr_ptr[hp.n_atoms]), dim3(256), 0, st, C, plan->d);
}

// E_P = T_P Dm for the atoms of the current chunk
static void launch_E(exx_plan plan, hipStream_t st) {
  launch_rowD(plan, plan->d.Dm, rowd_E(plan), cur_chunk(plan).n_e, st);
}

// the lane-ordered V and D operands of the V stage (DevPlan::Vr, Dr; with fp32 also the
// binary32 copies Vr32, Dr32) for these V and D
// maximum-norm estimates of C, V and D into plan->scr_nrm, then the screening flags of the
// plan's threshold into plan->scr_flags
static void launch_screening(exx_plan plan, const double* C, const double* V, const double* D, hipStream_t st,
                             const double* D1 = nullptr) {
  const int np = (int)plan->hp.pair_a.size(), na = plan->hp.n_atoms;
  if (np <= 0) return;
  hipLaunchKernelGGL(k_block_norms, dim3(np), dim3(256), 0, st, C, V, D, plan->d, plan->scr_nrm, D1);
  hipLaunchKernelGGL(k_atom_norms, dim3((na + 255) / 256), dim3(256), 0, st, plan->d, plan->scr_nrm, np, 0);
  hipLaunchKernelGGL(k_atom_norms, dim3((na + 255) / 256), dim3(256), 0, st, plan->d, plan->scr_nrm, np, 1);
  hipLaunchKernelGGL(k_screen, dim3((np + 255) / 256), dim3(256), 0, st, plan->d, plan->scr_nrm, np,
                     plan->scr_eps, plan->scr_flags);
}

static void launch_vd_operands(exx_plan plan, const double* V, const double* D, hipStream_t st, bool fp32 = false) {
  const unsigned np = (unsigned)plan->hp.pair_a.size();
  if (np) hipLaunchKernelGGL(k_vdrepack, dim3(np), dim3(256), 0, st, V, D, plan->d.Dr, plan->d, fp32 ? 1 : 0);
}

// V stage (binary64) of the current chunk's groups; the operands must be in place
static void launch_H(exx_plan plan, const double* V, const double* D, double gscale, int mode, hipStream_t st) {
  const DevPlan& d = plan->d;
  const ChunkDev& ch = cur_chunk(plan);
  launch_H_lists<double>(plan, V, D, HLists{d.g_tiles + ch.gt_beg, d.gq, d.gx, plan->h_vbase},
                         ch.gt_end - ch.gt_beg, gscale, mode, st);
}

// V stage of a mixed build (list set m): near pairs stored in binary64, far pairs added in binary32
static void stage_mark(exx_plan_s* pl, int i, hipStream_t st);
static void launch_H_mixed(exx_plan plan, int m, const double* V, const double* D, hipStream_t st) {
  const ChunkDev& ch = cur_chunk(plan);
  const MixedDev& md = plan->mdev[m];
  const std::vector<int>& src = plan->hp.mixed[m].far_src;
  const int fb = (int)(std::lower_bound(src.begin(), src.end(), ch.gt_beg) - src.begin());
  const int fe = (int)(std::lower_bound(src.begin(), src.end(), ch.gt_end) - src.begin());
  launch_H_lists<double>(plan, V, D, HLists{md.tiles_near + ch.gt_beg, md.q_near, md.x_near, plan->h_vbase},
                         ch.gt_end - ch.gt_beg, 2.0, H_WRITE, st);
  stage_mark(plan, 3, st);
  launch_H_lists<float>(plan, V, D, HLists{md.tiles_far + fb, md.q_far, md.x_far, plan->h_vbase},
                        fe - fb, 2.0, H_ADD, st);
}

// one launch per shape class (aux tiles of P, nu steps of Q) and precision
// spin: both spin density matrices in one pass (binary64 lists; K holds K^0 then K^1)
static void launch_T2_spin(exx_plan plan, const double* V, double* K, hipStream_t st) {
  const ChunkDev& ch = cur_chunk(plan);
  for (const T2Class& c : ch.t2_classes) launch_T2_class<double, 2>(plan, c, V, K, ch.t2_items, st);
}

// m < 0: the binary64 lists; else the classes of mixed set m in precision prec
static void launch_T2(exx_plan plan, const double* V, double* K, hipStream_t st, int m = -1, int prec = 0) {
  const ChunkDev& ch = cur_chunk(plan);
  if (m < 0) {
    for (const T2Class& c : ch.t2_classes) launch_T2_class<double>(plan, c, V, K, ch.t2_items, st);
    return;
  }
  for (const T2Class& c : ch.t2m_classes[m]) {
    if (c.prec != prec) continue;
    if (c.prec) launch_T2_class<float>(plan, c, V, K, ch.t2m_items[m], st);
    else launch_T2_class<double>(plan, c, V, K, ch.t2m_items[m], st);
  }
}

// device copies of the near / far lists of mixed set m at its split distance
static int prepare_mixed(exx_plan pl, int m) {
  MixedDev& md = pl->mdev[m];
  if (md.uploaded) return EXX_OK;
  if (!pl->d.Vr32) {
    const size_t np = pl->hp.pair_a.size();
    int64_t nvr = 0;
    for (size_t p = 0; p < np; ++p) {
      const int A = pl->hp.pair_a[p], B = pl->hp.pair_b[p];
      nvr += (int64_t)((pl->hp.na[A] + 15) / 16) * ((pl->hp.na[B] + 3) / 4) * 64;
      if (A != B) nvr += (int64_t)((pl->hp.na[B] + 15) / 16) * ((pl->hp.na[A] + 3) / 4) * 64;
    }
    HIP_TRY(hipMalloc((void**)&pl->d.Vr32, sizeof(float) * std::max<int64_t>(1, nvr)));
    pl->allocs.push_back(pl->d.Vr32);
    HIP_TRY(hipMalloc((void**)&pl->d.Dr32, sizeof(float) * 256 * std::max<size_t>(1, 2 * np)));
    pl->allocs.push_back(pl->d.Dr32);
    pl->dev_bytes += (int64_t)sizeof(float) * (nvr + 512 * (int64_t)np);
  }
  HostPlan& hp = pl->hp;
  MixedSet& ms = hp.mixed[m];
  if (!ms.ready) derive_mixed_lists(hp, m);
  free_mixed(md);
  int rc = 0;
  if ((rc = upload(pl, md.tiles_near, ms.tiles_near, &md))) return rc;
  if ((rc = upload(pl, md.tiles_far, ms.tiles_far, &md))) return rc;
  if ((rc = upload(pl, md.q_near, ms.q_near, &md))) return rc;
  if ((rc = upload(pl, md.x_near, ms.x_near, &md))) return rc;
  if ((rc = upload(pl, md.q_far, ms.q_far, &md))) return rc;
  if ((rc = upload(pl, md.x_far, ms.x_far, &md))) return rc;
  if (hp.chunks.empty()) {
    if ((rc = upload(pl, md.t2_items, ms.t2_items, &md))) return rc;
    pl->chunks[0].t2m_items[m] = md.t2_items;
    pl->chunks[0].t2m_classes[m] = ms.t2_classes;
  } else {
    for (size_t c = 0; c < hp.chunks.size(); ++c) {
      if ((rc = upload(pl, pl->chunks[c].t2m_items[m], ms.chunk_t2_items[c], &md))) return rc;
      pl->chunks[c].t2m_classes[m] = ms.chunk_t2_classes[c];
    }
  }
  md.uploaded = true;
  return EXX_OK;
}

static void launch_final(exx_plan plan, double* K, hipStream_t st) {
  if (plan->hp.periodic) {   // X on the pair pattern only
    launch_pgather(plan, K, st);
    return;
  }
  launch_Y(plan, plan->tune[TUNE_Y], st);
  launch_symreduce(plan, K, st);
}

static int n_chunks(exx_plan plan) { return (int)plan->chunks.size(); }

// The chunk loop of one K build (D masked into Dm, C repacked into T, K zeroed
// before): per chunk E, the V stage, T2 and the final contraction, in this
// order, every part added into K.  m < 0: binary64; else mixed set m.
static void build_chunks(exx_plan plan, const double* V, const double* D, double* K, int m, hipStream_t st) {
  for (int c = 0; c < n_chunks(plan); ++c) {
    set_chunk(plan, c);
    launch_E(plan, st);
    if (c == 0) stage_mark(plan, 2, st);
    if (m >= 0) {
      launch_H_mixed(plan, m, V, D, st);   // marks boundary 3 between its binary64 and binary32 parts
    } else {
      launch_H(plan, V, D, 2.0, H_WRITE, st);
      if (c == 0) stage_mark(plan, 3, st);
    }
    if (c == 0) stage_mark(plan, 4, st);
    launch_T2(plan, V, K, st, m, 0);
    if (c == 0) stage_mark(plan, 5, st);
    if (m >= 0) launch_T2(plan, V, K, st, m, 1);
    if (c == 0) stage_mark(plan, 6, st);
    launch_final(plan, K, st);
  }
  set_chunk(plan, 0);
}

// a call has written the workspace; fp64_build: E and H' are now those of a binary64,
// unscreened, single-chunk build_K of the call's inputs (fp64_spin: of such a build_K_spin)
static void ws_written(exx_plan plan, bool fp64_build, bool fp64_spin = false) {
  ++plan->ws_seq;
  plan->ws_fp64 = fp64_build ? plan->ws_seq : 0;
  plan->ws_fp64_spin = fp64_spin ? plan->ws_seq : 0;
}

// mixed list set of a precision, or -1 for binary64; -2: unknown, -3: reserved
static int precision_set(int precision) {
  switch (precision) {
    case EXX_PREC_FP64: return -1;
    case EXX_PREC_MIXED: return 0;
    case EXX_PREC_FP32: return 1;
    case EXX_PREC_BF16X3: return -3;
    default: return -2;
  }
}

static int check_precision(const char* who, int precision, int& m) {
  m = precision_set(precision);
  if (m == -3) return fail(EXX_EUNSUPPORTED, std::string(who) + ": EXX_PREC_BF16X3 is reserved, not implemented");
  if (m == -2) return fail(EXX_EINVAL, std::string(who) + ": unknown precision");
  return EXX_OK;
}

int build_K(exx_plan plan, const double* C, const double* V, const double* D, int precision,
            double* K, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "build_K: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "build_K: host-only plan");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "build_K: NULL array");
  int m = -1;
  int rc = check_precision("build_K", precision, m);
  if (rc != EXX_OK) return rc;
  if (m >= 0 && (rc = prepare_mixed(plan, m)) != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, hp.d_size);
  launch_dmask(plan, D, plan->d.Dm, st);
  launch_repack(plan, C, st);
  launch_vd_operands(plan, V, D, st, m >= 0);
  const bool screened = plan->scr_eps > 0;
  if (screened) {
    launch_screening(plan, C, V, D, st);
    plan->d.scr = plan->scr_flags;
  }
  stage_mark(plan, 1, st);
  build_chunks(plan, V, D, K, m, st);
  plan->d.scr = nullptr;
  if (screened) plan->scr_done = true;
  ws_written(plan, m < 0 && !screened && n_chunks(plan) == 1);
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
  if (Ex) rc = launch_energy(plan, K, D, Ex, st);
  stage_mark(plan, 8, st);
  return rc;
}

// E and H' workspaces of a second result (build_K_spin, build_K_two_kernels), allocated once
static int second_workspace(exx_plan plan) {
  if (plan->spin_E1) return EXX_OK;
  // E and H' of the second result in the layout of one chunk (the whole plan when unbounded)
  int64_t ne = plan->hp.e_total;
  if (!plan->hp.chunks.empty()) {
    ne = 0;
    for (const ChunkHost& c : plan->hp.chunks) ne = std::max(ne, std::max(c.e_total, c.h_total));
  }
  ne = std::max<int64_t>(1, ne);
  HIP_TRY(hipMalloc((void**)&plan->spin_E1, sizeof(double) * ne));
  plan->allocs.push_back(plan->spin_E1);
  HIP_TRY(hipMalloc((void**)&plan->spin_H1, sizeof(double) * ne));
  plan->allocs.push_back(plan->spin_H1);
  plan->dev_bytes += 2 * (int64_t)sizeof(double) * ne;
  const int64_t ndr = std::max<int64_t>(1, plan->dr_total);
  HIP_TRY(hipMalloc((void**)&plan->spin_Dr1, sizeof(double) * ndr));
  plan->allocs.push_back(plan->spin_Dr1);
  plan->dev_bytes += (int64_t)sizeof(double) * ndr;
  const int64_t nd = std::max<int64_t>(1, plan->hp.d_size);
  HIP_TRY(hipMalloc((void**)&plan->spin_Dm1, sizeof(double) * nd));
  plan->allocs.push_back(plan->spin_Dm1);
  plan->dev_bytes += (int64_t)sizeof(double) * nd;
  HIP_TRY(hipMemset(plan->spin_Dm1, 0, sizeof(double) * nd));
  return EXX_OK;
}

// Collinear spin: E^s = T D^s for both spins, then one V-stage pass for both (F shared), then
// T2 and the final contraction per spin with E and H' pointed at that spin's workspace.
int build_K_spin(exx_plan plan, const double* C, const double* V, const double* D, int precision, double* K,
                 double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "build_K_spin: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "build_K_spin: host-only plan");
  if (!C || !V || !D || !K) return fail(EXX_EINVAL, "build_K_spin: NULL array");
  int m = -1;
  int rc = check_precision("build_K_spin", precision, m);
  if (rc != EXX_OK) return rc;
  if (m >= 0 && (rc = prepare_mixed(plan, m)) != EXX_OK) return rc;
  const HostPlan& hp = plan->hp;
  const int64_t ds = hp.d_size;
  if (m < 0) {
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
  set_chunk(plan, 0);
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, 2 * ds);
  launch_dmask(plan, D, d.Dm, st);
  launch_dmask(plan, D + ds, plan->spin_Dm1, st);
  launch_repack(plan, C, st);
  const bool screened = plan->scr_eps > 0;
  if (screened) {   // one flag per pair for both spins: max|D| over D^0 and D^1
    launch_screening(plan, C, V, D, st, D + ds);
    d.scr = plan->scr_flags;
  }
  if (m < 0) {
    launch_vd_operands(plan, V, D, st);   // V and D^0 operands
    if (!hp.pair_a.empty())
      hipLaunchKernelGGL(k_vdrepack, dim3((unsigned)hp.pair_a.size()), dim3(256), 0, st, nullptr, D + ds,
                         plan->spin_Dr1, plan->d, 0);   // D^1 operands
  }
  stage_mark(plan, 1, st);
  // per chunk of aux atoms (one for an unbounded plan): E^s for both spins, then the rest
  for (int c = 0; c < n_chunks(plan); ++c) {
    set_chunk(plan, c);
    const ChunkDev& ch = cur_chunk(plan);
    launch_rowD_spin(plan, d.Dm, plan->spin_Dm1, plan->spin_E1, rowd_E(plan), ch.n_e, st);
    if (c == 0) stage_mark(plan, 2, st);
    double* const E0 = d.E;
    double* const H0 = d.H;
    if (m >= 0) {
      // mixed / FP32: per spin the V stage, T2 and the final contraction of a mixed build_K,
      // with E and H' pointed at that spin's workspace (F is not shared between the spins)
      for (int s = 0; s < 2; ++s) {
        d.E = s ? plan->spin_E1 : E0;
        d.H = s ? plan->spin_H1 : H0;
        launch_vd_operands(plan, V, D + s * ds, st, true);
        launch_H_mixed(plan, m, V, D + s * ds, st);
        launch_T2(plan, V, K + s * ds, st, m, 0);
        launch_T2(plan, V, K + s * ds, st, m, 1);
        launch_final(plan, K + s * ds, st);
      }
      d.E = E0;
      d.H = H0;
    } else {
      launch_H_lists<double, 2>(plan, V, D,
                                HLists{d.g_tiles + ch.gt_beg, d.gq, d.gx, plan->h_vbase, plan->spin_E1,
                                       plan->spin_H1, plan->spin_Dr1},
                                ch.gt_end - ch.gt_beg, 2.0, H_WRITE, st);
      if (c == 0) {
        stage_mark(plan, 3, st);
        stage_mark(plan, 4, st);
      }
      launch_T2_spin(plan, V, K, st);
      if (c == 0) {
        stage_mark(plan, 5, st);
        stage_mark(plan, 6, st);
      }
      launch_final(plan, K, st);
      d.H = plan->spin_H1;
      launch_final(plan, K + ds, st);
      d.H = H0;
    }
  }
  set_chunk(plan, 0);
  d.scr = nullptr;
  if (screened) plan->scr_done = true;
  ws_written(plan, false, m < 0 && !screened && n_chunks(plan) == 1);
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
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
  int m = -1;
  int rc = check_precision("build_K_two_kernels", precision, m);
  if (rc != EXX_OK) return rc;
  if (m >= 0 && (rc = prepare_mixed(plan, m)) != EXX_OK) return rc;
  const int rcw = second_workspace(plan);
  if (rcw != EXX_OK) return rcw;
  const HostPlan& hp = plan->hp;
  const int64_t ds = hp.d_size;
  hipStream_t st = (hipStream_t)stream;
  DevPlan& d = plan->d;
  set_chunk(plan, 0);
  stage_mark(plan, 0, st);
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, K, 2 * ds);
  launch_dmask(plan, D, d.Dm, st);
  launch_repack(plan, C, st);
  stage_mark(plan, 1, st);
  const double* Va[2] = {V, V2};
  for (int c = 0; c < n_chunks(plan); ++c) {
    set_chunk(plan, c);
    double* const H0 = d.H;
    launch_E(plan, st);
    if (c == 0) stage_mark(plan, 2, st);
    // T2 reads the lane-ordered copy of the V operands that the V stage reads: each Coulomb
    // matrix's operands (binary32 copies too for a mixed build) are written before its own
    // V stage, and its T2 blocks run before the next matrix's operands replace them
    for (int a = 0; a < 2; ++a) {
      d.H = a ? plan->spin_H1 : H0;
      if (plan->scr_eps > 0) {   // each Coulomb matrix screened by its own estimates
        launch_screening(plan, C, Va[a], D, st);
        d.scr = plan->scr_flags;
      }
      launch_vd_operands(plan, Va[a], D, st, m >= 0);
      if (m >= 0) launch_H_mixed(plan, m, Va[a], D, st);
      else launch_H(plan, Va[a], D, 2.0, H_WRITE, st);
      d.H = H0;
      launch_T2(plan, Va[a], K + a * ds, st, m, 0);
      if (m >= 0) launch_T2(plan, Va[a], K + a * ds, st, m, 1);
      d.scr = nullptr;
    }
    if (c == 0) {
      stage_mark(plan, 3, st);
      stage_mark(plan, 4, st);
      stage_mark(plan, 5, st);
      stage_mark(plan, 6, st);
    }
    launch_final(plan, K, st);
    d.H = plan->spin_H1;
    launch_final(plan, K + ds, st);
    d.H = H0;
  }
  set_chunk(plan, 0);
  if (plan->scr_eps > 0) plan->scr_done = true;
  ws_written(plan, false);
  stage_mark(plan, 7, st);
  HIP_TRY(hipGetLastError());
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
  int m = -1;
  int rc0 = check_precision("exx_graph_build", precision, m);
  if (rc0 != EXX_OK) return rc0;
  if (m >= 0 && (rc0 = prepare_mixed(plan, m)) != EXX_OK) return rc0;   // list uploads stay outside the capture
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
  ws_written(plan, false);   // the capture ran nothing
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
  ws_written(plan, false);
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
  int m = -1;
  int rc = check_precision("exx_plan_autotune", precision, m);
  if (rc != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const bool prof = plan->profiling;
  plan->profiling = false;
  // one build fills the workspace the stage kernels read (the last chunk's, for a chunked
  // plan: its lists are the ones timed)
  rc = build_K(plan, C, V, D, precision, K, nullptr, stream);
  if (rc == EXX_OK) HIP_TRY(hipStreamSynchronize(st));
  set_chunk(plan, n_chunks(plan) - 1);
  constexpr int REPS = 3;
  for (int stage = 0; stage < N_TUNE && rc == EXX_OK; ++stage) {
    for (int c = 0; c < kTuneCands[stage] && rc == EXX_OK; ++c) {
      plan->tune[stage] = c;
      float ms = 0.f;
      if (stage == TUNE_E) {
        rc = time_stage(st, REPS, [&] { launch_E(plan, st); }, ms);
      } else if (stage == TUNE_T2) {
        rc = time_stage(st, REPS, [&] {
          launch_T2(plan, V, K, st, m, 0);
          if (m >= 0) launch_T2(plan, V, K, st, m, 1);
        }, ms);
      } else {
        rc = time_stage(st, REPS, [&] { launch_Y(plan, c, st); }, ms);
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
  set_chunk(plan, 0);
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
  MixedSet& ms = plan->hp.mixed[0];
  if (ms.ready && ms.split == r_split) return EXX_OK;
  if (plan->graph_exec) { hipGraphExecDestroy(plan->graph_exec); plan->graph_exec = nullptr; }
  if (plan->graph) { hipGraphDestroy(plan->graph); plan->graph = nullptr; }
  ms.split = r_split;
  ms.ready = false;
  derive_mixed_lists(plan->hp, 0);
  if (plan->host_only) return EXX_OK;
  HIP_TRY(hipDeviceSynchronize());   // lists of an earlier split may still be in use
  plan->mdev[0].uploaded = false;
  return prepare_mixed(plan, 0);
}

int exx_block_norms(exx_plan plan, const double* C, const double* V, const double* D, double* norms,
                    void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_block_norms: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_block_norms: host-only plan");
  if (!C || !V || !D || !norms) return fail(EXX_EINVAL, "exx_block_norms: NULL array");
  const unsigned np = (unsigned)plan->hp.pair_a.size();
  if (np)
    hipLaunchKernelGGL(k_block_norms, dim3(np), dim3(256), 0, (hipStream_t)stream, C, V, D, plan->d, norms,
                       (const double*)nullptr);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exx_set_screening(exx_plan plan, double eps) {
  if (!plan) return fail(EXX_EINVAL, "exx_set_screening: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_set_screening: host-only plan");
  if (!(eps >= 0.0) || eps > 1e300) return fail(EXX_EINVAL, "exx_set_screening: eps must be finite and >= 0");
  if (eps > 0 && !plan->scr_nrm) {
    const int64_t np = (int64_t)plan->hp.pair_a.size(), na = plan->hp.n_atoms;
    HIP_TRY(hipMalloc((void**)&plan->scr_nrm, sizeof(double) * std::max<int64_t>(1, 3 * np + 3 * na)));
    plan->allocs.push_back(plan->scr_nrm);
    HIP_TRY(hipMalloc((void**)&plan->scr_flags, std::max<int64_t>(1, np)));
    plan->allocs.push_back(plan->scr_flags);
    plan->dev_bytes += (int64_t)sizeof(double) * (3 * np + 3 * na) + np;
  }
  plan->scr_eps = eps;
  return EXX_OK;
}

int exx_screened_pairs(exx_plan plan, uint8_t* flags, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_screened_pairs: NULL plan");
  if (!flags) return fail(EXX_EINVAL, "exx_screened_pairs: NULL array");
  if (!plan->scr_done) return fail(EXX_ESTATE, "exx_screened_pairs: no screened build has been issued");
  const size_t np = plan->hp.pair_a.size();
  if (np) HIP_TRY(hipMemcpyAsync(flags, plan->scr_flags, np, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return EXX_OK;
}

static int check_kpts(const char* who, int n_k, const double* k_frac) {
  if (n_k <= 0 || !k_frac) return fail(EXX_EINVAL, std::string(who) + ": need n_k > 0 and k-points");
  for (int i = 0; i < 3 * n_k; ++i)
    if (!(std::fabs(k_frac[i]) <= 1e6)) return fail(EXX_EINVAL, std::string(who) + ": k-points must be finite");
  return EXX_OK;
}

static KPts kpt_chunk(const double* k_frac, int k0, int n_k) {
  KPts kp{};
  kp.n = std::min(KPT_MAX, n_k - k0);
  for (int q = 0; q < kp.n; ++q)
    for (int x = 0; x < 3; ++x) kp.k[q][x] = k_frac[3 * (k0 + q) + x];
  return kp;
}

int exx_bloch_sum(exx_plan plan, const double* X, int n_k, const double* k_frac, double* Kk, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_bloch_sum: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_bloch_sum: host-only plan");
  if (!X || !Kk) return fail(EXX_EINVAL, "exx_bloch_sum: NULL array");
  int rc = check_kpts("exx_bloch_sum", n_k, k_frac);
  if (rc != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  const unsigned np = (unsigned)hp.pair_a.size();
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, Kk, 2 * (int64_t)n_k * hp.d_size);
  for (int k0 = 0; k0 < n_k && np; k0 += KPT_MAX)
    hipLaunchKernelGGL(k_bloch, dim3(np), dim3(256), 0, st, X, Kk, plan->d, kpt_chunk(k_frac, k0, n_k), k0);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exx_density_from_k(exx_plan plan, int n_k, const double* k_frac, const double* Dk, double* D, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_density_from_k: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_density_from_k: host-only plan");
  if (!Dk || !D) return fail(EXX_EINVAL, "exx_density_from_k: NULL array");
  int rc = check_kpts("exx_density_from_k", n_k, k_frac);
  if (rc != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  const unsigned np = (unsigned)hp.pair_a.size();
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, D, hp.d_size);
  for (int k0 = 0; k0 < n_k && np; k0 += KPT_MAX)
    hipLaunchKernelGGL(k_density_k, dim3(np), dim3(256), 0, st, Dk, D, plan->d, kpt_chunk(k_frac, k0, n_k), k0);
  if (np) hipLaunchKernelGGL(k_scale_pairs, dim3(np), dim3(256), 0, st, D, plan->d, 1.0 / n_k);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exx_strain_derivative(exx_plan plan, const double* C, const double* V, const double* dC, const double* dV,
                          double c_decay, double v_2s2, double* dEde, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exx_strain_derivative: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exx_strain_derivative: host-only plan");
  if (!C || !V || !dC || !dV || !dEde) return fail(EXX_EINVAL, "exx_strain_derivative: NULL array");
  if (!(c_decay > 0) || !(v_2s2 > 0)) return fail(EXX_EINVAL, "exx_strain_derivative: decay lengths must be positive");
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  if (!plan->strain_part) {
    HIP_TRY(hipMalloc((void**)&plan->strain_part, sizeof(double) * 9 * std::max(1, hp.n_atoms)));
    plan->allocs.push_back(plan->strain_part);
  }
  const unsigned np = (unsigned)hp.pair_a.size();
  if (np) {
    hipLaunchKernelGGL(k_block_dot, dim3(np), dim3(256), 0, st, dC, C, d.c_off, d.sC);
    hipLaunchKernelGGL(k_block_dot, dim3(np), dim3(256), 0, st, dV, V, d.v_off, d.sV);
  }
  hipLaunchKernelGGL(k_strain_part, dim3((hp.n_atoms + 127) / 128), dim3(128), 0, st, d.pos, d.sC, d.sV,
                     plan->strain_part, d, c_decay, v_2s2);
  hipLaunchKernelGGL(k_strain_sum, dim3(1), dim3(256), 0, st, plan->strain_part, hp.n_atoms, dEde);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exchange_energy(exx_plan plan, const double* K, const double* D, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exchange_energy: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exchange_energy: host-only plan");
  if (!K || !D || !Ex) return fail(EXX_EINVAL, "exchange_energy: NULL array");
  return launch_energy(plan, K, D, Ex, (hipStream_t)stream);
}

int exchange_energy_noalloc(exx_plan plan, const double* K, const double* D, double* Ex, void* stream) {
  if (!plan) return fail(EXX_EINVAL, "exchange_energy_noalloc: NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, "exchange_energy_noalloc: host-only plan");
  if (!K || !D || !Ex) return fail(EXX_EINVAL, "exchange_energy_noalloc: NULL array");
  const size_t nch = plan->hp.en_sys.size();
  if (nch > (size_t)EXX_NOALLOC_MAX_CHUNKS)
    return fail(EXX_EINVAL, "exchange_energy_noalloc: " + std::to_string(nch) + " energy chunks exceed the static "
                            "buffer of " + std::to_string(EXX_NOALLOC_MAX_CHUNKS));
  double* part = plan->device >= 0 && plan->device < MAX_DEVICES ? g_scratch_dev[plan->device] : nullptr;
  if (!part) return fail(EXX_ESTATE, "exchange_energy_noalloc: static buffer not set up for the plan's device");
  return launch_energy(plan, K, D, Ex, (hipStream_t)stream, 1, part);
}

// dE/dC and dE/dV of one chunk: E, the V stage with the G term taken once, the
// gradient product G_P = H_P D and the dV pair blocks.  (Launches only.)
static void backward_chunk(exx_plan plan, const double* V, const double* D, double* dVb, const double* gE,
                           bool needC, bool needV, bool h_ready, hipStream_t st) {
  if (!h_ready) launch_E(plan, st);
  if (needC) {
    if (!h_ready) launch_H(plan, V, D, 1.0, H_WRITE, st);
    const ChunkDev& ch = cur_chunk(plan);
    launch_rowD(plan, plan->d.Dm, rowd_GD(plan), ch.gd_end - ch.gd_beg, st);
  }
  if (needV) launch_dV(plan, V, D, dVb, gE, st);
}

// One density matrix's part of the backward pass: dD (if asked) from K or a rebuild, and the
// dC, dV blocks of sum_s gE[s] E_x[s] written (not added) into dCb, dVb.  C is repacked
// into T when repack is set (it does not depend on D).  (Launches only.)
// reuse: E and H' in the workspace are those of a binary64 build_K of these inputs (single
// chunk); they are taken instead of recomputed, with the G term brought back to once.
static void backward_density(exx_plan plan, const double* C, const double* V, const double* D, const double* K,
                             const double* gE, double* dCb, double* dVb, double* dD, bool needC, bool needV,
                             bool repack, hipStream_t st, bool reuse = false) {
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  const dim3 gsys(256, hp.n_sys);
  launch_dmask(plan, D, d.Dm, st);
  if (repack) launch_repack(plan, C, st);
  launch_vd_operands(plan, V, D, st);
  bool h_ready = false;   // E and H (G taken once) of the only chunk already in place
  if (dD && K) {
    // dE/dD = -1/2 gE K from the caller's K
    hipLaunchKernelGGL(k_scaled_copy_sys, gsys, dim3(256), 0, st, dD, K, gE, d, -0.5);
  } else if (dD) {
    // dE/dD = -1/2 gE K: the forward build into dD, then scaled
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, dD, hp.d_size);
    if (n_chunks(plan) == 1) {
      set_chunk(plan, 0);
      launch_E(plan, st);
      launch_H(plan, V, D, 2.0, H_WRITE, st);
      launch_T2(plan, V, dD, st);
      launch_final(plan, dD, st);
      if (needC) launch_H(plan, V, D, -1.0, H_G_ADD, st);   // G term taken once
      h_ready = true;
    } else {
      const bool prof = plan->profiling;
      plan->profiling = false;
      build_chunks(plan, V, D, dD, -1, st);
      plan->profiling = prof;
    }
    hipLaunchKernelGGL(k_scaled_copy_sys, gsys, dim3(256), 0, st, dD, dD, gE, d, -0.5);
  }
  if (reuse && !h_ready && (needC || needV)) {
    // the build wrote H' with the G term twice (factor 2); the gradient takes it once
    if (needC) launch_H(plan, V, D, -1.0, H_G_ADD, st);
    h_ready = true;
  }
  if (needC || needV) {
    for (int c = 0; c < n_chunks(plan); ++c) {
      set_chunk(plan, c);
      backward_chunk(plan, V, D, dVb, gE, needC, needV, h_ready && c == 0, st);
    }
    set_chunk(plan, 0);
  }
  if (needC) hipLaunchKernelGGL(k_unrepack, dim3(hp.nbr_ptr[hp.n_atoms]), dim3(256), 0, st, d.GD, dCb, d, gE, -1.0);
}

// forces from the summed dC, dV blocks (per-pair <gradient, block> sums, then per atom)
static void launch_forces(exx_plan plan, const double* C, const double* V, const double* dCb, const double* dVb,
                          double* forces, double c_decay, double v_2s2, hipStream_t st) {
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  hipLaunchKernelGGL(k_block_dot, dim3((int)hp.pair_a.size()), dim3(256), 0, st, dCb, C, d.c_off, d.sC);
  hipLaunchKernelGGL(k_block_dot, dim3((int)hp.pair_a.size()), dim3(256), 0, st, dVb, V, d.v_off, d.sV);
  hipLaunchKernelGGL(k_forces, dim3((hp.n_atoms + 127) / 128), dim3(128), 0, st, d.pos, d.sC, d.sV, forces, d,
                     c_decay, v_2s2);
}

static int backward_checks(exx_plan plan, const char* who, const double* C, const double* V, const double* D,
                           const double* gE, int precision, const double* forces, double c_decay, double v_2s2) {
  const std::string w(who);
  if (!plan) return fail(EXX_EINVAL, w + ": NULL plan");
  if (plan->host_only) return fail(EXX_ESTATE, w + ": host-only plan");
  if (!C || !V || !D || !gE) return fail(EXX_EINVAL, w + ": NULL input array");
  if (precision == EXX_PREC_MIXED || precision == EXX_PREC_FP32 || precision == EXX_PREC_BF16X3)
    return fail(EXX_EUNSUPPORTED, w + ": only the binary64 backward is implemented");
  if (precision != EXX_PREC_FP64) return fail(EXX_EINVAL, w + ": unknown precision");
  if (forces && (!(c_decay > 0) || !(v_2s2 > 0))) return fail(EXX_EINVAL, w + ": decay lengths must be positive");
  return EXX_OK;
}

// plan-owned gradient buffers of size n (allocated on first use)
static int scratch_buf(exx_plan plan, double*& buf, int64_t n) {
  if (buf) return EXX_OK;
  HIP_TRY(hipMalloc((void**)&buf, sizeof(double) * std::max<int64_t>(1, n)));
  plan->allocs.push_back(buf);
  return EXX_OK;
}

static int backward_one(exx_plan plan, const char* who, bool reuse, const double* C, const double* V,
                        const double* D, const double* K, const double* gE, int precision, double* dC, double* dV,
                        double* dD, double* forces, double c_decay, double v_2s2, void* stream) {
  int rc = backward_checks(plan, who, C, V, D, gE, precision, forces, c_decay, v_2s2);
  if (rc != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  const bool needC = dC || forces, needV = dV || forces;
  if (needC && !dC && (rc = scratch_buf(plan, plan->dC_scratch, hp.c_off.back())) != EXX_OK) return rc;
  if (needV && !dV && (rc = scratch_buf(plan, plan->dV_scratch, hp.v_off.back())) != EXX_OK) return rc;
  double* dCb = dC ? dC : plan->dC_scratch;
  double* dVb = dV ? dV : plan->dV_scratch;
  backward_density(plan, C, V, D, K, gE, dCb, dVb, dD, needC, needV, true, st, reuse);
  if (needC || needV || (dD && !K)) ws_written(plan, false);
  if (forces) launch_forces(plan, C, V, dCb, dVb, forces, c_decay, v_2s2, st);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exchange_backward(exx_plan plan, const double* C, const double* V, const double* D, const double* K,
                      const double* gE, int precision, double* dC, double* dV, double* dD, double* forces,
                      double c_decay, double v_2s2, void* stream) {
  return backward_one(plan, "exchange_backward", false, C, V, D, K, gE, precision, dC, dV, dD, forces, c_decay,
                      v_2s2, stream);
}

int exx_plan_build_id(exx_plan plan, uint64_t* id) {
  if (!plan || !id) return fail(EXX_EINVAL, "exx_plan_build_id: NULL argument");
  *id = plan->ws_seq;
  return EXX_OK;
}

int exchange_backward_reuse(exx_plan plan, uint64_t build_id, const double* C, const double* V, const double* D,
                            const double* K, const double* gE, int precision, double* dC, double* dV, double* dD,
                            double* forces, double c_decay, double v_2s2, int* reused, void* stream) {
  const bool reuse = plan && build_id != 0 && build_id == plan->ws_seq && build_id == plan->ws_fp64 &&
                     n_chunks(plan) == 1;
  const int rc = backward_one(plan, "exchange_backward_reuse", reuse, C, V, D, K, gE, precision, dC, dV, dD, forces,
                              c_decay, v_2s2, stream);
  if (reused) *reused = (rc == EXX_OK && reuse) ? 1 : 0;
  return rc;
}

// y += x over n doubles
__global__ void k_add(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// gE2 = a gE over n values
__global__ void k_scale_vec(double* __restrict__ y, const double* __restrict__ x, double a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// reuse: E^s and H'^s in the workspace are those of a binary64 build_K_spin of these inputs
// (single chunk): taken instead of recomputed, the G terms brought back to once.
static int backward_spin(exx_plan plan, const char* who, bool reuse, const double* C, const double* V,
                         const double* D, const double* K, const double* gE, int precision, double* dC, double* dV,
                         double* dD, double* forces, double c_decay, double v_2s2, void* stream) {
  int rc = backward_checks(plan, who, C, V, D, gE, precision, forces, c_decay, v_2s2);
  if (rc != EXX_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const HostPlan& hp = plan->hp;
  DevPlan& d = plan->d;
  const int64_t ds = hp.d_size, nc = hp.c_off.back(), nv = hp.v_off.back();
  const bool needC = dC || forces, needV = dV || forces;
  if (needC && !dC && (rc = scratch_buf(plan, plan->dC_scratch, nc)) != EXX_OK) return rc;
  if (needV && !dV && (rc = scratch_buf(plan, plan->dV_scratch, nv)) != EXX_OK) return rc;
  if (needC && (rc = scratch_buf(plan, plan->dC_spin1, nc)) != EXX_OK) return rc;
  if (needC && (rc = scratch_buf(plan, plan->spin_GD1, hp.t_total)) != EXX_OK) return rc;
  if (needV && (rc = scratch_buf(plan, plan->dV_spin1, nv)) != EXX_OK) return rc;
  if ((rc = scratch_buf(plan, plan->gE_spin, hp.n_sys)) != EXX_OK) return rc;
  if ((rc = second_workspace(plan)) != EXX_OK) return rc;
  double* dCb = dC ? dC : plan->dC_scratch;
  double* dVb = dV ? dV : plan->dV_scratch;
  // E_x = -1/2 sum_s K^s D^s is twice the one-density energy of each spin: every spin's part
  // is the one-density backward with upstream 2 gE
  hipLaunchKernelGGL(k_scale_vec, dim3((hp.n_sys + 255) / 256), dim3(256), 0, st, plan->gE_spin, gE, 2.0, hp.n_sys);
  const dim3 gsys(256, hp.n_sys);
  if (dD) {
    // dE/dD^s = -gE K^s: from the caller's K, or from a (never screened) spin build into dD
    if (!K) {
      const double eps = plan->scr_eps;
      const bool prof = plan->profiling;
      plan->scr_eps = 0;
      plan->profiling = false;
      rc = build_K_spin(plan, C, V, D, EXX_PREC_FP64, dD, nullptr, stream);
      plan->scr_eps = eps;
      plan->profiling = prof;
      if (rc != EXX_OK) return rc;
    }
    for (int s = 0; s < 2; ++s)
      hipLaunchKernelGGL(k_scaled_copy_sys, gsys, dim3(256), 0, st, dD + s * ds, (K ? K : dD) + s * ds,
                         plan->gE_spin, d, -0.5);
  }
  if (needC || needV) {
    // both spins in one pass per chunk: E^s together, the V stage with F shared (G term taken
    // once), then the gradient products and dV blocks per spin
    launch_dmask(plan, D, d.Dm, st);
    launch_dmask(plan, D + ds, plan->spin_Dm1, st);
    launch_repack(plan, C, st);
    launch_vd_operands(plan, V, D, st);
    if (!hp.pair_a.empty())
      hipLaunchKernelGGL(k_vdrepack, dim3((unsigned)hp.pair_a.size()), dim3(256), 0, st, nullptr, D + ds,
                         plan->spin_Dr1, d, 0);
    for (int c = 0; c < n_chunks(plan); ++c) {
      set_chunk(plan, c);
      const ChunkDev& ch = cur_chunk(plan);
      if (!reuse) launch_rowD_spin(plan, d.Dm, plan->spin_Dm1, plan->spin_E1, rowd_E(plan), ch.n_e, st);
      if (needC) {
        // recomputed with the G term once, or the build's (G twice) with one G-only pass of factor -1
        launch_H_lists<double, 2>(plan, V, D,
                                  HLists{d.g_tiles + ch.gt_beg, d.gq, d.gx, plan->h_vbase, plan->spin_E1,
                                         plan->spin_H1, plan->spin_Dr1},
                                  ch.gt_end - ch.gt_beg, reuse ? -1.0 : 1.0, reuse ? H_G_ADD : H_WRITE, st);
        launch_rowD(plan, d.Dm, rowd_GD(plan), ch.gd_end - ch.gd_beg, st);
        double* const H0 = d.H;
        double* const GD0 = d.GD;
        d.H = plan->spin_H1;
        d.GD = plan->spin_GD1;
        launch_rowD(plan, plan->spin_Dm1, rowd_GD(plan), ch.gd_end - ch.gd_beg, st);
        d.H = H0;
        d.GD = GD0;
      }
      if (needV) {
        launch_dV(plan, V, D, dVb, plan->gE_spin, st);
        double* const E0 = d.E;
        d.E = plan->spin_E1;
        launch_dV(plan, V, D + ds, plan->dV_spin1, plan->gE_spin, st);
        d.E = E0;
      }
    }
    set_chunk(plan, 0);
    if (needC) {
      const unsigned ne = (unsigned)hp.nbr_ptr[hp.n_atoms];
      hipLaunchKernelGGL(k_unrepack, dim3(ne), dim3(256), 0, st, d.GD, dCb, d, plan->gE_spin, -1.0);
      hipLaunchKernelGGL(k_unrepack, dim3(ne), dim3(256), 0, st, plan->spin_GD1, plan->dC_spin1, d, plan->gE_spin,
                         -1.0);
      hipLaunchKernelGGL(k_add, dim3(2048), dim3(256), 0, st, dCb, plan->dC_spin1, nc);
    }
    if (needV) hipLaunchKernelGGL(k_add, dim3(2048), dim3(256), 0, st, dVb, plan->dV_spin1, nv);
    ws_written(plan, false);
  }
  if (forces) launch_forces(plan, C, V, dCb, dVb, forces, c_decay, v_2s2, st);
  HIP_TRY(hipGetLastError());
  return EXX_OK;
}

int exchange_backward_spin(exx_plan plan, const double* C, const double* V, const double* D, const double* K,
                           const double* gE, int precision, double* dC, double* dV, double* dD, double* forces,
                           double c_decay, double v_2s2, void* stream) {
  return backward_spin(plan, "exchange_backward_spin", false, C, V, D, K, gE, precision, dC, dV, dD, forces, c_decay,
                       v_2s2, stream);
}

int exchange_backward_spin_reuse(exx_plan plan, uint64_t build_id, const double* C, const double* V,
                                 const double* D, const double* K, const double* gE, int precision, double* dC,
                                 double* dV, double* dD, double* forces, double c_decay, double v_2s2, int* reused,
                                 void* stream) {
  const bool reuse = plan && build_id != 0 && build_id == plan->ws_seq && build_id == plan->ws_fp64_spin &&
                     n_chunks(plan) == 1;
  const int rc = backward_spin(plan, "exchange_backward_spin_reuse", reuse, C, V, D, K, gE, precision, dC, dV, dD,
                               forces, c_decay, v_2s2, stream);
  if (reused) *reused = (rc == EXX_OK && reuse) ? 1 : 0;
  return rc;
}

}  // extern "C"
