// Shared declarations of the libexx device translation units (not part of the ABI).
//
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
#pragma once
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

// message of the last failure on the calling thread (exx_last_error)
extern thread_local std::string g_err;

static inline int fail(int code, const std::string& msg) {
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
  int64_t *t_off, *e_off, *h_off;   // offsets of T_P, E_P and H'_P (those of the current chunk)
  EItem* e_items;
  int *ct_run_ptr, *ct_klen;
  uint8_t* ct_kflag;
  int64_t* ct_kflag_off;
  Run* runs;
  EItem* gd_items;
  int *gd_run_ptr, *gd_klen;
  uint8_t* gd_kflag;
  int64_t* gd_kflag_off;
  Run* gd_runs;
  double* pos;
  int *grp_first, *grp_unit_ptr, *grp_col_ptr, *grp_cols;
  Unit* grp_units;
  GTile* g_tiles;
  Slot4 *gq, *gx;
  int* t2_items;
  int* t2col;           // E_P column of every T_Q column of a T2 pair (HostPlan::t2col)
  int64_t* t2col_off;
  int* dv_items;
  FItem* f_items;
  int* f_plist;
  int *en_sys, *en_pbeg, *en_pend;
  YTile* y_tiles;
  int64_t* y_off;
  double *T, *E, *H, *Y, *GD, *sC, *sV, *epart;
  // D restricted to the screened pair blocks (zero elsewhere), refreshed from the
  // caller's D before every contraction that reads D beyond pair blocks
  double* Dm;
  // The V-stage operands in MFMA lane order, rebuilt from V and D before every V stage:
  // per canonical pair p and orientation o (0: P = pair_a, Q = pair_b; 1: swapped) at
  // Vr + vr_off[2 p + o], [16-wide aux tile t of P][4-wide aux step q of Q][lane L] =
  // V_PQ[16 t + L % 16][4 q + L / 16], and at Dr + dr_off[2 p + o], [basis step q of Q][lane L] =
  // D_PQ[L % 16][L / 16 + 4 q] (zero outside the blocks).  Each MFMA operand is then one
  // coalesced 512-byte row instead of a gather over 16 rows of V or D.
  int64_t *vr_off, *dr_off;
  double *Vr, *Dr;
  // periodic plans (HostPlan): image codes and image-keyed column maps
  int periodic;
  int *pimg, *col2img, *col1img, *atom_of_col, *grp_colimg, *grp_cmap;
  double* nbr_sep;      // periodic: R_A - (R_J + image shift) per neighbour entry
  int64_t* dvcol_off;   // dV column maps (HostPlan::dvcol)
  int *dvcol, *dv_cp, *dv_cq;
  int *pg_beg, *pg_mid, *pg_end;
  PGEnt* pg_ent;
  PTile* pt_tiles;
  PTEnt* pt_ent;
  int* pg_pairs;
  // binary32 copies for the far pair terms of a mixed build: Vr32 in the layout of Vr; Dr32 at
  // (2 p + o) * 256, [k-step q < 4][lane L] = D_PQ[L % 16][4 (L / 16) + q] (the binary32 MFMA
  // accumulator puts rows 4 (L / 16) + v in lane L, so its D chain runs four k-steps)
  float *Vr32, *Dr32;
  // maximum-norm screening of a build_K (exx_set_screening): per canonical pair 1 where every
  // product through its V block is skipped; null when the build is not screened
  const uint8_t* scr;
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

// Device lists of one chunk of aux atoms (the whole plan when it is not
// workspace-bounded): pointers into device memory and host copies of the
// class tables the launchers loop over.
struct ChunkDev {
  EItem* e_items = nullptr;
  int n_e = 0;
  int gt_beg = 0, gt_end = 0, y_beg = 0, y_end = 0, gd_beg = 0, gd_end = 0;
  int* t2_items = nullptr;
  std::vector<T2Class> t2_classes;
  int* dv_items = nullptr;
  std::vector<DVClass> dv_classes;
  FItem* f_items = nullptr;
  int n_f = 0;
  int* f_plist = nullptr;
  int64_t *e_off = nullptr, *h_off = nullptr, *y_off = nullptr;
  int* t2m_items[2] = {nullptr, nullptr};   // per mixed set
  std::vector<T2Class> t2m_classes[2];
  int64_t h_base = 0, y_base = 0;           // H' and Y within the intermediate buffer (E at 0)
  // periodic plans: pattern tiles (classes on the host) and the per-pair gather
  PTile* pt_tiles = nullptr;
  PTEnt* pt_ent = nullptr;
  std::vector<PTClass> pt_classes;
  int *pg_beg = nullptr, *pg_mid = nullptr, *pg_end = nullptr, *pg_pairs = nullptr;
  PGEnt* pg_ent = nullptr;
  int n_pg = 0;
};

// Device copies of one mixed-precision list set (HostPlan::mixed).
struct MixedDev {
  GTile *tiles_near = nullptr, *tiles_far = nullptr;
  Slot4 *q_near = nullptr, *x_near = nullptr, *q_far = nullptr, *x_far = nullptr;
  int* t2_items = nullptr;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  bool uploaded = false;
};

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
  int h_vbase = 0;                  // elements of the T_Q tile k_H stages in LDS
  int h_smax_t2 = 1;                // largest n_aux * n_basis (T2 staging)
  int lds_max = 0;                  // LDS bytes a workgroup may use on the plan's device
  MixedDev mdev[2];                 // device copies of hp.mixed[0], hp.mixed[1]
  hipGraph_t graph = nullptr;       // captured build_K (exx_graph_build)
  hipGraphExec_t graph_exec = nullptr;
  double* dC_scratch = nullptr;     // gradient buffers used when the caller passes NULL
  double* dV_scratch = nullptr;
  double* dC_spin1 = nullptr;       // the second spin's dC, dV (exchange_backward_spin), and 2 gE
  double* dV_spin1 = nullptr;
  double* gE_spin = nullptr;
  double* strain_part = nullptr;    // per atom partial strain derivatives (9 each), on first use
  double* spin_E1 = nullptr;        // E and H' of the second spin (build_K_spin), allocated on first use
  double* spin_H1 = nullptr;
  double* spin_Dr1 = nullptr;       // lane-ordered D operands of the second spin
  double* spin_Dm1 = nullptr;       // pair-block copy of the second spin's D
  double* spin_GD1 = nullptr;       // the second spin's gradient product (exchange_backward_spin)
  int64_t dr_total = 0;             // doubles of the lane-ordered D operands (DevPlan::Dr)
  // chunks of aux atoms (one for an unbounded plan) and the one the launchers use
  std::vector<ChunkDev> chunks;
  int cur = 0;
  double* W = nullptr;              // the E, H' and Y workspace of the largest chunk
  GTile* g_tiles_all = nullptr;     // global (all-chunk) device lists the chunk ranges index
  YTile* y_tiles_all = nullptr;
  EItem* gd_items_all = nullptr;
  // maximum-norm screening: threshold (0: off); per pair max|C|, max|V|, max|D| (3 doubles),
  // then per atom tau, rho, sigma (n_atoms each); the flags of the last screened build
  double scr_eps = 0;
  double* scr_nrm = nullptr;
  uint8_t* scr_flags = nullptr;
  bool scr_done = false;
  // workspace generations: ws_seq counts the calls that write E and H'; ws_fp64 is the
  // generation whose E and H' are those of a binary64, unscreened, single-chunk build_K
  // (0: none), which exchange_backward_reuse may take instead of recomputing them
  uint64_t ws_seq = 0;
  uint64_t ws_fp64 = 0;
  uint64_t ws_fp64_spin = 0;   // the same for a binary64 build_K_spin (E, H' of both spins)
};

// Point the device plan and the launchers at chunk c.
void set_chunk(exx_plan plan, int c);

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
  // periodic plans (else nullptr): the image code of every output column; a D element
  // between a k-row atom J at image m (that of its run) and the column's atom L at image b
  // is used only if n_JL = b - m (everything else is beyond the cutoff)
  const int* ocolimg;
  // per column tile: one byte per 16 k rows, bit q set unless D is structurally zero on
  // those rows and tile columns 16q.. (the MFMAs of an all-zero block are skipped)
  const uint8_t* kflag;
  const int64_t* kflag_off;
};

// Batched GEMM: 64 x 64 output tile per workgroup of four wavefronts (32 x 32
// each), k in chunks staged through one LDS stage, the next chunk loaded into
// registers meanwhile.  The k index
// runs over the basis functions of the input atoms listed for the tile's
// column tile (runs of consecutive atoms: column lcol.. of A, row grow.. of D).
constexpr int ET = 64, EPITCH = ET + 4;

// V_PQ[mu][nu] (mu on P, nu on Q) from the canonical V block of pair p.
__device__ __forceinline__ double v_elem(const double* Vp, int P, int Q, int aP, int aQ, int mu, int nu) {
  return (P <= Q) ? Vp[mu * aQ + nu] : Vp[nu * aP + mu];
}

// V stage (k_H)
constexpr int LDS_PITCH = H_COLS + 1;   // doubles per staged row (one pad column: no bank conflicts)
constexpr int HQ_CHUNK = 64;            // Q-list entries whose metadata sits in LDS at once
constexpr int H_WAVES = 4;
constexpr int H_CPW = H_COLS / H_WAVES;

// Task lists of one k_H launch: tiles and their Q- and X-lists.
struct HLists {
  const GTile* tiles;
  const Slot4 *gq, *gx;
  int v_base;             // elements of the staged T_Q tile (cleared before the Q loop)
  // second density matrix (collinear spin): its E and H' workspaces and its lane-ordered
  // D operands
  const double* E1;
  double* H1;
  const double* Dr1;
};

// mode: H_WRITE stores H' = (Q part + G part); H_ADD adds both parts to H';
// H_G_ADD adds the G part only.
enum { H_WRITE = 0, H_ADD = 1, H_G_ADD = 2 };

// T2 pair kernel
constexpr int T2_COLS = 8;               // column chunk of the backward pair kernel
constexpr int T2_PITCH = T2_COLS + 1;

// backward pair kernel (dV)
constexpr int DV_WAVES = 8, DV_COLS = 8, DV_PITCH = DV_COLS + 1, DV_RSTEP = 64 * DV_WAVES / DV_COLS;

// kernel launchers (each defined in the translation unit of its kernels)
void launch_rowD(exx_plan plan, const double* D, const RowD& r, int n, hipStream_t st);
void launch_rowD_spin(exx_plan plan, const double* D, const double* D1, double* O1, const RowD& r, int n,
                      hipStream_t st);
void launch_Y(exx_plan plan, int choice, hipStream_t st);
void launch_symreduce(exx_plan plan, double* K, hipStream_t st);
void launch_pgather(exx_plan plan, double* K, hipStream_t st);
template <typename R, int NSP = 1>
void launch_H_lists(exx_plan plan, const double* V, const double* D, const HLists& hl, int n, double gscale,
                    int mode, hipStream_t st);
template <typename R, int NSP = 1>
void launch_T2_class(exx_plan plan, const T2Class& c, const double* V, double* K, const int* items,
                     hipStream_t st);
void launch_dV(exx_plan plan, const double* V, const double* D, double* dV, const double* gE, hipStream_t st);

