/*
 * exx.h -- C ABI of the MI355X RI-LVL exact-exchange library (libexx.so).
 *
 * The library evaluates the real-space exchange matrix of the localized
 * resolution-of-identity method (Kokott et al., Sec. "Description of the
 * real-space formalism", Eq. realspace_exchange, with the RI-LVL pair
 * restriction C^mu_ij = 0 unless the auxiliary function mu sits on the atom of
 * i or j), for clusters (lattice vector R = 0 only):
 *
 *     K_ik = sum_{j,l} sum_{mu,nu} C^mu_ij V_{mu nu} C^nu_kl D_jl
 *     E_x  = -1/4 sum_{i,k} K_ik D_ik
 *
 * and the derivatives of E_x, and for periodic systems (see "Periodic systems"
 * below).  All floating-point arrays are IEEE binary64.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Atoms carry a species s; species s has n_basis[s] basis and n_aux[s]
 * auxiliary functions.  Basis functions are numbered atom by atom inside each
 * system (a batch holds several independent systems / clusters).
 *
 * Screening: atoms A, B form a pair when (dx*dx + dy*dy) + dz*dz <= r_cut^2
 * (float64, no fused multiply-add), dx = x_A - x_B.  One cutoff is used for
 * the blocks of C, V and D (RI-LVL pair restriction for C, distance-screened
 * V, and the density-matrix pattern).  Pairs never cross systems.
 *
 * Canonical pairs are (A, B) with A <= B, in lexicographic order; their
 * storage offsets are returned by exx_pair_layout().
 *
 *   C (device, read-only): for pair (A, B), A < B, a block
 *       [n_aux(A) + n_aux(B)][n_basis(A)][n_basis(B)]; rows m < n_aux(A) hold
 *       C^mu_ij for mu = m-th aux of A, i on A, j on B; rows m >= n_aux(A)
 *       hold mu = (m - n_aux(A))-th aux of B.  C^mu_ji = C^mu_ij is implied.
 *       On-site pair (A, A): block [n_aux(A)][n_basis(A)][n_basis(A)] stored
 *       in full; the library uses (C_ij + C_ji)/2, so it should be symmetric.
 *   V (device, read-only): pair (A, B), a block [n_aux(A)][n_aux(B)] holding
 *       V_{mu nu} = V_{nu mu}, mu on A, nu on B.  On-site blocks in full.
 *   D, K (device): dense, row-major, symmetric, one n_s x n_s block per
 *       system s (n_s = sum of n_basis over its atoms), blocks concatenated
 *       in system order.  D entries of atom pairs beyond r_cut are ignored
 *       (treated as zero): the library contracts a copy of D restricted to the
 *       screened pair blocks, and E_x sums over those blocks only.
 *
 * Periodic systems (exx_system.lattice != NULL; one system per plan): every
 * atom A of the home cell has images A + n.L in all cells n.  The cutoff must
 * be below half the distance between opposite cell faces, so an atom pair
 * (A, B) has at most one image n_AB of B within r_cut of A: the pair is screened
 * as ((x_B + s_x) - x_A)^2 + ... (summed (dx*dx + dy*dy) + dz*dz, binary64,
 * s = (n0 a0 + n1 a1) + n2 a2 per component, n in {-1, 0, 1}^3) and its C, V and
 * D blocks are those of B at that image: C^mu_{i(A) j(B + n_AB)} for mu on A or
 * on B + n_AB, V_{mu(A) nu(B + n_AB)}, D_{A, B + n_AB}.  D and the output X keep
 * the dense layout: block (A, B) holds the pair's block at n_AB, zero for pairs
 * beyond the cutoff.  The output is the real-space X_ik(n) of Eq.
 * realspace_exchange restricted to that pattern (i on A in the home cell, k on
 * B at n_AB), and E_x = -1/4 sum over those blocks of X o D is the exchange
 * energy per cell.  exx_pair_images() returns n_AB.  Periodic plans take
 * build_K (every precision), graphs, the autotuner, the energy entry points
 * exchange_backward (gradients per stored entry of the home-cell blocks:
 * E_x per cell differentiated with every image of a block moving with it;
 * forces use the image separation x_A - (x_B + n_AB.L)), build_K_spin and
 * build_K_two_kernels (each result on the same pattern) and workspace
 * budgets (chunks, below; each chunk's part of the pattern-folded X is the
 * sum of the terms of its aux atoms).
 *
 * Ownership: the caller owns every device array passed in; the plan owns its
 * bookkeeping lists and workspace.  Output arrays are fully overwritten
 * (never accumulated into).  Calls are asynchronous on the HIP stream given
 * as `stream` (a hipStream_t, NULL = default stream); host outputs are
 * written before the call returns.
 *
 * Errors: every int-returning entry point returns EXX_OK (0) or a negative
 * code; exx_last_error() describes the last failure of the calling thread.
 * Nothing aborts or throws across the ABI.
 */
#ifndef EXX_H
#define EXX_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXX_OK            0
#define EXX_EINVAL       -1   /* bad argument: null pointer, size, range */
#define EXX_ENOMEM       -2   /* device or host allocation failed */
#define EXX_EDEVICE      -3   /* HIP runtime error */
#define EXX_ESTATE       -4   /* plan in the wrong state (e.g. host-only plan) */
#define EXX_EUNSUPPORTED -5   /* option not implemented */

/* arithmetic of the contraction stages */
#define EXX_PREC_FP64     0   /* binary64 everywhere (FP64 MFMA) */
#define EXX_PREC_MIXED    1   /* distance-split mixed precision, see exx_plan_set_mixed_split */
#define EXX_PREC_FP32     2   /* every pair term of the V stage and of the T2 blocks in binary32
                                 (the mixed build at split 0, whatever split the plan holds);
                                 a reported mode: it does not meet the mixed-precision bar */
#define EXX_PREC_BF16X3   3   /* reserved (bfloat16 hi/lo split products): EXX_EUNSUPPORTED */

/* plan flags */
#define EXX_PLAN_HOST_ONLY 1u /* build the lists on the host only; no device use */

typedef struct exx_plan_s* exx_plan;

typedef struct {
    int32_t n_atoms;
    int32_t n_species;
    const int32_t* species;      /* host [n_atoms], values 0..n_species-1 */
    const double* positions;     /* host [n_atoms][3], Angstrom */
    const int32_t* n_basis;      /* host [n_species], 1..16 */
    const int32_t* n_aux;        /* host [n_species], 1..64 */
    double r_cut;                /* Angstrom, > 0 */
    int32_t n_systems;           /* >= 1 */
    const int32_t* sys_atom_off; /* host [n_systems + 1], increasing, first 0,
                                    last n_atoms; may be NULL if n_systems == 1 */
    const double* lattice;       /* host [3][3] lattice vectors (rows, Angstrom) of a
                                    periodic system (n_systems must be 1; r_cut below
                                    half the cell width, else EXX_EINVAL), or NULL for
                                    clusters */
} exx_system;

typedef struct {
    int64_t n_atoms, n_systems, n_pairs;
    int64_t c_size, v_size, d_size;     /* element counts of C, V, D (= K) */
    int64_t n_basis_max;                /* largest system */
    int64_t workspace_bytes;            /* device bytes held by the plan */
    int64_t flops_fp64;                 /* algorithmic flops of one build_K */
    int64_t n_chunks;                   /* aux-atom chunks a build runs in (1: everything stored) */
    int64_t intermediate_bytes;         /* device bytes of the E, H' and Y workspaces */
    int64_t intermediate_bytes_stored;  /* what they take when nothing is recomputed */
} exx_info;

/* Build a plan for one geometry: screening, canonical pairs, neighbour
 * lists and all task lists (atom-pair / atom-quartet block lists) of the
 * exchange build.  The bookkeeping runs on the current HIP device unless
 * flags has EXX_PLAN_HOST_ONLY.  The plan keeps copies of everything it needs
 * from *sys.  Returns EXX_EINVAL for malformed systems.  Errors leave *out
 * NULL.
 *
 * ws_budget_bytes bounds the device memory of the C.D intermediates of a build
 * (E = M D of Eq. temp_E, H' of Eqs. temp_F-temp_H, Y = T^T H'; the
 * memory-driven sizing of Sec. "Initialization" and the force pass split of
 * Sec. "EXX force and stress contributions"); 0 = no bound.  When storing them
 * for all aux atoms at once would exceed the bound, builds and backward passes
 * run over consecutive chunks of aux atoms, and the E blocks of the atoms
 * neighbouring a chunk are recomputed for every chunk that needs them instead
 * of being stored.  The result equals the unbounded build up to the rounding
 * order of the final sum (the per-chunk parts of K are added in chunk order).
 * EXX_ENOMEM if one V-stage group (at most three neighbouring atoms) alone
 * needs more than the bound.  Clusters and periodic plans (in a small
 * periodic cell nearly every atom neighbours every group, so the smallest
 * budget there is close to the stored layout's).  Collinear-spin and
 * two-kernel builds on a chunked plan run chunk by chunk too; their second
 * result's E and H' take one more chunk-sized workspace (outside the bound). */
int exx_plan_create(const exx_system* sys, uint32_t flags, size_t ws_budget_bytes, exx_plan* out);

/* Release the plan and its device memory (after work on it has finished). */
int exx_plan_destroy(exx_plan plan);

/* Sizes and counts of the plan (host struct written). */
int exx_plan_info(exx_plan plan, exx_info* info);

/* Canonical pair layout, written to caller-owned host arrays: pair_a and
 * pair_b [n_pairs] (int32 atom indices), c_off and v_off [n_pairs + 1]
 * (int64 element offsets of each pair's C and V block).  Any pointer may be
 * NULL to skip that array.  n_pairs is in exx_plan_info(). */
int exx_pair_layout(exx_plan plan, int32_t* pair_a, int32_t* pair_b,
                    int64_t* c_off, int64_t* v_off);

/* Lattice image n_AB of every canonical pair (periodic plans; zeros for
 * clusters): host int32 [n_pairs][3]. */
int exx_pair_images(exx_plan plan, int32_t* images);

/* Neighbour lists as built on the device (for inspection and tests):
 * nbr_ptr [n_atoms + 1], nbr_atom [nbr_ptr[n_atoms]], host arrays.  Pass
 * nbr_atom = NULL to read nbr_ptr only (the total count). */
int exx_plan_neighbors(exx_plan plan, int32_t* nbr_ptr, int32_t* nbr_atom);

/* The exchange matrix K (definition above) and, if Ex != NULL, the energies
 * E_x of every system (device array [n_systems], binary64).
 * C, V, D: device inputs in the layouts above.  K: device output, d_size
 * doubles, exactly symmetric.  precision: EXX_PREC_*.
 * Sizes are those of exx_plan_info().  Returns EXX_ESTATE for a host-only
 * plan. */
int build_K(exx_plan plan, const double* C, const double* V, const double* D,
            int precision, double* K, double* Ex, void* stream);

/* Collinear spin: the spin index of Eq. realspace_exchange (Sec. "Description
 * of the real-space formalism") runs over two values, and each spin has its
 * own density matrix D^s and exchange matrix K^s = sum C V C D^s (the
 * definition above with D^s in place of D).
 * D: device, 2 * d_size doubles, D^0 then D^1, each laid out as D of build_K.
 * K: device output, 2 * d_size doubles, K^0 then K^1 (each exactly symmetric).
 * Ex: NULL, or device [n_systems]: E_x = -1/2 sum_s sum_ik K^s_ik D^s_ik
 * (with D^0 = D^1 = D/2 this is the E_x of build_K for D).
 * The repack of C and E = M D^s for both spins run once; in binary64 the
 * F = V C part of the V stage (Eq. temp_F) is also formed once for both
 * spins.  precision as in build_K: mixed and FP32 run the V stage, T2 and
 * the final contraction of that precision per spin (each K^s equals build_K
 * of D^s in that precision bit for bit).  Clusters and periodic plans,
 * chunked plans included (chunk by chunk).  The first call allocates a second
 * E and H' workspace (of the largest chunk's size on a chunked plan;
 * EXX_ENOMEM if that fails); calls on one plan must not overlap. */
int build_K_spin(exx_plan plan, const double* C, const double* V, const double* D,
                 int precision, double* K, double* Ex, void* stream);

/* Two Coulomb kernels in one call (Sec. "Introduction": functionals that mix
 * a full-range and a screened exchange part need one exchange matrix per
 * Coulomb kernel): K^a = sum C V^a C D for V^0 = V and V^1 = V2, where V2 is a
 * second Coulomb matrix in the pair layout of V.
 * K: device output, 2 * d_size doubles, K^0 then K^1.  Ex: NULL, or device
 * [2 * n_systems]: E_x of K^0 for every system, then of K^1 (each as in
 * exchange_energy).  The repack of C and E = M D (Eq. temp_E) are shared by
 * both kernels; the V stage, T2 and the final contraction run per kernel.
 * precision as in build_K (mixed and FP32 split each kernel's pair terms the
 * same way; each K^a equals build_K with V^a in that precision bit for bit).
 * Clusters and periodic plans, chunked plans included (chunk by chunk: E once
 * per chunk, then both kernels).  Uses the second workspace of build_K_spin
 * (allocated on first use). */
int build_K_two_kernels(exx_plan plan, const double* C, const double* V, const double* V2,
                        const double* D, int precision, double* K, double* Ex, void* stream);

/* Capture one build_K (these exact arrays, `precision` as in build_K) on
 * `stream` into a HIP graph owned by the plan, replacing any earlier one;
 * exx_graph_launch() replays it.  The arrays must stay valid while the graph is used.  The
 * captured work is kernel launches only (buffers are cleared by kernels).
 * `stream` must be a created stream (capture on the default stream is
 * rejected with EXX_EINVAL).  Replays on one plan must not overlap: they
 * share the plan's workspace. */
int exx_graph_build(exx_plan plan, const double* C, const double* V, const double* D,
                    int precision, double* K, double* Ex, void* stream);
int exx_graph_launch(exx_plan plan, void* stream);

/* Autotuner.  Tile shapes of three stages exist as compiled variants:
 *   choice[0]  E = M D GEMM: k-chunk per LDS stage, 0 -> 16, 1 -> 32;
 *   choice[1]  T2 pair blocks: columns per staged chunk x wavefronts per
 *              workgroup, 0 -> 4 x 4, 1 -> 8 x 4, 2 -> 8 x 8;
 *   choice[2]  Y = T^T H' GEMM: k-chunk per LDS stage, 0 -> 16, 1 -> 32.
 * exx_plan_autotune() runs one build_K (precision as given), then times
 * every variant of each stage on these inputs (best of 3, HIP events on
 * `stream`), keeps the fastest per stage for all later builds of the plan,
 * and ends with a build_K of the chosen configuration into K (no E_x).  It
 * blocks until done and must not be captured.  Every variant computes the
 * same K up to rounding order.  Defaults before tuning: {0, 1, 0}.
 * exx_plan_tuning() reports the choices (int32 [3]) and, if ms is not NULL
 * and the plan was tuned, the measured milliseconds (float [3][3], zero for
 * candidates a stage does not have); exx_plan_set_tuning() sets the choices
 * directly (in range for each stage, else EXX_EINVAL). */
int exx_plan_autotune(exx_plan plan, const double* C, const double* V, const double* D,
                      int precision, double* K, void* stream);
int exx_plan_tuning(exx_plan plan, int32_t* choices, float* ms);
int exx_plan_set_tuning(exx_plan plan, const int32_t* choices);

/* Mixed precision (EXX_PREC_MIXED in build_K).  K is linear in V, and every
 * pair term of the V stage and of the T2 blocks belongs to one aux-atom pair
 * (P, Q) (Eq. temp_F, temp_G, temp_H and the F-E term of Eq.
 * ri_lvl_exchange_matrix).  Terms of pairs with |R_P - R_Q| >= r_split (their
 * V, C and D blocks are the small ones, decaying with distance) run with
 * binary32 operands on FP32 MFMA with binary32 accumulation; all other terms,
 * E = M D, the final contraction, K itself and E_x stay binary64.  The
 * default split is 5.0 A; r_split = 0 puts every pair term in binary32.
 * Changing the split rebuilds the split lists (a blocking call) and drops a
 * captured graph.  Returns EXX_EINVAL unless 0 <= r_split <= 1e6. */
int exx_plan_set_mixed_split(exx_plan plan, double r_split);

/* Maximum-norm estimates (Sec. "Evaluation of the EXX matrix in real space":
 * whether a product of temporaries is formed is decided from estimates of the
 * maximum norms of the arrays involved, such as D and the RI coefficients).
 * exx_block_norms writes, in binary64, for every canonical pair p = (A, B) the
 * three doubles norms[3p..3p+2] = max|C| over the pair's stored C block, max|V|
 * over its V block, max|D| over the (A, B) and (B, A) blocks of D (device array
 * [n_pairs][3], caller-owned; C, V, D as in build_K).  Maxima are exact, so the
 * output does not depend on the order of evaluation.  Asynchronous on stream. */
int exx_block_norms(exx_plan plan, const double* C, const double* V, const double* D, double* norms,
                    void* stream);

/* Screening by those estimates (lossy; off by default).  With eps > 0 every
 * later build_K (any precision; graphs captured afterwards too; and the spin and
 * two-kernel builds, below) first forms the
 * norms of its C, V and D and, per atom A, tau_A = the largest max|C| of a pair
 * with A, rho_A = the largest max|D| of a pair with A, sigma_A = the largest
 * rho_J over J in N[A].  The estimate of pair (P, Q),
 *     est = ((max|V_PQ| * tau_P) * tau_Q) * min(sigma_P, sigma_Q)   (binary64),
 * bounds the modulus of every term C^mu_ij V_{mu nu} C^nu_kl D_jl with mu on P
 * and nu on Q.  Pairs with est < eps take no part in the build: every product
 * through their V block is skipped, so K equals the exact K of V with those
 * blocks set to zero.  eps = 0 switches screening off (the build is then the
 * unscreened one, bit for bit).  The first eps > 0 allocates the plan's norm
 * and flag buffers (n_pairs * 3 + n_atoms * 3 doubles, n_pairs bytes).
 * build_K_spin screens both spins with one flag per pair (max|D| over D^0 and
 * D^1); build_K_two_kernels screens each Coulomb matrix by its own estimates
 * (exx_screened_pairs then returns those of V2).  The backward passes are
 * never screened.  EXX_EINVAL unless eps is finite and
 * >= 0; EXX_ESTATE on a host-only plan. */
int exx_set_screening(exx_plan plan, double eps);

/* The screening flags of the last screened build_K issued (device uint8
 * [n_pairs], caller-owned: 1 = pair skipped), copied on stream after that
 * build.  EXX_ESTATE if no screened build has been issued. */
int exx_screened_pairs(exx_plan plan, uint8_t* flags, void* stream);

/* E_x = -1/4 sum_ik K_ik D_ik for every system (device Ex [n_systems]),
 * summed over the screened pair blocks (D beyond r_cut counts as zero), a
 * fixed-order binary64 reduction (bitwise reproducible).  The per-chunk
 * partial sums live in a plan-owned device buffer. */
int exchange_energy(exx_plan plan, const double* K, const double* D,
                    double* Ex, void* stream);

/* exchange_energy for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * result, bit for bit, with the partial sums in a static device array of
 * EXX_NOALLOC_MAX_CHUNKS doubles (512 KiB per GPU, held until the process
 * ends) instead of the plan's buffer.  The call allocates nothing.
 * EXX_EINVAL if the plan's energy reduction has more chunks than that (the
 * count is n_pairs / 64 rounded up per system, about 4 million canonical
 * pairs at most).  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams, threads or plans) race, and
 * must be ordered by the caller.  The array's device address is looked up
 * once per device on the first call. */
#define EXX_NOALLOC_MAX_CHUNKS 65536
int exchange_energy_noalloc(exx_plan plan, const double* K, const double* D,
                            double* Ex, void* stream);

/* Gradients of the scaled energy sum_s gE[s] * E_x[s] (gE: device [n_systems],
 * dL/dE_x of every system; each system's blocks are scaled by its own gE):
 *   dD (device, d_size, dense, symmetric): dE/dD_ik = -1/2 K_ik, the
 *       derivative with respect to each stored entry of the dense D;
 *   dC (device, c_size): derivative per stored C entry (the two mirrored
 *       uses of an off-site entry summed); on-site entries each counted once;
 *   dV (device, v_size): per stored V entry, off-site blocks counting both
 *       V_{mu nu} and V_{nu mu};
 *   forces (device [n_atoms][3], may be NULL): -d(gE E_x)/dR for the
 *       synthetic model C_AB ~ exp(-r_AB / c_decay), V_AB ~ exp(-r_AB^2 / v_2s2)
 *       (the position dependence the inputs are generated with; the paper's
 *       force terms, Sec. "EXX force and stress contributions", differentiate
 *       the real integrals instead)
 *       (on-site blocks position independent, D held fixed).
 * Any of dC, dV, dD may be NULL to skip it.  K (device, d_size, may be NULL)
 * is the exchange matrix of these same C, V, D from build_K (of either
 * precision): dD is then -1/2 gE K without a rebuild; with K NULL, dD needs a
 * binary64 rebuild of K inside the call.  The gradient arithmetic is binary64:
 * precision must be EXX_PREC_FP64 (EXX_PREC_MIXED returns EXX_EUNSUPPORTED;
 * a mixed forward pass is differentiated by passing its K here). */
int exchange_backward(exx_plan plan, const double* C, const double* V,
                      const double* D, const double* K, const double* gE, int precision,
                      double* dC, double* dV, double* dD, double* forces,
                      double c_decay, double v_2s2, void* stream);

/* Generation of the plan's workspace (the intermediates E and H' of
 * Eqs. temp_E and temp_H): a counter that every call writing them advances
 * (build_K, build_K_spin, build_K_two_kernels, graph builds and replays, and
 * the backward calls that form dC, dV or forces, or rebuild K for dD).  Read
 * it right after the build_K (or build_K_spin) whose intermediates a later
 * exchange_backward_reuse (exchange_backward_spin_reuse) is to take.
 * EXX_EINVAL on NULL arguments. */
int exx_plan_build_id(exx_plan plan, uint64_t* id);

/* exchange_backward (same arguments, results and errors) taking E and H' from
 * the workspace instead of recomputing them, when build_id is the current
 * generation and that generation is a binary64 build_K without screening on a
 * plan of one workspace chunk: H' then gets its G term back from factor 2 to
 * factor 1 (Eq. ri_lvl_exchange_matrix with Eqs. temp_G and temp_H) by one
 * G-only pass, and the rest is as in exchange_backward.  By passing build_id
 * the caller vouches that C, V and D are unchanged since that build_K.  In any
 * other case (another call wrote the workspace since, a mixed or screened
 * build, a chunked plan) the intermediates are recomputed as in
 * exchange_backward.  *reused (may be NULL) is set to 1 when they were taken,
 * else 0.  Results agree with exchange_backward to rounding. */
int exchange_backward_reuse(exx_plan plan, uint64_t build_id, const double* C,
                            const double* V, const double* D, const double* K,
                            const double* gE, int precision, double* dC,
                            double* dV, double* dD, double* forces, double c_decay,
                            double v_2s2, int* reused, void* stream);

/* Gradients of the collinear-spin energy sum_s gE[s] * E_x[s] with
 * E_x = -1/2 sum_sigma sum_ik K^sigma_ik D^sigma_ik (build_K_spin; the spin
 * index of Eq. realspace_exchange selects the density matrix): D, K (optional)
 * and dD hold two d_size blocks (spin 0, then spin 1); dC, dV, forces as in
 * exchange_backward.  Each spin's term is twice the one-density energy of
 * D^sigma, so dC and dV are twice the sum over the spins of the one-density
 * gradients (formed spin by spin, the second spin into plan-owned buffers and
 * then added), and dE/dD^sigma = -gE K^sigma.  Clusters, batches and periodic
 * plans, chunked plans included; precision EXX_PREC_FP64 only. */
int exchange_backward_spin(exx_plan plan, const double* C, const double* V,
                           const double* D, const double* K, const double* gE, int precision,
                           double* dC, double* dV, double* dD, double* forces,
                           double c_decay, double v_2s2, void* stream);

/* exchange_backward_spin taking E^s and H'^s of both spins from the workspace,
 * as exchange_backward_reuse does for one density matrix: when build_id is
 * the current generation and that generation is a binary64 build_K_spin
 * without screening on a plan of one workspace chunk (the caller vouches that
 * C, V and both density matrices are unchanged since); otherwise they are
 * recomputed.  *reused (may be NULL): 1 when they were taken, else 0. */
int exchange_backward_spin_reuse(exx_plan plan, uint64_t build_id, const double* C,
                                 const double* V, const double* D, const double* K,
                                 const double* gE, int precision, double* dC,
                                 double* dV, double* dD, double* forces,
                                 double c_decay, double v_2s2, int* reused,
                                 void* stream);

/* Strain derivative of the energy (the stress contribution of Sec. "EXX
 * force and stress contributions", for the synthetic model of exchange_backward):
 * dEde (device [3][3], row-major) = dE/d(eps_ab) for the homogeneous
 * deformation x -> (1 + eps) x of every position and lattice vector, given dC
 * and dV of exchange_backward (or exchange_backward_spin) for these C, V:
 *   dE/d(eps_ab) = sum over canonical pairs of g_a r_b,
 * r the pair's separation x_A - (x_B + n_AB L), g = dE/dr through C_AB ~
 * exp(-r / c_decay) and V_AB ~ exp(-r^2 / v_2s2) with D held fixed.  Divided by
 * the cell volume it is the stress tensor of this energy.  Clusters and
 * periodic plans; a fixed-order binary64 reduction.  The first call allocates
 * a per-atom buffer (9 doubles per atom). */
int exx_strain_derivative(exx_plan plan, const double* C, const double* V, const double* dC,
                          const double* dV, double c_decay, double v_2s2, double* dEde, void* stream);

/* Bloch sums (Eq. fock_operator_k and Eq. realspace_dm).  k-points are given in
 * fractional reciprocal coordinates (host [n_k][3]; k.R = 2 pi k.n for the
 * lattice vector R = n L); complex arrays are interleaved (re, im) doubles,
 * [n_k][d_size] complex.  With the cutoff below half the cell width every pair
 * (A, B) has the one image n_AB (exx_pair_images), so only R = n_AB enters:
 *   exx_bloch_sum:      Kk(k)_AB = e^{2 pi i k.n_AB} X_AB, Kk(k)_BA = e^{-2 pi i k.n_AB} X_BA
 *                       from the folded real-space X of build_K (device d_size);
 *                       entries outside the pair blocks are zero;
 *   exx_density_from_k: D_AB = Re (1 / n_k) sum_k e^{2 pi i k.n_AB} Dk(k)_AB (and the
 *                       conjugate phase for D_BA): the folded real-space density
 *                       matrix build_K takes, from D(k) on a k-grid (device
 *                       [n_k][d_size] complex); zero outside the pair blocks.  The
 *                       imaginary part vanishes for grids closed under k -> -k
 *                       with D(-k) = conj(D(k)); it is dropped.
 * A cluster plan has n = 0 for every pair.  EXX_EINVAL if n_k <= 0 or a
 * k-point is not finite.  Asynchronous on stream (k-points are read before the
 * call returns). */
int exx_bloch_sum(exx_plan plan, const double* X, int n_k, const double* k_frac, double* Kk, void* stream);
int exx_density_from_k(exx_plan plan, int n_k, const double* k_frac, const double* Dk, double* D,
                       void* stream);

/* Algorithmic flop count of one stage of build_K (stage -1 = total):
 * 0 repack, 1 E = M D, 2 V stage (F, H, G), 3 T2, 4 final contraction:
 * 2*m*n*k summed over the structurally nonzero blocks.  Stages 10..14 give
 * the flops the MFMA instructions of stage 0..4 actually issue (tile padding
 * included).  For the mixed build at the current split: 20..24 the
 * algorithmic flops run in binary32, 30..34 the issued binary32 MFMA flops,
 * 40..44 the issued binary64 MFMA flops. */
int64_t exx_plan_flops(exx_plan plan, int stage);

/* Instrumentation: when enabled, build_K records HIP events on its stream at
 * the boundaries of its EXX_N_STAGES stages, for up to 512 builds:
 *   0 zero-fill + repack of C, 1 E = M D, 2 V stage in binary64 (all pairs,
 *   or the near pairs of a mixed build), 3 V stage in binary32 (far pairs of
 *   a mixed build; empty otherwise), 4 T2 in binary64, 5 T2 in binary32
 *   (mixed only), 6 final contraction, 7 energy.
 * exx_plan_stage_times() waits for the recorded builds, adds their per-stage
 * durations into ms[EXX_N_STAGES] (milliseconds, host array), stores how many
 * builds were recorded in *n_builds and starts a new recording.  Enabling
 * (or re-enabling) clears earlier records. */
#define EXX_N_STAGES 8
int exx_plan_set_profiling(exx_plan plan, int enable);
int exx_plan_stage_times(exx_plan plan, double* ms, int64_t* n_builds);

/* Message of the last error on the calling thread ("" if none). */
const char* exx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EXX_H */
