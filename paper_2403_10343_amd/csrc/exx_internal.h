// Internal plan structure of libexx (not part of the ABI).
//
// Notation (non-periodic RI-LVL exchange, lattice vector R = 0):
//   N[P]   atoms within r_cut of atom P, P included, sorted by index.
//   N2[P]  union of N[J] over J in N[P], sorted.
//   T_P    row-owned RI coefficients of aux atom P: rows (mu, i) with mu and
//          i on P (s_P = n_aux(P) * n_basis(P) rows), columns the basis
//          functions of N[P] (n_P columns).  T_P[(mu,i), j] = C^mu_ij for
//          j off P and C^mu_ij / 2 for j on P, so that C^mu = M^mu + M^mu^T.
//   E_P    = T_P D restricted to columns N2[P]          (s_P x m_P)
//   H_P    = sum_Q (V_PQ (x) D_PQ) T_Q  + 2 G-part       (s_P x m_P)
//   T2     = sum V M D M^T (pair blocks, written into K first)
//   K      = T2 + sym(T^T H)
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace exx {

constexpr int NB_MAX = 16;   // basis functions per atom supported by the kernels
constexpr int NA_MAX = 64;   // auxiliary functions per atom supported by the kernels

struct Run { int lcol, grow, len, img; };      // k-range of the E GEMM (img: periodic image code of its rows)
struct EItem { int P, r0, c0, ct; };           // E tile: rows r0.., cols c0.., column tile ct
struct Unit { int P, mu0, slot, pad; };        // one wavefront of an H group: atom, aux tile, slot
struct GTile { int grp, col_beg, ncols, q_beg, q_end, x_beg, x_end, pad; };  // H group x 16 columns
// V-stage list entry: atom, pair id with group slots 0..2 (-1: none); periodic plans also
// the entry's lattice image (code) and, in G-part lists, per slot the column of E_X where
// the slot atom's basis starts
struct Slot4 { int atom, p0, p1, p2, img, e0, e1, e2; };

// Lattice images n (components in [-8, 8)) as one int: the sum of two codes minus
// IMG0 is the code of the sum of the images.
constexpr int IMG_OFF = 8, IMG_S = 16;
constexpr int img_code(int a, int b, int c) { return (a + IMG_OFF) + (b + IMG_OFF) * IMG_S + (c + IMG_OFF) * IMG_S * IMG_S; }
constexpr int IMG0 = img_code(0, 0, 0);
inline int img_add(int x, int y) { return x + y - IMG0; }
inline int img_neg(int x) { return 2 * IMG0 - x; }

constexpr int E_TILE = 64;           // output tile (rows and columns) of the E = M D GEMM
constexpr int GROUP_ATOMS = 3;       // atoms per H group (slots)
constexpr int H_COLS = 4;            // columns per V-stage tile (one per wavefront)
constexpr int GROUP_WAVES = 8;       // wavefronts per H workgroup at most
constexpr double GROUP_RADIUS = 2.5; // A, group atoms lie within this of the first
struct FItem { int sys, gI0, gL0, pbeg, pend, pad0, pad1, pad2; };  // final tile pair (32 x 32)
struct YTile { int P, m0, n0, pad; };          // 64 x 64 tile of Y_P = T_P^T H'_P
struct T2Class { int nt, ns, beg, end, prec; }; // items [beg, end) with this shape (prec 1: binary32)
struct DVClass { int ntp, ntq, nlq, nip, beg, end; };  // dV pairs [beg, end) of dv_items with this shape

// Near / far split of the V-stage and T2 lists at one split distance: pair
// terms (P, Q) with |R_P - R_Q| >= split run in binary32.
struct MixedSet {
  double split = 5.0;
  bool ready = false;
  std::vector<GTile> tiles_near, tiles_far;
  std::vector<int> far_src;                         // g_tiles index of every far tile
  std::vector<Slot4> q_near, x_near, q_far, x_far;
  std::vector<int> t2_items;                        // near classes first, then far
  std::vector<T2Class> t2_classes;
  // chunked plans: the T2 items of each chunk (rows on the chunk's atoms)
  std::vector<std::vector<int>> chunk_t2_items;
  std::vector<std::vector<T2Class>> chunk_t2_classes;
  int64_t flops32[5] = {0, 0, 0, 0, 0};             // algorithmic flops run in binary32
  int64_t issued32[5] = {0, 0, 0, 0, 0};            // issued binary32 MFMA flops
  int64_t issued64[5] = {0, 0, 0, 0, 0};            // issued binary64 MFMA flops
};

struct PGEnt { int P, tcol, hcol, pad; };       // pattern gather: T_P column, H'_P column
// Tiled pattern contraction: a tile is a pair of V-stage groups (ga <= gb); an entry is one
// P and one part (0: rows of T_P on the ga atoms times columns of H'_P on the gb atoms;
// 1: rows of H'_P on the ga atoms times columns of T_P on the gb atoms), with the first
// column of each group atom in the row and column matrices, or -1.
struct PTEnt { int P, part, rc[3], cc[3]; };
struct PTile { int a0, na, b0, nbt, e_beg, e_end, mask, pad; };   // mask bit 3 sa + sb: pair in the pattern
struct PTClass { int ta, tb, beg, end; };        // tiles with ta x tb 16 x 16 output tiles

// One chunk of a workspace-bounded plan: the aux atoms [a0, a1) (whole V-stage
// groups [g0, g1)), whose H' and Y are formed, and the atoms whose E is
// (re)computed for them: the chunk's atoms and their neighbours.
struct ChunkHost {
  int a0 = 0, a1 = 0, g0 = 0, g1 = 0;
  int gt_beg = 0, gt_end = 0, y_beg = 0, y_end = 0, gd_beg = 0, gd_end = 0;   // ranges of global lists
  std::vector<EItem> e_items;
  std::vector<int> t2_items;
  std::vector<T2Class> t2_classes;
  std::vector<int> dv_items;
  std::vector<DVClass> dv_classes;
  std::vector<FItem> f_items;
  std::vector<int> f_plist;
  std::vector<int64_t> e_off, h_off, y_off;         // per atom, element offsets in the chunk buffers
  int64_t e_total = 0, h_total = 0, y_total = 0;
  // periodic plans: the pattern-contraction tiles and the per-pair gather terms, each
  // restricted to the chunk's P (the X' terms of the chunk)
  std::vector<PTile> pt_tiles;
  std::vector<PTEnt> pt_ent;
  std::vector<PTClass> pt_classes;
  std::vector<int> pg_beg, pg_mid, pg_end, pg_pairs;
  std::vector<PGEnt> pg_ent;
};

constexpr int EN_PAIRS = 64;         // canonical pairs per energy chunk


struct HostPlan {
  // system description
  int n_atoms = 0, n_sys = 0;
  double r_cut = 0;
  // periodic systems (one system, lattice vectors as rows); entries of the
  // neighbour lists carry the image of the neighbour within the cutoff
  bool periodic = false;
  double lat[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int> nbr_img;                         // image code per neighbour entry
  std::vector<int> pair_img;                        // image code of B per canonical pair (A, B)
  std::vector<int> pimg;                            // [A * n_atoms + B]: image of B within r_cut of A, or -1
  std::vector<int> n2_img;                          // image code per N2 entry
  std::vector<int> col2img;                         // image code per E_P column
  std::vector<int> col1img;                         // image code per T_P column
  std::vector<double> nbr_sep;                      // per neighbour entry (A, J): R_A - (R_J + shift), 3 doubles
  std::vector<int> atom_of_col;                     // atom of every basis function
  std::vector<int> grp_colimg;                      // image code per V-stage group column
  std::vector<int> grp_cmap;                        // [group column * 3 + slot]: H' column of the slot atom, or -1
  std::vector<int> pg_beg, pg_mid, pg_end;          // per canonical pair: X'_AB terms [beg, mid), X'_BA [mid, end)
  std::vector<PGEnt> pg_ent;
  std::vector<PTile> pt_tiles;                      // tiled pattern contraction, sorted by class
  std::vector<PTEnt> pt_ent;
  std::vector<PTClass> pt_classes;
  std::vector<int> pg_pairs;                        // canonical pairs left to the per-pair gather
  std::vector<int> species, nb, na, atom_sys, bo;   // per atom
  std::vector<double> pos;                          // 3 * n_atoms
  std::vector<int> sys_atom_off;                    // n_sys + 1
  std::vector<int64_t> sys_n, sys_d_off;            // basis count, offset of dense block
  int64_t d_size = 0, n_basis_max = 0;
  // neighbour lists (CSR) and canonical pairs
  std::vector<int> nbr_ptr, nbr_atom, nbr_pair, nbr_lcol, nbr_owner;
  std::vector<int> pair_a, pair_b;
  std::vector<int64_t> c_off, v_off;
  std::vector<int> n_loc;                           // n_P
  // N2 lists
  std::vector<int> n2_ptr, n2_atom;
  std::vector<int> m_loc;                           // m_P
  // maps (per atom, over the basis of its system)
  std::vector<int64_t> map_off;
  std::vector<int> map1, map2;
  std::vector<int64_t> col1g_off, col2g_off;
  std::vector<int> col1g, col2g;
  // workspace layout
  std::vector<int64_t> t_off, e_off;
  int64_t t_total = 0, e_total = 0;
  // task lists
  std::vector<EItem> e_items;
  std::vector<int> ct_run_ptr, ct_klen;
  std::vector<uint8_t> ct_kflag;                    // per E column tile and 16 k rows: bit q set if the 16 columns
  std::vector<int64_t> ct_kflag_off;                // 16q.. of D are not all structurally zero there
  std::vector<Run> runs;
  std::vector<EItem> gd_items;                       // G_P = H_P D (backward)
  std::vector<int> gd_run_ptr, gd_klen;
  std::vector<uint8_t> gd_kflag;                    // the same for the gradient product
  std::vector<int64_t> gd_kflag_off;
  std::vector<Run> gd_runs;
  std::vector<int> grp_first, grp_unit_ptr, grp_col_ptr, grp_cols;
  std::vector<Unit> grp_units;
  std::vector<GTile> g_tiles;
  std::vector<Slot4> gq, gx;
  int h_waves = 1;
  std::vector<int> t2_items;                        // 2 * canonical pair id + orientation bit
  // per canonical pair (in the orientation of its T2 item: rows P, columns Q), the E_P
  // column of every column of T_Q (columns N[Q]) at t2col[t2col_off[p] + l]
  std::vector<int64_t> t2col_off;
  std::vector<int> t2col;
  std::vector<int> dv_items;                        // canonical pair ids sorted by dV shape class
  // per canonical pair p = (P, Q) = (pair_a, pair_b): the E_P column of every column of T_Q,
  // and the E_P column where Q's basis starts / the E_Q column where P's basis starts
  std::vector<int64_t> dvcol_off;
  std::vector<int> dvcol, dv_cp, dv_cq;
  std::vector<DVClass> dv_classes;
  std::vector<T2Class> t2_classes;
  std::vector<int64_t> y_off;                       // Y_P = T_P^T H'_P, n_P x m_P row-major
  int64_t y_total = 0;
  std::vector<YTile> y_tiles;
  std::vector<FItem> f_items;
  std::vector<int> f_plist;
  std::vector<int> en_sys;                          // system of each energy chunk
  // flop counts: [0] repack (0), [1] E, [2] H, [3] T2, [4] final
  int64_t flops[5] = {0, 0, 0, 0, 0};
  int64_t issued[5] = {0, 0, 0, 0, 0};
  // mixed precision: one list set per split distance (0: the plan's split,
  // 1: split 0, i.e. every pair term in binary32)
  MixedSet mixed[2];
  // energy reduction: chunks of at most EN_PAIRS canonical pairs of one system
  std::vector<int> en_pbeg, en_pend;
  // aux-atom chunks of a workspace-bounded plan (empty: one chunk, the global lists)
  int64_t ws_budget = 0;                            // bytes, 0 = unbounded
  int64_t inter_stored = 0;                         // bytes of E, H', Y stored for all atoms
  std::vector<ChunkHost> chunks;
  int64_t ws_total = 0;                             // doubles of the E + H' + Y buffer
};

// Validate a system and fill the description part of a HostPlan.
int describe_system(const int32_t n_atoms, const int32_t n_species, const int32_t* species,
                    const double* positions, const int32_t* n_basis, const int32_t* n_aux,
                    double r_cut, int32_t n_systems, const int32_t* sys_atom_off,
                    const double* lattice, HostPlan& hp, std::string& err);

// Host version of the screened neighbour lists (same arithmetic as the
// device builder): nbr_ptr / nbr_atom only.
void host_neighbors(HostPlan& hp);

// Everything derived from the neighbour lists: canonical pairs and their
// storage offsets, N2, maps, workspace layout, all task lists, flop counts.
int derive_lists(HostPlan& hp, std::string& err);

// Periodic plans: the same lists with image-labelled entries (after the
// neighbour lists with their images; see exx_plan_periodic.cpp).
// Structural zero blocks of one E (or gradient-product) column tile: krow lists the k-side
// entries in k order (atom, image code, first k, length), ccol the output entries (atom,
// image, first column inside the tile, length).  Appends ceil(klen / 16) bytes to out:
// bit q of byte g is set if D has a structurally nonzero element in k rows 16g.. and tile
// columns 16q.. (D_JL with L in N[J], at the matching image for periodic plans).
struct KEnt { int atom, img, beg, len; };
void tile_kflags(const HostPlan& hp, const std::vector<KEnt>& krow, const std::vector<KEnt>& ccol, int klen,
                 std::vector<uint8_t>& out);
int64_t kflag_issued(const uint8_t* f, int klen, int sP);
int derive_lists_periodic(HostPlan& hp, std::string& err);

// Host version of the periodic screening (the device builder's arithmetic):
// nbr_ptr / nbr_atom / nbr_img.
void host_neighbors_periodic(HostPlan& hp);

// Separation (R_B + image shift) - R_A of an image code, the shift summed as
// (n0 a0 + n1 a1) + n2 a2 per component.
void image_shift(const double* lat, int code, double* s);

// Near / far split of the V-stage and T2 lists of hp.mixed[set] at its split
// distance (after derive_lists and derive_chunks), with the binary32 flop counts.
void derive_mixed_lists(HostPlan& hp, int set);

// Aux-atom chunks whose E, H' and Y workspaces fit in budget bytes (0 = no
// bound).  Leaves hp.chunks empty when everything fits at once.  Returns 0,
// or -2 (with err) when a single V-stage group does not fit.
int derive_chunks(HostPlan& hp, int64_t budget, std::string& err);

}  // namespace exx
