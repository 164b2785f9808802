// Host-side interfaces shared by the translation units of libtmop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace tmop {

// Element operations: F and min det A (eq. 2.4), dF/dx, (d^2F/dx^2) v,
// F, min det A and dF/dx in one pass, the diagonal of d^2F/dx^2, the
// per-point sizes (det A)^(1/d) (with min det A), and the per-point target
// data W_0^{-1} = A^{-1} of the replication composite (Section 4.3.2, 2D).
enum { OP_ENERGY = 0, OP_GRAD = 1, OP_HESS = 2, OP_EG = 3, OP_DIAG = 4, OP_SIZE = 5, OP_JINV = 6 };
// timing slots: the element operations above, then the displacement penalty
constexpr int TIMING_PENALTY = 7;
constexpr int TIMING_SLOTS = 8;

// mu_98 = |T - I|^2 / tau on 3x3 T (the replication metric of Section
// 4.3.2 in 3D): an internal metric id of the 3D kernels
constexpr int MU98_3D = 398;
// mu_7 = |T - T^{-t}|^2 on 3x3 T: the internal id of TMOP_MU7 on 3D meshes
constexpr int MU7_3D = 307;

constexpr int MAXP = 5;   // nodes per direction (order p <= 4)
constexpr int MAXQ = 6;   // quadrature points per direction

// LDS values per element of the 2D element kernels: the forward data of
// both components and directions (2 x 2 x Q x P), or with split passes of
// one component at a time (2 x Q x P), padded against bank conflicts.
#ifndef TMOP_ELEM_PAD2
#define TMOP_ELEM_PAD2 5
#endif
constexpr int elem2d_lds_values(int P, int Q, bool split = false) { return (split ? 2 : 4) * Q * P + TMOP_ELEM_PAD2; }

// Owner-computes tiles of a 2D mesh: the gradient, energy + gradient and
// Hessian action in one launch over every element instead of one launch per
// colour.  A workgroup of TILE_BLOCK lanes holds in LDS its tile's node ids
// and an FP64 accumulator per node component, runs the tile's elements in
// rounds of node-disjoint elements (Q lanes each, TILE_BLOCK / Q per round)
// in a fixed order, adding each element's contribution to the accumulators,
// then writes every node only its tile touches and, for a node shared with
// other tiles, its partial sum into that node's slot for this tile.  The
// halo pass adds the slots of each shared node in tile order.  Every sum
// has a fixed order, so the results are reproducible.  One wave per
// workgroup: the rounds' barriers then hold no wave waiting on another
// (measured against 128 and 256 lanes: 512^2 Q2 FP64 Hessian tile launch
// 60.4 -> 53.5 us, 256^2 Q3 mixed 39.0 -> 34.1 us).
constexpr int TILE_BLOCK = 64;
// dynamic LDS of a tile workgroup: 64 KiB less room for its static arrays
constexpr int TILE_LDS_BYTES = 64 * 1024 - 256;
// the static LDS of a tile workgroup (its block-reduction buffer)
constexpr int TILE_STATIC_LDS_BYTES = 2 * (TILE_BLOCK / 64) * 8;
constexpr int tile_epr(int Q) { return TILE_BLOCK / Q; }
// The FP64 gradient tile kernels (gradient, energy + gradient) can stage
// one component at a time (TileParams::split): with both, a Q2 tile of FP64
// workgroups needs 24.9 KB of LDS and six fit on a compute unit, so the
// 512^2 mesh's eight tiles per unit would run in two batches; split, all
// eight are resident at once.  Where every tile is resident anyway the
// extra barriers only cost, and the Hessian action keeps both components
// (its six extra barriers per round cost more than the extra workgroups
// gain).
constexpr bool tile_can_split(int rsize, bool hess) { return rsize == 8 && !hess; }
// LDS bytes per tile node: two FP64 accumulators and the node id
constexpr int TILE_NODE_BYTES = 2 * 8 + 4;
// LDS bytes of a tile workgroup with nn nodes and element data of rsize bytes
constexpr int64_t tile_lds_bytes(int P, int Q, int rsize, bool split, int64_t nn) {
  return nn * TILE_NODE_BYTES + (int64_t)tile_epr(Q) * elem2d_lds_values(P, Q, split) * rsize;
}
struct TileParams {
  const int32_t* round_off;    // [n_tile + 1]: the rounds of tile t are round_off[t] .. round_off[t + 1] - 1
  const int32_t* slot_elem;    // [rounds][tile_epr(Q)]: the element of each round slot, -1: empty
  const uint16_t* slot_lnode;  // [rounds][tile_epr(Q)][P^2]: its nodes' tile-local ids (0 in empty slots)
  const int32_t* node_off;     // [n_tile + 1]: the nodes of tile t are node[node_off[t] ..]
  const int32_t* node;         // global node ids, ascending within each tile
  const int32_t* slot;         // per tile node: its halo slot, or -1 when no other tile touches it
  double* halo;                // [2][n_slot] the tiles' partial sums at shared nodes
  const int32_t* halo_node;    // [n_halo] the shared nodes, ascending
  const int32_t* halo_off;     // [n_halo + 1]: node halo_node[h] has slots halo_off[h] .. (tile order)
  int64_t n_slot, n_halo;
  int32_t n_tile;
  int32_t nn_max;              // most nodes of one tile: sizes the LDS of the launch
  int32_t split;               // 1: the FP64 gradient kernels stage one component at a time
};
// out[c][I] = the sum, in FP64, of node I's element-vector entries
// evec[c n_ent + k], k = off[I] .. off[I+1] - 1 (one entry per element
// holding the node, in ascending element order); nodes without entries
// get 0.  esize: bytes per entry, 8 (FP64) or 4 (FP32, the mixed path's
// element results, which are FP32 values).
hipError_t evec_gather(const void* evec, int esize, const int32_t* off, int64_t n_node, int64_t n_ent, int dim,
                       double* out, hipStream_t s);

// out[c][halo_node[h]] = sum of its slots, in order
hipError_t halo_sum(const TileParams& tp, int64_t n_node, double* out, hipStream_t s);
// The host form of the TileParams arrays (tmop_tiles.cpp).
struct TileLayout {
  std::vector<int32_t> round_off, slot_elem, node_off, node, slot, halo_node, halo_off;
  std::vector<uint16_t> slot_lnode;
  int32_t nn_max = 0;
  int64_t n_slot = 0;
};
// Tiles of a 2D mesh of order p with Q points per direction: elem_node
// [n_elem][npe], colour[e] its element colour.  0, or -1 when the mesh does
// not fit the tile limits (a round index or a node count out of range).
int build_tiles(const int32_t* elem_node, int64_t n_elem, int npe, int64_t n_node, const int32_t* colour, int p,
                int Q, TileLayout& out);

// Everything one element-kernel launch needs, in host form.
struct LaunchParams {
  const double* x;
  const double* v;
  double* out;
  const int32_t* elem_node;
  const int32_t* list;
  const uint32_t* first;   // first-touch bits of the scatter (see ElemArgs), or nullptr
  int32_t n_list;
  int64_t n_node;
  double* part;            // energy partials: sums (one per block)
  double* part_min;        // energy partials: minima of det A
  const double* scale;     // gradient: optional device scalar factor
  const double* tsize;     // per-point isotropic target sizes (in the order of elem_node), or nullptr
  const double* tmat;      // per-point targets [n_list][Q^dim][tms]: W^{-1} row-major and the weight
                           // omega_q (the term is sum_q w_q omega_q mu(A W_q^{-1})), or nullptr
  int tms;                 // values per point of tmat: dim^2 + 1, or 1 (omega_q alone, W^{-1} = Winv)
  int tm_el, tm_pt;        // tms == dim^2 + 1: values between elements and between points of tmat
                           // (tm_pt = 0: one target per element)
  double B[MAXQ][MAXP];
  double G[MAXQ][MAXP];
  double w[MAXQ];
  double Winv[3][3];
  double xi[MAXP];         // GLL node coordinates on [0,1]
  bool iso;                // W = s I: kernels fold 1/s into the G table instead of multiplying by W^{-1}
  double s_inv;
  double detW, detWinv;
  double wdetW;            // weight factor of a constant target: eta det W (OP_JINV: the omega it writes)
  // displacement penalty fused into the 3D FP64 constant-target Hessian action (eq. 4.2)
  bool pen;
  double M1[MAXP][MAXP];   // 1D mass matrix of the quadrature
  double kpen;             // 2 delta det W
  bool dry;                // only report the grid (*grid), launch nothing
  // 2D OP_GRAD / OP_EG / OP_HESS over every element in owner-computes tiles
  // (nullptr: the colour launch described by elem_node / list / first)
  const TileParams* tile;
  // 3D OP_GRAD / OP_EG / OP_HESS: each element's contributions go to this
  // element vector [3][n_ent] instead of the scatter to out (nullptr: the
  // scatter): element e's value for local node l, component c, to entry
  // c n_ent + evpos[e npe + l]; entries of evec_esize bytes, the element
  // kernels' arithmetic type
  void* evec;
  int evec_esize;
  const int32_t* evpos;
  int64_t n_ent;
};

// Everything one launch of the displacement-penalty kernels (eq. 4.2)
// needs.  Operations: OP_ENERGY, OP_GRAD, OP_HESS (field v in x, x0
// unused), OP_EG, OP_DIAG (no field).
struct MassParams {
  const double* x;
  const double* x0;
  double* out;
  const int32_t* elem_node;
  int32_t n_list;
  int64_t n_node;
  double* part;
  double* part_min;
  const double* scale;
  const double* tsize;
  double B[MAXQ][MAXP];
  double w[MAXQ];
  double k;                // 2 delta det W (per-point sizes: 2 delta, times s_q^d in the kernel)
  bool dry;                // only report the grid (*grid), launch nothing
};
int launch_mass(int dim, int p, int Q, int op, const MassParams& mp, hipStream_t s, int* grid);

// One colour of a sweep of the derivative-free solver (Section 3.4): one
// workgroup per node of `nodes`.
struct DfoParams {
  double* x;
  const double* mask;
  const int32_t* nodes;
  const int32_t* ne_off;
  const int32_t* ne;
  const int32_t* elem_node;
  double* move;
  int64_t n_node;
  int32_t n_list;
  int32_t max_evals;
  double B[MAXQ][MAXP];
  double G[MAXQ][MAXP];
  double w[MAXQ];
  double Winv[3][3];
  double detW, step, xtol;
};
int launch_dfo(int dim, int p, int Q, int metric, const DfoParams& dp, hipStream_t s);
// Elements a node's patch may have in the derivative-free kernel: its
// workgroup's lanes hold that many elements' quadrature points (at least 2^dim).
int dfo_patch_capacity(int dim, int Q);

// Launch one element operation (OP_ENERGY / OP_GRAD / OP_HESS / OP_EG) on
// n_list elements: element k has the nodes lp.elem_node[e * npe ...] with
// e = lp.list[k] (or e = k without a list).  Returns 0, -1 if no kernel
// exists for (p, Q, metric), or -2 on a launch error.  *grid receives the
// number of workgroups, i.e. the number of energy partials written to
// lp.part[0, grid) and lp.part_min[0, grid) (OP_ENERGY, OP_EG).
int launch_elem_2d_f64(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_2d_f32(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_2d_f64_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_2d_f32_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_3d_f64(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_3d_f32(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_3d_f64_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
int launch_elem_3d_f32_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid);
bool elem_supported(int dim, int p, int Q);

// The allocation-free energy entry point (tmop_noalloc.hip): its partials,
// the final reduction's scratch and the result live in one file-scope
// device array per GPU of NOALLOC_DOUBLES doubles: at most
// NOALLOC_MAX_BLOCKS workgroups of energy partials (sums, then minima),
// then 2 FIN_BLOCKS doubles of reduction scratch, then the result.
constexpr int64_t NOALLOC_MAX_BLOCKS = 65536;
// Device address of that array on `device`, which must be current;
// hipGetSymbolAddress once per device, cached.  0 or a HIP error code.
int noalloc_scratch(int device, double** out);

// BLAS-1 and reductions (tmop_blas.hip).  Every reduction is deterministic:
// fixed grid, fixed tree order.
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
hipError_t fill(double* y, double v, int64_t n, hipStream_t s);
constexpr int FIN_BLOCKS = 256;
constexpr int64_t NOALLOC_DOUBLES = 2 * NOALLOC_MAX_BLOCKS + 2 * FIN_BLOCKS + 8;
// res[0] = sum of part[0, n), res[1] = min of part[moff, moff + n)
// (scratch: >= 2 * FIN_BLOCKS doubles).
hipError_t finalize_sum_min(const double* part, int n, int moff, double* scratch, double* res, hipStream_t s);
// res[0] = x . y   (scratch: >= RED_BLOCKS doubles)
hipError_t dot(const double* x, const double* y, int64_t n, double* scratch, double* res, hipStream_t s);
hipError_t mul(const double* a, const double* x, double* y, int64_t n, hipStream_t s);    // y = a .* x
// Fused truncated-CG update: d += a p; r -= a (m .* Hp); z = minv .* r; res[0] = r . r, res[1] = r . z
// (m, minv may be nullptr: no mask, no preconditioner; then z is not written and res[1] is not set).
hipError_t cg_step(double a, const double* p, const double* Hp, const double* m, const double* minv, double* d,
                   double* r, double* z, int64_t n, double* scratch, double* res, hipStream_t s);
hipError_t jacobi_inv(const double* m, double* d, int64_t n, hipStream_t s);              // d = m && d ? 1/|d| : 1
// MINRES: Hv <- r_next = m .* Hv - a1 r_cur - a2 r_prev, y = minv .* r_next, res[0] = r_next . y
// (m, r_prev, minv may be nullptr: no mask, no r_prev term, y is r_next)
hipError_t minres_r(double* Hv, const double* m, double a1, const double* r_cur, double a2, const double* r_prev,
                    const double* minv, double* y, int64_t n, double* scratch, double* res, hipStream_t s);
// MINRES: w_prev <- (v - e w_prev - dl w_cur) sg; d += phi w_prev; v <- rb y (y may be nullptr: v kept)
hipError_t minres_wd(double* v, double e, double* w_prev, double dl, const double* w_cur, double sg, double phi,
                     double* d, const double* y, double rb, int64_t n, hipStream_t s);
// Krylov solvers with device-resident scalars: the run state lives in sc
// [SC_COUNT] doubles (indices below); see tmop_blas.hip.
enum {
  SC_ACTIVE = 0, SC_RUN, SC_ITERS, SC_MAXIT, SC_NEG,        // run control (flags as 0/1), counters
  SC_RZ, SC_ALPHA, SC_BETA, SC_PHP, SC_RR, SC_RZP,          // CG (SC_RZP: r . z of the next iteration)
  SC_BPREV, SC_CS, SC_SN, SC_DBAR, SC_EPS, SC_PHI, SC_PHIBAR, SC_BETA1, SC_TOL,   // MINRES
  SC_WE, SC_WDL, SC_WSG, SC_RB,
  SC_COUNT
};
// CG iteration, part 1: block partial sums of p . (Hp + tau p) into
// scratch[2 RED_BLOCKS, 3 RED_BLOCKS).
hipError_t cg_dev_curvature(const double* p, const double* Hp, double tau, int64_t n, double* scratch, double* sc,
                            hipStream_t s);
// CG iteration, part 2: pHp; non-positive curvature ends the run (SC_NEG,
// d unchanged); else alpha = rz / pHp, d += alpha p, r -= alpha (m .* Hp +
// tau p), z = minv .* r; the run ends once |r| <= tol_abs or after SC_MAXIT
// iterations; else p = z + beta p.  m: byte mask of the free DOFs or
// nullptr.  scratch: >= 3 RED_BLOCKS doubles; the run state starts with
// SC_RZP = SC_RZ = the first r . z.
hipError_t cg_dev_update(const double* p, const double* Hp, double tau, const uint8_t* m, const double* minv, double* d,
                         double* r, double* z, int64_t n, double tol_abs, double* scratch, double* sc, hipStream_t s);
// MINRES iteration: alpha = v . Hv, then the residual recurrence, the
// rotations and the direction update (the run ends at the tolerance
// SC_TOL * SC_BETA1 on |phibar|, a zero beta or SC_MAXIT iterations).
hipError_t mr_dev_alpha(const double* v, const double* Hv, int64_t n, double* scratch, double* sc, hipStream_t s);
hipError_t mr_dev_step(double* Hv, const double* m, const double* r_cur, const double* r_prev, const double* minv,
                       double* y, double* v, double* w_prev, const double* w_cur, double* d, int64_t n,
                       double* scratch, double* sc, hipStream_t s);
// res[0] = sum of |d| over the free DOFs (m > 0; m = nullptr: all), res[1] = their min.
hipError_t free_stats(const double* d, const double* m, int64_t n, double* scratch, double* res, hipStream_t s);
hipError_t axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);          // y += a x
hipError_t xpay(const double* x, double a, double* y, int64_t n, hipStream_t s);          // y = x + a y
hipError_t waxpy(const double* x, double a, const double* d, double* w, int64_t n, hipStream_t s);  // w = x + a d
hipError_t scale_copy(double a, const double* x, double* y, int64_t n, hipStream_t s);    // y = a x
hipError_t mask_mul(const double* m, double* y, int64_t n, hipStream_t s);                // y *= m
// dst[j][0..w) = src[rows[j]][0..w) for j < n
hipError_t gather_rows(const double* src, const int32_t* rows, int64_t n, int w, double* dst, hipStream_t s);

}  // namespace tmop

// The context behind the opaque tmop_ctx handle of the C ABI.
struct tmop_ctx {
  int dim = 0, p = 0, Q = 0, metric = 0, precision = 0;
  int64_t n_elem = 0, n_node = 0, n_dof = 0;
  int device = 0;
  tmop::LaunchParams base{};           // tables and target, pointers filled per call
  int32_t* d_elem_node = nullptr;
  int32_t* d_colors = nullptr;         // element ids grouped by colour
  int32_t* d_elem_node_col = nullptr;  // connectivity in colour order: colour launches index it directly
  uint32_t* d_first = nullptr;         // colour order: bit l of element j's words = first touch of local node l
  int first_words = 0;                 // words per element
  bool all_touched = false;            // every node belongs to an element: the colour launches initialize out
  int npe = 0;                         // nodes per element
  std::vector<int64_t> color_off;      // colour c = d_colors[color_off[c] .. color_off[c+1])
  int nq = 0;                          // quadrature points per element, Q^dim
  double* d_tsize = nullptr;           // TMOP_TGT_ISO_PER_QP: [n_elem][nq] sizes s_q, element order
  double* d_tsize_col = nullptr;       // the same in colour order
  double* d_ptgt = nullptr;            // TMOP_TGT_PER_ELEM / PER_QP: per element or per point W^{-1}
                                       // (row-major) and det W, ptgt_stride values each, element order
  double* d_ptgt_col = nullptr;        // the same in colour order
  bool ptgt_elem = false;              // d_ptgt holds one target per element
  int ptgt_stride = 0;                 // dim^2 + 1
  double* d_psize = nullptr;           // [n_elem][nq] (det W_q)^(1/dim) of those targets (the penalty's
  double* d_psize_col = nullptr;       // det W), element and colour order
  double* d_mask = nullptr;            // [n_dof], 1 = free DOF
  uint8_t* d_mask8 = nullptr;          // the same as bytes (the CG update reads it every iteration)
  bool has_fixed = false;
  double* d_part = nullptr;            // [2 * part_cap] energy partials: sums, then minima
  int64_t part_cap = 0;                // partials per kind (3 n_elem + 16: up to three terms)
  // Section 4 terms
  int metric2 = 0;                     // second metric term (0: none)
  int tm_stride = 0;                   // values per point of that data: dim^2 + 1 (W_q^{-1}, omega_q),
                                       // or 1 (omega_q alone, with the constant W2^{-1} below)
  double W2inv[3][3] = {};
  double* d_tmat = nullptr;            // its per-point data [n_elem][nq][tm_stride], element order
  double* d_tmat_col = nullptr;        // the same in colour order
  double delta = 0.0;                  // displacement penalty weight (eq. 4.2; 0: none)
  double* d_xinit = nullptr;           // its x_init [dim][n_node]
  // derivative-free solver (Section 3.4), built on first use
  bool dfo_ready = false;
  int32_t* d_dfo_nodes = nullptr;      // nodes grouped by colour
  std::vector<int64_t> dfo_col_off;    // colour c = d_dfo_nodes[dfo_col_off[c] .. dfo_col_off[c+1])
  int32_t* d_ne_off = nullptr;         // node -> (element, local node) CSR offsets
  int32_t* d_ne = nullptr;             // element * npe + local node
  double* d_dfo_move = nullptr;        // [n_node] per-node moves of a sweep (negated)
  double* d_scratch = nullptr;         // [4 * RED_BLOCKS] dot partials
  double* d_res = nullptr;             // [4] reduction results
  double* h_res = nullptr;             // [4] pinned mirror
  double* d_work = nullptr;            // Newton work vectors, allocated on first use
  double* d_sc = nullptr;              // [SC_COUNT] scalar state of the Krylov solvers
  double* h_sc = nullptr;              // its pinned host mirror
  int64_t n_free = 0;                  // free DOFs (mask 1)
  double* d_noalloc = nullptr;         // the allocation-free entry point's scratch on this device
  // 2D owner-computes tiles (TMOP_SCATTER_TILES), built on first use
  int scatter = 0;                     // TMOP_SCATTER_COLOURS or TMOP_SCATTER_TILES
  int tile_elems = 0;                  // elements per tile they were built for
  tmop::TileParams tile{};             // its device arrays, owned by the context
  // element-vector scatter (TMOP_SCATTER_ELEMENTS, 3D), built on first use
  void* d_evec = nullptr;              // [dim][n_elem npe]: each node's entries contiguous
  int evec_esize = 8;                  // bytes per entry: 8, or 4 in the mixed FP32 path
  int32_t* d_ev_off = nullptr;         // [n_node + 1] node -> its entries (ascending element order)
  int32_t* d_ev_pos = nullptr;         // [n_elem][npe] the entry of element e's local node l
  // optional per-launch timing of the element kernels (HIP events)
  struct TimedLaunch { int op; hipEvent_t a, b; };
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<TimedLaunch> ev_pending;
  double t_ms[tmop::TIMING_SLOTS] = {};        // per op: energy, gradient, Hessian action, energy+gradient,
  int64_t t_launches[tmop::TIMING_SLOTS] = {};  // Hessian diagonal, target sizes, W_0 data, penalty
};
