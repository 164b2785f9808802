// C ABI of libtmop: context set-up, element operations and the Newton /
// truncated-CG driver (arXiv:1807.09807, Sections 2-3).  Host code only;
// every step of the computation runs in the HIP kernels of this library.
#include <math.h>

#include <cmath>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <new>
#include <type_traits>
#include <vector>

#include <hip/hip_runtime.h>

#include "tmop.h"
#include "tmop_internal.h"

using namespace tmop;

// ---------------------------------------------------------------- 1D tables

namespace {

// Legendre polynomial P_n and its first two derivatives at t (three-term
// recurrence).
void legendre(int n, double t, double* P, double* dP, double* d2P) {
  double p0 = 1.0, p1 = t;
  if (n == 0) { *P = 1.0; *dP = 0.0; *d2P = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *P = p1;
  // (1 - t^2) P' = n (P_{n-1} - t P_n);  (1 - t^2) P'' = 2 t P' - n (n+1) P
  const double omt = 1.0 - t * t;
  *dP = n * (p0 - t * p1) / omt;
  *d2P = (2.0 * t * (*dP) - n * (n + 1.0) * p1) / omt;
}

// Gauss-Lobatto-Legendre points of order p on [0,1] (p+1 points): the
// endpoints and the roots of P_p', by Newton's method from the
// Chebyshev-Gauss-Lobatto points.
void gll_points(int p, double* xi) {
  xi[0] = 0.0;
  xi[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double t = -cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre(p, t, &P, &dP, &d2P);
      const double dt = dP / d2P;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    xi[j] = 0.5 * (t + 1.0);
  }
}

// Q-point Gauss-Legendre rule on [0,1].
void gauss_legendre(int Q, double* s, double* w) {
  for (int j = 0; j < Q; ++j) {
    double t = -cos(M_PI * (j + 0.75) / (Q + 0.5));
    double P = 0, dP = 0, d2P = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(Q, t, &P, &dP, &d2P);
      const double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    legendre(Q, t, &P, &dP, &d2P);
    s[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dP * dP);   // 2 / ((1-t^2) P'^2), halved for [0,1]
  }
}

// Q-point Gauss-Lobatto rule on [0,1].
void gauss_lobatto(int Q, double* s, double* w) {
  gll_points(Q - 1, s);
  for (int j = 0; j < Q; ++j) {
    double P, dP, d2P;
    const double t = 2.0 * s[j] - 1.0;
    if (j == 0 || j == Q - 1) {
      P = 1.0;   // |P_n(+-1)| = 1
    } else {
      legendre(Q - 1, t, &P, &dP, &d2P);
    }
    w[j] = 1.0 / (Q * (Q - 1.0) * P * P);
  }
}

// Lagrange basis through nodes xi (n of them) and its derivative at s.
void lagrange_at(int n, const double* xi, double s, double* L, double* dL) {
  for (int a = 0; a < n; ++a) {
    double v = 1.0, d = 0.0;
    for (int b = 0; b < n; ++b) {
      if (b == a) continue;
      const double f = 1.0 / (xi[a] - xi[b]);
      d = d * (s - xi[b]) * f + v * f;   // product rule, built up factor by factor
      v *= (s - xi[b]) * f;
    }
    L[a] = v;
    dL[a] = d;
  }
}

double det3(const double* W, int d) {
  if (d == 2) return W[0] * W[3] - W[1] * W[2];
  return W[0] * (W[4] * W[8] - W[5] * W[7]) - W[1] * (W[3] * W[8] - W[5] * W[6]) +
         W[2] * (W[3] * W[7] - W[4] * W[6]);
}

void inv3(const double* W, int d, double out[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i][j] = 0.0;
  const double D = det3(W, d);
  if (d == 2) {
    out[0][0] = W[3] / D; out[0][1] = -W[1] / D;
    out[1][0] = -W[2] / D; out[1][1] = W[0] / D;
    return;
  }
  out[0][0] = (W[4] * W[8] - W[5] * W[7]) / D;
  out[0][1] = (W[2] * W[7] - W[1] * W[8]) / D;
  out[0][2] = (W[1] * W[5] - W[2] * W[4]) / D;
  out[1][0] = (W[5] * W[6] - W[3] * W[8]) / D;
  out[1][1] = (W[0] * W[8] - W[2] * W[6]) / D;
  out[1][2] = (W[2] * W[3] - W[0] * W[5]) / D;
  out[2][0] = (W[3] * W[7] - W[4] * W[6]) / D;
  out[2][1] = (W[1] * W[6] - W[0] * W[7]) / D;
  out[2][2] = (W[0] * W[4] - W[1] * W[3]) / D;
}

}  // namespace

// ---------------------------------------------------------------- context


#define HIP_TRY(call)                         \
  do {                                        \
    if ((call) != hipSuccess) return TMOP_E_HIP; \
  } while (0)

namespace {

// Starts a timed region of timing slot `slot` (no-op unless timing is on).
int timing_begin(tmop_ctx* c, int slot, hipStream_t s, tmop_ctx::TimedLaunch& tl) {
  tl = tmop_ctx::TimedLaunch{slot, nullptr, nullptr};
  if (!c->timing) return TMOP_OK;
  for (hipEvent_t* e : {&tl.a, &tl.b}) {
    if (!c->ev_free.empty()) {
      *e = c->ev_free.back();
      c->ev_free.pop_back();
    } else if (hipEventCreate(e) != hipSuccess) {
      return TMOP_E_HIP;
    }
  }
  return hipEventRecord(tl.a, s) == hipSuccess ? TMOP_OK : TMOP_E_HIP;
}

// Ends it; a failed launch (r != 0) records nothing.
void timing_end(tmop_ctx* c, int r, hipStream_t s, tmop_ctx::TimedLaunch& tl) {
  if (!c->timing) return;
  if (r != 0 || hipEventRecord(tl.b, s) != hipSuccess) {
    c->ev_free.push_back(tl.a);
    c->ev_free.push_back(tl.b);
  } else {
    c->ev_pending.push_back(tl);
  }
}

// Where the energy partials and the final reduction of an energy call go:
// the context's buffers (nullptr), or the allocation-free scratch.  With
// dry set the launches only count their workgroups.
struct RedDst {
  double* part;        // sums at part[0, cap), minima at part[cap, 2 cap)
  int64_t cap;
  double* fin;         // >= 2 FIN_BLOCKS doubles of reduction scratch
  double* res;         // F and min det A
  bool dry;
};

// The metric term a launch evaluates: the primary one, or the second term
// of a composite objective (its metric and per-point targets).
struct TermSel {
  int metric = -1;                 // -1: the context's metric
  const double* tmat = nullptr;    // general targets: their data in the launch's element order
  int tms = 0;                     // values per point (or element) of tmat: dim^2 + 1, or 1 (omega_q alone)
  bool per_elem = false;           // tmat holds one target per element
  double omega = 0.0;              // OP_JINV: the weight omega_q it writes beside W_0^{-1}
  bool pen = false;                // the displacement penalty rides in this launch
};

// The primary metric term on elements [e0, ...) of the element order (col
// false) or the colour order (col true): general targets per element or per
// point (TMOP_TGT_PER_ELEM / TMOP_TGT_PER_QP) ride in tmat.
TermSel primary_term(const tmop_ctx* c, bool col, int64_t e0, bool pen) {
  TermSel t;
  t.pen = pen;
  if (c->d_ptgt) {
    const int64_t per = (c->ptgt_elem ? 1 : c->nq) * (int64_t)c->ptgt_stride;
    t.tmat = (col ? c->d_ptgt_col : c->d_ptgt) + e0 * per;
    t.tms = c->ptgt_stride;
    t.per_elem = c->ptgt_elem;
  }
  return t;
}

// The second metric term (Sections 4.2, 4.3.2) on elements [e0, ...).
TermSel second_term(const tmop_ctx* c, bool col, int64_t e0) {
  TermSel t;
  t.metric = c->metric2;
  t.tmat = (col ? c->d_tmat_col : c->d_tmat) + e0 * c->nq * c->tm_stride;
  t.tms = c->tm_stride;
  return t;
}

// Per-point sizes whose d-th powers are det W of the primary target, for the
// displacement penalty (nullptr: a constant target).
const double* penalty_sizes(const tmop_ctx* c, bool col, int64_t e0) {
  const double* p = c->d_tsize ? (col ? c->d_tsize_col : c->d_tsize) : (col ? c->d_psize_col : c->d_psize);
  return p ? p + e0 * c->nq : nullptr;
}

// Whether the displacement penalty (eq. 4.2) of op runs inside the primary
// term's element kernels: the Hessian action, 3D, FP64, constant target.
// Measured on the 64^3 Q2 hex workload: the fused Hessian colour launch
// takes 11% longer than the plain one, the separate penalty kernels add 29%
// to the operation.  Energy and energy + gradient gain nothing from fusion
// (the fused gradient kernels lose a wave per SIMD to registers, and the
// x_init gather stays), so they keep the separate kernels.
bool fused_penalty(const tmop_ctx* c, int op) {
  return c->delta > 0.0 && c->dim == 3 && c->precision == TMOP_FP64 && !c->d_tsize && !c->d_ptgt && op == OP_HESS;
}

// Element kernels over n_list elements: conn[k * npe ...] (list == nullptr)
// or conn[list[k] * npe ...].  Energy partials (OP_ENERGY, OP_EG) go to
// d_part[part_off + b] (sums) and d_part[part_cap + part_off + b] (minima).
int elem_launch(tmop_ctx* c, int op, const double* x, const double* v, double* out, const int32_t* conn,
                const int32_t* list, int64_t n_list, hipStream_t s, int* grid, const double* scale = nullptr,
                int64_t part_off = 0, const uint32_t* first = nullptr, const double* tsize = nullptr,
                TermSel term = TermSel{}, const RedDst* rd = nullptr, const TileParams* tile = nullptr,
                void* evec = nullptr) {
  LaunchParams lp = c->base;
  lp.tile = tile;
  lp.evec = evec;
  lp.evec_esize = c->evec_esize;
  lp.evpos = evec ? c->d_ev_pos : nullptr;
  lp.n_ent = c->n_elem * c->npe;
  lp.first = first;
  lp.tsize = tsize;
  lp.tmat = term.tmat;
  if (term.tmat) {
    lp.tms = term.tms;
    lp.tm_pt = term.per_elem ? 0 : term.tms;
    lp.tm_el = term.per_elem ? term.tms : c->nq * term.tms;
    if (term.tms == 1)   // constant second target: its W^{-1} rides in the kernel arguments
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) lp.Winv[i][j] = c->W2inv[i][j];
  }
  lp.pen = term.pen;
  if (term.pen) lp.kpen = 2.0 * c->delta * c->base.detW;
  lp.scale = scale;
  lp.x = x; lp.v = v; lp.out = out;
  lp.elem_node = conn;
  lp.list = list;
  lp.n_list = (int32_t)n_list;
  lp.n_node = c->n_node;
  lp.part = (rd ? rd->part : c->d_part) + part_off;
  lp.part_min = (rd ? rd->part + rd->cap : c->d_part + c->part_cap) + part_off;
  lp.dry = rd && rd->dry;
  const int metric = term.metric < 0 ? c->metric : term.metric;
  if (op == OP_JINV) {   // W_0 data of the replication composite: A of W = I, in FP64
    lp.iso = false;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) lp.Winv[i][j] = i == j ? 1.0 : 0.0;
    lp.detW = lp.detWinv = 1.0;
    lp.wdetW = term.omega;
  }
  tmop_ctx::TimedLaunch tl;
  const bool timed = !rd;   // the allocation-free call creates no events
  if (timed && timing_begin(c, op, s, tl) != TMOP_OK) return TMOP_E_HIP;
  const bool f64 = c->precision == TMOP_FP64 || op == OP_JINV;
  int r;
  if (c->dim == 2)
    r = f64 ? launch_elem_2d_f64(c->p, c->Q, metric, op, lp, s, grid)
            : launch_elem_2d_f32(c->p, c->Q, metric, op, lp, s, grid);
  else
    r = f64 ? launch_elem_3d_f64(c->p, c->Q, metric, op, lp, s, grid)
            : launch_elem_3d_f32(c->p, c->Q, metric, op, lp, s, grid);
  if (timed) timing_end(c, r, s, tl);
  if (r == -1) return TMOP_E_UNSUPPORTED;
  return r == 0 ? TMOP_OK : TMOP_E_HIP;
}

// Displacement-penalty kernels (eq. 4.2) over n_list elements of conn,
// adding to out; energy partials as elem_launch.  x is v for OP_HESS.
int mass_launch(tmop_ctx* c, int op, const double* x, double* out, const int32_t* conn, int64_t n_list,
                hipStream_t s, int* grid, const double* scale, int64_t part_off, const double* tsize,
                const RedDst* rd = nullptr) {
  MassParams mp{};
  mp.x = x;
  mp.x0 = c->d_xinit;
  mp.out = out;
  mp.elem_node = conn;
  mp.n_list = (int32_t)n_list;
  mp.n_node = c->n_node;
  mp.part = (rd ? rd->part : c->d_part) + part_off;
  mp.part_min = (rd ? rd->part + rd->cap : c->d_part + c->part_cap) + part_off;
  mp.dry = rd && rd->dry;
  mp.scale = scale;
  mp.tsize = tsize;
  for (int q = 0; q < MAXQ; ++q) {
    mp.w[q] = c->base.w[q];
    for (int i = 0; i < MAXP; ++i) mp.B[q][i] = c->base.B[q][i];
  }
  mp.k = 2.0 * c->delta * c->base.detW;   // per-point sizes: det W = 1 here, s_q^d in the kernel
  tmop_ctx::TimedLaunch tl;
  if (!rd && timing_begin(c, TIMING_PENALTY, s, tl) != TMOP_OK) return TMOP_E_HIP;
  const int r = launch_mass(c->dim, c->p, c->Q, op, mp, s, grid);
  if (!rd) timing_end(c, r, s, tl);
  if (r == -1) return TMOP_E_UNSUPPORTED;
  return r == 0 ? TMOP_OK : TMOP_E_HIP;
}

// Waits for the pending timed launches and adds their durations.
int collect_timing(tmop_ctx* c) {
  int st = TMOP_OK;
  for (auto& t : c->ev_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) {
      st = TMOP_E_HIP;
    } else {
      c->t_ms[t.op] += ms;
      c->t_launches[t.op] += 1;
    }
    c->ev_free.push_back(t.a);
    c->ev_free.push_back(t.b);
  }
  c->ev_pending.clear();
  return st;
}

// out = sum over colours of the element contributions (gradient / Hv /
// diagonal; with OP_EG also the energy partials of every colour, *nblocks
// of them): the primary metric term (its colour launches write first
// touches), then the Section 4 terms that are set, adding to out.
int assemble(tmop_ctx* c, int op, const double* x, const double* v, double* out, hipStream_t s,
             const double* scale = nullptr, int64_t* nblocks = nullptr) {
  // the first touch of every node writes instead of adding, so out needs no
  // zero fill unless some node belongs to no element
  if (!c->all_touched) HIP_TRY(fill(out, 0.0, c->n_dof, s));
  int64_t off = 0;
  const int ncol = (int)c->color_off.size() - 1;
  if (c->scatter == TMOP_SCATTER_TILES && (op == OP_GRAD || op == OP_EG || op == OP_HESS)) {
    // one launch in owner-computes tiles (2D), element order
    int grid = 0;
    const int r = elem_launch(c, op, x, v, out, nullptr, nullptr, c->n_elem, s, &grid, scale, off, nullptr,
                              c->d_tsize, primary_term(c, false, 0, fused_penalty(c, op)), nullptr, &c->tile);
    if (r != TMOP_OK) return r;
    off += grid;
  } else if (c->scatter == TMOP_SCATTER_ELEMENTS && (op == OP_GRAD || op == OP_EG || op == OP_HESS || op == OP_DIAG)) {
    // one launch over every element into the element vector, then the gather
    int grid = 0;
    const int r = elem_launch(c, op, x, v, out, c->d_elem_node, nullptr, c->n_elem, s, &grid, scale, off, nullptr,
                              c->d_tsize, primary_term(c, false, 0, fused_penalty(c, op)), nullptr, nullptr, c->d_evec);
    if (r != TMOP_OK) return r;
    off += grid;
    HIP_TRY(evec_gather(c->d_evec, c->evec_esize, c->d_ev_off, c->n_node, c->n_elem * c->npe, c->dim, out, s));
  } else {
    for (int k = 0; k < ncol; ++k) {
      const int64_t n = c->color_off[k + 1] - c->color_off[k];
      if (n == 0) continue;
      int grid = 0;
      const int r = elem_launch(c, op, x, v, out, c->d_elem_node_col + c->color_off[k] * c->npe, nullptr, n, s,
                                &grid, scale, off, c->d_first + c->color_off[k] * c->first_words,
                                c->d_tsize_col ? c->d_tsize_col + c->color_off[k] * c->nq : nullptr,
                                primary_term(c, true, c->color_off[k], fused_penalty(c, op)));
      if (r != TMOP_OK) return r;
      off += grid;
    }
  }
  for (int k = 0; c->metric2 && k < ncol; ++k) {   // second metric term (Sections 4.2, 4.3.2)
    const int64_t n = c->color_off[k + 1] - c->color_off[k];
    if (n == 0) continue;
    int grid = 0;
    const int r = elem_launch(c, op, x, v, out, c->d_elem_node_col + c->color_off[k] * c->npe, nullptr, n, s,
                              &grid, scale, off, nullptr, nullptr, second_term(c, true, c->color_off[k]));
    if (r != TMOP_OK) return r;
    off += grid;
  }
  for (int k = 0; c->delta > 0.0 && !fused_penalty(c, op) && k < ncol; ++k) {   // displacement penalty (eq. 4.2)
    const int64_t n = c->color_off[k + 1] - c->color_off[k];
    if (n == 0) continue;
    int grid = 0;
    const int r = mass_launch(c, op, op == OP_HESS ? v : x, out, c->d_elem_node_col + c->color_off[k] * c->npe, n,
                              s, &grid, scale, off, penalty_sizes(c, true, c->color_off[k]));
    if (r != TMOP_OK) return r;
    off += grid;
  }
  if (nblocks) *nblocks = off;
  return TMOP_OK;
}

// Enqueue F and min det A into c->d_res[0..1] (rd: into rd->res, the
// partials into rd->part; a dry rd only counts the workgroups into *nblocks):
// every term, element order.
int energy_async(tmop_ctx* c, const double* x, hipStream_t s, const RedDst* rd = nullptr,
                 int64_t* nblocks = nullptr) {
  int grid = 0;
  int r = elem_launch(c, OP_ENERGY, x, nullptr, nullptr, c->d_elem_node, nullptr, c->n_elem, s, &grid, nullptr, 0,
                      nullptr, c->d_tsize, primary_term(c, false, 0, fused_penalty(c, OP_ENERGY)), rd);
  if (r != TMOP_OK) return r;
  int64_t off = grid;
  if (c->metric2) {
    r = elem_launch(c, OP_ENERGY, x, nullptr, nullptr, c->d_elem_node, nullptr, c->n_elem, s, &grid, nullptr, off,
                    nullptr, nullptr, second_term(c, false, 0), rd);
    if (r != TMOP_OK) return r;
    off += grid;
  }
  if (c->delta > 0.0 && !fused_penalty(c, OP_ENERGY)) {
    r = mass_launch(c, OP_ENERGY, x, nullptr, c->d_elem_node, c->n_elem, s, &grid, nullptr, off,
                    penalty_sizes(c, false, 0), rd);
    if (r != TMOP_OK) return r;
    off += grid;
  }
  if (nblocks) *nblocks = off;
  if (rd && rd->dry) return TMOP_OK;
  if (rd) HIP_TRY(finalize_sum_min(rd->part, (int)off, (int)rd->cap, rd->fin, rd->res, s));
  else HIP_TRY(finalize_sum_min(c->d_part, (int)off, (int)c->part_cap, c->d_scratch, c->d_res, s));
  return TMOP_OK;
}

// F, min det A into c->d_res[0..1] and g (unmasked), in one pass.
int energy_gradient_async(tmop_ctx* c, const double* x, double* g, hipStream_t s) {
  int64_t nb = 0;
  const int r = assemble(c, OP_EG, x, nullptr, g, s, nullptr, &nb);
  if (r != TMOP_OK) return r;
  HIP_TRY(finalize_sum_min(c->d_part, (int)nb, (int)c->part_cap, c->d_scratch, c->d_res, s));
  return TMOP_OK;
}

int read_res(tmop_ctx* c, hipStream_t s, double* F, double* mind) {
  HIP_TRY(hipMemcpyAsync(c->h_res, c->d_res, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *F = c->h_res[0];
  *mind = c->h_res[1];
  return TMOP_OK;
}

int energy_sync(tmop_ctx* c, const double* x, hipStream_t s, double* F, double* mind) {
  const int r = energy_async(c, x, s);
  if (r != TMOP_OK) return r;
  return read_res(c, s, F, mind);
}

int dot_sync(tmop_ctx* c, const double* a, const double* b, hipStream_t s, double* out) {
  HIP_TRY(dot(a, b, c->n_dof, c->d_scratch, c->d_res + 2, s));
  HIP_TRY(hipMemcpyAsync(c->h_res + 2, c->d_res + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = c->h_res[2];
  return TMOP_OK;
}

// 3D meshes whose colours average at most this many elements default to the
// element-vector scatter.  Measured on MI355X against the colour launches,
// Q2 hex meshes, energy + gradient and Hessian action per step: its one
// launch over every element keeps the chip fuller than eight colour
// launches (VALU busy 55% against 40% for the 64^3 FP64 Hessian action),
// while its traffic grows with the mesh and larger colours fill the chip by
// themselves.  FP64 steps: 64^3 (32,768 per colour) 0.639 against 0.667 ms,
// 72^3 (46,656) 0.930 against 0.947 ms, 80^3 (64,000) 1.274 against
// 1.261 ms, 96^3 (110,592) 2.212 against 2.165 ms.  The mixed path's FP32
// entries halve the vector's traffic and it wins at every size measured:
// 80^3 0.921 against 1.027 ms, 96^3 1.575 against 1.724 ms.
constexpr int64_t EVEC_DEFAULT_ELEMS_PER_COLOUR = 49152;
constexpr int64_t EVEC_DEFAULT_ELEMS_PER_COLOUR_MIXED = 131072;

void free_tiles(tmop_ctx* c) {
  TileParams& t = c->tile;
  (void)hipFree((void*)t.round_off);
  (void)hipFree((void*)t.slot_elem);
  (void)hipFree((void*)t.slot_lnode);
  (void)hipFree((void*)t.node_off);
  (void)hipFree((void*)t.node);
  (void)hipFree((void*)t.slot);
  (void)hipFree(t.halo);
  (void)hipFree((void*)t.halo_node);
  (void)hipFree((void*)t.halo_off);
  t = TileParams{};
}

// Builds the owner-computes tiles of a 2D mesh on the host (connectivity
// en, the element order of the colouring) and uploads them.
// TMOP_E_UNSUPPORTED when the mesh does not fit the tile limits.
int make_tiles(tmop_ctx* c, const int32_t* en, const std::vector<int32_t>& order) {
  std::vector<int32_t> colour(c->n_elem);
  for (size_t k = 0; k + 1 < c->color_off.size(); ++k)
    for (int64_t j = c->color_off[k]; j < c->color_off[k + 1]; ++j) colour[order[j]] = (int32_t)k;
  TileLayout L;
  if (build_tiles(en, c->n_elem, c->npe, c->n_node, colour.data(), c->p, c->Q, L) != 0)
    return TMOP_E_UNSUPPORTED;
  TileParams t{};
  int st = TMOP_OK;
  auto up = [&](const auto& v, auto** dst) {
    using T = typename std::decay_t<decltype(v)>::value_type;
    *dst = nullptr;
    if (st != TMOP_OK) return;
    const size_t b = std::max<size_t>(v.size(), 1) * sizeof(T);
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) { st = TMOP_E_NOMEM; return; }
    *dst = static_cast<T*>(p);
    if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      st = TMOP_E_HIP;
  };
  int32_t *ro, *se, *no, *nd, *sl, *hn, *ho;
  uint16_t* ln;
  up(L.round_off, &ro); t.round_off = ro;
  up(L.slot_elem, &se); t.slot_elem = se;
  up(L.slot_lnode, &ln); t.slot_lnode = ln;
  up(L.node_off, &no); t.node_off = no;
  up(L.node, &nd); t.node = nd;
  up(L.slot, &sl); t.slot = sl;
  up(L.halo_node, &hn); t.halo_node = hn;
  up(L.halo_off, &ho); t.halo_off = ho;
  if (st == TMOP_OK && hipMalloc(&t.halo, std::max<int64_t>(2 * L.n_slot, 1) * sizeof(double)) != hipSuccess) {
    t.halo = nullptr;
    st = TMOP_E_NOMEM;
  }
  t.n_slot = L.n_slot;
  t.n_halo = (int64_t)L.halo_node.size();
  t.n_tile = (int32_t)(L.node_off.size() - 1);
  t.nn_max = L.nn_max;
  // FP64 gradient kernels: split passes when the tiles with both components
  // would not all be resident at once (LDS per compute unit); the
  // environment variable TMOP_TILE_SPLIT=0 / 1 forces the choice
  {
    int dev = 0, n_cu = 0, lds_cu = 0;
    bool split = false;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        n_cu > 0 && lds_cu > 0) {
      const int64_t per_tile = tile_lds_bytes(c->p + 1, c->Q, 8, false, t.nn_max) + TILE_STATIC_LDS_BYTES;
      split = (int64_t)(lds_cu / per_tile) * n_cu < t.n_tile;
    }
    if (const char* f = std::getenv("TMOP_TILE_SPLIT")) {
      if (f[0] == '0' && f[1] == 0) split = false;
      if (f[0] == '1' && f[1] == 0) split = true;
    }
    t.split = split ? 1 : 0;
  }
  c->tile = t;
  if (st != TMOP_OK) free_tiles(c);
  return st;
}

void free_evec(tmop_ctx* c) {
  (void)hipFree(c->d_evec);
  (void)hipFree(c->d_ev_off);
  (void)hipFree(c->d_ev_pos);
  c->d_evec = nullptr;
  c->d_ev_off = nullptr;
  c->d_ev_pos = nullptr;
}

// The element-vector scatter's buffer and its node -> entry map (3D), from
// the host connectivity en.  TMOP_E_UNSUPPORTED when the entries overflow
// 32-bit offsets.
int make_evec(tmop_ctx* c, const int32_t* en) {
  const int npe = c->npe, d = c->dim;
  const int64_t ne_tot = c->n_elem * npe;
  if (c->n_elem * d * npe > INT32_MAX) return TMOP_E_UNSUPPORTED;
  std::vector<int32_t> off(c->n_node + 1, 0), epos((size_t)ne_tot);
  for (int64_t k = 0; k < ne_tot; ++k) off[en[k] + 1]++;
  for (int64_t I = 0; I < c->n_node; ++I) off[I + 1] += off[I];
  {
    std::vector<int32_t> next(off.begin(), off.end() - 1);
    for (int64_t k = 0; k < ne_tot; ++k) epos[k] = next[en[k]]++;   // ascending element ids per node
  }
  int st = TMOP_OK;
  // the mixed path's element results are FP32 values: FP32 entries hold them exactly
  c->evec_esize = c->precision == TMOP_MIXED_FP32 ? 4 : 8;
  if (hipMalloc(&c->d_evec, (size_t)c->n_elem * d * npe * c->evec_esize) != hipSuccess ||
      hipMalloc(&c->d_ev_off, off.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_ev_pos, epos.size() * sizeof(int32_t)) != hipSuccess) {
    st = TMOP_E_NOMEM;
  } else if (hipMemcpy(c->d_ev_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->d_ev_pos, epos.data(), epos.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    st = TMOP_E_HIP;
  }
  if (st != TMOP_OK) free_evec(c);
  return st;
}

void free_ctx(tmop_ctx* c) {
  if (!c) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(c->device);
  (void)hipFree(c->d_elem_node);
  (void)hipFree(c->d_colors);
  (void)hipFree(c->d_elem_node_col);
  (void)hipFree(c->d_first);
  (void)hipFree(c->d_mask);
  (void)hipFree(c->d_mask8);
  (void)hipFree(c->d_tsize);
  (void)hipFree(c->d_tsize_col);
  (void)hipFree(c->d_tmat);
  (void)hipFree(c->d_tmat_col);
  (void)hipFree(c->d_ptgt);
  (void)hipFree(c->d_ptgt_col);
  (void)hipFree(c->d_psize);
  (void)hipFree(c->d_psize_col);
  (void)hipFree(c->d_xinit);
  (void)hipFree(c->d_dfo_nodes);
  (void)hipFree(c->d_ne_off);
  (void)hipFree(c->d_ne);
  (void)hipFree(c->d_dfo_move);
  (void)hipFree(c->d_part);
  (void)hipFree(c->d_scratch);
  (void)hipFree(c->d_res);
  (void)hipFree(c->d_work);
  (void)hipFree(c->d_sc);
  free_tiles(c);
  free_evec(c);
  if (c->h_res) (void)hipHostFree(c->h_res);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  (void)collect_timing(c);
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  (void)hipSetDevice(cur);
  delete c;
}

// Greedy element colouring: elements of one colour share no node.
void color_elements(const int32_t* en, int64_t n_elem, int npe, int64_t n_node, std::vector<int32_t>& order,
                    std::vector<int64_t>& off) {
  std::vector<int64_t> start(n_node + 1, 0);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int i = 0; i < npe; ++i) start[en[e * npe + i] + 1]++;
  for (int64_t I = 0; I < n_node; ++I) start[I + 1] += start[I];
  std::vector<int32_t> adj(start[n_node]);
  std::vector<int64_t> fillp(start.begin(), start.end() - 1);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int i = 0; i < npe; ++i) adj[fillp[en[e * npe + i]]++] = (int32_t)e;
  std::vector<int16_t> color(n_elem, -1);
  int ncolor = 0;
  std::vector<uint8_t> used;
  for (int64_t e = 0; e < n_elem; ++e) {
    used.assign(ncolor + 1, 0);
    for (int i = 0; i < npe; ++i) {
      const int32_t I = en[e * npe + i];
      for (int64_t k = start[I]; k < start[I + 1]; ++k) {
        const int16_t c = color[adj[k]];
        if (c >= 0) used[c] = 1;
      }
    }
    int c = 0;
    while (c < ncolor && used[c]) ++c;
    color[e] = (int16_t)c;
    if (c == ncolor) ++ncolor;
  }
  off.assign(ncolor + 1, 0);
  for (int64_t e = 0; e < n_elem; ++e) off[color[e] + 1]++;
  for (int c = 0; c < ncolor; ++c) off[c + 1] += off[c];
  order.resize(n_elem);
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (int64_t e = 0; e < n_elem; ++e) order[pos[color[e]]++] = (int32_t)e;
}

// Work vectors of the Newton driver: g, x_trial, g_trial, the direction d,
// the preconditioner and seven solver vectors.
constexpr int NEWTON_VECTORS = 12;
struct Inner {
  double* d;
  double* minv;
  double* v[7];
};

// The Krylov runs keep their scalars on the device (tmop_blas.hip) and the
// host reads them back only at these iteration counts: 1, 2, 4, 8, then every 8.
int next_check(int k) { return k < 8 ? 2 * k : k + 8; }

// Copies the run state in h_sc to the device (before the first iteration).
int sc_upload(tmop_ctx* c, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(c->d_sc, c->h_sc, SC_COUNT * sizeof(double), hipMemcpyHostToDevice, s));
  return TMOP_OK;
}

// Reads the run state back into h_sc; returns whether the run is still active.
int sc_read(tmop_ctx* c, hipStream_t s, bool* active) {
  HIP_TRY(hipMemcpyAsync(c->h_sc, c->d_sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *active = c->h_sc[SC_ACTIVE] != 0.0;
  return TMOP_OK;
}

// One preconditioned CG run on (m H m + tau I) d = -g from d = 0 (minv =
// 1 / diag M or nullptr), until |r|_2 <= tol |g|_2, max_it Hessian
// actions, or the first curvature p.(H + tau I)p <= 0 (*neg; d then holds
// the iterate before that step).  *ncg: Hessian actions used.  r, p, Hp and
// z are w.v[0..3]; p still holds the first direction -M^{-1} g when the run
// ends at its first step.
int cg_run(tmop_ctx* c, const double* x, const double* g, double gn, double tol, int max_it, const double* minv,
           double tau, Inner& w, hipStream_t s, int* ncg, bool* neg) {
  const int64_t N = c->n_dof;
  double* r = w.v[0];
  double* p = w.v[1];
  double* Hp = w.v[2];
  double* z = minv ? w.v[3] : r;
  const uint8_t* mask8 = c->has_fixed ? c->d_mask8 : nullptr;
  int st;
  HIP_TRY(fill(w.d, 0.0, N, s));
  HIP_TRY(scale_copy(-1.0, g, r, N, s));
  double rz;
  if (minv) {
    HIP_TRY(mul(minv, r, z, N, s));
    if ((st = dot_sync(c, r, z, s, &rz)) != TMOP_OK) return st;
  } else {
    rz = gn * gn;
  }
  HIP_TRY(hipMemcpyAsync(p, z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int k = 0; k < SC_COUNT; ++k) c->h_sc[k] = 0.0;
  c->h_sc[SC_ACTIVE] = 1.0;
  c->h_sc[SC_MAXIT] = max_it;
  c->h_sc[SC_RZ] = rz;
  c->h_sc[SC_RZP] = rz;
  if ((st = sc_upload(c, s)) != TMOP_OK) return st;
  bool active = true;
  for (int j = 1, check = 1; j <= max_it; ++j) {
    // H p over all DOFs; p vanishes on the fixed DOFs, so p . Hp equals
    // p . (m .* Hp), and the update applies the mask to Hp
    if ((st = assemble(c, OP_HESS, x, p, Hp, s)) != TMOP_OK) return st;
    HIP_TRY(cg_dev_curvature(p, Hp, tau, N, c->d_scratch, c->d_sc, s));
    HIP_TRY(cg_dev_update(p, Hp, tau, mask8, minv, w.d, r, z, N, tol * gn, c->d_scratch, c->d_sc, s));
    if (j == check || j == max_it) {
      if ((st = sc_read(c, s, &active)) != TMOP_OK) return st;
      if (!active) break;
      check = next_check(check);
    }
  }
  if (active && (st = sc_read(c, s, &active)) != TMOP_OK) return st;
  *ncg = (int)c->h_sc[SC_ITERS];
  *neg = c->h_sc[SC_NEG] != 0.0;
  return TMOP_OK;
}

// Steihaug's truncated CG for H d = -g from d = 0, optionally with the
// diagonal preconditioner minv = 1 / diag M.  Non-positive curvature at the
// first step returns -M^{-1} g (the steepest-descent direction, -g without
// M), later the current iterate; stops once |r|_2 <= tol |g|_2.
int inner_tcg(tmop_ctx* c, const double* x, const double* g, double gn, double tol, int max_it,
              const double* minv, Inner& w, hipStream_t s, int* ncg, bool* neg) {
  const int st = cg_run(c, x, g, gn, tol, max_it, minv, 0.0, w, s, ncg, neg);
  if (st != TMOP_OK) return st;
  if (*neg && *ncg == 1)
    HIP_TRY(hipMemcpyAsync(w.d, w.v[1], c->n_dof * sizeof(double), hipMemcpyDeviceToDevice, s));
  return TMOP_OK;
}

// CG on the modified Hessian H + tau I, the added multiple of the identity
// of Nocedal and Wright (Numerical Optimization, 2nd ed., Algorithm 3.3)
// with a CG run in place of their Cholesky factorization as the test of
// positive definiteness: beta = shift_beta mean |diag H| over the free DOFs
// (diag: the Hessian diagonal at x), tau_0 = 0 if every free diagonal entry
// is positive, else -min diag + beta; while CG meets curvature
// p.(H + tau I)p <= 0, tau <- max(2 tau, beta) and CG restarts from d = 0.
// The direction then solves a positive definite system, so it descends.
// After 64 restarts the direction is -M^{-1} g.  *nrestart: CG restarts.
int inner_shifted_cg(tmop_ctx* c, const double* x, const double* g, double gn, double tol, int max_it,
                     const double* minv, const double* diag, double shift_beta, Inner& w, hipStream_t s, int* ncg,
                     int* nrestart) {
  const int64_t N = c->n_dof;
  HIP_TRY(free_stats(diag, c->has_fixed ? c->d_mask : nullptr, N, c->d_scratch, c->d_res + 2, s));
  HIP_TRY(hipMemcpyAsync(c->h_res + 2, c->d_res + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double beta = shift_beta * c->h_res[2] / (double)std::max<int64_t>(c->n_free, 1);
  const double dmin = c->h_res[3];
  double tau = dmin > 0.0 ? 0.0 : -dmin + beta;
  *ncg = 0;
  *nrestart = 0;
  for (int k = 0; k < 64; ++k) {
    int n = 0;
    bool neg = false;
    const int st = cg_run(c, x, g, gn, tol, max_it, minv, tau, w, s, &n, &neg);
    if (st != TMOP_OK) return st;
    *ncg += n;
    if (!neg) return TMOP_OK;
    ++*nrestart;
    tau = std::max(2.0 * tau, beta);
  }
  HIP_TRY(scale_copy(-1.0, g, w.d, N, s));
  if (minv) HIP_TRY(mul(minv, w.d, w.d, N, s));
  return TMOP_OK;
}

// MINRES (Paige and Saunders) for H d = -g from d = 0, optionally with the
// symmetric positive definite diagonal preconditioner minv = 1 / diag M.
// Preconditioned Lanczos gives the tridiagonal of H in the M^{-1} inner
// product; Givens rotations keep its QR factorization current, so the
// iterate that minimizes the M^{-1}-norm of the residual over the Krylov
// space follows from a three-term recurrence of the directions w_k, and
// |phibar| is that residual norm.  Stops when |phibar| <= tol beta_1.  The
// scalar recurrences run on the device between the vector kernels.
int inner_minres(tmop_ctx* c, const double* x, const double* g, double tol, int max_it, const double* minv,
                 Inner& w, hipStream_t s, int* nit) {
  const int64_t N = c->n_dof;
  double* r_prev = w.v[0];
  double* r_cur = w.v[1];
  double* hbuf = w.v[2];       // H v, then r_next
  double* vbuf = w.v[3];
  double* ybuf = w.v[4];
  double* w_prev = w.v[5];
  double* w_cur = w.v[6];
  const double* mask = c->has_fixed ? c->d_mask : nullptr;
  int st;
  HIP_TRY(fill(w.d, 0.0, N, s));
  HIP_TRY(scale_copy(-1.0, g, r_cur, N, s));
  const double* y = r_cur;
  if (minv) {
    HIP_TRY(mul(minv, r_cur, ybuf, N, s));
    y = ybuf;
  }
  double beta1;
  if ((st = dot_sync(c, r_cur, y, s, &beta1)) != TMOP_OK) return st;
  beta1 = sqrt(beta1);
  *nit = 0;
  if (!(beta1 > 0.0)) return TMOP_OK;
  HIP_TRY(fill(w_prev, 0.0, N, s));
  HIP_TRY(fill(w_cur, 0.0, N, s));
  HIP_TRY(scale_copy(1.0 / beta1, y, vbuf, N, s));          // Lanczos vector v_1
  for (int k = 0; k < SC_COUNT; ++k) c->h_sc[k] = 0.0;
  c->h_sc[SC_ACTIVE] = 1.0;
  c->h_sc[SC_MAXIT] = max_it;
  c->h_sc[SC_BETA] = beta1;
  c->h_sc[SC_BETA1] = beta1;
  c->h_sc[SC_PHIBAR] = beta1;
  c->h_sc[SC_CS] = -1.0;
  c->h_sc[SC_TOL] = tol;
  if ((st = sc_upload(c, s)) != TMOP_OK) return st;
  bool active = true;
  for (int k = 1, check = 1; k <= max_it; ++k) {
    // H v over all DOFs; v vanishes on the fixed DOFs, so v . Hv = v . (m .* Hv)
    if ((st = assemble(c, OP_HESS, x, vbuf, hbuf, s)) != TMOP_OK) return st;
    HIP_TRY(mr_dev_alpha(vbuf, hbuf, N, c->d_scratch, c->d_sc, s));
    HIP_TRY(mr_dev_step(hbuf, mask, r_cur, r_prev, minv, ybuf, vbuf, w_prev, w_cur, w.d, N, c->d_scratch, c->d_sc,
                        s));
    std::swap(w_prev, w_cur);
    // r_{k-1} <- r_k <- r_{k+1}; the oldest buffer takes the next H v
    double* spare = r_prev;
    r_prev = r_cur;
    r_cur = hbuf;
    hbuf = spare;
    if (k == check || k == max_it) {
      if ((st = sc_read(c, s, &active)) != TMOP_OK) return st;
      if (!active) break;
      check = next_check(check);
    }
  }
  if (active && (st = sc_read(c, s, &active)) != TMOP_OK) return st;
  *nit = (int)c->h_sc[SC_ITERS];
  return TMOP_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

const char* tmop_strerror(int status) {
  switch (status) {
    case TMOP_OK: return "success";
    case TMOP_W_INVERTED: return "warning: det A <= 0 at a quadrature point (inverted mesh)";
    case TMOP_W_MAXIT: return "warning: Newton reached the iteration limit";
    case TMOP_W_LSFAIL: return "warning: line search found no admissible step";
    case TMOP_E_ARG: return "error: invalid argument";
    case TMOP_E_TARGET: return "error: target matrix with det W <= 0";
    case TMOP_E_NOMEM: return "error: out of memory";
    case TMOP_E_HIP: return "error: HIP runtime failure";
    case TMOP_E_UNSUPPORTED: return "error: no kernel built for this (dim, order, quadrature)";
    case TMOP_E_SCRATCH: return "error: the problem needs more than the fixed scratch of the allocation-free call";
    default: return "unknown status";
  }
}

void tmop_newton_default_opts(tmop_newton_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->rtol = 1e-12;
  o->atol = 0.0;
  o->max_it = 50;
  o->cg_rtol = 1e-8;
  o->cg_max_it = 1000;
  o->ls_shrink = 0.5;
  o->ls_max = 30;
  o->f_growth = 1.2;
  o->g_growth = 1.2;
  o->ftarget = -HUGE_VAL;
  o->cg_forcing = 0;
  o->inner = TMOP_INNER_SHIFTED_CG;
  o->precond = TMOP_PREC_NONE;
  o->shift_beta = 1e-3;
}

int tmop_setup(const tmop_mesh* mesh, const tmop_quadrature* quad, const tmop_target* target, int32_t metric,
               int32_t precision, tmop_ctx** out) {
  if (!out) return TMOP_E_ARG;
  *out = nullptr;
  if (!mesh || !quad || !target || !mesh->elem_node) return TMOP_E_ARG;
  const int d = mesh->dim, p = mesh->order, Q = quad->n1d;
  if (d != 2 && d != 3) return TMOP_E_ARG;
  if (p < 1 || mesh->n_elem < 1 || mesh->n_node < 1 || mesh->n_elem > (INT32_MAX - 16) / 3 ||
      mesh->n_node > INT32_MAX)
    return TMOP_E_ARG;
  if (quad->kind != TMOP_GAUSS_LEGENDRE && quad->kind != TMOP_GAUSS_LOBATTO) return TMOP_E_ARG;
  if (Q < p + 1) return TMOP_E_ARG;                      // Section 3.3: at least p+1 points
  if (quad->kind == TMOP_GAUSS_LOBATTO && Q < 2) return TMOP_E_ARG;
  if (d == 2 && metric != TMOP_MU1 && metric != TMOP_MU2 && metric != TMOP_MU7 && metric != TMOP_MU9 &&
      metric != TMOP_MU14 && metric != TMOP_MU77 && metric != TMOP_MU98)
    return TMOP_E_ARG;
  if (d == 3 && metric != TMOP_MU302 && metric != TMOP_MU303 && metric != TMOP_MU7) return TMOP_E_ARG;
  if (precision != TMOP_FP64 && precision != TMOP_MIXED_FP32) return TMOP_E_ARG;
  const int kind = target->kind;
  if ((kind != TMOP_TGT_CONST && kind != TMOP_TGT_ISO_PER_QP && kind != TMOP_TGT_PER_ELEM &&
       kind != TMOP_TGT_PER_QP) || !target->W)
    return TMOP_E_ARG;
  const int npe = d == 2 ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
  const int nq = d == 2 ? Q * Q : Q * Q * Q;
  for (int64_t k = 0; k < mesh->n_elem * npe; ++k)
    if (mesh->elem_node[k] < 0 || mesh->elem_node[k] >= mesh->n_node) return TMOP_E_ARG;
  const bool per_qp = kind == TMOP_TGT_ISO_PER_QP;
  const bool gen_tgt = kind == TMOP_TGT_PER_ELEM || kind == TMOP_TGT_PER_QP;
  static const double eye2[4] = {1, 0, 0, 1}, eye3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  const double* Wc = per_qp || gen_tgt ? (d == 2 ? eye2 : eye3) : target->W;
  if (per_qp) {                                          // Section 3.1: det W = s^d > 0
    for (int64_t k = 0; k < mesh->n_elem * nq; ++k)
      if (!(target->W[k] > 0.0)) return TMOP_E_TARGET;
  }
  // General targets per element or per point (Section 3.1: W may differ at
  // every point): W^{-1} row-major and det W > 0, d^2 + 1 values each, and
  // (det W_q)^(1/d) per point for the displacement penalty
  const int ts = d * d + 1;
  std::vector<double> ptgt, psize;
  if (gen_tgt) {
    const int64_t nt = kind == TMOP_TGT_PER_ELEM ? mesh->n_elem : mesh->n_elem * nq;
    ptgt.resize((size_t)nt * ts);
    psize.resize((size_t)mesh->n_elem * nq);
    for (int64_t k = 0; k < nt; ++k) {
      const double* Wk = target->W + k * d * d;
      for (int j = 0; j < d * d; ++j)
        if (!std::isfinite(Wk[j])) return TMOP_E_TARGET;
      const double dW = det3(Wk, d);
      if (!(dW > 0.0) || !std::isfinite(dW)) return TMOP_E_TARGET;
      double Wi[3][3];
      inv3(Wk, d, Wi);
      double* o = &ptgt[(size_t)k * ts];
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) o[i * d + j] = Wi[i][j];
      o[d * d] = dW;
    }
    for (int64_t e = 0; e < mesh->n_elem; ++e)
      for (int q = 0; q < nq; ++q) {
        const double dW = ptgt[(size_t)(kind == TMOP_TGT_PER_ELEM ? e : e * nq + q) * ts + d * d];
        psize[(size_t)(e * nq + q)] = d == 2 ? sqrt(dW) : cbrt(dW);
      }
  }
  const double detW = det3(Wc, d);
  if (!(detW > 0.0)) return TMOP_E_TARGET;               // Section 3.1: det W > 0
  if (!elem_supported(d, p, Q)) return TMOP_E_UNSUPPORTED;

  tmop_ctx* c = new (std::nothrow) tmop_ctx();
  if (!c) return TMOP_E_NOMEM;
  c->dim = d; c->p = p; c->Q = Q; c->precision = precision;
  c->metric = d == 3 && metric == TMOP_MU7 ? MU7_3D : metric;   // the kernels' id of the 3D form
  c->n_elem = mesh->n_elem; c->n_node = mesh->n_node; c->n_dof = (int64_t)d * mesh->n_node;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return TMOP_E_HIP; }
  // the allocation-free entry point's scratch on this device (its address,
  // taken once per device while the device is current)
  if (noalloc_scratch(c->device, &c->d_noalloc) != 0) { delete c; return TMOP_E_HIP; }

  // 1D tables: B[q][i] = l_i(s_q), G[q][i] = l_i'(s_q), weights w[q]
  double xi[MAXP], s[MAXQ], w[MAXQ];
  gll_points(p, xi);
  for (int i = 0; i <= p; ++i) c->base.xi[i] = xi[i];
  if (quad->kind == TMOP_GAUSS_LEGENDRE) gauss_legendre(Q, s, w);
  else gauss_lobatto(Q, s, w);
  for (int q = 0; q < Q; ++q) {
    lagrange_at(p + 1, xi, s[q], c->base.B[q], c->base.G[q]);
    c->base.w[q] = w[q];
  }
  inv3(Wc, d, c->base.Winv);
  c->base.iso = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (Wc[i * d + j] != (i == j ? Wc[0] : 0.0)) c->base.iso = false;
  c->base.s_inv = 1.0 / Wc[0];
  c->nq = nq;
  c->base.detW = detW;
  c->base.detWinv = 1.0 / detW;
  c->base.wdetW = detW;                                  // eta_1 = 1
  c->part_cap = 3 * mesh->n_elem + 16;

  // colouring and device copies
  std::vector<int32_t> order;
  color_elements(mesh->elem_node, mesh->n_elem, npe, mesh->n_node, order, c->color_off);
  c->npe = npe;
  const size_t en_bytes = (size_t)mesh->n_elem * npe * sizeof(int32_t);
  int st = TMOP_OK;
  do {
    if (hipMalloc(&c->d_elem_node, en_bytes) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMalloc(&c->d_colors, order.size() * sizeof(int32_t)) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMalloc(&c->d_part, 2 * (size_t)c->part_cap * sizeof(double)) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMalloc(&c->d_scratch, 4 * RED_BLOCKS * sizeof(double)) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMalloc(&c->d_res, 4 * sizeof(double)) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipHostMalloc(&c->h_res, 4 * sizeof(double), 0) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMalloc(&c->d_mask, c->n_dof * sizeof(double)) != hipSuccess) { st = TMOP_E_NOMEM; break; }
    if (hipMemcpy(c->d_elem_node, mesh->elem_node, en_bytes, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
    if (hipMemcpy(c->d_colors, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
    {   // the connectivity in colour order
      std::vector<int32_t> en_col((size_t)mesh->n_elem * npe);
      for (size_t j = 0; j < order.size(); ++j)
        memcpy(&en_col[j * npe], mesh->elem_node + (size_t)order[j] * npe, npe * sizeof(int32_t));
      if (hipMalloc(&c->d_elem_node_col, en_bytes) != hipSuccess) { st = TMOP_E_NOMEM; break; }
      if (hipMemcpy(c->d_elem_node_col, en_col.data(), en_bytes, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
      // first touches in colour order (colours run in order, their elements
      // share no node), and whether every node is touched at all
      c->first_words = (npe + 31) / 32;
      std::vector<uint32_t> first((size_t)mesh->n_elem * c->first_words, 0u);
      std::vector<uint8_t> seen(mesh->n_node, 0);
      for (int64_t j = 0; j < mesh->n_elem; ++j)
        for (int l = 0; l < npe; ++l) {
          const int32_t I = en_col[(size_t)j * npe + l];
          if (!seen[I]) {
            seen[I] = 1;
            first[(size_t)j * c->first_words + l / 32] |= 1u << (l % 32);
          }
        }
      c->all_touched = std::all_of(seen.begin(), seen.end(), [](uint8_t b) { return b != 0; });
      const size_t fb = first.size() * sizeof(uint32_t);
      if (hipMalloc(&c->d_first, fb) != hipSuccess) { st = TMOP_E_NOMEM; break; }
      if (hipMemcpy(c->d_first, first.data(), fb, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
    }
    if (per_qp) {   // per-point sizes, element order and colour order
      const size_t tb = (size_t)mesh->n_elem * nq * sizeof(double);
      if (hipMalloc(&c->d_tsize, tb) != hipSuccess) { c->d_tsize = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMalloc(&c->d_tsize_col, tb) != hipSuccess) { c->d_tsize_col = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMemcpy(c->d_tsize, target->W, tb, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
      if (gather_rows(c->d_tsize, c->d_colors, mesh->n_elem, nq, c->d_tsize_col, nullptr) != hipSuccess ||
          hipDeviceSynchronize() != hipSuccess) { st = TMOP_E_HIP; break; }
    }
    if (gen_tgt) {  // general targets and their penalty sizes, element order and colour order
      c->ptgt_elem = kind == TMOP_TGT_PER_ELEM;
      c->ptgt_stride = ts;
      const size_t pb = ptgt.size() * sizeof(double), sb = psize.size() * sizeof(double);
      const int width = (c->ptgt_elem ? 1 : nq) * ts;
      if (hipMalloc(&c->d_ptgt, pb) != hipSuccess) { c->d_ptgt = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMalloc(&c->d_ptgt_col, pb) != hipSuccess) { c->d_ptgt_col = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMalloc(&c->d_psize, sb) != hipSuccess) { c->d_psize = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMalloc(&c->d_psize_col, sb) != hipSuccess) { c->d_psize_col = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMemcpy(c->d_ptgt, ptgt.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->d_psize, psize.data(), sb, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
      if (gather_rows(c->d_ptgt, c->d_colors, mesh->n_elem, width, c->d_ptgt_col, nullptr) != hipSuccess ||
          gather_rows(c->d_psize, c->d_colors, mesh->n_elem, nq, c->d_psize_col, nullptr) != hipSuccess ||
          hipDeviceSynchronize() != hipSuccess) { st = TMOP_E_HIP; break; }
    }
    const int64_t evec_limit =
        precision == TMOP_MIXED_FP32 ? EVEC_DEFAULT_ELEMS_PER_COLOUR_MIXED : EVEC_DEFAULT_ELEMS_PER_COLOUR;
    if (d == 2 || mesh->n_elem <= evec_limit * (int64_t)(c->color_off.size() - 1)) {
      // the element vector, one launch over every element: the 2D default (faster than the tiles, whose
      // workgroups run their tile's colours one after the other) and that of 3D meshes whose colours
      // cannot fill the chip
      const int r = make_evec(c, mesh->elem_node);
      if (r == TMOP_OK) c->scatter = TMOP_SCATTER_ELEMENTS;
      else if (r != TMOP_E_UNSUPPORTED) { st = r; break; }
    }
    std::vector<double> mask(c->n_dof, 1.0);
    if (mesh->fixed)
      for (int64_t k = 0; k < c->n_dof; ++k)
        if (mesh->fixed[k]) { mask[k] = 0.0; c->has_fixed = true; }
    c->n_free = 0;
    for (int64_t k = 0; k < c->n_dof; ++k) c->n_free += mask[k] > 0.0;
    if (hipMemcpy(c->d_mask, mask.data(), c->n_dof * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
    {
      std::vector<uint8_t> m8(c->n_dof);
      for (int64_t k = 0; k < c->n_dof; ++k) m8[k] = mask[k] > 0.0 ? 1 : 0;
      if (hipMalloc(&c->d_mask8, c->n_dof) != hipSuccess) { c->d_mask8 = nullptr; st = TMOP_E_NOMEM; break; }
      if (hipMemcpy(c->d_mask8, m8.data(), c->n_dof, hipMemcpyHostToDevice) != hipSuccess) { st = TMOP_E_HIP; break; }
    }
  } while (0);
  if (st != TMOP_OK) { free_ctx(c); return st; }
  *out = c;
  return TMOP_OK;
}

void tmop_destroy(tmop_ctx* c) { free_ctx(c); }

int tmop_timing_enable(tmop_ctx* c, int enable) {
  if (!c) return TMOP_E_ARG;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(c->device) != hipSuccess) return TMOP_E_HIP;
  const int st = collect_timing(c);
  (void)hipSetDevice(cur);
  c->timing = enable != 0;
  for (int k = 0; k < TIMING_SLOTS; ++k) {
    c->t_ms[k] = 0.0;
    c->t_launches[k] = 0;
  }
  return st;
}

int tmop_timing_read(tmop_ctx* c, int op, double* ms_total, int64_t* launches) {
  if (!c || op < 0 || op >= TIMING_SLOTS || !ms_total || !launches) return TMOP_E_ARG;
  const int st = collect_timing(c);
  *ms_total = c->t_ms[op];
  *launches = c->t_launches[op];
  return st;
}

int tmop_energy_noalloc(tmop_ctx* c, const double* x, double* F, double* min_detA, void* stream) {
  if (!c || !x || !F || !min_detA) return TMOP_E_ARG;
  if (!c->d_noalloc) return TMOP_E_HIP;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return TMOP_E_HIP;
  if (cur != c->device) return TMOP_E_ARG;     // the scratch address belongs to the context's device
  hipStream_t s = (hipStream_t)stream;
  // count the workgroups of every term first: the partials must fit
  RedDst rd{c->d_noalloc, NOALLOC_MAX_BLOCKS, c->d_noalloc + 2 * NOALLOC_MAX_BLOCKS,
            c->d_noalloc + 2 * NOALLOC_MAX_BLOCKS + 2 * FIN_BLOCKS, true};
  int64_t nb = 0;
  int r = energy_async(c, x, s, &rd, &nb);
  if (r != TMOP_OK) return r;
  if (nb > NOALLOC_MAX_BLOCKS) return TMOP_E_SCRATCH;
  // every partial is written before it is read: nothing needs clearing
  rd.dry = false;
  if ((r = energy_async(c, x, s, &rd)) != TMOP_OK) return r;
  HIP_TRY(hipMemcpyAsync(c->h_res, rd.res, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *F = c->h_res[0];
  *min_detA = c->h_res[1];
  return *min_detA > 0.0 ? TMOP_OK : TMOP_W_INVERTED;
}

int tmop_energy(tmop_ctx* c, const double* x, double* F, double* min_detA, void* stream) {
  if (!c || !x || !F || !min_detA) return TMOP_E_ARG;
  double f = 0, m = 0;
  const int r = energy_sync(c, x, (hipStream_t)stream, &f, &m);
  if (r != TMOP_OK) return r;
  *F = f;
  *min_detA = m;
  return m > 0.0 ? TMOP_OK : TMOP_W_INVERTED;
}

int tmop_gradient(tmop_ctx* c, const double* x, double* g, void* stream) {
  if (!c || !x || !g || g == x) return TMOP_E_ARG;
  return assemble(c, OP_GRAD, x, nullptr, g, (hipStream_t)stream);
}

int tmop_gradient_scaled(tmop_ctx* c, const double* x, const double* scale, double* g, void* stream) {
  if (!c || !x || !g || g == x) return TMOP_E_ARG;
  return assemble(c, OP_GRAD, x, nullptr, g, (hipStream_t)stream, scale);
}

int tmop_energy_gradient(tmop_ctx* c, const double* x, double* F, double* min_detA, double* g, void* stream) {
  if (!c || !x || !F || !min_detA || !g || g == x) return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int r = energy_gradient_async(c, x, g, s);
  if (r != TMOP_OK) return r;
  double f = 0, m = 0;
  if ((r = read_res(c, s, &f, &m)) != TMOP_OK) return r;
  *F = f;
  *min_detA = m;
  return m > 0.0 ? TMOP_OK : TMOP_W_INVERTED;
}

int tmop_hessian_apply(tmop_ctx* c, const double* x, const double* v, double* Hv, void* stream) {
  if (!c || !x || !v || !Hv || Hv == x || Hv == v) return TMOP_E_ARG;
  return assemble(c, OP_HESS, x, v, Hv, (hipStream_t)stream);
}

int tmop_target_sizes_w3(tmop_ctx* c, const double* x0, double* sizes, void* stream) {
  if (!c || !x0 || !sizes || sizes == x0) return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int grid = 0;
  const int r = elem_launch(c, OP_SIZE, x0, nullptr, sizes, c->d_elem_node, nullptr, c->n_elem, s, &grid, nullptr, 0,
                            nullptr, c->d_tsize);
  if (r != TMOP_OK) return r;
  HIP_TRY(finalize_sum_min(c->d_part, grid, (int)c->part_cap, c->d_scratch, c->d_res, s));
  double F = 0, m = 0;
  const int st = read_res(c, s, &F, &m);
  if (st != TMOP_OK) return st;
  return m > 0.0 ? TMOP_OK : TMOP_W_INVERTED;
}

int tmop_set_target_sizes(tmop_ctx* c, const double* sizes, void* stream) {
  if (!c || !sizes) return TMOP_E_ARG;
  if (!c->d_tsize) return TMOP_E_ARG;                    // not a per-point target context
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = c->n_elem * c->nq;
  if (n > INT32_MAX) return TMOP_E_ARG;
  // Section 3.1: det W = s^d > 0 at every point, checked before anything changes
  HIP_TRY(finalize_sum_min(sizes, (int)n, 0, c->d_scratch, c->d_res, s));
  double sum = 0, m = 0;
  const int st = read_res(c, s, &sum, &m);
  if (st != TMOP_OK) return st;
  if (!(m > 0.0) || !std::isfinite(sum)) return TMOP_E_TARGET;
  HIP_TRY(hipMemcpyAsync(c->d_tsize, sizes, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(gather_rows(c->d_tsize, c->d_colors, c->n_elem, c->nq, c->d_tsize_col, s));
  return TMOP_OK;
}

int tmop_set_restriction(tmop_ctx* c, double delta, const double* x_init, void* stream) {
  if (!c || !(delta >= 0.0) || !std::isfinite(delta)) return TMOP_E_ARG;
  if (delta == 0.0) {          // Section 4.3.1 with delta = 0: the plain objective
    c->delta = 0.0;
    return TMOP_OK;
  }
  if (!x_init) return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!c->d_xinit && hipMalloc(&c->d_xinit, c->n_dof * sizeof(double)) != hipSuccess) {
    c->d_xinit = nullptr;
    return TMOP_E_NOMEM;
  }
  HIP_TRY(hipMemcpyAsync(c->d_xinit, x_init, c->n_dof * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  // 1D mass matrix of the quadrature, for the kernels that fuse the penalty
  for (int i = 0; i <= c->p; ++i)
    for (int j = 0; j <= c->p; ++j) {
      double m = 0.0;
      for (int q = 0; q < c->Q; ++q) m += c->base.w[q] * c->base.B[q][i] * c->base.B[q][j];
      c->base.M1[i][j] = m;
    }
  c->delta = delta;
  return TMOP_OK;
}

namespace {

bool metric_2d(int m) {
  return m == TMOP_MU1 || m == TMOP_MU2 || m == TMOP_MU7 || m == TMOP_MU9 || m == TMOP_MU14 || m == TMOP_MU77 ||
         m == TMOP_MU98;
}

// Installs per-point second-term data (element order, device; ts values
// per point) as the context's second metric term: its colour-order copy,
// then the switch.
int install_second_term(tmop_ctx* c, int metric2, double* d_tm, int ts, double eta1, hipStream_t s) {
  if (c->d_tmat_col && ts != c->tm_stride) {   // the colour-order copy has another size
    if (hipStreamSynchronize(s) != hipSuccess) {
      (void)hipFree(d_tm);
      return TMOP_E_HIP;
    }
    c->metric2 = 0;
    (void)hipFree(c->d_tmat_col);
    c->d_tmat_col = nullptr;
  }
  if (!c->d_tmat_col && hipMalloc(&c->d_tmat_col, (size_t)c->n_elem * c->nq * ts * sizeof(double)) != hipSuccess) {
    c->d_tmat_col = nullptr;
    c->metric2 = 0;
    (void)hipFree(d_tm);
    return TMOP_E_NOMEM;
  }
  if (gather_rows(d_tm, c->d_colors, c->n_elem, c->nq * ts, c->d_tmat_col, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    c->metric2 = 0;   // the colour-order copy may be half overwritten
    (void)hipFree(d_tm);
    return TMOP_E_HIP;
  }
  (void)hipFree(c->d_tmat);
  c->d_tmat = d_tm;
  c->tm_stride = ts;
  c->metric2 = metric2;
  c->base.wdetW = eta1 * c->base.detW;
  return TMOP_OK;
}

}  // namespace

int tmop_set_combo(tmop_ctx* c, int32_t metric2, const double* W2, double eta1, double eta2, const double* eta2_q,
                   void* stream) {
  if (!c || !(eta1 >= 0.0) || !std::isfinite(eta1)) return TMOP_E_ARG;
  if (c->d_tsize || c->d_ptgt) return TMOP_E_UNSUPPORTED;   // per-point targets carry their own weights
  if (metric2 == 0) {          // back to the single term eta_1 mu
    c->metric2 = 0;
    c->base.wdetW = eta1 * c->base.detW;
    return TMOP_OK;
  }
  const int d = c->dim;
  const bool metric_ok =
      d == 2 ? metric_2d(metric2) : (metric2 == TMOP_MU302 || metric2 == TMOP_MU303 || metric2 == TMOP_MU7);
  if (!metric_ok || !W2 || !(eta2 >= 0.0) || !std::isfinite(eta2)) return TMOP_E_ARG;
  const double det2 = det3(W2, d);
  if (!(det2 > 0.0)) return TMOP_E_TARGET;               // Section 3.1: det W > 0
  const int64_t n = c->n_elem * c->nq;
  if (eta2_q)
    for (int64_t k = 0; k < n; ++k)
      if (!(eta2_q[k] >= 0.0) || !std::isfinite(eta2_q[k])) return TMOP_E_ARG;
  // W2 is constant: per point only its weight omega_q = eta_2 eta_2(q) det W2
  std::vector<double> tm((size_t)n);
  for (int64_t k = 0; k < n; ++k) tm[(size_t)k] = eta2 * (eta2_q ? eta2_q[k] : 1.0) * det2;
  hipStream_t s = (hipStream_t)stream;
  double* d_tm = nullptr;
  if (hipMalloc(&d_tm, tm.size() * sizeof(double)) != hipSuccess) return TMOP_E_NOMEM;
  if (hipMemcpyAsync(d_tm, tm.data(), tm.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipFree(d_tm);
    return TMOP_E_HIP;
  }
  const int r = install_second_term(c, d == 3 && metric2 == TMOP_MU7 ? MU7_3D : metric2, d_tm, 1, eta1, s);
  if (r == TMOP_OK) {
    double Wi[3][3];
    inv3(W2, d, Wi);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) c->W2inv[i][j] = i < d && j < d ? Wi[i][j] : 0.0;
  }
  return r;
}

int tmop_set_replication(tmop_ctx* c, double gamma, const double* x_init, void* stream) {
  if (!c || !x_init || !(gamma >= 0.0 && gamma <= 1.0)) return TMOP_E_ARG;
  if (c->d_tsize || c->d_ptgt) return TMOP_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  double* d_tm = nullptr;
  const int ts = c->dim * c->dim + 1;
  if (hipMalloc(&d_tm, (size_t)c->n_elem * c->nq * ts * sizeof(double)) != hipSuccess) return TMOP_E_NOMEM;
  // W_0 = A(x_init) at every point; both parts weigh with the primary det W
  int grid = 0;
  int r = elem_launch(c, OP_JINV, x_init, nullptr, d_tm, c->d_elem_node, nullptr, c->n_elem, s, &grid, nullptr, 0,
                      nullptr, nullptr, [&] { TermSel t; t.omega = (1.0 - gamma) * c->base.detW; return t; }());
  double F = 0, m = 0;
  if (r == TMOP_OK) {
    r = finalize_sum_min(c->d_part, grid, (int)c->part_cap, c->d_scratch, c->d_res, s) == hipSuccess ? TMOP_OK
                                                                                                      : TMOP_E_HIP;
  }
  if (r == TMOP_OK) r = read_res(c, s, &F, &m);
  if (r == TMOP_OK && !(m > 0.0)) r = TMOP_E_TARGET;     // W_0 needs det A(x_init) > 0
  if (r != TMOP_OK) {
    (void)hipFree(d_tm);
    return r;
  }
  return install_second_term(c, c->dim == 2 ? TMOP_MU98 : MU98_3D, d_tm, ts, gamma, s);
}

namespace {

// Node colouring and node -> element adjacency of the derivative-free
// solver.  Greedy in node order: node I takes the smallest colour not used
// by a node that shares an element with it.
int dfo_prepare(tmop_ctx* c) {
  if (c->dfo_ready) return TMOP_OK;
  const int npe = c->npe;
  const int64_t ne_tot = c->n_elem * npe;
  std::vector<int32_t> en((size_t)ne_tot);
  HIP_TRY(hipMemcpy(en.data(), c->d_elem_node, ne_tot * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int32_t> off(c->n_node + 1, 0), code((size_t)ne_tot);
  for (int64_t k = 0; k < ne_tot; ++k) off[en[k] + 1]++;
  // every element holding a node must fit in that node's workgroup
  const int cap = dfo_patch_capacity(c->dim, c->Q);
  for (int64_t I = 0; I < c->n_node; ++I)
    if (off[I + 1] > cap) return TMOP_E_UNSUPPORTED;
  for (int64_t I = 0; I < c->n_node; ++I) off[I + 1] += off[I];
  {
    std::vector<int32_t> pos(off.begin(), off.end() - 1);
    for (int64_t e = 0; e < c->n_elem; ++e)   // ascending element ids per node
      for (int l = 0; l < npe; ++l) code[pos[en[e * npe + l]]++] = (int32_t)(e * npe + l);
  }
  std::vector<int32_t> colour(c->n_node, -1), mark;
  int ncol = 0;
  for (int64_t I = 0; I < c->n_node; ++I) {
    for (int32_t k = off[I]; k < off[I + 1]; ++k) {
      const int64_t e = code[k] / npe;
      for (int l = 0; l < npe; ++l) {
        const int32_t cj = colour[en[e * npe + l]];
        if (cj >= 0) mark[cj] = (int32_t)I;
      }
    }
    int col = 0;
    while (col < (int)mark.size() && mark[col] == (int32_t)I) ++col;
    if (col == (int)mark.size()) mark.push_back(-1);
    colour[I] = col;
    ncol = std::max(ncol, col + 1);
  }
  std::vector<int32_t> order;
  order.reserve(c->n_node);
  c->dfo_col_off.assign(1, 0);
  {
    std::vector<std::vector<int32_t>> by(ncol);
    for (int64_t I = 0; I < c->n_node; ++I) by[colour[I]].push_back((int32_t)I);
    for (auto& v : by) {
      order.insert(order.end(), v.begin(), v.end());
      c->dfo_col_off.push_back((int64_t)order.size());
    }
  }
  auto release = [c]() {
    for (void** p : {(void**)&c->d_dfo_nodes, (void**)&c->d_ne_off, (void**)&c->d_ne, (void**)&c->d_dfo_move}) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  };
  if (hipMalloc(&c->d_dfo_nodes, order.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_ne_off, off.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_ne, code.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_dfo_move, c->n_node * sizeof(double)) != hipSuccess) {
    release();
    return TMOP_E_NOMEM;
  }
  if (hipMemcpy(c->d_dfo_nodes, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_ne_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_ne, code.data(), code.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    release();
    return TMOP_E_HIP;
  }
  c->dfo_ready = true;
  return TMOP_OK;
}

bool dfo_opts_ok(const tmop_dfo_opts& o) {
  return o.t >= 0.0 && std::isfinite(o.t) && o.max_sweeps >= 0 && o.step > 0.0 && std::isfinite(o.step) &&
         o.xtol >= 0.0 && std::isfinite(o.xtol) && o.max_evals >= 1;
}

int dfo_sweep(tmop_ctx* c, double* x, const tmop_dfo_opts& o, hipStream_t s, double* max_move) {
  int st = dfo_prepare(c);
  if (st != TMOP_OK) return st;
  DfoParams dp{};
  dp.x = x;
  dp.mask = c->d_mask;
  dp.ne_off = c->d_ne_off;
  dp.ne = c->d_ne;
  dp.elem_node = c->d_elem_node;
  dp.n_node = c->n_node;
  dp.max_evals = o.max_evals;
  for (int q = 0; q < MAXQ; ++q) {
    dp.w[q] = c->base.w[q];
    for (int i = 0; i < MAXP; ++i) { dp.B[q][i] = c->base.B[q][i]; dp.G[q][i] = c->base.G[q][i]; }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) dp.Winv[i][j] = c->base.Winv[i][j];
  dp.detW = c->base.detW;
  dp.step = o.step * std::pow(c->base.detW, 1.0 / c->dim);   // in units of the target size
  dp.xtol = o.xtol;
  for (size_t k = 0; k + 1 < c->dfo_col_off.size(); ++k) {
    const int64_t a = c->dfo_col_off[k], n = c->dfo_col_off[k + 1] - a;
    dp.nodes = c->d_dfo_nodes + a;
    dp.move = c->d_dfo_move + a;
    dp.n_list = (int32_t)n;
    const int r = launch_dfo(c->dim, c->p, c->Q, c->metric, dp, s);
    if (r == -1) return TMOP_E_UNSUPPORTED;
    if (r != 0) return TMOP_E_HIP;
  }
  HIP_TRY(finalize_sum_min(c->d_dfo_move, (int)c->n_node, 0, c->d_scratch, c->d_res, s));
  double sum = 0, m = 0;
  if ((st = read_res(c, s, &sum, &m)) != TMOP_OK) return st;
  *max_move = -m;
  return TMOP_OK;
}

}  // namespace

void tmop_dfo_default_opts(tmop_dfo_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->t = 1e-5;
  o->max_sweeps = 100;
  o->step = 0.1;
  o->xtol = 1e-6;
  o->max_evals = 200;
}

int tmop_dfo_sweep(tmop_ctx* c, double* x, const tmop_dfo_opts* opts, double* max_move, void* stream) {
  if (!c || !x || !max_move) return TMOP_E_ARG;
  tmop_dfo_opts o;
  if (opts) o = *opts;
  else tmop_dfo_default_opts(&o);
  if (!dfo_opts_ok(o)) return TMOP_E_ARG;
  if (c->d_tsize || c->d_ptgt || c->metric2 || c->delta > 0.0) return TMOP_E_UNSUPPORTED;
  return dfo_sweep(c, x, o, (hipStream_t)stream, max_move);
}

int tmop_dfo_solve(tmop_ctx* c, double* x, const tmop_dfo_opts* opts, tmop_dfo_report* rep, void* stream) {
  if (!c || !x) return TMOP_E_ARG;
  tmop_dfo_opts o;
  if (opts) o = *opts;
  else tmop_dfo_default_opts(&o);
  if (!dfo_opts_ok(o)) return TMOP_E_ARG;
  if (c->d_tsize || c->d_ptgt || c->metric2 || c->delta > 0.0) return TMOP_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  tmop_dfo_report r{};
  double F = 0, m = 0;
  int st = energy_sync(c, x, s, &F, &m);
  if (st != TMOP_OK) return st;
  r.F0 = r.F = F;
  if (!(m > 0.0)) {
    if (rep) *rep = r;
    return TMOP_W_INVERTED;
  }
  for (int k = 0; k < o.max_sweeps; ++k) {
    double mv = 0;
    if ((st = dfo_sweep(c, x, o, s, &mv)) != TMOP_OK) return st;
    r.sweeps = k + 1;
    r.max_move = mv;
    if (mv < o.t) {
      r.converged = 1;
      break;
    }
  }
  if ((st = energy_sync(c, x, s, &F, &m)) != TMOP_OK) return st;
  r.F = F;
  if (rep) *rep = r;
  return r.converged ? TMOP_OK : TMOP_W_MAXIT;
}

int tmop_set_scatter(tmop_ctx* c, int32_t mode) {
  if (!c || (mode != TMOP_SCATTER_COLOURS && mode != TMOP_SCATTER_TILES && mode != TMOP_SCATTER_ELEMENTS))
    return TMOP_E_ARG;
  if (mode == TMOP_SCATTER_TILES && !c->tile.node) {   // built on first use, 2D only
    if (c->dim != 2) return TMOP_E_UNSUPPORTED;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    HIP_TRY(hipSetDevice(c->device));
    std::vector<int32_t> en((size_t)c->n_elem * c->npe), order((size_t)c->n_elem);
    int r = hipMemcpy(en.data(), c->d_elem_node, en.size() * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess &&
                    hipMemcpy(order.data(), c->d_colors, order.size() * sizeof(int32_t), hipMemcpyDeviceToHost) ==
                        hipSuccess
                ? make_tiles(c, en.data(), order)
                : TMOP_E_HIP;
    (void)hipSetDevice(cur);
    if (r != TMOP_OK) return r;   // TMOP_E_UNSUPPORTED: a mesh beyond the tile limits
  }
  if (mode == TMOP_SCATTER_ELEMENTS) {
    if (!c->d_evec) {
      int cur = 0;
      HIP_TRY(hipGetDevice(&cur));
      HIP_TRY(hipSetDevice(c->device));
      std::vector<int32_t> en((size_t)c->n_elem * c->npe);
      int r = hipMemcpy(en.data(), c->d_elem_node, en.size() * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess
                  ? make_evec(c, en.data())
                  : TMOP_E_HIP;
      (void)hipSetDevice(cur);
      if (r != TMOP_OK) return r;
    }
  }
  c->scatter = mode;
  return TMOP_OK;
}

int tmop_get_scatter(const tmop_ctx* c, int32_t* mode) {
  if (!c || !mode) return TMOP_E_ARG;
  *mode = c->scatter;
  return TMOP_OK;
}

int tmop_hessian_diagonal(tmop_ctx* c, const double* x, double* diag, void* stream) {
  if (!c || !x || !diag || diag == x) return TMOP_E_ARG;
  return assemble(c, OP_DIAG, x, nullptr, diag, (hipStream_t)stream);
}

int tmop_newton_solve(tmop_ctx* c, double* x, const tmop_newton_opts* opts_in, tmop_newton_report* rep_out,
                      void* stream) {
  if (!c || !x) return TMOP_E_ARG;
  tmop_newton_opts o;
  if (opts_in) o = *opts_in;
  else tmop_newton_default_opts(&o);
  if (o.max_it < 0 || o.cg_max_it < 1 || o.ls_max < 0 || !(o.ls_shrink > 0.0 && o.ls_shrink < 1.0))
    return TMOP_E_ARG;
  if ((o.inner != TMOP_INNER_CG && o.inner != TMOP_INNER_MINRES && o.inner != TMOP_INNER_SHIFTED_CG) ||
      (o.precond != TMOP_PREC_NONE && o.precond != TMOP_PREC_JACOBI) ||
      (o.inner == TMOP_INNER_SHIFTED_CG && !(o.shift_beta > 0.0 && std::isfinite(o.shift_beta))))
    return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  };
  const int64_t N = c->n_dof;
  if (!c->d_work) {
    if (hipMalloc(&c->d_work, (size_t)NEWTON_VECTORS * N * sizeof(double)) != hipSuccess) {
      c->d_work = nullptr;
      return TMOP_E_NOMEM;
    }
  }
  if (!c->d_sc) {
    if (hipMalloc(&c->d_sc, SC_COUNT * sizeof(double)) != hipSuccess) {
      c->d_sc = nullptr;
      return TMOP_E_NOMEM;
    }
  }
  if (!c->h_sc) {
    if (hipHostMalloc(&c->h_sc, SC_COUNT * sizeof(double), 0) != hipSuccess) {
      c->h_sc = nullptr;
      return TMOP_E_NOMEM;
    }
  }
  double* g = c->d_work;          // masked gradient at x
  double* xt = g + N;             // trial point
  double* gt = xt + N;            // masked gradient at the trial point
  Inner w;
  w.d = gt + N;                   // search direction
  w.minv = w.d + N;               // 1 / diag of the Jacobi preconditioner
  for (int k = 0; k < 7; ++k) w.v[k] = w.minv + (k + 1) * N;   // solver vectors

  tmop_newton_report rep;
  memset(&rep, 0, sizeof(rep));
  int st;
  double F, mind;
  if ((st = energy_gradient_async(c, x, g, s)) != TMOP_OK) return st;
  if ((st = read_res(c, s, &F, &mind)) != TMOP_OK) return st;
  rep.F0 = rep.F = F;
  rep.min_detA = mind;
  if (!(mind > 0.0)) {
    if (rep_out) *rep_out = rep;
    return TMOP_W_INVERTED;
  }
  HIP_TRY(mask_mul(c->d_mask, g, N, s));
  double gg;
  if ((st = dot_sync(c, g, g, s, &gg)) != TMOP_OK) return st;
  double gn = sqrt(gg);
  rep.gnorm0 = rep.gnorm = gn;
  if (o.hist_F) o.hist_F[0] = F;
  if (o.hist_gnorm) o.hist_gnorm[0] = gn;
  if (o.hist_cg) o.hist_cg[0] = 0;
  if (o.hist_time) o.hist_time[0] = elapsed();

  int status = TMOP_W_MAXIT;
  const double gtol = std::max(o.rtol * rep.gnorm0, o.atol);
  for (int it = 0;; ++it) {
    if (gn <= gtol || F <= o.ftarget) { status = TMOP_OK; break; }
    if (it >= o.max_it) { status = TMOP_W_MAXIT; break; }
    double cg_tol = o.cg_rtol;
    if (o.cg_forcing) cg_tol = std::max(o.cg_rtol, std::min(0.5, sqrt(gn / rep.gnorm0)));
    const double* minv = nullptr;
    double* diag = w.v[6];               // the shifted CG uses w.v[0..3]; MINRES overwrites it later
    if (o.precond == TMOP_PREC_JACOBI || o.inner == TMOP_INNER_SHIFTED_CG)
      if ((st = assemble(c, OP_DIAG, x, nullptr, diag, s)) != TMOP_OK) return st;
    if (o.precond == TMOP_PREC_JACOBI) {   // M = |diag H| at x on the free DOFs
      HIP_TRY(hipMemcpyAsync(w.minv, diag, N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIP_TRY(jacobi_inv(c->d_mask, w.minv, N, s));
      minv = w.minv;
    }
    int ncg = 0;
    if (o.inner == TMOP_INNER_MINRES) {
      st = inner_minres(c, x, g, cg_tol, o.cg_max_it, minv, w, s, &ncg);
    } else if (o.inner == TMOP_INNER_SHIFTED_CG) {
      int nrestart = 0;
      st = inner_shifted_cg(c, x, g, gn, cg_tol, o.cg_max_it, minv, diag, o.shift_beta, w, s, &ncg, &nrestart);
      rep.neg_curv += nrestart;
    } else {
      bool neg = false;
      st = inner_tcg(c, x, g, gn, cg_tol, o.cg_max_it, minv, w, s, &ncg, &neg);
      if (neg) rep.neg_curv++;
    }
    if (st != TMOP_OK) return st;
    rep.cg_iters += ncg;
    // ---- line search (Section 3.4): det A > 0, F and |g| growth below 1.2x
    bool accepted = false;
    double Ft = 0, mindt = 0, ggt = 0;
    double alpha = 1.0;
    for (int k = 0; k < o.ls_max; ++k) {
      HIP_TRY(waxpy(x, alpha, w.d, xt, N, s));
      // F, det A and g at the trial point in one pass (g is used only when
      // the first two tests pass)
      if ((st = energy_gradient_async(c, xt, gt, s)) != TMOP_OK) return st;
      if ((st = read_res(c, s, &Ft, &mindt)) != TMOP_OK) return st;
      if (mindt > 0.0 && Ft < o.f_growth * F) {
        HIP_TRY(mask_mul(c->d_mask, gt, N, s));
        if ((st = dot_sync(c, gt, gt, s, &ggt)) != TMOP_OK) return st;
        if (sqrt(ggt) < o.g_growth * gn) { accepted = true; break; }
      }
      rep.ls_shrinks++;
      alpha *= o.ls_shrink;
    }
    if (!accepted) { status = TMOP_W_LSFAIL; break; }
    HIP_TRY(hipMemcpyAsync(x, xt, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(g, gt, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    F = Ft;
    mind = mindt;
    gg = ggt;
    gn = sqrt(ggt);
    rep.iters = it + 1;
    if (o.hist_F) o.hist_F[it + 1] = F;
    if (o.hist_gnorm) o.hist_gnorm[it + 1] = gn;
    if (o.hist_cg) o.hist_cg[it + 1] = ncg;
    if (o.hist_time) o.hist_time[it + 1] = elapsed();
  }
  HIP_TRY(hipStreamSynchronize(s));
  rep.F = F;
  rep.gnorm = gn;
  rep.min_detA = mind;
  if (rep_out) *rep_out = rep;
  return status;
}

}  // extern "C"

namespace tmop {
bool elem_supported(int dim, int p, int Q) {
  (void)dim;
  return p >= 1 && p <= 4 && (Q == p + 1 || Q == p + 2);
}
}  // namespace tmop
