// Instantiation and dispatch of the element kernels for one dimension and
// one arithmetic type.  Included by one translation unit per (dim, type) so
// the instantiations compile in parallel.
#pragma once

#include "tmop_elem.h"
#include "tmop_internal.h"

namespace tmop {

template <int DIM, int P, int Q, int METRIC, typename R, int OP, bool ISO>
static int launch_one(const LaunchParams& lp, hipStream_t s, int* grid) {
  using C = Cfg<DIM, P, Q, R>;
  ElemArgs<P, Q, R> a;
  a.x = lp.x; a.v = lp.v; a.out = lp.out;
  a.elem_node = lp.elem_node; a.list = lp.list; a.first = lp.first; a.part = lp.part; a.part_min = lp.part_min; a.scale = lp.scale;
  a.n_node = lp.n_node; a.n_list = lp.n_list;
  const double gs = ISO ? lp.s_inv : 1.0;   // isotropic target: G carries 1/s
  for (int q = 0; q < Q; ++q) {
    a.w[q] = lp.w[q];
    for (int i = 0; i < P; ++i) { a.B[q][i] = (R)lp.B[q][i]; a.G[q][i] = (R)(lp.G[q][i] * gs); }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.Winv[i][j] = (R)lp.Winv[i][j];
  for (int i = 0; i < P; ++i) a.xi[i] = lp.xi[i];
  a.jscale = gs;
  a.detW = lp.detW;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.Winvd[i][j] = lp.Winv[i][j];
  const int g = (lp.n_list + C::EPB - 1) / C::EPB;
  *grid = g;
  if (g == 0) return 0;
  if constexpr (DIM == 3) hipLaunchKernelGGL((elem_kernel_3d<P, Q, METRIC, R, OP, ISO>), dim3(g), dim3(C::BLOCK), 0, s, a);
  else hipLaunchKernelGGL((elem_kernel_2d<P, Q, METRIC, R, OP, ISO>), dim3(g), dim3(C::BLOCK), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <int DIM, int P, int Q, int M, typename R, bool ISO>
static int launch_op(int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  if (op == OP_ENERGY) return launch_one<DIM, P, Q, M, R, OP_ENERGY, ISO>(lp, s, grid);
  if (op == OP_GRAD) return launch_one<DIM, P, Q, M, R, OP_GRAD, ISO>(lp, s, grid);
  if (op == OP_HESS) return launch_one<DIM, P, Q, M, R, OP_HESS, ISO>(lp, s, grid);
  if (op == OP_EG) return launch_one<DIM, P, Q, M, R, OP_EG, ISO>(lp, s, grid);
  return -1;
}

template <int DIM, int P, int Q, typename R>
static int launch_pq(int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  constexpr int M0 = DIM == 2 ? 2 : 302;
  constexpr int M1 = DIM == 2 ? 7 : 303;
  if (metric == M0)
    return lp.iso ? launch_op<DIM, P, Q, M0, R, true>(op, lp, s, grid) : launch_op<DIM, P, Q, M0, R, false>(op, lp, s, grid);
  if (metric == M1)
    return lp.iso ? launch_op<DIM, P, Q, M1, R, true>(op, lp, s, grid) : launch_op<DIM, P, Q, M1, R, false>(op, lp, s, grid);
  return -1;
}

// Orders p = 1..4 with Q = p+1 (the minimum of Section 3.3) and Q = p+2.
template <int DIM, typename R>
static int launch_dispatch(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  const int P = p + 1;
#define TMOP_PQ(P_, Q_) \
  if (P == P_ && Q == Q_) return launch_pq<DIM, P_, Q_, R>(metric, op, lp, s, grid);
  TMOP_PQ(2, 2) TMOP_PQ(2, 3)
  TMOP_PQ(3, 3) TMOP_PQ(3, 4)
  TMOP_PQ(4, 4) TMOP_PQ(4, 5)
  TMOP_PQ(5, 5) TMOP_PQ(5, 6)
#undef TMOP_PQ
  return -1;
}

}  // namespace tmop
