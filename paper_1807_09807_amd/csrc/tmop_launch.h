// Instantiation and dispatch of the element kernels for one dimension and
// one arithmetic type.  Included by one translation unit per (dim, type) so
// the instantiations compile in parallel.
#pragma once

#include <type_traits>

#include "tmop_elem.h"
#include "tmop_internal.h"

namespace tmop {

template <int DIM, int P, int Q, int METRIC, typename R, int OP, int TGT, bool PEN = false>
static int launch_one(const LaunchParams& lp, hipStream_t s, int* grid) {
  using C = Cfg<DIM, P, Q, R>;
  DiagArgs<P, Q, R> a;   // the element kernels take its ElemArgs part
  a.x = lp.x; a.v = lp.v; a.out = lp.out;
  a.elem_node = lp.elem_node; a.list = lp.list; a.first = lp.first; a.part = lp.part; a.part_min = lp.part_min; a.scale = lp.scale;
  a.n_node = lp.n_node; a.n_list = lp.n_list;
  a.tsize = lp.tsize;
  a.tmat = lp.tmat;
  a.tm_el = lp.tm_el;
  a.tm_pt = lp.tm_pt;
  a.wdetW = lp.wdetW;
  a.kpen = lp.kpen;
  a.evec = (OP == OP_GRAD || OP == OP_EG || OP == OP_HESS || OP == OP_DIAG) ? static_cast<R*>(lp.evec) : nullptr;
  if (a.evec && lp.evec_esize != (int)sizeof(R)) return -1;   // the vector holds the kernels' arithmetic type
  a.evpos = lp.evpos;
  a.n_ent = lp.n_ent;
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) a.M1[i][j] = lp.M1[i][j];
  const double gs = TGT == TGT_ISO ? lp.s_inv : 1.0;   // constant isotropic target: G carries 1/s
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
  if constexpr (DIM == 2 && (OP == OP_GRAD || OP == OP_EG || OP == OP_HESS)) {
    if (lp.tile) {   // owner-computes tiles: one workgroup per tile, then the halo sums
      const TileParams& tp = *lp.tile;
      *grid = tp.n_tile;
      if (tp.n_tile == 0 || lp.dry) return 0;
      const bool split = tile_can_split((int)sizeof(R), OP == OP_HESS) && tp.split;
      const int64_t lds = tile_lds_bytes(P, Q, (int)sizeof(R), split, tp.nn_max);
      if (lds > TILE_LDS_BYTES) return -2;
      const ElemArgs<P, Q, R>& ea = a;
      hipLaunchKernelGGL((tile_kernel_2d<P, Q, METRIC, R, OP, TGT>), dim3(tp.n_tile), dim3(TILE_BLOCK), (size_t)lds, s,
                         ea, tp);
      if (hipGetLastError() != hipSuccess) return -2;
      return halo_sum(tp, lp.n_node, lp.out, s) == hipSuccess ? 0 : -2;
    }
  }
  if (lp.tile) return -1;
  const int g = (lp.n_list + C::EPB - 1) / C::EPB;
  *grid = g;
  if (g == 0 || lp.dry) return 0;
  if constexpr (OP == OP_DIAG) {
    // products of the 1D tables for the squared gradients of the diagonal
    for (int q = 0; q < Q; ++q)
      for (int i = 0; i < P; ++i) {
        const double b = lp.B[q][i], gg = lp.G[q][i] * gs;
        a.BB[q][i] = (R)(b * b);
        a.BG[q][i] = (R)(b * gg);
        a.GG[q][i] = (R)(gg * gg);
      }
    if constexpr (DIM == 3) {
      if (a.evec) hipLaunchKernelGGL((diag_kernel_3d<P, Q, METRIC, R, TGT, true>), dim3(g), dim3(C::BLOCK), 0, s, a);
      else hipLaunchKernelGGL((diag_kernel_3d<P, Q, METRIC, R, TGT, false>), dim3(g), dim3(C::BLOCK), 0, s, a);
    } else {
      if (a.evec) hipLaunchKernelGGL((diag_kernel_2d<P, Q, METRIC, R, TGT, true>), dim3(g), dim3(C::BLOCK), 0, s, a);
      else hipLaunchKernelGGL((diag_kernel_2d<P, Q, METRIC, R, TGT, false>), dim3(g), dim3(C::BLOCK), 0, s, a);
    }
  } else {
    const ElemArgs<P, Q, R>& ea = a;
    if constexpr (DIM == 3) {
      // the element-vector stores are a separate instantiation: the colour
      // launches' kernels then hold no register for them
      constexpr bool SCATTER = OP == OP_GRAD || OP == OP_EG || OP == OP_HESS;
      if (SCATTER && a.evec)
        hipLaunchKernelGGL((elem_kernel_3d<P, Q, METRIC, R, OP, TGT, PEN, SCATTER>), dim3(g), dim3(C::BLOCK), 0, s, ea);
      else
        hipLaunchKernelGGL((elem_kernel_3d<P, Q, METRIC, R, OP, TGT, PEN, false>), dim3(g), dim3(C::BLOCK), 0, s, ea);
    } else {
      constexpr bool SCATTER = OP == OP_GRAD || OP == OP_EG || OP == OP_HESS;
      if (SCATTER && a.evec)
        hipLaunchKernelGGL((elem_kernel_2d<P, Q, METRIC, R, OP, TGT, SCATTER>), dim3(g), dim3(C::BLOCK), 0, s, ea);
      else
        hipLaunchKernelGGL((elem_kernel_2d<P, Q, METRIC, R, OP, TGT, false>), dim3(g), dim3(C::BLOCK), 0, s, ea);
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// OP_SIZE and OP_JINV do not depend on the metric: they are instantiated
// for the first metric of each dimension only (the caller routes them
// there), OP_JINV for the general constant target (W = I) only.
template <int DIM, int P, int Q, int M, typename R, int TGT>
static int launch_op(int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  // the displacement penalty fused into the 3D FP64 constant-target Hessian action
  if constexpr (DIM == 3 && std::is_same<R, double>::value && (TGT == TGT_ISO || TGT == TGT_GEN) && M != 398) {
    if (lp.pen) return op == OP_HESS ? launch_one<DIM, P, Q, M, R, OP_HESS, TGT, true>(lp, s, grid) : -1;
  }
  if (lp.pen) return -1;
  if (op == OP_ENERGY) return launch_one<DIM, P, Q, M, R, OP_ENERGY, TGT>(lp, s, grid);
  if (op == OP_GRAD) return launch_one<DIM, P, Q, M, R, OP_GRAD, TGT>(lp, s, grid);
  if (op == OP_HESS) return launch_one<DIM, P, Q, M, R, OP_HESS, TGT>(lp, s, grid);
  if (op == OP_EG) return launch_one<DIM, P, Q, M, R, OP_EG, TGT>(lp, s, grid);
  if (op == OP_DIAG) return launch_one<DIM, P, Q, M, R, OP_DIAG, TGT>(lp, s, grid);
  if constexpr (M == (DIM == 2 ? 1 : 302) && TGT != TGT_MAT && TGT != TGT_CW) {
    if (op == OP_SIZE) return launch_one<DIM, P, Q, M, R, OP_SIZE, TGT>(lp, s, grid);
    if constexpr (TGT == TGT_GEN)
      if (op == OP_JINV) return launch_one<DIM, P, Q, M, R, OP_JINV, TGT>(lp, s, grid);
  }
  return -1;
}

template <int DIM, int P, int Q, int M, typename R>
static int launch_metric(int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  if (lp.tmat) {
    if (lp.tms == 1) return launch_op<DIM, P, Q, M, R, TGT_CW>(op, lp, s, grid);
    return launch_op<DIM, P, Q, M, R, TGT_MAT>(op, lp, s, grid);
  }
  if (lp.tsize) return launch_op<DIM, P, Q, M, R, TGT_QPS>(op, lp, s, grid);
  return lp.iso ? launch_op<DIM, P, Q, M, R, TGT_ISO>(op, lp, s, grid) : launch_op<DIM, P, Q, M, R, TGT_GEN>(op, lp, s, grid);
}

// The metrics of each dimension (Table 3.1, Sections 3.2 and 4.3; mu_302 in
// 3D).  The metrics of each dimension come in two groups, instantiated by
// separate translation units so that they compile in parallel.
template <int DIM, int GROUP, int P, int Q, typename R>
static int launch_pq(int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  if (op == OP_SIZE || op == OP_JINV) metric = DIM == 2 ? 1 : 302;
  if constexpr (DIM == 2 && GROUP == 0) {
    switch (metric) {
      case 1: return launch_metric<2, P, Q, 1, R>(op, lp, s, grid);
      case 2: return launch_metric<2, P, Q, 2, R>(op, lp, s, grid);
      case 7: return launch_metric<2, P, Q, 7, R>(op, lp, s, grid);
      case 9: return launch_metric<2, P, Q, 9, R>(op, lp, s, grid);
      default: return -1;
    }
  } else if constexpr (DIM == 2) {
    switch (metric) {
      case 14: return launch_metric<2, P, Q, 14, R>(op, lp, s, grid);
      case 77: return launch_metric<2, P, Q, 77, R>(op, lp, s, grid);
      case 98: return launch_metric<2, P, Q, 98, R>(op, lp, s, grid);
      default: return -1;
    }
  } else if constexpr (GROUP == 0) {
    switch (metric) {
      case 302: return launch_metric<3, P, Q, 302, R>(op, lp, s, grid);
      case 303: return launch_metric<3, P, Q, 303, R>(op, lp, s, grid);
      case 398: return lp.tmat ? launch_op<3, P, Q, 398, R, TGT_MAT>(op, lp, s, grid) : -1;   // replication, 3D
      default: return -1;
    }
  } else {
    switch (metric) {
      case 307: return launch_metric<3, P, Q, 307, R>(op, lp, s, grid);   // mu_7, 3D
      default: return -1;
    }
  }
}

// Orders p = 1..4 with Q = p+1 (the minimum of Section 3.3) and Q = p+2.
template <int DIM, typename R, int GROUP = 0>
static int launch_dispatch(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  const int P = p + 1;
#define TMOP_PQ(P_, Q_) \
  if (P == P_ && Q == Q_) return launch_pq<DIM, GROUP, P_, Q_, R>(metric, op, lp, s, grid);
  TMOP_PQ(2, 2) TMOP_PQ(2, 3)
  TMOP_PQ(3, 3) TMOP_PQ(3, 4)
  TMOP_PQ(4, 4) TMOP_PQ(4, 5)
  TMOP_PQ(5, 5) TMOP_PQ(5, 6)
#undef TMOP_PQ
  return -1;
}

}  // namespace tmop
