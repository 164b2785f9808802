// Displacement penalty of the first restricted node movement algorithm
// (Section 4.3.1, eq. 4.2): delta |x - x_init|^2 integrated over the target
// elements,
//   E(x) = sum_E sum_q w_q det W_q delta |u(q)|^2,   u = x - x_init,
// with u(q) = sum_i u_i w_i(s_q) the finite element field of eq. 2.1.  E is
// a quadratic form in u with the constant matrix 2 delta M per component
// (M = the target-weighted mass matrix), so
//   dE/dx = 2 delta M u,   (d^2E/dx^2) v = 2 delta M v,
//   diag = 2 delta sum_q w_q det W_q w_i(s_q)^2 (the same for every component).
// The kernels add these to what the element kernels wrote (or, for the
// energy, write their own block sums beside theirs), so they run after them.
//
// Sum factorization with the value table B[q][i] = l_i(s_q) only: three 1D
// passes forward (z, y, x) and three transposed ones back; the diagonal
// runs the transposed passes alone with the squared table BB = B^2.  The
// lane mapping is that of the element kernels: Q*Q lanes per element in 3D
// (lane (a, b)), Q lanes in 2D.  FP64 throughout; the arithmetic per value
// is small, so the kernels are bound by the gather and scatter of the fields.
#include "tmop_elem.h"

namespace tmop {

template <int P, int Q>
struct MassArgs {
  const double* __restrict__ x;      // ENERGY / GRAD / EG: x; HESS: v   [dim][n_node]
  const double* __restrict__ x0;     // ENERGY / GRAD / EG: x_init       [dim][n_node]
  double* __restrict__ out;          // GRAD / HESS / EG / DIAG: out += the term  [dim][n_node]
  const int32_t* __restrict__ elem_node;   // [n_list][P^dim]
  double* __restrict__ part;         // ENERGY / EG: [gridDim.x] block sums
  double* __restrict__ part_min;     // ENERGY / EG: [gridDim.x] +inf (min det A is the element kernels')
  const double* __restrict__ scale;  // GRAD / EG: optional device scalar factor of the gradient
  const double* __restrict__ tsize;  // QPS: [n_list][Q^dim] sizes s_q, det W_q = s_q^dim
  int64_t n_node;
  int32_t n_list;
  double B[Q][P];
  double BB[Q][P];
  double w[Q];
  double k;                          // 2 delta det W (times s_q^dim per point when QPS)
};

template <int DIM, int P, int Q>
struct MassCfg {
  static constexpr int TPE = DIM == 3 ? Q * Q : Q;
  // values per element: 3D U1 [c][i0][i1][q2] and U2 [c][i0][q1][q2]; 2D U1 [c][i0][q1]
  static constexpr int NU1 = DIM == 3 ? 3 * P * P * Q : 2 * P * Q;
  static constexpr int NE = DIM == 3 ? 3 * P * Q * (P + Q) + 1 : 2 * P * Q + 1;
  static constexpr int EPB = pick_epb(TPE, NE * (int)sizeof(double));
  static constexpr int BLOCK = (EPB * TPE + 63) / 64 * 64;
};

template <int P, int Q, int OP, bool QPS>
__global__ void __launch_bounds__((MassCfg<3, P, Q>::BLOCK))
mass_kernel_3d(const MassArgs<P, Q> a) {
  using C = MassCfg<3, P, Q>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P * P, NE = C::NE;
  constexpr bool FWD = OP != OP_DIAG;
  constexpr bool SUM = OP == OP_ENERGY || OP == OP_EG;
  constexpr bool SCATTER = OP != OP_ENERGY;
  constexpr int NC = OP == OP_DIAG ? 1 : 3;   // fields carried by the transposed passes
  __shared__ double s_all[EPB * NE];
  __shared__ double red[2 * (C::BLOCK / 64)];

  const int tid = threadIdx.x;
  const int le_raw = tid / TPE;
  const int le = le_raw < EPB ? le_raw : EPB - 1;
  const int t = tid - le_raw * TPE;
  const int ta = le_raw < EPB ? t % Q : Q;   // idle pad lanes take no part
  const int tb = le_raw < EPB ? t / Q : Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int k = blk * EPB + le;
  const bool active = le_raw < EPB && k < a.n_list;
  const int kk = k < a.n_list ? k : a.n_list - 1;
  double* U1 = s_all + le * NE;              // [c][i0][i1][q2]
  double* U2 = U1 + C::NU1;                  // [c][i0][q1][q2]
  const bool p1 = ta < P && tb < P;          // lane (i0, i1)
  auto u1 = [](int c, int i0, int i1, int q2) { return ((c * P + i0) * P + i1) * Q + q2; };
  auto u2 = [](int c, int i0, int q1, int q2) { return ((c * P + i0) * Q + q1) * Q + q2; };

  const int32_t* en = a.elem_node + (int64_t)kk * NPE;
  int node[P];
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2) node[i2] = p1 ? en[ta + P * tb + P * P * i2] : en[0];
  double old[3][P];
  if constexpr (SCATTER) {
    if (active && p1) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) old[c][i2] = a.out[c * a.n_node + node[i2]];
    }
  }

  if constexpr (FWD) {
    if (p1) {   // z: lane (i0, i1)
      double u[3][P];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) {
          const int64_t j = c * a.n_node + node[i2];
          u[c][i2] = OP == OP_HESS ? a.x[j] : a.x[j] - a.x0[j];
        }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          double v = 0.0;
#pragma unroll
          for (int i2 = 0; i2 < P; ++i2) v += a.B[q2][i2] * u[c][i2];
          U1[u1(c, ta, tb, q2)] = v;
        }
    }
    __syncthreads();
    if (ta < P && tb < Q) {   // y: lane (i0, q2)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double r[P];
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) r[i1] = U1[u1(c, ta, i1, tb)];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          double v = 0.0;
#pragma unroll
          for (int i1 = 0; i1 < P; ++i1) v += a.B[q1][i1] * r[i1];
          U2[u2(c, ta, q1, tb)] = v;
        }
      }
    }
    __syncthreads();
  }

  // x and the point terms: lane (q1, q2)
  double acc = 0.0;
  double Rx[NC][P];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int i0 = 0; i0 < P; ++i0) Rx[c][i0] = 0.0;
  if (tb < Q) {
    const double w12 = a.w[ta] * a.w[tb] * a.k * (a.scale ? *a.scale : 1.0);
    double sq[Q];
    if constexpr (QPS) {
      const double* ts = a.tsize + (int64_t)kk * (Q * Q * Q) + Q * ta + Q * Q * tb;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    double x2[3][P];
    if constexpr (FWD) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) x2[c][i0] = U2[u2(c, i0, ta, tb)];
    }
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      double kq = w12 * a.w[q0];
      if constexpr (QPS) kq *= sq[q0] * sq[q0] * sq[q0];
      if constexpr (FWD) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double uq = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) uq += a.B[q0][i0] * x2[c][i0];
          if constexpr (SUM) acc += 0.5 * kq * uq * uq;
          if constexpr (SCATTER) {
            const double m = kq * uq;
#pragma unroll
            for (int i0 = 0; i0 < P; ++i0) Rx[c][i0] += a.B[q0][i0] * m;
          }
        }
      } else {
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) Rx[0][i0] += a.BB[q0][i0] * kq;
      }
    }
  }
  if constexpr (SUM) block_reduce_sum_min<C::BLOCK>(active ? acc : 0.0, __builtin_huge_val(), red, a.part + blk,
                                                    a.part_min + blk);
  if constexpr (SCATTER) {
    const double(&T)[Q][P] = OP == OP_DIAG ? a.BB : a.B;
    // lane (q1, q2) writes into exactly the U2 slots it read
    if (tb < Q) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) U2[u2(c, i0, ta, tb)] = Rx[c][i0];
    }
    __syncthreads();
    if (ta < P && tb < Q) {   // y': lane (i0, q2), into its own U1 slots
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double r[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) r[q1] = U2[u2(c, ta, q1, tb)];
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          double v = 0.0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) v += T[q1][i1] * r[q1];
          U1[u1(c, ta, i1, tb)] = v;
        }
      }
    }
    __syncthreads();
    if (active && p1) {       // z': lane (i0, i1), then the scatter
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int cc = NC == 1 ? 0 : c;
        double r[Q];
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) r[q2] = U1[u1(cc, ta, tb, q2)];
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) {
          double v = 0.0;
#pragma unroll
          for (int q2 = 0; q2 < Q; ++q2) v += T[q2][i2] * r[q2];
          a.out[c * a.n_node + node[i2]] = old[c][i2] + v;
        }
      }
    }
  }
}

template <int P, int Q, int OP, bool QPS>
__global__ void __launch_bounds__((MassCfg<2, P, Q>::BLOCK))
mass_kernel_2d(const MassArgs<P, Q> a) {
  using C = MassCfg<2, P, Q>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P, NE = C::NE;
  constexpr bool FWD = OP != OP_DIAG;
  constexpr bool SUM = OP == OP_ENERGY || OP == OP_EG;
  constexpr bool SCATTER = OP != OP_ENERGY;
  constexpr int NC = OP == OP_DIAG ? 1 : 2;
  __shared__ double s_all[EPB * NE];
  __shared__ double red[2 * (C::BLOCK / 64)];

  const int tid = threadIdx.x;
  const int le_raw = tid / TPE;
  const int le = le_raw < EPB ? le_raw : EPB - 1;
  const int ta = le_raw < EPB ? tid - le_raw * TPE : Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int k = blk * EPB + le;
  const bool active = le_raw < EPB && k < a.n_list;
  const int kk = k < a.n_list ? k : a.n_list - 1;
  double* U1 = s_all + le * NE;              // [c][i0][q1]
  const bool p1 = ta < P;                    // lane i0
  auto u1 = [](int c, int i0, int q1) { return (c * P + i0) * Q + q1; };

  const int32_t* en = a.elem_node + (int64_t)kk * NPE;
  int node[P];
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1) node[i1] = p1 ? en[ta + P * i1] : en[0];
  double old[2][P];
  if constexpr (SCATTER) {
    if (active && p1) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) old[c][i1] = a.out[c * a.n_node + node[i1]];
    }
  }

  if constexpr (FWD) {
    if (p1) {   // y: lane i0
      double u[2][P];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          const int64_t j = c * a.n_node + node[i1];
          u[c][i1] = OP == OP_HESS ? a.x[j] : a.x[j] - a.x0[j];
        }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          double v = 0.0;
#pragma unroll
          for (int i1 = 0; i1 < P; ++i1) v += a.B[q1][i1] * u[c][i1];
          U1[u1(c, ta, q1)] = v;
        }
    }
    __syncthreads();
  }

  double acc = 0.0;
  double Rx[NC][P];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int i0 = 0; i0 < P; ++i0) Rx[c][i0] = 0.0;
  if (ta < Q) {   // x and the point terms: lane q1
    const double w1 = a.w[ta] * a.k * (a.scale ? *a.scale : 1.0);
    double sq[Q];
    if constexpr (QPS) {
      const double* ts = a.tsize + (int64_t)kk * (Q * Q) + Q * ta;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    double x1[2][P];
    if constexpr (FWD) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) x1[c][i0] = U1[u1(c, i0, ta)];
    }
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      double kq = w1 * a.w[q0];
      if constexpr (QPS) kq *= sq[q0] * sq[q0];
      if constexpr (FWD) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          double uq = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) uq += a.B[q0][i0] * x1[c][i0];
          if constexpr (SUM) acc += 0.5 * kq * uq * uq;
          if constexpr (SCATTER) {
            const double m = kq * uq;
#pragma unroll
            for (int i0 = 0; i0 < P; ++i0) Rx[c][i0] += a.B[q0][i0] * m;
          }
        }
      } else {
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) Rx[0][i0] += a.BB[q0][i0] * kq;
      }
    }
  }
  if constexpr (SUM) block_reduce_sum_min<C::BLOCK>(active ? acc : 0.0, __builtin_huge_val(), red, a.part + blk,
                                                    a.part_min + blk);
  if constexpr (SCATTER) {
    const double(&T)[Q][P] = OP == OP_DIAG ? a.BB : a.B;
    if (ta < Q) {   // lane q1 writes into exactly the U1 slots it read
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) U1[u1(c, i0, ta)] = Rx[c][i0];
    }
    __syncthreads();
    if (active && p1) {   // y': lane i0, then the scatter
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int cc = NC == 1 ? 0 : c;
        double r[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) r[q1] = U1[u1(cc, ta, q1)];
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          double v = 0.0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) v += T[q1][i1] * r[q1];
          a.out[c * a.n_node + node[i1]] = old[c][i1] + v;
        }
      }
    }
  }
}

template <int DIM, int P, int Q, int OP, bool QPS>
static int mass_one(const MassParams& mp, hipStream_t s, int* grid) {
  using C = MassCfg<DIM, P, Q>;
  MassArgs<P, Q> a;
  a.x = mp.x; a.x0 = mp.x0; a.out = mp.out; a.elem_node = mp.elem_node;
  a.part = mp.part; a.part_min = mp.part_min; a.scale = mp.scale; a.tsize = mp.tsize;
  a.n_node = mp.n_node; a.n_list = mp.n_list; a.k = mp.k;
  for (int q = 0; q < Q; ++q) {
    a.w[q] = mp.w[q];
    for (int i = 0; i < P; ++i) { a.B[q][i] = mp.B[q][i]; a.BB[q][i] = mp.B[q][i] * mp.B[q][i]; }
  }
  const int g = (mp.n_list + C::EPB - 1) / C::EPB;
  *grid = g;
  if (g == 0 || mp.dry) return 0;
  if constexpr (DIM == 3) hipLaunchKernelGGL((mass_kernel_3d<P, Q, OP, QPS>), dim3(g), dim3(C::BLOCK), 0, s, a);
  else hipLaunchKernelGGL((mass_kernel_2d<P, Q, OP, QPS>), dim3(g), dim3(C::BLOCK), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <int DIM, int P, int Q, bool QPS>
static int mass_op(int op, const MassParams& mp, hipStream_t s, int* grid) {
  switch (op) {
    case OP_ENERGY: return mass_one<DIM, P, Q, OP_ENERGY, QPS>(mp, s, grid);
    case OP_GRAD: return mass_one<DIM, P, Q, OP_GRAD, QPS>(mp, s, grid);
    case OP_HESS: return mass_one<DIM, P, Q, OP_HESS, QPS>(mp, s, grid);
    case OP_EG: return mass_one<DIM, P, Q, OP_EG, QPS>(mp, s, grid);
    case OP_DIAG: return mass_one<DIM, P, Q, OP_DIAG, QPS>(mp, s, grid);
    default: return -1;
  }
}

template <int DIM>
static int mass_dispatch(int p, int Q, int op, const MassParams& mp, hipStream_t s, int* grid) {
  const int P = p + 1;
  const bool qps = mp.tsize != nullptr;
#define TMOP_MASS_PQ(P_, Q_) \
  if (P == P_ && Q == Q_) return qps ? mass_op<DIM, P_, Q_, true>(op, mp, s, grid) : mass_op<DIM, P_, Q_, false>(op, mp, s, grid);
  TMOP_MASS_PQ(2, 2) TMOP_MASS_PQ(2, 3)
  TMOP_MASS_PQ(3, 3) TMOP_MASS_PQ(3, 4)
  TMOP_MASS_PQ(4, 4) TMOP_MASS_PQ(4, 5)
  TMOP_MASS_PQ(5, 5) TMOP_MASS_PQ(5, 6)
#undef TMOP_MASS_PQ
  return -1;
}

int launch_mass(int dim, int p, int Q, int op, const MassParams& mp, hipStream_t s, int* grid) {
  return dim == 3 ? mass_dispatch<3>(p, Q, op, mp, s, grid) : mass_dispatch<2>(p, Q, op, mp, s, grid);
}

}  // namespace tmop
