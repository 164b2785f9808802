// Element kernels of the TMOP hot path on gfx950.
//
// One kernel template covers the three element operations of the method:
//   OP_ENERGY  sum_q w_q det W mu(T_q) and min det A    (eq. 2.4, Section 3.4)
//   OP_GRAD    dF/dx scattered to the nodes              (Section 3.4)
//   OP_HESS    (d^2F/dx^2) v scattered to the nodes      (Section 3.4)
//
// The Jacobian A = sum_i x_i (grad w_i)^T (eq. 2.2) of a tensor-product
// element is computed by sum factorization: one 1D contraction per
// reference direction with the tables B[q][i] = l_i(s_q) and
// G[q][i] = l_i'(s_q).  The gradient / Hessian action uses the transposed
// contractions in reverse order.
//
// Thread mapping (3D): each element gets Q*Q lanes, lane (a, b).  Each 1D
// pass gives a lane a full "pencil" along the contracted direction, so every
// value it loads is reused Q (or P) times from registers:
//   pass 1 (z):  lane (i0, i1) -- reads its P nodes from HBM, writes U to LDS
//   pass 2 (y):  lane (i0, q2) -- reads U, writes V to LDS
//   pass 3 (x):  lane (q1, q2) -- reads V into registers and walks q0:
//                A -> T = A W^-1 -> metric -> Y = w det W (dmu) W^-t,
//                accumulating the transposed x-contraction in registers
//   pass 3', 2', 1' mirror 3, 2, 1 and end with the scatter to the nodes.
// 2D is the same with one pass fewer and Q lanes per element.
//
// Scatter: the host launches one kernel per element colour; elements of a
// colour share no node, so the update out[node] += value is a plain
// read-modify-write and the result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmop_internal.h"
#include "tmop_metrics.h"

namespace tmop {

// Kernel arguments.  The 1D tables and the constant target travel in the
// kernel-argument segment, so the unrolled loops read them as scalars.
template <int P, int Q, typename R>
struct ElemArgs {
  const double* __restrict__ x;          // [dim][n_node]
  const double* __restrict__ v;          // [dim][n_node], OP_HESS only
  double* __restrict__ out;              // [dim][n_node], OP_GRAD / OP_HESS
  const int32_t* __restrict__ elem_node; // [n_elem][P^dim]
  const int32_t* __restrict__ list;      // elements to process (nullptr: 0..n_list-1)
  double* __restrict__ part;             // OP_ENERGY: [2 * gridDim.x] (sums, then mins)
  int64_t n_node;
  int32_t n_list;
  R B[Q][P];
  R G[Q][P];
  double w[Q];                           // 1D quadrature weights
  R Winv[3][3];                          // W^{-1} (constant target)
  double xi[P];                          // 1D GLL node coordinates
  double detW;
  double Winvd[3][3];                    // W^{-1} in FP64 (energy)
};

// Elements per block and block size: the smallest element count that best
// fills whole 64-lane waves, within 256 lanes and 64 KiB of LDS.
constexpr int pick_epb(int tpe, int lds_bytes_per_elem) {
  int best = 1;
  int best_num = 0, best_den = 1;        // utilisation as a fraction
  for (int epb = 1; epb * tpe <= 256; ++epb) {
    if (epb * lds_bytes_per_elem > 64 * 1024) break;
    const int threads = epb * tpe;
    const int padded = (threads + 63) / 64 * 64;
    if (threads * best_den > best_num * padded) { best_num = threads; best_den = padded; best = epb; }
  }
  return best;
}

template <int DIM, int P, int Q, typename R>
struct Cfg {
  static constexpr int TPE = DIM == 3 ? Q * Q : Q;
  static constexpr int NU = DIM == 3 ? 2 * 3 * Q * P * P : 2 * 2 * Q * P;
  static constexpr int NV = DIM == 3 ? 3 * 3 * Q * Q * P : 0;
  static constexpr int EPB = pick_epb(TPE, (NU + NV) * (int)sizeof(R));
  static constexpr int BLOCK = (EPB * TPE + 63) / 64 * 64;
};

// blockIdx -> logical block: consecutive logical blocks (neighbouring
// elements, which share nodes) land on the same XCD, whose L2 then serves
// the shared node reads.  Workgroups are dealt to the 8 XCDs round-robin.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int xcd = b & 7, q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

// Deterministic block reduction of (sum, min) in a fixed tree order.
template <int BLOCK>
__device__ __forceinline__ void block_reduce_sum_min(double s, double m, double* red, double* out_s,
                                                     double* out_m) {
  constexpr int NW = BLOCK / 64;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    m = fmin(m, __shfl_xor(m, off, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[wave] = s; red[NW + wave] = m; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ts = red[0], tm = red[NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) { ts += red[w]; tm = fmin(tm, red[NW + w]); }
    *out_s = ts;
    *out_m = tm;
  }
}

template <int D, typename R>
__device__ __forceinline__ double det_fp64(const R (&A)[D][D]) {
  double a[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) a[i][j] = (double)A[i][j];
  return det<D, double>(a);
}

// T = A W^{-1}
template <int D, typename R>
__device__ __forceinline__ void right_mul(const R (&A)[D][D], const R (&Wi)[3][3], R (&T)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R s = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += A[i][k] * Wi[k][j];
      T[i][j] = s;
    }
}

// Y = s * M W^{-t}
template <int D, typename R>
__device__ __forceinline__ void stress(const R (&M)[D][D], const R (&Wi)[3][3], R s, R (&Y)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R t = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) t += M[i][k] * Wi[j][k];
      Y[i][j] = s * t;
    }
}

// Per-point kernel of the three operations.  Given A (and dA), returns the
// energy contribution (OP_ENERGY) or fills Y (OP_GRAD / OP_HESS).
template <int D, int METRIC, typename R, int OP>
__device__ __forceinline__ void point_op(const R (&A)[D][D], const R (&dA)[D][D], const R (&Wi)[3][3],
                                         double wdet, const double (&Wid)[3][3], double& acc, double& mind,
                                         R (&Y)[D][D]) {
  if constexpr (OP == OP_ENERGY) {
    // The energy value, det A and their sums are FP64 in both paths: the
    // FP32 path promotes its contracted A (mu's "... - 1" would otherwise
    // leave an FP32 rounding floor under F).
    double Ad[D][D], Td[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) Ad[i][j] = (double)A[i][j];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += Ad[i][k] * Wid[k][j];
        Td[i][j] = s;
      }
    const double detA = det<D, double>(Ad);
    acc += wdet * mu_value<METRIC, double>(Td, det<D, double>(Td));
    mind = fmin(mind, detA);
    return;
  }
  R T[D][D];
  right_mul<D, R>(A, Wi, T);
  if constexpr (OP == OP_GRAD) {
    R Pm[D][D];
    mu_first<METRIC, R>(T, Pm);
    stress<D, R>(Pm, Wi, (R)wdet, Y);
  } else {
    R dT[D][D], dP[D][D];
    right_mul<D, R>(dA, Wi, dT);
    mu_second<METRIC, R>(T, dT, dP);
    stress<D, R>(dP, Wi, (R)wdet, Y);
  }
}

// ------------------------------------------------------------------ 3D

template <int P, int Q>
__device__ __forceinline__ constexpr int uidx3(int t, int c, int q2, int i1, int i0) {
  return ((t * 3 + c) * Q + q2) * (P * P) + i1 * P + i0;
}
template <int P, int Q>
__device__ __forceinline__ constexpr int vidx3(int t, int c, int q2, int q1, int i0) {
  return ((t * 3 + c) * Q + q2) * (Q * P) + q1 * P + i0;
}

// Both paths contract the field relative to the element: A only depends on
// node differences (the basis gradients sum to zero), so the summands stay
// at the element's size instead of the domain's, and so does the rounding
// error of A.  FP64 subtracts the element's first node.  FP32 subtracts the
// element's vertex-affine map f(0) + J0 xbar (J0 columns: corner minus
// origin, formed in FP64) and adds J0 back to the contracted Jacobian; the
// contracted values then shrink to the deviation from the affine map.
template <int DIM, int P, bool AFFINE>
__device__ __forceinline__ void element_frame(const double* __restrict__ f, int64_t n_node,
                                              const int32_t* __restrict__ en, double (&org)[3],
                                              double (&J0)[3][3]) {
  constexpr int corner[3] = {P - 1, P * (P - 1), P * P * (P - 1)};
  const int n0 = en[0];
#pragma unroll
  for (int c = 0; c < DIM; ++c) org[c] = f[c * n_node + n0];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int c = 0; c < 3; ++c) J0[c][l] = 0.0;
  if constexpr (AFFINE) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      const int nl = en[corner[l]];
#pragma unroll
      for (int c = 0; c < DIM; ++c) J0[c][l] = f[c * n_node + nl] - org[c];
    }
  }
}

// Passes 1 and 2 of the forward contraction of field f into sV.
template <int P, int Q, typename R, bool AFFINE>
__device__ __forceinline__ void fwd12_3d(const ElemArgs<P, Q, R>& a, const double* __restrict__ f,
                                         const int (&node)[P], const int32_t* __restrict__ en, int ta, int tb,
                                         R* __restrict__ sU, R* __restrict__ sV, R (&J0r)[3][3]) {
  double org[3], J0[3][3];
  element_frame<3, P, AFFINE>(f, a.n_node, en, org, J0);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int l = 0; l < 3; ++l) J0r[c][l] = (R)J0[c][l];
  if (ta < P && tb < P) {
    R X[3][P];
#pragma unroll
    for (int i2 = 0; i2 < P; ++i2)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (AFFINE)
          X[c][i2] = (R)(f[c * a.n_node + node[i2]] - org[c] - J0[c][0] * a.xi[ta] - J0[c][1] * a.xi[tb] -
                         J0[c][2] * a.xi[i2]);
        else
          X[c][i2] = (R)(f[c * a.n_node + node[i2]] - org[c]);
      }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        R ub = 0, ug = 0;
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) { ub += a.B[q2][i2] * X[c][i2]; ug += a.G[q2][i2] * X[c][i2]; }
        sU[uidx3<P, Q>(0, c, q2, tb, ta)] = ub;
        sU[uidx3<P, Q>(1, c, q2, tb, ta)] = ug;
      }
  }
  __syncthreads();
  if (ta < P) {   // lane (i0 = ta, q2 = tb)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R ub[P], ug[P];
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) { ub[i1] = sU[uidx3<P, Q>(0, c, tb, i1, ta)]; ug[i1] = sU[uidx3<P, Q>(1, c, tb, i1, ta)]; }
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        R bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          bb += a.B[q1][i1] * ub[i1];
          gb += a.G[q1][i1] * ub[i1];
          bg += a.B[q1][i1] * ug[i1];
        }
        sV[vidx3<P, Q>(0, c, tb, q1, ta)] = bb;
        sV[vidx3<P, Q>(1, c, tb, q1, ta)] = gb;
        sV[vidx3<P, Q>(2, c, tb, q1, ta)] = bg;
      }
    }
  }
  __syncthreads();
}

template <int P, int Q, int METRIC, typename R, int OP>
__global__ void __launch_bounds__((Cfg<3, P, Q, R>::BLOCK))
elem_kernel_3d(const ElemArgs<P, Q, R> a) {
  using C = Cfg<3, P, Q, R>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P * P;
  constexpr bool AFFINE = sizeof(R) == 4;   // FP32 contracts the deviation from the vertex-affine map
  __shared__ R sU_all[EPB * C::NU];
  __shared__ R sV_all[EPB * C::NV];
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
  const int e = a.list ? a.list[kk] : kk;
  R* sU = sU_all + le * C::NU;
  R* sV = sV_all + le * C::NV;

  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2)
    node[i2] = (ta < P && tb < P) ? en[ta + P * tb + P * P * i2] : 0;
  // forward for x, V into registers (lane (q1 = ta, q2 = tb))
  R J0x[3][3], J0v[3][3];
  fwd12_3d<P, Q, R, AFFINE>(a, a.x, node, en, ta, tb, sU, sV, J0x);
  R V[3][3][P];
  if (tb < Q) {
#pragma unroll
    for (int tt = 0; tt < 3; ++tt)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) V[tt][c][i0] = sV[vidx3<P, Q>(tt, c, tb, ta, i0)];
  }
  R dV[3][3][P];
  if constexpr (OP == OP_HESS) {
    __syncthreads();
    fwd12_3d<P, Q, R, AFFINE>(a, a.v, node, en, ta, tb, sU, sV, J0v);
    if (tb < Q) {
#pragma unroll
      for (int tt = 0; tt < 3; ++tt)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) dV[tt][c][i0] = sV[vidx3<P, Q>(tt, c, tb, ta, i0)];
    }
  }

  double acc = 0.0, mind = __builtin_huge_val();
  R Racc[3][3][P];
#pragma unroll
  for (int tt = 0; tt < 3; ++tt)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Racc[tt][c][i0] = 0;

  if (tb < Q) {
    const double w12 = a.w[ta] * a.w[tb] * a.detW;
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      R A[3][3], dA[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) {
          s0 += a.G[q0][i0] * V[0][c][i0];
          s1 += a.B[q0][i0] * V[1][c][i0];
          s2 += a.B[q0][i0] * V[2][c][i0];
        }
        if constexpr (AFFINE) { s0 += J0x[c][0]; s1 += J0x[c][1]; s2 += J0x[c][2]; }
        A[c][0] = s0; A[c][1] = s1; A[c][2] = s2;
        if constexpr (OP == OP_HESS) {
          R d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) {
            d0 += a.G[q0][i0] * dV[0][c][i0];
            d1 += a.B[q0][i0] * dV[1][c][i0];
            d2 += a.B[q0][i0] * dV[2][c][i0];
          }
          if constexpr (AFFINE) { d0 += J0v[c][0]; d1 += J0v[c][1]; d2 += J0v[c][2]; }
          dA[c][0] = d0; dA[c][1] = d1; dA[c][2] = d2;
        }
      }
      R Y[3][3];
      point_op<3, METRIC, R, OP>(A, dA, a.Winv, w12 * a.w[q0], a.Winvd, acc, mind, Y);
      if constexpr (OP != OP_ENERGY) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) {
            Racc[0][c][i0] += a.G[q0][i0] * Y[c][0];
            Racc[1][c][i0] += a.B[q0][i0] * Y[c][1];
            Racc[2][c][i0] += a.B[q0][i0] * Y[c][2];
          }
      }
    }
  }

  if constexpr (OP == OP_ENERGY) {
    if (!active) { acc = 0.0; mind = __builtin_huge_val(); }
    block_reduce_sum_min<C::BLOCK>(acc, mind, red, a.part + blk, a.part + gridDim.x + blk);
    return;
  } else {
    // pass 3': each lane writes its own V slots, so no barrier is needed first
    if (tb < Q) {
#pragma unroll
      for (int tt = 0; tt < 3; ++tt)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) sV[vidx3<P, Q>(tt, c, tb, ta, i0)] = Racc[tt][c][i0];
    }
    __syncthreads();
    // pass 2': lane (i0 = ta, q2 = tb)
    if (ta < P && tb < Q) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R r0[Q], r1[Q], r2[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          r0[q1] = sV[vidx3<P, Q>(0, c, tb, q1, ta)];
          r1[q1] = sV[vidx3<P, Q>(1, c, tb, q1, ta)];
          r2[q1] = sV[vidx3<P, Q>(2, c, tb, q1, ta)];
        }
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          R sb = 0, sg = 0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) {
            sb += a.B[q1][i1] * r0[q1] + a.G[q1][i1] * r1[q1];
            sg += a.B[q1][i1] * r2[q1];
          }
          sU[uidx3<P, Q>(0, c, tb, i1, ta)] = sb;
          sU[uidx3<P, Q>(1, c, tb, i1, ta)] = sg;
        }
      }
    }
    __syncthreads();
    // pass 1': lane (i0 = ta, i1 = tb), then the scatter
    if (active && ta < P && tb < P) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R sb[Q], sg[Q];
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) { sb[q2] = sU[uidx3<P, Q>(0, c, q2, tb, ta)]; sg[q2] = sU[uidx3<P, Q>(1, c, q2, tb, ta)]; }
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) {
          R s = 0;
#pragma unroll
          for (int q2 = 0; q2 < Q; ++q2) s += a.B[q2][i2] * sb[q2] + a.G[q2][i2] * sg[q2];
          double* o = a.out + c * a.n_node + node[i2];
          *o = *o + (double)s;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ 2D

template <int P, int Q>
__device__ __forceinline__ constexpr int uidx2(int t, int c, int q1, int i0) {
  return ((t * 2 + c) * Q + q1) * P + i0;
}

// Pass 1 of the forward contraction of f into sU, then U into registers of
// lane q1 = ta.
template <int P, int Q, typename R, bool AFFINE>
__device__ __forceinline__ void fwd1_2d(const ElemArgs<P, Q, R>& a, const double* __restrict__ f,
                                        const int (&node)[P], const int32_t* __restrict__ en, int ta,
                                        R* __restrict__ sU, R (&U)[2][2][P], R (&J0r)[2][2]) {
  double org[3], J0[3][3];
  element_frame<2, P, AFFINE>(f, a.n_node, en, org, J0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int l = 0; l < 2; ++l) J0r[c][l] = (R)J0[c][l];
  if (ta < P) {   // lane i0 = ta
    R X[2][P];
#pragma unroll
    for (int i1 = 0; i1 < P; ++i1)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if constexpr (AFFINE)
          X[c][i1] = (R)(f[c * a.n_node + node[i1]] - org[c] - J0[c][0] * a.xi[ta] - J0[c][1] * a.xi[i1]);
        else
          X[c][i1] = (R)(f[c * a.n_node + node[i1]] - org[c]);
      }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        R ub = 0, ug = 0;
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) { ub += a.B[q1][i1] * X[c][i1]; ug += a.G[q1][i1] * X[c][i1]; }
        sU[uidx2<P, Q>(0, c, q1, ta)] = ub;
        sU[uidx2<P, Q>(1, c, q1, ta)] = ug;
      }
  }
  __syncthreads();
  if (ta < Q) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) U[tt][c][i0] = sU[uidx2<P, Q>(tt, c, ta, i0)];
  }
}

template <int P, int Q, int METRIC, typename R, int OP>
__global__ void __launch_bounds__((Cfg<2, P, Q, R>::BLOCK))
elem_kernel_2d(const ElemArgs<P, Q, R> a) {
  using C = Cfg<2, P, Q, R>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P;
  constexpr bool AFFINE = sizeof(R) == 4;
  __shared__ R sU_all[EPB * C::NU];
  __shared__ double red[2 * (C::BLOCK / 64)];

  const int tid = threadIdx.x;
  const int le_raw = tid / TPE;
  const int le = le_raw < EPB ? le_raw : EPB - 1;
  const int ta = le_raw < EPB ? tid - le_raw * TPE : Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int k = blk * EPB + le;
  const bool active = le_raw < EPB && k < a.n_list;
  const int kk = k < a.n_list ? k : a.n_list - 1;
  const int e = a.list ? a.list[kk] : kk;
  R* sU = sU_all + le * C::NU;

  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1) node[i1] = ta < P ? en[ta + P * i1] : 0;
  R U[2][2][P], dU[2][2][P], J0x[2][2], J0v[2][2];
  fwd1_2d<P, Q, R, AFFINE>(a, a.x, node, en, ta, sU, U, J0x);
  if constexpr (OP == OP_HESS) {
    __syncthreads();
    fwd1_2d<P, Q, R, AFFINE>(a, a.v, node, en, ta, sU, dU, J0v);
  }

  double acc = 0.0, mind = __builtin_huge_val();
  R Racc[2][2][P];
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Racc[tt][c][i0] = 0;

  if (ta < Q) {   // lane q1 = ta
    const double w1 = a.w[ta] * a.detW;
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      R A[2][2], dA[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R s0 = 0, s1 = 0;
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) { s0 += a.G[q0][i0] * U[0][c][i0]; s1 += a.B[q0][i0] * U[1][c][i0]; }
        if constexpr (AFFINE) { s0 += J0x[c][0]; s1 += J0x[c][1]; }
        A[c][0] = s0; A[c][1] = s1;
        if constexpr (OP == OP_HESS) {
          R d0 = 0, d1 = 0;
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) { d0 += a.G[q0][i0] * dU[0][c][i0]; d1 += a.B[q0][i0] * dU[1][c][i0]; }
          if constexpr (AFFINE) { d0 += J0v[c][0]; d1 += J0v[c][1]; }
          dA[c][0] = d0; dA[c][1] = d1;
        }
      }
      R Y[2][2];
      point_op<2, METRIC, R, OP>(A, dA, a.Winv, w1 * a.w[q0], a.Winvd, acc, mind, Y);
      if constexpr (OP != OP_ENERGY) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) {
            Racc[0][c][i0] += a.G[q0][i0] * Y[c][0];
            Racc[1][c][i0] += a.B[q0][i0] * Y[c][1];
          }
      }
    }
  }

  if constexpr (OP == OP_ENERGY) {
    if (!active) { acc = 0.0; mind = __builtin_huge_val(); }
    block_reduce_sum_min<C::BLOCK>(acc, mind, red, a.part + blk, a.part + gridDim.x + blk);
    return;
  } else {
    // pass 2': lane q1 writes its own U slots, no barrier needed first
    if (ta < Q) {
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) sU[uidx2<P, Q>(tt, c, ta, i0)] = Racc[tt][c][i0];
    }
    __syncthreads();
    // pass 1': lane i0 = ta, then the scatter
    if (active && ta < P) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R rb[Q], rg[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) { rb[q1] = sU[uidx2<P, Q>(0, c, q1, ta)]; rg[q1] = sU[uidx2<P, Q>(1, c, q1, ta)]; }
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          R s = 0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) s += a.B[q1][i1] * rb[q1] + a.G[q1][i1] * rg[q1];
          double* o = a.out + c * a.n_node + node[i1];
          *o = *o + (double)s;
        }
      }
    }
  }
}

}  // namespace tmop
