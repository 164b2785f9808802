// Element kernels of the TMOP hot path on gfx950.
//
// One kernel template covers the element operations of the method:
//   OP_ENERGY  sum_q w_q det W mu(T_q) and min det A    (eq. 2.4, Section 3.4)
//   OP_GRAD    dF/dx scattered to the nodes              (Section 3.4)
//   OP_HESS    (d^2F/dx^2) v scattered to the nodes      (Section 3.4)
//   OP_EG      OP_ENERGY and OP_GRAD in one pass (the line search needs both
//              at every trial point)
//   OP_SIZE    (det A)^(1/d) at every quadrature point: the size of the
//              target W_3 = (det A(x_0))^(1/d) I of Section 3.1
//   OP_JINV    A^{-1} at every quadrature point: the target data of
//              W_0 = A(x_init) in the replication composite (Section 4.3.2)
//
// Targets (template parameter TGT): a constant general W (TGT_GEN), a
// constant isotropic W = s I (TGT_ISO), an isotropic W_q = s_q I given
// per quadrature point (TGT_QPS, Section 3.1: W may differ at every point),
// a general W_q with its own weight omega_q per point (TGT_MAT: the
// replication composite, Section 4.3.2), or a constant general W with a
// weight omega_q per point (TGT_CW: the second term of eq. 4.1).
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
//   pass 1 (z):   lane (i0, i1) -- its P nodes (loaded up front), U to LDS
//   pass 23 (y):  lane (q1, q2) -- contracts the slab of U at q2 for its own
//                 q1 into its x-pencils V (registers), then walks q0:
//                 A -> T = A W^-1 -> metric -> Y = w det W (dmu) W^-t,
//                 accumulating the transposed x-contraction in registers
//   pass 3', 2', 1' hand the transposed sums back through LDS one
//                 component at a time and end with the scatter to the nodes.
// All Q*Q lanes work in pass 23; LDS holds U (or one component's transposed
// data), 2 Q P^2 values per component and element.
// 2D is the same with one pass fewer and Q lanes per element.
//
// Scatter: the host launches one kernel per element colour; elements of a
// colour share no node, so the update out[node] += value is a plain
// read-modify-write (the old value is loaded early to hide its latency) and
// the result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmop_internal.h"
#include "tmop_metrics.h"

namespace tmop {

// Kernel arguments.  The 1D tables and the constant target travel in the
// kernel-argument segment, so the unrolled loops read them as scalars.
// Isotropic target W = s I: every term of A (and of the transposed
// contraction) holds exactly one G factor, so G carries the factor 1/s and
// the contraction yields T = A W^{-1} directly (and Y needs no W^{-t}).
template <int P, int Q, typename R>
struct ElemArgs {
  const double* __restrict__ x;          // [dim][n_node]
  const double* __restrict__ v;          // [dim][n_node], OP_HESS only
  double* __restrict__ out;              // [dim][n_node], OP_GRAD / OP_HESS
  const int32_t* __restrict__ elem_node; // [n_elem][P^dim]
  const int32_t* __restrict__ list;      // elements to process (nullptr: 0..n_list-1)
  const uint32_t* __restrict__ first;    // scatter: bit l of word k * ((P^dim + 31) / 32) + l / 32 set when
                                         // element k is the first to touch its local node l (its old value
                                         // is 0, not read); nullptr: read every old value
  double* __restrict__ part;             // OP_ENERGY, OP_EG: [gridDim.x] block sums of the energy
  double* __restrict__ part_min;         // OP_ENERGY, OP_EG: [gridDim.x] block minima of det A
  const double* __restrict__ scale;      // OP_GRAD: optional device scalar multiplying g (nullptr = 1)
  const double* __restrict__ tsize;      // TGT_QPS: [n_list][Q^dim] target sizes s_q (W_q = s_q I), point
                                         // index q0 + Q q1 (+ Q^2 q2), in the order of elem_node
  const double* __restrict__ tmat;       // TGT_MAT: W_q^{-1} (row-major) and omega_q, dim^2 + 1 values per point,
                                         // per point [n_list][Q^dim] or per element [n_list] (tm_el, tm_pt);
                                         // TGT_CW: [n_list][Q^dim] omega_q (W^{-1} = Winv)
  int32_t tm_el;                         // TGT_MAT: values between consecutive elements of tmat
  int32_t tm_pt;                         // TGT_MAT: values between consecutive points (0: one target per element)
  int64_t n_node;
  int32_t n_list;
  R B[Q][P];
  R G[Q][P];
  double w[Q];                           // 1D quadrature weights
  R Winv[3][3];                          // W^{-1} (constant target; unused when isotropic)
  double Winvd[3][3];                    // W^{-1} in FP64 (energy)
  double jscale;                         // factor of the affine-frame Jacobian: 1/s if isotropic, else 1
  double xi[P];                          // 1D GLL node coordinates
  double detW;
  double wdetW;                          // weight factor of a constant target: eta det W
  double M1[P][P];                       // PEN: 1D mass matrix sum_k w_k l_i(s_k) l_j(s_k)
  double kpen;                           // PEN: 2 delta det W
  R* evec;                               // 3D scatter ops: element vector [3][n_ent] instead of out, or nullptr
  const int32_t* evpos;                  // with evec: [n_elem][P^3] the entry of each element node
  int64_t n_ent;                         // with evec: entries per component
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

// LDS of one element (values).  Energy and gradient:
//   U [q2][c][i0][i1][t2]  pass 1 -> pass 23: the z-contraction, t2 = B, G
//   R [q2][i0][t][q1]      pass 3' -> pass 2': one component of the
//                          x-transposed contraction (t = the three terms)
//   S [i0][i1][q2][t2]     pass 2' -> pass 1': one component of the
//                          y-transposed contraction; S follows R
// U is dead before R and S are written, so they share the space.
// Hessian action: pass 2 on lanes (i0, q2), each with its own area of 9 Q
// values that holds first its U pencil, then its V pencils (read back by the
// pass-3 lanes); R and S reuse the space afterwards.
template <int P, int Q> struct Lds3 {
  static constexpr int NU = Q * 3 * P * P * 2;
  static constexpr int NR = Q * P * 3 * Q;
  static constexpr int NS = P * P * Q * 2;
  static constexpr int AREA = 9 * Q;
  static constexpr int NA = Q * P * AREA;
  static constexpr int N = NU > NR + NS ? NU : NR + NS;
  static constexpr int NH = NA > NR + NS ? NA : NR + NS;
  static __device__ __forceinline__ constexpr int u(int q2, int c, int i0, int i1) {
    return (((q2 * 3 + c) * P + i0) * P + i1) * 2;
  }
  static __device__ __forceinline__ constexpr int r(int q2, int i0, int t, int q1) {
    return ((q2 * P + i0) * 3 + t) * Q + q1;
  }
  static __device__ __forceinline__ constexpr int s(int i0, int i1, int q2) { return NR + ((i0 * P + i1) * Q + q2) * 2; }
  // area of pass-2 lane (i0, q2); U pencil at (t, c, i1), V pencil at (t, c, q1)
  static __device__ __forceinline__ constexpr int area(int q2, int i0) { return (q2 * P + i0) * AREA; }
  static __device__ __forceinline__ constexpr int au(int t, int c, int i1) { return (t * 3 + c) * P + i1; }
  static __device__ __forceinline__ constexpr int av(int t, int c, int q1) { return (t * 3 + c) * Q + q1; }
};

// LDS padding of the per-element block (values, 3D; the 2D padding,
// TMOP_ELEM_PAD2, sits with elem2d_lds_values): it sets the bank pattern of
// the accesses of neighbouring elements.  Measured on the 2D workloads, 5
// extra values cut the LDS bank conflicts of the 16
// elements of a wave: FP64 energy launch 24.0 -> 19.6 us (512^2 Q2),
// Hessian action 19.6 -> 16.8 us.
#ifndef TMOP_ELEM_PAD
#define TMOP_ELEM_PAD 2
#endif

template <int DIM, int P, int Q, typename R>
struct Cfg {
  static constexpr int TPE = DIM == 3 ? Q * Q : Q;
  // LDS values per element: energy / gradient, Hessian action
  static constexpr int NE = DIM == 3 ? Lds3<P, Q>::N + TMOP_ELEM_PAD : elem2d_lds_values(P, Q);
  static constexpr int NEH = DIM == 3 ? Lds3<P, Q>::NH + TMOP_ELEM_PAD : elem2d_lds_values(P, Q);
  static constexpr int EPB = pick_epb(TPE, NEH * (int)sizeof(R));
  static constexpr int BLOCK = (EPB * TPE + 63) / 64 * 64;
};

// blockIdx -> logical block: consecutive logical blocks (neighbouring
// elements, which share nodes) land on the same XCD, whose L2 then serves
// the shared node reads.  Workgroups are dealt to the 8 XCDs round-robin.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int xcd = b & 7, q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

// Whether element k (of this launch) is the first to touch its local node l.
template <int NPE>
__device__ __forceinline__ bool first_touch(const uint32_t* __restrict__ first, int k, int l) {
  constexpr int NW = (NPE + 31) / 32;
  return first && ((first[(int64_t)k * NW + l / 32] >> (l % 32)) & 1u);
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

// T = A W^{-1} (ISO: the contraction already produced T)
template <int D, typename R, bool ISO>
__device__ __forceinline__ void right_mul(const R (&A)[D][D], const R (&Wi)[3][3], R (&T)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if constexpr (ISO) {
        T[i][j] = A[i][j];
      } else {
        R s = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += A[i][k] * Wi[k][j];
        T[i][j] = s;
      }
    }
}

// Y = M W^{-t} (ISO: the transposed contraction's G carries W^{-t}, Y = M)
template <int D, typename R, bool ISO>
__device__ __forceinline__ void stress(const R (&M)[D][D], const R (&Wi)[3][3], R (&Y)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if constexpr (ISO) {
        Y[i][j] = M[i][j];
      } else {
        R t = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) t += M[i][k] * Wi[j][k];
        Y[i][j] = t;
      }
    }
}

enum { TGT_GEN = 0, TGT_ISO = 1, TGT_QPS = 2, TGT_MAT = 3, TGT_CW = 4 };

// TGT_MAT: this point's W^{-1} (in the arithmetic type and in FP64) and weight
template <typename R>
__device__ __forceinline__ double load_point_target2(const double* __restrict__ tm, R (&Wi)[3][3],
                                                     double (&Wid)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Wid[i][j] = 0.0;
  Wid[0][0] = tm[0]; Wid[0][1] = tm[1]; Wid[1][0] = tm[2]; Wid[1][1] = tm[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Wi[i][j] = (R)Wid[i][j];
  return tm[4];
}

template <typename R>
__device__ __forceinline__ double load_point_target3(const double* __restrict__ tm, R (&Wi)[3][3],
                                                     double (&Wid)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Wid[i][j] = tm[3 * i + j];
      Wi[i][j] = (R)Wid[i][j];
    }
  return tm[9];
}

// TGT_MAT / TGT_CW: the target data of point row `row` (q0 = 0 there) of
// element e; the row's points follow at steps of a.tm_pt (TGT_MAT) or 1.
template <int NQ, int TGT, typename Args>
__device__ __forceinline__ const double* target_row(const Args& a, int e, int row) {
  if constexpr (TGT == TGT_MAT) return a.tmat + (int64_t)e * a.tm_el + (int64_t)row * a.tm_pt;
  else if constexpr (TGT == TGT_CW) return a.tmat + (int64_t)e * NQ + row;
  else return nullptr;
}

// Per-point kernel of the operations.  Given A (and dA) -- already divided
// by s for isotropic targets, i.e. T -- adds the energy contribution
// wdet mu(T) (OP_ENERGY, OP_EG), fills Y (OP_GRAD / OP_HESS) with the weight
// kY folded into the metric's coefficients, or returns det A (OP_SIZE).
// detWq: det W at this point.
template <int D, int METRIC, typename R, int OP, bool ISO>
__device__ __forceinline__ void point_op(const R (&Wi)[3][3], const double (&Wid)[3][3], const R (&A)[D][D],
                                         const R (&dA)[D][D], double wdet, double detWq, double kY, double& acc,
                                         double& mind, R (&Y)[D][D], double& detA_out) {
  if constexpr (OP == OP_ENERGY || OP == OP_EG || OP == OP_SIZE || OP == OP_JINV) {
    // The energy value, det A and their sums are FP64 in both paths: the
    // FP32 path promotes its contracted A (mu's "... - 1" would otherwise
    // leave an FP32 rounding floor under F).
    double Ad[D][D], Td[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) Ad[i][j] = (double)A[i][j];
    double detA, tau;
    if constexpr (ISO) {          // the contraction gave T; det A = det T det W
      right_mul<D, double, true>(Ad, Wid, Td);
      tau = det<D, double>(Td);
      detA = tau * detWq;
    } else {
      detA = det<D, double>(Ad);
      right_mul<D, double, false>(Ad, Wid, Td);
      tau = det<D, double>(Td);
    }
    if constexpr (OP != OP_SIZE && OP != OP_JINV) acc += wdet * mu_value<METRIC, double>(Td, tau);
    mind = fmin(mind, detA);
    detA_out = detA;
  }
  if constexpr (OP == OP_GRAD || OP == OP_EG || OP == OP_HESS) {
    // the weight is folded into the metric's scalar coefficients
    R T[D][D];
    right_mul<D, R, ISO>(A, Wi, T);
    if constexpr (OP == OP_GRAD || OP == OP_EG) {
      R Pm[D][D];
      mu_first<METRIC, R>(T, (R)kY, Pm);
      stress<D, R, ISO>(Pm, Wi, Y);
    } else {
      R dT[D][D], dP[D][D];
      right_mul<D, R, ISO>(dA, Wi, dT);
      mu_second<METRIC, R>(T, dT, (R)kY, dP);
      stress<D, R, ISO>(dP, Wi, Y);
    }
  }
}

// (det A)^(1/d) with the real roots (NaN for det A < 0 in 2D, negative in 3D)
template <int D>
__device__ __forceinline__ double size_of(double detA) {
  if constexpr (D == 2) return sqrt(detA);
  else return cbrt(detA);
}

// Per-point target scaling (TGT_QPS): A, dA <- A / s, dA / s, and the
// weights: w det W = w s^d for the energy, w s^(d-1) for Y (W^{-t} = I / s
// is not in the G table then).
template <int D, typename R>
__device__ __forceinline__ void qp_scale(double s, R (&A)[D][D], R (&dA)[D][D], double& wdet, double& detWq,
                                         double& kY) {
  const double rs = 1.0 / s;
  const R r = (R)rs;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) { A[i][j] *= r; dA[i][j] *= r; }
  detWq = D == 2 ? s * s : s * s * s;
  wdet *= detWq;
  kY = wdet * rs;
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

// ------------------------------------------------------------------ 3D

// The pencil of pass-1 lane (i0, i1): its P nodes of field f relative to the
// element frame, for every component.  Only called by lanes with i0, i1 < P.
template <int P, int Q, typename R, bool AFFINE>
__device__ __forceinline__ void load_pencil_3d(const ElemArgs<P, Q, R>& a, const double* __restrict__ f,
                                               const int (&node)[P], const int32_t* __restrict__ en, int i0,
                                               int i1, R (&X)[3][P], R (&J0r)[3][3]) {
  double org[3], J0[3][3];
  element_frame<3, P, AFFINE>(f, a.n_node, en, org, J0);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int l = 0; l < 3; ++l) J0r[c][l] = (R)(J0[c][l] * a.jscale);
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (AFFINE)
        X[c][i2] = (R)(f[c * a.n_node + node[i2]] - org[c] - J0[c][0] * a.xi[i0] - J0[c][1] * a.xi[i1] -
                       J0[c][2] * a.xi[i2]);
      else
        X[c][i2] = (R)(f[c * a.n_node + node[i2]] - org[c]);
    }
}

// Forward contraction up to the x-pencils.  Pass 1 (lane (i0, i1)): z, into
// U.  Pass 23 (lane (q1, q2)): y for its own q1 straight from U, giving the
// three x-pencils V[t][c][i0] of point row (q1, q2):
//   t = 0: B_y B_z (used with G_x), 1: G_y B_z, 2: B_y G_z (used with B_x).
// Bq, Gq: row q1 of the tables.
template <int P, int Q, typename R>
__device__ __forceinline__ void fwd_3d(const ElemArgs<P, Q, R>& a, const R (&X)[3][P], int ta, int tb,
                                       const R (&Bq)[P], const R (&Gq)[P], R* __restrict__ s,
                                       R (&V)[3][3][P]) {
  using L = Lds3<P, Q>;
  if (ta < P && tb < P) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        R ub = 0, ug = 0;
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) { ub += a.B[q2][i2] * X[c][i2]; ug += a.G[q2][i2] * X[c][i2]; }
        R* p = s + L::u(q2, c, ta, tb);
        p[0] = ub;
        p[1] = ug;
      }
  }
  __syncthreads();
  if (tb < Q) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) {
        R ub[P], ug[P];
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          const R* p = s + L::u(tb, c, i0, i1);
          ub[i1] = p[0];
          ug[i1] = p[1];
        }
        R bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) { bb += Bq[i1] * ub[i1]; gb += Gq[i1] * ub[i1]; bg += Bq[i1] * ug[i1]; }
        V[0][c][i0] = bb;
        V[1][c][i0] = gb;
        V[2][c][i0] = bg;
      }
  }
}

// Forward contraction of the Hessian action (register pressure: its x-pencils
// come from LDS just before the point loop).  Pass 1 (lane (i0, i1)): z, into
// the areas.  Pass 2 (lane (i0, q2)): y for every q1, in its own area.  Then
// lane (q1, q2) reads its x-pencils V[t][c][i0].
template <int P, int Q, typename R>
__device__ __forceinline__ void fwd_3d_areas(const ElemArgs<P, Q, R>& a, const R (&X)[3][P], int ta, int tb,
                                             R* __restrict__ s, R (&V)[3][3][P]) {
  using L = Lds3<P, Q>;
  if (ta < P && tb < P) {   // pass 1, lane (i0 = ta, i1 = tb): U of all q2
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        R ub = 0, ug = 0;
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) { ub += a.B[q2][i2] * X[c][i2]; ug += a.G[q2][i2] * X[c][i2]; }
        R* ar = s + L::area(q2, ta);
        ar[L::au(0, c, tb)] = ub;
        ar[L::au(1, c, tb)] = ug;
      }
  }
  __syncthreads();
  if (ta < P && tb < Q) {   // pass 2, lane (i0 = ta, q2 = tb): own area, U in, V out
    R* ar = s + L::area(tb, ta);
    R ub[3][P], ug[3][P];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) { ub[c][i1] = ar[L::au(0, c, i1)]; ug[c][i1] = ar[L::au(1, c, i1)]; }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        R bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          bb += a.B[q1][i1] * ub[c][i1];
          gb += a.G[q1][i1] * ub[c][i1];
          bg += a.B[q1][i1] * ug[c][i1];
        }
        ar[L::av(0, c, q1)] = bb;
        ar[L::av(1, c, q1)] = gb;
        ar[L::av(2, c, q1)] = bg;
      }
  }
  __syncthreads();
  if (tb < Q) {             // lane (q1 = ta, q2 = tb) reads its x-pencils
#pragma unroll
    for (int i0 = 0; i0 < P; ++i0) {
      const R* ar = s + L::area(tb, i0);
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) V[t][c][i0] = ar[L::av(t, c, ta)];
    }
  }
}

// Displacement penalty of eq. 4.2 fused into the 3D Hessian action (PEN,
// FP64, constant target): with det W constant the target-weighted element
// mass matrix is det W (M1 x M1 x M1), M1 the 1D mass matrix of the
// quadrature, so M_E v is three P x P passes over the element's nodes.  Runs
// between the point loop and the transposed passes, in the LDS the forward
// passes leave free and while the point loop's registers are dead, on v
// re-read from global memory; lane (i0, i1) gets
// w[c][i2] = (M1 x M1 x M1 v)[c][i0][i1][i2].
template <int P, int Q>
__device__ __forceinline__ void penalty_pass_3d(const ElemArgs<P, Q, double>& a, const double* __restrict__ f,
                                                const int (&node)[P], bool p1, int ta, int tb,
                                                double* __restrict__ s, double (&w)[3][P]) {
  auto t = [](int c, int i0, int i1, int i2) { return ((c * P + i2) * P + i1) * P + i0; };
  double u[3][P];
  if (p1) {   // z, lane (i0, i1)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) u[c][i2] = f[c * a.n_node + node[i2]];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) {
        double v = 0.0;
#pragma unroll
        for (int j2 = 0; j2 < P; ++j2) v += a.M1[i2][j2] * u[c][j2];
        s[t(c, ta, tb, i2)] = v;
      }
  }
  __syncthreads();
  if (p1) {   // y: read all, then write in place
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) {
        double v = 0.0;
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1) v += a.M1[tb][j1] * s[t(c, ta, j1, i2)];
        w[c][i2] = v;
      }
  }
  __syncthreads();
  if (p1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) s[t(c, ta, tb, i2)] = w[c][i2];
  }
  __syncthreads();
  if (p1) {   // x
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) {
        double v = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < P; ++j0) v += a.M1[ta][j0] * s[t(c, j0, tb, i2)];
        w[c][i2] = v;
      }
  }
}

// EV: the element-vector instantiation.  Its gradient kinds with a constant
// target, up to order 3, are asked for two waves per SIMD: with no old
// values their schedule otherwise lands a register or two above 256 for the
// Q3 energy + gradient (one wave per SIMD).  Under the same request the
// Hessian action, order 4 and the per-point targets spill.
template <int P, int Q, int METRIC, typename R, int OP, int TGT, bool PEN = false, bool EV = false>
__global__ void __launch_bounds__((Cfg<3, P, Q, R>::BLOCK))
__attribute__((amdgpu_waves_per_eu(EV && OP != OP_HESS && P <= 4 && (TGT == TGT_GEN || TGT == TGT_ISO) ? 2 : 1)))
elem_kernel_3d(const ElemArgs<P, Q, R> a) {
  static_assert(!PEN || (sizeof(R) == 8 && OP == OP_HESS && (TGT == TGT_ISO || TGT == TGT_GEN)),
                "the fused penalty is the FP64 constant-target Hessian action");
  using C = Cfg<3, P, Q, R>;
  using L = Lds3<P, Q>;
  constexpr bool ISO = TGT == TGT_ISO || TGT == TGT_QPS;
  constexpr bool ENERGY_LIKE = OP == OP_ENERGY || OP == OP_SIZE || OP == OP_JINV;   // no transposed passes
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P * P;
  constexpr bool AFFINE = sizeof(R) == 4;   // FP32 contracts the deviation from the vertex-affine map
  constexpr int NE = OP == OP_HESS ? C::NEH : C::NE;
  __shared__ R s_all[EPB * NE];
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
  R* s = s_all + le * NE;
  const bool p1 = ta < P && tb < P;          // pass-1 lane (i0 = ta, i1 = tb)

  // all global loads of the element's fields first
  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2) node[i2] = p1 ? en[ta + P * tb + P * P * i2] : en[0];
  R X[3][P], dX[3][P], J0x[3][3], J0v[3][3];
  load_pencil_3d<P, Q, R, AFFINE>(a, a.x, node, en, p1 ? ta : 0, p1 ? tb : 0, X, J0x);
  if constexpr (OP == OP_HESS) load_pencil_3d<P, Q, R, AFFINE>(a, a.v, node, en, p1 ? ta : 0, p1 ? tb : 0, dX, J0v);

  R V[3][3][P], dV[3][3][P];
  if constexpr (OP == OP_HESS) {
    fwd_3d_areas<P, Q, R>(a, X, ta, tb, s, V);
    __syncthreads();
    fwd_3d_areas<P, Q, R>(a, dX, ta, tb, s, dV);
  } else {
    // row q1 = ta of the tables (pass 23 contracts y for its own q1)
    R Bq[P], Gq[P];
#pragma unroll
    for (int i = 0; i < P; ++i) { Bq[i] = a.B[0][i]; Gq[i] = a.G[0][i]; }
#pragma unroll
    for (int q = 1; q < Q; ++q)
      if (ta == q) {
#pragma unroll
        for (int i = 0; i < P; ++i) { Bq[i] = a.B[q][i]; Gq[i] = a.G[q][i]; }
      }
    fwd_3d<P, Q, R>(a, X, ta, tb, Bq, Gq, s, V);
    // keep the scheduler from starting the point loop inside the forward
    // passes (that raises the register peak of the kernel)
    __builtin_amdgcn_sched_barrier(0);
  }

  // pass 3, lane (q1, q2): x-contraction per point q0, the point kernel, and
  // the x-transposed contraction accumulated in registers
  double acc = 0.0, mind = __builtin_huge_val();
  R Racc[3][3][P];
#pragma unroll
  for (int tt = 0; tt < 3; ++tt)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Racc[tt][c][i0] = 0;

  if (tb < Q) {
    const double w12 =
        a.w[ta] * a.w[tb] * (TGT >= TGT_QPS ? 1.0 : a.wdetW) * (a.scale ? *a.scale : 1.0);
    double sq[Q];   // this lane's row of target sizes (q0 = 0..Q-1)
    if constexpr (TGT == TGT_QPS) {
      const double* ts = a.tsize + (int64_t)e * (Q * Q * Q) + Q * ta + Q * Q * tb;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    const double* tm = target_row<Q * Q * Q, TGT>(a, e, Q * ta + Q * Q * tb);
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
      double wdet = w12 * a.w[q0], detWq = a.detW, kY = wdet, detA = 0.0;
      if constexpr (TGT == TGT_QPS) qp_scale<3, R>(sq[q0], A, dA, wdet, detWq, kY);
      if constexpr (TGT == TGT_MAT) {
        R Wi[3][3];
        double Wid[3][3];
        wdet *= load_point_target3<R>(tm + a.tm_pt * q0, Wi, Wid);
        kY = wdet;
        point_op<3, METRIC, R, OP, false>(Wi, Wid, A, dA, wdet, detWq, kY, acc, mind, Y, detA);
      } else {
        if constexpr (TGT == TGT_CW) {
          wdet *= tm[q0];
          kY = wdet;
        }
        point_op<3, METRIC, R, OP, ISO>(a.Winv, a.Winvd, A, dA, wdet, detWq, kY, acc, mind, Y, detA);
      }
      if constexpr (OP == OP_SIZE) {
        if (active) a.out[(int64_t)e * (Q * Q * Q) + q0 + Q * ta + Q * Q * tb] = size_of<3>(detA);
      }
      if constexpr (OP == OP_JINV) {   // A^{-1} = cof(A)^t / det A, and the weight omega
        if (active) {
          double Ad[3][3], Cd[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ad[i][j] = (double)A[i][j];
          cofactor<3, double>(Ad, Cd);
          double* o = a.out + ((int64_t)e * (Q * Q * Q) + q0 + Q * ta + Q * Q * tb) * 10;
          const double r = 1.0 / detA;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) o[3 * i + j] = Cd[j][i] * r;
          o[9] = a.wdetW;
        }
      }
      if constexpr (!ENERGY_LIKE) {
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

  // the scatter's old values, loaded now so the passes below hide latency
  // (with the penalty: before it, which then adds its share to them)
  // (with an element vector: no old values, the element's own share only)
  double old[3][P];
  auto load_old = [&]() {
    if (active && p1) {
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) {
        const bool fresh = EV || first_touch<NPE>(a.first, kk, ta + P * tb + P * P * i2);
#pragma unroll
        for (int c = 0; c < 3; ++c) old[c][i2] = fresh ? 0.0 : a.out[c * a.n_node + node[i2]];
      }
    }
  };
  // the scatter of the value of local node (ta, tb, i2), component c (EV:
  // to the node's entry in the element vector)
  auto put = [&](int c, int i2, double val) {
    // (EV: val is the element's own FP64 or FP32 value, exact in R)
    if constexpr (EV) a.evec[(int64_t)c * a.n_ent + a.evpos[(int64_t)e * NPE + ta + P * tb + P * P * i2]] = (R)val;
    else a.out[c * a.n_node + node[i2]] = val;
  };
  if constexpr (PEN) {   // the penalty's share 2 delta det W (M1 x M1 x M1 v) joins the old values
    __syncthreads();   // the forward data is dead
    double w[3][P];
    penalty_pass_3d<P, Q>(a, a.v, node, p1, ta, tb, s, w);
    load_old();
    if (active && p1) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) old[c][i2] += a.kpen * w[c][i2];
    }
  }
  if constexpr (OP == OP_ENERGY || OP == OP_EG || OP == OP_SIZE || OP == OP_JINV) {
    if (!active) { acc = 0.0; mind = __builtin_huge_val(); }
    block_reduce_sum_min<C::BLOCK>(acc, mind, red, a.part + blk, a.part_min + blk);
  }
  if constexpr (!ENERGY_LIKE) {
    if constexpr (!PEN) load_old();
    __syncthreads();   // the forward data is dead
    if constexpr (OP == OP_HESS) {
      // all components at once through the lane areas.  Pass 3': lane
      // (q1, q2) writes into exactly the V slots it read.
      if (tb < Q) {
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) {
          R* ar = s + L::area(tb, i0);
#pragma unroll
          for (int tt = 0; tt < 3; ++tt)
#pragma unroll
            for (int c = 0; c < 3; ++c) ar[L::av(tt, c, ta)] = Racc[tt][c][i0];
        }
      }
      __syncthreads();
      // pass 2': lane (i0 = ta, q2 = tb), own area, sum over q1
      if (ta < P && tb < Q) {
        R* ar = s + L::area(tb, ta);
        R r[3][3][Q];
#pragma unroll
        for (int tt = 0; tt < 3; ++tt)
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1) r[tt][c][q1] = ar[L::av(tt, c, q1)];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int i1 = 0; i1 < P; ++i1) {
            R sb = 0, sg = 0;
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1) {
              sb += a.B[q1][i1] * r[0][c][q1] + a.G[q1][i1] * r[1][c][q1];
              sg += a.B[q1][i1] * r[2][c][q1];
            }
            ar[L::au(0, c, i1)] = sb;
            ar[L::au(1, c, i1)] = sg;
          }
      }
      __syncthreads();
      // pass 1': lane (i0 = ta, i1 = tb), sum over q2, then the scatter
      if (active && p1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          R sb[Q], sg[Q];
#pragma unroll
          for (int q2 = 0; q2 < Q; ++q2) {
            const R* ar = s + L::area(q2, ta);
            sb[q2] = ar[L::au(0, c, tb)];
            sg[q2] = ar[L::au(1, c, tb)];
          }
#pragma unroll
          for (int i2 = 0; i2 < P; ++i2) {
            R v = 0;
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2) v += a.B[q2][i2] * sb[q2] + a.G[q2][i2] * sg[q2];
            put(c, i2, old[c][i2] + (double)v);
          }
        }
      }
    } else {
    // the transposed y- and z-contractions, one component at a time
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (tb < Q) {    // pass 3': lane (q1, q2) hands over its x-transposed sums
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0)
#pragma unroll
          for (int tt = 0; tt < 3; ++tt) s[L::r(tb, i0, tt, ta)] = Racc[tt][c][i0];
      }
      __syncthreads();
      if (ta < P && tb < Q) {   // pass 2': lane (i0 = ta, q2 = tb), sum over q1
        R r[3][Q];
#pragma unroll
        for (int tt = 0; tt < 3; ++tt)
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) r[tt][q1] = s[L::r(tb, ta, tt, q1)];
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          R sb = 0, sg = 0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) {
            sb += a.B[q1][i1] * r[0][q1] + a.G[q1][i1] * r[1][q1];
            sg += a.B[q1][i1] * r[2][q1];
          }
          R* p = s + L::s(ta, i1, tb);
          p[0] = sb;
          p[1] = sg;
        }
      }
      __syncthreads();
      if (active && p1) {       // pass 1': lane (i0 = ta, i1 = tb), sum over q2, scatter
        R sb[Q], sg[Q];
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const R* p = s + L::s(ta, tb, q2);
          sb[q2] = p[0];
          sg[q2] = p[1];
        }
#pragma unroll
        for (int i2 = 0; i2 < P; ++i2) {
          R v = 0;
#pragma unroll
          for (int q2 = 0; q2 < Q; ++q2) v += a.B[q2][i2] * sb[q2] + a.G[q2][i2] * sg[q2];
          put(c, i2, old[c][i2] + (double)v);
        }
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

template <int P, int Q, typename R, bool AFFINE>
__device__ __forceinline__ void load_pencil_2d(const ElemArgs<P, Q, R>& a, const double* __restrict__ f,
                                               const int (&node)[P], const int32_t* __restrict__ en, int i0,
                                               R (&X)[2][P], R (&J0r)[2][2]) {
  double org[3], J0[3][3];
  element_frame<2, P, AFFINE>(f, a.n_node, en, org, J0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int l = 0; l < 2; ++l) J0r[c][l] = (R)(J0[c][l] * a.jscale);
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if constexpr (AFFINE)
        X[c][i1] = (R)(f[c * a.n_node + node[i1]] - org[c] - J0[c][0] * a.xi[i0] - J0[c][1] * a.xi[i1]);
      else
        X[c][i1] = (R)(f[c * a.n_node + node[i1]] - org[c]);
    }
}

// Pass 1 (y) of the forward contraction into LDS, then lane q1 = ta reads
// its U pencil.
template <int P, int Q, typename R>
__device__ __forceinline__ void fwd_2d(const ElemArgs<P, Q, R>& a, const R (&X)[2][P], int ta, R* __restrict__ s,
                                       R (&U)[2][2][P]) {
  if (ta < P) {   // lane i0 = ta
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        R ub = 0, ug = 0;
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) { ub += a.B[q1][i1] * X[c][i1]; ug += a.G[q1][i1] * X[c][i1]; }
        s[uidx2<P, Q>(0, c, q1, ta)] = ub;
        s[uidx2<P, Q>(1, c, q1, ta)] = ug;
      }
  }
  __syncthreads();
  if (ta < Q) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) U[tt][c][i0] = s[uidx2<P, Q>(tt, c, ta, i0)];
  }
}

// fwd_2d for one component c through an LDS area of 2 Q P values
// [t][q1][i0] (the split passes of elem2d_work).
template <int P, int Q, typename R>
__device__ __forceinline__ void fwd_2d_c(const ElemArgs<P, Q, R>& a, const R (&X)[2][P], int c, int ta,
                                         R* __restrict__ s, R (&U)[2][2][P]) {
  if (ta < P) {   // lane i0 = ta
#pragma unroll
    for (int q1 = 0; q1 < Q; ++q1) {
      R ub = 0, ug = 0;
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) { ub += a.B[q1][i1] * X[c][i1]; ug += a.G[q1][i1] * X[c][i1]; }
      s[q1 * P + ta] = ub;
      s[(Q + q1) * P + ta] = ug;
    }
  }
  __syncthreads();
  if (ta < Q) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) U[tt][c][i0] = s[(tt * Q + ta) * P + i0];
  }
}

// The forward contraction of one field: both components through the LDS
// area at once, or (split) one after the other through half the area.
template <int P, int Q, typename R>
__device__ __forceinline__ void fwd_2d_field(const ElemArgs<P, Q, R>& a, const R (&X)[2][P], int ta,
                                             R* __restrict__ s, R (&U)[2][2][P], bool split) {
  if (split) {
    fwd_2d_c<P, Q, R>(a, X, 0, ta, s, U);
    __syncthreads();
    fwd_2d_c<P, Q, R>(a, X, 1, ta, s, U);
  } else {
    fwd_2d<P, Q, R>(a, X, ta, s, U);
  }
}

// The work of one 2D element on lane ta once its field pencils X (and dX for
// the Hessian action) are in registers: the forward contraction through the
// element's LDS area s, the point loop (the energy terms add to acc and
// mind; OP_SIZE and OP_JINV write their per-point results), and for the
// operations with a scatter the transposed contraction back through s, after
// which lane ta < P holds in V[c][i1] the element's share of local node
// (ta, i1).  Every lane of the block calls it (it holds barriers); e is the
// element's index in the order of the per-point target data.  split (uniform
// over the block): the LDS area holds one component at a time
// (elem2d_lds_values(P, Q, true)), at the cost of four more barriers (six
// for the Hessian action); the sums and their order are the same.
template <int P, int Q, int METRIC, typename R, int OP, int TGT>
__device__ __forceinline__ void elem2d_work(const ElemArgs<P, Q, R>& a, int e, int ta, bool active, R* __restrict__ s,
                                            const R (&X)[2][P], const R (&dX)[2][P], const R (&J0x)[2][2],
                                            const R (&J0v)[2][2], double& acc, double& mind, R (&V)[2][P],
                                            bool split) {
  constexpr bool ISO = TGT == TGT_ISO || TGT == TGT_QPS;
  constexpr bool ENERGY_LIKE = OP == OP_ENERGY || OP == OP_SIZE || OP == OP_JINV;
  constexpr bool AFFINE = sizeof(R) == 4;
  R U[2][2][P], dU[2][2][P];
  fwd_2d_field<P, Q, R>(a, X, ta, s, U, split);
  if constexpr (OP == OP_HESS) {
    __syncthreads();
    fwd_2d_field<P, Q, R>(a, dX, ta, s, dU, split);
  }

  R Racc[2][2][P];
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Racc[tt][c][i0] = 0;

  if (ta < Q) {   // lane q1 = ta
    const double w1 = a.w[ta] * (TGT >= TGT_QPS ? 1.0 : a.wdetW) * (a.scale ? *a.scale : 1.0);
    double sq[Q];   // this lane's row of target sizes
    if constexpr (TGT == TGT_QPS) {
      const double* ts = a.tsize + (int64_t)e * (Q * Q) + Q * ta;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    const double* tm = target_row<Q * Q, TGT>(a, e, Q * ta);
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
      double wdet = w1 * a.w[q0], detWq = a.detW, kY = wdet, detA = 0.0;
      if constexpr (TGT == TGT_QPS) qp_scale<2, R>(sq[q0], A, dA, wdet, detWq, kY);
      if constexpr (TGT == TGT_MAT) {
        R Wi[3][3];
        double Wid[3][3];
        wdet *= load_point_target2<R>(tm + a.tm_pt * q0, Wi, Wid);
        kY = wdet;
        point_op<2, METRIC, R, OP, false>(Wi, Wid, A, dA, wdet, detWq, kY, acc, mind, Y, detA);
      } else {
        if constexpr (TGT == TGT_CW) {
          wdet *= tm[q0];
          kY = wdet;
        }
        point_op<2, METRIC, R, OP, ISO>(a.Winv, a.Winvd, A, dA, wdet, detWq, kY, acc, mind, Y, detA);
      }
      if constexpr (OP == OP_SIZE) {
        if (active) a.out[(int64_t)e * (Q * Q) + q0 + Q * ta] = size_of<2>(detA);
      }
      if constexpr (OP == OP_JINV) {   // A^{-1} = adj(A) / det A, and the weight omega
        if (active) {
          double* o = a.out + ((int64_t)e * (Q * Q) + q0 + Q * ta) * 5;
          const double r = 1.0 / detA;
          o[0] = (double)A[1][1] * r;
          o[1] = -(double)A[0][1] * r;
          o[2] = -(double)A[1][0] * r;
          o[3] = (double)A[0][0] * r;
          o[4] = a.wdetW;
        }
      }
      if constexpr (!ENERGY_LIKE) {
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

  if (!ENERGY_LIKE && split) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      // pass 2': lane q1 writes its own row of slots (the ones it read
      // last), so only the second component waits for the first's readers
      if (c == 1) __syncthreads();
      if (ta < Q) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) s[(tt * Q + ta) * P + i0] = Racc[tt][c][i0];
      }
      __syncthreads();
      // pass 1': lane i0 = ta
      if (ta < P) {
        R rb[Q], rg[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) { rb[q1] = s[q1 * P + ta]; rg[q1] = s[(Q + q1) * P + ta]; }
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          R v = 0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) v += a.B[q1][i1] * rb[q1] + a.G[q1][i1] * rg[q1];
          V[c][i1] = v;
        }
      }
    }
  }
  if (!ENERGY_LIKE && !split) {
    // pass 2': lane q1 writes its own U slots, no barrier needed first
    if (ta < Q) {
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int i0 = 0; i0 < P; ++i0) s[uidx2<P, Q>(tt, c, ta, i0)] = Racc[tt][c][i0];
    }
    __syncthreads();
    // pass 1': lane i0 = ta
    if (ta < P) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R rb[Q], rg[Q];
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) { rb[q1] = s[uidx2<P, Q>(0, c, q1, ta)]; rg[q1] = s[uidx2<P, Q>(1, c, q1, ta)]; }
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          R v = 0;
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) v += a.B[q1][i1] * rb[q1] + a.G[q1][i1] * rg[q1];
          V[c][i1] = v;
        }
      }
    }
  }
}

// EV: the element-vector instantiation (gradient kinds only): each lane
// stores its nodes' values at their entries of the element vector instead of
// the read-modify-write.
template <int P, int Q, int METRIC, typename R, int OP, int TGT, bool EV = false>
__global__ void __launch_bounds__((Cfg<2, P, Q, R>::BLOCK))
elem_kernel_2d(const ElemArgs<P, Q, R> a) {
  using C = Cfg<2, P, Q, R>;
  constexpr bool ENERGY_LIKE = OP == OP_ENERGY || OP == OP_SIZE || OP == OP_JINV;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P;
  constexpr bool AFFINE = sizeof(R) == 4;
  constexpr int NE = OP == OP_HESS ? C::NEH : C::NE;
  __shared__ R s_all[EPB * NE];
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
  R* s = s_all + le * C::NE;
  const bool p1 = ta < P;

  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1) node[i1] = p1 ? en[ta + P * i1] : en[0];
  R X[2][P], dX[2][P], J0x[2][2], J0v[2][2];
  load_pencil_2d<P, Q, R, AFFINE>(a, a.x, node, en, p1 ? ta : 0, X, J0x);
  if constexpr (OP == OP_HESS) load_pencil_2d<P, Q, R, AFFINE>(a, a.v, node, en, p1 ? ta : 0, dX, J0v);
  // the scatter's old values, loaded with the fields: a 2D colour launch
  // holds about one round of waves, so their latency would otherwise add to
  // the launch's dependent chain
  double old[2][P];
  if constexpr (!ENERGY_LIKE && !EV) {
    if (active && p1) {
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) {
        const bool fresh = first_touch<NPE>(a.first, kk, ta + P * i1);
#pragma unroll
        for (int c = 0; c < 2; ++c) old[c][i1] = fresh ? 0.0 : a.out[c * a.n_node + node[i1]];
      }
    }
  }

  double acc = 0.0, mind = __builtin_huge_val();
  R V[2][P];
  elem2d_work<P, Q, METRIC, R, OP, TGT>(a, e, ta, active, s, X, dX, J0x, J0v, acc, mind, V, false);

  if constexpr (OP == OP_ENERGY || OP == OP_EG || OP == OP_SIZE || OP == OP_JINV) {
    if (!active) { acc = 0.0; mind = __builtin_huge_val(); }
    block_reduce_sum_min<C::BLOCK>(acc, mind, red, a.part + blk, a.part_min + blk);
  }
  if constexpr (!ENERGY_LIKE) {
    if (active && p1) {   // the scatter
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) {
          if constexpr (EV) a.evec[(int64_t)c * a.n_ent + a.evpos[(int64_t)e * NPE + ta + P * i1]] = V[c][i1];
          else a.out[c * a.n_node + node[i1]] = old[c][i1] + (double)V[c][i1];
        }
    }
  }
}

// ------------------------------------------------- 2D owner-computes tiles

template <int P, int Q, typename R, int OP>
struct TileCfg {
  static constexpr int EPR = tile_epr(Q);              // elements per round
  static constexpr bool CAN_SPLIT = tile_can_split((int)sizeof(R), OP == OP_HESS);
  static constexpr int NE = elem2d_lds_values(P, Q);              // LDS values per element
  static constexpr int NE_SPLIT = elem2d_lds_values(P, Q, true);  // the same, split passes
};

// load_pencil_2d for an element of a tile: the same FP64 operations on the
// same global values, with the nodes' global ids gn (this lane's pencil)
// and c00, c10, c01 (the corners of the element frame).
template <int P, int Q, typename R, bool AFFINE>
__device__ __forceinline__ void tile_pencil_2d(const ElemArgs<P, Q, R>& a, const double* __restrict__ f,
                                               const int (&gn)[P], int c00, int c10, int c01, int i0,
                                               R (&X)[2][P], R (&J0r)[2][2]) {
  double org[2], J0[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int c = 0; c < 2; ++c) org[c] = f[c * a.n_node + c00];
  if constexpr (AFFINE) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      J0[c][0] = f[c * a.n_node + c10] - org[c];
      J0[c][1] = f[c * a.n_node + c01] - org[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int l = 0; l < 2; ++l) J0r[c][l] = (R)(J0[c][l] * a.jscale);
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if constexpr (AFFINE)
        X[c][i1] = (R)(f[c * a.n_node + gn[i1]] - org[c] - J0[c][0] * a.xi[i0] - J0[c][1] * a.xi[i1]);
      else
        X[c][i1] = (R)(f[c * a.n_node + gn[i1]] - org[c]);
    }
}

// One workgroup per tile (OP_GRAD, OP_EG, OP_HESS; see TileParams): the
// element work is elem2d_work, as in the colour launches, on the same
// gathered field values; only where the contributions go differs.  LDS:
// the accumulators [2][nn] (FP64), the element areas, the node ids [nn].
// Energy partials (OP_EG): one per tile.
template <int P, int Q, int METRIC, typename R, int OP, int TGT>
__global__ void __launch_bounds__(TILE_BLOCK)
tile_kernel_2d(const ElemArgs<P, Q, R> a, const TileParams tp) {
  using TC = TileCfg<P, Q, R, OP>;
  constexpr int NPE = P * P, EPR = TC::EPR;
  constexpr bool AFFINE = sizeof(R) == 4;
  constexpr bool HESS = OP == OP_HESS;
  extern __shared__ double lds[];
  __shared__ double red[2 * (TILE_BLOCK / 64)];

  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int n0 = tp.node_off[tile], nn = tp.node_off[tile + 1] - n0;
  const bool split = TC::CAN_SPLIT && tp.split;
  const int ne = split ? TC::NE_SPLIT : TC::NE;
  double* acc = lds;                                           // [2][nn]
  R* s_all = reinterpret_cast<R*>(acc + 2 * nn);               // [EPR][ne]
  int* ids = reinterpret_cast<int*>(s_all + EPR * ne);         // [nn]
  for (int l = tid; l < nn; l += TILE_BLOCK) {
    ids[l] = tp.node[n0 + l];
    acc[l] = 0.0;
    acc[nn + l] = 0.0;
  }
  __syncthreads();

  const int le_raw = tid / Q;
  const int le = le_raw < EPR ? le_raw : EPR - 1;
  const int ta = le_raw < EPR ? tid - le_raw * Q : Q;   // idle pad lanes take no part
  const bool p1 = ta < P;
  R* s = s_all + le * ne;
  const int r0 = tp.round_off[tile], nr = tp.round_off[tile + 1] - r0;
  double eacc = 0.0, emin = __builtin_huge_val();
  for (int r = 0; r < nr; ++r) {
    const int64_t slot = (int64_t)(r0 + r) * EPR + le;
    const int e_raw = le_raw < EPR ? tp.slot_elem[slot] : -1;
    const bool active = e_raw >= 0;
    const int e = active ? e_raw : 0;              // empty slots compute on local node 0, write nothing
    const uint16_t* en = tp.slot_lnode + slot * NPE;
    int ln[P], gn[P];
#pragma unroll
    for (int i1 = 0; i1 < P; ++i1) {
      ln[i1] = p1 ? en[ta + P * i1] : en[0];
      gn[i1] = ids[ln[i1]];
    }
    const int c00 = ids[en[0]], c10 = ids[en[P - 1]], c01 = ids[en[P * (P - 1)]];
    R X[2][P], dX[2][P], J0x[2][2], J0v[2][2];
    tile_pencil_2d<P, Q, R, AFFINE>(a, a.x, gn, c00, c10, c01, p1 ? ta : 0, X, J0x);
    if constexpr (HESS) tile_pencil_2d<P, Q, R, AFFINE>(a, a.v, gn, c00, c10, c01, p1 ? ta : 0, dX, J0v);
    double racc = 0.0, rmin = __builtin_huge_val();
    R V[2][P];
    elem2d_work<P, Q, METRIC, R, OP, TGT>(a, e, ta, active, s, X, dX, J0x, J0v, racc, rmin, V, split);
    if (active) {
      eacc += racc;
      emin = fmin(emin, rmin);
    }
    if (active && p1) {   // the elements of a round share no node, lanes of one element own distinct nodes
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i1 = 0; i1 < P; ++i1) acc[c * nn + ln[i1]] += (double)V[c][i1];
    }
    __syncthreads();   // the next round reuses the element areas and may share these nodes
  }

  for (int l = tid; l < nn; l += TILE_BLOCK) {
    const int64_t g = ids[l];
    const int sl = tp.slot[n0 + l];
    if (sl < 0) {
      a.out[g] = acc[l];
      a.out[a.n_node + g] = acc[nn + l];
    } else {
      tp.halo[sl] = acc[l];
      tp.halo[tp.n_slot + sl] = acc[nn + l];
    }
  }
  if constexpr (OP == OP_EG) block_reduce_sum_min<TILE_BLOCK>(eacc, emin, red, a.part + tile, a.part_min + tile);
}

// ------------------------------------------------------- Hessian diagonal
//
// diag(d^2F/dx^2) at DOF (c, I) collects, from every element E holding I as
// local node i,  sum_q w_q det W  g_i^T K_c g_i  with g_i = W^{-t} grad w_i
// at point q and K_c = d^2 mu / (dT_c. dT_c.) (mu_second_rows): the unit
// vector of the DOF moves row c of A by (grad w_i)^T.  In reference
// coordinates this is  sum_q sum_{l,m} Kt_c,lm (d_l w_i)(d_m w_i),
// Kt_c = w det W W^{-1} K_c W^{-t} (isotropic W = sI: G carries 1/s and
// Kt_c = w det W K_c).  The product (d_l w_i)(d_m w_i) of two tensor-product
// gradients is again a tensor product, of the squared tables BB = B^2,
// BG = B G, GG = G^2, so the diagonal is a transposed sum-factorized
// contraction of the d(d+1)/2 fields Kt_c,lm (times 2 for l != m) per
// component, with the table of pair (l, m) in direction d being GG if
// l = m = d, BG if exactly one of l, m is d, else BB.
template <int P, int Q, typename R>
struct DiagArgs : ElemArgs<P, Q, R> {
  R BB[Q][P];
  R BG[Q][P];
  R GG[Q][P];
};

// 3D pairs (l, m): 0 (0,0), 1 (1,1), 2 (2,2), 3 (0,1), 4 (0,2), 5 (1,2).
//   x tables: GG BB BB BG BG BB;  y tables: BB GG BB BG BB BG;
//   z tables: BB BB GG BB BG BG, so after the y-pass the pairs merge into
//   three z-groups: BB (pairs 0, 1, 3), BG (4, 5), GG (2).
// LDS per element: U of the forward passes, then per component the
// x-transposed sums R6 [q2][i0][pair][q1] and the y-transposed sums
// S3 [i0][i1][q2][group].
template <int P, int Q> struct LdsDiag3 {
  static constexpr int NR = Q * P * 6 * Q;
  static constexpr int NS = P * P * Q * 3;
  static constexpr int N = Lds3<P, Q>::NU > NR + NS ? Lds3<P, Q>::NU : NR + NS;
  static __device__ __forceinline__ constexpr int r(int q2, int i0, int pr, int q1) {
    return ((q2 * P + i0) * 6 + pr) * Q + q1;
  }
  static __device__ __forceinline__ constexpr int s(int i0, int i1, int q2) { return NR + ((i0 * P + i1) * Q + q2) * 3; }
};

// K_c <- W^{-1} K_c W^{-t} (general constant target), K_c symmetric and
// stored as its unique entries (SymPairs order)
template <int D, typename R>
__device__ __forceinline__ void target_congruence(const R (&Wi)[3][3], R (&K6)[D][SymPairs<D>::N]) {
  using SP = SymPairs<D>;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    R K[D][D], M[D][D];
#pragma unroll
    for (int pr = 0; pr < SP::N; ++pr) {
      K[SP::l[pr]][SP::m[pr]] = K6[c][pr];
      K[SP::m[pr]][SP::l[pr]] = K6[c][pr];
    }
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
      for (int m = 0; m < D; ++m) {
        R t = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) t += K[l][k] * Wi[m][k];
        M[l][m] = t;                         // (K_c W^{-t})_lm
      }
#pragma unroll
    for (int pr = 0; pr < SP::N; ++pr) {
      R t = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) t += Wi[SP::l[pr]][k] * M[k][SP::m[pr]];
      K6[c][pr] = t;
    }
  }
}

template <int P, int Q, int METRIC, typename R, int TGT, bool EV = false>
// EV (element-vector stores) asks for two waves per SIMD up to order 2 with
// a constant target: without the request the Q2 kernel lands 6 registers
// above 256, one wave.
__global__ void __launch_bounds__((Cfg<3, P, Q, R>::BLOCK))
__attribute__((amdgpu_waves_per_eu(EV && P <= 3 && (TGT == TGT_GEN || TGT == TGT_ISO) ? 2 : 1)))
diag_kernel_3d(const DiagArgs<P, Q, R> a) {
  constexpr bool ISO = TGT == TGT_ISO || TGT == TGT_QPS;
  using C = Cfg<3, P, Q, R>;
  using LD = LdsDiag3<P, Q>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P * P;
  constexpr bool AFFINE = sizeof(R) == 4;
  constexpr int NE = LD::N + TMOP_ELEM_PAD;
  __shared__ R s_all[EPB * NE];

  const int tid = threadIdx.x;
  const int le_raw = tid / TPE;
  const int le = le_raw < EPB ? le_raw : EPB - 1;
  const int t = tid - le_raw * TPE;
  const int ta = le_raw < EPB ? t % Q : Q;
  const int tb = le_raw < EPB ? t / Q : Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int k = blk * EPB + le;
  const bool active = le_raw < EPB && k < a.n_list;
  const int kk = k < a.n_list ? k : a.n_list - 1;
  const int e = a.list ? a.list[kk] : kk;
  R* s = s_all + le * NE;
  const bool p1 = ta < P && tb < P;

  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2) node[i2] = p1 ? en[ta + P * tb + P * P * i2] : en[0];
  R X[3][P], J0x[3][3];
  load_pencil_3d<P, Q, R, AFFINE>(a, a.x, node, en, p1 ? ta : 0, p1 ? tb : 0, X, J0x);

  R Bq[P], Gq[P];
#pragma unroll
  for (int i = 0; i < P; ++i) { Bq[i] = a.B[0][i]; Gq[i] = a.G[0][i]; }
#pragma unroll
  for (int q = 1; q < Q; ++q)
    if (ta == q) {
#pragma unroll
      for (int i = 0; i < P; ++i) { Bq[i] = a.B[q][i]; Gq[i] = a.G[q][i]; }
    }
  R V[3][3][P];
  fwd_3d<P, Q, R>(a, X, ta, tb, Bq, Gq, s, V);
  __builtin_amdgcn_sched_barrier(0);

  // x-transposed sums of the six pair fields, lane (q1, q2)
  R Rd[6][3][P];
#pragma unroll
  for (int pr = 0; pr < 6; ++pr)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Rd[pr][c][i0] = 0;
  if (tb < Q) {
    const double w12 = a.w[ta] * a.w[tb] * (TGT >= TGT_QPS ? 1.0 : a.wdetW);
    double sq[Q];
    if constexpr (TGT == TGT_QPS) {
      const double* ts = a.tsize + (int64_t)e * (Q * Q * Q) + Q * ta + Q * Q * tb;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    const double* tm = target_row<Q * Q * Q, TGT>(a, e, Q * ta + Q * Q * tb);
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      R A[3][3];
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
      }
      R T[3][3], K[3][6];
      double kK = w12 * a.w[q0];
      if constexpr (TGT == TGT_QPS) {   // T = A / s; W^{-1} K W^{-t} = K / s^2, det W = s^3
        const R r = (R)(1.0 / sq[q0]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) A[i][j] *= r;
        kK *= sq[q0];
      }
      if constexpr (TGT == TGT_MAT) {
        R Wi[3][3];
        double Wid[3][3];
        kK *= load_point_target3<R>(tm + a.tm_pt * q0, Wi, Wid);
        right_mul<3, R, false>(A, Wi, T);
        mu_second_rows<METRIC, R>(T, (R)kK, K);
        target_congruence<3, R>(Wi, K);
      } else {
        if constexpr (TGT == TGT_CW) kK *= tm[q0];
        right_mul<3, R, ISO>(A, a.Winv, T);
        mu_second_rows<METRIC, R>(T, (R)kK, K);
        if constexpr (!ISO) target_congruence<3, R>(a.Winv, K);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R f0 = K[c][0], f1 = K[c][1], f2 = K[c][2];
        const R f3 = R(2) * K[c][3], f4 = R(2) * K[c][4], f5 = R(2) * K[c][5];
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) {
          Rd[0][c][i0] += a.GG[q0][i0] * f0;
          Rd[1][c][i0] += a.BB[q0][i0] * f1;
          Rd[2][c][i0] += a.BB[q0][i0] * f2;
          Rd[3][c][i0] += a.BG[q0][i0] * f3;
          Rd[4][c][i0] += a.BG[q0][i0] * f4;
          Rd[5][c][i0] += a.BB[q0][i0] * f5;
        }
      }
    }
  }

  bool fresh[P];   // EV: each element stores its own share, no old values
#pragma unroll
  for (int i2 = 0; i2 < P; ++i2) fresh[i2] = EV || first_touch<NPE>(a.first, kk, ta + P * tb + P * P * i2);
  __syncthreads();   // U is dead
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // this component's old values, loaded before the passes that hide them
    double old[P];
    if (active && p1) {
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) old[i2] = fresh[i2] ? 0.0 : a.out[c * a.n_node + node[i2]];
    }
    if (tb < Q) {    // lane (q1, q2) hands over its x-transposed sums
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0)
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) s[LD::r(tb, i0, pr, ta)] = Rd[pr][c][i0];
    }
    __syncthreads();
    if (ta < P && tb < Q) {   // lane (i0 = ta, q2 = tb): y-transposed, grouped by z table
      R r[6][Q];
#pragma unroll
      for (int pr = 0; pr < 6; ++pr)
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) r[pr][q1] = s[LD::r(tb, ta, pr, q1)];
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) {
        R gbb = 0, gbg = 0, ggg = 0;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          gbb += a.BB[q1][i1] * r[0][q1] + a.GG[q1][i1] * r[1][q1] + a.BG[q1][i1] * r[3][q1];
          gbg += a.BB[q1][i1] * r[4][q1] + a.BG[q1][i1] * r[5][q1];
          ggg += a.BB[q1][i1] * r[2][q1];
        }
        R* p = s + LD::s(ta, i1, tb);
        p[0] = gbb;
        p[1] = gbg;
        p[2] = ggg;
      }
    }
    __syncthreads();
    if (active && p1) {       // lane (i0 = ta, i1 = tb): z-transposed, then the scatter
      R gbb[Q], gbg[Q], ggg[Q];
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const R* p = s + LD::s(ta, tb, q2);
        gbb[q2] = p[0];
        gbg[q2] = p[1];
        ggg[q2] = p[2];
      }
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) {
        R v = 0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) v += a.BB[q2][i2] * gbb[q2] + a.BG[q2][i2] * gbg[q2] + a.GG[q2][i2] * ggg[q2];
        if constexpr (EV) a.evec[(int64_t)c * a.n_ent + a.evpos[(int64_t)e * NPE + ta + P * tb + P * P * i2]] = v;
        else a.out[c * a.n_node + node[i2]] = old[i2] + (double)v;
      }
    }
  }
}

// 2D pairs (l, m): 0 (0,0), 1 (1,1), 2 (0,1); x tables GG BB BG, y tables
// BB GG BG.  LDS: the forward U, then the x-transposed sums [pair][c][q1][i0].
template <int P, int Q, int METRIC, typename R, int TGT, bool EV = false>
__global__ void __launch_bounds__((Cfg<2, P, Q, R>::BLOCK))
diag_kernel_2d(const DiagArgs<P, Q, R> a) {
  constexpr bool ISO = TGT == TGT_ISO || TGT == TGT_QPS;
  using C = Cfg<2, P, Q, R>;
  constexpr int TPE = C::TPE, EPB = C::EPB, NPE = P * P;
  constexpr bool AFFINE = sizeof(R) == 4;
  constexpr int NU = 2 * 2 * Q * P, NRD = 3 * 2 * Q * P;
  constexpr int NE = (NU > NRD ? NU : NRD) + TMOP_ELEM_PAD2;
  __shared__ R s_all[EPB * NE];

  const int tid = threadIdx.x;
  const int le_raw = tid / TPE;
  const int le = le_raw < EPB ? le_raw : EPB - 1;
  const int ta = le_raw < EPB ? tid - le_raw * TPE : Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int k = blk * EPB + le;
  const bool active = le_raw < EPB && k < a.n_list;
  const int kk = k < a.n_list ? k : a.n_list - 1;
  const int e = a.list ? a.list[kk] : kk;
  R* s = s_all + le * NE;
  const bool p1 = ta < P;

  const int32_t* en = a.elem_node + (int64_t)e * NPE;
  int node[P];
#pragma unroll
  for (int i1 = 0; i1 < P; ++i1) node[i1] = p1 ? en[ta + P * i1] : en[0];
  R X[2][P], J0x[2][2];
  load_pencil_2d<P, Q, R, AFFINE>(a, a.x, node, en, p1 ? ta : 0, X, J0x);
  R U[2][2][P];
  fwd_2d<P, Q, R>(a, X, ta, s, U);

  R Rd[3][2][P];
#pragma unroll
  for (int pr = 0; pr < 3; ++pr)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i0 = 0; i0 < P; ++i0) Rd[pr][c][i0] = 0;
  if (ta < Q) {   // lane q1 = ta
    const double w1 = a.w[ta] * (TGT >= TGT_QPS ? 1.0 : a.wdetW);
    double sq[Q];
    if constexpr (TGT == TGT_QPS) {
      const double* ts = a.tsize + (int64_t)e * (Q * Q) + Q * ta;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) sq[q0] = ts[q0];
    }
    const double* tm = target_row<Q * Q, TGT>(a, e, Q * ta);
#pragma unroll
    for (int q0 = 0; q0 < Q; ++q0) {
      R A[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R s0 = 0, s1 = 0;
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) { s0 += a.G[q0][i0] * U[0][c][i0]; s1 += a.B[q0][i0] * U[1][c][i0]; }
        if constexpr (AFFINE) { s0 += J0x[c][0]; s1 += J0x[c][1]; }
        A[c][0] = s0; A[c][1] = s1;
      }
      R T[2][2], K[2][3];
      double kK = w1 * a.w[q0];
      if constexpr (TGT == TGT_QPS) {   // T = A / s; W^{-1} K W^{-t} = K / s^2, det W = s^2
        const R r = (R)(1.0 / sq[q0]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) A[i][j] *= r;
      }
      if constexpr (TGT == TGT_MAT) {
        R Wi[3][3];
        double Wid[3][3];
        kK *= load_point_target2<R>(tm + a.tm_pt * q0, Wi, Wid);
        right_mul<2, R, false>(A, Wi, T);
        mu_second_rows<METRIC, R>(T, (R)kK, K);
        target_congruence<2, R>(Wi, K);
      } else {
        if constexpr (TGT == TGT_CW) kK *= tm[q0];
        right_mul<2, R, ISO>(A, a.Winv, T);
        mu_second_rows<METRIC, R>(T, (R)kK, K);
        if constexpr (!ISO) target_congruence<2, R>(a.Winv, K);
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const R f0 = K[c][0], f1 = K[c][1], f2 = R(2) * K[c][2];
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) {
          Rd[0][c][i0] += a.GG[q0][i0] * f0;
          Rd[1][c][i0] += a.BB[q0][i0] * f1;
          Rd[2][c][i0] += a.BG[q0][i0] * f2;
        }
      }
    }
  }

  double old[2][P];
  if (active && p1) {
#pragma unroll
    for (int i1 = 0; i1 < P; ++i1) {
      const bool fresh = EV || first_touch<NPE>(a.first, kk, ta + P * i1);   // EV: no old values
#pragma unroll
      for (int c = 0; c < 2; ++c) old[c][i1] = fresh ? 0.0 : a.out[c * a.n_node + node[i1]];
    }
  }
  __syncthreads();   // U is dead
  if (ta < Q) {
#pragma unroll
    for (int pr = 0; pr < 3; ++pr)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i0 = 0; i0 < P; ++i0) s[((pr * 2 + c) * Q + ta) * P + i0] = Rd[pr][c][i0];
  }
  __syncthreads();
  if (active && p1) {   // lane i0 = ta: y-transposed, then the scatter
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R r[3][Q];
#pragma unroll
      for (int pr = 0; pr < 3; ++pr)
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) r[pr][q1] = s[((pr * 2 + c) * Q + q1) * P + ta];
#pragma unroll
      for (int i1 = 0; i1 < P; ++i1) {
        R v = 0;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1)
          v += a.BB[q1][i1] * r[0][q1] + a.GG[q1][i1] * r[1][q1] + a.BG[q1][i1] * r[2][q1];
        if constexpr (EV) a.evec[(int64_t)c * a.n_ent + a.evpos[(int64_t)e * NPE + ta + P * i1]] = v;
        else a.out[c * a.n_node + node[i1]] = old[c][i1] + (double)v;
      }
    }
  }
}

}  // namespace tmop
