// Device library of TMOP quality metrics mu(T) and their derivatives in T.
//
// Section 3.2 / Table 3.1 define the metrics; Section 3.4 recommends writing
// them through matrix invariants so that first and second derivatives are
// easy to form.  Every metric here is mu = f(I1, I2, tau, J) with
//   I1 = |T|^2, tau = det T, C = cof T = d tau / dT, I2 = |C|^2 (3D only),
//   J = tr T (the metrics measured against T = I, dJ/dT = Id),
// and the derivatives follow from the chain rule:
//   P  = dmu/dT = 2 f1 T + f2 dI2 + ft C + fJ Id,    dI2 = 2 (I1 T - T T^t T)
//   dP = d/de P(T + e E)
//      = 2 f1 E + f2 ddI2[E] + ft dC[E]
//        + 2T (f11 a1 + f12 a2 + f1t at) + dI2 (f12 a1 + f22 a2 + f2t at)
//        + C (f1t a1 + f2t a2 + ftt at + fJt aJ) + Id fJt at,
//   a1 = 2 T:E, a2 = dI2:E, at = C:E, aJ = tr E,
//   ddI2[E] = 2 (2 (T:E) T + I1 E - E T^t T - T E^t T - T T^t E)
// (f11 = f22 = f1J = fJJ = 0 for every metric here).
// Metric values avoid the cancellation of "... - 1" where an exact identity
// allows it (2D: |T|^2 - 2 det T = (T00 - T11)^2 + (T01 + T10)^2).
#pragma once

#include <hip/hip_runtime.h>

namespace tmop {

template <typename R> __device__ __forceinline__ R rcp(R x) { return R(1) / x; }

// tau^(-1/3) with the real cube root (negative for tau < 0).  FP64: an FP32
// seed from the hardware log2/exp2 (relative error ~1e-7), then two Newton
// steps for y^-3 = tau, y <- y + y (1 - tau y^3) / 3, each of which squares
// the relative error.  No FP64 division or cube root is needed.
__device__ __forceinline__ double rcbrt(double t) {
  const float a = fabsf((float)t);
  float s = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(a) * (-1.0f / 3.0f));
  double y = (double)(t < 0.0 ? -s : s);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double y3 = y * y * y;
    y = fma(y * (1.0 / 3.0), fma(-t, y3, 1.0), y);
  }
  return y;
}
__device__ __forceinline__ float rcbrt(float t) {
  float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(t)) * (-1.0f / 3.0f));
  y = t < 0.0f ? -y : y;
  const float y3 = y * y * y;
  return fmaf(y * (1.0f / 3.0f), fmaf(-t, y3, 1.0f), y);
}

template <int D, typename R>
__device__ __forceinline__ void cofactor(const R T[D][D], R C[D][D]) {
  if constexpr (D == 2) {
    C[0][0] = T[1][1];  C[0][1] = -T[1][0];
    C[1][0] = -T[0][1]; C[1][1] = T[0][0];
  } else {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = (r + 1) % 3, b = (r + 2) % 3;   // C[r] = T[a] x T[b]
      C[r][0] = T[a][1] * T[b][2] - T[a][2] * T[b][1];
      C[r][1] = T[a][2] * T[b][0] - T[a][0] * T[b][2];
      C[r][2] = T[a][0] * T[b][1] - T[a][1] * T[b][0];
    }
  }
}

// Directional derivative of cof at T along E.
template <int D, typename R>
__device__ __forceinline__ void dcofactor(const R T[D][D], const R E[D][D], R dC[D][D]) {
  if constexpr (D == 2) {
    cofactor<2, R>(E, dC);
  } else {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = (r + 1) % 3, b = (r + 2) % 3;   // d(T[a] x T[b]) = E[a] x T[b] + T[a] x E[b]
      dC[r][0] = E[a][1] * T[b][2] - E[a][2] * T[b][1] + T[a][1] * E[b][2] - T[a][2] * E[b][1];
      dC[r][1] = E[a][2] * T[b][0] - E[a][0] * T[b][2] + T[a][2] * E[b][0] - T[a][0] * E[b][2];
      dC[r][2] = E[a][0] * T[b][1] - E[a][1] * T[b][0] + T[a][0] * E[b][1] - T[a][1] * E[b][0];
    }
  }
}

template <int D, typename R>
__device__ __forceinline__ R det(const R T[D][D]) {
  if constexpr (D == 2) return T[0][0] * T[1][1] - T[0][1] * T[1][0];
  else
    return T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1])
         - T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0])
         + T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0]);
}

// Partial derivatives of f(I1, I2, tau).  Flags tell which ones are
// identically zero so the compiler drops their terms.
template <typename R> struct Partials { R f1, f2, ft, fJ, f11, f12, f1t, f22, f2t, ftt, fJt; };

// dim, whether f depends on I2, whether it depends on J = tr T
template <int METRIC> struct MetricInfo;
template <> struct MetricInfo<1>   { static constexpr int dim = 2; static constexpr bool i2 = false, tr = false; };
template <> struct MetricInfo<2>   { static constexpr int dim = 2; static constexpr bool i2 = false, tr = false; };
template <> struct MetricInfo<7>   { static constexpr int dim = 2; static constexpr bool i2 = false, tr = false; };
template <> struct MetricInfo<9>   { static constexpr int dim = 2; static constexpr bool i2 = false, tr = false; };
template <> struct MetricInfo<14>  { static constexpr int dim = 2; static constexpr bool i2 = false, tr = true; };
template <> struct MetricInfo<77>  { static constexpr int dim = 2; static constexpr bool i2 = false, tr = false; };
template <> struct MetricInfo<98>  { static constexpr int dim = 2; static constexpr bool i2 = false, tr = true; };
// mu_98 = |T - I|^2 / tau for 3x3 T: the replication metric of Section 4.3.2 in 3D (an internal id; the
// 3D primary metrics are 302 and 303)
template <> struct MetricInfo<398> { static constexpr int dim = 3; static constexpr bool i2 = false, tr = true; };
template <> struct MetricInfo<302> { static constexpr int dim = 3; static constexpr bool i2 = true, tr = false; };
// mu_7 = |T - T^{-t}|^2 for 3x3 T (Section 3.2 gives it for any dimension): an internal id of the 3D kernels
template <> struct MetricInfo<307> { static constexpr int dim = 3; static constexpr bool i2 = true, tr = false; };
template <> struct MetricInfo<303> { static constexpr int dim = 3; static constexpr bool i2 = false, tr = false; };

template <int METRIC, typename R>
__device__ __forceinline__ Partials<R> partials(R I1, R I2, R tau, R J = R(0)) {
  Partials<R> p{};
  if constexpr (METRIC == 1) {            // f = I1
    p.f1 = R(1);
  } else if constexpr (METRIC == 9) {     // f = tau I1 + I1 / tau - 4 tau  (tau |T - T^-t|^2 in 2D)
    const R rt = rcp(tau);
    const R rt2 = rt * rt;
    p.f1 = tau + rt;  p.ft = I1 - I1 * rt2 - R(4);
    p.f1t = R(1) - rt2;  p.ftt = R(2) * I1 * rt2 * rt;
  } else if constexpr (METRIC == 77) {    // f = (tau - 1/tau)^2 / 2
    const R rt = rcp(tau);
    const R rt2 = rt * rt;
    p.ft = (tau - rt) * (R(1) + rt2);  p.ftt = R(1) + R(3) * rt2 * rt2;
  } else if constexpr (METRIC == 14) {    // f = I1 - 2 J + 2  (|T - I|^2)
    p.f1 = R(1);  p.fJ = R(-2);
  } else if constexpr (METRIC == 98 || METRIC == 398) {   // f = (I1 - 2 J + d) / tau  (|T - I|^2 / tau)
    const R rt = rcp(tau);
    const R n = I1 - R(2) * J + R(METRIC == 98 ? 2 : 3);
    p.f1 = rt;  p.fJ = R(-2) * rt;  p.ft = -n * rt * rt;
    p.f1t = -rt * rt;  p.fJt = R(2) * rt * rt;  p.ftt = R(2) * n * rt * rt * rt;
  } else if constexpr (METRIC == 2) {     // f = I1 / (2 tau) - 1
    const R rt = rcp(tau);
    const R rt2 = rt * rt;
    p.f1 = R(0.5) * rt;  p.ft = R(-0.5) * I1 * rt2;
    p.f1t = R(-0.5) * rt2; p.ftt = I1 * rt2 * rt;
  } else if constexpr (METRIC == 7) {     // f = I1 (1 + tau^-2) - 4
    const R rt = rcp(tau);
    const R rt2 = rt * rt, rt3 = rt2 * rt;
    p.f1 = R(1) + rt2;  p.ft = R(-2) * I1 * rt3;
    p.f1t = R(-2) * rt3; p.ftt = R(6) * I1 * rt3 * rt;
  } else if constexpr (METRIC == 303) {   // f = I1 tau^{-2/3} / 3 - 1
    const R y = rcbrt(tau);                   // tau^{-1/3}
    const R c = y * y;                        // tau^{-2/3}
    const R rt = c * y;                       // 1 / tau
    p.f1 = c * R(1.0 / 3.0);
    p.f1t = R(-2.0 / 9.0) * c * rt;
    p.ft = p.f1t * I1;
    p.ftt = R(10.0 / 27.0) * I1 * c * rt * rt;
  } else if constexpr (METRIC == 307) {   // f = I1 + I2 tau^-2 - 6  (|T^-1|^2 = |cof T|^2 / tau^2 in 3D)
    const R rt = rcp(tau);
    const R rt2 = rt * rt, rt3 = rt2 * rt;
    p.f1 = R(1);  p.f2 = rt2;  p.ft = R(-2) * I2 * rt3;
    p.f2t = R(-2) * rt3;  p.ftt = R(6) * I2 * rt2 * rt2;
  } else if constexpr (METRIC == 302) {   // f = I1 I2 tau^-2 / 9 - 1
    const R rt = rcp(tau);
    const R s = rt * rt * R(1.0 / 9.0);
    p.f1 = I2 * s;  p.f2 = I1 * s;  p.ft = R(-2) * I1 * I2 * s * rt;
    p.f12 = s;  p.f1t = R(-2) * I2 * s * rt;  p.f2t = R(-2) * I1 * s * rt;
    p.ftt = R(6) * I1 * I2 * s * rt * rt;
  }
  return p;
}

// mu(T) given tau = det T.
template <int METRIC, typename R>
__device__ __forceinline__ R mu_value(const R (&T)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim], R tau) {
  constexpr int D = MetricInfo<METRIC>::dim;
  if constexpr (METRIC == 2 || METRIC == 7 || METRIC == 9) {
    const R u = T[0][0] - T[1][1], w = T[0][1] + T[1][0];
    const R dev = u * u + w * w;                 // |T|^2 - 2 tau >= 0
    const R rt = rcp(tau);
    if constexpr (METRIC == 2) return R(0.5) * dev * rt;
    else if constexpr (METRIC == 7) return dev * (R(1) + rt * rt) + R(2) * (tau - R(1)) * (tau - R(1)) * rt;
    else return dev * (tau + rt) + R(2) * (tau - R(1)) * (tau - R(1));
  } else if constexpr (METRIC == 1) {
    return T[0][0] * T[0][0] + T[0][1] * T[0][1] + T[1][0] * T[1][0] + T[1][1] * T[1][1];
  } else if constexpr (METRIC == 77) {
    const R s = tau - rcp(tau);
    return R(0.5) * s * s;
  } else if constexpr (METRIC == 14 || METRIC == 98) {
    const R a = T[0][0] - R(1), b = T[1][1] - R(1);
    const R n = a * a + b * b + T[0][1] * T[0][1] + T[1][0] * T[1][0];
    if constexpr (METRIC == 14) return n;
    else return n * rcp(tau);
  } else if constexpr (METRIC == 307) {   // sum of squares of T - T^{-t} = T - cof(T) / tau, free of cancellation
    R C[3][3];
    cofactor<3, R>(T, C);
    const R rt = rcp(tau);
    R n = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R t = T[i][j] - C[i][j] * rt;
        n += t * t;
      }
    return n;
  } else if constexpr (METRIC == 398) {
    R n = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R t = T[i][j] - (i == j ? R(1) : R(0));
        n += t * t;
      }
    return n * rcp(tau);
  } else {
    R I1 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) I1 += T[i][j] * T[i][j];
    if constexpr (METRIC == 303) {
      const R y = rcbrt(tau);
      return I1 * (y * y) * R(1.0 / 3.0) - R(1);
    } else {
      R C[3][3];
      cofactor<3, R>(T, C);
      R I2 = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I2 += C[i][j] * C[i][j];
      const R rt = rcp(tau);
      return I1 * I2 * rt * rt * R(1.0 / 9.0) - R(1);
    }
  }
}

template <int D, typename R>
__device__ __forceinline__ void dI2_of(const R T[D][D], R I1, R out[D][D]) {
  // 2 (I1 T - T T^t T)
  R TTt[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R s = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += T[i][k] * T[j][k];
      TTt[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R s = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += TTt[i][k] * T[k][j];
      out[i][j] = R(2) * (I1 * T[i][j] - s);
    }
}

// P = k dmu/dT (k folds a caller's scalar weight into the coefficients).
template <int METRIC, typename R>
__device__ __forceinline__ void mu_first(const R (&T)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim], R k,
                                         R (&P)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim]) {
  constexpr int D = MetricInfo<METRIC>::dim;
  R C[D][D];
  cofactor<D, R>(T, C);
  R I1 = 0, tau = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) I1 += T[i][j] * T[i][j];
#pragma unroll
  for (int j = 0; j < D; ++j) tau += T[0][j] * C[0][j];
  R I2 = 0, J = 0;
  if constexpr (MetricInfo<METRIC>::i2) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) I2 += C[i][j] * C[i][j];
  }
  if constexpr (MetricInfo<METRIC>::tr) {
#pragma unroll
    for (int i = 0; i < D; ++i) J += T[i][i];
  }
  const Partials<R> f = partials<METRIC, R>(I1, I2, tau, J);
  const R k1 = R(2) * k * f.f1, kt = k * f.ft;
  if constexpr (MetricInfo<METRIC>::i2) {
    R dI2[D][D];
    dI2_of<D, R>(T, I1, dI2);
    const R k2 = k * f.f2;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) P[i][j] = k1 * T[i][j] + k2 * dI2[i][j] + kt * C[i][j];
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) P[i][j] = k1 * T[i][j] + kt * C[i][j];
  }
  if constexpr (MetricInfo<METRIC>::tr) {
    const R kJ = k * f.fJ;
#pragma unroll
    for (int i = 0; i < D; ++i) P[i][i] += kJ;
  }
}

// dP = k (d^2 mu / dT^2) : E (k folded into the coefficients).
template <int METRIC, typename R>
__device__ __forceinline__ void mu_second(const R (&T)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim],
                                          const R (&E)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim], R k,
                                          R (&dP)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim]) {
  constexpr int D = MetricInfo<METRIC>::dim;
  R C[D][D], dC[D][D];
  cofactor<D, R>(T, C);
  dcofactor<D, R>(T, E, dC);
  R I1 = 0, tau = 0, TE = 0, CE = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      I1 += T[i][j] * T[i][j];
      TE += T[i][j] * E[i][j];
      CE += C[i][j] * E[i][j];
    }
#pragma unroll
  for (int j = 0; j < D; ++j) tau += T[0][j] * C[0][j];
  if constexpr (!MetricInfo<METRIC>::i2) {
    R J = 0, aJ = 0;
    if constexpr (MetricInfo<METRIC>::tr) {
#pragma unroll
      for (int i = 0; i < D; ++i) { J += T[i][i]; aJ += E[i][i]; }
    }
    const Partials<R> f = partials<METRIC, R>(I1, R(0), tau, J);
    const R a1 = R(2) * TE, at = CE;
    const R kE = R(2) * k * f.f1, kd = k * f.ft;
    const R sT = R(2) * k * (f.f1t * at);         // f11 = 0 for these metrics
    R sC = k * (f.f1t * a1 + f.ftt * at);
    if constexpr (MetricInfo<METRIC>::tr) sC += k * f.fJt * aJ;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j)
        dP[i][j] = kE * E[i][j] + kd * dC[i][j] + sT * T[i][j] + sC * C[i][j];
    if constexpr (MetricInfo<METRIC>::tr) {
      const R sI = k * f.fJt * at;
#pragma unroll
      for (int i = 0; i < D; ++i) dP[i][i] += sI;
    }
  } else {
    R I2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) I2 += C[i][j] * C[i][j];
    const Partials<R> f = partials<METRIC, R>(I1, I2, tau);
    // T^t T, then the pieces of ddI2
    R TtT[D][D], TTt[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        R s = 0, u = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) { s += T[k][i] * T[k][j]; u += T[i][k] * T[j][k]; }
        TtT[i][j] = s;
        TTt[i][j] = u;
      }
    R dI2[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        R s = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += TTt[i][k] * T[k][j];
        dI2[i][j] = R(2) * (I1 * T[i][j] - s);
      }
    R a2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) a2 += dI2[i][j] * E[i][j];
    const R a1 = R(2) * TE, at = CE;
    const R sT = R(2) * k * (f.f12 * a2 + f.f1t * at);     // f11 = 0
    const R sI = k * (f.f12 * a1 + f.f2t * at);            // f22 = 0
    const R sC = k * (f.f1t * a1 + f.f2t * a2 + f.ftt * at);
    const R kE = R(2) * k * f.f1, k2 = k * f.f2, kd = k * f.ft;
    // E T^t T, T E^t T, T T^t E
    R ET[D][D], TEt[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        R s = 0, u = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) { s += E[i][k] * TtT[k][j]; u += T[i][k] * E[j][k]; }
        ET[i][j] = s;       // (E T^t T)_ij
        TEt[i][j] = u;      // (T E^t)_ij
      }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        R teT = 0, ttE = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) { teT += TEt[i][k] * T[k][j]; ttE += TTt[i][k] * E[k][j]; }
        const R ddI2 = R(2) * (R(2) * TE * T[i][j] + I1 * E[i][j] - ET[i][j] - teT - ttE);
        dP[i][j] = kE * E[i][j] + k2 * ddI2 + kd * dC[i][j]
                 + sT * T[i][j] + sI * dI2[i][j] + sC * C[i][j];
      }
  }
}

// Diagonal row blocks of the second derivative:
//   K[c][l][m] = k d^2 mu / (dT_cl dT_cm),
// the part of mu'' that a rank-one direction E = e_c g^T (one row of T
// moves) sees: E : mu''[E] = g^T K[c] g.  With E = e_c e_l^T and
// E' = e_c e_m^T the chain rule above gives, since det T is linear in each
// row (dC[E] : E' = 0) and
//   ddI2[E] : E' = 2 (T_cl T_cm + (I1 - |row c of T|^2) delta_lm - (T^t T)_lm),
//   K[c][l][m] = k (2 f1 delta_lm + f2 ddI2[E] : E' + sum_ab f_ab a_a(c,l) a_b(c,m)),
// a(c,l) = (2 T_cl, dI2_cl, C_cl, delta_cl) for (I1, I2, tau, J).
// K[c] is symmetric; its unique entries go to K6[c][pr] in the pair order
// (0,0), (1,1), (0,1) (2D) or (0,0), (1,1), (2,2), (0,1), (0,2), (1,2) (3D).
template <int D> struct SymPairs;
template <> struct SymPairs<2> {
  static constexpr int N = 3;
  static constexpr int l[3] = {0, 1, 0}, m[3] = {0, 1, 1};
};
template <> struct SymPairs<3> {
  static constexpr int N = 6;
  static constexpr int l[6] = {0, 1, 2, 0, 0, 1}, m[6] = {0, 1, 2, 1, 2, 2};
};

template <int METRIC, typename R>
__device__ __forceinline__ void mu_second_rows(const R (&T)[MetricInfo<METRIC>::dim][MetricInfo<METRIC>::dim], R k,
                                               R (&K6)[MetricInfo<METRIC>::dim][SymPairs<MetricInfo<METRIC>::dim>::N]) {
  constexpr int D = MetricInfo<METRIC>::dim;
  using SP = SymPairs<D>;
  R C[D][D];
  cofactor<D, R>(T, C);
  R I1 = 0, tau = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) I1 += T[i][j] * T[i][j];
#pragma unroll
  for (int j = 0; j < D; ++j) tau += T[0][j] * C[0][j];
  if constexpr (!MetricInfo<METRIC>::i2) {
    R J = 0;
    if constexpr (MetricInfo<METRIC>::tr) {
#pragma unroll
      for (int i = 0; i < D; ++i) J += T[i][i];
    }
    const Partials<R> f = partials<METRIC, R>(I1, R(0), tau, J);
    const R kE = R(2) * k * f.f1, k1t = R(2) * k * f.f1t, ktt = k * f.ftt, kJt = k * f.fJt;
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int pr = 0; pr < SP::N; ++pr) {
        const int l = SP::l[pr], m = SP::m[pr];
        K6[c][pr] = (l == m ? kE : R(0)) + k1t * (T[c][l] * C[c][m] + C[c][l] * T[c][m]) + ktt * C[c][l] * C[c][m];
        // d J / dT_cl = delta_cl
        if constexpr (MetricInfo<METRIC>::tr)
          K6[c][pr] += kJt * ((c == l ? C[c][m] : R(0)) + (c == m ? C[c][l] : R(0)));
      }
  } else {
    R I2 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) I2 += C[i][j] * C[i][j];
    const Partials<R> f = partials<METRIC, R>(I1, I2, tau);
    R dI2[D][D], rowsq[D];
    dI2_of<D, R>(T, I1, dI2);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      R r = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) r += T[i][j] * T[i][j];
      rowsq[i] = r;
    }
    const R kE = R(2) * k * f.f1, k2 = R(2) * k * f.f2;
    const R k12 = R(2) * k * f.f12, k1t = R(2) * k * f.f1t, k2t = k * f.f2t, ktt = k * f.ftt;
#pragma unroll
    for (int pr = 0; pr < SP::N; ++pr) {
      const int l = SP::l[pr], m = SP::m[pr];
      R tlm = 0;                                   // (T^t T)_lm
#pragma unroll
      for (int q = 0; q < D; ++q) tlm += T[q][l] * T[q][m];
#pragma unroll
      for (int c = 0; c < D; ++c)
        K6[c][pr] = (l == m ? kE + k2 * (I1 - rowsq[c]) : R(0)) + k2 * (T[c][l] * T[c][m] - tlm) +
                    k12 * (T[c][l] * dI2[c][m] + dI2[c][l] * T[c][m]) +
                    k1t * (T[c][l] * C[c][m] + C[c][l] * T[c][m]) +
                    k2t * (dI2[c][l] * C[c][m] + C[c][l] * dI2[c][m]) + ktt * C[c][l] * C[c][m];
    }
  }
}

}  // namespace tmop
