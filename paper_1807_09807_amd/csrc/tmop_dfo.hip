// Derivative-free solver of Section 3.4 (eq. 3.3, variational form): each
// node moves to the position that minimizes its patch quality
//   Q(x_i) = sum over the elements E holding node i of sum_q w_q det W mu(A W^{-1}),
// found by Nelder-Mead over the node's free components.  The sweeps run
// colour by colour: nodes of one colour share no element, so their patches
// are disjoint and one launch moves all of them at once; the result equals
// visiting them one after the other.
//
// One workgroup per node.  Its lanes own the patch's quadrature points
// (up to 2^d elements times Q^d points, PPL points per lane) and keep, per
// point, A at the node's current position, the node's basis gradient
// grad w_a(s_q) and the weight w_q det W.  A trial position y changes A by
// the rank-one term (y - x_i) grad w_a^T, so one evaluation of Q is d^2
// FMAs, det A, mu and a block reduction per point.  Every lane runs the
// same Nelder-Mead iteration on the reduced (uniform) values, so control
// flow stays uniform across the workgroup.
//
// Nelder-Mead as stated by Lagarias, Reeds, Wright and Wright (SIAM J.
// Optim. 9, 1998): reflection 1, expansion 2, contraction 1/2, shrink 1/2;
// initial simplex x_i, x_i + s e_k; stop when every vertex lies within xtol
// of the best (max norm) or after max_evals evaluations.  Q = +inf when
// det A <= 0 at a patch point.
#include "tmop_elem.h"

namespace tmop {

template <int D> struct DfoCfg {
  static constexpr int BLOCK = D == 2 ? 64 : 256;
};

template <int P, int Q>
struct DfoArgs {
  double* __restrict__ x;                  // [dim][n_node]; this colour's nodes are updated in place
  const double* __restrict__ mask;         // [dim][n_node], 1 = free component
  const int32_t* __restrict__ nodes;       // this colour's nodes [n_list]
  const int32_t* __restrict__ ne_off;      // node -> (element, local node) CSR offsets [n_node + 1]
  const int32_t* __restrict__ ne;          // element * P^dim + local node index
  const int32_t* __restrict__ elem_node;   // [n_elem][P^dim]
  double* __restrict__ move;               // [n_list]: minus the max-norm move of each node
  int64_t n_node;
  int32_t n_list;
  int32_t max_evals;
  double B[Q][P];
  double G[Q][P];
  double w[Q];
  double Winv[3][3];
  double detW;
  double step, xtol;
};

// Sum and min over the workgroup, returned to every lane (fixed order).
template <int BLOCK>
__device__ __forceinline__ void reduce_bcast(double& s, double& m, double* red) {
  constexpr int NW = BLOCK / 64;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    m = fmin(m, __shfl_xor(m, off, 64));
  }
  if constexpr (NW > 1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { red[wave] = s; red[NW + wave] = m; }
    __syncthreads();
    s = red[0];
    m = red[NW];
#pragma unroll
    for (int k = 1; k < NW; ++k) { s += red[k]; m = fmin(m, red[NW + k]); }
    __syncthreads();   // red is reused by the next reduction
  }
}

template <int D, int P, int Q, int METRIC>
__global__ void __launch_bounds__(DfoCfg<D>::BLOCK) dfo_kernel(const DfoArgs<P, Q> a) {
  constexpr int BLOCK = DfoCfg<D>::BLOCK;
  constexpr int NQ = D == 2 ? Q * Q : Q * Q * Q;
  constexpr int NPE = D == 2 ? P * P : P * P * P;
  constexpr int PPL = ((1 << D) * NQ + BLOCK - 1) / BLOCK;   // patch points per lane
  __shared__ double red[2 * (BLOCK / 64)];

  const int k = blockIdx.x;
  const int node = a.nodes[k];
  const int tid = threadIdx.x;
  // the free components (uniform)
  bool fr[D];
  int n = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    fr[c] = a.mask[c * a.n_node + node] > 0.5;
    n += fr[c] ? 1 : 0;
  }
  if (n == 0) {
    if (tid == 0) a.move[k] = -0.0;
    return;
  }
  double xi[D];
#pragma unroll
  for (int c = 0; c < D; ++c) xi[c] = a.x[c * a.n_node + node];
  const int off0 = a.ne_off[node];
  const int np = a.ne_off[node + 1] - off0;

  // per owned point: A at the current position, grad w_a and the weight
  double Ab[PPL][D][D], g[PPL][D], wq[PPL];
#pragma unroll
  for (int r = 0; r < PPL; ++r) {
    const int j = tid + r * BLOCK;
    const int pe = j / NQ, q = j - pe * NQ;
    wq[r] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      g[r][c] = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) Ab[r][c][l] = (c == l) ? 1.0 : 0.0;   // harmless filler (weight 0)
    }
    if (pe >= np) continue;
    const int code = a.ne[off0 + pe];
    const int e = code / NPE, la = code - e * NPE;
    const int32_t* en = a.elem_node + (int64_t)e * NPE;
    const int q0 = q % Q, q1 = (q / Q) % Q, q2 = D == 3 ? q / (Q * Q) : 0;
    wq[r] = a.w[q0] * a.w[q1] * (D == 3 ? a.w[q2] : 1.0) * a.detW;
    double org[D];
#pragma unroll
    for (int c = 0; c < D; ++c) org[c] = a.x[c * a.n_node + en[0]];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int l = 0; l < D; ++l) Ab[r][c][l] = 0.0;
    for (int b = 0; b < NPE; ++b) {
      const int b0 = b % P, b1 = (b / P) % P, b2 = D == 3 ? b / (P * P) : 0;
      double gw[D];
      if constexpr (D == 2) {
        gw[0] = a.G[q0][b0] * a.B[q1][b1];
        gw[1] = a.B[q0][b0] * a.G[q1][b1];
      } else {
        gw[0] = a.G[q0][b0] * a.B[q1][b1] * a.B[q2][b2];
        gw[1] = a.B[q0][b0] * a.G[q1][b1] * a.B[q2][b2];
        gw[2] = a.B[q0][b0] * a.B[q1][b1] * a.G[q2][b2];
      }
      const int nb = en[b];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double xb = a.x[c * a.n_node + nb] - org[c];
#pragma unroll
        for (int l = 0; l < D; ++l) Ab[r][c][l] += xb * gw[l];
      }
      if (b == la) {
#pragma unroll
        for (int l = 0; l < D; ++l) g[r][l] = gw[l];
      }
    }
  }

  // Q at the trial position y, the same on every lane.  The simplex
  // vertices are full d-vectors whose fixed components stay at x_i: every
  // simplex operation works component by component, and with at most two
  // free components the centroid of equal values is exact, so a fixed
  // component never moves and contributes nothing to the size test.
  auto quality = [&](const double (&y)[D]) -> double {
    double dy[D];
#pragma unroll
    for (int c = 0; c < D; ++c) dy[c] = y[c] - xi[c];
    double s = 0.0, m = __builtin_huge_val();
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
      if (wq[r] == 0.0) continue;
      double A[D][D], T[D][D];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int l = 0; l < D; ++l) A[c][l] = Ab[r][c][l] + dy[c] * g[r][l];
      m = fmin(m, det<D, double>(A));
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int l = 0; l < D; ++l) {
          double t = 0.0;
#pragma unroll
          for (int kk = 0; kk < D; ++kk) t += A[c][kk] * a.Winv[kk][l];
          T[c][l] = t;
        }
      s += wq[r] * mu_value<METRIC, double>(T, det<D, double>(T));
    }
    reduce_bcast<BLOCK>(s, m, red);
    return m > 0.0 ? s : __builtin_huge_val();
  };

  // Nelder-Mead over the n free components: vertices 0..n of V (static
  // indices with guards, so the state stays in registers)
  double V[D + 1][D], fv[D + 1];
#pragma unroll
  for (int v = 0; v <= D; ++v) {
#pragma unroll
    for (int c = 0; c < D; ++c) V[v][c] = xi[c];
    fv[v] = __builtin_huge_val();
  }
  {   // vertex t + 1 moves the t-th free component by the step
    int t = 0;
#pragma unroll
    for (int c = 0; c < D; ++c)
      if (fr[c]) {
        ++t;
#pragma unroll
        for (int v = 1; v <= D; ++v)
          if (v == t) V[v][c] += a.step;
      }
  }
#pragma unroll
  for (int v = 0; v <= D; ++v)
    if (v <= n) fv[v] = quality(V[v]);
  int evals = n + 1;
  while (true) {
    // stable sort of vertices 0..n by value (bubble passes: swap only on <)
#pragma unroll
    for (int pass = 0; pass < D; ++pass)
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j + 1 <= n && fv[j + 1] < fv[j]) {
          const double tf = fv[j]; fv[j] = fv[j + 1]; fv[j + 1] = tf;
#pragma unroll
          for (int c = 0; c < D; ++c) { const double tv = V[j][c]; V[j][c] = V[j + 1][c]; V[j + 1][c] = tv; }
        }
    double size = 0.0;
#pragma unroll
    for (int v = 1; v <= D; ++v)
      if (v <= n)
#pragma unroll
        for (int c = 0; c < D; ++c) size = fmax(size, fabs(V[v][c] - V[0][c]));
    if (size <= a.xtol || evals >= a.max_evals) break;
    // the worst vertex, its value and the second worst value
    double Vw[D], fw = fv[0], fw2 = fv[0];
#pragma unroll
    for (int c = 0; c < D; ++c) Vw[c] = V[0][c];
#pragma unroll
    for (int v = 1; v <= D; ++v) {
      if (v == n) {
        fw = fv[v];
#pragma unroll
        for (int c = 0; c < D; ++c) Vw[c] = V[v][c];
      }
      if (v == n - 1) fw2 = fv[v];
    }
    double xb[D], xr[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double sum = V[0][c];
#pragma unroll
      for (int v = 1; v < D; ++v)
        if (v < n) sum += V[v][c];
      xb[c] = sum / n;
      xr[c] = xb[c] + (xb[c] - Vw[c]);
    }
    double fnew, Vnew[D];
    bool replace = true;
    const double frv = quality(xr);
    ++evals;
    if (fv[0] <= frv && frv < fw2) {
      fnew = frv;
#pragma unroll
      for (int c = 0; c < D; ++c) Vnew[c] = xr[c];
    } else if (frv < fv[0]) {   // expansion
      double xe[D];
#pragma unroll
      for (int c = 0; c < D; ++c) xe[c] = xb[c] + 2.0 * (xr[c] - xb[c]);
      const double fe = quality(xe);
      ++evals;
      const bool take_e = fe < frv;
      fnew = take_e ? fe : frv;
#pragma unroll
      for (int c = 0; c < D; ++c) Vnew[c] = take_e ? xe[c] : xr[c];
    } else {                    // contraction, outside or inside
      const bool outside = frv < fw;
      double xc[D];
#pragma unroll
      for (int c = 0; c < D; ++c) xc[c] = outside ? xb[c] + 0.5 * (xr[c] - xb[c]) : xb[c] + 0.5 * (Vw[c] - xb[c]);
      const double fc = quality(xc);
      ++evals;
      replace = outside ? fc <= frv : fc < fw;
      fnew = fc;
#pragma unroll
      for (int c = 0; c < D; ++c) Vnew[c] = xc[c];
    }
    if (replace) {
#pragma unroll
      for (int v = 1; v <= D; ++v)
        if (v == n) {
          fv[v] = fnew;
#pragma unroll
          for (int c = 0; c < D; ++c) V[v][c] = Vnew[c];
        }
      continue;
    }
#pragma unroll
    for (int v = 1; v <= D; ++v)   // shrink towards the best vertex
      if (v <= n) {
#pragma unroll
        for (int c = 0; c < D; ++c) V[v][c] = V[0][c] + 0.5 * (V[v][c] - V[0][c]);
        fv[v] = quality(V[v]);
      }
    evals += n;
  }
  if (tid == 0) {
    double mv = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c)
      if (fr[c]) {
        mv = fmax(mv, fabs(V[0][c] - xi[c]));
        a.x[c * a.n_node + node] = V[0][c];
      }
    a.move[k] = -mv;
  }
}

template <int D, int P, int Q, int METRIC>
static int dfo_one(const DfoParams& dp, hipStream_t s) {
  DfoArgs<P, Q> a;
  a.x = dp.x; a.mask = dp.mask; a.nodes = dp.nodes; a.ne_off = dp.ne_off; a.ne = dp.ne;
  a.elem_node = dp.elem_node; a.move = dp.move; a.n_node = dp.n_node; a.n_list = dp.n_list;
  a.max_evals = dp.max_evals;
  for (int q = 0; q < Q; ++q) {
    a.w[q] = dp.w[q];
    for (int i = 0; i < P; ++i) { a.B[q][i] = dp.B[q][i]; a.G[q][i] = dp.G[q][i]; }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.Winv[i][j] = dp.Winv[i][j];
  a.detW = dp.detW;
  a.step = dp.step;
  a.xtol = dp.xtol;
  if (dp.n_list == 0) return 0;
  hipLaunchKernelGGL((dfo_kernel<D, P, Q, METRIC>), dim3(dp.n_list), dim3(DfoCfg<D>::BLOCK), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <int D, int P, int Q>
static int dfo_metric(int metric, const DfoParams& dp, hipStream_t s) {
  if constexpr (D == 2) {
    switch (metric) {
      case 1: return dfo_one<2, P, Q, 1>(dp, s);
      case 2: return dfo_one<2, P, Q, 2>(dp, s);
      case 7: return dfo_one<2, P, Q, 7>(dp, s);
      case 9: return dfo_one<2, P, Q, 9>(dp, s);
      case 14: return dfo_one<2, P, Q, 14>(dp, s);
      case 77: return dfo_one<2, P, Q, 77>(dp, s);
      case 98: return dfo_one<2, P, Q, 98>(dp, s);
      default: return -1;
    }
  } else {
    switch (metric) {
      case 302: return dfo_one<3, P, Q, 302>(dp, s);
      case 303: return dfo_one<3, P, Q, 303>(dp, s);
      case MU7_3D: return dfo_one<3, P, Q, MU7_3D>(dp, s);
      default: return -1;
    }
  }
}

template <int D>
static int dfo_dispatch(int p, int Q, int metric, const DfoParams& dp, hipStream_t s) {
  const int P = p + 1;
#define TMOP_DFO_PQ(P_, Q_) \
  if (P == P_ && Q == Q_) return dfo_metric<D, P_, Q_>(metric, dp, s);
  TMOP_DFO_PQ(2, 2) TMOP_DFO_PQ(2, 3)
  TMOP_DFO_PQ(3, 3) TMOP_DFO_PQ(3, 4)
  TMOP_DFO_PQ(4, 4) TMOP_DFO_PQ(4, 5)
  TMOP_DFO_PQ(5, 5) TMOP_DFO_PQ(5, 6)
#undef TMOP_DFO_PQ
  return -1;
}

int dfo_patch_capacity(int dim, int Q) {
  const int block = dim == 2 ? DfoCfg<2>::BLOCK : DfoCfg<3>::BLOCK;
  const int nq = dim == 2 ? Q * Q : Q * Q * Q;
  const int ppl = ((1 << dim) * nq + block - 1) / block;   // as PPL in dfo_kernel
  return ppl * block / nq;
}

int launch_dfo(int dim, int p, int Q, int metric, const DfoParams& dp, hipStream_t s) {
  return dim == 3 ? dfo_dispatch<3>(p, Q, metric, dp, s) : dfo_dispatch<2>(p, Q, metric, dp, s);
}

}  // namespace tmop
