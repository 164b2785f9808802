// Vector kernels of the Newton / truncated-CG driver and the deterministic
// reductions behind F, min det A and the CG dot products.  All are
// HBM-streaming kernels: grid-stride loops over contiguous FP64 vectors.
#include "tmop_internal.h"

namespace tmop {

namespace {

constexpr int VB = 256;   // threads per block for elementwise kernels

inline int vgrid(int64_t n) {
  int64_t g = (n + VB - 1) / VB;
  if (g > 8192) g = 8192;
  return (int)(g > 0 ? g : 1);
}

__global__ void __launch_bounds__(VB) k_fill(double* __restrict__ y, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] = v;
}

__global__ void __launch_bounds__(VB) k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] += a * x[i];
}

__global__ void __launch_bounds__(VB) k_xpay(const double* __restrict__ x, double a, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] = x[i] + a * y[i];
}

__global__ void __launch_bounds__(VB) k_waxpy(const double* __restrict__ x, double a, const double* __restrict__ d,
                                              double* __restrict__ w, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) w[i] = x[i] + a * d[i];
}

__global__ void __launch_bounds__(VB) k_scale_copy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] = a * x[i];
}

__global__ void __launch_bounds__(VB) k_mask_mul(const double* __restrict__ m, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] *= m[i];
}

__global__ void __launch_bounds__(VB) k_mul(const double* __restrict__ a, const double* __restrict__ x,
                                            double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) y[i] = a[i] * x[i];
}

// Jacobi preconditioner: d <- 1 / |d| on free DOFs (mask m = 1) with a
// nonzero diagonal, 1 elsewhere.
__global__ void __launch_bounds__(VB) k_jacobi_inv(const double* __restrict__ m, double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    const double a = fabs(d[i]);
    d[i] = (m[i] > 0.0 && a > 0.0) ? 1.0 / a : 1.0;
  }
}

__global__ void __launch_bounds__(VB) k_gather_rows(const double* __restrict__ src, const int32_t* __restrict__ rows,
                                                    int64_t n, int w, double* __restrict__ dst) {
  const int64_t total = n * w;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < total; i += (int64_t)gridDim.x * VB) {
    const int64_t j = i / w;
    dst[i] = src[(int64_t)rows[j] * w + (i - j * w)];
  }
}

// Fixed-order tree reduction of one value per thread in a RED_THREADS block.
__device__ __forceinline__ double block_sum(double s, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = s;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int w = 1; w < RED_THREADS / 64; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ double block_min(double s, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s = fmin(s, __shfl_xor(s, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = s;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int w = 1; w < RED_THREADS / 64; ++w) t = fmin(t, red[w]);
  return t;
}

// Stage 1 of a dot product: block b sums the chunk it owns, in order.
__global__ void __launch_bounds__(RED_THREADS) k_dot_part(const double* __restrict__ x, const double* __restrict__ y,
                                                          int64_t n, double* __restrict__ part) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS)
    s += x[i] * y[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One truncated-CG update, fused: d += a p; r -= a (m .* Hp) (m = nullptr:
// no fixed DOF); z = minv .* r (minv = nullptr: z is r); and the block
// partial sums of r . r into part[b] and, with minv, of r . z into
// part[RED_BLOCKS + b].  Same grid and summation order as k_dot_part.
__global__ void __launch_bounds__(RED_THREADS) k_cg_step(double a, const double* __restrict__ p,
                                                         const double* __restrict__ Hp, const double* __restrict__ m,
                                                         const double* __restrict__ minv, double* __restrict__ d,
                                                         double* __restrict__ r, double* __restrict__ z, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double red[2][RED_THREADS / 64];
  double srr = 0.0, srz = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    const double pi = p[i];
    const double hi = m ? Hp[i] * m[i] : Hp[i];
    d[i] += a * pi;
    const double ri = r[i] - a * hi;
    r[i] = ri;
    srr += ri * ri;
    if (minv) {
      const double zi = minv[i] * ri;
      z[i] = zi;
      srz += ri * zi;
    }
  }
  const double trr = block_sum(srr, red[0]);
  const double trz = block_sum(srz, red[1]);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = trr;
    part[RED_BLOCKS + blockIdx.x] = trz;
  }
}

// MINRES, fused: r_next = m .* Hv - a1 r_cur - a2 r_prev (r_prev = nullptr:
// no such term), written over Hv; y = minv .* r_next (minv = nullptr: y is
// r_next, not written); block partial sums of r_next . y into part[b].
__global__ void __launch_bounds__(RED_THREADS) k_minres_r(double* __restrict__ Hv, const double* __restrict__ m,
                                                          double a1, const double* __restrict__ r_cur, double a2,
                                                          const double* __restrict__ r_prev,
                                                          const double* __restrict__ minv, double* __restrict__ y,
                                                          int64_t n, double* __restrict__ part) {
  __shared__ double red[RED_THREADS / 64];
  double sum = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    double t = m ? Hv[i] * m[i] : Hv[i];
    t += a1 * r_cur[i];
    if (r_prev) t += a2 * r_prev[i];
    Hv[i] = t;
    if (minv) {
      const double yi = minv[i] * t;
      y[i] = yi;
      sum += t * yi;
    } else {
      sum += t * t;
    }
  }
  const double ts = block_sum(sum, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ts;
}

// MINRES, fused: w_prev <- (v - e w_prev - dl w_cur) sg (the new direction,
// in w_prev's storage); d += phi w_prev; and, when bnext > 0, the next
// Lanczos vector v <- y / bnext.
__global__ void __launch_bounds__(VB) k_minres_wd(double* __restrict__ v, double e, double* __restrict__ w_prev,
                                                  double dl, const double* __restrict__ w_cur, double sg, double phi,
                                                  double* __restrict__ d, const double* __restrict__ y, double rb,
                                                  int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    const double wn = (v[i] - e * w_prev[i] - dl * w_cur[i]) * sg;
    w_prev[i] = wn;
    d[i] += phi * wn;
    if (y) v[i] = rb * y[i];
  }
}

// Stage 2: one block folds n partial sums part[0, n) (and, optionally, n
// minima part[moff, moff + n)).
__global__ void __launch_bounds__(RED_THREADS) k_finalize(const double* __restrict__ part, int n, int moff,
                                                          int with_min, double* __restrict__ res) {
  __shared__ double red[2][RED_THREADS / 64];
  double s = 0.0, m = __builtin_huge_val();
  for (int i = threadIdx.x; i < n; i += RED_THREADS) {
    s += part[i];
    if (with_min) m = fmin(m, part[moff + i]);
  }
  const double ts = block_sum(s, red[0]);
  const double tm = block_min(m, red[1]);
  if (threadIdx.x == 0) {
    res[0] = ts;
    if (with_min) res[1] = tm;
  }
}

// Stage 1 of the energy fold: block b folds chunk b of the n sums part[0, n)
// and of the n minima part[moff, moff + n) into out[b] and out[FIN_BLOCKS + b].
__global__ void __launch_bounds__(RED_THREADS) k_fold_chunks(const double* __restrict__ part, int n, int moff,
                                                             int chunk, double* __restrict__ out) {
  __shared__ double red[2][RED_THREADS / 64];
  const int lo = blockIdx.x * chunk;
  const int hi = min(n, lo + chunk);
  double s = 0.0, m = __builtin_huge_val();
  for (int i = lo + threadIdx.x; i < hi; i += RED_THREADS) {
    s += part[i];
    m = fmin(m, part[moff + i]);
  }
  const double ts = block_sum(s, red[0]);
  const double tm = block_min(m, red[1]);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = ts;
    out[FIN_BLOCKS + blockIdx.x] = tm;
  }
}


// ------------------------------------------------------------------------
// Krylov solvers with device-resident scalars.  The scalar state of a CG or
// MINRES run lives in a small device array sc (layout SC_* in
// tmop_internal.h); one-block kernels update it between the vector kernels,
// which read their coefficients from it, so the host enqueues iterations
// without waiting and only reads sc back at check points.  An iteration
// runs while sc[SC_ACTIVE] is set: the first kernel of each iteration copies
// it to sc[SC_RUN], which every later kernel of the iteration tests; a run
// that ends clears SC_ACTIVE for the iterations still in the queue.

// Fixed-order fold of RED_BLOCKS partial sums by one block.
__device__ __forceinline__ double fold_parts(const double* __restrict__ part, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += RED_THREADS) s += part[i];
  return block_sum(s, red);
}

// Block partial sums of p . (m .* Hp + tau p) (p vanishes where m does).
__global__ void __launch_bounds__(RED_THREADS) k_dot_shift_part(const double* __restrict__ p,
                                                                const double* __restrict__ Hp, double tau, int64_t n,
                                                                const double* __restrict__ sc, double* __restrict__ part) {
  __shared__ double red[RED_THREADS / 64];
  if (sc[SC_ACTIVE] == 0.0) return;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    const double pi = p[i];
    s += pi * (Hp[i] + tau * pi);
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The CG scalars ride in the vector kernels that use them: every block
// folds the same partial sums in the same order, so every block takes the
// same decision and the same alpha or beta; block 0 alone writes the run
// state.  A value that the blocks of a kernel read is never written by that
// kernel: the new r . z goes to SC_RZP, which the next update commits to
// SC_RZ.

// CG update: pHp from the partials php_part (curvature test, alpha =
// rz / pHp), then d += alpha p; r -= alpha (m .* Hp + tau p); z = minv .* r
// and block partial sums of r . r (part[0, RED_BLOCKS)) and, with minv,
// r . z (part[RED_BLOCKS, 2 RED_BLOCKS)).  m: byte mask (1 = free DOF).
__global__ void __launch_bounds__(RED_THREADS) k_cg_update(const double* __restrict__ p, const double* __restrict__ Hp,
                                                           double tau, const uint8_t* __restrict__ m,
                                                           const double* __restrict__ minv, double* __restrict__ d,
                                                           double* __restrict__ r, double* __restrict__ z, int64_t n,
                                                           double* __restrict__ sc, const double* __restrict__ php_part,
                                                           double* __restrict__ part) {
  __shared__ double red[2][RED_THREADS / 64];
  if (sc[SC_ACTIVE] == 0.0) {   // ended earlier, or block 0 has just found non-positive curvature
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[SC_RUN] = 0.0;
    return;
  }
  const double pHp = fold_parts(php_part, red[0]);
  const double rz = sc[SC_RZP];
  const bool neg = !(pHp > 0.0);   // non-positive curvature (or NaN): the run ends here, d unchanged
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_ITERS] += 1.0;
    sc[SC_PHP] = pHp;
    sc[SC_RZ] = rz;
    sc[SC_RUN] = neg ? 0.0 : 1.0;
    if (neg) {
      sc[SC_NEG] = 1.0;
      sc[SC_ACTIVE] = 0.0;
    } else {
      sc[SC_ALPHA] = rz / pHp;
    }
  }
  if (neg) return;
  const double a = rz / pHp;
  double srr = 0.0, srz = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    const double pi = p[i];
    const double hi = (m && !m[i] ? 0.0 : Hp[i]) + tau * pi;
    d[i] += a * pi;
    const double ri = r[i] - a * hi;
    r[i] = ri;
    srr += ri * ri;
    if (minv) {
      const double zi = minv[i] * ri;
      z[i] = zi;
      srz += ri * zi;
    }
  }
  const double trr = block_sum(srr, red[0]);
  const double trz = block_sum(srz, red[1]);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = trr;
    part[RED_BLOCKS + blockIdx.x] = trz;
  }
}

// CG direction: r . r (and r . z) from the partials, the stopping test
// |r| <= tol_abs or the iteration cap, then beta = rz_new / rz and
// p = z + beta p.
__global__ void __launch_bounds__(RED_THREADS) k_cg_dir(const double* __restrict__ z, double* __restrict__ p, int64_t n,
                                                        const double* __restrict__ part, int precond, double tol_abs,
                                                        double* __restrict__ sc) {
  __shared__ double red[2][RED_THREADS / 64];
  if (sc[SC_RUN] == 0.0) return;   // ended, or block 0 has just stopped the run
  const double rr = fold_parts(part, red[0]);
  const double rz = precond ? fold_parts(part + RED_BLOCKS, red[1]) : rr;
  const bool stop = sqrt(rr) <= tol_abs || sc[SC_ITERS] >= sc[SC_MAXIT];
  const double b = rz / sc[SC_RZ];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_RR] = rr;
    if (stop) {
      sc[SC_RUN] = 0.0;
      sc[SC_ACTIVE] = 0.0;
    } else {
      sc[SC_BETA] = b;
      sc[SC_RZP] = rz;
    }
  }
  if (stop) return;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS)
    p[i] = z[i] + b * p[i];
}

// MINRES: alpha = v . Hv (iteration start: SC_ACTIVE -> SC_RUN).
__global__ void __launch_bounds__(RED_THREADS) k_mr_alpha(const double* __restrict__ part, double* __restrict__ sc) {
  __shared__ double red[RED_THREADS / 64];
  if (sc[SC_ACTIVE] == 0.0) {
    if (threadIdx.x == 0) sc[SC_RUN] = 0.0;
    return;
  }
  const double a = fold_parts(part, red);
  if (threadIdx.x == 0) {
    sc[SC_RUN] = 1.0;
    sc[SC_ITERS] += 1.0;
    sc[SC_ALPHA] = a;
  }
}

// MINRES: r_next = m .* Hv - (alpha / beta) r_cur - (beta / beta_prev) r_prev
// over Hv (first iteration: no r_prev term), y = minv .* r_next, partial sums
// of r_next . y.
__global__ void __launch_bounds__(RED_THREADS) k_mr_r(double* __restrict__ Hv, const double* __restrict__ m,
                                                      const double* __restrict__ r_cur,
                                                      const double* __restrict__ r_prev,
                                                      const double* __restrict__ minv, double* __restrict__ y,
                                                      int64_t n, const double* __restrict__ sc,
                                                      double* __restrict__ part) {
  __shared__ double red[RED_THREADS / 64];
  if (sc[SC_RUN] == 0.0) return;
  const double beta = sc[SC_BETA], bprev = sc[SC_BPREV];
  const double a1 = -sc[SC_ALPHA] / beta;
  const double a2 = bprev > 0.0 ? -beta / bprev : 0.0;
  double sum = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    double t = m ? Hv[i] * m[i] : Hv[i];
    t += a1 * r_cur[i];
    if (a2 != 0.0) t += a2 * r_prev[i];
    Hv[i] = t;
    if (minv) {
      const double yi = minv[i] * t;
      y[i] = yi;
      sum += t * yi;
    } else {
      sum += t * t;
    }
  }
  const double ts = block_sum(sum, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ts;
}

// MINRES scalars (Paige and Saunders): beta_{k+1}, the previous rotation on
// the new column, the rotation that annihilates beta_{k+1}, phi and phibar,
// the coefficients of the direction update, and the stopping test.
__global__ void __launch_bounds__(RED_THREADS) k_mr_rot(const double* __restrict__ part, double* __restrict__ sc) {
  __shared__ double red[RED_THREADS / 64];
  if (sc[SC_RUN] == 0.0) return;
  const double bn2 = fold_parts(part, red);
  if (threadIdx.x != 0) return;
  const double bnext = sqrt(fmax(bn2, 0.0));
  const double cs = sc[SC_CS], sn = sc[SC_SN], dbar = sc[SC_DBAR], alpha = sc[SC_ALPHA];
  const double eps_k = sc[SC_EPS];
  const double delta = cs * dbar + sn * alpha;
  const double gbar = sn * dbar - cs * alpha;
  sc[SC_EPS] = sn * bnext;
  sc[SC_DBAR] = -cs * bnext;
  double gamma = hypot(gbar, bnext);
  if (gamma == 0.0) gamma = 2.2250738585072014e-308;
  const double c2 = gbar / gamma, s2 = bnext / gamma;
  sc[SC_CS] = c2;
  sc[SC_SN] = s2;
  const double phibar = sc[SC_PHIBAR];
  sc[SC_PHI] = c2 * phibar;
  sc[SC_PHIBAR] = s2 * phibar;
  sc[SC_WE] = eps_k;
  sc[SC_WDL] = delta;
  sc[SC_WSG] = 1.0 / gamma;
  const bool last = fabs(s2 * phibar) <= sc[SC_TOL] * sc[SC_BETA1] || !(bnext > 0.0) || sc[SC_ITERS] >= sc[SC_MAXIT];
  sc[SC_RB] = last ? 0.0 : 1.0 / bnext;
  sc[SC_BPREV] = sc[SC_BETA];
  sc[SC_BETA] = bnext;
  if (last) sc[SC_ACTIVE] = 0.0;
}

// MINRES: w_prev <- (v - eps w_prev - delta w_cur) / gamma; d += phi w_prev;
// the next Lanczos vector v <- y / beta_{k+1} unless the run ends here.
__global__ void __launch_bounds__(VB) k_mr_wd(double* __restrict__ v, double* __restrict__ w_prev,
                                              const double* __restrict__ w_cur, double* __restrict__ d,
                                              const double* __restrict__ y, int64_t n, const double* __restrict__ sc) {
  if (sc[SC_RUN] == 0.0) return;
  const double e = sc[SC_WE], dl = sc[SC_WDL], sg = sc[SC_WSG], phi = sc[SC_PHI], rb = sc[SC_RB];
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    const double wn = (v[i] - e * w_prev[i] - dl * w_cur[i]) * sg;
    w_prev[i] = wn;
    d[i] += phi * wn;
    if (rb != 0.0) v[i] = rb * y[i];
  }
}

// Over the free DOFs (m > 0): partial sums of |d| and partial minima of d.
__global__ void __launch_bounds__(RED_THREADS) k_free_stats_part(const double* __restrict__ d,
                                                                 const double* __restrict__ m, int64_t n,
                                                                 double* __restrict__ part) {
  __shared__ double red[2][RED_THREADS / 64];
  double s = 0.0, mn = __builtin_huge_val();
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * RED_THREADS) {
    if (!m || m[i] > 0.0) {
      s += fabs(d[i]);
      mn = fmin(mn, d[i]);
    }
  }
  const double ts = block_sum(s, red[0]);
  const double tm = block_min(mn, red[1]);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ts;
    part[RED_BLOCKS + blockIdx.x] = tm;
  }
}

}  // namespace

hipError_t fill(double* y, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(vgrid(n)), dim3(VB), 0, s, y, v, n);
  return hipGetLastError();
}

hipError_t finalize_sum_min(const double* part, int n, int moff, double* scratch, double* res, hipStream_t s) {
  if (n <= 4 * RED_THREADS) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, part, n, moff, 1, res);
  } else {
    // stage 1: FIN_BLOCKS blocks fold contiguous chunks; stage 2 folds those
    const int chunk = (n + FIN_BLOCKS - 1) / FIN_BLOCKS;
    hipLaunchKernelGGL(k_fold_chunks, dim3(FIN_BLOCKS), dim3(RED_THREADS), 0, s, part, n, moff, chunk, scratch);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch, FIN_BLOCKS, FIN_BLOCKS, 1, res);
  }
  return hipGetLastError();
}

hipError_t dot(const double* x, const double* y, int64_t n, double* scratch, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_part, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, y, n, scratch);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch, RED_BLOCKS, 0, 0, res);
  return hipGetLastError();
}

hipError_t cg_step(double a, const double* p, const double* Hp, const double* m, const double* minv, double* d,
                   double* r, double* z, int64_t n, double* scratch, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_step, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, a, p, Hp, m, minv, d, r, z, n, scratch);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch, RED_BLOCKS, 0, 0, res);
  if (minv) hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch + RED_BLOCKS, RED_BLOCKS, 0, 0, res + 1);
  return hipGetLastError();
}

hipError_t minres_r(double* Hv, const double* m, double a1, const double* r_cur, double a2, const double* r_prev,
                    const double* minv, double* y, int64_t n, double* scratch, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_minres_r, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, Hv, m, a1, r_cur, a2, r_prev, minv, y, n,
                     scratch);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch, RED_BLOCKS, 0, 0, res);
  return hipGetLastError();
}

hipError_t minres_wd(double* v, double e, double* w_prev, double dl, const double* w_cur, double sg, double phi,
                     double* d, const double* y, double rb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_minres_wd, dim3(vgrid(n)), dim3(VB), 0, s, v, e, w_prev, dl, w_cur, sg, phi, d, y, rb, n);
  return hipGetLastError();
}

hipError_t mul(const double* a, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mul, dim3(vgrid(n)), dim3(VB), 0, s, a, x, y, n);
  return hipGetLastError();
}

hipError_t jacobi_inv(const double* m, double* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi_inv, dim3(vgrid(n)), dim3(VB), 0, s, m, d, n);
  return hipGetLastError();
}

hipError_t axpy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(vgrid(n)), dim3(VB), 0, s, a, x, y, n);
  return hipGetLastError();
}

hipError_t xpay(const double* x, double a, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_xpay, dim3(vgrid(n)), dim3(VB), 0, s, x, a, y, n);
  return hipGetLastError();
}

hipError_t waxpy(const double* x, double a, const double* d, double* w, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_waxpy, dim3(vgrid(n)), dim3(VB), 0, s, x, a, d, w, n);
  return hipGetLastError();
}

hipError_t scale_copy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(vgrid(n)), dim3(VB), 0, s, a, x, y, n);
  return hipGetLastError();
}

hipError_t gather_rows(const double* src, const int32_t* rows, int64_t n, int w, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3(vgrid(n * w)), dim3(VB), 0, s, src, rows, n, w, dst);
  return hipGetLastError();
}

namespace {
// Halo pass of the owner-computes tiles: each shared node's slots, one per
// touching tile, added in tile order.
__global__ void __launch_bounds__(VB) k_halo_sum(const TileParams tp, int64_t n_node, double* __restrict__ out) {
  const int64_t h = blockIdx.x * (int64_t)VB + threadIdx.x;
  if (h >= tp.n_halo) return;
  const int64_t g = tp.halo_node[h];
  const int j0 = tp.halo_off[h], j1 = tp.halo_off[h + 1];
  for (int c = 0; c < 2; ++c) {
    const double* hc = tp.halo + c * tp.n_slot;
    double sum = hc[j0];
    for (int j = j0 + 1; j < j1; ++j) sum += hc[j];
    out[c * n_node + g] = sum;
  }
}
}  // namespace

hipError_t halo_sum(const TileParams& tp, int64_t n_node, double* out, hipStream_t s) {
  if (tp.n_halo == 0) return hipSuccess;
  const int64_t g = (tp.n_halo + VB - 1) / VB;
  hipLaunchKernelGGL(k_halo_sum, dim3((unsigned)g), dim3(VB), 0, s, tp, n_node, out);
  return hipGetLastError();
}

namespace {
// Gather of the element-vector scatter: each node's entries, contiguous
// and in ascending element order, every component, summed in FP64 one by
// one in ascending order (so every variant below gives the same bits).
// Consecutive nodes read consecutive runs of entries.
//
// Per lane (FP64 entries, and the fallback of the staged form): the first
// RUN = 2^DIM entries of every component (a node of a structured quad or
// hex mesh has at most 2^DIM elements) are loaded before the first add, so
// a lane has DIM * RUN loads in flight instead of one. Slots past the
// node's run load an entry clamped to the last one (in bounds: a context
// always has elements) and add +0.0, which leaves the sum unchanged bit for
// bit (a sum that starts at +0.0 is never -0.0); longer runs (nodes of
// higher valence) finish in a plain loop.
template <typename E, int DIM>
__device__ __forceinline__ void gather_node(const E* __restrict__ evec, int k0, int n, int64_t n_ent, int64_t n_node,
                                            int64_t I, double* __restrict__ out) {
  constexpr int RUN = 1 << DIM;
  E v[DIM][RUN];
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < RUN; ++k) v[c][k] = evec[c * n_ent + min((int64_t)k0 + k, n_ent - 1)];
  // Every loaded value counts as used here, so the compiler cannot move a
  // load into the branch of its k < n test, behind the other loads' wait.
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < RUN; ++k) asm volatile("" : "+v"(v[c][k]));
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    double sum = 0.0 + (double)v[c][0];
#pragma unroll
    for (int k = 1; k < RUN; ++k) sum += k < n ? (double)v[c][k] : 0.0;
    for (int k = RUN; k < n; ++k) sum += (double)evec[c * n_ent + k0 + k];
    out[c * n_node + I] = n > 0 ? sum : 0.0;  // a node no element uses sums nothing
  }
}

// FP32 entries are staged: the block's VB nodes own one contiguous range of
// entries, which the block reads with coalesced loads into LDS (up to 2^DIM
// entries per node, 24 KB for hex meshes), and each lane then sums its run
// from there. Timed on 64^3 Q2 and 512^2 Q2 node runs, staging is the
// faster form for 4-byte entries (23.9 against 30.7 us per lane-wise call
// at 64^3) and the lane-wise form for 8-byte ones (35.2 against 36.5 us,
// where the staging buffer would be twice as large).
template <typename E, int DIM>
__global__ void __launch_bounds__(VB) k_evec_gather(const E* __restrict__ evec, const int32_t* __restrict__ off,
                                                    int64_t n_node, int64_t n_ent, double* __restrict__ out) {
  const int64_t I0 = blockIdx.x * (int64_t)VB;
  const int64_t I = I0 + threadIdx.x;
  if constexpr (sizeof(E) == 4) {
    constexpr int CAP = VB << DIM;   // entries per component the block stages
    constexpr int J = CAP / VB;
    __shared__ E lds[DIM][CAP];
    const int b0 = off[I0];
    const int len = off[min(I0 + VB, n_node)] - b0;
    if (len <= CAP) {                // block-uniform
      E t[DIM][J];
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const int e = threadIdx.x + j * VB;
          t[c][j] = e < len ? evec[c * n_ent + b0 + e] : E(0);
        }
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int c = 0; c < DIM; ++c) lds[c][threadIdx.x + j * VB] = t[c][j];
      __syncthreads();
      if (I < n_node) {
        const int k0 = off[I] - b0, k1 = off[I + 1] - b0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          double sum = 0.0;
          for (int k = k0; k < k1; ++k) sum += (double)lds[c][k];
          out[c * n_node + I] = sum;
        }
      }
      return;
    }
  }
  if (I >= n_node) return;
  const int k0 = off[I];
  gather_node<E, DIM>(evec, k0, off[I + 1] - k0, n_ent, n_node, I, out);
}

template <typename E>
hipError_t evec_gather_t(const E* evec, const int32_t* off, int64_t n_node, int64_t n_ent, int dim, double* out,
                         hipStream_t s) {
  const dim3 g((unsigned)((n_node + VB - 1) / VB));
  if (dim == 3)
    hipLaunchKernelGGL((k_evec_gather<E, 3>), g, dim3(VB), 0, s, evec, off, n_node, n_ent, out);
  else if (dim == 2)
    hipLaunchKernelGGL((k_evec_gather<E, 2>), g, dim3(VB), 0, s, evec, off, n_node, n_ent, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
}  // namespace

hipError_t evec_gather(const void* evec, int esize, const int32_t* off, int64_t n_node, int64_t n_ent, int dim,
                       double* out, hipStream_t s) {
  if (n_node == 0) return hipSuccess;
  if (n_ent < 1) return hipErrorInvalidValue;  // a context always has elements
  if (esize == 4) return evec_gather_t(static_cast<const float*>(evec), off, n_node, n_ent, dim, out, s);
  if (esize == 8) return evec_gather_t(static_cast<const double*>(evec), off, n_node, n_ent, dim, out, s);
  return hipErrorInvalidValue;
}

hipError_t mask_mul(const double* m, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_mul, dim3(vgrid(n)), dim3(VB), 0, s, m, y, n);
  return hipGetLastError();
}

hipError_t cg_dev_curvature(const double* p, const double* Hp, double tau, int64_t n, double* scratch, double* sc,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_dot_shift_part, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, p, Hp, tau, n, sc,
                     scratch + 2 * RED_BLOCKS);
  return hipGetLastError();
}

hipError_t cg_dev_update(const double* p, const double* Hp, double tau, const uint8_t* m, const double* minv, double* d,
                         double* r, double* z, int64_t n, double tol_abs, double* scratch, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, p, Hp, tau, m, minv, d, r, z, n, sc,
                     scratch + 2 * RED_BLOCKS, scratch);
  hipLaunchKernelGGL(k_cg_dir, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, minv ? z : r, (double*)p, n, scratch,
                     minv ? 1 : 0, tol_abs, sc);
  return hipGetLastError();
}

hipError_t mr_dev_alpha(const double* v, const double* Hv, int64_t n, double* scratch, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_shift_part, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, v, Hv, 0.0, n, sc, scratch);
  hipLaunchKernelGGL(k_mr_alpha, dim3(1), dim3(RED_THREADS), 0, s, scratch, sc);
  return hipGetLastError();
}

hipError_t mr_dev_step(double* Hv, const double* m, const double* r_cur, const double* r_prev, const double* minv,
                       double* y, double* v, double* w_prev, const double* w_cur, double* d, int64_t n,
                       double* scratch, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_mr_r, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, Hv, m, r_cur, r_prev, minv, y, n, sc, scratch);
  hipLaunchKernelGGL(k_mr_rot, dim3(1), dim3(RED_THREADS), 0, s, scratch, sc);
  hipLaunchKernelGGL(k_mr_wd, dim3(vgrid(n)), dim3(VB), 0, s, v, w_prev, w_cur, d, minv ? y : Hv, n, sc);
  return hipGetLastError();
}

hipError_t free_stats(const double* d, const double* m, int64_t n, double* scratch, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_free_stats_part, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, d, m, n, scratch);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_THREADS), 0, s, scratch, RED_BLOCKS, RED_BLOCKS, 1, res);
  return hipGetLastError();
}

}  // namespace tmop
