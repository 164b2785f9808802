// Learned initial guess for Newton: a per-element MLP that maps the 9 nodes
// of a Q2 quadrilateral (relative to the centroid, in units of the target
// size h) to a displacement of those nodes, trained on the method's own
// Newton solutions, plus the gather / merge kernels around it.
//
//   network   18 -> 64 -> 64 -> 64 -> 18, GELU(z) = z Phi(z) on the hidden
//             layers; weights take BF16 values, biases FP32
//   layers    FP32 matrix cores (v_mfma_f32_16x16x4f32): 16 samples per
//             wave, the BF16 weights widened exactly to FP32, FP32
//             accumulation; activations stay FP32
//   training  MSE loss, backward by the transposed products, weight
//             gradients summed per block and folded in a fixed order,
//             Adam on FP32 master weights (BF16 copy refreshed each step)
//   proposal  features -> MLP -> average of the element displacements at
//             shared nodes (colour launches, no atomics) -> fixed DOFs kept
//
// Everything is deterministic.  Parameter layout (flat, FP32 master):
// W1[18][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][18] b4[18].
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "tmop.h"
#include "tmop_internal.h"

namespace {

constexpr int NP = TMOP_MLP_NPARAMS;
constexpr int OW1 = 0, OB1 = 1152, OW2 = 1216, OB2 = 5312, OW3 = 5376, OB3 = 9472, OW4 = 9536, OB4 = 10688;
constexpr int NF = 18;            // features and outputs per element
constexpr int NH = 64;            // hidden width
constexpr int LDH = 65;           // LDS row stride of a 16 x 64 activation tile

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f2bf16(float f) {      // round to nearest, ties to even
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// acc[t] (16 x 16 tile t of a 16 x N product) += H (16 x K, LDS, stride LDH)
// times M, where M[k][n] = Wb[k * ldw + n] (TRANS = false) or Wb[n * ldw + k]
// (TRANS = true), zero outside k < Kr, n < Nr.  Lane l holds acc[t][r] =
// out[4 (l / 16) + r][16 t + l % 16].
template <int K, int NT, bool TRANS>
__device__ __forceinline__ void mm_tile(const float* Hl, const uint16_t* __restrict__ Wb, int ldw, int Kr, int Nr,
                                        f4 (&acc)[NT]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int kk = k0 + (l >> 4);
    const float a = kk < Kr ? Hl[(l & 15) * LDH + kk] : 0.0f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int nn = 16 * t + (l & 15);
      float b = 0.0f;
      if (kk < Kr && nn < Nr) b = bf16f(TRANS ? Wb[nn * ldw + kk] : Wb[kk * ldw + nn]);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
}

// Write an accumulator tile set to the LDS tile (rows = samples).
template <int NT>
__device__ __forceinline__ void store_tile(float* Hl, const f4 (&v)[NT], int Nr) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = 16 * t + (l & 15);
    if (n < Nr) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Hl[(4 * (l >> 4) + r) * LDH + n] = v[t][r];
    }
  }
}

// Forward over 16-sample tiles, one wave per block, grid-stride.  Saves the
// pre-activations Z and activations H of the hidden layers when asked.
__global__ void __launch_bounds__(64) k_mlp_fwd(const uint16_t* __restrict__ Wb, const float* __restrict__ P,
                                                const float* __restrict__ X, int64_t n, float* __restrict__ Y,
                                                float* __restrict__ Zs, float* __restrict__ Hs) {
  __shared__ float Hl[16 * LDH];
  const int l = threadIdx.x;
  const int64_t ntile = (n + 15) / 16;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * 16;
    // features into the tile (18 columns)
    for (int i = l; i < 16 * NF; i += 64) {
      const int r = i / NF, c = i % NF;
      Hl[r * LDH + c] = s0 + r < n ? X[(s0 + r) * NF + c] : 0.0f;
    }
    __syncthreads();
    const int wo[3] = {OW1, OW2, OW3}, bo[3] = {OB1, OB2, OB3};
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      f4 acc[4];
      if (layer == 0) mm_tile<20, 4, false>(Hl, Wb + wo[0], NH, NF, NH, acc);
      else mm_tile<64, 4, false>(Hl, Wb + wo[layer], NH, NH, NH, acc);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int nn = 16 * t + (l & 15);
        const float bias = P[bo[layer] + nn];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t s = s0 + 4 * (l >> 4) + r;
          const float z = acc[t][r] + bias;
          const float h = gelu(z);
          if (Zs && s < n) {
            Zs[((int64_t)layer * n + s) * NH + nn] = z;
            Hs[((int64_t)layer * n + s) * NH + nn] = h;
          }
          acc[t][r] = h;
        }
      }
      store_tile<4>(Hl, acc, NH);
      __syncthreads();
    }
    f4 out[2];
    mm_tile<64, 2, false>(Hl, Wb + OW4, NF, NH, NF, out);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int nn = 16 * t + (l & 15);
      if (nn < NF) {
        const float bias = P[OB4 + nn];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t s = s0 + 4 * (l >> 4) + r;
          if (s < n) Y[s * NF + nn] = out[t][r] + bias;
        }
      }
    }
    __syncthreads();
  }
}

// Backward through the data path: dZ of the hidden layers (and dX).
__global__ void __launch_bounds__(64) k_mlp_bwd_data(const uint16_t* __restrict__ Wb, const float* __restrict__ Zs,
                                                     const float* __restrict__ dY, int64_t n, float* __restrict__ dZ,
                                                     float* __restrict__ dX) {
  __shared__ float Dl[16 * LDH];
  const int l = threadIdx.x;
  const int64_t ntile = (n + 15) / 16;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t s0 = tile * 16;
    for (int i = l; i < 16 * NF; i += 64) {
      const int r = i / NF, c = i % NF;
      Dl[r * LDH + c] = s0 + r < n ? dY[(s0 + r) * NF + c] : 0.0f;
    }
    __syncthreads();
    // dH3 = dY W4^T (K = 18), then down through W3, W2
    const int wo[3] = {OW4, OW3, OW2};
#pragma unroll
    for (int step = 0; step < 3; ++step) {
      const int layer = 2 - step;                 // hidden layer whose dZ is formed
      f4 acc[4];
      if (step == 0) mm_tile<20, 4, true>(Dl, Wb + wo[0], NF, NF, NH, acc);
      else mm_tile<64, 4, true>(Dl, Wb + wo[step], NH, NH, NH, acc);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int nn = 16 * t + (l & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t s = s0 + 4 * (l >> 4) + r;
          float d = 0.0f;
          if (s < n) {
            d = acc[t][r] * gelu_d(Zs[((int64_t)layer * n + s) * NH + nn]);
            dZ[((int64_t)layer * n + s) * NH + nn] = d;
          }
          acc[t][r] = d;
        }
      }
      store_tile<4>(Dl, acc, NH);
      __syncthreads();
    }
    if (dX) {   // dX = dZ1 W1^T (N = 18)
      f4 acc[2];
      mm_tile<64, 2, true>(Dl, Wb + OW1, NH, NH, NF, acc);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int nn = 16 * t + (l & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t s = s0 + 4 * (l >> 4) + r;
          if (nn < NF && s < n) dX[s * NF + nn] = acc[t][r];
        }
      }
    }
    __syncthreads();
  }
}

// Weight gradients of one chunk of samples: dW = A^T dZ per layer, as
// 16 x 16 tiles over (input feature, output feature), contracted over the
// chunk's samples 4 at a time; db = column sums.  4 waves share the 48 tiles.
// Writes one partial gradient (NP values) per block.
__global__ void __launch_bounds__(256) k_mlp_bwd_weights(const float* __restrict__ X, const float* __restrict__ Hs,
                                                         const float* __restrict__ dZ, const float* __restrict__ dY,
                                                         int64_t n, int chunk, float* __restrict__ part) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = std::min<int64_t>(n, lo + chunk);
  float* out = part + (int64_t)blockIdx.x * NP;
  // tiles: layer 0: 2 x 4 (A = X, 18 rows), layers 1-2: 4 x 4, layer 3: 4 x 2 (18 columns)
  for (int tile = w; tile < 48; tile += 4) {
    int layer, mt, nt;
    if (tile < 8) { layer = 0; mt = tile / 4; nt = tile % 4; }
    else if (tile < 24) { layer = 1; mt = (tile - 8) / 4; nt = (tile - 8) % 4; }
    else if (tile < 40) { layer = 2; mt = (tile - 24) / 4; nt = (tile - 24) % 4; }
    else { layer = 3; mt = (tile - 40) / 2; nt = (tile - 40) % 2; }
    const int Kr = layer == 0 ? NF : NH;          // rows of dW (input features)
    const int Nr = layer == 3 ? NF : NH;          // columns of dW (output features)
    const int m = 16 * mt + (l & 15);
    const int nn = 16 * nt + (l & 15);
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t s0 = lo; s0 < hi; s0 += 4) {
      const int64_t s = s0 + (l >> 4);
      float a = 0.0f, b = 0.0f;
      if (s < hi) {
        if (m < Kr) a = layer == 0 ? X[s * NF + m] : Hs[((int64_t)(layer - 1) * n + s) * NH + m];
        if (nn < Nr) b = layer == 3 ? dY[s * NF + nn] : dZ[((int64_t)layer * n + s) * NH + nn];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    const int wofs = layer == 0 ? OW1 : layer == 1 ? OW2 : layer == 2 ? OW3 : OW4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * mt + 4 * (l >> 4) + r;
      if (row < Kr && nn < Nr) out[wofs + row * Nr + nn] = acc[r];
    }
  }
  // bias gradients: column sums in sample order
  for (int j = threadIdx.x; j < 3 * NH + NF; j += 256) {
    float s = 0.0f;
    if (j < 3 * NH) {
      const int layer = j / NH, c = j % NH;
      for (int64_t i = lo; i < hi; ++i) s += dZ[((int64_t)layer * n + i) * NH + c];
      out[(layer == 0 ? OB1 : layer == 1 ? OB2 : OB3) + c] = s;
    } else {
      const int c = j - 3 * NH;
      for (int64_t i = lo; i < hi; ++i) s += dY[i * NF + c];
      out[OB4 + c] = s;
    }
  }
}

__global__ void __launch_bounds__(256) k_fold_partials(const float* __restrict__ part, int nb, float* __restrict__ g) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NP) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * NP + p];
  g[p] = s;
}

// dY = 2 (Y - L) / (n 18); per-block sums of (Y - L)^2 in a fixed order.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ L, int64_t m,
                                             float scale, float* __restrict__ dY, double* __restrict__ lpart) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const float d = Y[i] - L[i];
    dY[i] = scale * d;
    acc += (double)d * d;
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(64) k_fold_loss(const double* __restrict__ lpart, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += lpart[b];
    *out = s;
  }
}

// Adam (Kingma & Ba) with bias correction on the FP32 master weights; the
// BF16 copy is refreshed from the updated master.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ P, float* __restrict__ m1, float* __restrict__ m2,
                                              const float* __restrict__ g, uint16_t* __restrict__ Wb, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NP) return;
  const float gi = g[p];
  const float a = b1 * m1[p] + (1.0f - b1) * gi;
  const float b = b2 * m2[p] + (1.0f - b2) * gi * gi;
  m1[p] = a;
  m2[p] = b;
  const float v = P[p] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  P[p] = v;
  Wb[p] = f2bf16(v);
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* __restrict__ P, uint16_t* __restrict__ Wb) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < NP) Wb[p] = f2bf16(P[p]);
}

// Element features (x_E - centroid) / h, index c * 9 + i, for Q2 quads.
__global__ void __launch_bounds__(256) k_features(const double* __restrict__ x, const double* __restrict__ xs,
                                                  const int32_t* __restrict__ en, int64_t n_elem, int64_t n_node,
                                                  double hinv, float* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (e >= n_elem) return;
  const int32_t* nd = en + e * 9;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double v[9], m = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      v[i] = x[c * n_node + nd[i]];
      if (xs) v[i] = xs[c * n_node + nd[i]] - v[i];     // labels: displacement to x*
      m += v[i];
    }
    m *= 1.0 / 9.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) out[e * NF + c * 9 + i] = (float)((v[i] - m) * hinv);
  }
}

// One colour of the merge: acc[c][I] += Y[e][c * 9 + i], cnt[I] += 1.
__global__ void __launch_bounds__(256) k_merge(const float* __restrict__ Y, const int32_t* __restrict__ list,
                                               int64_t n_list, const int32_t* __restrict__ en, int64_t n_node,
                                               double* __restrict__ acc, double* __restrict__ cnt) {
  const int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (k >= n_list) return;
  const int64_t e = list[k];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int32_t I = en[e * 9 + i];
    acc[I] += (double)Y[e * NF + i];
    acc[n_node + I] += (double)Y[e * NF + 9 + i];
    cnt[I] += 1.0;
  }
}

__global__ void __launch_bounds__(256) k_propose(const double* __restrict__ x, const double* __restrict__ acc,
                                                 const double* __restrict__ cnt, const double* __restrict__ mask,
                                                 int64_t n_node, double h, double* __restrict__ xo) {
  const int64_t I = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (I >= n_node) return;
  const double c = cnt[I] > 0.0 ? cnt[I] : 1.0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int64_t k = d * n_node + I;
    xo[k] = mask[k] != 0.0 ? x[k] + h * acc[k] / c : x[k];
  }
}

inline int grid_of(int64_t n, int per, int cap) {
  int64_t g = (n + per - 1) / per;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

struct tmop_mlp {
  int device = 0;
  float* P = nullptr;          // FP32 master [NP]
  uint16_t* Wb = nullptr;      // BF16 copy [NP]
  float* m1 = nullptr;         // Adam moments [NP]
  float* m2 = nullptr;
  float* g = nullptr;          // gradient [NP]
  int64_t step = 0;
  // scratch, grown on demand
  int64_t cap_n = 0;
  float* Zs = nullptr;         // [3][cap_n][64]
  float* Hs = nullptr;
  float* dZ = nullptr;
  float* Y = nullptr;          // [cap_n][18]
  float* dY = nullptr;
  float* part = nullptr;       // [nb][NP]
  int64_t cap_part = 0;
  double* lpart = nullptr;     // [1024 + 1]
  double* h_loss = nullptr;    // pinned
  int64_t cap_node = 0;
  double* acc = nullptr;       // [2][cap_node] + [cap_node]
};

#define HIP_OK(call) \
  do { if ((call) != hipSuccess) return TMOP_E_HIP; } while (0)

namespace {

constexpr int CHUNK = 256;     // samples per weight-gradient block

int grow(tmop_mlp* m, int64_t n) {
  if (n > m->cap_n) {
    (void)hipFree(m->Zs); (void)hipFree(m->Hs); (void)hipFree(m->dZ); (void)hipFree(m->Y); (void)hipFree(m->dY);
    m->Zs = m->Hs = m->dZ = m->Y = m->dY = nullptr;
    m->cap_n = 0;
    if (hipMalloc(&m->Zs, 3 * n * NH * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->Hs, 3 * n * NH * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->dZ, 3 * n * NH * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->Y, n * NF * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->dY, n * NF * sizeof(float)) != hipSuccess)
      return TMOP_E_NOMEM;
    m->cap_n = n;
  }
  const int64_t nb = (n + CHUNK - 1) / CHUNK;
  if (nb > m->cap_part) {
    (void)hipFree(m->part);
    m->part = nullptr;
    m->cap_part = 0;
    if (hipMalloc(&m->part, nb * NP * sizeof(float)) != hipSuccess) return TMOP_E_NOMEM;
    m->cap_part = nb;
  }
  return TMOP_OK;
}

// dparams = d(sum(dY * Y))/dparams for the samples X (forward re-run here).
int backward_impl(tmop_mlp* m, const float* X, const float* dY, int64_t n, float* dparams, float* dX, hipStream_t s) {
  int st = grow(m, n);
  if (st != TMOP_OK) return st;
  const int g = grid_of((n + 15) / 16, 1, 65536);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(64), 0, s, m->Wb, m->P, X, n, m->Y, m->Zs, m->Hs);
  hipLaunchKernelGGL(k_mlp_bwd_data, dim3(g), dim3(64), 0, s, m->Wb, m->Zs, dY, n, m->dZ, dX);
  const int nb = (int)((n + CHUNK - 1) / CHUNK);
  hipLaunchKernelGGL(k_mlp_bwd_weights, dim3(nb), dim3(256), 0, s, X, m->Hs, m->dZ, dY, n, CHUNK, m->part);
  hipLaunchKernelGGL(k_fold_partials, dim3((NP + 255) / 256), dim3(256), 0, s, m->part, nb, dparams);
  HIP_OK(hipGetLastError());
  return TMOP_OK;
}

}  // namespace

extern "C" {

int tmop_mlp_create(const float* params, tmop_mlp** out) {
  if (!out) return TMOP_E_ARG;
  *out = nullptr;
  if (!params) return TMOP_E_ARG;
  tmop_mlp* m = new (std::nothrow) tmop_mlp();
  if (!m) return TMOP_E_NOMEM;
  if (hipGetDevice(&m->device) != hipSuccess) { delete m; return TMOP_E_HIP; }
  bool ok = hipMalloc(&m->P, NP * sizeof(float)) == hipSuccess && hipMalloc(&m->Wb, NP * sizeof(uint16_t)) == hipSuccess &&
            hipMalloc(&m->m1, NP * sizeof(float)) == hipSuccess && hipMalloc(&m->m2, NP * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->g, NP * sizeof(float)) == hipSuccess && hipMalloc(&m->lpart, 1025 * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&m->h_loss, sizeof(double), 0) == hipSuccess;
  if (ok) ok = hipMemcpy(m->P, params, NP * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemset(m->m1, 0, NP * sizeof(float)) == hipSuccess && hipMemset(m->m2, 0, NP * sizeof(float)) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_to_bf16, dim3((NP + 255) / 256), dim3(256), 0, 0, m->P, m->Wb);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) { tmop_mlp_destroy(m); return TMOP_E_NOMEM; }
  *out = m;
  return TMOP_OK;
}

void tmop_mlp_destroy(tmop_mlp* m) {
  if (!m) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(m->device);
  (void)hipFree(m->P); (void)hipFree(m->Wb); (void)hipFree(m->m1); (void)hipFree(m->m2); (void)hipFree(m->g);
  (void)hipFree(m->Zs); (void)hipFree(m->Hs); (void)hipFree(m->dZ); (void)hipFree(m->Y); (void)hipFree(m->dY);
  (void)hipFree(m->part); (void)hipFree(m->lpart); (void)hipFree(m->acc);
  if (m->h_loss) (void)hipHostFree(m->h_loss);
  (void)hipSetDevice(cur);
  delete m;
}

int tmop_mlp_get_params(tmop_mlp* m, float* params) {
  if (!m || !params) return TMOP_E_ARG;
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(params, m->P, NP * sizeof(float), hipMemcpyDeviceToHost));
  return TMOP_OK;
}

int tmop_mlp_forward(tmop_mlp* m, const float* X, float* Y, int64_t n, void* stream) {
  if (!m || !X || !Y || n < 0) return TMOP_E_ARG;
  if (n == 0) return TMOP_OK;
  const int g = grid_of((n + 15) / 16, 1, 65536);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(64), 0, (hipStream_t)stream, m->Wb, m->P, X, n, Y, (float*)nullptr,
                     (float*)nullptr);
  HIP_OK(hipGetLastError());
  return TMOP_OK;
}

int tmop_mlp_backward(tmop_mlp* m, const float* X, const float* dY, int64_t n, float* dparams, float* dX,
                      void* stream) {
  if (!m || !X || !dY || !dparams || n < 1) return TMOP_E_ARG;
  return backward_impl(m, X, dY, n, dparams, dX, (hipStream_t)stream);
}

int tmop_mlp_train_step(tmop_mlp* m, const float* X, const float* L, int64_t n, float lr, double* loss,
                        void* stream) {
  if (!m || !X || !L || n < 1 || !(lr > 0.0f)) return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int st = grow(m, n);
  if (st != TMOP_OK) return st;
  const int g = grid_of((n + 15) / 16, 1, 65536);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(64), 0, s, m->Wb, m->P, X, n, m->Y, m->Zs, m->Hs);
  const int64_t cnt = n * NF;
  const int gl = grid_of(cnt, 256, 1024);
  hipLaunchKernelGGL(k_mse, dim3(gl), dim3(256), 0, s, m->Y, L, cnt, (float)(2.0 / (double)cnt), m->dY, m->lpart);
  hipLaunchKernelGGL(k_fold_loss, dim3(1), dim3(64), 0, s, m->lpart, gl, m->lpart + 1024);
  hipLaunchKernelGGL(k_mlp_bwd_data, dim3(g), dim3(64), 0, s, m->Wb, m->Zs, m->dY, n, m->dZ, (float*)nullptr);
  const int nb = (int)((n + CHUNK - 1) / CHUNK);
  hipLaunchKernelGGL(k_mlp_bwd_weights, dim3(nb), dim3(256), 0, s, X, m->Hs, m->dZ, m->dY, n, CHUNK, m->part);
  hipLaunchKernelGGL(k_fold_partials, dim3((NP + 255) / 256), dim3(256), 0, s, m->part, nb, m->g);
  m->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)m->step), c2 = 1.0f - powf(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, s, m->P, m->m1, m->m2, m->g, m->Wb, lr, b1, b2,
                     1e-8f, c1, c2);
  HIP_OK(hipGetLastError());
  if (loss) {
    HIP_OK(hipMemcpyAsync(m->h_loss, m->lpart + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *loss = *m->h_loss / (double)cnt;
  }
  return TMOP_OK;
}

// The network works in units of the constant isotropic target's size h
// (W = h I): per-point targets give no single h.
static int mlp_ctx_ok(const tmop_ctx* c) {
  if (!c) return TMOP_E_ARG;
  if (c->dim != 2 || c->p != 2 || !c->base.iso || c->d_tsize) return TMOP_E_UNSUPPORTED;
  return TMOP_OK;
}

int tmop_mlp_features(tmop_ctx* c, const double* x, float* X, void* stream) {
  int st = mlp_ctx_ok(c);
  if (st != TMOP_OK) return st;
  if (!x || !X) return TMOP_E_ARG;
  hipLaunchKernelGGL(k_features, dim3(grid_of(c->n_elem, 256, 1 << 30)), dim3(256), 0, (hipStream_t)stream, x,
                     (const double*)nullptr, c->d_elem_node, c->n_elem, c->n_node, c->base.s_inv, X);
  HIP_OK(hipGetLastError());
  return TMOP_OK;
}

int tmop_mlp_labels(tmop_ctx* c, const double* x, const double* xstar, float* L, void* stream) {
  int st = mlp_ctx_ok(c);
  if (st != TMOP_OK) return st;
  if (!x || !xstar || !L) return TMOP_E_ARG;
  hipLaunchKernelGGL(k_features, dim3(grid_of(c->n_elem, 256, 1 << 30)), dim3(256), 0, (hipStream_t)stream, x,
                     xstar, c->d_elem_node, c->n_elem, c->n_node, c->base.s_inv, L);
  HIP_OK(hipGetLastError());
  return TMOP_OK;
}

int tmop_mlp_propose(tmop_ctx* c, tmop_mlp* m, const double* x, double* x_out, void* stream) {
  int st = mlp_ctx_ok(c);
  if (st != TMOP_OK) return st;
  if (!m || !x || !x_out || x_out == x) return TMOP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if ((st = grow(m, c->n_elem)) != TMOP_OK) return st;
  if (c->n_node > m->cap_node) {
    (void)hipFree(m->acc);
    m->acc = nullptr;
    m->cap_node = 0;
    if (hipMalloc(&m->acc, 3 * c->n_node * sizeof(double)) != hipSuccess) return TMOP_E_NOMEM;
    m->cap_node = c->n_node;
  }
  float* X = m->dY;                                  // features (scratch)
  hipLaunchKernelGGL(k_features, dim3(grid_of(c->n_elem, 256, 1 << 30)), dim3(256), 0, s, x, (const double*)nullptr,
                     c->d_elem_node, c->n_elem, c->n_node, c->base.s_inv, X);
  const int g = grid_of((c->n_elem + 15) / 16, 1, 65536);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(64), 0, s, m->Wb, m->P, X, c->n_elem, m->Y, (float*)nullptr,
                     (float*)nullptr);
  double* acc = m->acc;
  double* cnt = m->acc + 2 * c->n_node;
  HIP_OK(tmop::fill(acc, 0.0, 3 * c->n_node, s));
  for (size_t k = 0; k + 1 < c->color_off.size(); ++k) {
    const int64_t nl = c->color_off[k + 1] - c->color_off[k];
    if (nl == 0) continue;
    hipLaunchKernelGGL(k_merge, dim3(grid_of(nl, 256, 1 << 30)), dim3(256), 0, s, m->Y, c->d_colors + c->color_off[k],
                       nl, c->d_elem_node, c->n_node, acc, cnt);
  }
  hipLaunchKernelGGL(k_propose, dim3(grid_of(c->n_node, 256, 1 << 30)), dim3(256), 0, s, x, acc, cnt, c->d_mask,
                     c->n_node, 1.0 / c->base.s_inv, x_out);
  HIP_OK(hipGetLastError());
  return TMOP_OK;
}

}  // extern "C"
