// Dense kernels of the learned stray-field operator: one strided, batched
// BF16 matrix product on the CDNA matrix cores (v_mfma_f32_32x32x8bf16_1k,
// float32 accumulation) and the element-wise kernels around it (GELU and its
// derivative, bias, residual sums, mean-square loss, Adam).
//
// C[b](m, n) = alpha * sum_k A[b](m, k) B[b](k, n) + beta * C[b](m, n)
// with A(m, k) = A[b*sa + m*am + k*ak], B(k, n) = B[b*sb + k*bk + n*bn],
// C(m, n) = C[b*sc + m*cm + n*cn]; A and B are float32 in memory and rounded
// to bfloat16 (nearest-even) as they enter the matrix cores.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mmv_nn.h"

namespace mmv {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Block of four 64-lane waves, WM x WN waves of 32 x 32 output tiles each
// (64 x 64, or 128 x 32 / 32 x 128 for a narrow N / M).  K advances in
// chunks of KC: the block loads the A and B pieces of a chunk with every
// element's load in flight at once, along whichever index is contiguous in
// memory (coalesced for row- and column-major views alike), rounds them to
// bfloat16 into LDS, and while the matrix cores consume the chunk from LDS
// the next chunk's loads are already issued.  Each wave's accumulation runs
// through the same 8-wide k steps in the same order as a single-wave loop.
// MFMA operands: lane l feeds A(i, k) with i = l % 32, k = k0 + 4 (l / 32) + v
// and B(k, j) with j = l % 32; accumulator register r holds
// C(8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
constexpr int GEMM_KC = 32;
constexpr int GEMM_PAD = 4;  // bf16 elements of padding per LDS row

__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int WM, int WN>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  constexpr int TM = 32 * WM, TN = 32 * WN, KC = GEMM_KC, RS = KC + GEMM_PAD;
  constexpr int NA = TM * KC / 256, NB = TN * KC / 256;  // elements per thread and chunk
  __shared__ __align__(16) short sA[TM * RS];
  __shared__ __align__(16) short sB[TN * RS];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int nsplit = g.kchunk > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  const long long b = blockIdx.z / nsplit;
  const int split = blockIdx.z - (int)b * nsplit;
  const int kbeg = g.kchunk > 0 ? split * g.kchunk : 0;
  const int kend = g.kchunk > 0 ? min(g.K, kbeg + g.kchunk) : g.K;
  const int bm0 = blockIdx.y * TM, bn0 = blockIdx.x * TN;
  const float* A = g.A + b * g.sa;
  const float* B = g.B + b * g.sb;
  float* C = g.C + b * g.sc + split * g.ps;
  // element e of a chunk -> (row, k): k fastest where it is contiguous
  const bool a_kfast = g.ak == 1, b_kfast = g.bn != 1;
  float ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
      const int gm = bm0 + m, gk = k0 + k;
      ra[u] = (gm < g.M && gk < kend) ? A[(long long)gm * g.am + (long long)gk * g.ak] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
      const int gn = bn0 + n, gk = k0 + k;
      rb[u] = (gn < g.N && gk < kend) ? B[(long long)gk * g.bk + (long long)gn * g.bn] : 0.0f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
      sA[m * RS + k] = to_bf16(ra[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
      sB[n * RS + k] = to_bf16(rb[u]);
    }
  };
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 31, lk = (lane >> 5) * 4;
  const short* pa = sA + (wm * 32 + li) * RS + lk;
  const short* pb = sB + (wn * 32 + li) * RS + lk;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  if (kbeg < kend) load(kbeg);
#pragma unroll 1
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    store();
    lds_sync();
    if (k0 + KC < kend) load(k0 + KC);
    // k steps past kend hold zeros in both operands
    const int nk = min(KC, ((kend - k0) + 7) & ~7);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 8) {
      if (kk < nk) {
        const bf16x4 av = *reinterpret_cast<const bf16x4*>(pa + kk);
        const bf16x4 bv = *reinterpret_cast<const bf16x4*>(pb + kk);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
      }
    }
    lds_sync();
  }
  const int m0 = bm0 + wm * 32, n0 = bn0 + wn * 32;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int j = n0 + (lane & 31);
    if (i < g.M && j < g.N) {
      float* c = C + (long long)i * g.cm + (long long)j * g.cn;
      *c = g.alpha * acc[r] + (g.beta != 0.0f ? g.beta * *c : 0.0f);
    }
  }
}

// Small products (M, N <= 32; the batched transforms over the kept modes):
// one 32 x 32 output tile per block, K in chunks of 128 whose loads are all in
// flight at once, and the four waves taking interleaved 8-wide k steps of a
// chunk (wave w: steps w, w + 4, ...); their partial tiles are summed in
// wave order at the end.
__global__ void __launch_bounds__(256) k_gemm_bf16_small(GemmArgs g) {
  constexpr int KC = 128, RS = KC + GEMM_PAD, NE = 32 * KC / 256;
  __shared__ __align__(16) short sA[32 * RS];
  __shared__ __align__(16) short sB[32 * RS];
  __shared__ float red[3][16][64];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int nsplit = g.kchunk > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  const long long b = blockIdx.z / nsplit;
  const int split = blockIdx.z - (int)b * nsplit;
  const int kbeg = g.kchunk > 0 ? split * g.kchunk : 0;
  const int kend = g.kchunk > 0 ? min(g.K, kbeg + g.kchunk) : g.K;
  const float* A = g.A + b * g.sa;
  const float* B = g.B + b * g.sb;
  float* C = g.C + b * g.sc + split * g.ps;
  const bool a_kfast = g.ak == 1, b_kfast = g.bn != 1;
  const int li = lane & 31, lk = (lane >> 5) * 4;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll 1
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    float ra[NE], rb[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = t + 256 * u;
      const int m = a_kfast ? e / KC : e % 32, k = a_kfast ? e % KC : e / 32;
      ra[u] = (m < g.M && k0 + k < kend) ? A[(long long)m * g.am + (long long)(k0 + k) * g.ak] : 0.0f;
      const int n = b_kfast ? e / KC : e % 32, kb = b_kfast ? e % KC : e / 32;
      rb[u] = (n < g.N && k0 + kb < kend) ? B[(long long)(k0 + kb) * g.bk + (long long)n * g.bn] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = t + 256 * u;
      const int m = a_kfast ? e / KC : e % 32, k = a_kfast ? e % KC : e / 32;
      sA[m * RS + k] = to_bf16(ra[u]);
      const int n = b_kfast ? e / KC : e % 32, kb = b_kfast ? e % KC : e / 32;
      sB[n * RS + kb] = to_bf16(rb[u]);
    }
    lds_sync();
    const int nk = min(KC, ((kend - k0) + 7) & ~7);
#pragma unroll
    for (int kk = 8 * wave; kk < KC; kk += 32) {
      if (kk < nk) {
        const bf16x4 av = *reinterpret_cast<const bf16x4*>(sA + li * RS + lk + kk);
        const bf16x4 bv = *reinterpret_cast<const bf16x4*>(sB + li * RS + lk + kk);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
      }
    }
    lds_sync();
  }
  if (wave > 0)
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave - 1][r][lane] = acc[r];
  lds_sync();
  if (wave == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int j = lane & 31;
      if (i < g.M && j < g.N) {
        float* c = C + (long long)i * g.cm + (long long)j * g.cn;
        *c = g.alpha * v + (g.beta != 0.0f ? g.beta * *c : 0.0f);
      }
    }
  }
}

hipError_t launch_gemm(const GemmArgs& g, int batch, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  const int nsplit = g.kchunk > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  if (g.M <= 32 && g.N <= 32 && g.K > 32) {
    hipLaunchKernelGGL(k_gemm_bf16_small, dim3(1, 1, batch * nsplit), dim3(256), 0, st, g);
  } else if (g.N <= 32) {
    dim3 grid((g.N + 31) / 32, (g.M + 127) / 128, batch * nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<4, 1>), grid, dim3(256), 0, st, g);
  } else if (g.M <= 32) {
    dim3 grid((g.N + 127) / 128, (g.M + 31) / 32, batch * nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<1, 4>), grid, dim3(256), 0, st, g);
  } else {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, batch * nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<2, 2>), grid, dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

__global__ void k_sum_parts(int nparts, long long n, const float* __restrict__ src, float* __restrict__ dst,
                            int accumulate) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float s = accumulate ? dst[i] : 0.0f;
    for (int p = 0; p < nparts; ++p) s += src[(long long)p * n + i];
    dst[i] = s;
  }
}

// ------------------------------------------------------------ element-wise
__device__ __forceinline__ float gelu(float x) {
  // tanh form of the Gaussian error linear unit
  const float c = 0.7978845608028654f, a = 0.044715f;
  return 0.5f * x * (1.0f + tanhf(c * (x + a * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float c = 0.7978845608028654f, a = 0.044715f;
  const float u = c * (x + a * x * x * x);
  const float t = tanhf(u);
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * a * x * x);
}

// y = act(s + u + bias[channel]); pre = s + u + bias (kept for the backward)
__global__ void k_bias_act(long long n, int hw, int C, const float* __restrict__ s, const float* __restrict__ u,
                           const float* __restrict__ bias, float* __restrict__ pre, float* __restrict__ y, int act) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int c = (int)((i / hw) % C);
    const float v = (s ? s[i] : 0.0f) + (u ? u[i] : 0.0f) + (bias ? bias[c] : 0.0f);
    if (pre) pre[i] = v;
    y[i] = act ? gelu(v) : v;
  }
}

// g = dy * gelu'(pre)
__global__ void k_act_grad(long long n, const float* __restrict__ pre, const float* __restrict__ dy,
                           float* __restrict__ g) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    g[i] = dy[i] * gelu_grad(pre[i]);
}

// per-channel sum over (batch, pixels) of g: db[c] (+)= sum
__global__ void __launch_bounds__(256)
    k_channel_sum(int B, int C, int hw, const float* __restrict__ g, float* __restrict__ db, int accumulate) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (long long t = threadIdx.x; t < (long long)B * hw; t += blockDim.x) {
    const long long b = t / hw, p = t - b * hw;
    s += g[(b * C + c) * hw + p];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = (accumulate ? db[c] : 0.0f) + red[0];
}

// d = 2 (p - t) / n, and per-block partial sums of (p - t)^2 and t^2
__global__ void __launch_bounds__(256)
    k_mse(long long n, const float* __restrict__ p, const float* __restrict__ t, float* __restrict__ d,
          double* __restrict__ part) {
  __shared__ double r1[256], r2[256];
  double e = 0.0, q = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float diff = p[i] - t[i];
    if (d) d[i] = 2.0f * diff / (float)n;
    e += (double)diff * diff;
    q += (double)t[i] * t[i];
  }
  r1[threadIdx.x] = e;
  r2[threadIdx.x] = q;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      r1[threadIdx.x] += r1[threadIdx.x + k];
      r2[threadIdx.x] += r2[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

// Adam with bias correction (step t >= 1), float32 master weights
__global__ void k_adam(long long n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// out = x + y (element-wise), or out = a x when y is null
// (out may alias x: each element is read before it is written by the same thread)
__global__ void k_axpy(long long n, float a, const float* x, const float* y, float* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (y ? y[i] : 0.0f);
}

static inline dim3 g1(long long n) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_sum_parts(int nparts, long long n, const float* src, float* dst, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, g1(n), dim3(256), 0, st, nparts, n, src, dst, accumulate);
  return hipGetLastError();
}

hipError_t launch_bias_act(long long n, int hw, int C, const float* s, const float* u, const float* bias, float* pre,
                           float* y, int act, hipStream_t st) {
  hipLaunchKernelGGL(k_bias_act, g1(n), dim3(256), 0, st, n, hw, C, s, u, bias, pre, y, act);
  return hipGetLastError();
}
hipError_t launch_act_grad(long long n, const float* pre, const float* dy, float* g, hipStream_t st) {
  hipLaunchKernelGGL(k_act_grad, g1(n), dim3(256), 0, st, n, pre, dy, g);
  return hipGetLastError();
}
hipError_t launch_channel_sum(int B, int C, int hw, const float* g, float* db, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_channel_sum, dim3(C), dim3(256), 0, st, B, C, hw, g, db, accumulate);
  return hipGetLastError();
}
int mse_blocks(long long n) { return (int)g1(n).x; }
hipError_t launch_mse(long long n, const float* p, const float* t, float* d, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, g1(n), dim3(256), 0, st, n, p, t, d, part);
  return hipGetLastError();
}
hipError_t launch_adam(long long n, float* w, const float* g, float* m1, float* m2, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, g1(n), dim3(256), 0, st, n, w, g, m1, m2, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_axpy(long long n, float a, const float* x, const float* y, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, g1(n), dim3(256), 0, st, n, a, x, y, out);
  return hipGetLastError();
}

}  // namespace mmv
