// Tricubic B-spline of a three-dimensional scalar field: the prefilter
// along x, y and z (Sec. III.A: coefficients whose spline passes through
// the lattice values, whole-sample mirror ends) and the 4 x 4 x 4 gather at
// arbitrary points (the 64 nearest-neighbour lookups of Sec. IV.D), the
// interpolation that motion along more than one axis needs.
//
// The prefilter applies the exact inverse of the cubic B-spline's sampling
// filter (z + 4 + 1/z) / 6 on the mirror-periodic extension of each line:
// c_i = sum_j sqrt(3) z1^|j| f(i - j), z1 = sqrt(3) - 2, truncated at
// |j| <= K (|z1|^K below the precision's rounding: K = 16 in float32, 30
// in float64).  On the mirror-periodic extension this equals the
// tridiagonal solve with mirror rows at any line length.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mmv_kernels.h"

namespace mmv {

namespace {

template <typename T> struct Spl3Taps { static constexpr int K = 16; };
template <> struct Spl3Taps<double> { static constexpr int K = 30; };

__device__ __forceinline__ int mirror(int k, int M) {
  if (M == 1) return 0;
  const int P = 2 * M - 2;
  k %= P;
  if (k < 0) k += P;
  return k > M - 1 ? P - k : k;
}

template <typename T>
__device__ __forceinline__ T bspline3(T t) {
  const T a = fabs(t);
  if (a <= T(1)) return T(2) / T(3) - a * a + T(0.5) * a * a * a;
  if (a <= T(2)) {
    const T b = T(2) - a;
    return b * b * b / T(6);
  }
  return T(0);
}

// One output coefficient per thread along axis `ax` of a [nz][ny][nx] array:
// c_i = w_0 f_i + sum_{j=1..K} w_j (f_{i-j} + f_{i+j}), w_j = sqrt(3) z1^j,
// the block's weights in LDS; mirror indices only near the line's ends.
template <typename T>
__global__ void __launch_bounds__(256)
    k_spline3_prefilter(const T* __restrict__ in, T* __restrict__ out, int nx, int ny, int nz, int ax) {
  constexpr int K = Spl3Taps<T>::K;
  __shared__ T w[K + 1];
  if (threadIdx.x <= K) w[threadIdx.x] = (T)(1.7320508075688772935 * pow(-0.26794919243112270647, (double)threadIdx.x));
  __syncthreads();
  const long long n = (long long)nx * ny * nz;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int ix = (int)(id % nx);
  const int iy = (int)((id / nx) % ny);
  const int iz = (int)(id / ((long long)nx * ny));
  const int M = ax == 0 ? nx : (ax == 1 ? ny : nz);
  const int i = ax == 0 ? ix : (ax == 1 ? iy : iz);
  const long long stride = ax == 0 ? 1 : (ax == 1 ? nx : (long long)nx * ny);
  const T* line = in + (id - (long long)i * stride);
  T acc = w[0] * line[(long long)i * stride];
  if (i >= K && i + K < M) {
    const T* f = line + (long long)i * stride;
#pragma unroll
    for (int j = 1; j <= K; ++j) acc += w[j] * (f[-(long long)j * stride] + f[(long long)j * stride]);
  } else {
#pragma unroll 4
    for (int j = 1; j <= K; ++j)
      acc += w[j] * (line[(long long)mirror(i - j, M) * stride] + line[(long long)mirror(i + j, M) * stride]);
  }
  out[id] = acc;
}

// One point per thread: s(p) = sum over the 4 x 4 x 4 nearest coefficients
// of beta3 products, z outermost, x innermost; mirror-extended indices.
template <typename T>
__global__ void __launch_bounds__(256)
    k_spline3_gather(const T* __restrict__ c, int nx, int ny, int nz, const T* __restrict__ pts, int npts,
                     T* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const T u = pts[3 * (size_t)p], v = pts[3 * (size_t)p + 1], w = pts[3 * (size_t)p + 2];
  const int ku = (int)floor(u), kv = (int)floor(v), kw = (int)floor(w);
  T wx[4], wy[4], wz[4];
  int ix[4], iy[4], iz[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    wx[t] = bspline3<T>(u - (T)(ku + t - 1));
    wy[t] = bspline3<T>(v - (T)(kv + t - 1));
    wz[t] = bspline3<T>(w - (T)(kw + t - 1));
    ix[t] = mirror(ku + t - 1, nx);
    iy[t] = mirror(kv + t - 1, ny);
    iz[t] = mirror(kw + t - 1, nz);
  }
  T acc = T(0);
#pragma unroll
  for (int tz = 0; tz < 4; ++tz)
#pragma unroll
    for (int ty = 0; ty < 4; ++ty) {
      const T* row = c + ((size_t)iz[tz] * ny + iy[ty]) * nx;
      const T wzy = wz[tz] * wy[ty];
#pragma unroll
      for (int tx = 0; tx < 4; ++tx) acc += (wzy * wx[tx]) * row[ix[tx]];
    }
  out[p] = acc;
}

}  // namespace

template <typename T>
hipError_t launch_spline3_prefilter(const T* field, T* coef, T* work, int nx, int ny, int nz, hipStream_t st) {
  const long long n = (long long)nx * ny * nz;
  const dim3 grid((unsigned)((n + 255) / 256));
  // x: field -> coef, y: coef -> work, z: work -> coef
  hipLaunchKernelGGL(k_spline3_prefilter<T>, grid, dim3(256), 0, st, field, coef, nx, ny, nz, 0);
  hipLaunchKernelGGL(k_spline3_prefilter<T>, grid, dim3(256), 0, st, (const T*)coef, work, nx, ny, nz, 1);
  hipLaunchKernelGGL(k_spline3_prefilter<T>, grid, dim3(256), 0, st, (const T*)work, coef, nx, ny, nz, 2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spline3_gather(const T* coef, int nx, int ny, int nz, const T* pts, int npts, T* out,
                                 hipStream_t st) {
  if (npts <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_spline3_gather<T>, dim3((npts + 255) / 256), dim3(256), 0, st, coef, nx, ny, nz, pts, npts,
                     out);
  return hipGetLastError();
}

template hipError_t launch_spline3_prefilter<float>(const float*, float*, float*, int, int, int, hipStream_t);
template hipError_t launch_spline3_prefilter<double>(const double*, double*, double*, int, int, int, hipStream_t);
template hipError_t launch_spline3_gather<float>(const float*, int, int, int, const float*, int, float*, hipStream_t);
template hipError_t launch_spline3_gather<double>(const double*, int, int, int, const double*, int, double*,
                                                  hipStream_t);

}  // namespace mmv
