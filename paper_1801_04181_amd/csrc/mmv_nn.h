// Dense kernels of the learned stray-field operator (host launchers).
#pragma once
#include <hip/hip_runtime.h>

namespace mmv {

// C[b](m, n) = alpha sum_k A[b](m, k) B[b](k, n) + beta C[b](m, n), strided
// views of float32 arrays; A and B enter the matrix cores as bfloat16.
struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int M, N, K;
  long long am, ak, sa;
  long long bk, bn, sb;
  long long cm, cn, sc;
  float alpha, beta;
  // split-K: blockIdx.z = batch * nsplit + split covers K range
  // [split * kchunk, (split + 1) * kchunk) and writes C + b * sc + split * ps
  int kchunk;
  long long ps;
};

hipError_t launch_gemm(const GemmArgs& g, int batch, hipStream_t st);
// dst[i] = (accumulate ? dst[i] : 0) + sum_p src[p * n + i], fixed order
hipError_t launch_sum_parts(int nparts, long long n, const float* src, float* dst, int accumulate, hipStream_t st);
hipError_t launch_bias_act(long long n, int hw, int C, const float* s, const float* u, const float* bias, float* pre,
                           float* y, int act, hipStream_t st);
hipError_t launch_act_grad(long long n, const float* pre, const float* dy, float* g, hipStream_t st);
hipError_t launch_channel_sum(int B, int C, int hw, const float* g, float* db, int accumulate, hipStream_t st);
int mse_blocks(long long n);
hipError_t launch_mse(long long n, const float* p, const float* t, float* d, double* part, hipStream_t st);
hipError_t launch_adam(long long n, float* w, const float* g, float* m1, float* m2, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st);
hipError_t launch_axpy(long long n, float a, const float* x, const float* y, float* out, hipStream_t st);

}  // namespace mmv
