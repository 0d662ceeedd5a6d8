// Launch wrappers of the HIP kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "mmv_internal.h"

namespace mmv {

template <typename T>
hipError_t launch_row_fwd(const T* src, void* dst, int nrows, int nin, int N2x, int Kx, const FftPlan& P,
                          const void* tw, const void* twp, hipStream_t st);
template <typename T>
hipError_t launch_col(const void* spec1, void* spec2, const T* kern, int Kx, int Ly, int Kyh, int ny, int nin_ch,
                      int ngroup, const FftPlan& P, const void* twy, const OutTable& tab, hipStream_t st);
template <typename T>
hipError_t launch_row_stage(const RowParams& p, const void* spec2, const T* mst, const T* m0, T* mnext, T* acc,
                            T* hout, const void* tw, const void* twp, RigidState* rigid, double* partial,
                            unsigned* counter, hipStream_t st);
hipError_t launch_kernel_real(double* out, int Lx, int Ly, int kind, int comp, double dzc, double dx, double dy,
                              double dz, double rc, double scale, hipStream_t st);
template <typename T>
hipError_t launch_colpack(const void* spec, T* out, int Kx, int Ly, int Kyh, const FftPlan& P, const void* twy,
                          int imag, hipStream_t st);
template <typename T>
size_t row_lds_bytes(const RowParams& p);
template <typename T>
size_t col_lds_bytes(int Ly, int nbuf);

}  // namespace mmv
