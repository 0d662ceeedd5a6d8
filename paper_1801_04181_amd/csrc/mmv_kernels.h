// Launch wrappers of the HIP kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "mmv_internal.h"

namespace mmv {

template <typename T>
hipError_t launch_row_fwd(const T* src, void* dst, int nrows, int nin, int N2x, int Kx, const FftPlan& P,
                          const void* tw, const void* twp, hipStream_t st, int ny3 = 0);
template <typename T>
hipError_t launch_col(const void* spec1, void* spec2, const T* kern, int Kx, int Ly, int Kyh, int ny, int nin_ch,
                      int ngroup, const FftPlan& P, const void* twy, const OutTable& tab, hipStream_t st,
                      const TickArgs* tick = nullptr, int tick_stage = -1, double tick_dt = 0.0);
// the pending slider update alone (after the last row launch of a call)
hipError_t launch_tick(const TickArgs& tick, int stage, double dt, hipStream_t st);
hipError_t launch_tick_batch(const ColDesc* d, int n, int stage, double dt, hipStream_t st);
template <typename T>
hipError_t launch_row_stage(const RowParams& p, const void* spec2, const T* mst, const T* m0, T* mnext, T* acc,
                            T* hout, const void* tw, const void* twp, RigidState* rigid, double* partial,
                            unsigned* counter, hipStream_t st);
hipError_t launch_kernel_real(double* out, int Lx, int Ly, int kind, int comp, double dzc, double dx, double dy,
                              double dz, double rc, double scale, int pbc, int images, hipStream_t st);
template <typename T>
hipError_t launch_colpack(const void* spec, T* out, int Kx, int Ly, int Kyh, const FftPlan& P, const void* twy,
                          int imag, hipStream_t st);
template <typename T>
size_t row_lds_bytes(const RowParams& p);

// batched launches over many film pairs
template <typename T>
hipError_t launch_row_fwd_batch(const RowFwdDesc* d, const int* start, int n, int nblk, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_col_batch(const ColDesc* d, const int* start, int n, int nblk, size_t lds, hipStream_t st,
                            int tick_stage = -1, double tick_dt = 0.0);
template <typename T>
hipError_t launch_row_stage_batch(const RowStageDesc* d, const int* start, int n, int nblk, size_t lds, int stage,
                                  double dt, bool inplace, int nt, hipStream_t st);
// Whether the batched row kernel exists with nt threads per block (512; 128
// and 256 for float32 in-place row lengths).
template <typename T>
bool row_batch_threads_ok(int nt, bool inplace);
// Adaptive Dormand-Prince run: end of an attempt (slider's last stage, error,
// decision, next step) and the commit of an accepted state.
hipError_t launch_dp_control(const TickArgs& tick, DpCtrl* ctrl, const double* errpart, int ntask, hipStream_t st);
template <typename T>
hipError_t launch_dp_commit(const T* y5, T* m, int nfilm, size_t plane, const DpCtrl* ctrl, int* flags,
                            hipStream_t st);
// Eq. 13: per slider row, sums of |div H| and |curl H| of the base field on
// the stencil points written by the force pass.
template <typename T>
hipError_t launch_div_curl(const T* G, int nx, int ny, double dx, double dy, double dz, int pbc_y, double* part,
                           hipStream_t st);
// The row kernel can transform rows of this length in place.
bool row_inplace_length(int L);
size_t row_fwd_lds_bytes(int N2x, int esz);
template <typename T>
hipError_t prepare_batch_kernels(size_t lds_fwd, size_t lds_col, size_t lds_stage);

// single-magnet three-dimensional path
struct CubeLaunch {
  int nx, ny, nz;
  double dx, dy, dz;
  double pref_ex, pref_an, u[3], hext[3], gam, alpha;
  int pbc;  // periodic in-plane axes (bit 0 = x, 1 = y) of the exchange stencil and the Neumann problem
};
template <typename T>
hipError_t launch_fft_axis(const void* in, void* out, int nplanes, int ncols, int CB, int n_in, long long in_ps,
                           int n_out, long long out_ps, const FftPlan& P, const void* tw, bool inv, hipStream_t st);
template <typename T>
hipError_t launch_zmul(void* buf, const T* kern, int Kx, int Ly, int nz, int CB, int mode, double sgn,
                       const FftPlan& P, const void* twz, hipStream_t st);
template <typename T>
hipError_t launch_row_inv(const void* spec, T* out, int nrows, int R, int nx, int N2x, int Kx, const FftPlan& P,
                          const void* tw, const void* twp, hipStream_t st);
template <typename T>
hipError_t launch_stage3(const CubeLaunch& c, int mode, int stage, int mask, double dt, const T* ms, const T* m0,
                         T* mnext, T* acc, const T* hd, const T* he, T* hout, int* flags, RigidState* tick,
                         T* dmstep, hipStream_t st);
template <typename T>
hipError_t launch_eddy_bdot(size_t N, const T* dm, const T* hdm, T* bdot, double mu0, double Ms, double idt,
                            int first, hipStream_t st);
template <typename T>
hipError_t launch_sor_rhs(const CubeLaunch& c, const T* es, T* r, double* part, double* mean, hipStream_t st);
// float64 partial sums (res^2, r^2) of the Neumann residual, nblk blocks
template <typename T>
hipError_t launch_sor_residual(const CubeLaunch& c, const T* phi, const T* r, double* part, int nblk, hipStream_t st);
template <typename T>
hipError_t launch_sor(const CubeLaunch& c, int nbox, T* phi, T* phi2, const T* r, double omega, int sweeps,
                      double* part, double* mean, hipStream_t st);
// The nbox Neumann problems solved exactly in the cosine basis (r -> phi,
// zero mean; work: scratch of the same size); P, tw: FFT plans and twiddle
// tables of lengths nx, ny, nz ({2,3,5,7}-smooth).
template <typename T>
hipError_t launch_neumann_solve(const CubeLaunch& c, int nbox, const T* r, T* phi, T* work, const FftPlan* P,
                                const void* const* tw, hipStream_t st);
template <typename T>
hipError_t launch_current(const CubeLaunch& c, const T* phi, const T* es, T* J, double sigma, hipStream_t st);
hipError_t launch_kernel_real3(double* out, int Lx, int Ly, int Lz, int kind, int comp, double dx, double dy,
                               double dz, double rc, double scale, hipStream_t st);
template <typename T>
hipError_t launch_pack3(const void* spec, T* out, int Kx, int Ly, int Lz, int imag, hipStream_t st);
template <typename T>
size_t col_lds_bytes(int Ly, int nbuf);
template <typename T>
int col_blocks_per_cu(size_t lds);

// LDS of one CU, and the parts of it reserved for what the row and y-pass
// kernels declare statically (row and output tables, reduction slots): a
// launch's dynamic LDS must fit in the rest.
constexpr size_t LDS_PER_CU = 160 * 1024;
constexpr size_t ROW_STATIC_LDS = 512;
constexpr size_t COL_STATIC_LDS = 640;
// true if the compiled row and y-pass kernels stay within those reserves
template <typename T>
bool static_lds_within_reserve();

// Tricubic B-spline of a [nz][ny][nx] field: prefilter along x, y, z
// (field -> coef, using work; the three must not overlap) and the 64-tap
// gather at npts points [npts][3] (x, y, z in cells).
template <typename T>
hipError_t launch_spline3_prefilter(const T* field, T* coef, T* work, int nx, int ny, int nz, hipStream_t st);
template <typename T>
hipError_t launch_spline3_gather(const T* coef, int nx, int ny, int nz, const T* pts, int npts, T* out,
                                 hipStream_t st);

}  // namespace mmv
