// Launch wrappers and launch tables of the thick two-film path (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "mmv_internal.h"

namespace mmv {

// One target window of a layer-coupled product: the source film's spectra
// times the kernel of each layer offset, summed over the source layers, for
// the target layers tz0 .. tz0 + ntz - 1 (in the source film's lattice).
// The window starts at lattice x0 = xs * s_int + xoff, y0 = yoff; its
// spectra [3][ntz][Ly][Kx] start at element `out` of the product buffer.
struct SlabGroup {
  int src;
  int tz0, ntz;
  int xs, xoff, yoff;
  long long out;
};

struct SlabMulTable {
  int n;
  SlabGroup g[4];
};

template <typename T>
hipError_t launch_slab_pack(const void* spec, T* out, int n, int imag, hipStream_t st);
// mode 0: out_a = sum_b N_ab v_b (six tensor components); mode 1: out =
// sgn * S x v (three components); sgn also scales mode 0
template <typename T>
hipError_t launch_slab_mul(const void* in, void* out, const T* kern, const SlabMulTable& tab, int nz, int D, int Lx,
                           int Ly, int Kx, int mode, double sgn, const RigidState* rigid, hipStream_t st);
size_t slab_sample_lds(int M, int esz);
// The rows of a sampling launch: nch channels of nrow output rows; output
// row r of a block of orows reads input row (r + roff) mod wrows of the
// block (nrow_in input rows per channel), whose window is the M elements from
// column cs * s_int + c_off (rows ld apart), modulo period when period > 0.
struct SlabRows {
  int nch, nrow, nrow_in;
  int orows, wrows, roff;
  int M, ld, cs, c_off, period;
};
// rows of their own (one block, identity row map, no column offset)
inline SlabRows slab_rows(int nch, int nrow, int M) { return SlabRows{nch, nrow, nrow, nrow, nrow, 0, M, M, 0, 0, 0}; }
template <typename T>
hipError_t launch_slab_sample(const T* win, const SlabRows& R, int h, T* out, int i0, int nw, int sgn, int add,
                              int interp, double inv_dx, const RigidState* rigid, hipStream_t st);
// scalar potential sgn * S . v per target layer (one channel), groups as
// launch_slab_mul
template <typename T>
hipError_t launch_slab_pot(const void* in, void* out, const T* kern, const SlabMulTable& tab, int nz, int D, int Lx,
                           int Ly, int Kx, double sgn, const RigidState* rigid, hipStream_t st);
// -grad of a sampled potential P[.][py][px] by four-point differences on
// [3][ol][oy][ox], output (l, j, i) at P[l + o0][j + o0][i + o0]
template <typename T>
hipError_t launch_slab_potgrad(const T* P, int py, int px, int o0, int ol, int oy, int ox, T* out, int add, double dx,
                               double dy, double dz, hipStream_t st);
template <typename T>
hipError_t launch_slab_add(int n, const T* src, T* dst, hipStream_t st);
int slab_force_blocks(int ncell);
template <typename T>
hipError_t launch_slab_force(const T* G, const T* m, T* hd, int nx, int ny, int nz, int add, double dx, double dy,
                             double dz, double* part, hipStream_t st);
template <typename T>
hipError_t launch_slab_bdot(int n, int ncell, const T* hd, const T* m, const double hext[3], double mu0, double Ms,
                            double idt, int first, double* Bprev, T* bdot, hipStream_t st);

}  // namespace mmv
