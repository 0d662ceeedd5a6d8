// HIP kernels of the thick two-film path: films nx x ny x nz cells (nz > 1)
// in relative motion along x, with eddy currents in both (Sec. II.A end,
// Sec. III.A-B, Eqs. 3, 6, 9-12; Sec. IV.C-D).
//
// Every field of one film on another film's cells (or its own) is a sum over
// the source film's layers of in-plane convolutions: the m (or dB/dt, or J)
// of each source layer is transformed along x and y once, and each target
// layer t takes sum_l K(t - l) * mhat_l with the kernel of the layer offset
// t - l (2-D spectra of the tensor N of Eq. 6, or of the potential kernel S of
// Eq. 8 for the eddy sums).  A target window that starts at lattice point
// (x0, y0) is shifted to the origin by the phase exp(2 pi i (kx x0 / Lx +
// ky y0 / Ly)) in the product, so the inverse transforms write it from index
// 0; x0 follows the slider's seat s_int, read from device memory.
//
//   k_slab_pack    one real part (or imaginary part) of a float64 kernel
//                  spectrum, in the mesh precision
//   k_slab_mul     the layer-coupled product of the source spectra with the
//                  kernel spectra, per target window (tensor or S x v)
//   k_slab_sample  one window row: cubic B-spline coefficients (mirror
//                  boundaries, a truncated symmetric filter) and samples at
//                  the other film's shifted cells, or linear interpolation
//   k_slab_force   the base field on the slider's cells and Eq. 3's force
//                  partials from the sampled stencil points
//   k_slab_bdot    B = mu0 (H_d + H_ext + Ms m) per cell and its backward
//                  difference over the step
#include <hip/hip_runtime.h>
#include <math.h>
#include "mmv_device.h"
#include "mmv_slab.h"

namespace mmv {

constexpr int SLAB_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_pack(const cpx<double>* __restrict__ spec, T* __restrict__ out, int n, int imag) {
  const int i = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (i < n) out[i] = (T)(imag ? spec[i].y : spec[i].x);
}

// exp(2 pi i (kx x0 / Lx + ky y0 / Ly)) with the integer products reduced
// first (an exact argument for any offset), times sgn.
template <typename T>
__device__ __forceinline__ cpx<T> slab_phase(int kx, int ky, int x0, int y0, int Lx, int Ly, T sgn) {
  long long px = ((long long)kx * x0) % Lx;
  if (px < 0) px += Lx;
  long long py = ((long long)ky * y0) % Ly;
  if (py < 0) py += Ly;
  const double frac = (double)px / (double)Lx + (double)py / (double)Ly;
  T ps, pc;
  if constexpr (sizeof(T) == 8)
    sincospi(2.0 * frac, &ps, &pc);
  else
    sincospif((float)(2.0 * frac), &ps, &pc);
  return mk<T>(pc * sgn, ps * sgn);
}

// out += K v for one layer pair: the six tensor components (xz, yz
// imaginary) in mode 0, S x v (S = (i sx, i sy, sz)) in mode 1.
template <typename T>
__device__ __forceinline__ void slab_mac(int mode, const T* kv, const cpx<T>& v0, const cpx<T>& v1, const cpx<T>& v2,
                                         cpx<T>& o0, cpx<T>& o1, cpx<T>& o2) {
  if (mode == 0) {
    const T nxx = kv[0], nyy = kv[1], nzz = kv[2], nxy = kv[3], ixz = kv[4], iyz = kv[5];
    // i * a for a complex v: (-v.y, v.x)
    o0 = o0 + scale(v0, nxx) + scale(v1, nxy) + mk<T>(-ixz * v2.y, ixz * v2.x);
    o1 = o1 + scale(v0, nxy) + scale(v1, nyy) + mk<T>(-iyz * v2.y, iyz * v2.x);
    o2 = o2 + mk<T>(-(ixz * v0.y + iyz * v1.y), ixz * v0.x + iyz * v1.x) + scale(v2, nzz);
  } else {
    // (S x v) = (i sy v2 - sz v1, sz v0 - i sx v2, i (sx v1 - sy v0))
    const T sx = kv[0], sy = kv[1], sz = kv[2];
    o0 = o0 + mk<T>(-sy * v2.y, sy * v2.x) - scale(v1, sz);
    o1 = o1 + scale(v0, sz) - mk<T>(-sx * v2.y, sx * v2.x);
    const cpx<T> d = scale(v1, sx) - scale(v0, sy);
    o2 = o2 + mk<T>(-d.y, d.x);
  }
}

// The product for a compile-time layer count NZ: one thread per spectral
// point and target window holds the NZ source layers and the (at most
// NZ + 2) target layers in registers and reads each layer offset's kernel
// once (offsets tz0 - NZ + 1 .. tz0 + ntz - 1).  Grid: (points / SLAB_THREADS,
// groups).
template <typename T, int NZ>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_mul_nz(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const T* __restrict__ kern,
                  SlabMulTable tab, int D, int Lx, int Ly, int Kx, int mode, T sgn,
                  const RigidState* __restrict__ rigid) {
  constexpr int NT = NZ + 2;
  const int plane = Ly * Kx;
  const int q = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (q >= plane) return;
  const SlabGroup G = tab.g[blockIdx.y];
  const int ky = q / Kx, kx = q - ky * Kx;
  const size_t ks = (size_t)plane * (2 * D + 1);  // stride of one component
  const cpx<T>* src = in + (size_t)G.src * 3 * NZ * plane + q;
  cpx<T> v[3][NZ];
#pragma unroll
  for (int l = 0; l < NZ; ++l)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a][l] = src[(size_t)(a * NZ + l) * plane];
  cpx<T> o[3][NT];
#pragma unroll
  for (int k = 0; k < NT; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a][k] = mk<T>(0, 0);
  const int ncomp = mode == 0 ? 6 : 3;
  // e = k - l + NZ - 1 runs over the layer offsets dz = tz0 - NZ + 1 + e
#pragma unroll
  for (int e = 0; e < NT + NZ - 1; ++e) {
    if (e < G.ntz + NZ - 1) {
      const T* K = kern + (size_t)(G.tz0 - NZ + 1 + e + D) * plane + q;
      T kv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) kv[c] = c < ncomp ? K[c * ks] : T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const int k = e - (NZ - 1) + l;
        if (k >= 0 && k < NT && k < G.ntz) slab_mac<T>(mode, kv, v[0][l], v[1][l], v[2][l], o[0][k], o[1][k], o[2][k]);
      }
    }
  }
  const cpx<T> ph = slab_phase<T>(kx, ky, G.xs * rigid->s_int + G.xoff, G.yoff, Lx, Ly, sgn);
  cpx<T>* dst = out + G.out + q;
#pragma unroll
  for (int k = 0; k < NT; ++k)
    if (k < G.ntz)
#pragma unroll
      for (int a = 0; a < 3; ++a) dst[(size_t)(a * G.ntz + k) * plane] = cmul(o[a][k], ph);
}

// Kernel spectra: kern[(comp * ndz + dz + D) * Ly * Kx + ky * Kx + kx], one
// real number per point: tensor components xx yy zz xy (real spectra) and
// xz yz (imaginary, value = i * stored); S components x, y (imaginary) and z
// (real).  Grid: (points / SLAB_THREADS, groups, target layers): one
// thread per spectral point and target layer.
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_mul(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const T* __restrict__ kern, SlabMulTable tab,
               int nz, int D, int Lx, int Ly, int Kx, int mode, T sgn, const RigidState* __restrict__ rigid) {
  const int plane = Ly * Kx;
  const int q = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (q >= plane) return;
  const SlabGroup G = tab.g[blockIdx.y];
  const int k = blockIdx.z;
  if (k >= G.ntz) return;
  const int ky = q / Kx, kx = q - ky * Kx;
  const size_t ks = (size_t)plane * (2 * D + 1);  // stride of one component
  const cpx<T>* src = in + (size_t)G.src * 3 * nz * plane + q;
  cpx<T>* dst = out + G.out + q;
  {
    const int t = G.tz0 + k;
    cpx<T> o0 = mk<T>(0, 0), o1 = mk<T>(0, 0), o2 = mk<T>(0, 0);
    const int ncomp = mode == 0 ? 6 : 3;
    for (int l = 0; l < nz; ++l) {
      const T* K = kern + (size_t)(t - l + D) * plane + q;
      T kv[6];
      for (int c = 0; c < 6; ++c) kv[c] = c < ncomp ? K[c * ks] : T(0);
      slab_mac<T>(mode, kv, src[(size_t)(0 * nz + l) * plane], src[(size_t)(1 * nz + l) * plane],
                  src[(size_t)(2 * nz + l) * plane], o0, o1, o2);
    }
    const cpx<T> ph = slab_phase<T>(kx, ky, G.xs * rigid->s_int + G.xoff, G.yoff, Lx, Ly, sgn);
    dst[(size_t)(0 * G.ntz + k) * plane] = cmul(o0, ph);
    dst[(size_t)(1 * G.ntz + k) * plane] = cmul(o1, ph);
    dst[(size_t)(2 * G.ntz + k) * plane] = cmul(o2, ph);
  }
}

// Scalar-potential product (Eqs. 7-8): phi_t = sgn * sum_l S(t - l) . mhat_l
// with S = (i sx, i sy, sz), one channel per target layer; the same groups,
// phases and kernel layout as k_slab_mul.  Grid: (points / SLAB_THREADS,
// groups, target layers).
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_pot(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const T* __restrict__ kern, SlabMulTable tab,
               int nz, int D, int Lx, int Ly, int Kx, T sgn, const RigidState* __restrict__ rigid) {
  const int plane = Ly * Kx;
  const int q = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (q >= plane) return;
  const SlabGroup G = tab.g[blockIdx.y];
  const int k = blockIdx.z;
  if (k >= G.ntz) return;
  const int ky = q / Kx, kx = q - ky * Kx;
  const size_t ks = (size_t)plane * (2 * D + 1);
  const cpx<T>* src = in + (size_t)G.src * 3 * nz * plane + q;
  const int t = G.tz0 + k;
  cpx<T> o = mk<T>(0, 0);
  for (int l = 0; l < nz; ++l) {
    const T* K = kern + (size_t)(t - l + D) * plane + q;
    const T sx = K[0], sy = K[ks], sz = K[2 * ks];
    const cpx<T> v0 = src[(size_t)(0 * nz + l) * plane], v1 = src[(size_t)(1 * nz + l) * plane],
                 v2 = src[(size_t)(2 * nz + l) * plane];
    const cpx<T> a = scale(v0, sx) + scale(v1, sy);
    o = o + mk<T>(-a.y, a.x) + scale(v2, sz);
  }
  out[G.out + (size_t)k * plane + q] = cmul(o, slab_phase<T>(kx, ky, G.xs * rigid->s_int + G.xoff, G.yoff, Lx, Ly, sgn));
}

// H = -grad phi by four-point central differences (Sec. III.A) on an output
// box [3][ol][oy][ox] from a sampled potential P[pl][py][px]: output point
// (l, j, i) sits at P[l + o0][j + o0][i + o0] (o0 >= 2).  add: out += H.
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_potgrad(const T* __restrict__ P, int py, int px, int o0, int ol, int oy, int ox, T* __restrict__ out,
                   int add, T c12x, T c12y, T c12z) {
  const int n = ol * oy * ox;
  const int id = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (id >= n) return;
  const int i = id % ox, j = (id / ox) % oy, l = id / (ox * oy);
  const size_t sy = px, sz = (size_t)px * py;
  const T* p = P + (size_t)(l + o0) * sz + (size_t)(j + o0) * sy + (i + o0);
  auto d4 = [&](size_t s) { return (p[-2 * (long long)s] - T(8) * p[-(long long)s] + T(8) * p[s] - p[2 * s]); };
  const T hx = -d4(1) * c12x, hy = -d4(sy) * c12y, hz = -d4(sz) * c12z;
  T* o = out + id;
  const size_t N = (size_t)n;
  if (add) {
    o[0] += hx;
    o[N] += hy;
    o[2 * N] += hz;
  } else {
    o[0] = hx;
    o[N] = hy;
    o[2 * N] = hz;
  }
}

// Whole-sample mirror index of k into [0, M) (M >= 2).
__device__ __forceinline__ int slab_reflect(int k, int M) {
  if (k >= 0 && k < M) return k;
  const int P = 2 * M - 2;
  k %= P;
  if (k < 0) k += P;
  return k > M - 1 ? P - k : k;
}

// Window rows -> out[nch][nrow][nw] at u = i + h + sgn * x_p, i = i0 .. i0 +
// nw - 1, x_p = x_s / dx - s_int of the current stage.  Output row r (in
// blocks of R.orows) reads input row (r + R.roff) mod R.wrows of the same
// block (R.nrow_in input rows per channel); its window is the M elements
// from column c0 = R.cs * s_int + R.c_off of that row (ld apart), taken
// modulo R.period when it is set (a periodic x: the row holds one period).
// interp 0: cubic B-spline; its coefficients solve the mirror-bounded
// system (c_{k-1} + 4 c_k + c_{k+1}) / 6 = f_k, i.e. the symmetric filter
// sqrt(3) z^|j| (z = sqrt(3) - 2) on the mirror-periodic extension of the
// row, truncated at |j| <= KF where |z|^KF is below the precision.
// interp 1: linear interpolation of the samples.  One block per row; the
// row is staged in LDS with its mirror images KF samples past each end, so
// the filter taps index it directly.
constexpr int SLAB_KF_MAX = 30;
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_sample(const T* __restrict__ win, SlabRows R, int h, T* __restrict__ out, int i0, int nw, int sgn, int add,
                  int interp, double inv_dx, const RigidState* __restrict__ rigid) {
  constexpr int KF = sizeof(T) == 8 ? 30 : 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  static_assert(KF <= SLAB_KF_MAX, "LDS sized for SLAB_KF_MAX");
  const int nch = R.nch, nrow = R.nrow, M = R.M;
  const int ME = M + 2 * KF;
  T* fe = reinterpret_cast<T*>(smem_raw);  // [3][M + 2 KF]: f_{k - KF}, mirror-extended
  T* c = fe + 3 * ME;                       // [3][M]
  __shared__ T w[KF + 1];
  const int r = blockIdx.x;
  if (r >= nrow) return;
  if (threadIdx.x <= KF) w[threadIdx.x] = (T)(1.7320508075688772935 * pow(1.7320508075688772935 - 2.0, (double)threadIdx.x));
  const int blk = r / R.orows;
  int ri = (r - blk * R.orows + R.roff) % R.wrows;
  if (ri < 0) ri += R.wrows;
  const int rin = blk * R.wrows + ri;
  const int c0 = R.cs * rigid->s_int + R.c_off;
  for (int t = threadIdx.x; t < nch * ME; t += SLAB_THREADS) {
    const int a = t / ME, k = t - a * ME - KF;
    int col = c0 + slab_reflect(k, M);
    if (R.period > 0) {
      col %= R.period;
      if (col < 0) col += R.period;
    }
    fe[t] = win[((size_t)a * R.nrow_in + rin) * R.ld + col];
  }
  __syncthreads();
  const T* src = fe + KF;
  int stride = ME;
  if (interp == 0) {
    for (int t = threadIdx.x; t < nch * M; t += SLAB_THREADS) {
      const int a = t / M, k = t - a * M;
      const T* fa = fe + a * ME + KF + k;
      T s = w[0] * fa[0];
#pragma unroll
      for (int j = 1; j <= KF; ++j) s += w[j] * (fa[j] + fa[-j]);
      c[t] = s;
    }
    __syncthreads();
    src = c;
    stride = M;
  }
  const double xp = sgn * (rigid->xs * inv_dx - (double)rigid->s_int);
  const double fl = floor(xp);
  const int k0 = (int)fl + h;
  const T tt = (T)(xp - fl);
  T wb[4];
  if (interp == 0) {
    const T u = T(1) - tt;
    wb[0] = u * u * u / T(6);
    wb[1] = T(2) / T(3) - tt * tt + T(0.5) * tt * tt * tt;
    wb[2] = T(2) / T(3) - u * u + T(0.5) * u * u * u;
    wb[3] = tt * tt * tt / T(6);
  } else {
    wb[0] = T(0);
    wb[1] = T(1) - tt;
    wb[2] = tt;
    wb[3] = T(0);
  }
  for (int t = threadIdx.x; t < nch * nw; t += SLAB_THREADS) {
    const int a = t / nw, o = t - a * nw;
    const int k = k0 + i0 + o;
    const T* sa = src + a * stride;
    const T v = wb[0] * sa[slab_reflect(k - 1, M)] + wb[1] * sa[slab_reflect(k, M)] +
                wb[2] * sa[slab_reflect(k + 1, M)] + wb[3] * sa[slab_reflect(k + 2, M)];
    T* d = out + ((size_t)a * nrow + r) * nw + o;
    *d = add ? *d + v : v;
  }
}

// Stencil G[3][nz+2][ny+2][nx+2]: the base field at window layer t (slider
// layer t - 1), row y (lattice row y - 1), point i (slider column i - 1).
// Per slider cell: the centre value is added to hd (when add), and the force
// density (m . grad) H with two-point central differences is summed in
// float64; block b writes its sums to part[3 b .. 3 b + 2].
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_force(const T* __restrict__ G, const T* __restrict__ m, T* __restrict__ hd, int nx, int ny, int nz, int add,
                 double i2dx, double i2dy, double i2dz, double* __restrict__ part) {
  __shared__ double red[3][SLAB_THREADS / 64];
  const int N = nx * ny * nz;
  const int id = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  double F0 = 0.0, F1 = 0.0, F2 = 0.0;
  if (id < N) {
    const int i = id % nx, j = (id / nx) % ny, l = id / (nx * ny);
    const int W = nx + 2, Hh = ny + 2, Zl = nz + 2;
    auto at = [&](int a, int t, int y, int x) { return G[(((size_t)a * Zl + t) * Hh + y) * W + x]; };
    const double mx = m[id], my = m[N + id], mz = m[2 * N + id];
    double Fa[3];
    for (int a = 0; a < 3; ++a) {
      const T cv = at(a, l + 1, j + 1, i + 1);
      if (add) hd[(size_t)a * N + id] += cv;
      const double gx = ((double)at(a, l + 1, j + 1, i + 2) - (double)at(a, l + 1, j + 1, i)) * i2dx;
      const double gy = ((double)at(a, l + 1, j + 2, i + 1) - (double)at(a, l + 1, j, i + 1)) * i2dy;
      const double gz = ((double)at(a, l + 2, j + 1, i + 1) - (double)at(a, l, j + 1, i + 1)) * i2dz;
      Fa[a] = mx * gx + my * gy + mz * gz;
    }
    F0 = Fa[0];
    F1 = Fa[1];
    F2 = Fa[2];
  }
  F0 = wave_sum(F0);
  F1 = wave_sum(F1);
  F2 = wave_sum(F2);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = F0;
    red[1][wv] = F1;
    red[2][wv] = F2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int k = 0; k < SLAB_THREADS / 64; ++k) s += red[threadIdx.x][k];
    part[3 * (size_t)blockIdx.x + threadIdx.x] = s;
  }
}

// dst[i] += src[i]
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS) k_slab_add(int n, const T* __restrict__ src, T* __restrict__ dst) {
  const int i = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (i < n) dst[i] += src[i];
}

// Per element id of [film][3][ncell]: B = mu0 (hd + hext_c + Ms m) in
// float64, bdot = (B - Bprev) / dt (zero on the first update), Bprev = B.
template <typename T>
__global__ void __launch_bounds__(SLAB_THREADS)
    k_slab_bdot(int n, int ncell, const T* __restrict__ hd, const T* __restrict__ m, double hx, double hy, double hz,
                double mu0, double Ms, double idt, int first, double* __restrict__ Bprev, T* __restrict__ bdot) {
  const int id = (int)(blockIdx.x * SLAB_THREADS + threadIdx.x);
  if (id >= n) return;
  const int c = (id / ncell) % 3;
  const double he = c == 0 ? hx : (c == 1 ? hy : hz);
  const double B = mu0 * ((double)hd[id] + he + Ms * (double)m[id]);
  bdot[id] = first ? T(0) : (T)((B - Bprev[id]) * idt);
  Bprev[id] = B;
}

// ------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_slab_pack(const void* spec, T* out, int n, int imag, hipStream_t st) {
  hipLaunchKernelGGL(k_slab_pack<T>, dim3((n + SLAB_THREADS - 1) / SLAB_THREADS), dim3(SLAB_THREADS), 0, st,
                     (const cpx<double>*)spec, out, n, imag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slab_mul(const void* in, void* out, const T* kern, const SlabMulTable& tab, int nz, int D, int Lx,
                           int Ly, int Kx, int mode, double sgn, const RigidState* rigid, hipStream_t st) {
  const int plane = Ly * Kx;
  int ntz = 1;
  for (int g = 0; g < tab.n; ++g) {
    ntz = tab.g[g].ntz > ntz ? tab.g[g].ntz : ntz;
    if (tab.g[g].ntz > nz + 2) return hipErrorInvalidValue;  // the register form holds nz + 2 target layers
  }
  const dim3 grid2((plane + SLAB_THREADS - 1) / SLAB_THREADS, tab.n);
#define MMV_SLAB_MUL_NZ(N)                                                                                      \
  case N:                                                                                                       \
    hipLaunchKernelGGL((k_slab_mul_nz<T, N>), grid2, dim3(SLAB_THREADS), 0, st, (const cpx<T>*)in, (cpx<T>*)out, \
                       kern, tab, D, Lx, Ly, Kx, mode, (T)sgn, rigid);                                          \
    return hipGetLastError();
  switch (nz) {
    MMV_SLAB_MUL_NZ(2)
    MMV_SLAB_MUL_NZ(3)
    MMV_SLAB_MUL_NZ(4)
    MMV_SLAB_MUL_NZ(5)
    MMV_SLAB_MUL_NZ(6)
    MMV_SLAB_MUL_NZ(7)
    MMV_SLAB_MUL_NZ(8)
    default: break;
  }
#undef MMV_SLAB_MUL_NZ
  dim3 grid((plane + SLAB_THREADS - 1) / SLAB_THREADS, tab.n, ntz);
  hipLaunchKernelGGL(k_slab_mul<T>, grid, dim3(SLAB_THREADS), 0, st, (const cpx<T>*)in, (cpx<T>*)out, kern, tab, nz,
                     D, Lx, Ly, Kx, mode, (T)sgn, rigid);
  return hipGetLastError();
}

size_t slab_sample_lds(int M, int esz) { return ((size_t)6 * M + 6 * SLAB_KF_MAX) * esz; }

template <typename T>
hipError_t launch_slab_sample(const T* win, const SlabRows& R, int h, T* out, int i0, int nw, int sgn, int add,
                              int interp, double inv_dx, const RigidState* rigid, hipStream_t st) {
  const size_t lds = slab_sample_lds(R.M, sizeof(T));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_slab_sample<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_slab_sample<T>, dim3(R.nrow), dim3(SLAB_THREADS), lds, st, win, R, h, out, i0, nw, sgn, add,
                     interp, inv_dx, rigid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slab_pot(const void* in, void* out, const T* kern, const SlabMulTable& tab, int nz, int D, int Lx,
                           int Ly, int Kx, double sgn, const RigidState* rigid, hipStream_t st) {
  const int plane = Ly * Kx;
  int ntz = 1;
  for (int g = 0; g < tab.n; ++g) ntz = tab.g[g].ntz > ntz ? tab.g[g].ntz : ntz;
  dim3 grid((plane + SLAB_THREADS - 1) / SLAB_THREADS, tab.n, ntz);
  hipLaunchKernelGGL(k_slab_pot<T>, grid, dim3(SLAB_THREADS), 0, st, (const cpx<T>*)in, (cpx<T>*)out, kern, tab, nz, D,
                     Lx, Ly, Kx, (T)sgn, rigid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slab_potgrad(const T* P, int py, int px, int o0, int ol, int oy, int ox, T* out, int add, double dx,
                               double dy, double dz, hipStream_t st) {
  const int n = ol * oy * ox;
  hipLaunchKernelGGL(k_slab_potgrad<T>, dim3((n + SLAB_THREADS - 1) / SLAB_THREADS), dim3(SLAB_THREADS), 0, st, P, py,
                     px, o0, ol, oy, ox, out, add, (T)(1.0 / (12.0 * dx)), (T)(1.0 / (12.0 * dy)),
                     (T)(1.0 / (12.0 * dz)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slab_add(int n, const T* src, T* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_slab_add<T>, dim3((n + SLAB_THREADS - 1) / SLAB_THREADS), dim3(SLAB_THREADS), 0, st, n, src,
                     dst);
  return hipGetLastError();
}

int slab_force_blocks(int ncell) { return (ncell + SLAB_THREADS - 1) / SLAB_THREADS; }

template <typename T>
hipError_t launch_slab_force(const T* G, const T* m, T* hd, int nx, int ny, int nz, int add, double dx, double dy,
                             double dz, double* part, hipStream_t st) {
  const int nb = slab_force_blocks(nx * ny * nz);
  hipLaunchKernelGGL(k_slab_force<T>, dim3(nb), dim3(SLAB_THREADS), 0, st, G, m, hd, nx, ny, nz, add,
                     0.5 / dx, 0.5 / dy, 0.5 / dz, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slab_bdot(int n, int ncell, const T* hd, const T* m, const double hext[3], double mu0, double Ms,
                            double idt, int first, double* Bprev, T* bdot, hipStream_t st) {
  hipLaunchKernelGGL(k_slab_bdot<T>, dim3((n + SLAB_THREADS - 1) / SLAB_THREADS), dim3(SLAB_THREADS), 0, st, n,
                     ncell, hd, m, hext[0], hext[1], hext[2], mu0, Ms, idt, first, Bprev, bdot);
  return hipGetLastError();
}

#define MMV_SLAB_INST(T)                                                                                        \
  template hipError_t launch_slab_pack<T>(const void*, T*, int, int, hipStream_t);                              \
  template hipError_t launch_slab_mul<T>(const void*, void*, const T*, const SlabMulTable&, int, int, int, int,  \
                                         int, int, double, const RigidState*, hipStream_t);                    \
  template hipError_t launch_slab_sample<T>(const T*, const SlabRows&, int, T*, int, int, int, int, int, double, \
                                            const RigidState*, hipStream_t);                                    \
  template hipError_t launch_slab_pot<T>(const void*, void*, const T*, const SlabMulTable&, int, int, int, int,  \
                                         int, double, const RigidState*, hipStream_t);                          \
  template hipError_t launch_slab_potgrad<T>(const T*, int, int, int, int, int, int, T*, int, double, double,    \
                                             double, hipStream_t);                                              \
  template hipError_t launch_slab_add<T>(int, const T*, T*, hipStream_t);                                       \
  template hipError_t launch_slab_force<T>(const T*, const T*, T*, int, int, int, int, double, double, double,   \
                                           double*, hipStream_t);                                               \
  template hipError_t launch_slab_bdot<T>(int, int, const T*, const T*, const double*, double, double, double,  \
                                          int, double*, T*, hipStream_t);

MMV_SLAB_INST(float)
MMV_SLAB_INST(double)

}  // namespace mmv
