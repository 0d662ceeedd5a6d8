// HIP kernels of the single-magnet three-dimensional path: the demagnetising
// convolution of Eq. (6) on a zero-padded Lx x Ly x Lz grid and the
// eddy-current field of Sec. III.B (Eqs. 9-12).
//
//   k_fft_axis   batched column transforms along one strided axis (y or z),
//                zero-padded input rows, truncated output rows.
//   k_zmul       per (ky, kx) pencil: z transform of three channels,
//                multiplication by the tensor N (Eq. 6) or by the cross
//                product with the potential kernel S (Eqs. 9 and the
//                Biot-Savart field of J), inverse z transform.
//   k_row_inv    inverse real x transform of each row into cell values.
//   k_stage3     local terms, LLG (Eq. 1) and the RK4 stage on each cell.
//   k_bdot, k_sor_rhs, k_sor, k_current, k_sum_*, k_shift
//                B and dB/dt, the finite-volume Neumann problem for the
//                electric potential and its red-black SOR sweeps, J.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mmv_device.h"
#include "mmv_kernels.h"
#include "mmv_kernel_fn.h"

namespace mmv {

// ------------------------------------------------------------ strided column FFT
// Block size of the LDS transform kernels (used as a compile-time constant
// by the kernels and their helpers).
constexpr int CUBE_THREADS = 256;

template <typename T, bool INV>
__global__ void __launch_bounds__(CUBE_THREADS)
    k_fft_axis(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int ncols, int CB, int n_in,
               long long in_ps, int n_out, long long out_ps, FftPlan P, const cpx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = P.L;
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = stw + L;
  cpx<T>* B = A + (size_t)CB * L;
  const int c0 = blockIdx.x * CB;
  if (c0 >= ncols) return;
  const int nc = min(CB, ncols - c0);
  const long long p = blockIdx.y;
  const cpx<T>* src = in + p * in_ps + c0;
  cpx<T>* dst = out + p * out_ps + c0;
  for (int t = threadIdx.x; t < L; t += CUBE_THREADS) stw[t] = tw[t];
  const float inc = 1.0f / (float)nc;
  for (int t = threadIdx.x; t < nc * L; t += CUBE_THREADS) {
    const int r = fdiv(t, inc);
    const int c = t - r * nc;
    A[c * L + r] = r < n_in ? src[(size_t)r * ncols + c] : mk<T>(0, 0);
  }
  lds_barrier();
  const cpx<T>* R = fft_lds_pow2<T, INV, CUBE_THREADS>(A, B, P, nc, L, stw);
  for (int t = threadIdx.x; t < nc * n_out; t += CUBE_THREADS) {
    const int r = fdiv(t, inc);
    const int c = t - r * nc;
    dst[(size_t)r * ncols + c] = R[c * L + r];
  }
}

// ------------------------------------------------------------ z pencils with the kernel
// Kernel spectra are stored for kx < Kx, ky <= Ly/2, kz <= Lz/2 as one real
// number (all tensor components have real spectra, all S components
// imaginary); the other half follows from the parity in y and z.
// mode 0: out_a = sum_b N_ab v_b (six components xx yy zz xy xz yz)
// mode 1: out = sgn * S x v (components Sx Sy Sz)
template <typename T>
__global__ void __launch_bounds__(CUBE_THREADS)
    k_zmul(cpx<T>* __restrict__ buf, const T* __restrict__ kern, int Kx, int Ly, int nz, int CB, int mode,
           T sgn, FftPlan P, const cpx<T>* __restrict__ twz) {
  // block b: the CB pencils q = ky * Kx + kx from b * CB (fewer in the last
  // block); pencil q of plane z sits at z * Ly * Kx + q
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int Lz = P.L;
  const int Kyh = Ly / 2 + 1, Kzh = Lz / 2 + 1;
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = stw + Lz;
  cpx<T>* B = A + (size_t)3 * CB * Lz;
  const int ncol = Ly * Kx;
  const int q0 = blockIdx.x * CB;
  if (q0 >= ncol) return;
  const int nc = min(CB, ncol - q0);
  const long long zs = ncol, cs = (long long)nz * ncol;  // plane and channel strides
  for (int t = threadIdx.x; t < Lz; t += CUBE_THREADS) stw[t] = twz[t];
  const float inc = 1.0f / (float)nc;
  for (int t = threadIdx.x; t < 3 * nz * nc; t += CUBE_THREADS) {
    const int cz = fdiv(t, inc);  // c * nz + z
    const int cc = t - cz * nc;
    const int c = cz / nz, z = cz - c * nz;
    A[(c * nc + cc) * Lz + z] = buf[c * cs + z * zs + q0 + cc];
  }
  for (int t = threadIdx.x; t < 3 * nc * (Lz - nz); t += CUBE_THREADS) {
    const int b = t / (Lz - nz), z = nz + t - b * (Lz - nz);
    A[b * Lz + z] = mk<T>(0, 0);
  }
  lds_barrier();
  cpx<T>* X = fft_lds_pow2<T, false, CUBE_THREADS>(A, B, P, 3 * nc, Lz, stw);
  for (int t = threadIdx.x; t < nc * Lz; t += CUBE_THREADS) {
    const int cc = t / Lz, kz = t - cc * Lz;
    const int ky = (q0 + cc) / Kx, kx = q0 + cc - ky * Kx;
    const bool yup = ky >= Kyh;
    const int kyr = yup ? Ly - ky : ky;
    const bool zup = kz >= Kzh;
    const int kzr = zup ? Lz - kz : kz;
    const size_t kb = (((size_t)kx * Kyh + kyr) * Kzh + kzr);
    const size_t ks = (size_t)Kx * Kyh * Kzh;
    cpx<T> v0 = X[(0 * nc + cc) * Lz + kz], v1 = X[(1 * nc + cc) * Lz + kz], v2 = X[(2 * nc + cc) * Lz + kz];
    cpx<T> o0, o1, o2;
    if (mode == 0) {
      // parities (x, y, z): xx yy zz even; xy (1,1,0); xz (1,0,1); yz (0,1,1)
      const T nxx = kern[0 * ks + kb], nyy = kern[1 * ks + kb], nzz = kern[2 * ks + kb];
      const T nxy = kern[3 * ks + kb] * T(yup ? -1 : 1);
      const T nxz = kern[4 * ks + kb] * T(zup ? -1 : 1);
      const T nyz = kern[5 * ks + kb] * T((yup != zup) ? -1 : 1);
      o0 = scale(v0, nxx) + scale(v1, nxy) + scale(v2, nxz);
      o1 = scale(v0, nxy) + scale(v1, nyy) + scale(v2, nyz);
      o2 = scale(v0, nxz) + scale(v1, nyz) + scale(v2, nzz);
    } else {
      // S_x odd in x, S_y odd in y, S_z odd in z: spectra i * stored
      const T sx = kern[0 * ks + kb] * sgn;
      const T sy = kern[1 * ks + kb] * sgn * T(yup ? -1 : 1);
      const T sz = kern[2 * ks + kb] * sgn * T(zup ? -1 : 1);
      // (S x v) with S = i s: i * (s x v)
      const cpx<T> c0 = scale(v2, sy) - scale(v1, sz);
      const cpx<T> c1 = scale(v0, sz) - scale(v2, sx);
      const cpx<T> c2 = scale(v1, sx) - scale(v0, sy);
      o0 = mk<T>(-c0.y, c0.x);
      o1 = mk<T>(-c1.y, c1.x);
      o2 = mk<T>(-c2.y, c2.x);
    }
    X[(0 * nc + cc) * Lz + kz] = o0;
    X[(1 * nc + cc) * Lz + kz] = o1;
    X[(2 * nc + cc) * Lz + kz] = o2;
  }
  lds_barrier();
  cpx<T>* Y = fft_lds_pow2<T, true, CUBE_THREADS>(X, (X == A) ? B : A, P, 3 * nc, Lz, stw);
  for (int t = threadIdx.x; t < 3 * nz * nc; t += CUBE_THREADS) {
    const int cz = fdiv(t, inc);
    const int cc = t - cz * nc;
    const int c = cz / nz, z = cz - c * nz;
    buf[c * cs + z * zs + q0 + cc] = Y[(c * nc + cc) * Lz + z];
  }
}

// ------------------------------------------------------------ inverse x transform
// Block b turns the R consecutive spectrum rows from b * R (fewer in the
// last block) into cell values.
template <typename T>
__global__ void __launch_bounds__(CUBE_THREADS)
    k_row_inv(const cpx<T>* __restrict__ spec, T* __restrict__ out, int nrows, int R, int nx, int N2x, int Kx,
              FftPlan P, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* stp = stw + N2x;
  cpx<T>* a = stp + N2x + 1;
  cpx<T>* b = a + (size_t)R * N2x;
  const int row0 = (int)blockIdx.x * R;
  if (row0 >= nrows) return;
  const int nb = min(R, nrows - row0);
  for (int t = threadIdx.x; t < N2x; t += CUBE_THREADS) stw[t] = tw[t];
  for (int t = threadIdx.x; t <= N2x; t += CUBE_THREADS) stp[t] = twp[t];
  lds_barrier();
  const float ink = 1.0f / (float)N2x;
  for (int t = threadIdx.x; t < nb * N2x; t += CUBE_THREADS) {
    const int r = fdiv(t, ink);
    const int k = t - r * N2x;
    const cpx<T>* X = spec + (size_t)(row0 + r) * Kx;
    cpx<T> xk = X[k];
    cpx<T> xm = X[N2x - k];
    xm.y = -xm.y;
    cpx<T> s = xk + xm;
    cpx<T> d = cmulc(xk - xm, stp[k]);
    a[t] = mk<T>(s.x - d.y, s.y + d.x);
  }
  lds_barrier();
  const T* xr = reinterpret_cast<const T*>(fft_lds_pow2<T, true, CUBE_THREADS>(a, b, P, nb, N2x, stw));
  const float inx = 1.0f / (float)nx;
  for (int t = threadIdx.x; t < nb * nx; t += CUBE_THREADS) {
    const int r = fdiv(t, inx);
    const int i = t - r * nx;
    out[(size_t)(row0 + r) * nx + i] = xr[(size_t)r * 2 * N2x + i];
  }
}

// ------------------------------------------------------------ cell kernels
struct CubeParams {
  int nx, ny, nz;
  int mode;  // MODE_EVAL or MODE_STAGE
  int stage;
  int term_mask;
  double dx, dy, dz;
  double pref_ex, pref_an, u[3], hext[3], gam, alpha, dt;
};

// (i, j, k) of cell id on an nx x ny x nz grid of fewer than 2^31 cells
// (checked at set-up), in 32-bit arithmetic.
__device__ __forceinline__ void cell_ijk(size_t id, int nx, int ny, int& i, int& j, int& k) {
  const unsigned u = (unsigned)id, unx = (unsigned)nx, uny = (unsigned)ny;
  const unsigned q = u / unx;
  i = (int)(u - q * unx);
  k = (int)(q / uny);
  j = (int)(q - (unsigned)k * uny);
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_stage3(CubeParams p, const T* __restrict__ ms, const T* m0, T* mnext, T* __restrict__ acc,
             const T* __restrict__ hd, const T* __restrict__ he, T* __restrict__ hout, int* __restrict__ flags) {
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
  int i, j, k;
  cell_ijk(id, p.nx, p.ny, i, j, k);
  const T mx = ms[id], my = ms[N + id], mz = ms[2 * N + id];
  T hx = 0, hy = 0, hz = 0;
  if (p.term_mask & 8) {
    hx += hd[id];
    hy += hd[N + id];
    hz += hd[2 * N + id];
  }
  if (p.term_mask & 32) {
    hx += he[id];
    hy += he[N + id];
    hz += he[2 * N + id];
  }
  if (p.term_mask & 1) {
    T ex = 0, ey = 0, ez = 0;
    const T ix2 = T(1.0 / (p.dx * p.dx)), iy2 = T(1.0 / (p.dy * p.dy)), iz2 = T(1.0 / (p.dz * p.dz));
    const size_t sx = 1, sy = p.nx, sz = (size_t)p.nx * p.ny;
    auto add = [&](size_t nb, T w) {
      ex += (ms[nb] - mx) * w;
      ey += (ms[N + nb] - my) * w;
      ez += (ms[2 * N + nb] - mz) * w;
    };
    if (i > 0) add(id - sx, ix2);
    if (i < p.nx - 1) add(id + sx, ix2);
    if (j > 0) add(id - sy, iy2);
    if (j < p.ny - 1) add(id + sy, iy2);
    if (k > 0) add(id - sz, iz2);
    if (k < p.nz - 1) add(id + sz, iz2);
    hx += (T)p.pref_ex * ex;
    hy += (T)p.pref_ex * ey;
    hz += (T)p.pref_ex * ez;
  }
  if (p.term_mask & 2) {
    const T mu = mx * (T)p.u[0] + my * (T)p.u[1] + mz * (T)p.u[2];
    hx += (T)p.pref_an * mu * (T)p.u[0];
    hy += (T)p.pref_an * mu * (T)p.u[1];
    hz += (T)p.pref_an * mu * (T)p.u[2];
  }
  if (p.term_mask & 4) {
    hx += (T)p.hext[0];
    hy += (T)p.hext[1];
    hz += (T)p.hext[2];
  }
  if (p.mode == MODE_EVAL) {
    hout[id] = hx;
    hout[N + id] = hy;
    hout[2 * N + id] = hz;
    continue;
  }
  const T gam = (T)p.gam, alp = (T)p.alpha, h = (T)p.dt;
  const T cx = my * hz - mz * hy, cy = mz * hx - mx * hz, cz = mx * hy - my * hx;
  const T dx_ = my * cz - mz * cy, dy_ = mz * cx - mx * cz, dz_ = mx * cy - my * cx;
  const T kx = -gam * (cx + alp * dx_), ky = -gam * (cy + alp * dy_), kz = -gam * (cz + alp * dz_);
  const T ox = m0[id], oy = m0[N + id], oz = m0[2 * N + id];
  if (p.stage == 0) {
    acc[id] = kx;
    acc[N + id] = ky;
    acc[2 * N + id] = kz;
    mnext[id] = ox + T(0.5) * h * kx;
    mnext[N + id] = oy + T(0.5) * h * ky;
    mnext[2 * N + id] = oz + T(0.5) * h * kz;
  } else if (p.stage < 3) {
    acc[id] += T(2) * kx;
    acc[N + id] += T(2) * ky;
    acc[2 * N + id] += T(2) * kz;
    const T c = p.stage == 1 ? T(0.5) * h : h;
    mnext[id] = ox + c * kx;
    mnext[N + id] = oy + c * ky;
    mnext[2 * N + id] = oz + c * kz;
  } else {
    const T c = h / T(6);
    const T nx_ = ox + c * (acc[id] + kx), ny_ = oy + c * (acc[N + id] + ky), nz_ = oz + c * (acc[2 * N + id] + kz);
    const T nrm = sqrt(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
    if (!(nrm > T(0)) || !isfinite(nrm)) atomicOr(flags, (int)FLAG_NUMERIC);
    mnext[id] = nx_ / nrm;
    mnext[N + id] = ny_ / nrm;
    mnext[2 * N + id] = nz_ / nrm;
  }
  }
}

// B = mu0 (H_d + H_ext + Ms m); dB/dt = (B - B_prev) / dt (zero on the first
// update); B_prev = B.
template <typename T>
__global__ void k_bdot(size_t N, const T* __restrict__ m, const T* __restrict__ hd, T* __restrict__ bprev,
                       T* __restrict__ bdot, double mu0, double Ms, double h0, double h1, double h2, double idt,
                       int first) {
  const double he[3] = {h0, h1, h2};
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x)
    for (int a = 0; a < 3; ++a) {
      const size_t q = a * N + id;
      const T B = (T)(mu0 * ((double)hd[q] + he[a] + Ms * (double)m[q]));
      bdot[q] = first ? T(0) : (B - bprev[q]) * (T)idt;
      bprev[q] = B;
    }
}

// Right-hand side of sum_interior (phi_j - phi_i)/d^2 = r_i (surface faces
// carry the normal component of E_sol), plus per-block partial sums.
template <typename T>
__global__ void __launch_bounds__(256)
    k_sor_rhs(int nx, int ny, int nz, double dx, double dy, double dz, const T* __restrict__ es,
              T* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[256];
  const size_t N = (size_t)nx * ny * nz;
  double acc = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    int i, j, k;
    cell_ijk(id, nx, ny, i, j, k);
    const double ex = es[id], ey = es[N + id], ez = es[2 * N + id];
    if (i == nx - 1) v -= ex / dx;
    if (i == 0) v += ex / dx;
    if (j == ny - 1) v -= ey / dy;
    if (j == 0) v += ey / dy;
    if (k == nz - 1) v -= ez / dz;
    if (k == 0) v += ez / dz;
    r[id] = (T)v;
    acc += v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Sum of an array (float64, fixed order): per-block partials, then one block.
template <typename T>
__global__ void __launch_bounds__(256) k_sum_part(size_t N, const T* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x)
    acc += (double)x[id];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_final(int n, const double* __restrict__ part, double* __restrict__ mean,
                                                   double inv_count) {
  __shared__ double red[256];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) s += part[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mean = red[0] * inv_count;
}

template <typename T>
__global__ void k_shift(size_t N, T* __restrict__ x, const double* __restrict__ mean) {
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x)
    x[id] = (T)((double)x[id] - *mean);
}

// One colour of a red-black SOR sweep (colour = (i + j + k) mod 2).
template <typename T>
__global__ void __launch_bounds__(256)
    k_sor(int nx, int ny, int nz, double dx, double dy, double dz, T* __restrict__ phi,
          const T* __restrict__ r, double omega, int colour) {
  // thread (x, y) owns the x-th cell of this colour in row (j = y, k):
  // i = 2 x + ((colour + j + k) & 1), no index division (the launch covers
  // every cell with one pass of the strided loops)
  const int k = blockIdx.z;
  const int nxh = (nx + 1) / 2;
  const T wx = T(1.0 / (dx * dx)), wy = T(1.0 / (dy * dy)), wz = T(1.0 / (dz * dz));
  const size_t sy = nx, sz = (size_t)nx * ny;
  for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < ny; j += gridDim.y * blockDim.y)
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < nxh; x += gridDim.x * blockDim.x) {
      const int i = 2 * x + ((colour + j + k) & 1);
      if (i >= nx) continue;
      const size_t id = (size_t)k * sz + (size_t)j * sy + i;
      T s = 0, w = 0;
      if (i > 0) { s += phi[id - 1] * wx; w += wx; }
      if (i < nx - 1) { s += phi[id + 1] * wx; w += wx; }
      if (j > 0) { s += phi[id - sy] * wy; w += wy; }
      if (j < ny - 1) { s += phi[id + sy] * wy; w += wy; }
      if (k > 0) { s += phi[id - sz] * wz; w += wz; }
      if (k < nz - 1) { s += phi[id + sz] * wz; w += wz; }
      if (w == T(0)) continue;
      const T upd = (s - r[id]) / w;
      phi[id] = (T(1) - (T)omega) * phi[id] + (T)omega * upd;
    }
}

// J = sigma (E_sol + E_irrot), E_irrot,a = -(g+ + g-)/2, surface faces take E_sol,a.
template <typename T>
__global__ void k_current(int nx, int ny, int nz, double dx, double dy, double dz, const T* __restrict__ phi,
                          const T* __restrict__ es, T* __restrict__ J, double sigma) {
  const size_t N = (size_t)nx * ny * nz;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
  int i, j, k;
  cell_ijk(id, nx, ny, i, j, k);
  const int idx[3] = {i, j, k};
  const int n[3] = {nx, ny, nz};
  const size_t st[3] = {1, (size_t)nx, (size_t)nx * ny};
  const double d[3] = {dx, dy, dz};
  for (int a = 0; a < 3; ++a) {
    const T e = es[a * N + id];
    const T gp = idx[a] < n[a] - 1 ? (phi[id + st[a]] - phi[id]) / (T)d[a] : e;
    const T gm = idx[a] > 0 ? (phi[id] - phi[id - st[a]]) / (T)d[a] : e;
    J[a * N + id] = (T)sigma * (e - T(0.5) * (gp + gm));
  }
  }
}

// Time and step count of a mesh without a moving magnet.
__global__ void k_rigid_tick(RigidState* R, double dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    R->t0 = R->t0 + dt;
    R->ts = R->t0;
    R->step += 1;
  }
}

// ------------------------------------------------------------ kernel construction (float64)
__global__ void k_kernel_real3(double* __restrict__ out, int Lx, int Ly, int Lz, int kind, int comp, double dx,
                               double dy, double dz, double rc, double scale) {
  const int ry = blockIdx.y, rz = blockIdx.z;
  const int iy = ry <= Ly / 2 ? ry : ry - Ly;
  const int iz = rz <= Lz / 2 ? rz : rz - Lz;
  for (int rx = blockIdx.x * blockDim.x + threadIdx.x; rx < Lx; rx += gridDim.x * blockDim.x) {
    const int ix = rx <= Lx / 2 ? rx : rx - Lx;
    int ox, oy, oz;
    double v;
    if (kind == 0) {
      const int px[6] = {0, 0, 0, 1, 1, 0}, py[6] = {0, 0, 0, 1, 0, 1}, pz[6] = {0, 0, 0, 0, 1, 1};
      ox = px[comp];
      oy = py[comp];
      oz = pz[comp];
      v = tensor_comp(comp, ix * dx, iy * dy, iz * dz, dx, dy, dz, rc);
    } else {
      ox = comp == 0;
      oy = comp == 1;
      oz = comp == 2;
      v = s_comp(comp, ix * dx, iy * dy, iz * dz, dx, dy, dz);
    }
    if ((Lx % 2 == 0 && rx == Lx / 2 && ox) || (Ly % 2 == 0 && ry == Ly / 2 && oy) ||
        (Lz % 2 == 0 && rz == Lz / 2 && oz))
      v = 0.0;
    out[((size_t)rz * Ly + ry) * Lx + rx] = scale * v;
  }
}

// spectrum [Lz][Ly][Kx] (complex float64) -> stored [Kx][Ly/2+1][Lz/2+1]
template <typename T>
__global__ void k_pack3(const cpx<double>* __restrict__ spec, T* __restrict__ out, int Kx, int Ly, int Lz,
                        int imag) {
  const int Kyh = Ly / 2 + 1, Kzh = Lz / 2 + 1;
  const size_t n = (size_t)Kx * Kyh * Kzh;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
    const int kz = id % Kzh;
    const int ky = (id / Kzh) % Kyh;
    const int kx = id / ((size_t)Kzh * Kyh);
    const cpx<double> v = spec[((size_t)kz * Ly + ky) * Kx + kx];
    out[id] = (T)(imag ? v.y : v.x);
  }
}

// ------------------------------------------------------------ launchers
static inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <typename T>
hipError_t launch_fft_axis(const void* in, void* out, int nplanes, int ncols, int CB, int n_in, long long in_ps,
                           int n_out, long long out_ps, const FftPlan& P, const void* tw, bool inv, hipStream_t st) {
  if (CB <= 0) {
    CB = (int)((65536 / sizeof(cpx<T>) - P.L) / (2 * (size_t)P.L));
    if (CB > 16) CB = 16;
    if (CB < 1) CB = 1;
    const int nblk = (ncols + CB - 1) / CB;  // spread the columns evenly over the blocks
    CB = (ncols + nblk - 1) / nblk;
  }
  const size_t lds = sizeof(cpx<T>) * ((size_t)P.L + 2 * (size_t)CB * P.L);
  if (lds > 65536) {  // one column per block past 64 KB (the set-up bounds L so that it fits)
    hipError_t e = inv ? hipFuncSetAttribute((const void*)k_fft_axis<T, true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                       : hipFuncSetAttribute((const void*)k_fft_axis<T, false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((ncols + CB - 1) / CB, nplanes);
  if (inv)
    hipLaunchKernelGGL((k_fft_axis<T, true>), grid, dim3(CUBE_THREADS), lds, st, (const cpx<T>*)in, (cpx<T>*)out, ncols, CB,
                       n_in, in_ps, n_out, out_ps, P, (const cpx<T>*)tw);
  else
    hipLaunchKernelGGL((k_fft_axis<T, false>), grid, dim3(CUBE_THREADS), lds, st, (const cpx<T>*)in, (cpx<T>*)out, ncols, CB,
                       n_in, in_ps, n_out, out_ps, P, (const cpx<T>*)tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zmul(void* buf, const T* kern, int Kx, int Ly, int nz, int CB, int mode, double sgn,
                       const FftPlan& P, const void* twz, hipStream_t st) {
  // columns per block: at most CB, as many as the CU's LDS holds (at least
  // one fits: the set-up bounds Lz)
  while (CB > 1 && sizeof(cpx<T>) * ((size_t)P.L + 6 * (size_t)CB * P.L) > 160 * 1024) --CB;
  const size_t lds = sizeof(cpx<T>) * ((size_t)P.L + 6 * (size_t)CB * P.L);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_zmul<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((Ly * Kx + CB - 1) / CB);
  hipLaunchKernelGGL(k_zmul<T>, grid, dim3(CUBE_THREADS), lds, st, (cpx<T>*)buf, kern, Kx, Ly, nz, CB, mode, (T)sgn, P,
                     (const cpx<T>*)twz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_inv(const void* spec, T* out, int nrows, int R, int nx, int N2x, int Kx, const FftPlan& P,
                          const void* tw, const void* twp, hipStream_t st) {
  const size_t lds = sizeof(cpx<T>) * (2 * (size_t)N2x + 1 + 2 * (size_t)R * N2x);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_row_inv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_row_inv<T>, dim3((nrows + R - 1) / R), dim3(CUBE_THREADS), lds, st, (const cpx<T>*)spec, out,
                     nrows, R, nx, N2x, Kx, P, (const cpx<T>*)tw, (const cpx<T>*)twp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage3(const CubeLaunch& c, int mode, int stage, int mask, double dt, const T* ms, const T* m0,
                         T* mnext, T* acc, const T* hd, const T* he, T* hout, int* flags, hipStream_t st) {
  CubeParams p;
  p.nx = c.nx;
  p.ny = c.ny;
  p.nz = c.nz;
  p.mode = mode;
  p.stage = stage;
  p.term_mask = mask;
  p.dx = c.dx;
  p.dy = c.dy;
  p.dz = c.dz;
  p.pref_ex = c.pref_ex;
  p.pref_an = c.pref_an;
  for (int i = 0; i < 3; ++i) {
    p.u[i] = c.u[i];
    p.hext[i] = c.hext[i];
  }
  p.gam = c.gam;
  p.alpha = c.alpha;
  p.dt = dt;
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  hipLaunchKernelGGL(k_stage3<T>, grid1(N), dim3(256), 0, st, p, ms, m0, mnext, acc, hd, he, hout, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_eddy_bdot(size_t N, const T* m, const T* hd, T* bprev, T* bdot, double mu0, double Ms,
                            const double* hext, double idt, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_bdot<T>, grid1(N), dim3(256), 0, st, N, m, hd, bprev, bdot, mu0, Ms, hext[0], hext[1],
                     hext[2], idt, first);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sor_rhs(const CubeLaunch& c, const T* es, T* r, double* part, double* mean, hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  const int nb = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_sor_rhs<T>, dim3(nb), dim3(256), 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, es, r, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, nb, (const double*)part, mean, 1.0 / (double)N);
  hipLaunchKernelGGL(k_shift<T>, grid1(N), dim3(256), 0, st, N, r, (const double*)mean);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sor(const CubeLaunch& c, T* phi, const T* r, double omega, int sweeps, double* part, double* mean,
                      hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  // one thread per cell of the swept colour: rows of (nx + 1) / 2, 32 x 8
  // threads per block, one z layer per grid slice
  const dim3 blk(32, 8), grid((unsigned)(((c.nx + 1) / 2 + 31) / 32), (unsigned)((c.ny + 7) / 8), (unsigned)c.nz);
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < 2; ++col)
      hipLaunchKernelGGL(k_sor<T>, grid, blk, 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, phi, r, omega, col);
  const int nb = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_sum_part<T>, dim3(nb), dim3(256), 0, st, N, (const T*)phi, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, nb, (const double*)part, mean, 1.0 / (double)N);
  hipLaunchKernelGGL(k_shift<T>, grid1(N), dim3(256), 0, st, N, phi, (const double*)mean);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_current(const CubeLaunch& c, const T* phi, const T* es, T* J, double sigma, hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  hipLaunchKernelGGL(k_current<T>, grid1(N), dim3(256), 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, phi, es, J,
                     sigma);
  return hipGetLastError();
}

hipError_t launch_rigid_tick(RigidState* r, double dt, hipStream_t st) {
  hipLaunchKernelGGL(k_rigid_tick, dim3(1), dim3(64), 0, st, r, dt);
  return hipGetLastError();
}

hipError_t launch_kernel_real3(double* out, int Lx, int Ly, int Lz, int kind, int comp, double dx, double dy,
                               double dz, double rc, double scale, hipStream_t st) {
  dim3 grid((Lx + 127) / 128, Ly, Lz);
  hipLaunchKernelGGL(k_kernel_real3, grid, dim3(128), 0, st, out, Lx, Ly, Lz, kind, comp, dx, dy, dz, rc, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pack3(const void* spec, T* out, int Kx, int Ly, int Lz, int imag, hipStream_t st) {
  const size_t n = (size_t)Kx * (Ly / 2 + 1) * (Lz / 2 + 1);
  hipLaunchKernelGGL(k_pack3<T>, grid1(n), dim3(256), 0, st, (const cpx<double>*)spec, out, Kx, Ly, Lz, imag);
  return hipGetLastError();
}

#define MMV_CUBE_INST(T)                                                                                          \
  template hipError_t launch_fft_axis<T>(const void*, void*, int, int, int, int, long long, int, long long,       \
                                         const FftPlan&, const void*, bool, hipStream_t);                         \
  template hipError_t launch_zmul<T>(void*, const T*, int, int, int, int, int, double, const FftPlan&,           \
                                     const void*, hipStream_t);                                                   \
  template hipError_t launch_row_inv<T>(const void*, T*, int, int, int, int, int, const FftPlan&, const void*,        \
                                        const void*, hipStream_t);                                                \
  template hipError_t launch_stage3<T>(const CubeLaunch&, int, int, int, double, const T*, const T*, T*, T*,    \
                                       const T*, const T*, T*, int*, hipStream_t);                                \
  template hipError_t launch_eddy_bdot<T>(size_t, const T*, const T*, T*, T*, double, double, const double*,     \
                                          double, int, hipStream_t);                                              \
  template hipError_t launch_sor_rhs<T>(const CubeLaunch&, const T*, T*, double*, double*, hipStream_t);         \
  template hipError_t launch_sor<T>(const CubeLaunch&, T*, const T*, double, int, double*, double*, hipStream_t); \
  template hipError_t launch_current<T>(const CubeLaunch&, const T*, const T*, T*, double, hipStream_t);         \
  template hipError_t launch_pack3<T>(const void*, T*, int, int, int, int, hipStream_t);

MMV_CUBE_INST(float)
MMV_CUBE_INST(double)

}  // namespace mmv
