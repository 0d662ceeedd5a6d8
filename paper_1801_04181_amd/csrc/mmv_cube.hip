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
//   k_bdot, k_sor_rhs, k_sor_tile, k_current, k_sum_*, k_shift
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
  // the column groups of one plane share cache lines: keep them on one XCD
  const int lb = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int by = lb / gridDim.x;
  const int c0 = (lb - by * gridDim.x) * CB;
  if (c0 >= ncols) return;
  const int nc = min(CB, ncols - c0);
  const long long p = by;
  const cpx<T>* src = in + p * in_ps + c0;
  cpx<T>* dst = out + p * out_ps + c0;
  for (int t = threadIdx.x; t < L; t += CUBE_THREADS) stw[t] = tw[t];
  const float inc = 1.0f / (float)nc;
  stage_move<4, CUBE_THREADS>(
      nc * L,
      [&](int t) {
        const int r = fdiv(t, inc);
        return r < n_in ? src[(size_t)r * ncols + (t - r * nc)] : mk<T>(0, 0);
      },
      [&](int t, cpx<T> v) {
        const int r = fdiv(t, inc);
        A[(t - r * nc) * L + r] = v;
      });
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
// IP: Lz of 64 or 128 points, transformed in place (one LDS buffer, at most
// ZMUL_IP_CB pencils per block); else ping-pong buffers.
constexpr int ZMUL_IP_CB = 5;

template <typename T, bool IP>
__global__ void __launch_bounds__(CUBE_THREADS)
    k_zmul(cpx<T>* __restrict__ buf, const T* __restrict__ kern, int Kx, int Ly, int nz, int CB, int mode,
           T sgn, FftPlan P, const cpx<T>* __restrict__ twz) {
  // logical block b (XCD-remapped): the CB pencils q = ky * Kx + kx from
  // b * CB (fewer in the last block); pencil q of plane z sits at
  // z * Ly * Kx + q
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int Lz = P.L;
  const int Kyh = Ly / 2 + 1, Kzh = Lz / 2 + 1;
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = stw + Lz;
  cpx<T>* B = IP ? A : A + (size_t)3 * CB * Lz;
  const int ncol = Ly * Kx;
  // neighbouring pencil groups share cache lines: keep them on one XCD
  const int q0 = xcd_remap(blockIdx.x, gridDim.x) * CB;
  if (q0 >= ncol) return;
  const int nc = min(CB, ncol - q0);
  const long long zs = ncol, cs = (long long)nz * ncol;  // plane and channel strides
  for (int t = threadIdx.x; t < Lz; t += CUBE_THREADS) stw[t] = twz[t];
  const float inc = 1.0f / (float)nc;
  stage_move<4, CUBE_THREADS>(
      3 * nz * nc,
      [&](int t) {
        const int cz = fdiv(t, inc);  // c * nz + z
        const int c = cz / nz, z = cz - c * nz;
        return buf[c * cs + z * zs + q0 + (t - cz * nc)];
      },
      [&](int t, cpx<T> v) {
        const int cz = fdiv(t, inc);
        const int c = cz / nz, z = cz - c * nz;
        A[(c * nc + t - cz * nc) * Lz + z] = v;
      });
  for (int t = threadIdx.x; t < 3 * nc * (Lz - nz); t += CUBE_THREADS) {
    const int b = t / (Lz - nz), z = nz + t - b * (Lz - nz);
    A[b * Lz + z] = mk<T>(0, 0);
  }
  lds_barrier();
  cpx<T>* X = A;
  if constexpr (IP) {
    if (Lz == 128)
      fft_inplace<T, 128, CUBE_THREADS, false, 3 * ZMUL_IP_CB>(A, 3 * nc, stw);
    else
      fft_inplace<T, 64, CUBE_THREADS, false, 3 * ZMUL_IP_CB>(A, 3 * nc, stw);
  } else {
    X = fft_lds_pow2<T, false, CUBE_THREADS>(A, B, P, 3 * nc, Lz, stw);
  }
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
  cpx<T>* Y = X;
  if constexpr (IP) {
    if (Lz == 128)
      fft_inplace<T, 128, CUBE_THREADS, true, 3 * ZMUL_IP_CB>(X, 3 * nc, stw);
    else
      fft_inplace<T, 64, CUBE_THREADS, true, 3 * ZMUL_IP_CB>(X, 3 * nc, stw);
  } else {
    Y = fft_lds_pow2<T, true, CUBE_THREADS>(X, (X == A) ? B : A, P, 3 * nc, Lz, stw);
  }
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
  stage_copy<4, CUBE_THREADS>(a, nb * N2x, [&](int t) {
    const int r = fdiv(t, ink);
    const int k = t - r * N2x;
    const cpx<T>* X = spec + (size_t)(row0 + r) * Kx;
    cpx<T> xk = X[k];
    cpx<T> xm = X[N2x - k];
    xm.y = -xm.y;
    cpx<T> s = xk + xm;
    cpx<T> d = cmulc(xk - xm, stp[k]);
    return mk<T>(s.x - d.y, s.y + d.x);
  });
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
  int pbc;  // periodic x (bit 0) and y (bit 1) neighbours in the exchange
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
             const T* __restrict__ hd, const T* __restrict__ he, T* __restrict__ hout, int* __restrict__ flags,
             RigidState* tick, T* __restrict__ dmstep) {
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  // the step's clock (time, step count) advances with its last stage
  if (tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
    tick->t0 = tick->t0 + p.dt;
    tick->ts = tick->t0;
    tick->step += 1;
  }
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
    if (p.pbc & 1) {
      add(id - i + (i == 0 ? p.nx - 1 : i - 1), ix2);
      add(id - i + (i == p.nx - 1 ? 0 : i + 1), ix2);
    } else {
      if (i > 0) add(id - sx, ix2);
      if (i < p.nx - 1) add(id + sx, ix2);
    }
    if (p.pbc & 2) {
      const size_t row0 = id - (size_t)j * sy;
      add(row0 + (size_t)(j == 0 ? p.ny - 1 : j - 1) * sy, iy2);
      add(row0 + (size_t)(j == p.ny - 1 ? 0 : j + 1) * sy, iy2);
    } else {
      if (j > 0) add(id - sy, iy2);
      if (j < p.ny - 1) add(id + sy, iy2);
    }
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
    const T ix = c * (acc[id] + kx), iy = c * (acc[N + id] + ky), iz = c * (acc[2 * N + id] + kz);
    const T nx_ = ox + ix, ny_ = oy + iy, nz_ = oz + iz;
    const T nrm = sqrt(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
    if (!(nrm > T(0)) || !isfinite(nrm)) atomicOr(flags, (int)FLAG_NUMERIC);
    mnext[id] = nx_ / nrm;
    mnext[N + id] = ny_ / nrm;
    mnext[2 * N + id] = nz_ / nrm;
    if (dmstep != nullptr) {
      // the step's change of m, normalise(m + inc) - m for a unit m, formed
      // from the increment (no difference of two rounded states):
      // q = |m + inc|^2 - 1 = 2 m.inc + |inc|^2, 1/|m + inc| - 1 = -q / (s (1 + s))
      const T q = T(2) * (ox * ix + oy * iy + oz * iz) + (ix * ix + iy * iy + iz * iz);
      const T sn = sqrt(T(1) + q);
      const T rm1 = -q / (sn * (T(1) + sn));
      const T r = T(1) + rm1;
      dmstep[id] = ix * r + ox * rm1;
      dmstep[N + id] = iy * r + oy * rm1;
      dmstep[2 * N + id] = iz * r + oz * rm1;
    }
  }
  }
}

// dB/dt over the last step.  B = mu0 (H_d + H_ext + Ms m) with H_d linear in
// m and H_ext constant, so B_n - B_{n-1} = mu0 (H_d(dm) + Ms dm) for the
// step's change dm: bdot = mu0 (hdm + Ms dm) / dt (zero on the first update).
// bdot may alias hdm.
template <typename T>
__global__ void k_bdot(size_t N, const T* dm, const T* hdm, T* bdot, double mu0, double Ms, double idt, int first) {
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x)
    for (int a = 0; a < 3; ++a) {
      const size_t q = a * N + id;
      bdot[q] = first ? T(0) : (T)(mu0 * ((double)hdm[q] + Ms * (double)dm[q]) * idt);
    }
}

// Right-hand side of sum_interior (phi_j - phi_i)/d^2 = r_i (surface faces
// carry the normal component of E_sol; a periodic in-plane axis, pbc bit 0 =
// x, 1 = y, has no surface), plus per-block partial sums.
template <typename T>
__global__ void __launch_bounds__(256)
    k_sor_rhs(int nx, int ny, int nz, double dx, double dy, double dz, int pbc, const T* __restrict__ es,
              T* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[256];
  const size_t N = (size_t)nx * ny * nz;
  double acc = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    int i, j, k;
    cell_ijk(id, nx, ny, i, j, k);
    const double ex = es[id], ey = es[N + id], ez = es[2 * N + id];
    if (!(pbc & 1)) {
      if (i == nx - 1) v -= ex / dx;
      if (i == 0) v += ex / dx;
    }
    if (!(pbc & 2)) {
      if (j == ny - 1) v -= ey / dy;
      if (j == 0) v += ey / dy;
    }
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

// dst = src - mean (src may be dst)
template <typename T>
__global__ void k_shift(size_t N, const T* src, T* dst, const double* __restrict__ mean) {
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x)
    dst[id] = (T)((double)src[id] - *mean);
}

// Residual of the Neumann problem after the sweeps: per cell
// res_i = sum over interior faces (phi_j - phi_i) / d^2 - r_i (faces through
// a periodic axis' period included); each block writes its float64 sums of
// res^2 and r^2 (part[2 b], part[2 b + 1]).
template <typename T>
__global__ void __launch_bounds__(256)
    k_sor_residual(int nx, int ny, int nz, double dx, double dy, double dz, int pbc, const T* __restrict__ phi,
                   const T* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[2][256];
  const size_t N = (size_t)nx * ny * nz;
  const double wx = 1.0 / (dx * dx), wy = 1.0 / (dy * dy), wz = 1.0 / (dz * dz);
  double a = 0.0, b = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(id, nx, ny, i, j, k);
    const double p = phi[id];
    double s = 0.0;
    const size_t rx = (size_t)(nx - 1), ry = (size_t)(ny - 1) * nx;  // a period's wrap
    if (i > 0) s += wx * ((double)phi[id - 1] - p);
    else if (pbc & 1) s += wx * ((double)phi[id + rx] - p);
    if (i < nx - 1) s += wx * ((double)phi[id + 1] - p);
    else if (pbc & 1) s += wx * ((double)phi[id - rx] - p);
    if (j > 0) s += wy * ((double)phi[id - nx] - p);
    else if (pbc & 2) s += wy * ((double)phi[id + ry] - p);
    if (j < ny - 1) s += wy * ((double)phi[id + nx] - p);
    else if (pbc & 2) s += wy * ((double)phi[id - ry] - p);
    if (k > 0) s += wz * ((double)phi[id - (size_t)nx * ny] - p);
    if (k < nz - 1) s += wz * ((double)phi[id + (size_t)nx * ny] - p);
    const double res = s - (double)r[id];
    a += res * res;
    b += (double)r[id] * (double)r[id];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

// Red-black SOR sweeps (colour = (i + j + k) mod 2, red = 0 first) on 3-D
// tiles.  A cell's update is
//   phi <- (1 - omega) phi + omega (sum_nb w_nb phi_nb - r) / sum_nb w_nb
// over its face neighbours inside the mesh (w = 1/d^2 of the axis; a mesh
// face contributes nothing, the Neumann condition being in r); all cells of
// one colour update from the other colour's values, so the order within a
// half-sweep does not matter.  Along a periodic in-plane axis (even period)
// the box holds the wrapped cells, which update like interior ones.
constexpr int SOR_THREADS = 256;
constexpr int SOR_T = 8;                    // tile edge
constexpr int SOR_S = 2;                    // sweeps per launch at most
constexpr int SOR_H = 2 * SOR_S;            // halo
constexpr int SOR_D = SOR_T + 2 * SOR_H;    // loaded box edge

// One half-sweep of `colour` over the centred E^3 region of the LDS box
// (E even).  Every neighbour of the region lies in the box.  A thread
// computes all of its new values before storing any: the half-sweep reads
// only the other colour and each updated cell's own old value.
template <typename T, int E, int PBC>
__device__ __forceinline__ void sor_half(T* sp, const T* sr, int colour, int ox, int oy, int oz, int nx, int ny,
                                         int nz, T wx, T wy, T wz, T om) {
  constexpr int D = SOR_D, D2 = D * D, O = (SOR_D - E) / 2, EH = E / 2;
  constexpr int NC = E * E * E / 2, NU = (NC + SOR_THREADS - 1) / SOR_THREADS;
  static_assert(E % 2 == 0 && O >= 1, "the region and its neighbours lie in the box");
  T val[NU];
  int cell[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = (int)threadIdx.x + u * SOR_THREADS;
    const int row = t / EH, xh = t - row * EH;
    const int lj = O + row % E, lk = O + row / E;
    const int j = oy + lj, k = oz + lk;
    const int li = O + 2 * xh + ((colour - ox - O - j - k) & 1);
    const int i = ox + li;
    constexpr bool px = (PBC & 1) != 0, py = (PBC & 2) != 0;
    const bool upd = t < NC && (px || (i >= 0 && i < nx)) && (py || (j >= 0 && j < ny)) && k >= 0 && k < nz;
    const bool x0 = px || i > 0, x1 = px || i < nx - 1, y0 = py || j > 0, y1 = py || j < ny - 1, z0 = k > 0,
               z1 = k < nz - 1;
    const int c = upd ? lk * D2 + lj * D + li : D2 + D + 1;  // an in-box cell for the lanes past the region
    const T px0 = sp[c - 1], px1 = sp[c + 1], py0 = sp[c - D], py1 = sp[c + D], pz0 = sp[c - D2],
            pz1 = sp[c + D2], pc = sp[c], rc = sr[c];
    // absent neighbours enter with weight 0 (s + 0 * 0 and w + 0 are exact)
    T s = 0, w = 0;
    s = fma(x0 ? px0 : T(0), x0 ? wx : T(0), s);
    w += x0 ? wx : T(0);
    s = fma(x1 ? px1 : T(0), x1 ? wx : T(0), s);
    w += x1 ? wx : T(0);
    s = fma(y0 ? py0 : T(0), y0 ? wy : T(0), s);
    w += y0 ? wy : T(0);
    s = fma(y1 ? py1 : T(0), y1 ? wy : T(0), s);
    w += y1 ? wy : T(0);
    s = fma(z0 ? pz0 : T(0), z0 ? wz : T(0), s);
    w += z0 ? wz : T(0);
    s = fma(z1 ? pz1 : T(0), z1 ? wz : T(0), s);
    w += z1 ? wz : T(0);
    const bool ok = upd && w != T(0);
    val[u] = (T(1) - om) * pc + om * ((s - rc) / (ok ? w : T(1)));
    cell[u] = ok ? c : -1;
  }
#pragma unroll
  for (int u = 0; u < NU; ++u)
    if (cell[u] >= 0) sp[cell[u]] = val[u];
  lds_barrier();
}

// Half-sweeps HS .. 2 NSW - 1 of a launch: half-sweep h updates the region
// of edge SOR_T + 2 (2 NSW - 1 - h), the cells the tile still depends on,
// which reads the region of half-sweep h - 1 (the whole box for h = 0).
template <typename T, int NSW, int HS, int PBC>
__device__ __forceinline__ void sor_halves(T* sp, const T* sr, int ox, int oy, int oz, int nx, int ny, int nz, T wx,
                                           T wy, T wz, T om) {
  if constexpr (HS < 2 * NSW) {
    sor_half<T, SOR_T + 2 * (2 * NSW - 1 - HS), PBC>(sp, sr, HS & 1, ox, oy, oz, nx, ny, nz, wx, wy, wz, om);
    sor_halves<T, NSW, HS + 1, PBC>(sp, sr, ox, oy, oz, nx, ny, nz, wx, wy, wz, om);
  }
}

// NSW <= SOR_S sweeps in one launch.  Tile (bx, by, bz) loads the box of
// the 8^3 tile of cells from (8 bx, 8 by, 8 bz) with a halo of 2 SOR_S
// cells (the parts inside the mesh) from pin into LDS, runs the 2 NSW
// half-sweeps there and writes the tile's cells (those inside the mesh) to
// pout, as global half-sweeps would leave them.  Several independent meshes
// of the same size (consecutive, bstride cells apart) share a launch: grid z
// runs over tz tiles of each mesh in turn.  A periodic axis (pbc) loads the
// box's cells past the mesh from the other side of the period (PBC: the
// periodic axes, bit 0 = x, 1 = y, fixed at compile time so that the open
// mesh's sweep carries no wrap arithmetic).
template <typename T, int NSW, int PBC>
__global__ void __launch_bounds__(SOR_THREADS)
    k_sor_tile(int nx, int ny, int nz, double dx, double dy, double dz, const T* __restrict__ pin,
               T* __restrict__ pout, const T* __restrict__ r, double omega, int tz, size_t bstride) {
  static_assert(NSW >= 1 && NSW <= SOR_S, "the halo covers the half-sweeps");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int D = SOR_D, D2 = D * D, D3 = D * D * D;
  T* sp = reinterpret_cast<T*>(smem_raw);
  T* sr = sp + D3;
  // neighbouring tiles share halo cells: consecutive tiles (x fastest, then
  // y, z) go to one XCD
  const int gx = gridDim.x, gy = gridDim.y;
  const int lb = xcd_remap((blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x, gx * gy * gridDim.z);
  const int bzb = lb / (gx * gy), byx = lb - bzb * gx * gy, by = byx / gx, bx = byx - by * gx;
  const int box = bzb / tz, bz = bzb - box * tz;
  pin += box * bstride;
  pout += box * bstride;
  r += box * bstride;
  const int ox = bx * SOR_T - SOR_H, oy = by * SOR_T - SOR_H, oz = bz * SOR_T - SOR_H;
  const size_t sy = nx, sz = (size_t)nx * ny;
  // all of a thread's loads in flight before the first LDS store
  constexpr int NL = D3 / SOR_THREADS;
  static_assert(NL * SOR_THREADS == D3, "the box is a whole number of block passes");
  T vp[NL], vr[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int t = (int)threadIdx.x + u * SOR_THREADS;
    const int li = t % D, lj = (t / D) % D, lk = t / D2;
    int i = ox + li, j = oy + lj;
    const int k = oz + lk;
    if constexpr ((PBC & 1) != 0) i = ((i % nx) + nx) % nx;
    if constexpr ((PBC & 2) != 0) j = ((j % ny) + ny) % ny;
    vp[u] = vr[u] = T(0);
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) {
      const size_t id = (size_t)k * sz + (size_t)j * sy + i;
      vp[u] = pin[id];
      vr[u] = r[id];
    }
  }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int t = (int)threadIdx.x + u * SOR_THREADS;
    sp[t] = vp[u];
    sr[t] = vr[u];
  }
  lds_barrier();
  const T wx = T(1.0 / (dx * dx)), wy = T(1.0 / (dy * dy)), wz = T(1.0 / (dz * dz));
  sor_halves<T, NSW, 0, PBC>(sp, sr, ox, oy, oz, nx, ny, nz, wx, wy, wz, (T)omega);
  for (int t = threadIdx.x; t < SOR_T * SOR_T * SOR_T; t += SOR_THREADS) {
    const int li = SOR_H + t % SOR_T, lj = SOR_H + (t / SOR_T) % SOR_T, lk = SOR_H + t / (SOR_T * SOR_T);
    const int i = ox + li, j = oy + lj, k = oz + lk;
    if (i < nx && j < ny && k < nz) pout[(size_t)k * sz + (size_t)j * sy + i] = sp[lk * D2 + lj * D + li];
  }
}

// ------------------------------------------------------------ exact Neumann solve
// The finite-volume Neumann Laplacian of a box is diagonal in the cosine
// basis cos(pi k (i + 1/2) / n) per axis, eigenvalue sum over axes of
// (2 cos(pi k / n) - 2) / d^2.  Cosine transforms along one axis of
// [nbox][nz][ny][nx] arrays take an n-point complex FFT of the reordered
// line (Makhoul, IEEE Trans. ASSP 28, 27, 1980): the DCT-II
// C_k = sum_i x_i cos(pi k (2 i + 1) / (2 n)) = Re(exp(-i pi k / (2 n)) V_k)
// with V = DFT(v), v_p = x_{2p}, v_{n-1-p} = x_{2p+1}; the inverse builds
// V_k = exp(i pi k / (2 n)) (C_k - i C_{n-k}) (C_n = 0) and v = IDFT(V).
// A periodic in-plane axis (pbc) has no faces at its ends: its Laplacian is
// the symmetric circulant one, diagonal in the Hartley basis
// cas(2 pi k i / n) = cos + sin with eigenvalue (2 cos(2 pi k / n) - 2) / d^2
// (cas k and cas n - k span the Fourier pair of one eigenvalue).  The real
// Hartley transform H_k = Re X_k - Im X_k of X = DFT(x), and x = (Re Y +
// Im Y) / n of Y = IDFT(H), keep the line real like the cosine one.
// Line l of a launch: element i at (l / inner) hs + l % inner + i es.
// SOLVE (the last forward axis, z): C / lambda(kx, ky, kz), the k = 0 mode
// (the gauge) set to zero.
struct DctSolve {
  int nx, ny;
  double idx2, idy2, idz2;
  int pbc;  // periodic x (bit 0) and y (bit 1): Hartley eigenvalues there
};

template <typename T, bool INV, bool SOLVE>
__global__ void __launch_bounds__(CUBE_THREADS)
    k_dct_axis(const T* __restrict__ in, T* __restrict__ out, int nlines, int n, int inner, long long hs,
               long long es, int CB, FftPlan P, const cpx<T>* __restrict__ tw, DctSolve sv, int hart) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = stw + n;
  cpx<T>* B = A + (size_t)CB * n;
  const int l0 = xcd_remap(blockIdx.x, gridDim.x) * CB;
  if (l0 >= nlines) return;
  const int nc = min(CB, nlines - l0);
  for (int t = threadIdx.x; t < n; t += CUBE_THREADS) stw[t] = tw[t];
  // element (c, i) of thread slot t: along the line for contiguous lines,
  // across lines otherwise (coalesced either way)
  auto slot = [&](int t, int& c, int& i) {
    if (es == 1) {
      c = t / n;
      i = t - c * n;
    } else {
      i = t / nc;
      c = t - i * nc;
    }
  };
  auto addr = [&](int c, int i) {
    const int l = l0 + c;
    return (long long)(l / inner) * hs + (l % inner) + (long long)i * es;
  };
  if constexpr (!INV) {
    for (int t = threadIdx.x; t < nc * n; t += CUBE_THREADS) {
      int c, i;
      slot(t, c, i);
      const int p = hart ? i : ((i & 1) ? n - 1 - (i >> 1) : (i >> 1));
      A[c * n + p] = mk<T>(in[addr(c, i)], T(0));
    }
  } else if (hart) {
    for (int t = threadIdx.x; t < nc * n; t += CUBE_THREADS) {
      int c, i;
      slot(t, c, i);
      A[c * n + i] = mk<T>(in[addr(c, i)], T(0));
    }
  } else {
    T* Cs = reinterpret_cast<T*>(B);
    for (int t = threadIdx.x; t < nc * n; t += CUBE_THREADS) {
      int c, i;
      slot(t, c, i);
      Cs[c * n + i] = in[addr(c, i)];
    }
    lds_barrier();
    for (int t = threadIdx.x; t < nc * n; t += CUBE_THREADS) {
      const int c = t / n, k = t - c * n;
      const T ck = Cs[c * n + k], cm = k ? Cs[c * n + n - k] : T(0);
      T sn, cs;
      if constexpr (sizeof(T) == 8)
        sincospi((double)k / (2.0 * n), &sn, &cs);
      else
        sincospif((float)k / (2.0f * (float)n), &sn, &cs);
      A[t] = mk<T>(ck * cs + cm * sn, ck * sn - cm * cs);
    }
  }
  lds_barrier();
  const cpx<T>* R = fft_lds_pow2<T, INV, CUBE_THREADS>(A, B, P, nc, n, stw);
  for (int t = threadIdx.x; t < nc * n; t += CUBE_THREADS) {
    int c, i;
    slot(t, c, i);
    T v;
    if constexpr (!INV) {
      const cpx<T> V = R[c * n + i];
      if (hart) {
        v = V.x - V.y;
      } else {
        T sn, cs;
        if constexpr (sizeof(T) == 8)
          sincospi((double)i / (2.0 * n), &sn, &cs);
        else
          sincospif((float)i / (2.0f * (float)n), &sn, &cs);
        v = V.x * cs + V.y * sn;
      }
      if constexpr (SOLVE) {
        const int lo = (l0 + c) % inner;
        const int ky = lo / sv.nx, kx = lo - ky * sv.nx;
        const double fx = (sv.pbc & 1) ? 2.0 : 1.0, fy = (sv.pbc & 2) ? 2.0 : 1.0;
        const double lam = (2.0 * cospi(fx * kx / sv.nx) - 2.0) * sv.idx2 +
                           (2.0 * cospi(fy * ky / sv.ny) - 2.0) * sv.idy2 +
                           (2.0 * cospi((double)i / n) - 2.0) * sv.idz2;
        v = (kx == 0 && ky == 0 && i == 0) ? T(0) : (T)((double)v / lam);
      }
    } else if (hart) {
      v = (R[c * n + i].x + R[c * n + i].y) / (T)n;
    } else {
      const int p = (i & 1) ? n - 1 - (i >> 1) : (i >> 1);
      v = R[c * n + p].x / (T)n;
    }
    out[addr(c, i)] = v;
  }
}

// J = sigma (E_sol + E_irrot), E_irrot,a = -(g+ + g-)/2, surface faces take
// E_sol,a; along a periodic axis (pbc) the faces through the period are
// interior ones.
template <typename T>
__global__ void k_current(int nx, int ny, int nz, double dx, double dy, double dz, int pbc,
                          const T* __restrict__ phi, const T* __restrict__ es, T* __restrict__ J, double sigma) {
  const size_t N = (size_t)nx * ny * nz;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (size_t)gridDim.x * blockDim.x) {
  int i, j, k;
  cell_ijk(id, nx, ny, i, j, k);
  const int idx[3] = {i, j, k};
  const int n[3] = {nx, ny, nz};
  const size_t st[3] = {1, (size_t)nx, (size_t)nx * ny};
  const double d[3] = {dx, dy, dz};
  const bool per[3] = {(pbc & 1) != 0, (pbc & 2) != 0, false};
  for (int a = 0; a < 3; ++a) {
    const T e = es[a * N + id];
    const size_t wrap = (size_t)(n[a] - 1) * st[a];
    const size_t up = idx[a] < n[a] - 1 ? id + st[a] : id - wrap, dn = idx[a] > 0 ? id - st[a] : id + wrap;
    const T gp = (idx[a] < n[a] - 1 || per[a]) ? (phi[up] - phi[id]) / (T)d[a] : e;
    const T gm = (idx[a] > 0 || per[a]) ? (phi[id] - phi[dn]) / (T)d[a] : e;
    J[a * N + id] = (T)sigma * (e - T(0.5) * (gp + gm));
  }
  }
}

// Time and step count of a mesh without a moving magnet.
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
  // 64 or 128 points: in place, ZMUL_IP_CB pencils per block in float32 and
  // 3 in float64 (one LDS buffer).  Else ping-pong buffers with at most CB
  // pencils, as many as the CU's LDS holds (at least one fits: the set-up
  // bounds Lz).
  const bool ip = P.L == 64 || P.L == 128;
  if (ip) CB = sizeof(T) == 4 ? ZMUL_IP_CB : 3;
  const int nbuf = ip ? 3 : 6;
  while (CB > 1 && sizeof(cpx<T>) * ((size_t)P.L + nbuf * (size_t)CB * P.L) > 160 * 1024) --CB;
  const size_t lds = sizeof(cpx<T>) * ((size_t)P.L + nbuf * (size_t)CB * P.L);
  const void* fn = ip ? (const void*)k_zmul<T, true> : (const void*)k_zmul<T, false>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((Ly * Kx + CB - 1) / CB);
  if (ip)
    hipLaunchKernelGGL((k_zmul<T, true>), grid, dim3(CUBE_THREADS), lds, st, (cpx<T>*)buf, kern, Kx, Ly, nz, CB, mode,
                       (T)sgn, P, (const cpx<T>*)twz);
  else
    hipLaunchKernelGGL((k_zmul<T, false>), grid, dim3(CUBE_THREADS), lds, st, (cpx<T>*)buf, kern, Kx, Ly, nz, CB,
                       mode, (T)sgn, P, (const cpx<T>*)twz);
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
                         T* mnext, T* acc, const T* hd, const T* he, T* hout, int* flags, RigidState* tick,
                         T* dmstep, hipStream_t st) {
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
  p.pbc = c.pbc;
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  hipLaunchKernelGGL(k_stage3<T>, grid1(N), dim3(256), 0, st, p, ms, m0, mnext, acc, hd, he, hout, flags, tick,
                     dmstep);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_eddy_bdot(size_t N, const T* dm, const T* hdm, T* bdot, double mu0, double Ms, double idt,
                            int first, hipStream_t st) {
  hipLaunchKernelGGL(k_bdot<T>, grid1(N), dim3(256), 0, st, N, dm, hdm, bdot, mu0, Ms, idt, first);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sor_rhs(const CubeLaunch& c, const T* es, T* r, double* part, double* mean, hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  const int nb = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_sor_rhs<T>, dim3(nb), dim3(256), 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.pbc, es, r,
                     part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, nb, (const double*)part, mean, 1.0 / (double)N);
  hipLaunchKernelGGL(k_shift<T>, grid1(N), dim3(256), 0, st, N, (const T*)r, r, (const double*)mean);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sor_residual(const CubeLaunch& c, const T* phi, const T* r, double* part, int nblk,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_sor_residual<T>, dim3(nblk), dim3(256), 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.pbc,
                     phi, r, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sor(const CubeLaunch& c, int nbox, T* phi, T* phi2, const T* r, double omega, int sweeps,
                      double* part, double* mean, hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  // SOR_S sweeps per launch on tiles, alternating between phi and phi2; the
  // nbox meshes (N cells apart) in one launch
  const int tz = (c.nz + SOR_T - 1) / SOR_T;
  const dim3 grid((unsigned)((c.nx + SOR_T - 1) / SOR_T), (unsigned)((c.ny + SOR_T - 1) / SOR_T),
                  (unsigned)(tz * nbox));
  const size_t lds = 2 * sizeof(T) * SOR_D * SOR_D * SOR_D;
  T* cur = phi;
  T* nxt = phi2;
  // one instantiation per sweep count and set of periodic axes
  for (int s = 0; s < sweeps; s += SOR_S) {
    const int two = sweeps - s >= 2;
#define MMV_SOR_TILE(NSW, PBC)                                                                                  \
  hipLaunchKernelGGL((k_sor_tile<T, NSW, PBC>), grid, dim3(SOR_THREADS), lds, st, c.nx, c.ny, c.nz, c.dx, c.dy, \
                     c.dz, (const T*)cur, nxt, r, omega, tz, N)
    switch ((c.pbc & 3) * 2 + two) {
      case 0: MMV_SOR_TILE(1, 0); break;
      case 1: MMV_SOR_TILE(2, 0); break;
      case 2: MMV_SOR_TILE(1, 1); break;
      case 3: MMV_SOR_TILE(2, 1); break;
      case 4: MMV_SOR_TILE(1, 2); break;
      case 5: MMV_SOR_TILE(2, 2); break;
      case 6: MMV_SOR_TILE(1, 3); break;
      default: MMV_SOR_TILE(2, 3); break;
    }
#undef MMV_SOR_TILE
    T* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  // each mesh's potential to zero mean (the reduction buffers serve the
  // meshes in turn, in stream order)
  const int nb = (int)((N + 255) / 256);
  for (int b = 0; b < nbox; ++b) {
    hipLaunchKernelGGL(k_sum_part<T>, dim3(nb), dim3(256), 0, st, N, (const T*)cur + b * N, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, nb, (const double*)part, mean, 1.0 / (double)N);
    hipLaunchKernelGGL(k_shift<T>, grid1(N), dim3(256), 0, st, N, (const T*)cur + b * N, phi + b * N,
                       (const double*)mean);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_current(const CubeLaunch& c, const T* phi, const T* es, T* J, double sigma, hipStream_t st) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  hipLaunchKernelGGL(k_current<T>, grid1(N), dim3(256), 0, st, c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.pbc, phi, es,
                     J, sigma);
  return hipGetLastError();
}


// Exact solve of the nbox Neumann problems (r -> phi, zero mean), work of
// the same size: forward x, y, z (with the division), inverse z, y, x.
template <typename T>
hipError_t launch_neumann_solve(const CubeLaunch& c, int nbox, const T* r, T* phi, T* work, const FftPlan* P,
                                const void* const* tw, hipStream_t st) {
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const long long N = (long long)nx * ny * nz;
  DctSolve sv{nx, ny, 1.0 / (c.dx * c.dx), 1.0 / (c.dy * c.dy), 1.0 / (c.dz * c.dz), c.pbc};
  struct Ax {
    int n, inner;
    long long hs, es;
    int nlines;
  };
  const Ax ax[3] = {{nx, 1, nx, 1, (int)(nbox * N / nx)},
                    {ny, nx, (long long)nx * ny, nx, (int)(nbox * N / ny)},
                    {nz, nx * ny, N, (long long)nx * ny, (int)(nbox * N / nz)}};
  auto run = [&](int a, bool inv, bool solve, const T* src, T* dst) -> hipError_t {
    const Ax& x = ax[a];
    int CB = (int)((65536 / sizeof(cpx<T>) - x.n) / (2 * (size_t)x.n));
    if (CB > 16) CB = 16;
    if (CB < 1) CB = 1;
    const size_t lds = sizeof(cpx<T>) * ((size_t)x.n + 2 * (size_t)CB * x.n);
    const void* fn = inv ? (const void*)k_dct_axis<T, true, false>
                         : (solve ? (const void*)k_dct_axis<T, false, true> : (const void*)k_dct_axis<T, false, false>);
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    const dim3 grid((x.nlines + CB - 1) / CB);
    // axes 0 (x) and 1 (y) take the Hartley transform where periodic
    const int hart = a < 2 && ((c.pbc >> a) & 1);
    if (inv)
      hipLaunchKernelGGL((k_dct_axis<T, true, false>), grid, dim3(CUBE_THREADS), lds, st, src, dst, x.nlines, x.n,
                         x.inner, x.hs, x.es, CB, P[a], (const cpx<T>*)tw[a], sv, hart);
    else if (solve)
      hipLaunchKernelGGL((k_dct_axis<T, false, true>), grid, dim3(CUBE_THREADS), lds, st, src, dst, x.nlines, x.n,
                         x.inner, x.hs, x.es, CB, P[a], (const cpx<T>*)tw[a], sv, hart);
    else
      hipLaunchKernelGGL((k_dct_axis<T, false, false>), grid, dim3(CUBE_THREADS), lds, st, src, dst, x.nlines, x.n,
                         x.inner, x.hs, x.es, CB, P[a], (const cpx<T>*)tw[a], sv, hart);
    return hipGetLastError();
  };
  hipError_t e = run(0, false, false, r, work);
  if (e == hipSuccess) e = run(1, false, false, work, phi);
  if (e == hipSuccess) e = run(2, false, true, phi, work);
  if (e == hipSuccess) e = run(2, true, false, work, phi);
  if (e == hipSuccess) e = run(1, true, false, phi, work);
  if (e == hipSuccess) e = run(0, true, false, work, phi);
  return e;
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
                                       const T*, const T*, T*, int*, RigidState*, T*, hipStream_t);               \
  template hipError_t launch_eddy_bdot<T>(size_t, const T*, const T*, T*, double, double, double, int,           \
                                          hipStream_t);                                                           \
  template hipError_t launch_sor_rhs<T>(const CubeLaunch&, const T*, T*, double*, double*, hipStream_t);         \
  template hipError_t launch_sor<T>(const CubeLaunch&, int, T*, T*, const T*, double, int, double*, double*,     \
                                     hipStream_t);                                                             \
  template hipError_t launch_current<T>(const CubeLaunch&, const T*, const T*, T*, double, hipStream_t);         \
  template hipError_t launch_sor_residual<T>(const CubeLaunch&, const T*, const T*, double*, int, hipStream_t);  \
  template hipError_t launch_neumann_solve<T>(const CubeLaunch&, int, const T*, T*, T*, const FftPlan*,          \
                                              const void* const*, hipStream_t);                                 \
  template hipError_t launch_pack3<T>(const void*, T*, int, int, int, int, hipStream_t);

MMV_CUBE_INST(float)
MMV_CUBE_INST(double)

}  // namespace mmv
