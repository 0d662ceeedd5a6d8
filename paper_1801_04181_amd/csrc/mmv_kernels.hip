// HIP kernels of the two-film hot path (gfx950).
//
//   k_row_fwd    forward real-to-complex transform of each row of m (the
//                x pass of the zero-padded demagnetising convolution,
//                Sec. III.A, Eq. 6), one row per block.
//   k_col        per kx column: y transform of the six magnetisation
//                channels, multiplication by the kernel spectra (tensor N of
//                Eq. 6 or potential kernel S of Eq. 8), inverse y transform
//                of each requested output channel.
//   k_row_stage  per film row: inverse x transforms, prefiltered cubic
//                B-spline sampling of the other film's field at the sub-cell
//                offset (Sec. II.A, III.A), exchange / anisotropy / Zeeman
//                terms, LLG torque (Eq. 1) and RK4 stage update, partial sums
//                of the force of Eq. (3); the last block to finish reduces the
//                partials in float64 and advances the slider (Eq. 15).
//   k_kernel_real, k_colpack
//                one-time float64 construction of the kernel spectra.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <algorithm>
#include "mmv_device.h"
#include "mmv_kernels.h"
#include "mmv_kernel_fn.h"

namespace mmv {

// Block sizes of the launches.  Kernels and their helpers use these
// compile-time values instead of blockDim.x.
constexpr int FWD_THREADS = 256;      // x pass
constexpr int COL_THREADS = 256;      // y pass (its block 0 also runs the slider tick)
constexpr int TICK_THREADS = 256;     // slider tick
constexpr int COLPACK_THREADS = 256;  // kernel-spectrum packing
static_assert(TICK_THREADS == COL_THREADS, "the y pass runs the tick with its own block");

// Rows per batch of the row kernel's transforms, at most.
constexpr int MAX_NBR = 9;

// Lengths with a compiled plan that the row kernel can transform in place
// (half the LDS of the ping-pong form).
__host__ __device__ constexpr bool inplace_length(int L) { return L == 525 || L == 270 || L == 140 || L == 72; }

// In-place batched transform of `batch` <= MAX_NBR contiguous rows of
// length P.L (one of inplace_length); returns a.
template <typename T, bool INV, int NT>
__device__ __forceinline__ cpx<T>* fft_rows_inplace(cpx<T>* a, const FftPlan& P, int batch,
                                                   const cpx<T>* __restrict__ tw) {
  switch (P.L) {
    case 525: fft_inplace<T, 525, NT, INV, MAX_NBR>(a, batch, tw); break;
    case 270: fft_inplace<T, 270, NT, INV, MAX_NBR>(a, batch, tw); break;
    case 140: fft_inplace<T, 140, NT, INV, MAX_NBR>(a, batch, tw); break;
    case 72: fft_inplace<T, 72, NT, INV, MAX_NBR>(a, batch, tw); break;
    default: break;  // the host only selects the in-place kernel for these lengths
  }
  return a;
}

// The row kernel's transforms: in place (INPL) or ping-pong between a and b.
template <typename T, bool INV, int NT, bool INPL>
__device__ __forceinline__ cpx<T>* row_fft(cpx<T>* a, cpx<T>* b, const FftPlan& P, int batch,
                                           const cpx<T>* __restrict__ tw) {
  if constexpr (INPL)
    return fft_rows_inplace<T, INV, NT>(a, P, batch, tw);
  else
    return fft_lds<T, INV, NT>(a, b, P, batch, P.L, tw);
}

// ------------------------------------------------------------ x transform
// Rows handled by one block of the x pass: `nb` rows at `row0`, `rstride`
// rows apart (the three components of one film row, or one row).  Output
// layout: tny == 0, row-major [row][Kx]; tny > 0 (film spectra), column-major
// [row / tny][Kx][row % tny], so the y pass reads each column contiguously.
// POW2: compiled transforms for 64 and 128 points (the 3-D path's rows).
template <typename T, bool POW2 = false>
__device__ __forceinline__ void row_fwd_body(int row0, int nb, int rstride, const T* __restrict__ src,
                                             cpx<T>* __restrict__ dst, int nin, int N2x, int Kx, const FftPlan& P,
                                             const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twp,
                                             int tny = 0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* stp = stw + N2x;
  cpx<T>* a = stp + N2x + 1;
  cpx<T>* b = a + (size_t)nb * N2x;
  for (int t = threadIdx.x; t < N2x; t += FWD_THREADS) stw[t] = tw[t];
  for (int t = threadIdx.x; t <= N2x; t += FWD_THREADS) stp[t] = twp[t];
  const float inv = 1.0f / (float)N2x;
  stage_copy<4, FWD_THREADS>(a, nb * N2x, [&](int t) {
    const int r = fdiv(t, inv);
    const int n = t - r * N2x;
    const T* s = src + (size_t)(row0 + r * rstride) * nin;
    const int i0 = 2 * n, i1 = 2 * n + 1;
    return mk<T>(i0 < nin ? s[i0] : T(0), i1 < nin ? s[i1] : T(0));
  });
  lds_barrier();
  // the film lengths run in place, as in the row kernel's fused forward
  // transform, so both produce the same spectra
  cpx<T>* Z = POW2 ? fft_lds_pow2<T, false, FWD_THREADS>(a, b, P, nb, N2x, stw)
              : (inplace_length(P.L) && nb <= MAX_NBR) ? fft_rows_inplace<T, false, FWD_THREADS>(a, P, nb, stw)
                                                       : fft_lds<T, false, FWD_THREADS>(a, b, P, nb, N2x, stw);
  const int K1 = N2x + 1;
  const float ink = 1.0f / (float)K1;
  for (int t = threadIdx.x; t < nb * K1; t += FWD_THREADS) {
    const int r = fdiv(t, ink);
    const int k = t - r * K1;
    const cpx<T>* z = Z + (size_t)r * N2x;
    cpx<T> zk = z[k == N2x ? 0 : k];
    cpx<T> zm = z[k == 0 ? 0 : N2x - k];
    zm.y = -zm.y;
    cpx<T> e = zk + zm;
    cpx<T> p = cmul(stp[k], zk - zm);
    const int row = row0 + r * rstride;
    const size_t o = tny > 0 ? ((size_t)(row / tny) * Kx + k) * tny + (row % tny) : (size_t)row * Kx + k;
    dst[o] = mk<T>(T(0.5) * (e.x + p.y), T(0.5) * (e.y - p.x));
  }
}

// ny3 > 0: block b transforms the x, y, z components of one film row (ny3
// rows apart); ny3 < 0: block b transforms the -ny3 consecutive rows from
// b * -ny3 (fewer in the last block); ny3 == 0: block b transforms row b.
template <typename T>
__global__ void __launch_bounds__(FWD_THREADS)
    k_row_fwd(const T* __restrict__ src, cpx<T>* __restrict__ dst, int nrows, int nin, int N2x,
              int Kx, FftPlan P, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twp, int ny3) {
  if (ny3 > 0) {
    // rows are [film][comp][y]; block = (film, y), XCD-contiguous in y so the
    // column-major writes of neighbouring rows meet in one L2
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int f = b / ny3, y = b - f * ny3;
    row_fwd_body<T>(f * 3 * ny3 + y, 3, ny3, src, dst, nin, N2x, Kx, P, tw, twp, ny3);
  } else if (ny3 < 0) {
    const int row0 = (int)blockIdx.x * -ny3;
    if (row0 >= nrows) return;
    row_fwd_body<T, true>(row0, min(-ny3, nrows - row0), 1, src, dst, nin, N2x, Kx, P, tw, twp);
  } else {
    if ((int)blockIdx.x >= nrows) return;
    row_fwd_body<T>(blockIdx.x, 1, 0, src, dst, nin, N2x, Kx, P, tw, twp);
  }
}

// Instance of a batched launch owning block b: start[i] <= b < start[i+1].
__device__ __forceinline__ int find_instance(const int* __restrict__ start, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void __launch_bounds__(FWD_THREADS) k_row_fwd_batch(const RowFwdDesc* __restrict__ d, const int* __restrict__ start,
                                                       int n) {
  const int bl = xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_instance(start, n, bl);
  const RowFwdDesc& q = d[i];
  const int b = bl - start[i];
  const int f = b / q.ny, y = b - f * q.ny;
  row_fwd_body<T>(f * 3 * q.ny + y, 3, q.ny, gptr((const T*)q.src), gptr((cpx<T>*)q.dst), q.nin, q.N2x, q.Kx, q.P,
                  gptr((const cpx<T>*)q.tw), gptr((const cpx<T>*)q.twp), q.ny);
}

// ------------------------------------------------------------ y pass
// One block per (kx column, output group): the column's nin_ch magnetisation
// spectra are y-transformed (recomputed by each group, an L2 hit), multiplied
// by the kernel spectra into the group's output channels, inverse
// y-transformed and the requested rows written.
template <typename T>
__device__ __forceinline__ void col_body(int blk, const cpx<T>* __restrict__ spec1, cpx<T>* __restrict__ spec2,
                                         const T* __restrict__ kern, int Kx, int Ly, int Kyh, int ny, int nin_ch,
                                         int ngroup, int nbuf, const FftPlan& P, const cpx<T>* __restrict__ twy,
                                         const OutTable& tab) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // twiddles: half table for even Ly (tw[t + Ly/2] = -tw[t])
  const int Lh = (Ly & 1) ? Ly : Ly / 2;
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = stw + Lh;
  cpx<T>* B = A + (size_t)nbuf * Ly;
  // this group's output channels, staged in LDS: per (output, source comp)
  // the kernel offset (kc Kx + kx) Kyh and flags, per output the source film
  __shared__ int s_koff[MAX_OUT][3];
  __shared__ unsigned char s_fl[MAX_OUT][3];
  __shared__ unsigned char s_src[MAX_OUT];
  const int kx = blk / ngroup;
  const int g = blk - kx * ngroup;
  if (kx >= Kx) return;
  const int o0 = (g * tab.n) / ngroup;
  const int o1 = ((g + 1) * tab.n) / ngroup;
  const int no = o1 - o0;
  for (int t = threadIdx.x; t < 3 * no; t += COL_THREADS) {
    const int o = t / 3, b = t - 3 * o;
    const int kc = tab.ch[o0 + o].kc[b];
    s_koff[o][b] = kc < 0 ? -1 : (kc * Kx + kx) * Kyh;
    s_fl[o][b] = tab.ch[o0 + o].fl[b];
    if (b == 0) s_src[o] = tab.ch[o0 + o].src;
  }
  for (int t = threadIdx.x; t < Lh; t += COL_THREADS) stw[t] = twy[t];
  const int nload = nin_ch * Ly;
  const float invLy = 1.0f / (float)Ly;
  stage_copy<4, COL_THREADS>(A, nload, [&](int t) {
    const int ch = fdiv(t, invLy);
    const int y = t - ch * Ly;
    return (y < ny) ? spec1[((size_t)ch * Kx + kx) * ny + y] : mk<T>(0, 0);
  });
  lds_barrier();
  // one thread per (output, |ky|): the kernel value at |ky| (the stored half)
  // serves both ky and Ly - ky.  The kernel values of PF pairs per thread
  // are loaded together; the first PF are issued before the forward
  // transforms, so their latency overlaps them.
  const int npair = no * Kyh;
  const float invK = 1.0f / (float)Kyh;
  constexpr int PF = 4;
  T kv[PF][3];
  auto load_kv = [&](int t0) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = t0 + u * COL_THREADS + (int)threadIdx.x;
      const int o = fdiv(t, invK);
      const int kyr = t - o * Kyh;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int ko = t < npair ? s_koff[o][b] : -1;
        kv[u][b] = ko < 0 ? T(0) : kern[ko + kyr];
      }
    }
  };
  load_kv(0);
  const int twh = (Ly & 1) ? 0 : Lh;
  cpx<T>* X = fft_lds<T, false, COL_THREADS>(A, B, P, nin_ch, Ly, stw, twh);
  cpx<T>* W = (X == A) ? B : A;
#pragma unroll 1
  for (int t0 = 0; t0 < npair; t0 += PF * COL_THREADS) {
    if (t0 > 0) load_kv(t0);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = t0 + u * COL_THREADS + (int)threadIdx.x;
      if (t >= npair) break;
      const int o = fdiv(t, invK);
      const int kyr = t - o * Kyh;
      const int ky2 = Ly - kyr;
      const bool two = kyr > 0 && ky2 > kyr;
      const int src = s_src[o];
      cpx<T> a1 = mk<T>(0, 0), a2 = mk<T>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (s_koff[o][b] < 0) continue;
        const int fl = s_fl[o][b];
        const T s = kv[u][b];
        const T s1 = (fl & 4) ? -s : s;                                // ky <= Ly/2
        const T s2 = (((fl & 4) != 0) != ((fl & 2) != 0)) ? -s : s;   // ky > Ly/2 (odd in ky)
        const cpx<T>* xb = X + (src * 3 + b) * Ly;
        const cpx<T> m1 = xb[kyr];
        if (fl & 1)
          a1 = a1 + mk<T>(-s1 * m1.y, s1 * m1.x);
        else
          a1 = a1 + mk<T>(s1 * m1.x, s1 * m1.y);
        if (two) {
          const cpx<T> m2 = xb[ky2];
          if (fl & 1)
            a2 = a2 + mk<T>(-s2 * m2.y, s2 * m2.x);
          else
            a2 = a2 + mk<T>(s2 * m2.x, s2 * m2.y);
        }
      }
      W[o * Ly + kyr] = a1;
      if (two) W[o * Ly + ky2] = a2;
    }
  }
  lds_barrier();
  cpx<T>* Y = fft_lds<T, true, COL_THREADS>(W, X, P, no, Ly, stw, twh);
  for (int o = 0; o < no; ++o) {
    const OutCh& oc = tab.ch[o0 + o];
    for (int r = threadIdx.x; r < oc.nrows; r += COL_THREADS) {
      int yy = (oc.row0 + r) % Ly;
      if (yy < 0) yy += Ly;
      spec2[oc.off + (size_t)r * Kx + kx] = Y[o * Ly + yy];
    }
  }
}

__device__ void rigid_stage(RigidState* R, const DriveP& d, int stage, double F, double h, double dxc, int travel);

// ------------------------------------------------------------ Dormand-Prince pair
// Nodes, stage coefficients (row i, j < i), fifth-order weights (the last
// row) and embedded fourth-order weights of the Dormand-Prince RK5(4) pair
// (Dormand & Prince, J. Comput. Appl. Math. 6, 19, 1980).
__device__ __forceinline__ double dp_c(int i) {
  switch (i) {
    case 1: return 1.0 / 5.0;
    case 2: return 3.0 / 10.0;
    case 3: return 4.0 / 5.0;
    case 4: return 8.0 / 9.0;
    case 5: case 6: return 1.0;
    default: return 0.0;
  }
}

__device__ __forceinline__ double dp_a(int i, int j) {
  switch (i * 8 + j) {
    case 8 + 0: return 1.0 / 5.0;
    case 16 + 0: return 3.0 / 40.0;
    case 16 + 1: return 9.0 / 40.0;
    case 24 + 0: return 44.0 / 45.0;
    case 24 + 1: return -56.0 / 15.0;
    case 24 + 2: return 32.0 / 9.0;
    case 32 + 0: return 19372.0 / 6561.0;
    case 32 + 1: return -25360.0 / 2187.0;
    case 32 + 2: return 64448.0 / 6561.0;
    case 32 + 3: return -212.0 / 729.0;
    case 40 + 0: return 9017.0 / 3168.0;
    case 40 + 1: return -355.0 / 33.0;
    case 40 + 2: return 46732.0 / 5247.0;
    case 40 + 3: return 49.0 / 176.0;
    case 40 + 4: return -5103.0 / 18656.0;
    case 48 + 0: return 35.0 / 384.0;
    case 48 + 2: return 500.0 / 1113.0;
    case 48 + 3: return 125.0 / 192.0;
    case 48 + 4: return -2187.0 / 6784.0;
    case 48 + 5: return 11.0 / 84.0;
    default: return 0.0;
  }
}

// Error weights: fifth-order minus embedded fourth-order weights.
__device__ __forceinline__ double dp_e(int j) {
  const double b5 = j < 6 ? dp_a(6, j) : 0.0;
  double b4 = 0.0;
  switch (j) {
    case 0: b4 = 5179.0 / 57600.0; break;
    case 2: b4 = 7571.0 / 16695.0; break;
    case 3: b4 = 393.0 / 640.0; break;
    case 4: b4 = -92097.0 / 339200.0; break;
    case 5: b4 = 187.0 / 2100.0; break;
    case 6: b4 = 1.0 / 40.0; break;
    default: break;
  }
  return b5 - b4;
}

// The slider's Dormand-Prince stage: its derivative at the stage state
// (Eq. 15) is kept, and the next stage's state x_n + h sum_j a_(i+1)j k_j
// (stages 0..5) formed.  At stage 6 the state stays (it is the fifth-order
// solution); the step control decides.
__device__ void rigid_stage_dp(RigidState* R, const DriveP& d, int stage, double F, double h) {
  const double x = R->xs, v = R->vs, t = R->ts;
  double dxdt = 0.0, dvdt = 0.0;
  if (d.mode == 1) {
    dxdt = d.v_d;
  } else if (d.mode == 2) {
    dxdt = v;
    dvdt = (d.k * (d.v_d * t + d.xa0 - x) - d.gamma_v * d.mass * v + F) / d.mass;
  }
  R->F[0] = F;
  R->kx[stage] = dxdt;
  R->kv[stage] = dvdt;
  if (stage < 6) {
    double sx = 0.0, sv = 0.0;
    for (int j = 0; j <= stage; ++j) {
      const double a = dp_a(stage + 1, j);
      sx += a * R->kx[j];
      sv += a * R->kv[j];
    }
    R->xs = R->x0 + h * sx;
    R->vs = R->v0 + h * sv;
    R->ts = R->t0 + dp_c(stage + 1) * h;
  }
}

// Slider stage update from a finished row launch's force partials, by one
// whole block: fixed-order float64 sum (strided per thread, then per wave,
// then over the waves), then Eq. 15's RK4 stage.
__device__ __forceinline__ void tick_body(const TickArgs& a, int stage, double dt) {
  __shared__ double s_red[16];
  double v = 0.0;
  for (int t = threadIdx.x; t < a.ntask; t += TICK_THREADS) v += a.partial[(size_t)t * 3];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  lds_barrier();
  if (threadIdx.x == 0) {
    double F = 0.0;
    for (int w = 0; w < (TICK_THREADS + 63) >> 6; ++w) F += s_red[w];
    if (a.scheme == 1)
      rigid_stage_dp(a.rigid, a.drive, stage, a.force_scale * F, a.ctrl->h);
    else
      rigid_stage(a.rigid, a.drive, stage, a.force_scale * F, dt, a.dx, a.travel);
  }
  lds_barrier();
}

template <typename T>
__global__ void __launch_bounds__(COL_THREADS)
    k_col(const cpx<T>* __restrict__ spec1, cpx<T>* __restrict__ spec2, const T* __restrict__ kern,
          int Kx, int Ly, int Kyh, int ny, int nin_ch, int ngroup, int nbuf, FftPlan P,
          const cpx<T>* __restrict__ twy, OutTable tab, TickArgs tick, int tick_stage, double tick_dt) {
  if (tick.ctrl != nullptr && tick.ctrl->done) return;  // adaptive run finished
  if (tick_stage >= 0 && blockIdx.x == 0) tick_body(tick, tick_stage, tick_dt);
  col_body<T>(xcd_remap(blockIdx.x, gridDim.x), spec1, spec2, kern, Kx, Ly, Kyh, ny, nin_ch, ngroup, nbuf, P, twy,
              tab);
}

__global__ void __launch_bounds__(TICK_THREADS) k_tick(TickArgs tick, int stage, double dt) { tick_body(tick, stage, dt); }

__global__ void __launch_bounds__(TICK_THREADS) k_tick_batch(const ColDesc* __restrict__ d, int stage, double dt) {
  tick_body(d[blockIdx.x].tick, stage, dt);
}

// End of a Dormand-Prince attempt (one block): the slider's last stage from
// the last row launch's force partials, the error ratio over the cells'
// block maxima and the slider's position and velocity errors, the decision
// and the next step size.  An accepted step takes the fifth-order state,
// advances t and re-seats s_int; the commit kernel then renormalises m.
constexpr double DP_END_REL = 1e-9;  // t_end reached when t_end - t <= DP_END_REL * t_end

__global__ void __launch_bounds__(TICK_THREADS)
    k_dp_control(TickArgs a, DpCtrl* ctrl, const double* __restrict__ errpart, int ntask) {
  __shared__ double s_max[16];
  if (ctrl->done) {
    if (threadIdx.x == 0) ctrl->accept = 0;
    return;
  }
  tick_body(a, 6, 0.0);
  double m = 0.0;
  for (int t = threadIdx.x; t < ntask; t += TICK_THREADS) m = (errpart[t] > m || errpart[t] != errpart[t]) ? errpart[t] : m;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double q = __shfl_down(m, o, 64);
    m = (q > m || q != q) ? q : m;
  }
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = m;
  lds_barrier();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < TICK_THREADS / 64; ++w) m = (s_max[w] > m || s_max[w] != s_max[w]) ? s_max[w] : m;
  m = (s_max[0] > m || s_max[0] != s_max[0]) ? s_max[0] : m;
  RigidState* R = a.rigid;
  const double h = ctrl->h;
  double ex = 0.0, ev = 0.0;
  for (int j = 0; j < 7; ++j) {
    ex += dp_e(j) * R->kx[j];
    ev += dp_e(j) * R->kv[j];
  }
  ex *= h;
  ev *= h;
  const double err = fmax(m, fmax(fabs(ex) / a.dx, fabs(ev) * h / a.dx));
  const double ratio = (m != m) ? m : err / ctrl->tol;
  const bool ok = ratio <= 1.0;
  double fac = ratio == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(ratio, -0.2)));
  if (!ok) fac = fmin(fac, 1.0);
  double hn = h * fac;
  if (ok) {
    R->x0 = R->xs;
    R->v0 = R->vs;
    R->t0 = R->t0 + h;
    R->step += 1;
    ctrl->accepted += 1;
    if (isfinite(R->x0)) {
      const double sc = floor(R->x0 / a.dx);
      if (fabs(sc) > (double)a.travel)
        R->flags |= FLAG_RANGE;
      else
        R->s_int = (int)sc;
    } else {
      R->flags |= FLAG_NUMERIC;
    }
    if (ctrl->t_end - R->t0 <= DP_END_REL * ctrl->t_end) {
      R->t0 = ctrl->t_end;
      ctrl->done = 1;
    }
  } else {
    ctrl->rejected += 1;
  }
  R->xs = R->x0;
  R->vs = R->v0;
  R->ts = R->t0;
  if (!ctrl->done) hn = fmin(hn, ctrl->t_end - R->t0);
  if (!isfinite(ratio) || !(hn > 0.0)) {
    // non-finite error or no step left: stop the run
    R->flags |= FLAG_NUMERIC;
    ctrl->done = 1;
  }
  ctrl->err = ratio;
  ctrl->accept = ok ? 1 : 0;
  ctrl->h = hn;
}

// Eq. 13: per slider row y, the sums over its cells of |div H| and |curl H|
// with two-point central differences of the base field on the stencil
// points written by the force pass (layout of RowParams::fieldout); rows
// wrap along a periodic y.  One block per row; fixed-order float64 sums.
template <typename T>
__global__ void __launch_bounds__(256)
    k_div_curl(const T* __restrict__ G, int nx, int ny, double dx, double dy, double dz, int pbc_y,
               double* __restrict__ part) {
  __shared__ double s_red[2][4];
  const int y = blockIdx.x;
  const size_t gcs = (size_t)(ny + 2) * (nx + 2), cs = (size_t)ny * nx;
  const int yl = pbc_y ? (y - 1 + ny) % ny : y - 1, yh = pbc_y ? (y + 1) % ny : y + 1;
  auto c = [&](int a, int row, int i) -> double { return (double)G[a * gcs + (size_t)(row + 1) * (nx + 2) + i + 1]; };
  auto zp = [&](int a, int i) -> double { return (double)G[3 * gcs + a * cs + (size_t)y * nx + i]; };
  auto zm = [&](int a, int i) -> double { return (double)G[3 * gcs + 3 * cs + a * cs + (size_t)y * nx + i]; };
  const double i2x = 1.0 / (2.0 * dx), i2y = 1.0 / (2.0 * dy), i2z = 1.0 / (2.0 * dz);
  double sd = 0.0, sc = 0.0;
  for (int i = threadIdx.x; i < nx; i += 256) {
    double dH[3][3];  // dH[a][b] = d_b H_a
    for (int a = 0; a < 3; ++a) {
      dH[a][0] = (c(a, y, i + 1) - c(a, y, i - 1)) * i2x;
      dH[a][1] = (c(a, yh, i) - c(a, yl, i)) * i2y;
      dH[a][2] = (zp(a, i) - zm(a, i)) * i2z;
    }
    const double div = dH[0][0] + dH[1][1] + dH[2][2];
    const double cx = dH[2][1] - dH[1][2], cy = dH[0][2] - dH[2][0], cz = dH[1][0] - dH[0][1];
    sd += fabs(div);
    sc += sqrt(cx * cx + cy * cy + cz * cz);
  }
  sd = wave_sum(sd);
  sc = wave_sum(sc);
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = sd;
    s_red[1][threadIdx.x >> 6] = sc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * y] = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
    part[2 * y + 1] = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
  }
}

// Accepted attempt: m = the fifth-order state renormalised (y5 and m are
// [film][3][plane]).
template <typename T>
__global__ void k_dp_commit(const T* __restrict__ y5, T* __restrict__ m, int nfilm, size_t plane,
                            const DpCtrl* __restrict__ ctrl, int* __restrict__ flags) {
  if (!ctrl->accept) return;
  const size_t n = (size_t)nfilm * plane;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const size_t f = q / plane, i = q - f * plane;
    const size_t o = f * 3 * plane + i;
    const T x = y5[o], y = y5[o + plane], z = y5[o + 2 * plane];
    const T nrm = sqrt(x * x + y * y + z * z);
    if (!(nrm > T(0)) || !isfinite(nrm)) atomicOr(flags, (int)FLAG_NUMERIC);
    m[o] = x / nrm;
    m[o + plane] = y / nrm;
    m[o + 2 * plane] = z / nrm;
  }
}

template <typename T>
__global__ void __launch_bounds__(COL_THREADS) k_col_batch(const ColDesc* __restrict__ d, const int* __restrict__ start,
                                                   int n, int tick_stage, double tick_dt) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_instance(start, n, b);
  const ColDesc& q = d[i];
  if (tick_stage >= 0 && b == start[i]) tick_body(q.tick, tick_stage, tick_dt);
  col_body<T>(b - start[i], gptr((const cpx<T>*)q.spec1), gptr((cpx<T>*)q.spec2), gptr((const T*)q.kern), q.Kx,
              q.Ly, q.Kyh, q.ny, q.nin_ch, q.ngroup, q.nbuf, q.P, gptr((const cpx<T>*)q.twy), q.tab);
}

// ------------------------------------------------------------ row kernel
// Threads per row block: 1024 for the float32 single-mesh kernel (four
// waves per SIMD at its register count), 512 where more registers are needed
// (float64, batched descriptors).
template <typename T, bool BATCH>
struct RowThreads { static constexpr int n = (sizeof(T) == 4 && !BATCH) ? 1024 : 512; };

template <typename T> struct FirHalf { static constexpr int K = 16; };
template <> struct FirHalf<double> { static constexpr int K = 30; };

__device__ __forceinline__ int reflect_idx(int k, int M) {
  if (M == 1) return 0;
  const int P = 2 * M - 2;
  k %= P;
  if (k < 0) k += P;
  return k > M - 1 ? P - k : k;
}

__device__ __forceinline__ double beta3(double t) {
  double a = fabs(t);
  if (a <= 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a <= 2.0) {
    double b = 2.0 - a;
    return b * b * b / 6.0;
  }
  return 0.0;
}

// Half-length complex input of the inverse real transform from the
// Hermitian half: Z[k] = (X[k] + conj X[N2x-k]) + i conj(w_k) (X[k] - conj X[N2x-k]).
template <typename T>
__device__ __forceinline__ cpx<T> c2r_twist(cpx<T> xk, cpx<T> xm, cpx<T> w) {
  xm.y = -xm.y;
  const cpx<T> s = xk + xm;
  const cpx<T> d = cmulc(xk - xm, w);
  return mk<T>(s.x - d.y, s.y + d.x);
}

// Inverse real transform of nb rows (Hermitian halves X[0..N2x] at base + rowo[b])
// into LDS; result buffer viewed as T* holds x[0..Lx) of each row at stride
// 2*N2x reals.
template <typename T, int NT, bool INPL = false>
__device__ __forceinline__ cpx<T>* c2r_rows(const cpx<T>* __restrict__ base, const long long* rowo, int nb, cpx<T>* fa, cpx<T>* fb,
                            int N2x,
                            const FftPlan& P, const cpx<T>* stw, const cpx<T>* stp) {
  const int tot = nb * N2x;
  const float inv = 1.0f / (float)N2x;
  stage_copy<4, NT>(fa, tot, [&](int t) {
    const int b = fdiv(t, inv);
    const int k = t - b * N2x;
    const cpx<T>* X = base + rowo[b];
    return c2r_twist(X[k], X[N2x - k], stp[k]);
  });
  lds_barrier();
  return row_fft<T, true, NT, INPL>(fa, fb, P, nb, stw);
}

// Inputs of the first batch of inverse row transforms, held in registers:
// issued early in the row kernel's set-up, they stay in flight across the
// LDS-only barriers and are folded into the half-length input by finish()
// once the twiddles are in LDS.  A thread holds CP elements; finish() loads
// and folds any further ones itself.
template <typename T, int NT, int CP>
struct C2rInputs {
  cpx<T> xk[CP], xm[CP];
  __device__ __forceinline__ void issue(const cpx<T>* __restrict__ base, const long long* rowo, int tot, int N2x) {
    const float inv = 1.0f / (float)N2x;
#pragma unroll
    for (int u = 0; u < CP; ++u) {
      const int t = (int)threadIdx.x + u * NT;
      if (t < tot) {
        const int b = fdiv(t, inv);
        const int k = t - b * N2x;
        const cpx<T>* X = base + rowo[b];
        xk[u] = X[k];
        xm[u] = X[N2x - k];
      }
    }
  }
  __device__ __forceinline__ void finish(const cpx<T>* __restrict__ base, const long long* rowo, int tot, int N2x,
                                         cpx<T>* fa, const cpx<T>* stp) {
    const float inv = 1.0f / (float)N2x;
#pragma unroll
    for (int u = 0; u < CP; ++u) {
      const int t = (int)threadIdx.x + u * NT;
      if (t < tot) {
        const int k = t - fdiv(t, inv) * N2x;
        fa[t] = c2r_twist(xk[u], xm[u], stp[k]);
      }
    }
#pragma unroll 1
    for (int t = (int)threadIdx.x + CP * NT; t < tot; t += NT) {
      const int b = fdiv(t, inv);
      const int k = t - b * N2x;
      const cpx<T>* X = base + rowo[b];
      fa[t] = c2r_twist(X[k], X[N2x - k], stp[k]);
    }
  }
};

template <typename T> struct alignas(2 * sizeof(T)) Pair { T x, y; };

// NO consecutive spline values at window coordinates k0 + j + frac,
// j = 0 .. NO-1: o_j = sum_q g_q ext(k0 + j - K - 1 + q), q = 0 .. 2K+3,
// summed in q order, from one register window read one sample at a time
// (neighbouring lanes NO samples apart: conflict-free LDS reads for odd NO).
// g (16-byte aligned) is read in 16-byte vectors.
template <typename T, int K, int NO>
__device__ __forceinline__ void fir_evaln(const T* ext, const T* g, int k0, int E, T* o) {
  constexpr int NQ = 2 * K + 4;
  constexpr int GV = 16 / sizeof(T);
  const T* p = ext + E + k0 - K - 1;
  T w[NQ + NO - 1];
#pragma unroll
  for (int q = 0; q < NQ + NO - 1; ++q) w[q] = p[q];
  T a[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) a[j] = 0;
#pragma unroll
  for (int q0 = 0; q0 < NQ; q0 += GV) {
    T gv[GV];
    if constexpr (GV == 4) {
      const float4 v = *reinterpret_cast<const float4*>(g + q0);
      gv[0] = v.x; gv[1] = v.y; gv[2] = v.z; gv[3] = v.w;
    } else {
      const Pair<T> v = *reinterpret_cast<const Pair<T>*>(g + q0);
      gv[0] = v.x; gv[1] = v.y;
    }
#pragma unroll
    for (int u = 0; u < GV; ++u)
#pragma unroll
      for (int j = 0; j < NO; ++j) a[j] += gv[u] * w[q0 + u + j];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) o[j] = a[j];
}

__device__ void rigid_stage(RigidState* R, const DriveP& d, int stage, double F, double h,
                            double dxc, int travel) {
  // every field is read before the first store, so the loads issue together
  const double x = R->xs, v = R->vs, t = R->ts;
  const double x0 = R->x0, v0 = R->v0, t0 = R->t0, ax = R->ax, av = R->av;
  double dxdt = 0.0, dvdt = 0.0;
  if (d.mode == 1) {
    dxdt = d.v_d;
  } else if (d.mode == 2) {
    dxdt = v;
    dvdt = (d.k * (d.v_d * t + d.xa0 - x) - d.gamma_v * d.mass * v + F) / d.mass;
  }
  R->F[0] = F;
  if (stage == 0) {
    R->ax = dxdt;
    R->av = dvdt;
    R->xs = x0 + 0.5 * h * dxdt;
    R->vs = v0 + 0.5 * h * dvdt;
    R->ts = t0 + 0.5 * h;
  } else if (stage == 1) {
    R->ax = ax + 2.0 * dxdt;
    R->av = av + 2.0 * dvdt;
    R->xs = x0 + 0.5 * h * dxdt;
    R->vs = v0 + 0.5 * h * dvdt;
    R->ts = t0 + 0.5 * h;
  } else if (stage == 2) {
    R->ax = ax + 2.0 * dxdt;
    R->av = av + 2.0 * dvdt;
    R->xs = x0 + h * dxdt;
    R->vs = v0 + h * dvdt;
    R->ts = t0 + h;
  } else {
    const double xn = x0 + h / 6.0 * (ax + dxdt);
    const double vn = v0 + h / 6.0 * (av + dvdt);
    R->t0 = t0 + h;
    R->ts = t0 + h;
    R->x0 = R->xs = xn;
    R->v0 = R->vs = vn;
    R->step += 1;
    if (isfinite(xn)) {
      const double s = floor(xn / dxc);
      if (fabs(s) > (double)travel) {
        R->flags |= FLAG_RANGE;
      } else {
        R->s_int = (int)s;
      }
    } else {
      R->flags |= FLAG_NUMERIC;
    }
  }
}

// Row kinds of the fused row kernel.
enum { RK_SELF = 0, RK_CROSS = 3, RK_FP = 6, RK_FM = 9, RK_PHI = 12, RK_XB = 40 };
constexpr int MAX_ROWS = 24;

// Block layout: tasks [film 0 rows][film 1 rows] (MODE_STAGE; in potential
// mode with a spring drive also [film 1 rows -1 and ny]), [eval_film rows]
// (MODE_EVAL), [film 1 rows -1..ny] (MODE_FORCE).  In direct mode the
// force's boundary rows -1 and ny (the y term summed by parts needs the
// x-component of the base field there) ride along with the tasks of film 1
// rows 0 and ny-1, one more inverse transform each, so that a stage
// launches exactly nfilm * ny blocks.  All inverse row transforms of a task run as one batch (or
// batches of p.nbr rows); every spline window is filtered in parallel.
template <typename T, int NT, bool INPL = false>
__device__ __forceinline__ void row_stage_body(const RowParams& p, int stage, double dt, int task, int ntask,
                                               const cpx<T>* __restrict__ spec2, const T* __restrict__ mst,
                                               const T* m0, T* mnext, T* __restrict__ acc, T* __restrict__ hout,
                                               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twp,
                                               RigidState* __restrict__ rigid, double* __restrict__ partial,
                                               unsigned int* __restrict__ counter) {
  constexpr int K = FirHalf<T>::K;
  constexpr int NQ = 2 * K + 4;
  constexpr int E = K + 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nx = p.nx, ny = p.ny, N2x = p.N2x, M = p.M, Lx = 2 * N2x, nbr = p.nbr;
  const int MW = M + 2 * E;
  const int MWS = (MW + 5) & ~1;  // row stride of the windows, >= MW + 4 (slack for the FIR reads past a row)
  const int nfc = p.full_force ? 3 : 1;
  cpx<T>* stw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* stp = stw + N2x;
  cpx<T>* fa = stp + N2x + 1;
  cpx<T>* fb = INPL ? fa : fa + (size_t)nbr * N2x;  // ping-pong partner (none in place)
  T* ext = reinterpret_cast<T*>(fb + (size_t)nbr * N2x);  // [nbr][MW]
  // weights, slider samples base field (16-byte aligned for vector reads)
  T* gs = reinterpret_cast<T*>(smem_raw + ((static_cast<size_t>(reinterpret_cast<unsigned char*>(ext + (size_t)nbr * MWS) - smem_raw) + 15) & ~size_t(15)));
  T* gb = gs + NQ;                 // weights, base samples slider field
  T* H = gb + NQ;                  // [3][nx] demag accumulation
  T* gc = H + 3 * nx;              // [3][nx+2] slider cross field at i = -1..nx
  T* gp = gc + 3 * (nx + 2);       // [nfc][nx] force layer z_s+1
  T* gm = gp + nfc * nx;           // [nfc][nx] force layer z_s-1
  T* phit = gm + nfc * nx;         // [nslot][nx+6] potential at i = -3..nx+2
  const int nslot_max = p.pot ? (p.full_force ? 19 : 9) : 0;
  T* gxb = phit + (size_t)nslot_max * (nx + 6);  // [2][nx] base field x at slider rows -1, ny
  // (offset arithmetic from smem_raw keeps the LDS address space)
  const size_t red_off = ((size_t)(reinterpret_cast<unsigned char*>(gxb + 2 * nx + 2) - smem_raw) + 15) & ~size_t(15);
  double* red = reinterpret_cast<double*>(smem_raw + red_off);
  __shared__ long long rowo[MAX_ROWS];  // element offsets of the rows in spec2
  __shared__ int rowkind[MAX_ROWS];
  __shared__ int slot_of[7][5];  // (layer d + 3, row offset + 2) -> slot, -1 if absent
  __shared__ int s_nrow;
  __shared__ int s_last;
  __shared__ int s_bad;

  int film, y;
  if (p.mode == MODE_STAGE) {
    if (task < p.nfilm * ny) {
      film = task / ny;
      y = task - film * ny;
    } else {
      film = 1;
      y = (task == p.nfilm * ny) ? -1 : ny;
    }
  } else if (p.mode == MODE_EVAL) {
    film = p.eval_film;
    y = task;
  } else {
    film = 1;
    y = task - 1;
  }
  const bool cell_row = (y >= 0 && y < ny);
  const bool two = (p.nfilm == 2);
  // periodic y: the rows -1 and ny are rows of the film, summed by parts
  // with wrapped neighbours; the tasks outside the film add nothing
  const bool pbc_y = (p.pbc & 2) != 0, pbc_x = (p.pbc & 1) != 0;
  const bool need_force = two && film == 1 && (cell_row || !pbc_y) &&
                          ((p.mode == MODE_STAGE && p.with_force) || p.mode == MODE_FORCE);
  const bool ext_cross = two && film == 0 && p.hsur != nullptr;
  const float* __restrict__ hsur = gptr(p.hsur);
  const bool need_cross = two && !ext_cross && ((p.term_mask & 16) || need_force);
  // boundary force rows carried by this task (direct mode, stage launches)
  const bool xb_lo = p.mode == MODE_STAGE && need_force && !p.pot && !pbc_y && y == 0;
  const bool xb_hi = p.mode == MODE_STAGE && need_force && !p.pot && !pbc_y && y == ny - 1;
  // direct-mode stage launches: the force's z_s - 1 layer row of slider row y
  // is transformed and filtered by the base-film task of row y, which adds
  // that part of the z term (seven rows per task on both films)
  const bool fm_split = p.mode == MODE_STAGE && p.with_force && !p.pot && two;
  const bool fm_here = fm_split && film == 0 && cell_row;
  const int h = p.halo;

  // direct mode: the row table in closed form (row i -> spec2 offset, kind)
  const bool closed = !(need_cross && p.pot);
  const int n_self = (cell_row && (p.term_mask & 8)) ? 3 : 0;
  const int n_cross = need_cross ? ((cell_row || p.full_force) ? 3 : 1) : 0;
  const int n_frc = (need_force && cell_row) ? (fm_split ? nfc : 2 * nfc) : (fm_here ? 1 : 0);
  const int n_tot = n_self + n_cross + n_frc + (xb_lo ? 1 : 0) + (xb_hi ? 1 : 0);
  auto row_entry = [&](int i, int& kind) -> long long {
    long long r;
    if (i < n_self) {
      r = p.off_self[film][i] + (long long)y * p.Kx;
      kind = RK_SELF + i;
    } else if (i < n_self + n_cross) {
      const int c = i - n_self;
      r = p.off_cross[film][c] + (long long)(y - p.cross_row0[film]) * p.Kx;
      kind = RK_CROSS + c;
    } else if (i < n_self + n_cross + n_frc) {
      const int j = i - n_self - n_cross;
      if (fm_here) {
        r = p.off_fm[0] + (long long)y * p.Kx;
        kind = RK_FM;
      } else if (fm_split) {
        r = p.off_fp[j] + (long long)y * p.Kx;
        kind = RK_FP + j;
      } else {
        const int c = j >> 1;
        r = ((j & 1) ? p.off_fm[c] : p.off_fp[c]) + (long long)y * p.Kx;
        kind = ((j & 1) ? RK_FM : RK_FP) + c;
      }
    } else {
      const bool lo = xb_lo && i == n_self + n_cross + n_frc;
      r = p.off_cross[1][0] + (long long)((lo ? -1 : ny) - p.cross_row0[1]) * p.Kx;
      kind = RK_XB + (lo ? 0 : 1);
    }
    return r;
  };

  // slider offset of this stage (issued first; the slider state is written
  // only after every block of the launch has read it)
  const DpCtrl* ctrl = gptr(p.ctrl);
  if (p.scheme == 1 && ctrl->done) return;  // adaptive run finished
  if (p.scheme == 1) dt = ctrl->h;
  const double xs = rigid->xs;
  const int s_int = rigid->s_int;
  // twiddles (stw: N2x, stp: N2x + 1, contiguous): loads issued before the
  // row table is built, stored after it
  constexpr int TWR = 2;
  const int ntw = 2 * N2x + 1;
  cpx<T> tv[TWR];
#pragma unroll
  for (int u = 0; u < TWR; ++u) {
    const int t = (int)threadIdx.x + u * NT;
    if (t < ntw) tv[u] = t < N2x ? tw[t] : twp[t - N2x];
  }
  if (closed) {
#pragma unroll 1
    for (int i = threadIdx.x; i < n_tot; i += NT) {
      int kind;
      rowo[i] = row_entry(i, kind);
      rowkind[i] = kind;
    }
    if (threadIdx.x == 0) {
      s_bad = 0;
      s_nrow = n_tot;
    }
  } else if (threadIdx.x == 0) {
    s_bad = 0;
    int n = 0;
    if (cell_row && (p.term_mask & 8))
      for (int c = 0; c < 3; ++c) {
        rowo[n] = p.off_self[film][c] + (size_t)y * p.Kx;
        rowkind[n++] = RK_SELF + c;
      }
    for (int a = 0; a < 7; ++a)
      for (int b = 0; b < 5; ++b) slot_of[a][b] = -1;
    if (need_cross && p.pot) {
      // potential rows needed by this task (layer offset d, row offset r)
      int ns = 0;
      auto add = [&](int d, int r) {
        slot_of[d + 3][r + 2] = ns;
        rowo[n] = p.off_phi[film][d + 3] + (size_t)(y + r - p.phi_row0[film][d + 3]) * p.Kx;
        rowkind[n++] = RK_PHI + ns;
        ++ns;
      };
      const bool full = p.mode == MODE_FORCE;
      if (cell_row || full) {
        for (int r = -2; r <= 2; ++r) add(0, r);
        if (full && cell_row) {
          for (int r = -2; r <= 2; ++r) add(1, r);
          for (int r = -2; r <= 2; ++r) add(-1, r);
          add(2, 0);
          add(-2, 0);
          add(3, 0);
          add(-3, 0);
        } else {
          add(1, 0);
          add(-1, 0);
          add(2, 0);
          add(-2, 0);
        }
      } else {
        add(0, 0);
      }
    } else if (need_cross) {
      const int ncomp = (cell_row || p.full_force) ? 3 : 1;
      const int stored = y - p.cross_row0[film];
      for (int c = 0; c < ncomp; ++c) {
        rowo[n] = p.off_cross[film][c] + (size_t)stored * p.Kx;
        rowkind[n++] = RK_CROSS + c;
      }
    }
    if (need_force && cell_row && !p.pot)
      for (int c = 0; c < nfc; ++c) {
        rowo[n] = p.off_fp[c] + (size_t)y * p.Kx;
        rowkind[n++] = RK_FP + c;
        rowo[n] = p.off_fm[c] + (size_t)y * p.Kx;
        rowkind[n++] = RK_FM + c;
      }
    if (xb_lo) {
      rowo[n] = p.off_cross[1][0] + (size_t)(-1 - p.cross_row0[1]) * p.Kx;
      rowkind[n++] = RK_XB;
    }
    if (xb_hi) {
      rowo[n] = p.off_cross[1][0] + (size_t)(ny - p.cross_row0[1]) * p.Kx;
      rowkind[n++] = RK_XB + 1;
    }
    s_nrow = n;
  }
#pragma unroll
  for (int u = 0; u < TWR; ++u) {
    const int t = (int)threadIdx.x + u * NT;
    if (t < ntw) stw[t] = tv[u];
  }
#pragma unroll 1
  for (int t = (int)threadIdx.x + TWR * NT; t < ntw; t += NT) stw[t] = t < N2x ? tw[t] : twp[t - N2x];
  lds_barrier();  // row table, twiddles
  const int nrow = s_nrow;
  // the first batch's transform inputs: issued now, consumed after the
  // spline weights
  constexpr int CP = (sizeof(T) == 4 && 4096 / NT > 4) ? (4096 / NT > 8 ? 8 : 4096 / NT) : 4;
  C2rInputs<T, NT, CP> in0;
  const int tot0 = min(nbr, nrow) * N2x;
  in0.issue(spec2, rowo, tot0, N2x);
#pragma unroll 1
  for (int t = threadIdx.x; t < 3 * nx; t += NT) H[t] = T(0);

  double xp = xs / p.dx - (double)s_int;
  const bool xp_bad = !(xp >= -1.0 && xp < 2.0);
  if (xp_bad) xp = 0.0;
  const double fls = floor(xp), flb = floor(-xp);
  const double frs = xp - fls, frb = -xp - flb;
  const int ifs = (int)fls, ifb = (int)flb;
  // spline weights: the four terms of each weight on their own threads,
  // then summed in tap order
  {
    double* wterm = red + 96;  // [2 NQ][4]
#pragma unroll 1
    for (int u = threadIdx.x; u < 8 * NQ; u += NT) {
      const int tq = u >> 2, t = (u & 3) - 1;
      const int q = (tq % NQ) - K - 1;
      const double fr = tq < NQ ? frs : frb;
      const double z1 = -0.26794919243112270647;  // sqrt(3) - 2, pole of the cubic B-spline prefilter
      const int j = t - q;
      double v = 0.0;
      if (j >= -K && j <= K) {
        // z1^|j| by binary exponentiation (|j| <= K)
        double zp = 1.0, b = z1;
        for (int e = abs(j); e; e >>= 1) {
          if (e & 1) zp *= b;
          b *= b;
        }
        v = beta3(fr - t) * 1.7320508075688772935 * zp;
      }
      wterm[u] = v;
    }
    lds_barrier();
#pragma unroll 1
    for (int tq = threadIdx.x; tq < 2 * NQ; tq += NT) {
      double g = 0.0;
      for (int t = 0; t < 4; ++t) g += wterm[tq * 4 + t];
      if (p.interp == 1) {
        // linear interpolation: taps at offsets 0 and 1 of the window
        const int q = tq % NQ;
        const double fr = tq < NQ ? frs : frb;
        g = q == K + 1 ? 1.0 - fr : (q == K + 2 ? fr : 0.0);
      }
      (tq < NQ ? gs : gb)[tq % NQ] = (T)g;
    }
  }
  in0.finish(spec2, rowo, tot0, N2x, fa, stp);
  lds_barrier();
  const int W0c = (film == 1) ? s_int - h : -s_int - h;  // cross window start
  const int W0f = s_int - h;                              // force windows (base field)

  for (int b0 = 0; b0 < nrow; b0 += nbr) {
    const int bn = min(nbr, nrow - b0);
    // the first batch's half-length inputs were formed during the set-up
    cpx<T>* Z = b0 == 0 ? row_fft<T, true, NT, INPL>(fa, fb, p.px, bn, stw)
                        : c2r_rows<T, NT, INPL>(spec2, rowo + b0, bn, fa, fb, N2x, p.px, stw, stp);
    const T* xr = reinterpret_cast<const T*>(Z);
    // self rows -> H, spline rows -> windows with mirror extension
    const float invMW = 1.0f / (float)MW;
#pragma unroll 1
    for (int t = threadIdx.x; t < bn * MW; t += NT) {
      const int r = fdiv(t, invMW);
      const int k = t - r * MW;
      const int kind = rowkind[b0 + r];
      const T* row = xr + (size_t)r * Lx;
      if (kind < RK_CROSS) {
        if (k < nx) H[kind * nx + k] = row[k];
      } else {
        // mirror only the 2E samples outside the window; the lattice index
        // then lies within one period of [0, Lx)
        int w = k - E;
        if (w < 0 || w >= M) w = reflect_idx(w, M);
        int X = ((kind < RK_FP || kind >= RK_PHI) ? W0c : W0f) + w;
        if (X < 0)
          X += Lx;
        else if (X >= Lx)
          X -= Lx;
        if (X < 0 || X >= Lx) {
          X %= Lx;
          if (X < 0) X += Lx;
        }
        ext[(size_t)r * MWS + k] = row[X];
      }
    }
    lds_barrier();
    const int NP = nx + 6;  // potential outputs i = -3 .. nx+2
    // spline outputs: NO consecutive i per thread, over the spline rows of
    // the batch only, each row over the outputs its kind needs (potential
    // -3..nx+2, the slider's cross field -1..nx, otherwise 0..nx-1), so a
    // float32 task fits one pass of the block
    constexpr int NO = sizeof(T) == 4 ? 3 : 2;
    auto out_range = [&](int kind, int& lo, int& cnt) {
      lo = 0;
      cnt = nx;
      if (kind < RK_CROSS) {
        cnt = 0;
      } else if (kind >= RK_PHI && kind < RK_XB) {
        lo = -3;
        cnt = NP;
      } else if (kind < RK_FP && film == 1) {
        lo = -1;
        cnt = nx + 2;
      }
    };
    int nitem = 0;
    for (int r = 0; r < bn; ++r) {
      int lo, cnt;
      out_range(rowkind[b0 + r], lo, cnt);
      nitem += (cnt + NO - 1) / NO;
    }
#pragma unroll 1
    for (int t = threadIdx.x; t < nitem; t += NT) {
      int r = 0, first = 0, lo = 0, cnt = 0;
      for (;; ++r) {
        out_range(rowkind[b0 + r], lo, cnt);
        const int ng = (cnt + NO - 1) / NO;
        if (t < first + ng) break;
        first += ng;
      }
      const int kind = rowkind[b0 + r];
      const int i0 = lo + NO * (t - first);
      const T* e = ext + (size_t)r * MWS;
      // the base film samples the slider's field (and potential) at -x_p
      const bool base = film == 0 && (kind < RK_FP || (kind >= RK_PHI && kind < RK_XB));
      T v[NO];
      if constexpr (sizeof(T) == 8) {  // float64: two call sites keep its wide window in registers
        if (base)
          fir_evaln<T, K, NO>(e, gb, i0 + h + ifb, E, v);
        else
          fir_evaln<T, K, NO>(e, gs, i0 + h + ifs, E, v);
      } else {
        fir_evaln<T, K, NO>(e, base ? gb : gs, i0 + h + (base ? ifb : ifs), E, v);
      }
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        const int i = i0 + j;
        if (i >= lo + cnt) break;
        if (kind >= RK_XB) {
          gxb[(kind - RK_XB) * nx + i] = v[j];
        } else if (kind >= RK_PHI) {
          phit[(size_t)(kind - RK_PHI) * NP + i + 3] = v[j];
        } else if (kind < RK_FP) {
          const int c = kind - RK_CROSS;
          if (film == 1) {
            gc[c * (nx + 2) + i + 1] = v[j];
            if (cell_row && i >= 0 && i < nx && (p.term_mask & 16)) H[c * nx + i] += v[j];
          } else {
            H[c * nx + i] += v[j];
          }
        } else if (kind < RK_FM) {
          gp[(kind - RK_FP) * nx + i] = v[j];
        } else {
          gm[(kind - RK_FM) * nx + i] = v[j];
        }
      }
    }
    lds_barrier();
  }

  // non-uniform applied field (Sec. II.A): the base film's cells take the
  // frame values; the slider's cells the samples of the frame field at their
  // moved positions, interpolated along x like its cross field (same window,
  // mirror ends and weights)
  if (cell_row && (p.term_mask & 4)) {
    if (film == 0 && p.hext_b != nullptr) {
      const T* src = gptr(reinterpret_cast<const T*>(p.hext_b)) + (size_t)y * nx;
#pragma unroll 1
      for (int t = threadIdx.x; t < 3 * nx; t += NT) {
        const int c = t / nx, i = t - c * nx;
        H[t] += src[(size_t)c * ny * nx + i];
      }
      lds_barrier();
    } else if (film == 1 && p.hext_s != nullptr) {
      const T* src = gptr(reinterpret_cast<const T*>(p.hext_s)) + (size_t)y * p.hext_w;
      const size_t cs = (size_t)ny * p.hext_w;
      const float invMW = 1.0f / (float)MW;
      for (int c0 = 0; c0 < 3; c0 += nbr) {
        const int nc = min(nbr, 3 - c0);
#pragma unroll 1
        for (int t = threadIdx.x; t < nc * MW; t += NT) {
          const int r = fdiv(t, invMW), k = t - r * MW;
          int w = k - E;
          if (w < 0 || w >= M) w = reflect_idx(w, M);
          int X = W0f + w;
          if (pbc_x) {
            X %= nx;
            if (X < 0) X += nx;
          } else {
            X += p.hext_off;
          }
          ext[(size_t)r * MWS + k] = src[(size_t)(c0 + r) * cs + X];
        }
        lds_barrier();
        // one output per thread, taps streamed from LDS (an optional term:
        // kept off the register window of the spline rows' FIR)
#pragma unroll 1
        for (int t = threadIdx.x; t < nc * nx; t += NT) {
          const int r = t / nx, i = t - r * nx;
          const T* e = ext + (size_t)r * MWS + E + i + h + ifs - K - 1;
          T a = T(0);
#pragma unroll 4
          for (int q = 0; q < NQ; ++q) a += gs[q] * e[q];
          H[(c0 + r) * nx + i] += a;
        }
        lds_barrier();
      }
    }
  }

  if (need_cross && p.pot) {
    // H = -grad phi with the four-point central difference on the shifted
    // lattice (far field from the scalar potential, Sec. III.A)
    const int NP = nx + 6;
    const T c1 = T(8.0 / 12.0), c2 = T(1.0 / 12.0);
    const T ix = T(1.0 / p.dx), iy = T(1.0 / p.dy), iz = T(1.0 / p.dz);
    auto ph = [&](int d, int r, int i) -> T { return phit[(size_t)slot_of[d + 3][r + 2] * NP + i + 3]; };
    auto hcomp = [&](int a, int d, int i) -> T {
      if (a == 0)
        return -(c1 * (ph(d, 0, i + 1) - ph(d, 0, i - 1)) - c2 * (ph(d, 0, i + 2) - ph(d, 0, i - 2))) * ix;
      if (a == 1)
        return -(c1 * (ph(d, 1, i) - ph(d, -1, i)) - c2 * (ph(d, 2, i) - ph(d, -2, i))) * iy;
      return -(c1 * (ph(d + 1, 0, i) - ph(d - 1, 0, i)) - c2 * (ph(d + 2, 0, i) - ph(d - 2, 0, i))) * iz;
    };
    const bool full = p.mode == MODE_FORCE;
    if (cell_row) {
#pragma unroll 1
      for (int t = threadIdx.x; t < 3 * nx; t += NT) {
        const int c = t / nx, i = t - c * nx;
        if (p.term_mask & 16) H[t] += hcomp(c, 0, i);
      }
    }
    if (need_force) {
#pragma unroll 1
      for (int t = threadIdx.x; t < nfc * (nx + 2); t += NT) {
        const int a = t / (nx + 2), i = t - a * (nx + 2) - 1;
        gc[a * (nx + 2) + i + 1] = hcomp(a, 0, i);
      }
      if (cell_row)
#pragma unroll 1
        for (int t = threadIdx.x; t < nfc * nx; t += NT) {
          const int a = t / nx, i = t - a * nx;
          if (a == 0 || full) {
            gp[a * nx + i] = hcomp(a, 1, i);
            gm[a * nx + i] = hcomp(a, -1, i);
          }
        }
    }
    lds_barrier();
  }

  if (p.mode == MODE_FORCE && p.fieldout != nullptr && need_force) {
    // the base field on the slider's stencil points, for Eq. 13's
    // divergence and curl (gc holds i = -1..nx of this row; gp, gm the
    // layers z_s +- 1 on the cells)
    T* G = gptr(reinterpret_cast<T*>(p.fieldout));
    const size_t gcs = (size_t)(ny + 2) * (nx + 2), cs = (size_t)ny * nx;
#pragma unroll 1
    for (int t = threadIdx.x; t < 3 * (nx + 2); t += NT) {
      const int a = t / (nx + 2), i = t - a * (nx + 2);
      G[a * gcs + (size_t)(y + 1) * (nx + 2) + i] = gc[a * (nx + 2) + i];
    }
    if (cell_row)
#pragma unroll 1
      for (int t = threadIdx.x; t < 3 * nx; t += NT) {
        const int a = t / nx, i = t - a * nx;
        G[3 * gcs + a * cs + (size_t)y * nx + i] = gp[a * nx + i];
        G[3 * gcs + 3 * cs + a * cs + (size_t)y * nx + i] = gm[a * nx + i];
      }
  }
  // --- per cell: local terms, LLG stage, force partials
  const size_t plane = (size_t)ny * nx;
  if (ext_cross && cell_row && (p.term_mask & 16)) {
    const T sc = (T)p.sur_scale;
#pragma unroll 1
    for (int t = threadIdx.x; t < 3 * nx; t += NT) {
      const int c = t / nx, i = t - c * nx;
      H[t] += sc * (T)hsur[(size_t)c * plane + (size_t)y * nx + i];
    }
    lds_barrier();
  }
  double fpart[3] = {0.0, 0.0, 0.0};
  const T* ms = mst + (size_t)film * 3 * plane;
  const T idx2 = T(1.0 / (p.dx * p.dx)), idy2 = T(1.0 / (p.dy * p.dy));
  const T pex = (T)p.pref_ex, pan = (T)p.pref_an;
  const T u0 = (T)p.u[0], u1 = (T)p.u[1], u2 = (T)p.u[2];
  const T gam = (T)p.gam, alp = (T)p.alpha;
  const T hdt = (T)dt;
  bool bad = false;
  double errmax = 0.0;  // Dormand-Prince last stage: largest |error| of m
  // fused x transform of the new row: real rows packed in fa (Lx reals each)
  const bool fuse = p.spec1_out != nullptr && p.mode == MODE_STAGE && cell_row;
  T* fr = reinterpret_cast<T*>(fa);
  if (fuse)
#pragma unroll 1
    for (int t = threadIdx.x; t < 3 * (Lx - nx); t += NT) {
      const int c = t / (Lx - nx);
      fr[c * Lx + nx + (t - c * (Lx - nx))] = T(0);
    }
  if (cell_row && p.mode != MODE_FORCE) {
#pragma unroll 1
    for (int i = threadIdx.x; i < nx; i += NT) {
      const size_t id = (size_t)y * nx + i;
      const T mx = ms[id], my = ms[plane + id], mz = ms[2 * plane + id];
      T hx = H[i], hy = H[nx + i], hz = H[2 * nx + i];
      if (p.term_mask & 1) {
        T ex = 0, ey = 0, ez = 0;
        // neighbours (free boundaries, or wrapped along a periodic axis)
        auto nb = [&](size_t q, T w) {
          ex += (ms[q] - mx) * w;
          ey += (ms[plane + q] - my) * w;
          ez += (ms[2 * plane + q] - mz) * w;
        };
        if (i > 0)
          nb(id - 1, idx2);
        else if (pbc_x && nx > 1)
          nb(id + nx - 1, idx2);
        if (i < nx - 1)
          nb(id + 1, idx2);
        else if (pbc_x && nx > 1)
          nb(id + 1 - nx, idx2);
        if (y > 0)
          nb(id - nx, idy2);
        else if (pbc_y && ny > 1)
          nb(id + plane - nx, idy2);
        if (y < ny - 1)
          nb(id + nx, idy2);
        else if (pbc_y && ny > 1)
          nb(id + nx - plane, idy2);
        hx += pex * ex;
        hy += pex * ey;
        hz += pex * ez;
      }
      if (p.term_mask & 2) {
        const T mu = mx * u0 + my * u1 + mz * u2;
        hx += pan * mu * u0;
        hy += pan * mu * u1;
        hz += pan * mu * u2;
      }
      if (p.term_mask & 4) {
        hx += (T)p.hext[0];
        hy += (T)p.hext[1];
        hz += (T)p.hext[2];
      }
      if (p.mode == MODE_EVAL) {
        hout[id] = hx;
        hout[plane + id] = hy;
        hout[2 * plane + id] = hz;
        continue;
      }
      // LLG right-hand side, Landau-Lifshitz form of Eq. (1)
      const T cx = my * hz - mz * hy, cy = mz * hx - mx * hz, cz = mx * hy - my * hx;
      const T dx_ = my * cz - mz * cy, dy_ = mz * cx - mx * cz, dz_ = mx * cy - my * cx;
      const T kx = -gam * (cx + alp * dx_), ky = -gam * (cy + alp * dy_), kz = -gam * (cz + alp * dz_);
      const size_t fo = (size_t)film * 3 * plane + id;
      const T ox = m0[fo], oy = m0[fo + plane], oz = m0[fo + 2 * plane];
      if (p.scheme == 1) {
        // Dormand-Prince stage: keep k_stage; form the next stage's state
        // m_n + h sum_j a_(stage+1)j k_j (j ascending), or at the last stage
        // the error h sum_j e_j k_j
        T* K = gptr(reinterpret_cast<T*>(p.kdp));
        const size_t kst = (size_t)p.nfilm * 3 * plane;
        K[stage * kst + fo] = kx;
        K[stage * kst + fo + plane] = ky;
        K[stage * kst + fo + 2 * plane] = kz;
        if (stage < 6) {
          T sx = 0, sy = 0, sz = 0;
          for (int j = 0; j < stage; ++j) {
            const T a = (T)dp_a(stage + 1, j);
            if (a == T(0)) continue;
            sx += a * K[j * kst + fo];
            sy += a * K[j * kst + fo + plane];
            sz += a * K[j * kst + fo + 2 * plane];
          }
          const T a = (T)dp_a(stage + 1, stage);
          sx += a * kx;
          sy += a * ky;
          sz += a * kz;
          const T nx_ = ox + hdt * sx, ny_ = oy + hdt * sy, nz_ = oz + hdt * sz;
          mnext[fo] = nx_;
          mnext[fo + plane] = ny_;
          mnext[fo + 2 * plane] = nz_;
          if (fuse) {
            fr[i] = nx_;
            fr[Lx + i] = ny_;
            fr[2 * Lx + i] = nz_;
          }
        } else {
          T ex = 0, ey = 0, ez = 0;
          for (int j = 0; j < 6; ++j) {
            const T e = (T)dp_e(j);
            if (e == T(0)) continue;
            ex += e * K[j * kst + fo];
            ey += e * K[j * kst + fo + plane];
            ez += e * K[j * kst + fo + 2 * plane];
          }
          const T e6 = (T)dp_e(6);
          ex = hdt * (ex + e6 * kx);
          ey = hdt * (ey + e6 * ky);
          ez = hdt * (ez + e6 * kz);
          const double en = sqrt((double)ex * ex + (double)ey * ey + (double)ez * ez);
          errmax = (en > errmax || en != en) ? en : errmax;
        }
      } else if (stage == 0) {
        acc[fo] = kx;
        acc[fo + plane] = ky;
        acc[fo + 2 * plane] = kz;
        const T c = T(0.5) * hdt;
        mnext[fo] = ox + c * kx;
        mnext[fo + plane] = oy + c * ky;
        mnext[fo + 2 * plane] = oz + c * kz;
        if (fuse) {
          fr[i] = ox + c * kx;
          fr[Lx + i] = oy + c * ky;
          fr[2 * Lx + i] = oz + c * kz;
        }
      } else if (stage < 3) {
        acc[fo] += T(2) * kx;
        acc[fo + plane] += T(2) * ky;
        acc[fo + 2 * plane] += T(2) * kz;
        const T c = (stage == 1) ? T(0.5) * hdt : hdt;
        mnext[fo] = ox + c * kx;
        mnext[fo + plane] = oy + c * ky;
        mnext[fo + 2 * plane] = oz + c * kz;
        if (fuse) {
          fr[i] = ox + c * kx;
          fr[Lx + i] = oy + c * ky;
          fr[2 * Lx + i] = oz + c * kz;
        }
      } else {
        const T c = hdt / T(6);
        T nx_ = ox + c * (acc[fo] + kx);
        T ny_ = oy + c * (acc[fo + plane] + ky);
        T nz_ = oz + c * (acc[fo + 2 * plane] + kz);
        const T nrm = sqrt(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
        if (!(nrm > T(0)) || !isfinite(nrm)) bad = true;
        const T inv = T(1) / nrm;
        mnext[fo] = nx_ * inv;
        mnext[fo + plane] = ny_ * inv;
        mnext[fo + 2 * plane] = nz_ * inv;
        if (fuse) {
          fr[i] = nx_ * inv;
          fr[Lx + i] = ny_ * inv;
          fr[2 * Lx + i] = nz_ * inv;
        }
      }
    }
  }
  if (fuse) {
    // forward real transform of the three rows (as the x pass computes it)
    lds_barrier();
    const cpx<T>* Z = row_fft<T, false, NT, INPL>(fa, fb, p.px, 3, stw);
    cpx<T>* dst = gptr(reinterpret_cast<cpx<T>*>(p.spec1_out));
    const int K1 = N2x + 1;
#pragma unroll 1
    for (int t = threadIdx.x; t < 3 * K1; t += NT) {
      const int r = t / K1;
      const int k = t - r * K1;
      const cpx<T>* z = Z + (size_t)r * N2x;
      cpx<T> zk = z[k == N2x ? 0 : k];
      cpx<T> zm = z[k == 0 ? 0 : N2x - k];
      zm.y = -zm.y;
      const cpx<T> e = zk + zm;
      const cpx<T> q = cmul(stp[k], zk - zm);
      dst[((size_t)(film * 3 + r) * p.Kx + k) * ny + y] = mk<T>(T(0.5) * (e.x + q.y), T(0.5) * (e.y - q.x));
    }
  }
  if (need_force) {
    // Eq. (3), component a: sum_i m_x d_x G_a + m_y d_y G_a + m_z d_z G_a,
    // the y term summed by parts over rows -1..ny.
    const double i2dx = 1.0 / (2.0 * p.dx), i2dy = 1.0 / (2.0 * p.dy), i2dz = 1.0 / (2.0 * p.dz);
    // neighbouring rows of m_y (wrapped along a periodic y: no boundary rows)
    const int yl = pbc_y ? (y - 1 + ny) % ny : y - 1, yh = pbc_y ? (y + 1) % ny : y + 1;
#pragma unroll 1
    for (int i = threadIdx.x; i < nx; i += NT) {
      const double myl = (yl >= 0 && yl < ny) ? (double)ms[plane + (size_t)yl * nx + i] : 0.0;
      const double myh = (yh >= 0 && yh < ny) ? (double)ms[plane + (size_t)yh * nx + i] : 0.0;
      double mx = 0, mz = 0;
      if (cell_row) {
        mx = ms[(size_t)y * nx + i];
        mz = ms[2 * plane + (size_t)y * nx + i];
      }
      for (int a = 0; a < nfc; ++a) {
        const T* ga = gc + a * (nx + 2);
        double v = (double)ga[i + 1] * (myl - myh) * i2dy;
        if (cell_row) {
          v += mx * ((double)ga[i + 2] - (double)ga[i]) * i2dx;
          v += mz * ((double)gp[a * nx + i] - (fm_split ? 0.0 : (double)gm[a * nx + i])) * i2dz;
        }
        fpart[a] += v;
      }
      // rows -1 and ny: m_y is zero outside the film
      if (xb_lo) fpart[0] -= (double)gxb[i] * (double)ms[plane + i] * i2dy;
      if (xb_hi) fpart[0] += (double)gxb[nx + i] * (double)ms[plane + (size_t)(ny - 1) * nx + i] * i2dy;
    }
  }
  if (fm_here) {
    // the slider's m_z at row y times the base field's x component on the
    // layer below it (the z_s - 1 half of the central difference)
    const double i2dz = 1.0 / (2.0 * p.dz);
    const T* mz1 = mst + (size_t)5 * plane + (size_t)y * nx;
#pragma unroll 1
    for (int i = threadIdx.x; i < nx; i += NT) fpart[0] -= (double)mz1[i] * (double)gm[i] * i2dz;
  }
  if (bad) atomicOr(&s_bad, 1);
  // block reduction of the force partials, fixed order: within each wave,
  // then over the waves
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (NT + 63) >> 6;
  for (int a = 0; a < 3; ++a) {
    const double v = wave_sum(fpart[a]);
    if (lane == 0) red[wv * 3 + a] = v;
  }
  lds_barrier();
  if (p.mode == MODE_EVAL) return;
  if (p.mode == MODE_STAGE && p.scheme == 1 && stage == 6) {
    // the block's largest error (a maximum: independent of order)
    double e = errmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double q = __shfl_down(e, o, 64);
      e = (q > e || q != q) ? q : e;
    }
    if (lane == 0) red[48 + wv] = e;
    lds_barrier();
    if (threadIdx.x == 0) {
      double m = 0.0;
      for (int w = 0; w < nw; ++w) m = (red[48 + w] > m || red[48 + w] != red[48 + w]) ? red[48 + w] : m;
      gptr(p.errpart)[task] = m;
    }
  }
  if (p.mode == MODE_STAGE && p.defer_tick) {
    // partials only; the slider update runs after this launch
    if (threadIdx.x == 0) {
      for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        for (int w = 0; w < nw; ++w) v += red[w * 3 + a];
        partial[(size_t)task * 3 + a] = v;
      }
      if (s_bad || xp_bad) atomicOr(&rigid->flags, s_bad ? (int)FLAG_NUMERIC : (int)FLAG_RANGE);
    }
    return;
  }
  if (threadIdx.x == 0) {
    for (int a = 0; a < 3; ++a) {
      double v = 0.0;
      for (int w = 0; w < nw; ++w) v += red[w * 3 + a];
      partial[(size_t)task * 3 + a] = v;
    }
    if (s_bad || xp_bad) atomicOr(&rigid->flags, s_bad ? (int)FLAG_NUMERIC : (int)FLAG_RANGE);
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == (unsigned)ntask - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double sum[3] = {0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < ntask; t += NT)
    for (int a = 0; a < 3; ++a)
      sum[a] += __hip_atomic_load(&partial[(size_t)t * 3 + a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int a = 0; a < 3; ++a) {
    const double v = wave_sum(sum[a]);
    if (lane == 0) red[48 + wv * 3 + a] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[3];
    for (int a = 0; a < 3; ++a) {
      tot[a] = 0.0;
      for (int w = 0; w < nw; ++w) tot[a] += red[48 + w * 3 + a];
    }
    const double F0 = p.force_scale * tot[0];
    if (p.mode == MODE_FORCE) {
      double* Fo = p.fout != nullptr ? gptr(p.fout) : rigid->F;
      for (int a = 0; a < 3; ++a) Fo[a] = p.force_scale * tot[a];
    } else {
      rigid_stage(rigid, p.drive, stage, F0, dt, p.dx, p.travel);
    }
    __threadfence();
    atomicExch(counter, 0u);
  }
}

template <typename T, bool INPL>
__global__ void __launch_bounds__((RowThreads<T, false>::n))
    k_row_stage(RowParams p, const cpx<T>* __restrict__ spec2, const T* __restrict__ mst, const T* m0, T* mnext,
                T* __restrict__ acc, T* __restrict__ hout, const cpx<T>* __restrict__ tw,
                const cpx<T>* __restrict__ twp, RigidState* __restrict__ rigid, double* __restrict__ partial,
                unsigned int* __restrict__ counter) {
  // XCD-contiguous tasks: the column-major spectrum writes of neighbouring
  // rows meet in one L2
  row_stage_body<T, RowThreads<T, false>::n, INPL>(p, p.stage, p.dt, xcd_remap(blockIdx.x, gridDim.x), gridDim.x,
                                                    spec2, mst, m0, mnext, acc, hout, tw, twp, rigid, partial,
                                                    counter);
}

// NT: 512, or 128 / 256 for the float32 in-place classes of short rows
// (more blocks per CU; the batch picks it per row length, never below nx, so
// every thread sums at most one cell of the force and the sums equal those
// of the single-mesh kernel bit for bit).
template <typename T, bool INPL, int NT>
__global__ void __launch_bounds__(NT) k_row_stage_batch(const RowStageDesc* __restrict__ d,
                                                        const int* __restrict__ start, int n, int stage, double dt) {
  const int bl = xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_instance(start, n, bl);
  const RowStageDesc& q = d[i];
  row_stage_body<T, NT, INPL>(q.p, stage, dt, bl - start[i], start[i + 1] - start[i], gptr((const cpx<T>*)q.spec2),
                              gptr((const T*)q.mst), gptr((const T*)q.m0), gptr((T*)q.mnext), gptr((T*)q.acc),
                              nullptr, gptr((const cpx<T>*)q.tw), gptr((const cpx<T>*)q.twp), gptr(q.rigid),
                              gptr(q.partial), gptr(q.counter));
}

// ------------------------------------------------------------ kernel init (float64)
// Real kernel on the cyclic Lx x Ly grid of one layer (dzc cells apart):
// displacement index r maps to r (r <= L/2) or r - L; odd components are
// zeroed on the Nyquist index of an even length so that every spectrum is
// purely real or imaginary.
// Periodic axes (pbc bit 0 = x, 1 = y; the transform length is then the
// period): the displacement on the cyclic grid is its minimum image, and the
// kernel is summed over `images` repetitions of the period on each side.
__global__ void k_kernel_real(double* __restrict__ out, int Lx, int Ly, int kind, int comp, double dzc,
                              double dx, double dy, double dz, double rc, double scale, int pbc, int images) {
  const int ry = blockIdx.y;
  if (ry >= Ly) return;
  for (int rx = blockIdx.x * blockDim.x + threadIdx.x; rx < Lx; rx += gridDim.x * blockDim.x) {
  const int ix = rx <= Lx / 2 ? rx : rx - Lx;
  const int iy = ry <= Ly / 2 ? ry : ry - Ly;
  int oddx, oddy;
  double v;
  if (kind == 0) {
    const int px[6] = {0, 0, 0, 1, 1, 0}, py[6] = {0, 0, 0, 1, 0, 1};
    oddx = px[comp];
    oddy = py[comp];
    const int qx = (pbc & 1) ? images : 0, qy = (pbc & 2) ? images : 0;
    v = 0.0;
    for (int a = -qx; a <= qx; ++a)
      for (int b = -qy; b <= qy; ++b)
        v += tensor_comp(comp, (ix + a * Lx) * dx, (iy + b * Ly) * dy, dzc * dz, dx, dy, dz, rc);
  } else {
    oddx = (comp == 0);
    oddy = (comp == 1);
    const int qx = (pbc & 1) ? images : 0, qy = (pbc & 2) ? images : 0;
    v = 0.0;
    for (int a = -qx; a <= qx; ++a)
      for (int b = -qy; b <= qy; ++b) v += s_comp(comp, (ix + a * Lx) * dx, (iy + b * Ly) * dy, dzc * dz, dx, dy, dz);
  }
  if ((Lx % 2 == 0 && rx == Lx / 2 && oddx) || (Ly % 2 == 0 && ry == Ly / 2 && oddy)) v = 0.0;
  out[(size_t)ry * Lx + rx] = scale * v;
  }
}

// y transform of the row spectra of a real kernel, keeping the real or
// imaginary part for ky in [0, Kyh).
template <typename T>
__global__ void __launch_bounds__(COLPACK_THREADS)
    k_colpack(const cpx<double>* __restrict__ spec, T* __restrict__ out, int Kx, int Ly, int Kyh,
              FftPlan P, const cpx<double>* __restrict__ twy, int imag) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<double>* stw = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* a = stw + Ly;
  cpx<double>* b = a + Ly;
  const int kx = blockIdx.x;
  for (int t = threadIdx.x; t < Ly; t += COLPACK_THREADS) {
    stw[t] = twy[t];
    a[t] = spec[(size_t)t * Kx + kx];
  }
  __syncthreads();
  cpx<double>* Y = fft_lds<double, false, COLPACK_THREADS>(a, b, P, 1, Ly, stw);
  for (int t = threadIdx.x; t < Kyh; t += COLPACK_THREADS) out[(size_t)kx * Kyh + t] = (T)(imag ? Y[t].y : Y[t].x);
}

// ------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_row_fwd(const T* src, void* dst, int nrows, int nin, int N2x, int Kx, const FftPlan& P,
                          const void* tw, const void* twp, hipStream_t st, int ny3) {
  const int nb = ny3 > 0 ? 3 : ny3 < 0 ? -ny3 : 1;
  const size_t lds = sizeof(cpx<T>) * (2 * (size_t)N2x + 1 + 2 * (size_t)nb * N2x);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_row_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int nblk = ny3 > 0 ? nrows / 3 : ny3 < 0 ? (nrows - ny3 - 1) / -ny3 : nrows;
  hipLaunchKernelGGL(k_row_fwd<T>, dim3(nblk), dim3(FWD_THREADS), lds, st, src, (cpx<T>*)dst, nrows, nin, N2x, Kx,
                     P, (const cpx<T>*)tw, (const cpx<T>*)twp, ny3);
  return hipGetLastError();
}

template <typename T>
size_t col_lds_bytes(int Ly, int nbuf) {
  const size_t Lh = (Ly & 1) ? Ly : Ly / 2;
  return sizeof(cpx<T>) * (Lh + 2 * (size_t)nbuf * Ly);
}

// Resident blocks per CU of the y-pass kernel (256 threads = 4 waves, one
// per SIMD) at `lds` bytes of dynamic LDS on a CDNA CU: 160 KiB of LDS
// (512-byte granules), 512 VGPRs per SIMD lane (8-register granules), at
// most 8 waves per SIMD.
template <typename T>
int col_blocks_per_cu(size_t lds) {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, (const void*)k_col<T>) != hipSuccess) return 0;
  const size_t per = ((lds + a.sharedSizeBytes + 511) / 512) * 512;
  const int by_lds = (int)((160 * 1024) / per);
  if (getenv("MMV_VERBOSE"))
    fprintf(stderr, "mmv: k_col registers %d, static LDS %zu\n", a.numRegs, (size_t)a.sharedSizeBytes);
  const int vg = ((a.numRegs > 0 ? a.numRegs : 128) + 7) / 8 * 8;
  int waves = 512 / vg;
  if (waves > 8) waves = 8;
  return by_lds < waves ? by_lds : waves;
}

template <typename T>
bool static_lds_within_reserve() {
  hipFuncAttributes a{};
  constexpr int NB = RowThreads<T, true>::n;
  for (const void* k : {(const void*)k_row_stage<T, false>, (const void*)k_row_stage<T, true>,
                        (const void*)k_row_stage_batch<T, false, NB>, (const void*)k_row_stage_batch<T, true, NB>,
                        (const void*)k_row_stage_batch<T, true, 128>, (const void*)k_row_stage_batch<T, true, 256>}) {
    if (hipFuncGetAttributes(&a, k) != hipSuccess || a.sharedSizeBytes > ROW_STATIC_LDS) return false;
  }
  for (const void* k : {(const void*)k_col<T>, (const void*)k_col_batch<T>}) {
    if (hipFuncGetAttributes(&a, k) != hipSuccess || a.sharedSizeBytes > COL_STATIC_LDS) return false;
  }
  return true;
}

template <typename T>
hipError_t launch_col(const void* spec1, void* spec2, const T* kern, int Kx, int Ly, int Kyh, int ny,
                      int nin_ch, int ngroup, const FftPlan& P, const void* twy, const OutTable& tab,
                      hipStream_t st, const TickArgs* tick, int tick_stage, double tick_dt) {
  const int per = (tab.n + ngroup - 1) / ngroup;
  const int nbuf = nin_ch > per ? nin_ch : per;
  const size_t lds = col_lds_bytes<T>(Ly, nbuf);
  const int nblk = Kx * ngroup;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_col<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  TickArgs ta{};
  if (tick) ta = *tick;
  hipLaunchKernelGGL(k_col<T>, dim3(nblk), dim3(COL_THREADS), lds, st, (const cpx<T>*)spec1, (cpx<T>*)spec2, kern, Kx,
                     Ly, Kyh, ny, nin_ch, ngroup, nbuf, P, (const cpx<T>*)twy, tab, ta, tick ? tick_stage : -1,
                     tick_dt);
  return hipGetLastError();
}

hipError_t launch_tick(const TickArgs& tick, int stage, double dt, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(TICK_THREADS), 0, st, tick, stage, dt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div_curl(const T* G, int nx, int ny, double dx, double dy, double dz, int pbc_y, double* part,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_div_curl<T>, dim3(ny), dim3(256), 0, st, G, nx, ny, dx, dy, dz, pbc_y, part);
  return hipGetLastError();
}

hipError_t launch_dp_control(const TickArgs& tick, DpCtrl* ctrl, const double* errpart, int ntask, hipStream_t st) {
  hipLaunchKernelGGL(k_dp_control, dim3(1), dim3(TICK_THREADS), 0, st, tick, ctrl, errpart, ntask);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dp_commit(const T* y5, T* m, int nfilm, size_t plane, const DpCtrl* ctrl, int* flags,
                            hipStream_t st) {
  const size_t n = (size_t)nfilm * plane;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_dp_commit<T>, dim3(nb), dim3(256), 0, st, y5, m, nfilm, plane, ctrl, flags);
  return hipGetLastError();
}

hipError_t launch_tick_batch(const ColDesc* d, int n, int stage, double dt, hipStream_t st) {
  hipLaunchKernelGGL(k_tick_batch, dim3(n), dim3(TICK_THREADS), 0, st, d, stage, dt);
  return hipGetLastError();
}

template <typename T>
size_t row_lds_bytes(const RowParams& p) {
  const int K = FirHalf<T>::K, NQ = 2 * K + 4, E = K + 4;
  const int nfc = p.full_force ? 3 : 1;
  size_t b = sizeof(cpx<T>) * (size_t)(2 * p.N2x + 1 + (p.inplace ? 1 : 2) * (size_t)p.nbr * p.N2x);
  const int nslot = p.pot ? (p.full_force ? 19 : 9) : 0;
  b += sizeof(T) * ((size_t)p.nbr * ((p.M + 2 * E + 5) & ~1) + 2 * NQ + 3 * p.nx + 3 * (p.nx + 2) + 2 * nfc * p.nx +
                    (size_t)nslot * (p.nx + 6) + 2 * (size_t)p.nx + 2) + 16;  // + alignment of the weights
  b = (b + 15) & ~size_t(15);
  b += sizeof(double) * (96 + 8 * NQ) + 16;  // wave partials of the force reduction, spline-weight terms
  return b;
}

template <typename T>
hipError_t launch_row_stage(const RowParams& p, const void* spec2, const T* mst, const T* m0, T* mnext, T* acc,
                            T* hout, const void* tw, const void* twp, RigidState* rigid, double* partial,
                            unsigned* counter, hipStream_t st) {
  const size_t lds = row_lds_bytes<T>(p);
  const void* kf = p.inplace ? (const void*)k_row_stage<T, true> : (const void*)k_row_stage<T, false>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (p.inplace)
    hipLaunchKernelGGL((k_row_stage<T, true>), dim3(p.ntask), dim3(RowThreads<T, false>::n), lds, st, p,
                       (const cpx<T>*)spec2, mst, m0, mnext, acc, hout, (const cpx<T>*)tw, (const cpx<T>*)twp, rigid,
                       partial, counter);
  else
    hipLaunchKernelGGL((k_row_stage<T, false>), dim3(p.ntask), dim3(RowThreads<T, false>::n), lds, st, p,
                       (const cpx<T>*)spec2, mst, m0, mnext, acc, hout, (const cpx<T>*)tw, (const cpx<T>*)twp, rigid,
                       partial, counter);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_fwd_batch(const RowFwdDesc* d, const int* start, int n, int nblk, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_row_fwd_batch<T>, dim3(nblk), dim3(FWD_THREADS), lds, st, d, start, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_batch(const ColDesc* d, const int* start, int n, int nblk, size_t lds, hipStream_t st,
                            int tick_stage, double tick_dt) {
  hipLaunchKernelGGL(k_col_batch<T>, dim3(nblk), dim3(COL_THREADS), lds, st, d, start, n, tick_stage, tick_dt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_stage_batch(const RowStageDesc* d, const int* start, int n, int nblk, size_t lds, int stage,
                                  double dt, bool inplace, int nt, hipStream_t st) {
  constexpr int NB = RowThreads<T, true>::n;
  if (!inplace) {
    hipLaunchKernelGGL((k_row_stage_batch<T, false, NB>), dim3(nblk), dim3(NB), lds, st, d, start, n, stage, dt);
    return hipGetLastError();
  }
  if constexpr (sizeof(T) == 4) {
    if (nt == 128) {
      hipLaunchKernelGGL((k_row_stage_batch<T, true, 128>), dim3(nblk), dim3(128), lds, st, d, start, n, stage, dt);
      return hipGetLastError();
    }
    if (nt == 256) {
      hipLaunchKernelGGL((k_row_stage_batch<T, true, 256>), dim3(nblk), dim3(256), lds, st, d, start, n, stage, dt);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_row_stage_batch<T, true, NB>), dim3(nblk), dim3(NB), lds, st, d, start, n, stage, dt);
  return hipGetLastError();
}

template <typename T>
bool row_batch_threads_ok(int nt, bool inplace) {
  constexpr int NB = RowThreads<T, true>::n;
  if (nt == NB) return true;
  return sizeof(T) == 4 && inplace && (nt == 128 || nt == 256);
}

// Dynamic-LDS limits of the batched kernels, set outside any graph capture.
template <typename T>
hipError_t prepare_batch_kernels(size_t lds_fwd, size_t lds_col, size_t lds_stage) {
  hipError_t e = hipSuccess;
  if (lds_fwd > 65536)
    e = hipFuncSetAttribute((const void*)k_row_fwd_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_fwd);
  if (e == hipSuccess && lds_col > 65536)
    e = hipFuncSetAttribute((const void*)k_col_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_col);
  constexpr int NB = RowThreads<T, true>::n;
  for (const void* k : {(const void*)k_row_stage_batch<T, false, NB>, (const void*)k_row_stage_batch<T, true, NB>,
                        (const void*)k_row_stage_batch<T, true, 128>, (const void*)k_row_stage_batch<T, true, 256>})
    if (e == hipSuccess && lds_stage > 65536)
      e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_stage);
  return e;
}

bool row_inplace_length(int L) { return inplace_length(L); }

size_t row_fwd_lds_bytes(int N2x, int esz) { return (size_t)2 * esz * (8 * (size_t)N2x + 1); }

hipError_t launch_kernel_real(double* out, int Lx, int Ly, int kind, int comp, double dzc, double dx, double dy,
                              double dz, double rc, double scale, int pbc, int images, hipStream_t st) {
  dim3 grid((Lx + 127) / 128, Ly);
  hipLaunchKernelGGL(k_kernel_real, grid, dim3(128), 0, st, out, Lx, Ly, kind, comp, dzc, dx, dy, dz, rc, scale,
                     pbc, images);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_colpack(const void* spec, T* out, int Kx, int Ly, int Kyh, const FftPlan& P, const void* twy,
                          int imag, hipStream_t st) {
  const size_t lds = sizeof(cpx<double>) * 3 * (size_t)Ly;
  hipLaunchKernelGGL(k_colpack<T>, dim3(Kx), dim3(COLPACK_THREADS), lds, st, (const cpx<double>*)spec, out, Kx, Ly, Kyh, P,
                     (const cpx<double>*)twy, imag);
  return hipGetLastError();
}

#define MMV_INST(T)                                                                                             \
  template hipError_t launch_row_fwd<T>(const T*, void*, int, int, int, int, const FftPlan&, const void*,      \
                                        const void*, hipStream_t, int);                                             \
  template hipError_t launch_col<T>(const void*, void*, const T*, int, int, int, int, int, int, const FftPlan&, \
                                    const void*, const OutTable&, hipStream_t, const TickArgs*, int, double);  \
  template hipError_t launch_row_stage<T>(const RowParams&, const void*, const T*, const T*, T*, T*, T*,       \
                                          const void*, const void*, RigidState*, double*, unsigned*,           \
                                          hipStream_t);                                                        \
  template hipError_t launch_colpack<T>(const void*, T*, int, int, int, const FftPlan&, const void*, int,      \
                                        hipStream_t);                                                          \
  template size_t row_lds_bytes<T>(const RowParams&);                                                           \
  template size_t col_lds_bytes<T>(int, int);                                                                    \
  template int col_blocks_per_cu<T>(size_t);\
  template bool static_lds_within_reserve<T>();                                                                     \
  template hipError_t prepare_batch_kernels<T>(size_t, size_t, size_t);                                         \
  template hipError_t launch_row_fwd_batch<T>(const RowFwdDesc*, const int*, int, int, size_t, hipStream_t);      \
  template hipError_t launch_col_batch<T>(const ColDesc*, const int*, int, int, size_t, hipStream_t, int, double);             \
  template hipError_t launch_row_stage_batch<T>(const RowStageDesc*, const int*, int, int, size_t, int, double,   \
                                                bool, int, hipStream_t);                                        \
  template bool row_batch_threads_ok<T>(int, bool);                                                             \
  template hipError_t launch_dp_commit<T>(const T*, T*, int, size_t, const DpCtrl*, int*, hipStream_t);         \
  template hipError_t launch_div_curl<T>(const T*, int, int, double, double, double, int, double*, hipStream_t);

MMV_INST(float)
MMV_INST(double)

}  // namespace mmv
