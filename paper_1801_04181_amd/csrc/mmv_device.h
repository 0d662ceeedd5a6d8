// Device-side building blocks: complex arithmetic, mixed-radix Stockham FFT
// passes in LDS, XCD-aware block remapping.
#pragma once
#include <hip/hip_runtime.h>
#include "mmv_internal.h"

namespace mmv {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }

// Blocks are dispatched round-robin over the 8 XCDs.  Map the hardware block
// id to a logical id so that each XCD works on one contiguous range of
// logical ids (neighbouring columns / rows then share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int nx = 8;
  int per = G / nx, rem = G % nx;
  int x = b % nx, local = b / nx;
  return (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// ---------------------------------------------------------------- small DFTs
// cos / sin of 2 pi m / R for m = 1..(R-1)/2.
template <int R> struct Roots;
template <> struct Roots<3> {
  static __device__ __forceinline__ double c(int m) { return -0.5; }
  static __device__ __forceinline__ double s(int m) { return 0.86602540378443864676; }
};
template <> struct Roots<5> {
  static __device__ __forceinline__ double c(int m) {
    return m == 1 ? 0.3090169943749474241 : -0.8090169943749474241;
  }
  static __device__ __forceinline__ double s(int m) {
    return m == 1 ? 0.95105651629515357212 : 0.58778525229247312917;
  }
};
template <> struct Roots<7> {
  static __device__ __forceinline__ double c(int m) {
    return m == 1 ? 0.62348980185873353053 : (m == 2 ? -0.22252093395631440429 : -0.90096886790241912624);
  }
  static __device__ __forceinline__ double s(int m) {
    return m == 1 ? 0.78183148246802980871 : (m == 2 ? 0.97492791218182360702 : 0.43388373911755812048);
  }
};

template <> struct Roots<9> {
  static __device__ __forceinline__ double c(int m) {
    return m == 1 ? 0.766044443118978035202
                  : (m == 2 ? 0.173648177666930348852 : (m == 3 ? -0.5 : -0.939692620785908384054));
  }
  static __device__ __forceinline__ double s(int m) {
    return m == 1 ? 0.642787609686539326323
                  : (m == 2 ? 0.984807753012208059367 : (m == 3 ? 0.866025403784438646764 : 0.342020143325668733044));
  }
};

// In-register DFT of odd length R, forward (e^{-2 pi i rq/R}) or inverse.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_odd(cpx<T>* v) {
  constexpr int H = (R - 1) / 2;
  cpx<T> s[H], d[H];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    s[r - 1] = v[r] + v[R - r];
    d[r - 1] = v[r] - v[R - r];
  }
  cpx<T> out[R];
  cpx<T> o0 = v[0];
#pragma unroll
  for (int r = 0; r < H; ++r) o0 = o0 + s[r];
  out[0] = o0;
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    cpx<T> A = v[0];
    cpx<T> B = mk<T>(0, 0);
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      int m = (r * q) % R;
      T c, sn;
      if (m == 0) {  // composite R (9): r q can be a multiple of R
        c = T(1);
        sn = T(0);
      } else if (m <= H) {
        c = (T)Roots<R>::c(m);
        sn = (T)Roots<R>::s(m);
      } else {
        c = (T)Roots<R>::c(R - m);
        sn = -(T)Roots<R>::s(R - m);
      }
      A = A + scale(s[r - 1], c);
      B = B + scale(d[r - 1], sn);
    }
    if (!INV) {
      out[q] = mk(A.x + B.y, A.y - B.x);
      out[R - q] = mk(A.x - B.y, A.y + B.x);
    } else {
      out[q] = mk(A.x - B.y, A.y + B.x);
      out[R - q] = mk(A.x + B.y, A.y - B.x);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = out[r];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cpx<T> t2 = v[1] + v[3], d = v[1] - v[3];
    // forward: t3 = -i d ; inverse: t3 = +i d
    cpx<T> t3 = INV ? mk(-d.y, d.x) : mk(d.y, -d.x);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
  } else if constexpr (R == 8) {
    // two length-4 DFTs of the even and odd samples, odd half twiddled by
    // w^k = exp(-+2 pi i k / 8), combined as X[k], X[k + 4] = e_k +- w^k o_k
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft<T, 4, INV>(e);
    dft<T, 4, INV>(o);
    const T h = T(0.70710678118654752440);
    const cpx<T> o1 = INV ? mk((o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h)
                          : mk((o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h);
    const cpx<T> o2 = INV ? mk(-o[2].y, o[2].x) : mk(o[2].y, -o[2].x);
    const cpx<T> o3 = INV ? mk((-o[3].x - o[3].y) * h, (o[3].x - o[3].y) * h)
                          : mk((o[3].y - o[3].x) * h, (-o[3].x - o[3].y) * h);
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  } else if constexpr (R == 6) {
    // prime-factor 2 x 3 (no twiddles): inputs n = (3 n1 + 2 n2) mod 6,
    // outputs k = (3 k1 + 4 k2) mod 6
    cpx<T> a[3] = {v[0], v[2], v[4]};
    cpx<T> b[3] = {v[3], v[5], v[1]};
    dft_odd<T, 3, INV>(a);
    dft_odd<T, 3, INV>(b);
    v[0] = a[0] + b[0];
    v[3] = a[0] - b[0];
    v[4] = a[1] + b[1];
    v[1] = a[1] - b[1];
    v[2] = a[2] + b[2];
    v[5] = a[2] - b[2];
  } else {
    dft_odd<T, R, INV>(v);
  }
}

// Exact quotient floor(n / d) for 0 <= n < 2^20, 1 <= d < 2^20 from a float
// reciprocal: (n + 1/2) / d lies at least 1/(2d) from an integer, far more
// than the float rounding of the product.
__device__ __forceinline__ int fdiv(int n, float inv_d) { return (int)(((float)n + 0.5f) * inv_d); }

// dst[t] = load(t) for t < n, block-strided over the NT threads of the
// block, with U independent loads in flight per thread before the first
// store (one global-memory latency per U elements instead of one per
// element).
//
// Every device helper takes the block size NT as a compile-time constant:
// the runtime block size lives in the dispatch's hidden arguments, and the
// compiler re-reads it with a vector load after each barrier.
template <int U, int NT, typename V, typename F>
__device__ __forceinline__ void stage_copy(V* dst, int n, F load) {
#pragma unroll 1
  for (int t0 = threadIdx.x; t0 < n; t0 += U * NT) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * NT;
      if (t < n) v[u] = load(t);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * NT;
      if (t < n) dst[t] = v[u];
    }
  }
}

// As stage_copy, for a destination that is not dst[t]: store(t, load(t)).
template <int U, int NT, typename F, typename S>
__device__ __forceinline__ void stage_move(int n, F load, S store) {
  using V = decltype(load(0));
#pragma unroll 1
  for (int t0 = threadIdx.x; t0 < n; t0 += U * NT) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * NT;
      if (t < n) v[u] = load(t);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * NT;
      if (t < n) store(t, v[u]);
    }
  }
}

// Block barrier for data exchanged through LDS only.  It waits for this
// wave's LDS operations but not for its global loads: on this architecture
// the workgroup fence of __syncthreads() waits for every outstanding
// vector-memory operation, loads included, so a load issued ahead of its use
// could not stay in flight across a barrier.  Not a fence for global memory.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// threadIdx.x, opaque to the optimiser: index arithmetic derived from it
// is then recomputed where it is used instead of being hoisted out of an
// enclosing loop and kept live (in registers or spilled) across it.
__device__ __forceinline__ int local_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// A pointer read from memory (a batch descriptor, a parameter struct in
// device memory) is a generic pointer to the compiler, and its loads and
// stores become flat instructions (both wait counters, full 64-bit
// addresses).  Every such pointer here addresses device global memory; the
// round trip through the global address space lets the compiler emit global
// instructions instead.
template <typename P>
__device__ __forceinline__ P* gptr(P* p) {
  typedef __attribute__((address_space(1))) P GP;
  return (P*)(GP*)(unsigned long long)p;
}

// Sum over the 64 lanes of a wave; the total is returned in lane 0.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// One radix-R Stockham pass over `batch` transforms of length L at stride
// `stride`: reads src[j + r*nb], twiddles by exp(-+2 pi i r k / (Ns R)),
// DFT_R, writes dst[(j - k) R + k + r Ns] with k = j mod Ns.
// tw[t] = exp(-2 pi i t / L).  Threads are spread over (butterfly j,
// transform group g); a thread reuses its index arithmetic and twiddles for
// every transform t = g, g + G, ... of its group.  twh > 0: only tw[0..twh)
// is stored (L = 2 twh) and tw[t + twh] = -tw[t].
template <typename T, int R, bool INV, int NT>
__device__ __forceinline__ void stockham_pass(const cpx<T>* __restrict__ a, cpx<T>* __restrict__ b, int L,
                                              int Ns, int batch, int stride,
                                              const cpx<T>* __restrict__ tw, int twh) {
  const int nb = L / R;
  const int tws = L / (Ns * R);
  int G = NT / nb;
  if (G < 1) G = 1;
  if (G > batch) G = batch;
  const float inb = 1.0f / (float)nb;
  const float ins = 1.0f / (float)Ns;
  const int total = nb * G;
#pragma unroll 1
  for (int w = local_tid(); w < total; w += NT) {
    const int g = fdiv(w, inb);
    const int j = w - g * nb;
    const int q = fdiv(j, ins);
    const int k = j - q * Ns;
    cpx<T> wv[R];
    if (k) {
      const int kt = k * tws;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        // branch-free: one load from the stored half, sign by select
        const int id = r * kt;
        const bool hi = twh != 0 && id >= twh;
        const cpx<T> w = tw[hi ? id - twh : id];
        wv[r] = hi ? mk(-w.x, -w.y) : w;
      }
    }
    const int din = j;
    const int dout = q * Ns * R + k;
    for (int t = g; t < batch; t += G) {
      const cpx<T>* s = a + t * stride + din;
      cpx<T>* d = b + t * stride + dout;
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = s[r * nb];
      if (k) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], wv[r]) : cmul(v[r], wv[r]);
      }
      dft<T, R, INV>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) d[r * Ns] = v[r];
    }
  }
}

// ---------------------------------------------------------------- compile-time plans
// For the lengths the workloads use, the radix plan, butterfly counts, thread
// mapping and LDS strides are compile-time constants: index arithmetic folds,
// LDS accesses take immediate offsets.  Radices: 7, 5, then 3s paired into 9,
// then 4s, and a remaining 2 paired with a 3 into 6; a power of two takes
// 8s, then a 4 or a 2.
struct CPlan {
  int np;
  int r[12];
};

constexpr CPlan make_cplan(int L) {
  CPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int n = L, n3 = 0, n2 = 0;
  while (n % 7 == 0) { p.r[p.np++] = 7; n /= 7; }
  while (n % 5 == 0) { p.r[p.np++] = 5; n /= 5; }
  while (n % 3 == 0) { ++n3; n /= 3; }
  while (n % 2 == 0) { ++n2; n /= 2; }
  if (n == 1 && p.np == 0 && n3 == 0) {  // power of two
    while (n2 >= 3) { p.r[p.np++] = 8; n2 -= 3; }
    if (n2 > 0) p.r[p.np++] = n2 == 2 ? 4 : 2;
    return p;
  }
  if (n2 % 2 == 1 && n3 > 0) { p.r[p.np++] = 6; --n3; --n2; }
  while (n3 >= 2) { p.r[p.np++] = 9; n3 -= 2; }
  if (n3 == 1) p.r[p.np++] = 3;
  while (n2 >= 2) { p.r[p.np++] = 4; n2 -= 2; }
  if (n2 == 1) p.r[p.np++] = 2;
  return p;
}

// One radix-R pass of `batch` contiguous transforms of length L with NT
// threads per block (butterflies are block-strided).
// HALF: only tw[0..L/2) is stored and tw[t + L/2] = -tw[t].
template <typename T, int L, int NT, int R, int Ns, bool INV, bool HALF>
__device__ __forceinline__ void stockham_ct(const cpx<T>* __restrict__ a, cpx<T>* __restrict__ b, int batch,
                                            const cpx<T>* __restrict__ tw) {
  constexpr int nb = L / R;
  constexpr int G = NT / nb >= 1 ? NT / nb : 1;
  constexpr int tws = L / (Ns * R);
#pragma unroll 1
  for (int w = local_tid(); w < nb * G; w += NT) {
    const int g = w / nb;
    const int j = w - g * nb;
    const int q = j / Ns;
    const int k = j - q * Ns;
    cpx<T> wv[R];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int id = r * k * tws;
        if constexpr (HALF) {
          const bool hi = id >= L / 2;
          const cpx<T> x = tw[hi ? id - L / 2 : id];
          wv[r] = hi ? mk(-x.x, -x.y) : x;
        } else {
          wv[r] = tw[id];
        }
      }
    }
    const cpx<T>* s0 = a + j;
    cpx<T>* d0 = b + q * Ns * R + k;
    for (int t = g; t < batch; t += G) {
      const cpx<T>* s = s0 + t * L;
      cpx<T>* d = d0 + t * L;
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = s[r * nb];
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], wv[r]) : cmul(v[r], wv[r]);
      }
      dft<T, R, INV>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) d[r * Ns] = v[r];
    }
  }
}

template <typename T, int L, int NT, bool INV, bool HALF, int P, int Ns>
__device__ __forceinline__ cpx<T>* fft_ct_from(cpx<T>* a, cpx<T>* b, int batch, const cpx<T>* __restrict__ tw) {
  constexpr CPlan pl = make_cplan(L);
  if constexpr (P == pl.np) {
    return a;
  } else {
    constexpr int R = pl.r[P];
    stockham_ct<T, L, NT, R, Ns, INV, HALF>(a, b, batch, tw);
    lds_barrier();
    return fft_ct_from<T, L, NT, INV, HALF, P + 1, Ns * R>(b, a, batch, tw);
  }
}

// In-place batched FFT of `batch` <= MAXBATCH contiguous transforms of
// length L in LDS (the compiled plan's Stockham passes).  Each pass reads all
// inputs of the thread's butterflies into registers, waits for the block,
// and writes the outputs over the inputs: half the LDS of the ping-pong form
// for two barriers per pass.  Unnormalised; entered by the whole block after
// an lds_barrier(), ends with one.
template <typename T, int L, int NT, bool INV, int MAXBATCH, int P = 0, int Ns = 1>
__device__ __forceinline__ void fft_inplace(cpx<T>* a, int batch, const cpx<T>* __restrict__ tw) {
  constexpr CPlan pl = make_cplan(L);
  if constexpr (P < pl.np) {
    constexpr int R = pl.r[P];
    constexpr int nb = L / R;
    constexpr int tws = L / (Ns * R);
    constexpr int MB = (MAXBATCH * nb + NT - 1) / NT;  // butterflies per thread at most
    const int total = batch * nb;
    cpx<T> v[MB][R];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int w = local_tid() + m * NT;
      if (w < total) {
        const int t = w / nb, j = w - t * nb;
        const int k = j % Ns;
        const cpx<T>* s = a + t * L + j;
#pragma unroll
        for (int r = 0; r < R; ++r) v[m][r] = s[r * nb];
        if constexpr (Ns > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const cpx<T> wv = tw[r * k * tws];
            v[m][r] = INV ? cmulc(v[m][r], wv) : cmul(v[m][r], wv);
          }
        }
        dft<T, R, INV>(v[m]);
      }
    }
    lds_barrier();
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int w = local_tid() + m * NT;
      if (w < total) {
        const int t = w / nb, j = w - t * nb;
        const int q = j / Ns, k = j - q * Ns;
        cpx<T>* d = a + t * L + q * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) d[r * Ns] = v[m][r];
      }
    }
    lds_barrier();
    fft_inplace<T, L, NT, INV, MAXBATCH, P + 1, Ns * R>(a, batch, tw);
  }
}

// Batched in-LDS FFT of `batch` transforms of length P.L, transform t at
// a + t*stride.  Ping-pongs between a and b; returns the buffer holding the
// result.  Unnormalised.  Must be entered by the whole block after the data
// are in place and visible (an lds_barrier() before the call); ends with
// an lds_barrier().
template <typename T, bool INV, int NT>
__device__ __forceinline__ cpx<T>* fft_lds_generic(cpx<T>* a, cpx<T>* b, const FftPlan& P, int batch, int stride,
                                   const cpx<T>* __restrict__ tw, int twh) {
  const int L = P.L;
  int Ns = 1;
  for (int p = 0; p < P.np; ++p) {
    const int R = P.r[p];
    switch (R) {
      case 2: stockham_pass<T, 2, INV, NT>(a, b, L, Ns, batch, stride, tw, twh); break;
      case 3: stockham_pass<T, 3, INV, NT>(a, b, L, Ns, batch, stride, tw, twh); break;
      case 4: stockham_pass<T, 4, INV, NT>(a, b, L, Ns, batch, stride, tw, twh); break;
      case 5: stockham_pass<T, 5, INV, NT>(a, b, L, Ns, batch, stride, tw, twh); break;
      default: stockham_pass<T, 7, INV, NT>(a, b, L, Ns, batch, stride, tw, twh); break;
    }
    lds_barrier();
    cpx<T>* tmp = a;
    a = b;
    b = tmp;
    Ns *= R;
  }
  return a;
}

// Dispatch: compiled plans for contiguous transforms of the workloads'
// lengths (270, 525, 135, 140, 72 points), else the generic runtime-plan
// passes; NT = the launch's block size.
template <typename T, bool INV, int NT>
__device__ __forceinline__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, const FftPlan& P, int batch, int stride,
                           const cpx<T>* __restrict__ tw, int twh = 0) {
  if (stride == P.L) {
    if (twh == 0) {
      switch (P.L) {
        case 270: return fft_ct_from<T, 270, NT, INV, false, 0, 1>(a, b, batch, tw);
        case 525: return fft_ct_from<T, 525, NT, INV, false, 0, 1>(a, b, batch, tw);
        case 135: return fft_ct_from<T, 135, NT, INV, false, 0, 1>(a, b, batch, tw);
        case 140: return fft_ct_from<T, 140, NT, INV, false, 0, 1>(a, b, batch, tw);
        case 72: return fft_ct_from<T, 72, NT, INV, false, 0, 1>(a, b, batch, tw);
        default: break;
      }
    } else if (twh * 2 == P.L) {
      switch (P.L) {
        case 270: return fft_ct_from<T, 270, NT, INV, true, 0, 1>(a, b, batch, tw);
        case 140: return fft_ct_from<T, 140, NT, INV, true, 0, 1>(a, b, batch, tw);
        case 72: return fft_ct_from<T, 72, NT, INV, true, 0, 1>(a, b, batch, tw);
        default: break;
      }
    }
  }
  return fft_lds_generic<T, INV, NT>(a, b, P, batch, stride, tw, twh);
}

// Dispatch of the three-dimensional path: compiled plans for contiguous
// transforms of 64 and 128 points, else as fft_lds.
template <typename T, bool INV, int NT>
__device__ __forceinline__ cpx<T>* fft_lds_pow2(cpx<T>* a, cpx<T>* b, const FftPlan& P, int batch, int stride,
                                                const cpx<T>* __restrict__ tw) {
  if (stride == P.L) {
    switch (P.L) {
      case 64: return fft_ct_from<T, 64, NT, INV, false, 0, 1>(a, b, batch, tw);
      case 128: return fft_ct_from<T, 128, NT, INV, false, 0, 1>(a, b, batch, tw);
      default: break;
    }
  }
  return fft_lds<T, INV, NT>(a, b, P, batch, stride, tw);
}

}  // namespace mmv
