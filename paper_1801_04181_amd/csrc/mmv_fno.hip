// Learned stray-field operator: a Fourier neural operator that maps the
// slider's magnetisation and its sub-cell offset to the stray field it
// makes on the base film (the operator whose exact form is the cross term
// of Eqs. 6-8 sampled with the spline of Sec. III.A).
//
//   input a0 [B][4][H][W]   (m_x, m_y, m_z of the slider, x_p everywhere)
//   lift     v0 = Wl a0 + bl                         (pointwise 4 -> C)
//   layer l  v_{l+1} = GELU( K_l v_l + Wp_l v_l + bp_l ),  l = 0 .. L-1
//            K_l v = Re IDFT2[ R_l(k) DFT2[v](k) ] over the retained modes
//            kx in [0, Mx), ky in [0, My/2) U [H - My/2, H), R_l(k) complex C x C
//   project  out = Wq v_L + bq                       (pointwise C -> 3)
//
// Every contraction (the truncated DFTs as products with cos/sin bases, the
// per-mode complex mixing, the pointwise layers, and all their adjoints in
// the backward pass) runs through the BF16 matrix-core product of
// mmv_nn.hip with float32 accumulation; parameters and Adam state are
// float32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string>
#include <algorithm>
#include <vector>
#include "mmv.h"
#include "mmv_internal.h"
#include "mmv_nn.h"

using namespace mmv;

struct mmv_sur {
  hipStream_t st = nullptr;
  int H = 0, W = 0, C = 0, Mx = 0, My = 0, L = 0, Bmax = 0;
  long long HW = 0, P = 0;
  long long o_wl = 0, o_bl = 0, o_wq = 0, o_bq = 0, nparam = 0;
  std::vector<long long> o_R, o_wp, o_bp;
  float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  int adam_t = 0;
  float *Dx = nullptr, *Cy = nullptr, *Sy = nullptr, *Ex = nullptr;
  std::vector<float*> v, pre, x2;
  float *x1 = nullptr, *yb = nullptr, *zb = nullptr, *s = nullptr, *u = nullptr, *pred = nullptr;
  float *dv = nullptr, *dv2 = nullptr, *dpre = nullptr, *dpred = nullptr, *parts = nullptr;
  long long nparts_cap = 0;
  double* mse_part = nullptr;
  std::vector<void*> allocs;
};

namespace {

int sfail(int code, const std::string& m) { return report_error(code, m); }

#define SCHK(call)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return sfail(MMV_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int salloc(mmv_sur* h, float** p, long long n) {
  hipError_t e = hipMalloc((void**)p, sizeof(float) * (size_t)(n > 0 ? n : 1));
  if (e != hipSuccess) return sfail(MMV_ENOMEM, "hipMalloc failed");
  h->allocs.push_back(*p);
  return MMV_OK;
}

GemmArgs G(const float* A, long long am, long long ak, long long sa, const float* B, long long bk, long long bn,
           long long sb, float* C, long long cm, long long cn, long long sc, int M, int N, int K, float alpha = 1.0f,
           float beta = 0.0f) {
  GemmArgs g{};
  g.A = A;
  g.am = am;
  g.ak = ak;
  g.sa = sa;
  g.B = B;
  g.bk = bk;
  g.bn = bn;
  g.sb = sb;
  g.C = C;
  g.cm = cm;
  g.cn = cn;
  g.sc = sc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.kchunk = 0;
  g.ps = 0;
  return g;
}

// grad (+)= sum over batch b of A_b (M x K, K = pixels) B_b^T, split-K with a
// deterministic reduction of the partial tiles
int wgrad(mmv_sur* h, const float* A, long long a_b, const float* Bm, long long b_b, int M, int N, long long K,
          int nb, float* grad, int accumulate) {
  const int kchunk = 2048;
  const int nsplit = (int)((K + kchunk - 1) / kchunk);
  const long long need = (long long)nb * nsplit * M * N;
  if (need > h->nparts_cap) return sfail(MMV_EINVAL, "partial buffer too small");
  // A_b(m, k) = A[b a_b + m K + k];  B(k, n) = Bm[b b_b + n K + k]
  GemmArgs g = G(A, K, 1, a_b, Bm, 1, K, b_b, h->parts, N, 1, (long long)nsplit * M * N, M, N, (int)K);
  g.kchunk = kchunk;
  g.ps = (long long)M * N;
  SCHK(launch_gemm(g, nb, h->st));
  SCHK(launch_sum_parts(nb * nsplit, (long long)M * N, h->parts, grad, accumulate, h->st));
  return MMV_OK;
}

// spectral convolution of layer l: v -> s
int spectral_fwd(mmv_sur* h, int l, const float* v, float* s, int B) {
  const int C = h->C, H = h->H, W = h->W, Mx = h->Mx, My = h->My;
  const long long P = h->P, HW = h->HW;
  const long long BCH = (long long)B * C * H;
  const float* R = h->w + h->o_R[l];
  float* x2 = h->x2[l];
  // x DFT: x1 = v Dx  ([B C H] x W) (W x 2Mx)
  SCHK(launch_gemm(G(v, W, 1, 0, h->Dx, 2 * Mx, 1, 0, h->x1, 2 * Mx, 1, 0, (int)BCH, 2 * Mx, W), 1, h->st));
  // y DFT per (b, c): x2r = Cy xr1 + Sy xi1, x2i = Cy xi1 - Sy xr1
  const long long s1 = (long long)H * 2 * Mx;
  const float* xr1 = h->x1;
  const float* xi1 = h->x1 + Mx;
  float* x2r = x2;
  float* x2i = x2 + P;
  const int nbc = B * C;
  SCHK(launch_gemm(G(h->Cy, H, 1, 0, xr1, 2 * Mx, 1, s1, x2r, Mx, 1, 2 * P, My, Mx, H), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, H, 1, 0, xi1, 2 * Mx, 1, s1, x2r, Mx, 1, 2 * P, My, Mx, H, 1.0f, 1.0f), nbc, h->st));
  SCHK(launch_gemm(G(h->Cy, H, 1, 0, xi1, 2 * Mx, 1, s1, x2i, Mx, 1, 2 * P, My, Mx, H), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, H, 1, 0, xr1, 2 * Mx, 1, s1, x2i, Mx, 1, 2 * P, My, Mx, H, -1.0f, 1.0f), nbc, h->st));
  // mode mixing, batched over the P modes: y = R x (complex C x C)
  const float* Rr = R;
  const float* Ri = R + (long long)C * C;
  const long long sR = 2LL * C * C, sX = 2LL * C * P;
  float* yr = h->yb;
  float* yi = h->yb + P;
  const int Pn = (int)P;
  SCHK(launch_gemm(G(Rr, C, 1, sR, x2r, 2 * P, sX, 1, yr, 2 * P, sX, 1, C, B, C), Pn, h->st));
  SCHK(launch_gemm(G(Ri, C, 1, sR, x2i, 2 * P, sX, 1, yr, 2 * P, sX, 1, C, B, C, -1.0f, 1.0f), Pn, h->st));
  SCHK(launch_gemm(G(Ri, C, 1, sR, x2r, 2 * P, sX, 1, yi, 2 * P, sX, 1, C, B, C), Pn, h->st));
  SCHK(launch_gemm(G(Rr, C, 1, sR, x2i, 2 * P, sX, 1, yi, 2 * P, sX, 1, C, B, C, 1.0f, 1.0f), Pn, h->st));
  // inverse y per (b, o): zr = Cy^T yr - Sy^T yi, zi = Sy^T yr + Cy^T yi
  float* zr = h->zb;
  float* zi = h->zb + Mx;
  SCHK(launch_gemm(G(h->Cy, 1, H, 0, yr, Mx, 1, 2 * P, zr, 2 * Mx, 1, s1, H, Mx, My), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, 1, H, 0, yi, Mx, 1, 2 * P, zr, 2 * Mx, 1, s1, H, Mx, My, -1.0f, 1.0f), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, 1, H, 0, yr, Mx, 1, 2 * P, zi, 2 * Mx, 1, s1, H, Mx, My), nbc, h->st));
  SCHK(launch_gemm(G(h->Cy, 1, H, 0, yi, Mx, 1, 2 * P, zi, 2 * Mx, 1, s1, H, Mx, My, 1.0f, 1.0f), nbc, h->st));
  // inverse x: s = z Ex  ([B C H] x 2Mx) (2Mx x W)
  SCHK(launch_gemm(G(h->zb, 2 * Mx, 1, 0, h->Ex, W, 1, 0, s, W, 1, 0, (int)BCH, W, 2 * Mx), 1, h->st));
  (void)HW;
  return MMV_OK;
}

// adjoint of the spectral convolution: ds -> dv (accumulated), and dR
int spectral_bwd(mmv_sur* h, int l, const float* ds, float* dv, int B) {
  const int C = h->C, H = h->H, W = h->W, Mx = h->Mx, My = h->My;
  const long long P = h->P;
  const long long BCH = (long long)B * C * H;
  const float* R = h->w + h->o_R[l];
  float* gR = h->g + h->o_R[l];
  const float* x2 = h->x2[l];
  const long long s1 = (long long)H * 2 * Mx;
  const int nbc = B * C;
  // dz = ds Ex^T
  SCHK(launch_gemm(G(ds, W, 1, 0, h->Ex, 1, W, 0, h->zb, 2 * Mx, 1, 0, (int)BCH, 2 * Mx, W), 1, h->st));
  // dy from dz: dyr = Cy dzr + Sy dzi ; dyi = -Sy dzr + Cy dzi
  const float* dzr = h->zb;
  const float* dzi = h->zb + Mx;
  float* dyr = h->yb;
  float* dyi = h->yb + P;
  SCHK(launch_gemm(G(h->Cy, H, 1, 0, dzr, 2 * Mx, 1, s1, dyr, Mx, 1, 2 * P, My, Mx, H), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, H, 1, 0, dzi, 2 * Mx, 1, s1, dyr, Mx, 1, 2 * P, My, Mx, H, 1.0f, 1.0f), nbc, h->st));
  SCHK(launch_gemm(G(h->Cy, H, 1, 0, dzi, 2 * Mx, 1, s1, dyi, Mx, 1, 2 * P, My, Mx, H), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, H, 1, 0, dzr, 2 * Mx, 1, s1, dyi, Mx, 1, 2 * P, My, Mx, H, -1.0f, 1.0f), nbc, h->st));
  // dR per mode: dRr = dyr xr^T + dyi xi^T ; dRi = dyi xr^T - dyr xi^T (sum over batch)
  const long long sR = 2LL * C * C, sX = 2LL * C * P;
  const float* xr = x2;
  const float* xi = x2 + P;
  float* gRr = gR;
  float* gRi = gR + (long long)C * C;
  const int Pn = (int)P;
  SCHK(launch_gemm(G(dyr, 2 * P, sX, 1, xr, sX, 2 * P, 1, gRr, C, 1, sR, C, C, B), Pn, h->st));
  SCHK(launch_gemm(G(dyi, 2 * P, sX, 1, xi, sX, 2 * P, 1, gRr, C, 1, sR, C, C, B, 1.0f, 1.0f), Pn, h->st));
  SCHK(launch_gemm(G(dyi, 2 * P, sX, 1, xr, sX, 2 * P, 1, gRi, C, 1, sR, C, C, B), Pn, h->st));
  SCHK(launch_gemm(G(dyr, 2 * P, sX, 1, xi, sX, 2 * P, 1, gRi, C, 1, sR, C, C, B, -1.0f, 1.0f), Pn, h->st));
  // dx2: dxr = Rr^T dyr + Ri^T dyi ; dxi = Rr^T dyi - Ri^T dyr   (into the x1 scratch, layout of x2)
  const float* Rr = R;
  const float* Ri = R + (long long)C * C;
  float* dxr = h->x1;
  float* dxi = h->x1 + P;
  SCHK(launch_gemm(G(Rr, 1, C, sR, dyr, 2 * P, sX, 1, dxr, 2 * P, sX, 1, C, B, C), Pn, h->st));
  SCHK(launch_gemm(G(Ri, 1, C, sR, dyi, 2 * P, sX, 1, dxr, 2 * P, sX, 1, C, B, C, 1.0f, 1.0f), Pn, h->st));
  SCHK(launch_gemm(G(Rr, 1, C, sR, dyi, 2 * P, sX, 1, dxi, 2 * P, sX, 1, C, B, C), Pn, h->st));
  SCHK(launch_gemm(G(Ri, 1, C, sR, dyr, 2 * P, sX, 1, dxi, 2 * P, sX, 1, C, B, C, -1.0f, 1.0f), Pn, h->st));
  // dx1 from dx2: dxr1 = Cy^T dxr - Sy^T dxi ; dxi1 = Sy^T dxr + Cy^T dxi   (into zb, layout of x1)
  float* dxr1 = h->zb;
  float* dxi1 = h->zb + Mx;
  SCHK(launch_gemm(G(h->Cy, 1, H, 0, dxr, Mx, 1, 2 * P, dxr1, 2 * Mx, 1, s1, H, Mx, My), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, 1, H, 0, dxi, Mx, 1, 2 * P, dxr1, 2 * Mx, 1, s1, H, Mx, My, -1.0f, 1.0f), nbc, h->st));
  SCHK(launch_gemm(G(h->Sy, 1, H, 0, dxr, Mx, 1, 2 * P, dxi1, 2 * Mx, 1, s1, H, Mx, My), nbc, h->st));
  SCHK(launch_gemm(G(h->Cy, 1, H, 0, dxi, Mx, 1, 2 * P, dxi1, 2 * Mx, 1, s1, H, Mx, My, 1.0f, 1.0f), nbc, h->st));
  // dv += dx1 Dx^T
  SCHK(launch_gemm(G(h->zb, 2 * Mx, 1, 0, h->Dx, 1, 2 * Mx, 0, dv, W, 1, 0, (int)BCH, W, 2 * Mx, 1.0f, 1.0f), 1,
                   h->st));
  return MMV_OK;
}

int forward(mmv_sur* h, const float* a0, int B) {
  const int C = h->C, L = h->L;
  const long long HW = h->HW;
  const float* w = h->w;
  // lift
  SCHK(launch_gemm(G(w + h->o_wl, 4, 1, 0, a0, HW, 1, 4 * HW, h->v[0], HW, 1, C * HW, C, (int)HW, 4), B, h->st));
  SCHK(launch_bias_act((long long)B * C * HW, (int)HW, C, nullptr, h->v[0], w + h->o_bl, nullptr, h->v[0], 0, h->st));
  for (int l = 0; l < L; ++l) {
    int rc = spectral_fwd(h, l, h->v[l], h->s, B);
    if (rc) return rc;
    SCHK(launch_gemm(G(w + h->o_wp[l], C, 1, 0, h->v[l], HW, 1, C * HW, h->u, HW, 1, C * HW, C, (int)HW, C), B,
                     h->st));
    SCHK(launch_bias_act((long long)B * C * HW, (int)HW, C, h->s, h->u, w + h->o_bp[l], h->pre[l + 1], h->v[l + 1], 1,
                         h->st));
  }
  SCHK(launch_gemm(G(w + h->o_wq, C, 1, 0, h->v[L], HW, 1, C * HW, h->pred, HW, 1, 3 * HW, 3, (int)HW, C), B, h->st));
  SCHK(launch_bias_act((long long)B * 3 * HW, (int)HW, 3, nullptr, h->pred, w + h->o_bq, nullptr, h->pred, 0, h->st));
  return MMV_OK;
}

// gradients of the mean-square loss at (a0, target); h->g receives them
int backward(mmv_sur* h, const float* a0, const float* target, int B, double* loss, double* rel) {
  const int C = h->C, L = h->L;
  const long long HW = h->HW, n = (long long)B * 3 * HW;
  const float* w = h->w;
  float* g = h->g;
  const int nb = mse_blocks(n);
  SCHK(launch_mse(n, h->pred, target, h->dpred, h->mse_part, h->st));
  // projection
  int rc = wgrad(h, h->dpred, 3 * HW, h->v[L], C * HW, 3, C, HW, B, g + h->o_wq, 0);
  if (rc) return rc;
  SCHK(launch_channel_sum(B, 3, (int)HW, h->dpred, g + h->o_bq, 0, h->st));
  SCHK(launch_gemm(G(w + h->o_wq, 1, C, 0, h->dpred, HW, 1, 3 * HW, h->dv, HW, 1, C * HW, C, (int)HW, 3), B, h->st));
  for (int l = L - 1; l >= 0; --l) {
    SCHK(launch_act_grad((long long)B * C * HW, h->pre[l + 1], h->dv, h->dpre, h->st));
    SCHK(launch_channel_sum(B, C, (int)HW, h->dpre, g + h->o_bp[l], 0, h->st));
    if ((rc = wgrad(h, h->dpre, C * HW, h->v[l], C * HW, C, C, HW, B, g + h->o_wp[l], 0))) return rc;
    SCHK(launch_gemm(G(w + h->o_wp[l], 1, C, 0, h->dpre, HW, 1, C * HW, h->dv2, HW, 1, C * HW, C, (int)HW, C), B,
                     h->st));
    if ((rc = spectral_bwd(h, l, h->dpre, h->dv2, B))) return rc;
    std::swap(h->dv, h->dv2);
  }
  if ((rc = wgrad(h, h->dv, C * HW, a0, 4 * HW, C, 4, HW, B, g + h->o_wl, 0))) return rc;
  SCHK(launch_channel_sum(B, C, (int)HW, h->dv, g + h->o_bl, 0, h->st));
  std::vector<double> part(2 * (size_t)nb);
  SCHK(hipMemcpyAsync(part.data(), h->mse_part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, h->st));
  SCHK(hipStreamSynchronize(h->st));
  double e = 0, q = 0;
  for (int i = 0; i < nb; ++i) {
    e += part[2 * i];
    q += part[2 * i + 1];
  }
  if (loss) *loss = e / (double)n;
  if (rel) *rel = q > 0 ? sqrt(e / q) : 0.0;
  return MMV_OK;
}

void host_bases(mmv_sur* h, std::vector<float>& Dx, std::vector<float>& Cy, std::vector<float>& Sy,
                std::vector<float>& Ex) {
  const int H = h->H, W = h->W, Mx = h->Mx, My = h->My;
  Dx.assign((size_t)W * 2 * Mx, 0.0f);
  Ex.assign((size_t)2 * Mx * W, 0.0f);
  for (int x = 0; x < W; ++x)
    for (int j = 0; j < Mx; ++j) {
      const double a = 2.0 * M_PI * (double)j * x / W;
      Dx[(size_t)x * 2 * Mx + j] = (float)cos(a);
      Dx[(size_t)x * 2 * Mx + Mx + j] = (float)(-sin(a));
      const double wgt = (j == 0 ? 1.0 : 2.0) / ((double)H * W);
      Ex[(size_t)j * W + x] = (float)(wgt * cos(a));
      Ex[(size_t)(Mx + j) * W + x] = (float)(-wgt * sin(a));
    }
  Cy.assign((size_t)My * H, 0.0f);
  Sy.assign((size_t)My * H, 0.0f);
  for (int k = 0; k < My; ++k) {
    const int kv = k < My / 2 ? k : H - My + k;
    for (int y = 0; y < H; ++y) {
      const double a = 2.0 * M_PI * (double)kv * y / H;
      Cy[(size_t)k * H + y] = (float)cos(a);
      Sy[(size_t)k * H + y] = (float)sin(a);
    }
  }
}

__global__ void k_sur_input(const float* __restrict__ m, const RigidState* __restrict__ rigid, double inv_dx,
                            long long plane, float* __restrict__ a) {
  const float xp = (float)(rigid->xs * inv_dx);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < plane;
       i += (long long)gridDim.x * blockDim.x) {
    a[i] = m[i];
    a[plane + i] = m[plane + i];
    a[2 * plane + i] = m[2 * plane + i];
    a[3 * plane + i] = xp;
  }
}

}  // namespace

namespace mmv {

int sur_infer(mmv_sur* s, const float* a, int B, hipStream_t st, const float** out) {
  if (B < 1 || B > s->Bmax) return sfail(MMV_EINVAL, "batch out of range");
  hipStream_t keep = s->st;
  s->st = st;
  const int rc = forward(s, a, B);
  s->st = keep;
  *out = s->pred;
  return rc;
}

void sur_shape(const mmv_sur* s, int* H, int* W) {
  *H = s->H;
  *W = s->W;
}

void sur_max_batch(const mmv_sur* s, int* Bmax) { *Bmax = s->Bmax; }

const float* sur_output(const mmv_sur* s) { return s->pred; }

hipError_t launch_sur_input(const float* m_slider, const RigidState* rigid, double inv_dx, int ny, int nx, float* a,
                            hipStream_t st) {
  const long long plane = (long long)ny * nx;
  const unsigned nb = (unsigned)std::min<long long>((plane + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sur_input, dim3(nb), dim3(256), 0, st, m_slider, rigid, inv_dx, plane, a);
  return hipGetLastError();
}

int sur_rel_err(mmv_sur* s, const float* pred, float* exact, long long n, double scale, hipStream_t st, double* rel) {
  // compare in the network's units: exact / scale against pred
  SCHK(launch_axpy(n, (float)(1.0 / scale), exact, nullptr, exact, st));
  const int nb = mse_blocks(n);
  if (2LL * nb > 2LL * mse_blocks((long long)s->Bmax * 3 * s->HW)) return sfail(MMV_EINVAL, "judge size");
  SCHK(launch_mse(n, pred, exact, nullptr, s->mse_part, st));
  std::vector<double> part(2 * (size_t)nb);
  SCHK(hipMemcpyAsync(part.data(), s->mse_part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
  SCHK(hipStreamSynchronize(st));
  double e = 0, q = 0;
  for (int i = 0; i < nb; ++i) {
    e += part[2 * i];
    q += part[2 * i + 1];
  }
  *rel = q > 0 ? sqrt(e / q) : (e > 0 ? INFINITY : 0.0);
  return MMV_OK;
}

}  // namespace mmv

extern "C" {

int sur_create(const mmv_sur_desc* d, void* hip_stream, mmv_sur_handle* out) {
  if (!d || !out) return sfail(MMV_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->H < 8 || d->W < 8 || d->H > 4096 || d->W > 4096) return sfail(MMV_EINVAL, "H, W must be in [8, 4096]");
  if (d->width < 1 || d->width > 256) return sfail(MMV_EINVAL, "width must be in [1, 256]");
  if (d->modes_x < 1 || 2 * d->modes_x > d->W) return sfail(MMV_EINVAL, "modes_x must be in [1, W/2]");
  if (d->modes_y < 2 || d->modes_y % 2 || d->modes_y > d->H) return sfail(MMV_EINVAL, "modes_y must be even, <= H");
  if (d->layers < 1 || d->layers > 16) return sfail(MMV_EINVAL, "layers must be in [1, 16]");
  if (d->max_batch < 1 || d->max_batch > 256) return sfail(MMV_EINVAL, "max_batch must be in [1, 256]");
  mmv_sur* h = new mmv_sur();
  h->st = (hipStream_t)hip_stream;
  h->H = d->H;
  h->W = d->W;
  h->C = d->width;
  h->Mx = d->modes_x;
  h->My = d->modes_y;
  h->L = d->layers;
  h->Bmax = d->max_batch;
  h->HW = (long long)h->H * h->W;
  h->P = (long long)h->Mx * h->My;
  const long long C = h->C, P = h->P, HW = h->HW, B = h->Bmax;
  long long o = 0;
  h->o_wl = o;
  o += C * 4;
  h->o_bl = o;
  o += C;
  for (int l = 0; l < h->L; ++l) {
    h->o_R.push_back(o);
    o += P * 2 * C * C;
    h->o_wp.push_back(o);
    o += C * C;
    h->o_bp.push_back(o);
    o += C;
  }
  h->o_wq = o;
  o += 3 * C;
  h->o_bq = o;
  o += 3;
  h->nparam = o;
  int rc = 0;
  float** pp[] = {&h->w, &h->g, &h->m1, &h->m2};
  for (float** p : pp)
    if (!rc) rc = salloc(h, p, o);
  if (!rc) rc = salloc(h, &h->Dx, (long long)h->W * 2 * h->Mx);
  if (!rc) rc = salloc(h, &h->Ex, (long long)h->W * 2 * h->Mx);
  if (!rc) rc = salloc(h, &h->Cy, (long long)h->My * h->H);
  if (!rc) rc = salloc(h, &h->Sy, (long long)h->My * h->H);
  h->v.assign(h->L + 1, nullptr);
  h->pre.assign(h->L + 1, nullptr);
  h->x2.assign(h->L, nullptr);
  for (int l = 0; l <= h->L && !rc; ++l) rc = salloc(h, &h->v[l], B * C * HW);
  for (int l = 1; l <= h->L && !rc; ++l) rc = salloc(h, &h->pre[l], B * C * HW);
  for (int l = 0; l < h->L && !rc; ++l) rc = salloc(h, &h->x2[l], B * C * 2 * P);
  const long long xs = std::max(B * C * h->H * 2 * h->Mx, B * C * 2 * P);
  if (!rc) rc = salloc(h, &h->x1, xs);
  if (!rc) rc = salloc(h, &h->zb, xs);
  if (!rc) rc = salloc(h, &h->yb, B * C * 2 * P);
  if (!rc) rc = salloc(h, &h->s, B * C * HW);
  if (!rc) rc = salloc(h, &h->u, B * C * HW);
  if (!rc) rc = salloc(h, &h->dv, B * C * HW);
  if (!rc) rc = salloc(h, &h->dv2, B * C * HW);
  if (!rc) rc = salloc(h, &h->dpre, B * C * HW);
  if (!rc) rc = salloc(h, &h->pred, B * 3 * HW);
  if (!rc) rc = salloc(h, &h->dpred, B * 3 * HW);
  h->nparts_cap = B * ((HW + 2047) / 2048) * C * C;
  if (!rc) rc = salloc(h, &h->parts, h->nparts_cap);
  if (!rc) {
    hipError_t e = hipMalloc((void**)&h->mse_part, sizeof(double) * 2 * mse_blocks(B * 3 * HW));
    if (e != hipSuccess)
      rc = sfail(MMV_ENOMEM, "hipMalloc failed");
    else
      h->allocs.push_back(h->mse_part);
  }
  if (!rc) {
    std::vector<float> Dx, Cy, Sy, Ex;
    host_bases(h, Dx, Cy, Sy, Ex);
    if (hipMemcpy(h->Dx, Dx.data(), Dx.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->Ex, Ex.data(), Ex.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->Cy, Cy.data(), Cy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->Sy, Sy.data(), Sy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->m1, 0, sizeof(float) * o) != hipSuccess || hipMemset(h->m2, 0, sizeof(float) * o) != hipSuccess ||
        hipMemset(h->w, 0, sizeof(float) * o) != hipSuccess)
      rc = sfail(MMV_EHIP, "upload failed");
  }
  if (rc) {
    for (void* p : h->allocs) hipFree(p);
    delete h;
    return rc;
  }
  *out = h;
  return MMV_OK;
}

long long sur_param_count(mmv_sur_handle h) { return h ? h->nparam : -1; }

int sur_param_offsets(mmv_sur_handle h, long long* offs, int n) {
  // wl, bl, (R, wp, bp) per layer, wq, bq
  if (!h || !offs || n < 4 + 3 * h->L) return sfail(MMV_EINVAL, "need 4 + 3 layers offsets");
  int k = 0;
  offs[k++] = h->o_wl;
  offs[k++] = h->o_bl;
  for (int l = 0; l < h->L; ++l) {
    offs[k++] = h->o_R[l];
    offs[k++] = h->o_wp[l];
    offs[k++] = h->o_bp[l];
  }
  offs[k++] = h->o_wq;
  offs[k++] = h->o_bq;
  return MMV_OK;
}

int sur_set_params(mmv_sur_handle h, const float* w_dev) {
  if (!h || !w_dev) return sfail(MMV_EINVAL, "NULL argument");
  SCHK(hipMemcpyAsync(h->w, w_dev, sizeof(float) * h->nparam, hipMemcpyDeviceToDevice, h->st));
  SCHK(hipMemsetAsync(h->m1, 0, sizeof(float) * h->nparam, h->st));
  SCHK(hipMemsetAsync(h->m2, 0, sizeof(float) * h->nparam, h->st));
  h->adam_t = 0;
  return MMV_OK;
}

int sur_get_params(mmv_sur_handle h, float* w_dev) {
  if (!h || !w_dev) return sfail(MMV_EINVAL, "NULL argument");
  SCHK(hipMemcpyAsync(w_dev, h->w, sizeof(float) * h->nparam, hipMemcpyDeviceToDevice, h->st));
  return MMV_OK;
}

int sur_forward(mmv_sur_handle h, const float* in_dev, int B, float* out_dev) {
  if (!h || !in_dev || !out_dev) return sfail(MMV_EINVAL, "NULL argument");
  if (B < 1 || B > h->Bmax) return sfail(MMV_EINVAL, "batch out of range");
  int rc = forward(h, in_dev, B);
  if (rc) return rc;
  SCHK(hipMemcpyAsync(out_dev, h->pred, sizeof(float) * B * 3 * h->HW, hipMemcpyDeviceToDevice, h->st));
  return MMV_OK;
}

int sur_gradient(mmv_sur_handle h, const float* in_dev, const float* target_dev, int B, float* grad_dev,
                 double* loss) {
  if (!h || !in_dev || !target_dev) return sfail(MMV_EINVAL, "NULL argument");
  if (B < 1 || B > h->Bmax) return sfail(MMV_EINVAL, "batch out of range");
  int rc = forward(h, in_dev, B);
  if (!rc) rc = backward(h, in_dev, target_dev, B, loss, nullptr);
  if (rc) return rc;
  if (grad_dev) SCHK(hipMemcpyAsync(grad_dev, h->g, sizeof(float) * h->nparam, hipMemcpyDeviceToDevice, h->st));
  return MMV_OK;
}

int sur_train_step(mmv_sur_handle h, const float* in_dev, const float* target_dev, int B, float lr, double* loss,
                   double* rel_err) {
  if (!h || !in_dev || !target_dev) return sfail(MMV_EINVAL, "NULL argument");
  if (B < 1 || B > h->Bmax) return sfail(MMV_EINVAL, "batch out of range");
  if (!(lr > 0) || !isfinite(lr)) return sfail(MMV_EINVAL, "lr must be > 0");
  int rc = forward(h, in_dev, B);
  if (!rc) rc = backward(h, in_dev, target_dev, B, loss, rel_err);
  if (rc) return rc;
  h->adam_t += 1;
  SCHK(launch_adam(h->nparam, h->w, h->g, h->m1, h->m2, lr, 0.9f, 0.999f, 1e-8f, h->adam_t, h->st));
  return MMV_OK;
}

int sur_gemm_bf16(const float* A, long long am, long long ak, const float* B, long long bk, long long bn, float* C,
                  long long cm, long long cn, int M, int N, int K, float alpha, float beta, void* hip_stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return sfail(MMV_EINVAL, "bad GEMM arguments");
  GemmArgs g = G(A, am, ak, 0, B, bk, bn, 0, C, cm, cn, 0, M, N, K, alpha, beta);
  SCHK(launch_gemm(g, 1, (hipStream_t)hip_stream));
  return MMV_OK;
}

int sur_destroy(mmv_sur_handle h) {
  if (!h) return MMV_OK;
  hipStreamSynchronize(h->st);
  for (void* p : h->allocs) hipFree(p);
  delete h;
  return MMV_OK;
}

}  // extern "C"
