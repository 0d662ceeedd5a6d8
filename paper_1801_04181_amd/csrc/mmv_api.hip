// C ABI of the two-film hot path: descriptor validation, FFT plans, device
// buffers, one-time kernel construction and the per-step launch sequence.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>
#include <string>
#include <vector>
#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include "mmv.h"
#include "mmv_internal.h"
#include "mmv_kernels.h"
#include "mmv_slab.h"

using namespace mmv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(MMV_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double MU0 = 4e-7 * M_PI;
constexpr double GAMMA0 = MU0 * 1.7595e11;  // gamma_e = 1.7595e11 rad/(s T)

bool smooth2357(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}
int next_smooth(int n, bool even) {
  for (int m = n < 1 ? 1 : n;; ++m)
    if (smooth2357(m) && (!even || m % 2 == 0)) return m;
}
bool make_plan(int L, FftPlan& P) {
  P.L = L;
  P.np = 0;
  int n = L;
  for (int r : {7, 5, 3}) {
    while (n % r == 0) {
      if (P.np >= MAX_PASSES) return false;
      P.r[P.np++] = r;
      n /= r;
    }
  }
  while (n % 4 == 0) {
    if (P.np >= MAX_PASSES) return false;
    P.r[P.np++] = 4;
    n /= 4;
  }
  while (n % 2 == 0) {
    if (P.np >= MAX_PASSES) return false;
    P.r[P.np++] = 2;
    n /= 2;
  }
  return n == 1;
}

// Kernel component order: xx yy zz xy xz yz; parities in (x, y).
const int PX[6] = {0, 0, 0, 1, 1, 0};
const int PY[6] = {0, 0, 0, 1, 0, 1};
int comp_index(int a, int b) {
  static const int t[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  return t[a][b];
}

struct LayerSet {
  int kc[6];  // kernel channel per component, -1 = identically zero
};

}  // namespace

namespace mmv {
int report_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace mmv

struct mmv_mesh {
  mmv_mesh_desc d;
  hipStream_t st = nullptr;
  int esz = 4;  // bytes per real
  int nfilm = 2, nx = 0, ny = 0;
  int Lx = 0, Ly = 0, N2x = 0, Kx = 0, Kyh = 0, ngroup = 1, M = 0;
  int row_nt = 0;  // batched row kernel's block size (0: by row length)
  void* hext_buf[2] = {nullptr, nullptr};  // non-uniform applied field per film (owned)
  long hext_gen = 0;                       // bumped by every set_hext_field
  FftPlan px{}, py{};
  void* m0 = nullptr;
  void* mb[2] = {nullptr, nullptr};
  void* acc = nullptr;
  void* spec1 = nullptr;
  void* spec2 = nullptr;
  void* kern = nullptr;
  void* twx = nullptr;
  void* twp = nullptr;
  void* twy = nullptr;
  RigidState* rigid = nullptr;
  double* partial = nullptr;
  unsigned* counter = nullptr;
  int nkc = 0;
  LayerSet self{}, cross{}, fp{}, fm{};
  int pot_kc[7][3];  // potential kernel S at dz = z_s + d (d = -3..3), components x, y, z
  OutTable tab_hot{}, tab_force{};
  RowParams rp_hot{}, rp_force{};
  DriveP drive{};
  std::vector<void*> allocs;
  // single-magnet three-dimensional path
  bool cube = false;
  int nz = 1, Lz = 1;
  FftPlan pz{};
  void* twz = nullptr;
  void* specB = nullptr;
  void* kern_s = nullptr;  // potential kernel S (eddy currents)
  void *hd = nullptr, *he = nullptr, *dmstep = nullptr, *bdot = nullptr, *es = nullptr, *phi = nullptr, *phi2 = nullptr,
       *rr = nullptr;
  double* red = nullptr;   // reduction partials + mean
  CubeLaunch cl{};
  bool eddy_first = true;
  bool in_batch = false;  // owned by a batch: destroy_mesh refuses it
  bool fuse_fwd = false;  // the row kernel x-transforms its new rows (nbr >= 3)
  // learned operator for film 0's cross field (not owned)
  mmv_sur* sur = nullptr;
  int sur_every = 10;
  double sur_tol = 1e-3;
  int sur_fallback = 0;
  double sur_err = -1.0;
  long sur_judged = 0, sur_steps = 0;
  float* sur_in = nullptr;
  float* sur_exact = nullptr;
  // adaptive Dormand-Prince run (allocated at its first use)
  void* kdp = nullptr;         // stage derivatives [7][film][3][y][x]
  double* errpart = nullptr;   // per row block largest error
  DpCtrl* dpc = nullptr;       // step control
  // divergence / curl of the interpolated field (allocated at first use)
  void* divfield = nullptr;    // base field on the slider's stencil points
  double* divpart = nullptr;   // per row: sum |div|, sum |curl|
  OutTable tab_sur{};
  int sor_sweeps = 40;         // < 0: the exact Neumann solve
  double sor_omega = 1.0;
  FftPlan pdct[3]{};           // exact solve: plans and twiddles of lengths nx, ny, nz
  void* twdct[3] = {nullptr, nullptr, nullptr};
  // two films more than one cell thick (uses m0, mb, acc, hd, he, spec1,
  // kern_s and the eddy buffers above for both films)
  bool slab = false;
  int sD = 0;                  // kernel spectra for layer offsets -sD..sD
  void* kern_t = nullptr;      // tensor spectra [6][2 sD + 1][Ly][Kx]
  void* specM = nullptr;       // source spectra [2][3][nz][Ly][Kx]
  void* specP = nullptr;       // product spectra of the target windows
  void* specI = nullptr;       // after the inverse y transforms
  void* win_s2b = nullptr;     // slider field on the base's window [3][nz][ny][M]
  void* win_b2s = nullptr;     // base field on the slider's window [3][nz+2][ny+2][M]
  void* win_e = nullptr;       // eddy sums on both windows [2][3][nz][ny][M]
  void* stencil = nullptr;     // base field at the slider's stencil points [3][nz+2][ny+2][nx+2]
  double* Bprev = nullptr;     // B at the last eddy update [2][3][nz][ny][nx]
  const void* slab_hext[2] = {nullptr, nullptr};  // applied field in use (hext_buf or NULL)
  SlabMulTable tab_t{}, tab_e{};
  SlabMulTable tab_p{};        // scalar-potential mode: the two potential windows
  void *pot_w[2] = {nullptr, nullptr};  // potential windows: slider side [nz+6][ny+6][M], base side [nz+4][ny+4][M]
  void *pot_s[2] = {nullptr, nullptr};  // their samples [nz+6][ny+6][nx+6], [nz+4][ny+4][nx+4]
  // launch timing (diagnostics)
  int prof_kernel = 0;
  size_t prof_used = 0;
  std::vector<hipEvent_t> prof_ev;
};

namespace {

template <typename T>
size_t rsz() {
  return sizeof(T);
}

int dalloc(mmv_mesh* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(MMV_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  h->allocs.push_back(*p);
  return MMV_OK;
}

void free_all(mmv_mesh* h) {
  for (void* p : h->allocs) hipFree(p);
  h->allocs.clear();
}

int validate(const mmv_mesh_desc* d) {
  if (!d) return fail(MMV_EINVAL, "descriptor is NULL");
  if (d->n_films != 1 && d->n_films != 2) return fail(MMV_EINVAL, "n_films must be 1 or 2");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(MMV_EINVAL, "nx, ny, nz must be >= 1");
  if (d->nx > 8192 || d->ny > 8192) return fail(MMV_EINVAL, "nx, ny must be <= 8192");
  if (d->nz > 8192) return fail(MMV_EINVAL, "nz must be <= 8192");
  auto pos = [](double v) { return isfinite(v) && v > 0; };
  if (!pos(d->dx) || !pos(d->dy) || !pos(d->dz)) return fail(MMV_EINVAL, "cell edges must be finite and > 0");
  if (!pos(d->Ms)) return fail(MMV_EINVAL, "Ms must be finite and > 0");
  if (!isfinite(d->Aex) || d->Aex < 0) return fail(MMV_EINVAL, "Aex must be finite and >= 0");
  if (!isfinite(d->alpha) || d->alpha < 0) return fail(MMV_EINVAL, "alpha must be finite and >= 0");
  if (!isfinite(d->Ku)) return fail(MMV_EINVAL, "Ku must be finite");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(d->u[i]) || !isfinite(d->Hext[i])) return fail(MMV_EINVAL, "u and Hext must be finite");
  if (d->precision != 32 && d->precision != 64) return fail(MMV_EINVAL, "precision must be 32 or 64");
  if (d->cross_mode < 0 || d->cross_mode > 2) return fail(MMV_EINVAL, "cross_mode must be 0, 1 or 2");
  if (d->cross_mode != 0 && d->n_films != 2) return fail(MMV_EINVAL, "cross_mode 1 and 2 need two films");
  // the four-point difference of the potential and the force stencil around
  // it reach two cells towards the other film: the films must be more than
  // two cells apart (Sec. IV.D)
  if (d->cross_mode == 1 && d->gap_cells < 3)
    return fail(MMV_EINVAL, "cross_mode 1 (scalar potential) needs gap_cells >= 3: its four-point difference "
                            "would reach into the other film");
  if (!isfinite(d->sigma) || d->sigma < 0) return fail(MMV_EINVAL, "sigma must be finite and >= 0");
  if (d->sigma != 0.0 && !(d->nz > 1 && d->ny > 1 && d->nx > 1))
    return fail(MMV_EINVAL,
                "eddy currents need magnets more than one cell thick in every direction (sigma must be 0)");
  if (d->sor_sweeps < -1 || d->sor_sweeps > 100000)
    return fail(MMV_EINVAL, "sor_sweeps must be -1 (the exact solve) or in [0, 100000]");
  if (d->sor_sweeps == -1 && d->sigma != 0.0 && !(smooth2357(d->nx) && smooth2357(d->ny) && smooth2357(d->nz)))
    return fail(MMV_EINVAL, "sor_sweeps -1 (the exact solve) needs nx, ny, nz {2,3,5,7}-smooth");
  if (!isfinite(d->sor_omega) || d->sor_omega < 0 || d->sor_omega >= 2) return fail(MMV_EINVAL, "sor_omega must be in [0, 2)");
  if (d->gap_cells < 0) return fail(MMV_EINVAL, "gap_cells must be >= 0");
  if (d->max_travel_cells < 0 || d->max_travel_cells > 4096)
    return fail(MMV_EINVAL, "max_travel_cells must be in [0, 4096]");
  if (d->n_films == 2 && (d->halo < 2 || d->halo > 64)) return fail(MMV_EINVAL, "halo must be in [2, 64]");
  if (!pos(d->rc_cells)) return fail(MMV_EINVAL, "rc_cells must be finite and > 0");
  if (d->fft_lx < 0 || d->fft_ly < 0 || d->fft_lz < 0) return fail(MMV_EINVAL, "FFT lengths must be >= 0");
  if (d->pbc < 0 || d->pbc > 3) return fail(MMV_EINVAL, "pbc must be 0..3 (bit 0 = x, bit 1 = y)");
  if (d->pbc_images < 0 || d->pbc_images > 1024) return fail(MMV_EINVAL, "pbc_images must be in [0, 1024]");
  if (d->pbc) {
    if (d->nz != 1 && d->n_films != 2)
      return fail(MMV_EINVAL, "pbc: periodic boundaries need films one cell thick (nz == 1), or two thicker films");
    if (d->sigma > 0.0 && (d->pbc & 2) && d->ny % 2)
      return fail(MMV_EINVAL, "pbc: eddy currents with a periodic y need ny even (red-black colouring over the "
                              "period)");
    if ((d->pbc & 1) && (d->nx % 2 || !smooth2357(d->nx)))
      return fail(MMV_EINVAL, "pbc: a periodic x needs nx even and {2,3,5,7}-smooth (the transform length)");
    if ((d->pbc & 2) && !smooth2357(d->ny))
      return fail(MMV_EINVAL, "pbc: a periodic y needs ny {2,3,5,7}-smooth (the transform length)");
    if (((d->pbc & 1) && d->fft_lx && d->fft_lx != d->nx) || ((d->pbc & 2) && d->fft_ly && d->fft_ly != d->ny))
      return fail(MMV_EINVAL, "pbc: the transform length of a periodic axis is its period (fft_lx/fft_ly 0 or n)");
  }
  return MMV_OK;
}

void host_twiddles(int L, int count, std::vector<double>& re, std::vector<double>& im) {
  re.resize(count);
  im.resize(count);
  for (int t = 0; t < count; ++t) {
    const double a = -2.0 * M_PI * (double)t / (double)L;
    re[t] = cos(a);
    im[t] = sin(a);
  }
}

int upload_tw(mmv_mesh* h, void** dst, int L, int count, bool dbl) {
  std::vector<double> re, im;
  host_twiddles(L, count, re, im);
  const size_t es = dbl ? 8 : 4;
  std::vector<unsigned char> buf(2 * es * count);
  for (int t = 0; t < count; ++t) {
    if (dbl) {
      double v[2] = {re[t], im[t]};
      memcpy(&buf[2 * es * t], v, 2 * es);
    } else {
      float v[2] = {(float)re[t], (float)im[t]};
      memcpy(&buf[2 * es * t], v, 2 * es);
    }
  }
  int rc = dalloc(h, dst, buf.size());
  if (rc) return rc;
  HIPCHK(hipMemcpy(*dst, buf.data(), buf.size(), hipMemcpyHostToDevice));
  return MMV_OK;
}

// Output channel for component a of the field of film `src` through layer set L.
OutCh make_out(const LayerSet& L, int src, int a, int zsign, int row0, int nrows) {
  OutCh o{};
  o.src = src;
  for (int b = 0; b < 3; ++b) {
    const int c = comp_index(a, b);
    o.kc[b] = L.kc[c];
    const int imag = (PX[c] + PY[c]) & 1;
    const int oddy = PY[c];
    const int neg = (zsign < 0 && (c == 4 || c == 5)) ? 1 : 0;  // xz, yz are odd in z
    o.fl[b] = imag | (oddy << 1) | (neg << 2);
  }
  o.row0 = row0;
  o.nrows = nrows;
  o.off = 0;
  return o;
}

// Kernel-channel numbering: the film's own layer (xz, yz vanish in the film
// plane), the other film's layer z_s and the force layers z_s +/- 1.
void assign_channels(mmv_mesh* h) {
  int n = 0;
  for (int c = 0; c < 6; ++c) h->self.kc[c] = (c < 4) ? n++ : -1;
  for (int c = 0; c < 6; ++c) h->cross.kc[c] = h->fp.kc[c] = h->fm.kc[c] = -1;
  for (int d = 0; d < 7; ++d)
    for (int c = 0; c < 3; ++c) h->pot_kc[d][c] = -1;
  if (h->nfilm == 2 && h->d.cross_mode != 1) {
    for (int c = 0; c < 6; ++c) h->cross.kc[c] = n++;
    for (int c = 0; c < 6; ++c) h->fp.kc[c] = n++;
    for (int c = 0; c < 6; ++c) h->fm.kc[c] = n++;
  }
  if (h->nfilm == 2 && h->d.cross_mode == 1)
    for (int d = 0; d < 7; ++d)
      for (int c = 0; c < 3; ++c) h->pot_kc[d][c] = n++;
  h->nkc = n;
}

// Potential channel of film `src` sampled on the layer zsign * z_s + d of
// the other film: phi = sum_b S_b * m_b with S at dz = zsign (z_s + zsign d).
// S_x and S_y have imaginary spectra, S_y is odd in y, S_z flips with dz.
OutCh make_phi(const mmv_mesh* h, int src, int zsign, int d, int row0, int nrows) {
  OutCh o{};
  o.src = src;
  const int layer = zsign > 0 ? d : -d;  // index into S at dz = z_s + layer
  for (int b = 0; b < 3; ++b) {
    o.kc[b] = h->pot_kc[layer + 3][b];
    const int imag = (b < 2) ? 1 : 0;
    const int oddy = (b == 1) ? 1 : 0;
    const int neg = (zsign < 0 && b == 2) ? 1 : 0;
    o.fl[b] = imag | (oddy << 1) | (neg << 2);
  }
  o.row0 = row0;
  o.nrows = nrows;
  return o;
}

// Column-pass table and the matching row-kernel offsets.
void build_tables(mmv_mesh* h, bool full_force, OutTable& tab, RowParams& rp, long long& total) {
  const int ny = h->ny;
  tab.n = 0;
  long long off = 0;
  auto add = [&](OutCh o) -> long long {
    o.off = off;
    off += (long long)o.nrows * h->Kx;
    tab.ch[tab.n++] = o;
    return o.off;
  };
  rp.pot = h->d.cross_mode == 1;
  if (rp.pot) {
    // potential rows each task reads: the stage / eval table carries layers
    // d = -2..2 (rows y-2..y+2 on the film's own layer), the force table
    // d = -3..3 with the extra rows of the y and z differences of H.
    if (!full_force)
      for (int f = 0; f < 2; ++f)
        for (int a = 0; a < 3; ++a) rp.off_self[f][a] = add(make_out(h->self, f, a, +1, 0, ny));
    for (int tgt = 1; tgt >= 0; --tgt) {
      if (full_force && tgt == 0) break;
      const int src = 1 - tgt, zsign = tgt == 1 ? +1 : -1;
      for (int d = -3; d <= 3; ++d) {
        int r0, r1;
        if (full_force) {
          const int ext = 3 - (d < 0 ? -d : d);
          r0 = -ext;
          r1 = ny - 1 + ext;
        } else {
          if (d < -2 || d > 2) {
            rp.off_phi[tgt][d + 3] = 0;
            rp.phi_row0[tgt][d + 3] = 0;
            continue;
          }
          r0 = d == 0 ? -2 : 0;
          r1 = d == 0 ? ny + 1 : ny - 1;
        }
        rp.off_phi[tgt][d + 3] = add(make_phi(h, src, zsign, d, r0, r1 - r0 + 1));
        rp.phi_row0[tgt][d + 3] = r0;
      }
    }
    total = off;
    return;
  }
  for (int f = 0; f < h->nfilm; ++f)
    for (int a = 0; a < 3; ++a) rp.off_self[f][a] = add(make_out(h->self, f, a, +1, 0, ny));
  if (h->nfilm == 2) {
    for (int a = 0; a < 3; ++a) rp.off_cross[1][a] = add(make_out(h->cross, 0, a, +1, -1, ny + 2));
    rp.cross_row0[1] = -1;
    const int nfc = full_force ? 3 : 1;
    for (int a = 0; a < nfc; ++a) rp.off_fp[a] = add(make_out(h->fp, 0, a, +1, 0, ny));
    for (int a = 0; a < nfc; ++a) rp.off_fm[a] = add(make_out(h->fm, 0, a, +1, 0, ny));
    for (int a = 0; a < 3; ++a) rp.off_cross[0][a] = add(make_out(h->cross, 1, a, -1, 0, ny));
    rp.cross_row0[0] = 0;
  }
  total = off;
}

template <typename T>
int build_kernels(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  const int n = h->nkc;
  int rc = dalloc(h, &h->kern, sizeof(T) * (size_t)n * h->Kx * h->Kyh);
  if (rc) return rc;
  void *tmp = nullptr, *tspec = nullptr, *twxd = nullptr, *twpd = nullptr, *twyd = nullptr;
  HIPCHK(hipMalloc(&tmp, sizeof(double) * (size_t)h->Lx * h->Ly));
  HIPCHK(hipMalloc(&tspec, 2 * sizeof(double) * (size_t)h->Kx * h->Ly));
  mmv_mesh tmp_owner;
  rc = upload_tw(&tmp_owner, &twxd, h->N2x, h->N2x, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twpd, h->Lx, h->N2x + 1, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twyd, h->Ly, h->Ly, true);
  if (rc) {
    hipFree(tmp);
    hipFree(tspec);
    free_all(&tmp_owner);
    return rc;
  }
  // tensor spectra carry -Ms (Eq. 6), potential spectra +Ms (Eq. 7); both
  // the 1/(Lx Ly) of the unnormalised inverse transforms
  const double scale = d.Ms / ((double)h->Lx * (double)h->Ly);
  struct Job {
    int kc, kind, comp;
    double dzc;
  };
  std::vector<Job> jobs;
  const int zs = d.nz + d.gap_cells;
  for (int c = 0; c < 6; ++c) {
    if (h->self.kc[c] >= 0) jobs.push_back({h->self.kc[c], 0, c, 0.0});
    if (h->cross.kc[c] >= 0) {
      jobs.push_back({h->cross.kc[c], 0, c, (double)zs});
      jobs.push_back({h->fp.kc[c], 0, c, (double)(zs + 1)});
      jobs.push_back({h->fm.kc[c], 0, c, (double)(zs - 1)});
    }
  }
  for (int dd = -3; dd <= 3; ++dd)
    for (int c = 0; c < 3; ++c)
      if (h->pot_kc[dd + 3][c] >= 0) jobs.push_back({h->pot_kc[dd + 3][c], 1, c, (double)(zs + dd)});
  hipError_t err = hipSuccess;
  for (const Job& j : jobs) {
    err = launch_kernel_real((double*)tmp, h->Lx, h->Ly, j.kind, j.comp, j.dzc, d.dx, d.dy, d.dz, d.rc_cells,
                             j.kind == 0 ? -scale : scale, d.pbc, d.pbc_images, h->st);
    if (err != hipSuccess) break;
    err = launch_row_fwd<double>((const double*)tmp, tspec, h->Ly, h->Lx, h->N2x, h->Kx, h->px, twxd, twpd, h->st);
    if (err != hipSuccess) break;
    const int imag = j.kind == 0 ? ((PX[j.comp] + PY[j.comp]) & 1) : (j.comp < 2 ? 1 : 0);
    err = launch_colpack<T>(tspec, (T*)h->kern + (size_t)j.kc * h->Kx * h->Kyh, h->Kx, h->Ly, h->Kyh, h->py, twyd,
                            imag, h->st);
    if (err != hipSuccess) break;
  }
  if (err == hipSuccess) err = hipStreamSynchronize(h->st);
  hipFree(tmp);
  hipFree(tspec);
  free_all(&tmp_owner);
  if (err != hipSuccess) return fail(MMV_EHIP, std::string("kernel construction: ") + hipGetErrorString(err));
  return MMV_OK;
}

// Size limits set by the LDS of the row and y-pass kernels (the CU's 160 KB
// less what the kernels declare statically) and by the 32-bit
// kernel-spectrum index, from the descriptor and the channel tables alone
// (checked before any device call).
template <typename T>
int check_sizes(const mmv_mesh* h) {
  const size_t lds_limit = LDS_PER_CU - ROW_STATIC_LDS;
  RowParams probe{};
  probe.nx = h->nx;
  probe.N2x = h->N2x;
  probe.M = h->M;
  probe.nbr = 1;
  probe.full_force = 1;
  probe.pot = h->d.cross_mode == 1;
  if (row_lds_bytes<T>(probe) > lds_limit) return fail(MMV_EINVAL, "nx too large for the row kernel's LDS");
  if (sizeof(T) * 2 * (4 * (size_t)h->N2x + 1) > LDS_PER_CU) return fail(MMV_EINVAL, "nx too large");
  if ((long long)h->nkc * h->Kx * h->Kyh >= (1LL << 31)) return fail(MMV_EINVAL, "kernel spectra too large");
  const int nin = 3 * h->nfilm;
  const int nmax = h->tab_force.n > h->tab_hot.n ? h->tab_force.n : h->tab_hot.n;
  for (int g = 1; g <= 8; ++g) {
    const int per = (nmax + g - 1) / g;
    if (col_lds_bytes<T>(h->Ly, nin > per ? nin : per) <= LDS_PER_CU - COL_STATIC_LDS) return MMV_OK;
  }
  return fail(MMV_EINVAL, "ny too large for the y pass");
}

template <typename T>
int init_typed(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  h->esz = sizeof(T);
  const size_t ncell = (size_t)h->nfilm * h->nx * h->ny;
  int rc;
  long long n_hot = 0, n_force = 0;
  assign_channels(h);
  build_tables(h, false, h->tab_hot, h->rp_hot, n_hot);
  build_tables(h, true, h->tab_force, h->rp_force, n_force);
  if ((rc = check_sizes<T>(h))) return rc;
  if ((rc = dalloc(h, &h->m0, 3 * ncell * sizeof(T)))) return rc;
  if (!static_lds_within_reserve<T>())
    return fail(MMV_EHIP, "the film kernels' static LDS exceeds the reserve the size limits assume");
  if ((rc = dalloc(h, &h->mb[0], 3 * ncell * sizeof(T)))) return rc;
  if ((rc = dalloc(h, &h->mb[1], 3 * ncell * sizeof(T)))) return rc;
  if ((rc = dalloc(h, &h->acc, 3 * ncell * sizeof(T)))) return rc;
  if ((rc = dalloc(h, &h->spec1, 2 * sizeof(T) * 3 * (size_t)h->nfilm * h->ny * h->Kx))) return rc;
  const long long n2 = n_hot > n_force ? n_hot : n_force;
  if ((rc = dalloc(h, &h->spec2, 2 * sizeof(T) * (size_t)n2))) return rc;
  if ((rc = upload_tw(h, &h->twx, h->N2x, h->N2x, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twp, h->Lx, h->N2x + 1, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twy, h->Ly, h->Ly, sizeof(T) == 8))) return rc;
  const int ntask_max = h->nfilm * h->ny + 2;
  if ((rc = dalloc(h, (void**)&h->partial, sizeof(double) * 3 * (size_t)ntask_max))) return rc;
  if ((rc = dalloc(h, (void**)&h->counter, sizeof(unsigned) * 4))) return rc;
  if ((rc = dalloc(h, (void**)&h->rigid, sizeof(RigidState)))) return rc;
  HIPCHK(hipMemsetAsync(h->counter, 0, sizeof(unsigned) * 4, h->st));
  RigidState r{};
  HIPCHK(hipMemcpyAsync(h->rigid, &r, sizeof(r), hipMemcpyHostToDevice, h->st));
  // m = +z
  std::vector<T> mz(3 * ncell, T(0));
  for (int f = 0; f < h->nfilm; ++f)
    for (size_t i = 0; i < (size_t)h->nx * h->ny; ++i) mz[(size_t)f * 3 * h->nx * h->ny + 2 * h->nx * h->ny + i] = T(1);
  HIPCHK(hipMemcpy(h->m0, mz.data(), mz.size() * sizeof(T), hipMemcpyHostToDevice));
  if ((rc = build_kernels<T>(h))) return rc;

  // row-kernel parameters common to both tables
  for (RowParams* rp : {&h->rp_hot, &h->rp_force}) {
    rp->nfilm = h->nfilm;
    rp->nx = h->nx;
    rp->ny = h->ny;
    rp->N2x = h->N2x;
    rp->Kx = h->Kx;
    rp->halo = d.halo;
    rp->M = h->M;
    // a periodic x lets the slider travel without bound
    rp->travel = (d.pbc & 1) ? (1 << 30) : d.max_travel_cells;
    rp->pbc = d.pbc;
    rp->dx = d.dx;
    rp->dy = d.dy;
    rp->dz = d.dz;
    rp->pref_ex = 2.0 * d.Aex / (MU0 * d.Ms);
    rp->pref_an = 2.0 * d.Ku / (MU0 * d.Ms);
    const double un = sqrt(d.u[0] * d.u[0] + d.u[1] * d.u[1] + d.u[2] * d.u[2]);
    for (int i = 0; i < 3; ++i) {
      rp->u[i] = un > 0 ? d.u[i] / un : 0.0;
      rp->hext[i] = d.Hext[i];
    }
    rp->gam = GAMMA0 / (1.0 + d.alpha * d.alpha);
    rp->alpha = d.alpha;
    rp->force_scale = MU0 * d.Ms * d.dx * d.dy * d.dz;
    rp->interp = d.cross_mode == 2 ? 1 : 0;
    rp->px = h->px;
  }
  // LDS limits (the CU's 160 KB less the kernels' static LDS)
  const size_t lds_limit = LDS_PER_CU - ROW_STATIC_LDS;
  const size_t col_limit = LDS_PER_CU - COL_STATIC_LDS;
  // inverse row transforms per batch of the row kernel: as many as fit
  int nbr = 0;
  for (int b : {9, 8, 6, 4, 3, 2, 1}) {
    RowParams probe = h->rp_force;
    probe.full_force = 1;
    probe.nbr = b;
    probe.pot = h->d.cross_mode == 1;
    if (row_lds_bytes<T>(probe) <= lds_limit) {
      nbr = b;
      break;
    }
  }
  if (!nbr) return fail(MMV_EINVAL, "nx too large for the row kernel's LDS");
  h->rp_hot.nbr = h->rp_force.nbr = nbr;
  h->fuse_fwd = nbr >= 3;
  // compiled lengths: the row transforms run in place (the batched kernel
  // does the same, so batch and single-mesh launches compute alike)
  h->rp_hot.inplace = h->rp_force.inplace = row_inplace_length(h->N2x) ? 1 : 0;
  if (sizeof(T) * 2 * (4 * (size_t)h->N2x + 1) > LDS_PER_CU) return fail(MMV_EINVAL, "nx too large");
  // output groups per column of the y pass.  Each group recomputes the
  // column's forward transforms (an L2 hit); more groups give shorter blocks,
  // and the launch should fit in one round of resident blocks.  Estimated
  // cost: rounds x (fixed load/store overhead of ~4 transforms + forward and
  // inverse transforms per block).
  const int nin = 3 * h->nfilm;
  const int nmax = h->tab_force.n > h->tab_hot.n ? h->tab_force.n : h->tab_hot.n;
  if ((long long)h->nkc * h->Kx * h->Kyh >= (1LL << 31)) return fail(MMV_EINVAL, "kernel spectra too large");
  int ncu = 0, dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  h->ngroup = 0;
  double best = 0.0;
  for (int g = 1; g <= 4; ++g) {
    // LDS of the stage launches (the force table only has to fit)
    const int pf = (nmax + g - 1) / g;
    if (col_lds_bytes<T>(h->Ly, nin > pf ? nin : pf) > col_limit) continue;
    const int pg = (h->tab_hot.n + g - 1) / g;
    const size_t lds = col_lds_bytes<T>(h->Ly, nin > pg ? nin : pg);
    const int occ = col_blocks_per_cu<T>(lds);
    if (occ < 1) continue;
    const long long slots = (long long)ncu * occ;
    const long long rounds = ((long long)h->Kx * g + slots - 1) / slots;
    const double cost = (double)rounds * (4.0 + nin + (h->tab_hot.n + g - 1) / g);
    if (getenv("MMV_VERBOSE"))
      fprintf(stderr, "mmv: y pass groups %d: lds %zu, blocks/CU %d, CUs %d, rounds %lld, cost %.0f\n", g, lds, occ,
              ncu, rounds, cost);
    if (!h->ngroup || cost < best) {
      h->ngroup = g;
      best = cost;
    }
  }
  if (!h->ngroup) h->ngroup = 1;
  if (const char* e = getenv("MMV_COL_GROUPS")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 8) h->ngroup = v;
  }
  const int per = (nmax + h->ngroup - 1) / h->ngroup;
  if (col_lds_bytes<T>(h->Ly, nin > per ? nin : per) > col_limit)
    return fail(MMV_EINVAL, "ny too large for the y pass");
  return MMV_OK;
}

// Record a timing event before (begin = true) or after a launch of `kernel`.
int prof_mark(mmv_mesh* h, int kernel) {
  if (h->prof_kernel != kernel) return MMV_OK;
  if (h->prof_used == h->prof_ev.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    h->prof_ev.push_back(e);
  }
  HIPCHK(hipEventRecord(h->prof_ev[h->prof_used++], h->st));
  return MMV_OK;
}

#define PROF(k)                      \
  do {                               \
    int rc_ = prof_mark(h, (k));     \
    if (rc_) return rc_;             \
  } while (0)

// Plans and twiddles of the exact Neumann solve (eddy currents with
// sor_sweeps < 0).
template <typename T>
int init_dct(mmv_mesh* h) {
  if (!(h->d.sigma > 0) || h->sor_sweeps >= 0) return MMV_OK;
  const int n[3] = {h->nx, h->ny, h->nz};
  for (int a = 0; a < 3; ++a) {
    if (!make_plan(n[a], h->pdct[a])) return fail(MMV_EINVAL, "exact Neumann solve: an axis length has too many factors");
    int rc = upload_tw(h, &h->twdct[a], n[a], n[a], sizeof(T) == 8);
    if (rc) return rc;
  }
  return MMV_OK;
}

// ---------------------------------------------------------------- single magnet, 3-D
template <typename T>
int build_kernels_cube(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  const size_t nk = (size_t)h->Kx * (h->Ly / 2 + 1) * (h->Lz / 2 + 1);
  int rc = dalloc(h, &h->kern, sizeof(T) * 6 * nk);
  if (rc) return rc;
  if (d.sigma > 0 && (rc = dalloc(h, &h->kern_s, sizeof(T) * 3 * nk))) return rc;
  mmv_mesh tmp_owner;
  void *grid = nullptr, *s1 = nullptr, *s2 = nullptr, *twxd = nullptr, *twpd = nullptr, *twyd = nullptr, *twzd = nullptr;
  const size_t ng = (size_t)h->Lx * h->Ly * h->Lz;
  const size_t ns = (size_t)h->Kx * h->Ly * h->Lz;
  rc = dalloc(&tmp_owner, &grid, sizeof(double) * ng);
  if (!rc) rc = dalloc(&tmp_owner, &s1, 2 * sizeof(double) * ns);
  if (!rc) rc = dalloc(&tmp_owner, &s2, 2 * sizeof(double) * ns);
  if (!rc) rc = upload_tw(&tmp_owner, &twxd, h->N2x, h->N2x, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twpd, h->Lx, h->N2x + 1, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twyd, h->Ly, h->Ly, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twzd, h->Lz, h->Lz, true);
  if (rc) {
    free_all(&tmp_owner);
    return rc;
  }
  const double inv = 1.0 / ((double)h->Lx * h->Ly * h->Lz);
  hipError_t err = hipSuccess;
  const int nkind = d.sigma > 0 ? 2 : 1;
  for (int kind = 0; kind < nkind && err == hipSuccess; ++kind) {
    for (int comp = 0; comp < (kind == 0 ? 6 : 3) && err == hipSuccess; ++comp) {
      // tensor spectra carry -Ms (Eq. 6); S spectra enter the eddy sums bare
      const double scale = kind == 0 ? -d.Ms * inv : inv;
      err = launch_kernel_real3((double*)grid, h->Lx, h->Ly, h->Lz, kind, comp, d.dx, d.dy, d.dz, d.rc_cells, scale,
                                h->st);
      if (err == hipSuccess)
        err = launch_row_fwd<double>((const double*)grid, s1, h->Ly * h->Lz, h->Lx, h->N2x, h->Kx, h->px, twxd, twpd,
                                     h->st);
      if (err == hipSuccess)
        err = launch_fft_axis<double>(s1, s2, h->Lz, h->Kx, 0, h->Ly, (long long)h->Ly * h->Kx, h->Ly,
                                      (long long)h->Ly * h->Kx, h->py, twyd, false, h->st);
      if (err == hipSuccess)
        err = launch_fft_axis<double>(s2, s1, 1, h->Ly * h->Kx, 0, h->Lz, 0, h->Lz, 0, h->pz, twzd, false, h->st);
      T* dst = (T*)(kind == 0 ? h->kern : h->kern_s) + (size_t)comp * nk;
      if (err == hipSuccess) err = launch_pack3<T>(s1, dst, h->Kx, h->Ly, h->Lz, kind == 1 ? 1 : 0, h->st);
    }
  }
  if (err == hipSuccess) err = hipStreamSynchronize(h->st);
  free_all(&tmp_owner);
  if (err != hipSuccess) return fail(MMV_EHIP, std::string("kernel construction: ") + hipGetErrorString(err));
  return MMV_OK;
}

template <typename T>
int init_cube(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  h->esz = sizeof(T);
  const size_t N = (size_t)h->nx * h->ny * h->nz;
  int rc;
  void** bufs3[] = {&h->m0, &h->mb[0], &h->mb[1], &h->acc, &h->hd, &h->he};
  for (void** b : bufs3)
    if ((rc = dalloc(h, b, 3 * N * sizeof(T)))) return rc;
  if ((rc = dalloc(h, &h->spec1, 2 * sizeof(T) * 3 * (size_t)h->nz * h->ny * h->Kx))) return rc;
  if ((rc = dalloc(h, &h->specB, 2 * sizeof(T) * 3 * (size_t)h->nz * h->Ly * h->Kx))) return rc;
  if (d.sigma > 0) {
    void** e3[] = {&h->dmstep, &h->bdot, &h->es};
    for (void** b : e3)
      if ((rc = dalloc(h, b, 3 * N * sizeof(T)))) return rc;
    if ((rc = dalloc(h, &h->phi, N * sizeof(T)))) return rc;
    if ((rc = dalloc(h, &h->phi2, N * sizeof(T)))) return rc;
    if ((rc = dalloc(h, &h->rr, N * sizeof(T)))) return rc;
    HIPCHK(hipMemsetAsync(h->phi, 0, N * sizeof(T), h->st));
  }
  if ((rc = dalloc(h, (void**)&h->red, sizeof(double) * (N / 256 + 4)))) return rc;
  HIPCHK(hipMemsetAsync(h->he, 0, 3 * N * sizeof(T), h->st));
  if ((rc = upload_tw(h, &h->twx, h->N2x, h->N2x, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twp, h->Lx, h->N2x + 1, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twy, h->Ly, h->Ly, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twz, h->Lz, h->Lz, sizeof(T) == 8))) return rc;
  if ((rc = dalloc(h, (void**)&h->rigid, sizeof(RigidState)))) return rc;
  RigidState r{};
  HIPCHK(hipMemcpyAsync(h->rigid, &r, sizeof(r), hipMemcpyHostToDevice, h->st));
  std::vector<T> mz(3 * N, T(0));
  for (size_t i = 0; i < N; ++i) mz[2 * N + i] = T(1);
  HIPCHK(hipMemcpyAsync(h->m0, mz.data(), mz.size() * sizeof(T), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if ((rc = build_kernels_cube<T>(h))) return rc;
  CubeLaunch& c = h->cl;
  c.nx = h->nx;
  c.ny = h->ny;
  c.nz = h->nz;
  c.dx = d.dx;
  c.dy = d.dy;
  c.dz = d.dz;
  c.pref_ex = 2.0 * d.Aex / (MU0 * d.Ms);
  c.pref_an = 2.0 * d.Ku / (MU0 * d.Ms);
  const double un = sqrt(d.u[0] * d.u[0] + d.u[1] * d.u[1] + d.u[2] * d.u[2]);
  for (int i = 0; i < 3; ++i) {
    c.u[i] = un > 0 ? d.u[i] / un : 0.0;
    c.hext[i] = d.Hext[i];
  }
  c.gam = GAMMA0 / (1.0 + d.alpha * d.alpha);
  c.alpha = d.alpha;
  h->sor_sweeps = d.sor_sweeps != 0 ? d.sor_sweeps : 40;
  const int nmax = std::max(h->nx, std::max(h->ny, h->nz));
  h->sor_omega = d.sor_omega > 0 ? d.sor_omega : 2.0 / (1.0 + sin(M_PI / nmax));
  return init_dct<T>(h);
}

// Demagnetising-type convolution of a three-channel cell field:
// x transform, y transform, z pencils with the kernel, inverse y, inverse x.
// The x transforms take about 1024 points (at most 16 rows) per block.
static int cube_rows_per_block(int N2x) { return std::max(1, std::min(16, 1024 / N2x)); }

template <typename T>
int conv3(mmv_mesh* h, const void* src, void* dst, const T* kern, int mode, double sgn) {
  const int nrow = 3 * h->nz * h->ny;
  const int R = cube_rows_per_block(h->N2x);
  HIPCHK(launch_row_fwd<T>((const T*)src, h->spec1, nrow, h->nx, h->N2x, h->Kx, h->px, h->twx, h->twp, h->st, -R));
  HIPCHK(launch_fft_axis<T>(h->spec1, h->specB, 3 * h->nz, h->Kx, 0, h->ny, (long long)h->ny * h->Kx, h->Ly,
                            (long long)h->Ly * h->Kx, h->py, h->twy, false, h->st));
  const int CBz = 4;  // pencils per block of the z pass
  HIPCHK(launch_zmul<T>(h->specB, kern, h->Kx, h->Ly, h->nz, CBz, mode, sgn, h->pz, h->twz, h->st));
  HIPCHK(launch_fft_axis<T>(h->specB, h->spec1, 3 * h->nz, h->Kx, 0, h->Ly, (long long)h->Ly * h->Kx, h->ny,
                            (long long)h->ny * h->Kx, h->py, h->twy, true, h->st));
  HIPCHK(launch_row_inv<T>(h->spec1, (T*)dst, nrow, R, h->nx, h->N2x, h->Kx, h->px, h->twx, h->twp, h->st));
  return MMV_OK;
}

// Eddy-current update at the start of a step (field held through its stages).
template <typename T>
int eddy_update(mmv_mesh* h, double dt) {
  const size_t N = (size_t)h->nx * h->ny * h->nz;
  const double* part = h->red;
  double* mean = h->red + (N / 256 + 2);
  // dmstep holds the last step's change of m (written by its last stage):
  // dB/dt = mu0 (H_d(dm) + Ms dm) / dt
  int rc;
  if (!h->eddy_first && (rc = conv3<T>(h, h->dmstep, h->bdot, (const T*)h->kern, 0, 1.0))) return rc;
  HIPCHK(launch_eddy_bdot<T>(N, (const T*)h->dmstep, (const T*)h->bdot, (T*)h->bdot, MU0, h->d.Ms, 1.0 / dt,
                             h->eddy_first ? 1 : 0, h->st));
  h->eddy_first = false;
  rc = conv3<T>(h, h->bdot, h->es, (const T*)h->kern_s, 1, +1.0);
  if (rc) return rc;
  HIPCHK(launch_sor_rhs<T>(h->cl, (const T*)h->es, (T*)h->rr, h->red, mean, h->st));
  if (h->sor_sweeps < 0)
    HIPCHK(launch_neumann_solve<T>(h->cl, 1, (const T*)h->rr, (T*)h->phi, (T*)h->phi2, h->pdct, h->twdct, h->st));
  else
    HIPCHK(launch_sor<T>(h->cl, 1, (T*)h->phi, (T*)h->phi2, (const T*)h->rr, h->sor_omega, h->sor_sweeps, h->red,
                         mean, h->st));
  HIPCHK(launch_current<T>(h->cl, (const T*)h->phi, (const T*)h->es, (T*)h->bdot, h->d.sigma, h->st));
  (void)part;
  return conv3<T>(h, h->bdot, h->he, (const T*)h->kern_s, 1, -1.0);
}

template <typename T>
int step_cube(mmv_mesh* h, double dt, int nsteps) {
  T* m0 = (T*)h->m0;
  T* b1 = (T*)h->mb[0];
  T* b2 = (T*)h->mb[1];
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 4; ++s) {
      T* in = s == 0 ? m0 : (s == 1 ? b1 : (s == 2 ? b2 : b1));
      T* out = s == 0 ? b1 : (s == 1 ? b2 : (s == 2 ? b1 : m0));
      int rc = conv3<T>(h, in, h->hd, (const T*)h->kern, 0, 1.0);
      if (rc) return rc;
      if (s == 0 && h->d.sigma > 0 && (rc = eddy_update<T>(h, dt))) return rc;
      PROF(3);
      HIPCHK(launch_stage3<T>(h->cl, MODE_STAGE, s, MMV_TERM_ALL, dt, in, m0, out, (T*)h->acc, (const T*)h->hd,
                              (const T*)h->he, nullptr, &h->rigid->flags, s == 3 ? h->rigid : nullptr,
                              (s == 3 && h->d.sigma > 0) ? (T*)h->dmstep : nullptr, h->st));
      PROF(3);
    }
  }
  return MMV_OK;
}

template <typename T>
int eval_cube(mmv_mesh* h, int mask, void* hout) {
  if (mask & MMV_TERM_DEMAG_SELF) {
    int rc = conv3<T>(h, h->m0, h->hd, (const T*)h->kern, 0, 1.0);
    if (rc) return rc;
  }
  HIPCHK(launch_stage3<T>(h->cl, MODE_EVAL, 0, mask & (1 | 2 | 4 | 8 | 32), 0.0, (const T*)h->m0, (const T*)h->m0,
                          nullptr, nullptr, (const T*)h->hd, (const T*)h->he, (T*)hout, &h->rigid->flags, nullptr,
                          nullptr, h->st));
  return MMV_OK;
}

// ---------------------------------------------------------------- two thick films
// Films of nz > 1 layers in relative motion (Sec. II.A, III.A-B, IV.C-D).
// Each field is a layer-coupled in-plane convolution (mmv_slab.hip): the
// films' own fields, the base's field on the slider's window (layers z_s - 1
// .. z_s + nz, rows -1..ny: the force stencil) and the slider's field on the
// base's window, then the spline (or linear) sampling along x.
constexpr int SLAB_KIND_TENSOR = 0, SLAB_KIND_S = 1;

int slab_rows_per_block(int N2x) { return std::max(1, std::min(16, 1024 / N2x)); }

template <typename T>
int build_kernels_slab(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  const int ndz = 2 * h->sD + 1;
  const size_t plane = (size_t)h->Ly * h->Kx;
  int rc = dalloc(h, &h->kern_t, sizeof(T) * 6 * ndz * plane);
  if (rc) return rc;
  const bool need_s = d.sigma > 0 || d.cross_mode == 1;
  if (need_s && (rc = dalloc(h, &h->kern_s, sizeof(T) * 3 * ndz * plane))) return rc;
  mmv_mesh tmp_owner;
  void *grid = nullptr, *s1 = nullptr, *s2 = nullptr, *twxd = nullptr, *twpd = nullptr, *twyd = nullptr;
  rc = dalloc(&tmp_owner, &grid, sizeof(double) * (size_t)h->Lx * h->Ly);
  if (!rc) rc = dalloc(&tmp_owner, &s1, 2 * sizeof(double) * plane);
  if (!rc) rc = dalloc(&tmp_owner, &s2, 2 * sizeof(double) * plane);
  if (!rc) rc = upload_tw(&tmp_owner, &twxd, h->N2x, h->N2x, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twpd, h->Lx, h->N2x + 1, true);
  if (!rc) rc = upload_tw(&tmp_owner, &twyd, h->Ly, h->Ly, true);
  if (rc) {
    free_all(&tmp_owner);
    return rc;
  }
  const double inv = 1.0 / ((double)h->Lx * h->Ly);
  // stored part of each spectrum: tensor xz, yz and S x, y are imaginary
  const int imag_t[6] = {0, 0, 0, 0, 1, 1}, imag_s[3] = {1, 1, 0};
  hipError_t err = hipSuccess;
  for (int kind = 0; kind < (need_s ? 2 : 1) && err == hipSuccess; ++kind) {
    const int ncomp = kind == SLAB_KIND_TENSOR ? 6 : 3;
    for (int comp = 0; comp < ncomp && err == hipSuccess; ++comp) {
      for (int dz = -h->sD; dz <= h->sD && err == hipSuccess; ++dz) {
        // tensor spectra carry -Ms (Eq. 6); S spectra enter the eddy sums bare
        const double sc = kind == SLAB_KIND_TENSOR ? -d.Ms * inv : inv;
        err = launch_kernel_real((double*)grid, h->Lx, h->Ly, kind, comp, (double)dz, d.dx, d.dy, d.dz, d.rc_cells,
                                 sc, d.pbc, d.pbc_images, h->st);
        if (err == hipSuccess)
          err = launch_row_fwd<double>((const double*)grid, s1, h->Ly, h->Lx, h->N2x, h->Kx, h->px, twxd, twpd, h->st);
        if (err == hipSuccess)
          err = launch_fft_axis<double>(s1, s2, 1, h->Kx, 0, h->Ly, 0, h->Ly, 0, h->py, twyd, false, h->st);
        T* dst = (T*)(kind == SLAB_KIND_TENSOR ? h->kern_t : h->kern_s) + ((size_t)comp * ndz + dz + h->sD) * plane;
        if (err == hipSuccess)
          err = launch_slab_pack<T>(s2, dst, (int)plane, kind == SLAB_KIND_TENSOR ? imag_t[comp] : imag_s[comp], h->st);
      }
    }
  }
  if (err == hipSuccess) err = hipStreamSynchronize(h->st);
  free_all(&tmp_owner);
  if (err != hipSuccess) return fail(MMV_EHIP, std::string("kernel construction: ") + hipGetErrorString(err));
  return MMV_OK;
}

template <typename T>
int init_slab(mmv_mesh* h) {
  const mmv_mesh_desc& d = h->d;
  h->esz = sizeof(T);
  const int nz = h->nz, ny = h->ny, nx = h->nx, M = h->M;
  const size_t ncell = (size_t)nx * ny * nz, F = 3 * ncell;
  const size_t plane = (size_t)h->Ly * h->Kx, cs = 2 * sizeof(T);
  const int zs = nz + d.gap_cells, hl = d.halo;
  const bool pot = d.cross_mode == 1;
  // layer offsets of the kernel spectra: the windows reach z_s + nz (direct)
  // or z_s + nz + 2 with the potential's layers below the base reaching -3
  h->sD = pot ? zs + nz + 3 : zs + nz;
  int rc;
  void** bufs[] = {&h->m0, &h->mb[0], &h->mb[1], &h->acc, &h->hd, &h->he};
  for (void** b : bufs)
    if ((rc = dalloc(h, b, 2 * F * sizeof(T)))) return rc;
  const bool eddy = d.sigma > 0;
  size_t chP = std::max<size_t>(9 * (size_t)nz + 3 * (size_t)(nz + 2), eddy ? 12 * (size_t)nz : 0);
  size_t rowsI = std::max<size_t>(9 * (size_t)nz * ny + 3 * (size_t)(nz + 2) * (ny + 2),
                                  eddy ? 12 * (size_t)nz * ny : 0);
  if (pot) {
    chP = std::max<size_t>(chP, 6 * (size_t)nz + (nz + 6) + (nz + 4));
    rowsI = std::max<size_t>(rowsI, 6 * (size_t)nz * ny + (size_t)(nz + 6) * (ny + 6) + (size_t)(nz + 4) * (ny + 4));
    if ((rc = dalloc(h, &h->pot_w[0], sizeof(T) * (size_t)(nz + 6) * (ny + 6) * M))) return rc;
    if ((rc = dalloc(h, &h->pot_w[1], sizeof(T) * (size_t)(nz + 4) * (ny + 4) * M))) return rc;
    if ((rc = dalloc(h, &h->pot_s[0], sizeof(T) * (size_t)(nz + 6) * (ny + 6) * (nx + 6)))) return rc;
    if ((rc = dalloc(h, &h->pot_s[1], sizeof(T) * (size_t)(nz + 4) * (ny + 4) * (nx + 4)))) return rc;
  }
  if ((rc = dalloc(h, &h->spec1, cs * 2 * 3 * nz * (size_t)ny * h->Kx))) return rc;
  if ((rc = dalloc(h, &h->specM, cs * 2 * 3 * nz * plane))) return rc;
  if ((rc = dalloc(h, &h->specP, cs * chP * plane))) return rc;
  if ((rc = dalloc(h, &h->specI, cs * rowsI * h->Kx))) return rc;
  if ((rc = dalloc(h, &h->win_s2b, sizeof(T) * 3 * (size_t)nz * ny * M))) return rc;
  if ((rc = dalloc(h, &h->win_b2s, sizeof(T) * 3 * (size_t)(nz + 2) * (ny + 2) * M))) return rc;
  if ((rc = dalloc(h, &h->stencil, sizeof(T) * 3 * (size_t)(nz + 2) * (ny + 2) * (nx + 2)))) return rc;
  if ((rc = dalloc(h, (void**)&h->partial, sizeof(double) * 3 * (size_t)slab_force_blocks((int)ncell)))) return rc;
  if (eddy) {
    void** e2[] = {&h->bdot, &h->es};
    for (void** b : e2)
      if ((rc = dalloc(h, b, 2 * F * sizeof(T)))) return rc;
    void** e1[] = {&h->phi, &h->phi2, &h->rr};
    for (void** b : e1)
      if ((rc = dalloc(h, b, 2 * ncell * sizeof(T)))) return rc;
    if ((rc = dalloc(h, (void**)&h->Bprev, 2 * F * sizeof(double)))) return rc;
    if ((rc = dalloc(h, &h->win_e, sizeof(T) * 2 * 3 * (size_t)nz * ny * M))) return rc;
    if ((rc = dalloc(h, (void**)&h->red, sizeof(double) * (ncell / 256 + 4)))) return rc;
    HIPCHK(hipMemsetAsync(h->phi, 0, 2 * ncell * sizeof(T), h->st));
  }
  HIPCHK(hipMemsetAsync(h->he, 0, 2 * F * sizeof(T), h->st));
  if ((rc = upload_tw(h, &h->twx, h->N2x, h->N2x, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twp, h->Lx, h->N2x + 1, sizeof(T) == 8))) return rc;
  if ((rc = upload_tw(h, &h->twy, h->Ly, h->Ly, sizeof(T) == 8))) return rc;
  if ((rc = dalloc(h, (void**)&h->rigid, sizeof(RigidState)))) return rc;
  RigidState r{};
  HIPCHK(hipMemcpyAsync(h->rigid, &r, sizeof(r), hipMemcpyHostToDevice, h->st));
  std::vector<T> mz(2 * F, T(0));
  for (int f = 0; f < 2; ++f)
    for (size_t i = 0; i < ncell; ++i) mz[f * F + 2 * ncell + i] = T(1);
  HIPCHK(hipMemcpyAsync(h->m0, mz.data(), mz.size() * sizeof(T), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if ((rc = build_kernels_slab<T>(h))) return rc;
  // target windows of the two products (mmv_slab.h): the films' own fields,
  // the slider's field on the base (x0 = -s_int - h), the base's field on
  // the slider (x0 = s_int - h; with rows -1..ny and layers z_s-1..z_s+nz
  // for the tensor product); every group [3][ntz][Ly][Kx]
  const long long P = (long long)plane;
  // potential mode: the films' own fields (the tensor table's first two
  // groups) and the potentials of the other film on the windows
  // a periodic x keeps the windows' period unshifted (columns from 0; the
  // sampling reads them modulo nx), a periodic y the rows of the period
  const bool px = (d.pbc & 1) != 0, py = (d.pbc & 2) != 0;
  h->tab_p.n = 2;
  h->tab_p.g[0] = SlabGroup{0, zs - 3, nz + 6, px ? 0 : 1, px ? 0 : -hl, py ? 0 : -3, 6LL * nz * P};
  h->tab_p.g[1] = SlabGroup{1, -zs - 2, nz + 4, px ? 0 : -1, px ? 0 : -hl, py ? 0 : -2, (6LL * nz + nz + 6) * P};
  h->tab_t.n = 4;
  h->tab_t.g[0] = SlabGroup{0, 0, nz, 0, 0, 0, 0};
  h->tab_t.g[1] = SlabGroup{1, 0, nz, 0, 0, 0, 3LL * nz * P};
  h->tab_t.g[2] = SlabGroup{1, -zs, nz, px ? 0 : -1, px ? 0 : -hl, 0, 6LL * nz * P};
  h->tab_t.g[3] = SlabGroup{0, zs - 1, nz + 2, px ? 0 : 1, px ? 0 : -hl, py ? 0 : -1, 9LL * nz * P};
  h->tab_e.n = 4;
  h->tab_e.g[0] = SlabGroup{0, 0, nz, 0, 0, 0, 0};
  h->tab_e.g[1] = SlabGroup{1, 0, nz, 0, 0, 0, 3LL * nz * P};
  h->tab_e.g[2] = SlabGroup{1, -zs, nz, px ? 0 : -1, px ? 0 : -hl, 0, 6LL * nz * P};
  h->tab_e.g[3] = SlabGroup{0, zs, nz, px ? 0 : 1, px ? 0 : -hl, 0, 9LL * nz * P};
  CubeLaunch& c = h->cl;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.dx = d.dx;
  c.dy = d.dy;
  c.dz = d.dz;
  c.pref_ex = 2.0 * d.Aex / (MU0 * d.Ms);
  c.pref_an = 2.0 * d.Ku / (MU0 * d.Ms);
  const double un = sqrt(d.u[0] * d.u[0] + d.u[1] * d.u[1] + d.u[2] * d.u[2]);
  for (int i = 0; i < 3; ++i) {
    c.u[i] = un > 0 ? d.u[i] / un : 0.0;
    c.hext[i] = d.Hext[i];
  }
  c.gam = GAMMA0 / (1.0 + d.alpha * d.alpha);
  c.alpha = d.alpha;
  h->sor_sweeps = d.sor_sweeps != 0 ? d.sor_sweeps : 40;
  const int nmax = std::max(nx, std::max(ny, nz));
  h->sor_omega = d.sor_omega > 0 ? d.sor_omega : 2.0 / (1.0 + sin(M_PI / nmax));
  if ((rc = init_dct<T>(h))) return rc;
  // a periodic x lets the slider travel without bound
  h->rp_hot.travel = h->rp_force.travel = px ? (1 << 30) : d.max_travel_cells;
  h->rp_hot.halo = h->rp_force.halo = hl;
  c.pbc = d.pbc;
  return MMV_OK;
}

// Fields of both films at the state m ([2][3][nz][ny][nx]) and the current
// slider stage: hd = the films' own fields (self) plus the other film's
// sampled field (cross) plus the non-uniform applied field (zee: film 0's
// values, the slider's samples of the frame field); the force partials of
// Eq. 3 (always, from the stray field alone).
template <typename T>
int slab_fields(mmv_mesh* h, const T* m, bool self_on, bool cross_on, bool zee_on) {
  const int nz = h->nz, ny = h->ny, nx = h->nx, Kx = h->Kx, M = h->M;
  const size_t F = 3 * (size_t)nx * ny * nz;
  const size_t P = (size_t)h->Ly * Kx;
  const int R = slab_rows_per_block(h->N2x);
  const double idx = 1.0 / h->d.dx;
  const int interp = h->d.cross_mode == 2 ? 1 : 0;
  HIPCHK(launch_row_fwd<T>(m, h->spec1, 6 * nz * ny, nx, h->N2x, Kx, h->px, h->twx, h->twp, h->st, -R));
  HIPCHK(launch_fft_axis<T>(h->spec1, h->specM, 6 * nz, Kx, 0, ny, (long long)ny * Kx, h->Ly, (long long)P, h->py,
                            h->twy, false, h->st));
  char* pI = (char*)h->specI;
  const size_t cs = 2 * sizeof(T);
  if (h->d.cross_mode == 1) {
    // the films' own fields (tensor groups 0, 1), the other film's potential
    // on the windows (Eqs. 7-8), sampled along x, four-point differences
    SlabMulTable own = h->tab_t;
    own.n = 2;
    HIPCHK(launch_slab_mul<T>(h->specM, h->specP, (const T*)h->kern_t, own, nz, h->sD, h->Lx, h->Ly, Kx, 0, 1.0,
                              h->rigid, h->st));
    HIPCHK(launch_slab_pot<T>(h->specM, h->specP, (const T*)h->kern_s, h->tab_p, nz, h->sD, h->Lx, h->Ly, Kx,
                              h->d.Ms, h->rigid, h->st));
    const int L1 = nz + 6, R1 = ny + 6, L2 = nz + 4, R2 = ny + 4;
    // periodic axes: the windows hold the period (WC columns, W1 / W2 rows
    // per layer); the sampler reads window rows -3..ny+2 (-2..ny+1) and the
    // columns from +-s_int - halo modulo the period, the copy of the
    // potential from the other side
    const bool px = (h->d.pbc & 1) != 0, py = (h->d.pbc & 2) != 0;
    const int WC = px ? nx : M, W1 = py ? ny : R1, W2 = py ? ny : R2, hl = h->d.halo;
    const size_t o1 = 6 * (size_t)nz * ny, o2 = o1 + (size_t)L1 * W1;
    HIPCHK(launch_fft_axis<T>(h->specP, pI, 6 * nz, Kx, 0, h->Ly, (long long)P, ny, (long long)ny * Kx, h->py, h->twy,
                              true, h->st));
    HIPCHK(launch_fft_axis<T>((char*)h->specP + cs * 6 * nz * P, pI + cs * o1 * Kx, L1, Kx, 0, h->Ly, (long long)P, W1,
                              (long long)W1 * Kx, h->py, h->twy, true, h->st));
    HIPCHK(launch_fft_axis<T>((char*)h->specP + cs * (6 * nz + L1) * P, pI + cs * o2 * Kx, L2, Kx, 0, h->Ly,
                              (long long)P, W2, (long long)W2 * Kx, h->py, h->twy, true, h->st));
    HIPCHK(launch_row_inv<T>(pI, (T*)h->hd, 6 * nz * ny, R, nx, h->N2x, Kx, h->px, h->twx, h->twp, h->st));
    HIPCHK(launch_row_inv<T>(pI + cs * o1 * Kx, (T*)h->pot_w[0], L1 * W1, R, WC, h->N2x, Kx, h->px, h->twx, h->twp,
                             h->st));
    HIPCHK(launch_row_inv<T>(pI + cs * o2 * Kx, (T*)h->pot_w[1], L2 * W2, R, WC, h->N2x, Kx, h->px, h->twx, h->twp,
                             h->st));
    if (!self_on) HIPCHK(hipMemsetAsync(h->hd, 0, 2 * F * sizeof(T), h->st));
    const SlabRows r1{1, L1 * R1, L1 * W1, R1, W1, py ? -3 : 0, M, WC, px ? 1 : 0, px ? -hl : 0, px ? nx : 0};
    const SlabRows r2{1, L2 * R2, L2 * W2, R2, W2, py ? -2 : 0, M, WC, px ? -1 : 0, px ? -hl : 0, px ? nx : 0};
    // slider side: samples at i = -3 .. nx + 2, then H on the force stencil
    // (stencil point (l', j', i') at window layer l' + 2, row j' + 2, sample i' + 2)
    HIPCHK(launch_slab_sample<T>((const T*)h->pot_w[0], r1, h->d.halo, (T*)h->pot_s[0], -3, nx + 6, 1, 0, 0, idx,
                                 h->rigid, h->st));
    HIPCHK(launch_slab_potgrad<T>((const T*)h->pot_s[0], R1, nx + 6, 2, nz + 2, ny + 2, nx + 2, (T*)h->stencil, 0,
                                  h->d.dx, h->d.dy, h->d.dz, h->st));
    if (cross_on) {
      // base side: samples at i = -2 .. nx + 1; base cell (k, j, i) at window
      // layer k + 2, row j + 2, sample i + 2
      HIPCHK(launch_slab_sample<T>((const T*)h->pot_w[1], r2, h->d.halo, (T*)h->pot_s[1], -2, nx + 4, -1, 0, 0, idx,
                                   h->rigid, h->st));
      HIPCHK(launch_slab_potgrad<T>((const T*)h->pot_s[1], R2, nx + 4, 2, nz, ny, nx, (T*)h->hd, 1, h->d.dx, h->d.dy,
                                    h->d.dz, h->st));
    }
  } else {
    // window widths and rows: a periodic x keeps the period (the windows'
    // columns are read modulo nx), a periodic y the ny rows of the period
    // (the force's rows -1 and ny are rows ny - 1 and 0)
    const bool px = (h->d.pbc & 1) != 0, py = (h->d.pbc & 2) != 0;
    const int WC = px ? nx : M, WR = py ? ny : ny + 2;
    HIPCHK(launch_slab_mul<T>(h->specM, h->specP, (const T*)h->kern_t, h->tab_t, nz, h->sD, h->Lx, h->Ly, Kx, 0, 1.0,
                              h->rigid, h->st));
    HIPCHK(launch_fft_axis<T>(h->specP, pI, 9 * nz, Kx, 0, h->Ly, (long long)P, ny, (long long)ny * Kx, h->py, h->twy,
                              true, h->st));
    HIPCHK(launch_fft_axis<T>((char*)h->specP + cs * 9 * nz * P, pI + cs * 9 * (size_t)nz * ny * Kx, 3 * (nz + 2), Kx,
                              0, h->Ly, (long long)P, WR, (long long)WR * Kx, h->py, h->twy, true, h->st));
    HIPCHK(launch_row_inv<T>(pI, (T*)h->hd, 6 * nz * ny, R, nx, h->N2x, Kx, h->px, h->twx, h->twp, h->st));
    HIPCHK(launch_row_inv<T>(pI + cs * 6 * (size_t)nz * ny * Kx, (T*)h->win_s2b, 3 * nz * ny, R, WC, h->N2x, Kx,
                             h->px, h->twx, h->twp, h->st));
    HIPCHK(launch_row_inv<T>(pI + cs * 9 * (size_t)nz * ny * Kx, (T*)h->win_b2s, 3 * (nz + 2) * WR, R, WC, h->N2x, Kx,
                             h->px, h->twx, h->twp, h->st));
    if (!self_on) HIPCHK(hipMemsetAsync(h->hd, 0, 2 * F * sizeof(T), h->st));
    // base side: lattice columns -s_int - h + k of the slider's field; slider
    // side: s_int - h + k of the base's (periodic x), rows -1..ny
    const int hl = h->d.halo;
    const SlabRows rs{3, nz * ny, nz * ny, nz * ny, nz * ny, 0, M, WC, px ? -1 : 0, px ? -hl : 0, px ? nx : 0};
    const SlabRows rb{3, (nz + 2) * (ny + 2), (nz + 2) * WR, ny + 2, WR, py ? -1 : 0, M, WC, px ? 1 : 0, px ? -hl : 0,
                      px ? nx : 0};
    if (cross_on)
      HIPCHK(launch_slab_sample<T>((const T*)h->win_s2b, rs, hl, (T*)h->hd, 0, nx, -1, 1, interp, idx, h->rigid, h->st));
    HIPCHK(launch_slab_sample<T>((const T*)h->win_b2s, rb, hl, (T*)h->stencil, -1, nx + 2, 1, 0, interp, idx, h->rigid,
                                 h->st));
  }
  HIPCHK(launch_slab_force<T>((const T*)h->stencil, m + F, (T*)h->hd + F, nx, ny, nz, cross_on ? 1 : 0, h->d.dx,
                              h->d.dy, h->d.dz, h->partial, h->st));
  if (zee_on && h->slab_hext[0]) HIPCHK(launch_slab_add<T>((int)F, (const T*)h->slab_hext[0], (T*)h->hd, h->st));
  if (zee_on && h->slab_hext[1]) {
    // the slider's window of the frame rows starts at column s_int + travel
    // (periodic x: the frame is the period, the window from s_int - halo)
    const bool px = (h->d.pbc & 1) != 0;
    const int W = px ? nx : nx + 2 * (h->d.max_travel_cells + h->d.halo);
    const SlabRows rz{3, nz * ny, nz * ny, nz * ny, nz * ny, 0, M, W, 1,
                      px ? -h->d.halo : h->d.max_travel_cells, px ? nx : 0};
    HIPCHK(launch_slab_sample<T>((const T*)h->slab_hext[1], rz, h->d.halo, (T*)h->hd + F, 0, nx, 1, 1, interp, idx,
                                 h->rigid, h->st));
  }
  return MMV_OK;
}

// sgn * sum over both films of S x src (own film: lattice sum; other film:
// sampled window), src and dst [2][3][nz][ny][nx]
template <typename T>
int slab_s_sum(mmv_mesh* h, const T* src, T* dst, double sgn) {
  const int nz = h->nz, ny = h->ny, nx = h->nx, Kx = h->Kx, M = h->M;
  const size_t F = 3 * (size_t)nx * ny * nz;
  const size_t P = (size_t)h->Ly * Kx;
  const int R = slab_rows_per_block(h->N2x);
  const size_t cs = 2 * sizeof(T);
  const int interp = h->d.cross_mode == 2 ? 1 : 0;
  char* pI = (char*)h->specI;
  HIPCHK(launch_row_fwd<T>(src, h->spec1, 6 * nz * ny, nx, h->N2x, Kx, h->px, h->twx, h->twp, h->st, -R));
  HIPCHK(launch_fft_axis<T>(h->spec1, h->specM, 6 * nz, Kx, 0, ny, (long long)ny * Kx, h->Ly, (long long)P, h->py,
                            h->twy, false, h->st));
  HIPCHK(launch_slab_mul<T>(h->specM, h->specP, (const T*)h->kern_s, h->tab_e, nz, h->sD, h->Lx, h->Ly, Kx, 1, sgn,
                            h->rigid, h->st));
  HIPCHK(launch_fft_axis<T>(h->specP, pI, 12 * nz, Kx, 0, h->Ly, (long long)P, ny, (long long)ny * Kx, h->py, h->twy,
                            true, h->st));
  HIPCHK(launch_row_inv<T>(pI, dst, 6 * nz * ny, R, nx, h->N2x, Kx, h->px, h->twx, h->twp, h->st));
  // a periodic x keeps the windows' period (columns read modulo nx from
  // -s_int - h on the base and s_int - h on the slider)
  const bool px = (h->d.pbc & 1) != 0;
  const int WC = px ? nx : M, hl = h->d.halo;
  HIPCHK(launch_row_inv<T>(pI + cs * 6 * (size_t)nz * ny * Kx, (T*)h->win_e, 6 * nz * ny, R, WC, h->N2x, Kx, h->px,
                           h->twx, h->twp, h->st));
  const size_t wsz = 3 * (size_t)nz * ny * WC;
  const int nr = nz * ny;
  const SlabRows rs{3, nr, nr, nr, nr, 0, M, WC, px ? -1 : 0, px ? -hl : 0, px ? nx : 0};
  const SlabRows rb{3, nr, nr, nr, nr, 0, M, WC, px ? 1 : 0, px ? -hl : 0, px ? nx : 0};
  HIPCHK(launch_slab_sample<T>((const T*)h->win_e, rs, hl, dst, 0, nx, -1, 1, interp, 1.0 / h->d.dx, h->rigid,
                               h->st));
  HIPCHK(launch_slab_sample<T>((const T*)h->win_e + wsz, rb, hl, dst + F, 0, nx, 1, 1, interp, 1.0 / h->d.dx,
                               h->rigid, h->st));
  return MMV_OK;
}

// Eddy-current update at the start of a step, from the fields hd of its
// first stage (held through the step's stages).
template <typename T>
int slab_eddy(mmv_mesh* h, const T* m, double dt) {
  const size_t ncell = (size_t)h->nx * h->ny * h->nz, F = 3 * ncell;
  double* mean = h->red + (ncell / 256 + 2);
  HIPCHK(launch_slab_bdot<T>((int)(2 * F), (int)ncell, (const T*)h->hd, m, h->d.Hext, MU0, h->d.Ms, 1.0 / dt,
                             h->eddy_first ? 1 : 0, h->Bprev, (T*)h->bdot, h->st));
  h->eddy_first = false;
  int rc = slab_s_sum<T>(h, (const T*)h->bdot, (T*)h->es, +1.0);
  if (rc) return rc;
  for (int f = 0; f < 2; ++f)
    HIPCHK(launch_sor_rhs<T>(h->cl, (T*)h->es + f * F, (T*)h->rr + f * ncell, h->red, mean, h->st));
  // the two films' Neumann problems in the same launches
  if (h->sor_sweeps < 0)
    HIPCHK(launch_neumann_solve<T>(h->cl, 2, (const T*)h->rr, (T*)h->phi, (T*)h->phi2, h->pdct, h->twdct, h->st));
  else
    HIPCHK(launch_sor<T>(h->cl, 2, (T*)h->phi, (T*)h->phi2, (const T*)h->rr, h->sor_omega, h->sor_sweeps, h->red,
                         mean, h->st));
  for (int f = 0; f < 2; ++f)
    HIPCHK(launch_current<T>(h->cl, (T*)h->phi + f * ncell, (T*)h->es + f * F, (T*)h->bdot + f * F, h->d.sigma,
                             h->st));
  return slab_s_sum<T>(h, (const T*)h->bdot, (T*)h->he, -1.0);
}

TickArgs slab_tick(mmv_mesh* h) {
  TickArgs a{};
  a.partial = h->partial;
  a.rigid = h->rigid;
  a.drive = h->drive;
  a.force_scale = MU0 * h->d.Ms * h->d.dx * h->d.dy * h->d.dz;
  a.dx = h->d.dx;
  a.ntask = slab_force_blocks(h->nx * h->ny * h->nz);
  a.travel = h->rp_hot.travel;
  a.scheme = 0;
  a.ctrl = nullptr;
  return a;
}

template <typename T>
int step_slab(mmv_mesh* h, double dt, int nsteps) {
  T* m0 = (T*)h->m0;
  T* b1 = (T*)h->mb[0];
  T* b2 = (T*)h->mb[1];
  const size_t F = 3 * (size_t)h->nx * h->ny * h->nz;
  const TickArgs tick = slab_tick(h);
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 4; ++s) {
      T* in = s == 0 ? m0 : (s == 1 ? b1 : (s == 2 ? b2 : b1));
      T* out = s == 0 ? b1 : (s == 1 ? b2 : (s == 2 ? b1 : m0));
      int rc = slab_fields<T>(h, in, true, true, true);
      if (rc) return rc;
      if (s == 0 && h->d.sigma > 0 && (rc = slab_eddy<T>(h, m0, dt))) return rc;
      // the slider's stage from this stage's force (after every sampling of
      // the stage has read its position)
      HIPCHK(launch_tick(tick, s, dt, h->st));
      for (int f = 0; f < 2; ++f)
        HIPCHK(launch_stage3<T>(h->cl, MODE_STAGE, s, MMV_TERM_ALL, dt, in + f * F, m0 + f * F, out + f * F,
                                (T*)h->acc + f * F, (const T*)h->hd + f * F, (const T*)h->he + f * F, nullptr,
                                &h->rigid->flags, nullptr, nullptr, h->st));
    }
  }
  return MMV_OK;
}

template <typename T>
int eval_slab(mmv_mesh* h, int film, int mask, void* hout) {
  const size_t F = 3 * (size_t)h->nx * h->ny * h->nz;
  const bool zee = (mask & MMV_TERM_ZEEMAN) && (h->slab_hext[0] || h->slab_hext[1]);
  const bool dem = (mask & (MMV_TERM_DEMAG_SELF | MMV_TERM_DEMAG_CROSS)) != 0 || zee;
  if (dem) {
    int rc = slab_fields<T>(h, (const T*)h->m0, (mask & MMV_TERM_DEMAG_SELF) != 0, (mask & MMV_TERM_DEMAG_CROSS) != 0,
                            zee);
    if (rc) return rc;
  }
  const int m3 = (mask & (MMV_TERM_EXCHANGE | MMV_TERM_ANISOTROPY | MMV_TERM_ZEEMAN | MMV_TERM_EDDY)) |
                 (dem ? MMV_TERM_DEMAG_SELF : 0);
  const T* m0 = (const T*)h->m0 + film * F;
  HIPCHK(launch_stage3<T>(h->cl, MODE_EVAL, 0, m3, 0.0, m0, m0, nullptr, nullptr, (const T*)h->hd + film * F,
                          (const T*)h->he + film * F, (T*)hout, &h->rigid->flags, nullptr, nullptr, h->st));
  return MMV_OK;
}

// Eq. 3's force at the current state [N] (blocks on the stream).
template <typename T>
int force_slab(mmv_mesh* h, double F_out[3]) {
  int rc = slab_fields<T>(h, (const T*)h->m0, true, true, false);
  if (rc) return rc;
  const int nb = slab_force_blocks(h->nx * h->ny * h->nz);
  std::vector<double> part(3 * (size_t)nb);
  HIPCHK(hipMemcpyAsync(part.data(), h->partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  const double sc = MU0 * h->d.Ms * h->d.dx * h->d.dy * h->d.dz;
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[3 * (size_t)b + a];
    F_out[a] = sc * s;
  }
  return MMV_OK;
}

template <typename T>
void* mptr(mmv_mesh* h, void* base, int film) {
  return (char*)base + (size_t)film * 3 * h->nx * h->ny * sizeof(T);
}

int check_handle(mmv_handle h) {
  if (!h) return fail(MMV_EINVAL, "handle is NULL");
  return MMV_OK;
}

TickArgs tick_args(mmv_mesh* h, int ntask) {
  TickArgs a{};
  a.partial = h->partial;
  a.rigid = h->rigid;
  a.drive = h->drive;
  a.force_scale = h->rp_hot.force_scale;
  a.dx = h->d.dx;
  a.ntask = ntask;
  a.travel = h->rp_hot.travel;
  return a;
}

// tick_stage >= 0: the y pass also applies the slider update of the row
// launch of that stage (whose force partials are in h->partial)
template <typename T>
int run_fields(mmv_mesh* h, const void* m_in, const OutTable& tab, bool fwd = true, int tick_stage = -1,
               int tick_ntask = 0, double tick_dt = 0.0) {
  if (fwd) {
    PROF(1);
    HIPCHK(launch_row_fwd<T>((const T*)m_in, h->spec1, 3 * h->nfilm * h->ny, h->nx, h->N2x, h->Kx, h->px, h->twx,
                             h->twp, h->st, h->ny));
    PROF(1);
  }
  PROF(2);
  const TickArgs ta = tick_args(h, tick_ntask);
  HIPCHK(launch_col<T>(h->spec1, h->spec2, (const T*)h->kern, h->Kx, h->Ly, h->Kyh, h->ny, 3 * h->nfilm, h->ngroup,
                       h->py, h->twy, tab, h->st, tick_stage >= 0 ? &ta : nullptr, tick_stage, tick_dt));
  PROF(2);
  return MMV_OK;
}

template <typename T>
int eval_typed(mmv_mesh* h, int film, int mask, void* hout);

// Error judge of the learned operator: exact cross field on film 0 against
// the network's, at the state at the start of the step.
template <typename T>
int sur_judge(mmv_mesh* h) {
  int rc = eval_typed<T>(h, 0, MMV_TERM_DEMAG_CROSS, h->sur_exact);
  if (rc) return rc;
  const size_t plane = (size_t)h->ny * h->nx;
  HIPCHK(launch_sur_input((const float*)h->m0 + 3 * plane, h->rigid, 1.0 / h->d.dx, h->ny, h->nx, h->sur_in, h->st));
  const float* pred = nullptr;
  if ((rc = sur_infer(h->sur, h->sur_in, 1, h->st, &pred))) return rc;
  double e = 0.0;
  if ((rc = sur_rel_err(h->sur, pred, h->sur_exact, (long long)3 * plane, h->d.Ms, h->st, &e))) return rc;
  h->sur_err = e;
  h->sur_judged += 1;
  if (!(e <= h->sur_tol)) h->sur_fallback = 1;
  return MMV_OK;
}

template <typename T>
int step_typed(mmv_mesh* h, double dt, int nsteps) {
  RowParams rp = h->rp_hot;
  rp.mode = MODE_STAGE;
  rp.term_mask = MMV_TERM_ALL;
  rp.dt = dt;
  rp.drive = h->drive;
  rp.with_force = (h->nfilm == 2 && h->drive.mode == MMV_DRIVE_SPRING) ? 1 : 0;
  rp.full_force = 0;
  rp.ntask = h->nfilm * h->ny + ((rp.with_force && rp.pot) ? 2 : 0);
  // after the first stage the x-pass input comes from the row kernel
  rp.spec1_out = h->fuse_fwd ? h->spec1 : nullptr;
  // the slider update of each row launch is applied by the next y pass (or
  // by a one-block kernel when something else must see it first)
  rp.defer_tick = 1;
  const TickArgs ta = tick_args(h, rp.ntask);
  int pending = -1;
  T* m0 = (T*)h->m0;
  T* b1 = (T*)h->mb[0];
  T* b2 = (T*)h->mb[1];
  const size_t plane = (size_t)h->ny * h->nx;
  for (int n = 0; n < nsteps; ++n) {
    if (h->sur && !h->sur_fallback && h->sur_steps % h->sur_every == 0) {
      if (pending >= 0) HIPCHK(launch_tick(ta, pending, dt, h->st));
      pending = -1;
      int rc = sur_judge<T>(h);
      if (rc) return rc;
    }
    const bool use_sur = h->sur && !h->sur_fallback;
    for (int s = 0; s < 4; ++s) {
      T* in = s == 0 ? m0 : (s == 1 ? b1 : (s == 2 ? b2 : b1));
      T* out = s == 0 ? b1 : (s == 1 ? b2 : (s == 2 ? b1 : m0));
      int rc;
      const bool fwd = !h->fuse_fwd || (n == 0 && s == 0);
      if (use_sur) {
        // the network reads this stage's slider offset: apply the update first
        if (pending >= 0) HIPCHK(launch_tick(ta, pending, dt, h->st));
        pending = -1;
        // film 0's cross field from the network at this stage's slider state
        HIPCHK(launch_sur_input((const float*)in + 3 * plane, h->rigid, 1.0 / h->d.dx, h->ny, h->nx, h->sur_in,
                                h->st));
        const float* pred = nullptr;
        if ((rc = sur_infer(h->sur, h->sur_in, 1, h->st, &pred))) return rc;
        rp.hsur = pred;
        rp.sur_scale = h->d.Ms;
        rc = run_fields<T>(h, in, h->tab_sur, fwd);
      } else {
        rp.hsur = nullptr;
        rc = run_fields<T>(h, in, h->tab_hot, fwd, pending, rp.ntask, dt);
        pending = -1;
      }
      if (rc) return rc;
      rp.stage = s;
      PROF(3);
      HIPCHK(launch_row_stage<T>(rp, h->spec2, in, m0, out, (T*)h->acc, nullptr, h->twx, h->twp, h->rigid,
                                 h->partial, h->counter, h->st));
      PROF(3);
      pending = s;
    }
    if (h->sur) h->sur_steps += 1;
  }
  if (pending >= 0) HIPCHK(launch_tick(ta, pending, dt, h->st));
  return MMV_OK;
}

template <typename T>
int eval_typed(mmv_mesh* h, int film, int mask, void* hout) {
  if (mask & (MMV_TERM_DEMAG_SELF | MMV_TERM_DEMAG_CROSS)) {
    int rc = run_fields<T>(h, h->m0, h->tab_hot);
    if (rc) return rc;
  }
  RowParams rp = h->rp_hot;
  rp.mode = MODE_EVAL;
  rp.eval_film = film;
  rp.term_mask = mask & 31;
  rp.with_force = 0;
  rp.full_force = 0;
  rp.ntask = h->ny;
  rp.drive = h->drive;
  HIPCHK(launch_row_stage<T>(rp, h->spec2, (const T*)h->m0, (const T*)h->m0, nullptr, nullptr, (T*)hout, h->twx,
                             h->twp, h->rigid, h->partial, h->counter, h->st));
  return MMV_OK;
}

// Eq. 3 force at the current state: the force rows' field pass, then one
// row-kernel launch whose blocks write float64 partials [ny + 2][3] and whose
// last block (arrival counter) sums them in a fixed order into fout (NULL:
// the slider state's F).
template <typename T>
int force_typed(mmv_mesh* h, double* partial, unsigned* counter, double* fout) {
  int rc = run_fields<T>(h, h->m0, h->tab_force);
  if (rc) return rc;
  RowParams rp = h->rp_force;
  rp.mode = MODE_FORCE;
  rp.term_mask = 0;
  rp.with_force = 1;
  rp.full_force = 1;
  rp.ntask = h->ny + 2;
  rp.drive = h->drive;
  rp.fout = fout;
  HIPCHK(launch_row_stage<T>(rp, h->spec2, (const T*)h->m0, (const T*)h->m0, nullptr, nullptr, nullptr, h->twx,
                             h->twp, h->rigid, partial, counter, h->st));
  return MMV_OK;
}

// Attempts of the adaptive Dormand-Prince run (Sec. III): per attempt the x
// pass of m, seven stages (y pass with the previous stage's slider update,
// row kernel writing the stage derivative and the next stage's state), the
// step control and the commit of an accepted state.  Every launch reads the
// step size from the device; after t_end they return at once.
template <typename T>
int dp_attempts(mmv_mesh* h, int n) {
  RowParams rp = h->rp_hot;
  rp.mode = MODE_STAGE;
  rp.term_mask = MMV_TERM_ALL;
  rp.drive = h->drive;
  rp.with_force = (h->nfilm == 2 && h->drive.mode == MMV_DRIVE_SPRING) ? 1 : 0;
  rp.full_force = 0;
  rp.ntask = h->nfilm * h->ny + ((rp.with_force && rp.pot) ? 2 : 0);
  rp.defer_tick = 1;
  rp.hsur = nullptr;
  rp.scheme = 1;
  rp.kdp = h->kdp;
  rp.errpart = h->errpart;
  rp.ctrl = h->dpc;
  TickArgs ta = tick_args(h, rp.ntask);
  ta.scheme = 1;
  ta.ctrl = h->dpc;
  T* m0 = (T*)h->m0;
  T* b1 = (T*)h->mb[0];
  T* b2 = (T*)h->mb[1];
  const size_t plane = (size_t)h->ny * h->nx;
  for (int a = 0; a < n; ++a) {
    int pending = -1;
    for (int i = 0; i < 7; ++i) {
      T* in = i == 0 ? m0 : ((i & 1) ? b1 : b2);
      T* out = (i & 1) ? b2 : b1;
      if (i == 0 || !h->fuse_fwd)
        HIPCHK(launch_row_fwd<T>(in, h->spec1, 3 * h->nfilm * h->ny, h->nx, h->N2x, h->Kx, h->px, h->twx, h->twp,
                                 h->st, h->ny));
      HIPCHK(launch_col<T>(h->spec1, h->spec2, (const T*)h->kern, h->Kx, h->Ly, h->Kyh, h->ny, 3 * h->nfilm,
                           h->ngroup, h->py, h->twy, h->tab_hot, h->st, &ta, pending, 0.0));
      rp.stage = i;
      rp.spec1_out = (i < 6 && h->fuse_fwd) ? h->spec1 : nullptr;
      HIPCHK(launch_row_stage<T>(rp, h->spec2, in, m0, out, (T*)h->acc, nullptr, h->twx, h->twp, h->rigid,
                                 h->partial, h->counter, h->st));
      pending = i;
    }
    HIPCHK(launch_dp_control(ta, h->dpc, h->errpart, rp.ntask, h->st));
    HIPCHK(launch_dp_commit<T>(b2, m0, h->nfilm, plane, h->dpc, &h->rigid->flags, h->st));
  }
  return MMV_OK;
}

// Eq. 13 at the current state: the force pass writes the base field on the
// slider's stencil points, then per row the sums of |div| and |curl|.
template <typename T>
int div_curl_typed(mmv_mesh* h, double* D, double* C) {
  const size_t gsz = (size_t)3 * (h->ny + 2) * (h->nx + 2) + (size_t)6 * h->ny * h->nx;
  int rc;
  if (!h->divfield && (rc = dalloc(h, &h->divfield, sizeof(T) * gsz))) return rc;
  if (!h->divpart && (rc = dalloc(h, (void**)&h->divpart, sizeof(double) * 2 * (size_t)h->ny))) return rc;
  if ((rc = run_fields<T>(h, h->m0, h->tab_force))) return rc;
  RowParams rp = h->rp_force;
  rp.mode = MODE_FORCE;
  rp.term_mask = 0;
  rp.with_force = 1;
  rp.full_force = 1;
  rp.ntask = h->ny + 2;
  rp.drive = h->drive;
  rp.fieldout = h->divfield;
  HIPCHK(launch_row_stage<T>(rp, h->spec2, (const T*)h->m0, (const T*)h->m0, nullptr, nullptr, nullptr, h->twx,
                             h->twp, h->rigid, h->partial, h->counter, h->st));
  HIPCHK(launch_div_curl<T>((const T*)h->divfield, h->nx, h->ny, h->d.dx, h->d.dy, h->d.dz, (h->d.pbc & 2) ? 1 : 0,
                            h->divpart, h->st));
  std::vector<double> part(2 * (size_t)h->ny);
  HIPCHK(hipMemcpyAsync(part.data(), h->divpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  double sd = 0.0, sc = 0.0;
  for (int y = 0; y < h->ny; ++y) {
    sd += part[2 * y];
    sc += part[2 * y + 1];
  }
  const double n = (double)h->nx * h->ny;
  *D = sd / n;
  *C = sc / n;
  return MMV_OK;
}

int read_rigid(mmv_mesh* h, RigidState& r) {
  HIPCHK(hipMemcpyAsync(&r, h->rigid, sizeof(r), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return MMV_OK;
}

int write_rigid(mmv_mesh* h, const RigidState& r) {
  HIPCHK(hipMemcpyAsync(h->rigid, &r, sizeof(r), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return MMV_OK;
}

int report_flags(mmv_mesh* h, RigidState& r) {
  if (r.flags == 0) return MMV_OK;
  const int f = r.flags;
  r.flags = 0;
  int rc = write_rigid(h, r);
  if (rc) return rc;
  if (f & FLAG_NUMERIC) return fail(MMV_ENUMERIC, "non-finite magnetisation or slider state");
  return fail(MMV_ERANGE, "slider left the window the FFT lengths were sized for (max_travel_cells)");
}

// Static scratch of stray_force_noalloc (the entry point for callers that
// cannot allocate): the float64 force partials of the row blocks followed by
// the launch's arrival counter.  One copy per device, held until the process
// ends; its device address is resolved once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64 * 1024;
constexpr size_t NOALLOC_COUNTER_BYTES = 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

size_t noalloc_partial_bytes(int ntask) { return ((size_t)ntask * 3 * sizeof(double) + 255) & ~size_t(255); }

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;

// Device address of this device's scratch (host code must not use the
// array's name: on the host it only stands in for the symbol).
int noalloc_scratch(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MMV_EHIP, "hipGetSymbolAddress returned NULL for the static scratch");
    it = g_scratch_ptr.emplace(dev, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return MMV_OK;
}

}  // namespace


// ---------------------------------------------------------------- batches
// One launch of a batched pass over a class of instances: their descriptors
// at [off, off + n) of the pass's array, block starts at soff.
struct BatchLaunch {
  int off = 0, n = 0, soff = 0, nblk = 0;
  size_t lds = 0;
  bool inplace = false;
  int nt = 0;  // row kernel: threads per block
};

struct mmv_batch {
  std::vector<mmv_mesh*> inst;
  hipStream_t st = nullptr;
  hipStream_t gst = nullptr;
  int esz = 4;
  int flags = 0;
  std::vector<void*> allocs;
  // Descriptor arrays (device), instances ordered by launch class, and the
  // classes' block-start tables (class c's table at its soff, n + 1 entries).
  RowFwdDesc* d_fwd[4] = {};
  ColDesc* d_col = nullptr;
  ColDesc* d_col_all = nullptr;  // every instance in batch order (closing slider tick)
  RowStageDesc* d_stage[4] = {};
  bool fuse = false;  // every instance x-transforms its new rows in the row kernel
  int *s_fwd = nullptr, *s_col = nullptr, *s_stage = nullptr;
  // one launch per class of instances with the same launch shape (dynamic
  // LDS, transform variant): small meshes are not held to the LDS of the
  // largest, so more of their blocks share a CU
  std::vector<BatchLaunch> l_fwd, l_col, l_stage;
  std::vector<int> stage_inst;  // instance of each row-stage descriptor (class order)
  // learned operator for every instance's film-0 cross field (not owned):
  // one batched inference per RK stage over all instances
  mmv_sur* sur = nullptr;
  int sur_every = 10, sur_fallback = 0;
  double sur_tol = 1e-3, sur_err = -1.0;
  long sur_judged = 0, sur_steps = 0;
  float* sur_in = nullptr;     // [n][4][ny][nx]
  float* sur_exact = nullptr;  // [n][3][ny][nx]
  bool built_sur = false;      // the descriptors read the operator's output
  std::vector<DriveP> drive_sig;  // drives the stage and tick descriptors were built for
  std::vector<long> hext_sig;     // applied-field generations they were built for
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  double g_dt = 0.0;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // the launch classes of one pass touch disjoint instances: they run on
  // side streams forked from the launching stream and joined back into it
  // (in a captured graph, parallel branches), so that one class's blocks
  // fill the CUs another class's tail leaves idle
  static constexpr int NSIDE = 3;
  hipStream_t side[NSIDE] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[NSIDE] = {};
};

namespace {

int balloc(mmv_batch* b, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) return fail(MMV_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  b->allocs.push_back(*p);
  return MMV_OK;
}

RowParams stage_params(mmv_mesh* h, bool fuse) {
  RowParams rp = h->rp_hot;
  rp.spec1_out = fuse ? h->spec1 : nullptr;
  rp.defer_tick = 1;
  rp.mode = MODE_STAGE;
  rp.term_mask = MMV_TERM_ALL;
  rp.drive = h->drive;
  rp.with_force = (h->drive.mode == MMV_DRIVE_SPRING) ? 1 : 0;
  rp.full_force = 0;
  rp.ntask = h->nfilm * h->ny + ((rp.with_force && rp.pot) ? 2 : 0);
  return rp;
}

// Threads per block of the batched row kernel for one instance: the tuned
// value if it is valid, else the smallest of 128, 256, 512 that is at least
// nx (one cell per thread in the force sums, as in the single-mesh kernel).
template <typename T>
int batch_row_threads(const mmv_mesh* h, const RowParams& rp) {
  if (h->row_nt >= h->nx && row_batch_threads_ok<T>(h->row_nt, rp.inplace != 0)) return h->row_nt;
  for (int nt : {128, 256})
    if (nt >= h->nx && row_batch_threads_ok<T>(nt, rp.inplace != 0)) return nt;
  return 512;
}

// Rows per transform batch of the batched row kernel for one instance:
// a direct-mode stage task needs at most 8 inverse transforms (7 except the
// slider's first and last rows).  Pick the batch size that lets the most
// blocks share a CU (LDS, and 2048 threads per CU), then the largest at that
// occupancy (at least 3: the fused forward transform of the new row's three
// components).
template <typename T>
int batch_rows_per_transform(const RowParams& rp, size_t limit, int nt) {
  if (rp.pot) return rp.nbr;
  int best = 0, best_occ = 0;
  for (int nb = std::min(rp.nbr, 8); nb >= 3; --nb) {
    RowParams q = rp;
    q.nbr = nb;
    const size_t lds = row_lds_bytes<T>(q) + ROW_STATIC_LDS;
    if (lds > limit) continue;
    const int occ = std::min(2048 / nt, (int)((160 * 1024) / (((lds + 511) / 512) * 512)));
    if (occ > best_occ) {
      best_occ = occ;
      best = nb;
    }
  }
  return best ? best : rp.nbr;
}

// Group instance indices by key (stable), one class per distinct key.
template <typename K>
std::vector<std::vector<int>> group_by(const std::vector<K>& key) {
  std::vector<int> idx(key.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return key[a] < key[c]; });
  std::vector<std::vector<int>> out;
  for (size_t k = 0; k < idx.size(); ++k) {
    if (k == 0 || key[idx[k]] != key[idx[k - 1]]) out.emplace_back();
    out.back().push_back(idx[k]);
  }
  return out;
}

// (Re)build the per-instance descriptors, launch classes and block tables.
template <typename T>
int batch_build(mmv_batch* b) {
  const int n = (int)b->inst.size();
  std::vector<RowFwdDesc> fwd_i[4], fwd[4];
  std::vector<RowStageDesc> stg_i[4], stg[4];
  std::vector<ColDesc> col_i(n), col;
  std::vector<int> sf, sc, ss;
  std::vector<size_t> k_fwd(n), k_col(n);
  std::vector<std::tuple<size_t, int, int>> k_stage(n);
  const bool use_sur = b->sur != nullptr && !b->sur_fallback;
  const float* sur_out = use_sur ? sur_output(b->sur) : nullptr;
  b->built_sur = use_sur;
  b->drive_sig.assign(n, DriveP{});
  b->hext_sig.assign(n, 0);
  b->fuse = true;
  for (int i = 0; i < n; ++i) b->fuse = b->fuse && b->inst[i]->fuse_fwd;
  const size_t lds_limit = LDS_PER_CU - ROW_STATIC_LDS;
  for (int i = 0; i < n; ++i) {
    mmv_mesh* h = b->inst[i];
    b->drive_sig[i] = h->drive;
    b->hext_sig[i] = h->hext_gen;
    T* m0 = (T*)h->m0;
    T* b1 = (T*)h->mb[0];
    T* b2 = (T*)h->mb[1];
    RowParams rp = stage_params(h, b->fuse);
    const int nt = batch_row_threads<T>(h, rp);
    rp.nbr = batch_rows_per_transform<T>(rp, lds_limit, nt);
    if (use_sur) {
      // film 0's cross field from the operator's output of this instance
      rp.hsur = sur_out + (size_t)i * 3 * h->ny * h->nx;
      rp.sur_scale = h->d.Ms;
    }
    for (int s = 0; s < 4; ++s) {
      T* in = s == 0 ? m0 : (s == 1 ? b1 : (s == 2 ? b2 : b1));
      T* out = s == 0 ? b1 : (s == 1 ? b2 : (s == 2 ? b1 : m0));
      RowFwdDesc f{};
      f.src = in;
      f.dst = h->spec1;
      f.nin = h->nx;
      f.N2x = h->N2x;
      f.Kx = h->Kx;
      f.ny = h->ny;
      f.P = h->px;
      f.tw = h->twx;
      f.twp = h->twp;
      fwd_i[s].push_back(f);
      RowStageDesc r{};
      r.p = rp;
      r.spec2 = h->spec2;
      r.mst = in;
      r.m0 = m0;
      r.mnext = out;
      r.acc = h->acc;
      r.tw = h->twx;
      r.twp = h->twp;
      r.rigid = h->rigid;
      r.partial = h->partial;
      r.counter = h->counter;
      stg_i[s].push_back(r);
    }
    ColDesc& c = col_i[i];
    c.spec1 = h->spec1;
    c.spec2 = h->spec2;
    c.kern = h->kern;
    c.Kx = h->Kx;
    c.Ly = h->Ly;
    c.Kyh = h->Kyh;
    c.ny = h->ny;
    c.nin_ch = 3 * h->nfilm;
    c.ngroup = h->ngroup;
    const int per = ((use_sur ? h->tab_sur.n : h->tab_hot.n) + h->ngroup - 1) / h->ngroup;
    c.nbuf = c.nin_ch > per ? c.nin_ch : per;
    c.P = h->py;
    c.twy = h->twy;
    c.tab = use_sur ? h->tab_sur : h->tab_hot;
    c.tick = tick_args(h, rp.ntask);
    k_fwd[i] = row_fwd_lds_bytes(h->N2x, sizeof(T));
    k_col[i] = col_lds_bytes<T>(h->Ly, c.nbuf);
    k_stage[i] = std::make_tuple(row_lds_bytes<T>(rp), rp.inplace, nt);
  }
  // launch classes: descriptors in class order, one block-start table each
  auto make = [&](const std::vector<std::vector<int>>& groups, std::vector<BatchLaunch>& L, std::vector<int>& st,
                  auto blocks, auto lds_of, auto fill) {
    L.clear();
    st.clear();
    int off = 0;
    for (const auto& g : groups) {
      BatchLaunch c;
      c.off = off;
      c.n = (int)g.size();
      c.soff = (int)st.size();
      int acc = 0;
      for (int i : g) {
        st.push_back(acc);
        acc += blocks(i);
        c.lds = std::max(c.lds, lds_of(i));
        fill(i);
      }
      st.push_back(acc);
      c.nblk = acc;
      c.inplace = std::get<1>(k_stage[g[0]]) != 0;
      c.nt = std::get<2>(k_stage[g[0]]);
      off += c.n;
      L.push_back(c);
    }
  };
  for (int s = 0; s < 4; ++s) {
    fwd[s].clear();
    stg[s].clear();
  }
  make(group_by(k_fwd), b->l_fwd, sf, [&](int i) { return b->inst[i]->nfilm * b->inst[i]->ny; },
       [&](int i) { return k_fwd[i]; }, [&](int i) {
         for (int s = 0; s < 4; ++s) fwd[s].push_back(fwd_i[s][i]);
       });
  make(group_by(k_col), b->l_col, sc, [&](int i) { return b->inst[i]->Kx * b->inst[i]->ngroup; },
       [&](int i) { return k_col[i]; }, [&](int i) { col.push_back(col_i[i]); });
  b->stage_inst.clear();
  make(group_by(k_stage), b->l_stage, ss, [&](int i) { return stg_i[0][i].p.ntask; },
       [&](int i) { return std::get<0>(k_stage[i]); }, [&](int i) {
         for (int s = 0; s < 4; ++s) stg[s].push_back(stg_i[s][i]);
         b->stage_inst.push_back(i);
       });
  int rc;
  if (!b->d_col) {
    for (int s = 0; s < 4; ++s) {
      if ((rc = balloc(b, (void**)&b->d_fwd[s], sizeof(RowFwdDesc) * n))) return rc;
      if ((rc = balloc(b, (void**)&b->d_stage[s], sizeof(RowStageDesc) * n))) return rc;
    }
    if ((rc = balloc(b, (void**)&b->d_col, sizeof(ColDesc) * n))) return rc;
    if ((rc = balloc(b, (void**)&b->d_col_all, sizeof(ColDesc) * n))) return rc;
    // at most one class per instance: n + 1 + (classes - 1) <= 2 n entries
    if ((rc = balloc(b, (void**)&b->s_fwd, sizeof(int) * 2 * (n + 1)))) return rc;
    if ((rc = balloc(b, (void**)&b->s_col, sizeof(int) * 2 * (n + 1)))) return rc;
    if ((rc = balloc(b, (void**)&b->s_stage, sizeof(int) * 2 * (n + 1)))) return rc;
  }
  for (int s = 0; s < 4; ++s) {
    HIPCHK(hipMemcpyAsync(b->d_fwd[s], fwd[s].data(), sizeof(RowFwdDesc) * n, hipMemcpyHostToDevice, b->st));
    HIPCHK(hipMemcpyAsync(b->d_stage[s], stg[s].data(), sizeof(RowStageDesc) * n, hipMemcpyHostToDevice, b->st));
  }
  HIPCHK(hipMemcpyAsync(b->d_col, col.data(), sizeof(ColDesc) * n, hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->d_col_all, col_i.data(), sizeof(ColDesc) * n, hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->s_fwd, sf.data(), sizeof(int) * sf.size(), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->s_col, sc.data(), sizeof(int) * sc.size(), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->s_stage, ss.data(), sizeof(int) * ss.size(), hipMemcpyHostToDevice, b->st));
  size_t mf = 0, mc = 0, ms = 0;
  for (auto& c : b->l_fwd) mf = std::max(mf, c.lds);
  for (auto& c : b->l_col) mc = std::max(mc, c.lds);
  for (auto& c : b->l_stage) ms = std::max(ms, c.lds);
  HIPCHK(prepare_batch_kernels<T>(mf, mc, ms));
  HIPCHK(hipStreamSynchronize(b->st));
  if (getenv("MMV_VERBOSE"))
    for (auto& c : b->l_stage)
      fprintf(stderr, "mmv: batch row class: %d instances, %d blocks of %d threads, LDS %zu, in place %d\n", c.n,
              c.nblk, c.nt, c.lds, (int)c.inplace);
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  return MMV_OK;
}

// Launch every class of a pass, class k on side stream k - 1 (class 0, and
// classes past the side streams, on st), forked from and joined into st.
template <typename F>
int batch_classes(mmv_batch* b, hipStream_t st, const std::vector<BatchLaunch>& L, F launch) {
  const int n = (int)L.size();
  if (n <= 1) {
    for (const BatchLaunch& c : L) HIPCHK(launch(c, st));
    return MMV_OK;
  }
  HIPCHK(hipEventRecord(b->ev_fork, st));
  const int nside = std::min(n - 1, mmv_batch::NSIDE);
  for (int k = 0; k < nside; ++k) HIPCHK(hipStreamWaitEvent(b->side[k], b->ev_fork, 0));
  for (int k = 0; k < n; ++k) {
    hipStream_t s = (k >= 1 && k <= nside) ? b->side[k - 1] : st;
    HIPCHK(launch(L[k], s));
  }
  for (int k = 0; k < nside; ++k) {
    HIPCHK(hipEventRecord(b->ev_join[k], b->side[k]));
    HIPCHK(hipStreamWaitEvent(st, b->ev_join[k], 0));
  }
  return MMV_OK;
}

// The y pass of every class (its block 0 per instance applies the pending
// slider stage when tick_stage >= 0).
template <typename T>
int batch_col_launches(mmv_batch* b, hipStream_t st, int tick_stage, double dt) {
  return batch_classes(b, st, b->l_col, [&](const BatchLaunch& c, hipStream_t s) {
    return launch_col_batch<T>(b->d_col + c.off, b->s_col + c.soff, c.n, c.nblk, c.lds, s, tick_stage, dt);
  });
}

// The row kernel of every class at stage s.
template <typename T>
int batch_stage_launches(mmv_batch* b, hipStream_t st, int s, double dt) {
  return batch_classes(b, st, b->l_stage, [&](const BatchLaunch& c, hipStream_t q) {
    return launch_row_stage_batch<T>(b->d_stage[s] + c.off, b->s_stage + c.soff, c.n, c.nblk, c.lds, s, dt,
                                     c.inplace, c.nt, q);
  });
}

template <typename T>
int eval_typed(mmv_mesh* h, int film, int mask, void* hout);

// Inputs of the batched operator: each instance's slider magnetisation of
// the stage and its offset x_s / dx.
template <typename T>
int batch_sur_inputs(mmv_batch* b, int stage, hipStream_t st) {
  for (size_t i = 0; i < b->inst.size(); ++i) {
    mmv_mesh* h = b->inst[i];
    const T* in = stage == 0 ? (const T*)h->m0 : (stage == 2 ? (const T*)h->mb[1] : (const T*)h->mb[0]);
    const size_t plane = (size_t)h->ny * h->nx;
    HIPCHK(launch_sur_input((const float*)in + 3 * plane, h->rigid, 1.0 / h->d.dx, h->ny, h->nx,
                            b->sur_in + i * 4 * plane, st));
  }
  return MMV_OK;
}

// Error judge of the batched operator at the step-start state: the exact
// cross field of every instance against the network's, relative L2 over the
// whole batch; above tol every instance falls back to the exact path.
template <typename T>
int batch_sur_judge(mmv_batch* b, hipStream_t st) {
  const int n = (int)b->inst.size();
  const size_t plane = (size_t)b->inst[0]->ny * b->inst[0]->nx;
  for (int i = 0; i < n; ++i) {
    int rc = eval_typed<T>(b->inst[i], 0, MMV_TERM_DEMAG_CROSS, b->sur_exact + (size_t)i * 3 * plane);
    if (rc) return rc;
  }
  int rc = batch_sur_inputs<T>(b, 0, st);
  if (rc) return rc;
  const float* pred = nullptr;
  if ((rc = sur_infer(b->sur, b->sur_in, n, st, &pred))) return rc;
  double e = 0.0;
  if ((rc = sur_rel_err(b->sur, pred, b->sur_exact, (long long)n * 3 * plane, b->inst[0]->d.Ms, st, &e)))
    return rc;
  b->sur_err = e;
  b->sur_judged += 1;
  if (!(e <= b->sur_tol)) b->sur_fallback = 1;
  return MMV_OK;
}

// Steps with the operator: before each stage the pending slider stage is
// applied (the network reads the stage offset), the operator runs once over
// all instances, then the y pass without film 0's cross channels and the
// row kernel reading the operator's output.
template <typename T>
int batch_sur_steps(mmv_batch* b, hipStream_t st, double dt, int nsteps, int* done) {
  const int n = (int)b->inst.size();
  int pending = -1;
  *done = 0;
  for (int k = 0; k < nsteps; ++k) {
    if (b->sur_steps % b->sur_every == 0) {
      if (pending >= 0) HIPCHK(launch_tick_batch(b->d_col_all, n, pending, dt, st));
      pending = -1;
      int rc = batch_sur_judge<T>(b, st);
      if (rc) return rc;
      if (b->sur_fallback) break;
    }
    for (int s = 0; s < 4; ++s) {
      if (pending >= 0) HIPCHK(launch_tick_batch(b->d_col_all, n, pending, dt, st));
      pending = -1;
      int rc = batch_sur_inputs<T>(b, s, st);
      if (rc) return rc;
      const float* pred = nullptr;
      if ((rc = sur_infer(b->sur, b->sur_in, n, st, &pred))) return rc;
      if (!b->fuse || (k == 0 && s == 0))
        for (const BatchLaunch& c : b->l_fwd)
          HIPCHK(launch_row_fwd_batch<T>(b->d_fwd[s] + c.off, b->s_fwd + c.soff, c.n, c.nblk, c.lds, st));
      if ((rc = batch_col_launches<T>(b, st, -1, dt))) return rc;
      if ((rc = batch_stage_launches<T>(b, st, s, dt))) return rc;
      pending = s;
    }
    b->sur_steps += 1;
    *done += 1;
  }
  if (pending >= 0) HIPCHK(launch_tick_batch(b->d_col_all, n, pending, dt, st));
  return MMV_OK;
}

template <typename T>
int batch_launch_steps(mmv_batch* b, hipStream_t st, double dt, int nsteps) {
  const int n = (int)b->inst.size();
  mmv_mesh* h0 = b->inst[0];  // timing events of the first instance's profile slot
  int pending = -1;           // stage whose slider update the next y pass applies
  for (int k = 0; k < nsteps; ++k)
    for (int s = 0; s < 4; ++s) {
      mmv_mesh* h = h0;
      if (!b->fuse || (k == 0 && s == 0)) {
        PROF(1);
        for (const BatchLaunch& c : b->l_fwd)
          HIPCHK(launch_row_fwd_batch<T>(b->d_fwd[s] + c.off, b->s_fwd + c.soff, c.n, c.nblk, c.lds, st));
        PROF(1);
      }
      PROF(2);
      int rc = batch_col_launches<T>(b, st, pending, dt);
      if (rc) return rc;
      PROF(2);
      PROF(3);
      if ((rc = batch_stage_launches<T>(b, st, s, dt))) return rc;
      PROF(3);
      pending = s;
    }
  if (pending >= 0) HIPCHK(launch_tick_batch(b->d_col_all, n, pending, dt, st));
  return MMV_OK;
}

constexpr int GRAPH_STEPS = 8;

bool same_drive(const DriveP& a, const DriveP& c) {
  return a.mode == c.mode && a.v_d == c.v_d && a.k == c.k && a.mass == c.mass && a.gamma_v == c.gamma_v &&
         a.xa0 == c.xa0;
}

template <typename T>
int batch_step_typed(mmv_batch* b, double dt, int nsteps) {
  // the descriptors carry each instance's drive by value: any change made by
  // set_drive since they were built rebuilds them (and drops the graph)
  bool rebuild = b->built_sur != (b->sur != nullptr && !b->sur_fallback);
  for (size_t i = 0; i < b->inst.size(); ++i)
    if (!same_drive(b->inst[i]->drive, b->drive_sig[i]) || b->inst[i]->hext_gen != b->hext_sig[i]) rebuild = true;
  if (rebuild) {
    int rc = batch_build<T>(b);
    if (rc) return rc;
  }
  if (b->sur && !b->sur_fallback) {
    int done = 0;
    int rc = batch_sur_steps<T>(b, b->st, dt, nsteps, &done);
    if (rc) return rc;
    if (done == nsteps) return MMV_OK;
    // the judge sent the batch back to the exact path
    if ((rc = batch_build<T>(b))) return rc;
    return batch_launch_steps<T>(b, b->st, dt, nsteps - done);
  }
  const bool graph = (b->flags & MMV_BATCH_GRAPH) && b->inst[0]->prof_kernel == 0;
  if (!graph) return batch_launch_steps<T>(b, b->st, dt, nsteps);
  int done = 0;
  if (nsteps >= GRAPH_STEPS) {
    if (!b->exec || b->g_dt != dt) {
      if (b->exec) {
        hipGraphExecDestroy(b->exec);
        hipGraphDestroy(b->graph);
        b->exec = nullptr;
      }
      HIPCHK(hipStreamBeginCapture(b->gst, hipStreamCaptureModeThreadLocal));
      int rc = batch_launch_steps<T>(b, b->gst, dt, GRAPH_STEPS);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->gst, &g);
      if (rc) return rc;
      if (e != hipSuccess) return fail(MMV_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      b->graph = g;
      HIPCHK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
      b->g_dt = dt;
    }
    HIPCHK(hipEventRecord(b->ev_in, b->st));
    HIPCHK(hipStreamWaitEvent(b->gst, b->ev_in, 0));
    for (; done + GRAPH_STEPS <= nsteps; done += GRAPH_STEPS) HIPCHK(hipGraphLaunch(b->exec, b->gst));
    HIPCHK(hipEventRecord(b->ev_out, b->gst));
    HIPCHK(hipStreamWaitEvent(b->st, b->ev_out, 0));
  }
  return batch_launch_steps<T>(b, b->st, dt, nsteps - done);
}

// Tuning cache on disk (process-wide path; empty = none).  One line per
// tuned mesh size: "<key>\t<groups>", the key naming the device (arch, CU
// count), the precision, the batch's size mix (FNV-1a over the instances'
// (Kx, Ly) in order) and the size.  Unreadable or malformed lines are
// ignored; the file is rewritten whole (temporary file + rename).
std::string g_tune_cache;

std::map<std::string, int> tune_cache_read(const std::string& path) {
  std::map<std::string, int> m;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return m;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char* tab = strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    char* end = nullptr;
    const long g = strtol(tab + 1, &end, 10);
    if (end == tab + 1 || g < 1 || g > 8) continue;
    m[line] = (int)g;
  }
  fclose(f);
  return m;
}

bool tune_cache_write(const std::string& path, const std::map<std::string, int>& m) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = true;
  for (const auto& kv : m) ok = ok && fprintf(f, "%s\t%d\n", kv.first.c_str(), kv.second) > 0;
  ok = (fclose(f) == 0) && ok;
  if (ok) ok = rename(tmp.c_str(), path.c_str()) == 0;
  if (!ok) remove(tmp.c_str());
  return ok;
}

std::string tune_key(const mmv_batch* b, const std::pair<int, int>& sz) {
  int dev = 0;
  hipDeviceProp_t prop;
  memset(&prop, 0, sizeof prop);
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
  unsigned long long hsh = 1469598103934665603ull;
  auto mix = [&](unsigned v) {
    for (int k = 0; k < 4; ++k) {
      hsh ^= (v >> (8 * k)) & 0xffu;
      hsh *= 1099511628211ull;
    }
  };
  for (const mmv_mesh* h : b->inst) {
    mix((unsigned)h->Kx);
    mix((unsigned)h->Ly);
  }
  char buf[320];
  snprintf(buf, sizeof buf, "%s cu%d f%d n%d mix%016llx Kx%d Ly%d", prop.gcnArchName, prop.multiProcessorCount,
           b->esz * 8, (int)b->inst.size(), hsh, sz.first, sz.second);
  return std::string(buf);
}

// Autotuner: per mesh size, time the batched y pass for each grouping of
// that size's instances (others fixed) and keep the fastest.  With a tuning
// cache, sizes tuned before for the same device, precision and size mix take
// the stored grouping without timing; new results are added to the file.
template <typename T>
int batch_autotune(mmv_batch* b) {
  std::vector<std::pair<int, int>> sizes;
  for (mmv_mesh* h : b->inst) {
    std::pair<int, int> k(h->Kx, h->Ly);
    if (std::find(sizes.begin(), sizes.end(), k) == sizes.end()) sizes.push_back(k);
  }
  const bool use_cache = !g_tune_cache.empty();
  std::map<std::string, int> cache;
  if (use_cache) cache = tune_cache_read(g_tune_cache);
  bool added = false;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int n = (int)b->inst.size();
  for (auto& sz : sizes) {
    const std::string key = use_cache ? tune_key(b, sz) : std::string();
    auto hit = key.empty() ? cache.end() : cache.find(key);
    if (hit != cache.end()) {
      for (mmv_mesh* h : b->inst)
        if (h->Kx == sz.first && h->Ly == sz.second) h->ngroup = hit->second;
      continue;
    }
    int best = b->inst[0]->ngroup;
    float best_ms = 1e30f;
    for (int g : {1, 2, 3, 4}) {
      for (mmv_mesh* h : b->inst)
        if (h->Kx == sz.first && h->Ly == sz.second) h->ngroup = g;
      int rc = batch_build<T>(b);
      if (rc) return rc;
      if ((rc = batch_col_launches<T>(b, b->st, -1, 0.0))) return rc;
      HIPCHK(hipEventRecord(e0, b->st));
      for (int r = 0; r < 5; ++r)
        if ((rc = batch_col_launches<T>(b, b->st, -1, 0.0))) return rc;
      HIPCHK(hipEventRecord(e1, b->st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = g;
      }
    }
    for (mmv_mesh* h : b->inst)
      if (h->Kx == sz.first && h->Ly == sz.second) h->ngroup = best;
    if (!key.empty()) {
      cache[key] = best;
      added = true;
    }
  }
  // Row kernel: per row length, the block size (128, 256 or 512 threads, at
  // least the widest nx of that length), timed over the stage-0 row launches
  // of the whole batch (they write only stage buffers, the accumulator and
  // the next x pass's spectra, all rewritten by the next step).  Cached as
  // threads / 64.
  std::vector<int> lens;
  for (mmv_mesh* h : b->inst)
    if (std::find(lens.begin(), lens.end(), h->N2x) == lens.end()) lens.push_back(h->N2x);
  for (int len : lens) {
    int nxmax = 0;
    for (mmv_mesh* h : b->inst)
      if (h->N2x == len) nxmax = std::max(nxmax, h->nx);
    std::vector<int> cand;
    for (int nt : {128, 256, 512})
      if (nt >= nxmax && row_batch_threads_ok<T>(nt, row_inplace_length(len))) cand.push_back(nt);
    if (cand.size() < 2) continue;
    const std::string key = use_cache ? tune_key(b, std::make_pair(len, 0)) + " row" : std::string();
    auto hit = key.empty() ? cache.end() : cache.find(key);
    if (hit != cache.end()) {
      for (mmv_mesh* h : b->inst)
        if (h->N2x == len) h->row_nt = 64 * hit->second;
      continue;
    }
    int best = cand.back();
    float best_ms = 1e30f;
    for (int nt : cand) {
      for (mmv_mesh* h : b->inst)
        if (h->N2x == len) h->row_nt = nt;
      int rc = batch_build<T>(b);
      if (rc) return rc;
      auto launches = [&]() -> int { return batch_stage_launches<T>(b, b->st, 0, 0.0); };
      if ((rc = launches())) return rc;
      HIPCHK(hipEventRecord(e0, b->st));
      for (int r = 0; r < 5; ++r)
        if ((rc = launches())) return rc;
      HIPCHK(hipEventRecord(e1, b->st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = nt;
      }
    }
    for (mmv_mesh* h : b->inst)
      if (h->N2x == len) h->row_nt = best;
    if (!key.empty()) {
      cache[key] = best / 64;
      added = true;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (added && !tune_cache_write(g_tune_cache, cache))
    fprintf(stderr, "mmv: could not write the tuning cache %s\n", g_tune_cache.c_str());
  return batch_build<T>(b);
}

bool same_kernel(const mmv_mesh_desc& a, const mmv_mesh_desc& c) {
  return a.nx == c.nx && a.ny == c.ny && a.dx == c.dx && a.dy == c.dy && a.dz == c.dz && a.gap_cells == c.gap_cells &&
         a.Ms == c.Ms && a.rc_cells == c.rc_cells && a.cross_mode == c.cross_mode && a.halo == c.halo &&
         a.max_travel_cells == c.max_travel_cells && a.fft_lx == c.fft_lx && a.fft_ly == c.fft_ly &&
         a.pbc == c.pbc && a.pbc_images == c.pbc_images;
}

void batch_free(mmv_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (void* p : b->allocs) hipFree(p);
  for (mmv_mesh* h : b->inst) {
    for (hipEvent_t e : h->prof_ev) hipEventDestroy(e);
    free_all(h);
    delete h;
  }
  if (b->gst) hipStreamDestroy(b->gst);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  for (int k = 0; k < mmv_batch::NSIDE; ++k) {
    if (b->side[k]) hipStreamDestroy(b->side[k]);
    if (b->ev_join[k]) hipEventDestroy(b->ev_join[k]);
  }
  delete b;
}

}  // namespace

extern "C" {

const char* mmv_last_error(void) { return g_err.c_str(); }

int init_mesh(const mmv_mesh_desc* d, void* hip_stream, mmv_handle* out) {
  g_err.clear();
  if (!out) return fail(MMV_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  mmv_mesh* h = new mmv_mesh();
  h->d = *d;
  h->st = (hipStream_t)hip_stream;
  h->nfilm = d->n_films;
  h->nx = d->nx;
  h->ny = d->ny;
  if (d->n_films == 1 && d->nz > 1) {
    h->cube = true;
    h->nz = d->nz;
    h->Lx = d->fft_lx ? d->fft_lx : next_smooth(2 * d->nx - 1, true);
    h->Ly = d->fft_ly ? d->fft_ly : next_smooth(2 * d->ny - 1, false);
    h->Lz = d->fft_lz ? d->fft_lz : next_smooth(2 * d->nz - 1, false);
    if (h->Lx < 2 * d->nx - 1 || h->Lx % 2 || !smooth2357(h->Lx) || h->Ly < 2 * d->ny - 1 || !smooth2357(h->Ly) ||
        h->Lz < 2 * d->nz - 1 || !smooth2357(h->Lz)) {
      delete h;
      return fail(MMV_EINVAL, "FFT lengths must be {2,3,5,7}-smooth and >= 2n-1 per axis (Lx even)");
    }
    h->N2x = h->Lx / 2;
    h->Kx = h->N2x + 1;
    h->Kyh = h->Ly / 2 + 1;
    if (!make_plan(h->N2x, h->px) || !make_plan(h->Ly, h->py) || !make_plan(h->Lz, h->pz)) {
      delete h;
      return fail(MMV_EINVAL, "FFT length has too many factors");
    }
    // LDS of one block of each 3-D pass at its smallest batch (one row or
    // column): x transforms (4 N2x + 1), y and z transforms (3 L) in float64
    // for the kernel build and in the mesh precision, the z pass with the
    // kernel product (7 Lz) in the mesh precision
    const size_t es = d->precision == 64 ? 16 : 8, lim = 160 * 1024;
    const bool lds_ok = 16 * (4 * (size_t)h->N2x + 1) <= lim && 16 * 3 * (size_t)h->Ly <= lim &&
                        16 * 3 * (size_t)h->Lz <= lim && es * 7 * (size_t)h->Lz <= lim;
    if (!lds_ok || (long long)d->nx * d->ny * d->nz >= (1LL << 31)) {
      delete h;
      return fail(MMV_EINVAL, "mesh too large for the three-dimensional path");
    }
    rc = d->precision == 64 ? init_cube<double>(h) : init_cube<float>(h);
    if (rc) {
      free_all(h);
      delete h;
      return rc;
    }
    *out = h;
    return MMV_OK;
  }
  if (d->n_films == 2 && d->nz > 1) {
    // two thick films: in-plane transforms sized as for one-layer films
    h->slab = true;
    h->nz = d->nz;
    // the windows reach one row past the films (direct mode: the force's
    // rows) or three (the potential's four-point differences and the force)
    // a periodic axis is transformed over its period
    const int lx_min = (d->pbc & 1) ? d->nx : 2 * (d->nx + d->halo + d->max_travel_cells),
              ly_min = (d->pbc & 2) ? d->ny : 2 * (d->ny + (d->cross_mode == 1 ? 3 : 1));
    h->Lx = d->fft_lx ? d->fft_lx : ((d->pbc & 1) ? d->nx : next_smooth(lx_min, true));
    h->Ly = d->fft_ly ? d->fft_ly : ((d->pbc & 2) ? d->ny : next_smooth(ly_min, false));
    if (h->Lx < lx_min || h->Lx % 2 || !smooth2357(h->Lx) || h->Ly < ly_min || !smooth2357(h->Ly)) {
      delete h;
      return fail(MMV_EINVAL, "fft_lx must be even, {2,3,5,7}-smooth and >= " + std::to_string(lx_min) +
                                  "; fft_ly {2,3,5,7}-smooth and >= " + std::to_string(ly_min));
    }
    h->N2x = h->Lx / 2;
    h->Kx = h->N2x + 1;
    h->Kyh = h->Ly / 2 + 1;
    h->M = d->nx + 2 * d->halo;
    // LDS of the transforms (one row or column, float64 at set-up), the
    // sampling rows, and 32-bit indexing of every array
    const size_t es = d->precision == 64 ? 8 : 4, lim = 160 * 1024;
    const bool lds_ok = 16 * (4 * (size_t)h->N2x + 1) <= lim && 16 * 3 * (size_t)h->Ly <= lim &&
                        slab_sample_lds(h->M, (int)es) + 1024 <= lim;
    const long long chans = 9LL * d->nz + 3LL * (d->nz + 2) + 12LL * d->nz;
    if (!lds_ok || chans * h->Ly * h->Kx >= (1LL << 31) || 2LL * 3 * d->nx * d->ny * d->nz >= (1LL << 31) ||
        2LL * (2 * d->nz + d->gap_cells) + 1 > 4096) {
      delete h;
      return fail(MMV_EINVAL, "films too large for the thick-film path");
    }
    if (!make_plan(h->N2x, h->px) || !make_plan(h->Ly, h->py)) {
      delete h;
      return fail(MMV_EINVAL, "FFT length has too many factors");
    }
    rc = d->precision == 64 ? init_slab<double>(h) : init_slab<float>(h);
    if (rc) {
      free_all(h);
      delete h;
      return rc;
    }
    *out = h;
    return MMV_OK;
  }
  const int hx = d->n_films == 2 ? d->halo : 0;
  const int T = d->n_films == 2 ? d->max_travel_cells : 0;
  int lx_min = d->n_films == 2 ? 2 * (d->nx + hx + T) : 2 * d->nx;
  int ly_min = d->n_films == 2 ? 2 * (d->ny + (d->cross_mode == 1 ? 3 : 1)) : 2 * d->ny;
  // a periodic axis is transformed over one period
  if (d->pbc & 1) lx_min = d->nx;
  if (d->pbc & 2) ly_min = d->ny;
  if (d->fft_lx) {
    if (d->fft_lx < lx_min || d->fft_lx % 2 || !smooth2357(d->fft_lx)) {
      delete h;
      return fail(MMV_EINVAL, "fft_lx must be even, {2,3,5,7}-smooth and >= " + std::to_string(lx_min));
    }
    h->Lx = d->fft_lx;
  } else {
    h->Lx = (d->pbc & 1) ? d->nx : next_smooth(lx_min, true);
  }
  if (d->fft_ly) {
    if (d->fft_ly < ly_min || !smooth2357(d->fft_ly)) {
      delete h;
      return fail(MMV_EINVAL, "fft_ly must be {2,3,5,7}-smooth and >= " + std::to_string(ly_min));
    }
    h->Ly = d->fft_ly;
  } else {
    h->Ly = (d->pbc & 2) ? d->ny : next_smooth(ly_min, false);
  }
  h->N2x = h->Lx / 2;
  h->Kx = h->N2x + 1;
  h->Kyh = h->Ly / 2 + 1;
  h->M = d->nx + 2 * hx;
  if (!make_plan(h->N2x, h->px) || !make_plan(h->Ly, h->py)) {
    delete h;
    return fail(MMV_EINVAL, "FFT length has too many factors");
  }
  rc = d->precision == 64 ? init_typed<double>(h) : init_typed<float>(h);
  // two films: resolve this device's static scratch of stray_force_noalloc
  // now, so that its calls (possibly under graph capture) only look it up
  unsigned char* scratch_dev = nullptr;
  if (!rc && d->n_films == 2) rc = noalloc_scratch(&scratch_dev);
  if (rc) {
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return MMV_OK;
}

int profile_begin(mmv_handle h, int kernel) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (kernel < 1 || kernel > 3) return fail(MMV_EINVAL, "kernel must be 1, 2 or 3");
  h->prof_kernel = kernel;
  h->prof_used = 0;
  return MMV_OK;
}

int profile_end(mmv_handle h, double* total_ms, long* launches) {
  int rc = check_handle(h);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->st));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, h->prof_ev[i], h->prof_ev[i + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (long)(h->prof_used / 2);
  h->prof_kernel = 0;
  h->prof_used = 0;
  return MMV_OK;
}

}  // extern "C"

namespace {
template <typename T>
int repeat_typed(mmv_mesh* h, int kernel, int reps, double* avg_ms) {
  RowParams rp = h->rp_hot;
  rp.mode = MODE_STAGE;
  rp.term_mask = MMV_TERM_ALL;
  rp.stage = 1;
  rp.dt = 0.0;
  rp.drive = h->drive;
  rp.with_force = (h->drive.mode == MMV_DRIVE_SPRING) ? 1 : 0;
  rp.full_force = 0;
  rp.ntask = h->nfilm * h->ny + ((rp.with_force && rp.pot) ? 2 : 0);
  rp.spec1_out = h->fuse_fwd ? h->spec1 : nullptr;
  rp.defer_tick = 1;
  rp.hsur = nullptr;
  T* b1 = (T*)h->mb[0];
  T* b2 = (T*)h->mb[1];
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = MMV_OK;
  auto one = [&]() -> hipError_t {
    if (kernel == 1)
      return launch_row_fwd<T>((const T*)h->m0, h->spec1, 3 * h->nfilm * h->ny, h->nx, h->N2x, h->Kx, h->px, h->twx,
                               h->twp, h->st, h->ny);
    if (kernel == 2)
      return launch_col<T>(h->spec1, h->spec2, (const T*)h->kern, h->Kx, h->Ly, h->Kyh, h->ny, 3 * h->nfilm,
                           h->ngroup, h->py, h->twy, h->tab_hot, h->st);
    return launch_row_stage<T>(rp, h->spec2, b1, (const T*)h->m0, b2, (T*)h->acc, nullptr, h->twx, h->twp, h->rigid,
                               h->partial, h->counter, h->st);
  };
  hipError_t e = one();  // warm
  if (e == hipSuccess) e = hipEventRecord(e0, h->st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = one();
  if (e == hipSuccess) e = hipEventRecord(e1, h->st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e != hipSuccess) rc = fail(MMV_EHIP, std::string("profile_repeat: ") + hipGetErrorString(e));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!rc && avg_ms) *avg_ms = (double)ms / reps;
  return rc;
}
}  // namespace

extern "C" {

int profile_repeat(mmv_handle h, int kernel, int reps, double* avg_ms) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (kernel < 1 || kernel > 3) return fail(MMV_EINVAL, "kernel must be 1, 2 or 3");
  if (reps < 1 || reps > 100000) return fail(MMV_EINVAL, "reps must be in [1, 100000]");
  if (h->cube || h->slab || h->nfilm != 2 || h->in_batch)
    return fail(MMV_ESTATE, "profile_repeat needs a two-film mesh of one-cell-thick films");
  return h->esz == 8 ? repeat_typed<double>(h, kernel, reps, avg_ms) : repeat_typed<float>(h, kernel, reps, avg_ms);
}

int init_batch(const mmv_mesh_desc* descs, int n, void* hip_stream, int flags, mmv_batch_handle* out) {
  g_err.clear();
  if (!out) return fail(MMV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || n < 1 || n > 4096) return fail(MMV_EINVAL, "need 1..4096 descriptors");
  for (int i = 0; i < n; ++i) {
    int rc = validate(&descs[i]);
    if (rc) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
    if (descs[i].n_films != 2 || descs[i].nz != 1) return fail(MMV_EINVAL, "batch instances need two films, nz == 1");
    if (descs[i].precision != descs[0].precision) return fail(MMV_EINVAL, "batch instances need one precision");
  }
  mmv_batch* b = new mmv_batch();
  b->st = (hipStream_t)hip_stream;
  b->flags = flags;
  b->esz = descs[0].precision == 64 ? 8 : 4;
  for (int i = 0; i < n; ++i) {
    mmv_handle h = nullptr;
    // reuse the kernel spectra of an earlier instance of the same geometry
    int rc = init_mesh(&descs[i], hip_stream, &h);
    if (rc) {
      batch_free(b);
      return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
    }
    h->in_batch = true;
    for (int j = 0; j < i; ++j)
      if (same_kernel(descs[i], descs[j])) {
        auto it = std::find(h->allocs.begin(), h->allocs.end(), h->kern);
        if (it != h->allocs.end()) {
          hipFree(*it);
          h->allocs.erase(it);
        }
        h->kern = b->inst[j]->kern;
        break;
      }
    b->inst.push_back(h);
  }
  int rc = hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking) == hipSuccess ? MMV_OK
                                                                                   : fail(MMV_EHIP, "stream create");
  if (!rc && (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess))
    rc = fail(MMV_EHIP, "event create");
  for (int k = 0; !rc && k < mmv_batch::NSIDE; ++k)
    if (hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming) != hipSuccess)
      rc = fail(MMV_EHIP, "side stream create");
  if (!rc) rc = b->esz == 8 ? batch_build<double>(b) : batch_build<float>(b);
  if (!rc && (flags & MMV_BATCH_AUTOTUNE)) rc = b->esz == 8 ? batch_autotune<double>(b) : batch_autotune<float>(b);
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return MMV_OK;
}

int batch_instance(mmv_batch_handle b, int i, mmv_handle* out) {
  if (!b || !out) return fail(MMV_EINVAL, "NULL argument");
  if (i < 0 || i >= (int)b->inst.size()) return fail(MMV_EINVAL, "instance out of range");
  *out = b->inst[i];
  return MMV_OK;
}

int batch_step(mmv_batch_handle b, double dt, int nsteps) {
  if (!b) return fail(MMV_EINVAL, "batch is NULL");
  if (!(dt > 0) || !isfinite(dt)) return fail(MMV_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(MMV_EINVAL, "nsteps must be >= 0");
  return b->esz == 8 ? batch_step_typed<double>(b, dt, nsteps) : batch_step_typed<float>(b, dt, nsteps);
}

int set_tune_cache(const char* path) {
  if (path && strlen(path) >= 4096) return fail(MMV_EINVAL, "tuning cache path too long");
  g_tune_cache = path ? path : "";
  return MMV_OK;
}

int batch_tuning(mmv_batch_handle b, int i, int* col_groups, int* row_threads) {
  if (!b || !col_groups) return fail(MMV_EINVAL, "NULL argument");
  if (i < 0 || i >= (int)b->inst.size()) return fail(MMV_EINVAL, "instance out of range");
  *col_groups = b->inst[i]->ngroup;
  if (row_threads) {
    int nt = 0;
    for (const BatchLaunch& c : b->l_stage)
      for (int k = c.off; k < c.off + c.n; ++k)
        if (b->stage_inst[k] == i) nt = c.nt;
    *row_threads = nt;
  }
  return MMV_OK;
}

int batch_sur_attach(mmv_batch_handle b, mmv_sur_handle s, int judge_every, double tol) {
  if (!b) return fail(MMV_EINVAL, "batch is NULL");
  if (!s) {
    b->sur = nullptr;
    return MMV_OK;
  }
  if (b->esz != 4) return fail(MMV_ESTATE, "the learned operator runs with precision 32");
  if (judge_every < 1) return fail(MMV_EINVAL, "judge_every must be >= 1");
  if (!(tol > 0) || !isfinite(tol)) return fail(MMV_EINVAL, "tol must be finite and > 0");
  int H = 0, W = 0, Bmax = 0;
  sur_shape(s, &H, &W);
  sur_max_batch(s, &Bmax);
  const int n = (int)b->inst.size();
  if (n > Bmax) return fail(MMV_EINVAL, "the operator's max_batch is smaller than the batch");
  for (mmv_mesh* h : b->inst) {
    if (h->d.cross_mode != 0) return fail(MMV_ESTATE, "the learned operator replaces the direct cross term");
    if (H != h->ny || W != h->nx) return fail(MMV_EINVAL, "every instance must have the operator's grid");
    const OutTable& t = h->tab_hot;
    if (t.n < 3 || t.ch[t.n - 3].off != h->rp_hot.off_cross[0][0])
      return fail(MMV_ESTATE, "unexpected channel table");
  }
  const size_t plane = (size_t)H * W;
  int rc;
  if (!b->sur_in && (rc = balloc(b, (void**)&b->sur_in, sizeof(float) * 4 * plane * (size_t)n))) return rc;
  if (!b->sur_exact && (rc = balloc(b, (void**)&b->sur_exact, sizeof(float) * 3 * plane * (size_t)n))) return rc;
  for (mmv_mesh* h : b->inst) {
    h->tab_sur = h->tab_hot;
    h->tab_sur.n = h->tab_hot.n - 3;
  }
  b->sur = s;
  b->sur_every = judge_every;
  b->sur_tol = tol;
  b->sur_fallback = 0;
  b->sur_err = -1.0;
  b->sur_judged = 0;
  b->sur_steps = 0;
  return MMV_OK;
}

int batch_sur_status(mmv_batch_handle b, double* last_rel_err, int* fallback, long* judged) {
  if (!b) return fail(MMV_EINVAL, "batch is NULL");
  if (last_rel_err) *last_rel_err = b->sur_err;
  if (fallback) *fallback = b->sur_fallback;
  if (judged) *judged = b->sur_judged;
  return MMV_OK;
}

int destroy_batch(mmv_batch_handle b) {
  if (!b) return MMV_OK;
  hipStreamSynchronize(b->st);
  if (b->gst) hipStreamSynchronize(b->gst);
  for (hipStream_t q : b->side)
    if (q) hipStreamSynchronize(q);
  batch_free(b);
  return MMV_OK;
}

int destroy_mesh(mmv_handle h) {
  if (!h) return MMV_OK;
  if (h->in_batch) return fail(MMV_ESTATE, "instance handles are owned by their batch");
  hipStreamSynchronize(h->st);
  for (hipEvent_t e : h->prof_ev) hipEventDestroy(e);
  free_all(h);
  delete h;
  return MMV_OK;
}

int set_m(mmv_handle h, int film, const void* m_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (film < 0 || film >= h->nfilm) return fail(MMV_EINVAL, "film out of range");
  if (!m_dev) return fail(MMV_EINVAL, "m_dev is NULL");
  const size_t bytes = (size_t)3 * h->nx * h->ny * h->nz * h->esz;
  HIPCHK(hipMemcpyAsync((char*)h->m0 + film * bytes, m_dev, bytes, hipMemcpyDeviceToDevice, h->st));
  h->eddy_first = true;
  return MMV_OK;
}

int get_m(mmv_handle h, int film, void* m_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (film < 0 || film >= h->nfilm) return fail(MMV_EINVAL, "film out of range");
  if (!m_dev) return fail(MMV_EINVAL, "m_dev is NULL");
  const size_t bytes = (size_t)3 * h->nx * h->ny * h->nz * h->esz;
  HIPCHK(hipMemcpyAsync(m_dev, (char*)h->m0 + film * bytes, bytes, hipMemcpyDeviceToDevice, h->st));
  return MMV_OK;
}

int set_offset(mmv_handle h, double x_cells) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->nfilm != 2) return fail(MMV_ESTATE, "set_offset needs two films");
  if (!isfinite(x_cells)) return fail(MMV_EINVAL, "offset must be finite");
  const double s = floor(x_cells);
  if (fabs(s) > h->rp_hot.travel)
    return fail(MMV_ERANGE, "offset outside the window sized by max_travel_cells");
  RigidState r;
  if ((rc = read_rigid(h, r))) return rc;
  r.x0 = r.xs = x_cells * h->d.dx;
  r.s_int = (int)s;
  return write_rigid(h, r);
}

int set_drive(mmv_handle h, const mmv_drive* drv) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!drv) return fail(MMV_EINVAL, "drive is NULL");
  if (drv->mode < 0 || drv->mode > 2) return fail(MMV_EINVAL, "unknown drive mode");
  if (drv->mode != MMV_DRIVE_FROZEN && h->nfilm != 2) return fail(MMV_ESTATE, "a moving drive needs two films");
  if (drv->mode == MMV_DRIVE_SPRING && !(drv->mass > 0 && isfinite(drv->mass)))
    return fail(MMV_EINVAL, "spring drive needs mass > 0");
  if (!isfinite(drv->v_d) || !isfinite(drv->k) || !isfinite(drv->gamma_v) || !isfinite(drv->x_anchor0) ||
      !isfinite(drv->x0) || !isfinite(drv->v0))
    return fail(MMV_EINVAL, "drive parameters must be finite");
  const double s = floor(drv->x0 / h->d.dx);
  if (fabs(s) > h->rp_hot.travel) return fail(MMV_ERANGE, "x0 outside the window sized by max_travel_cells");
  RigidState r;
  if ((rc = read_rigid(h, r))) return rc;
  r.x0 = r.xs = drv->x0;
  r.v0 = r.vs = (drv->mode == MMV_DRIVE_VELOCITY) ? drv->v_d : (drv->mode == MMV_DRIVE_FROZEN ? 0.0 : drv->v0);
  r.s_int = (int)s;
  h->drive.mode = drv->mode;
  h->drive.v_d = drv->v_d;
  h->drive.k = drv->k;
  h->drive.mass = drv->mode == MMV_DRIVE_SPRING ? drv->mass : 1.0;
  h->drive.gamma_v = drv->gamma_v;
  h->drive.xa0 = drv->x_anchor0;
  return write_rigid(h, r);
}

int eddy_residual(mmv_handle h, double* rel) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!rel) return fail(MMV_EINVAL, "rel is NULL");
  if (!(h->cube || h->slab) || !(h->d.sigma > 0)) return fail(MMV_ESTATE, "no eddy-current solve on this mesh");
  if (h->eddy_first) return fail(MMV_ESTATE, "no step has run the eddy solve yet");
  const size_t N = (size_t)h->nx * h->ny * h->nz;
  // the partials reuse the eddy update's reduction buffer (N/256 + 2 doubles
  // before the mean), free between steps; two thick films: both problems
  // summed, ||L phi - r|| and ||r|| over the two films together
  const int nblk = (int)std::max<size_t>(1, std::min<size_t>(512, (N / 256 + 2) / 2));
  double a = 0.0, b = 0.0;
  for (int f = 0; f < (h->slab ? 2 : 1); ++f) {
    const size_t off = (size_t)f * N * h->esz;
    if (h->esz == 8)
      HIPCHK(launch_sor_residual<double>(h->cl, (const double*)((char*)h->phi + off),
                                         (const double*)((char*)h->rr + off), h->red, nblk, h->st));
    else
      HIPCHK(launch_sor_residual<float>(h->cl, (const float*)((char*)h->phi + off), (const float*)((char*)h->rr + off),
                                        h->red, nblk, h->st));
    std::vector<double> part(2 * (size_t)nblk);
    HIPCHK(hipMemcpyAsync(part.data(), h->red, sizeof(double) * part.size(), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    for (int k = 0; k < nblk; ++k) {
      a += part[2 * (size_t)k];
      b += part[2 * (size_t)k + 1];
    }
  }
  *rel = b > 0 ? sqrt(a / b) : sqrt(a);
  return MMV_OK;
}

int spline3_prefilter(int precision, const void* field, void* coef, void* work, int nx, int ny, int nz,
                      void* hip_stream) {
  g_err.clear();
  if (precision != 32 && precision != 64) return fail(MMV_EINVAL, "precision must be 32 or 64");
  if (!field || !coef || !work) return fail(MMV_EINVAL, "NULL buffer");
  if (nx < 1 || ny < 1 || nz < 1) return fail(MMV_EINVAL, "nx, ny, nz must be >= 1");
  if ((long long)nx * ny * nz >= (1LL << 31)) return fail(MMV_EINVAL, "field too large");
  const size_t bytes = (size_t)nx * ny * nz * (precision / 8);
  auto overlap = [&](const void* a, const void* b) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bytes && y < x + bytes;
  };
  if (overlap(field, coef) || overlap(field, work) || overlap(coef, work))
    return fail(MMV_EINVAL, "field, coef and work must not overlap");
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == 64)
    HIPCHK(launch_spline3_prefilter<double>((const double*)field, (double*)coef, (double*)work, nx, ny, nz, st));
  else
    HIPCHK(launch_spline3_prefilter<float>((const float*)field, (float*)coef, (float*)work, nx, ny, nz, st));
  return MMV_OK;
}

int spline3_gather(int precision, const void* coef, int nx, int ny, int nz, const void* points, int npts, void* out,
                   void* hip_stream) {
  g_err.clear();
  if (precision != 32 && precision != 64) return fail(MMV_EINVAL, "precision must be 32 or 64");
  if (nx < 1 || ny < 1 || nz < 1) return fail(MMV_EINVAL, "nx, ny, nz must be >= 1");
  if ((long long)nx * ny * nz >= (1LL << 31)) return fail(MMV_EINVAL, "field too large");
  if (npts < 0) return fail(MMV_EINVAL, "npts must be >= 0");
  if (npts > 0 && (!coef || !points || !out)) return fail(MMV_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == 64)
    HIPCHK(launch_spline3_gather<double>((const double*)coef, nx, ny, nz, (const double*)points, npts, (double*)out,
                                         st));
  else
    HIPCHK(launch_spline3_gather<float>((const float*)coef, nx, ny, nz, (const float*)points, npts, (float*)out, st));
  return MMV_OK;
}

int set_hext_field(mmv_handle h, int film, const void* field) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->cube) return fail(MMV_ESTATE, "the applied-field array belongs to the film paths");
  if (film < 0 || film >= h->nfilm) return fail(MMV_EINVAL, "film out of range");
  if (h->slab) {
    // thick films: [3][nz][ny][nx] for film 0, [3][nz][ny][nx + 2 (travel +
    // halo)] for the slider's layers; read by slab_fields
    const int w = (film == 0 || (h->d.pbc & 1)) ? h->nx : h->nx + 2 * (h->d.max_travel_cells + h->d.halo);
    const size_t bytes = (size_t)3 * h->nz * h->ny * w * h->esz;
    h->slab_hext[film] = nullptr;
    if (field) {
      if (!h->hext_buf[film] && (rc = dalloc(h, &h->hext_buf[film], bytes))) return rc;
      HIPCHK(hipMemcpyAsync(h->hext_buf[film], field, bytes, hipMemcpyDefault, h->st));
      h->slab_hext[film] = h->hext_buf[film];
    }
    return MMV_OK;
  }
  const bool px = (h->d.pbc & 1) != 0;
  const int w = (film == 0 || px) ? h->nx : h->nx + 2 * (h->rp_hot.travel + h->d.halo);
  const size_t bytes = (size_t)3 * h->ny * w * h->esz;
  void* buf = nullptr;
  if (field) {
    if (!h->hext_buf[film] && (rc = dalloc(h, &h->hext_buf[film], bytes))) return rc;
    HIPCHK(hipMemcpyAsync(h->hext_buf[film], field, bytes, hipMemcpyDefault, h->st));
    buf = h->hext_buf[film];
  }
  for (RowParams* rp : {&h->rp_hot, &h->rp_force}) {
    if (film == 0) {
      rp->hext_b = buf;
    } else {
      rp->hext_s = buf;
      rp->hext_w = w;
      rp->hext_off = px ? 0 : h->rp_hot.travel + h->d.halo;
    }
  }
  h->hext_gen += 1;
  return MMV_OK;
}

int eval_heff(mmv_handle h, int film, int term_mask, void* h_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (film < 0 || film >= h->nfilm) return fail(MMV_EINVAL, "film out of range");
  if (!h_dev) return fail(MMV_EINVAL, "h_dev is NULL");
  if (term_mask & ~MMV_TERM_ALL) return fail(MMV_EINVAL, "unknown term bits");
  if (h->cube) return h->esz == 8 ? eval_cube<double>(h, term_mask, h_dev) : eval_cube<float>(h, term_mask, h_dev);
  if (h->slab)
    return h->esz == 8 ? eval_slab<double>(h, film, term_mask, h_dev) : eval_slab<float>(h, film, term_mask, h_dev);
  return h->esz == 8 ? eval_typed<double>(h, film, term_mask, h_dev) : eval_typed<float>(h, film, term_mask, h_dev);
}

int llg_step(mmv_handle h, double dt, int nsteps) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!(dt > 0) || !isfinite(dt)) return fail(MMV_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(MMV_EINVAL, "nsteps must be >= 0");
  if (h->cube) return h->esz == 8 ? step_cube<double>(h, dt, nsteps) : step_cube<float>(h, dt, nsteps);
  if (h->slab) return h->esz == 8 ? step_slab<double>(h, dt, nsteps) : step_slab<float>(h, dt, nsteps);
  return h->esz == 8 ? step_typed<double>(h, dt, nsteps) : step_typed<float>(h, dt, nsteps);
}

int sur_attach(mmv_handle h, mmv_sur_handle s, int judge_every, double tol) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!s) {
    h->sur = nullptr;
    return MMV_OK;
  }
  if (h->cube || h->nfilm != 2 || h->nz != 1) return fail(MMV_ESTATE, "the learned operator needs two films, nz = 1");
  if (h->in_batch) return fail(MMV_ESTATE, "batch instances cannot use the learned operator");
  if (h->esz != 4) return fail(MMV_ESTATE, "the learned operator runs with precision 32");
  if (h->d.cross_mode != 0) return fail(MMV_ESTATE, "the learned operator replaces the direct cross term (cross_mode 0)");
  int H = 0, W = 0;
  sur_shape(s, &H, &W);
  if (H != h->ny || W != h->nx) return fail(MMV_EINVAL, "operator grid differs from the film grid");
  if (judge_every < 1) return fail(MMV_EINVAL, "judge_every must be >= 1");
  if (!(tol > 0) || !isfinite(tol)) return fail(MMV_EINVAL, "tol must be finite and > 0");
  // the film-0 cross channels are the last three of the stage table
  const OutTable& t = h->tab_hot;
  if (t.n < 3 || t.ch[t.n - 3].off != h->rp_hot.off_cross[0][0]) return fail(MMV_ESTATE, "unexpected channel table");
  const size_t plane = (size_t)h->ny * h->nx;
  if (!h->sur_in && (rc = dalloc(h, (void**)&h->sur_in, sizeof(float) * 4 * plane))) return rc;
  if (!h->sur_exact && (rc = dalloc(h, (void**)&h->sur_exact, sizeof(float) * 3 * plane))) return rc;
  h->tab_sur = t;
  h->tab_sur.n = t.n - 3;
  h->sur = s;
  h->sur_every = judge_every;
  h->sur_tol = tol;
  h->sur_fallback = 0;
  h->sur_err = -1.0;
  h->sur_judged = 0;
  h->sur_steps = 0;
  return MMV_OK;
}

int sur_status(mmv_handle h, double* last_rel_err, int* fallback, long* judged) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (last_rel_err) *last_rel_err = h->sur_err;
  if (fallback) *fallback = h->sur_fallback;
  if (judged) *judged = h->sur_judged;
  return MMV_OK;
}

int stray_force(mmv_handle h, double F_out[3]) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!F_out) return fail(MMV_EINVAL, "F_out is NULL");
  if (h->nfilm != 2) return fail(MMV_ESTATE, "stray_force needs two films");
  if (h->slab) {
    rc = h->esz == 8 ? force_slab<double>(h, F_out) : force_slab<float>(h, F_out);
    if (rc) return rc;
    RigidState r;
    if ((rc = read_rigid(h, r))) return rc;
    return report_flags(h, r);
  }
  rc = h->esz == 8 ? force_typed<double>(h, h->partial, h->counter, nullptr)
                    : force_typed<float>(h, h->partial, h->counter, nullptr);
  if (rc) return rc;
  RigidState r;
  if ((rc = read_rigid(h, r))) return rc;
  for (int a = 0; a < 3; ++a) F_out[a] = r.F[a];
  return report_flags(h, r);
}

int stray_force_noalloc(mmv_handle h, double* F_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!F_dev) return fail(MMV_EINVAL, "F_dev is NULL");
  if (h->nfilm != 2 || h->slab) return fail(MMV_ESTATE, "stray_force_noalloc needs two one-cell-thick films");
  const size_t part_bytes = noalloc_partial_bytes(h->ny + 2);
  if (part_bytes + NOALLOC_COUNTER_BYTES > NOALLOC_SCRATCH_BYTES)
    return fail(MMV_EINVAL, "stray_force_noalloc: ny + 2 force rows need " + std::to_string(part_bytes) +
                                " bytes of partials, more than the static scratch of " +
                                std::to_string(NOALLOC_SCRATCH_BYTES - NOALLOC_COUNTER_BYTES) + " bytes");
  unsigned char* base = nullptr;
  if ((rc = noalloc_scratch(&base))) return rc;
  double* partial = reinterpret_cast<double*>(base);
  unsigned* counter = reinterpret_cast<unsigned*>(base + part_bytes);
  // the arrival counter must start at zero (a fill kernel, not a memset node)
  HIPCHK(launch_fill_u32(counter, (int)(NOALLOC_COUNTER_BYTES / sizeof(unsigned)), 0u, h->st));
  return h->esz == 8 ? force_typed<double>(h, partial, counter, F_dev) : force_typed<float>(h, partial, counter, F_dev);
}

int llg_run_dp(mmv_handle h, double t_end, double tol, double* h_io, int max_attempts, long* accepted,
               long* rejected) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->cube || h->slab) return fail(MMV_ESTATE, "llg_run_dp runs on the film path (nz == 1)");
  if (h->in_batch) return fail(MMV_ESTATE, "llg_run_dp does not run on batch instances");
  if (h->sur) return fail(MMV_ESTATE, "llg_run_dp does not run with a learned operator attached");
  if (!h_io) return fail(MMV_EINVAL, "h_io is NULL");
  if (!(*h_io > 0) || !isfinite(*h_io)) return fail(MMV_EINVAL, "the initial step must be finite and > 0");
  if (!(tol > 0) || !isfinite(tol)) return fail(MMV_EINVAL, "tol must be finite and > 0");
  if (!isfinite(t_end)) return fail(MMV_EINVAL, "t_end must be finite");
  if (max_attempts < 1) return fail(MMV_EINVAL, "max_attempts must be >= 1");
  RigidState r;
  if ((rc = read_rigid(h, r))) return rc;
  if (!(t_end > r.t0)) return fail(MMV_EINVAL, "t_end must lie after the current time");
  const size_t plane = (size_t)h->ny * h->nx;
  if (!h->kdp && (rc = dalloc(h, &h->kdp, (size_t)7 * h->nfilm * 3 * plane * h->esz))) return rc;
  if (!h->errpart && (rc = dalloc(h, (void**)&h->errpart, sizeof(double) * (size_t)(h->nfilm * h->ny + 2))))
    return rc;
  if (!h->dpc && (rc = dalloc(h, (void**)&h->dpc, sizeof(DpCtrl)))) return rc;
  DpCtrl c{};
  c.h = std::min(*h_io, t_end - r.t0);
  c.t_end = t_end;
  c.tol = tol;
  r.xs = r.x0;
  r.vs = r.v0;
  r.ts = r.t0;
  HIPCHK(hipMemcpyAsync(h->dpc, &c, sizeof(c), hipMemcpyHostToDevice, h->st));
  if ((rc = write_rigid(h, r))) return rc;
  // attempts in chunks between host checks of the run's end
  constexpr int CHUNK = 8;
  int done_attempts = 0;
  while (done_attempts < max_attempts) {
    const int n = std::min(CHUNK, max_attempts - done_attempts);
    rc = h->esz == 8 ? dp_attempts<double>(h, n) : dp_attempts<float>(h, n);
    if (rc) return rc;
    done_attempts += n;
    HIPCHK(hipMemcpyAsync(&c, h->dpc, sizeof(c), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (c.done) break;
  }
  *h_io = c.h;
  if (accepted) *accepted = (long)c.accepted;
  if (rejected) *rejected = (long)c.rejected;
  if ((rc = read_rigid(h, r))) return rc;
  return report_flags(h, r);
}

int div_curl(mmv_handle h, double* D, double* C) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!D || !C) return fail(MMV_EINVAL, "D and C must not be NULL");
  if (h->cube || h->slab || h->nfilm != 2) return fail(MMV_ESTATE, "div_curl needs two one-cell-thick films");
  return h->esz == 8 ? div_curl_typed<double>(h, D, C) : div_curl_typed<float>(h, D, C);
}

int get_state(mmv_handle h, double* t, double* x_s, double* v_s, long* step) {
  int rc = check_handle(h);
  if (rc) return rc;
  RigidState r;
  if ((rc = read_rigid(h, r))) return rc;
  if (t) *t = r.t0;
  if (x_s) *x_s = r.x0;
  if (v_s) *v_s = r.v0;
  if (step) *step = (long)r.step;
  return report_flags(h, r);
}

int tune_fft_lengths(const mmv_mesh_desc* d, double dt, int nsteps, int ncand, void* hip_stream, int* fft_lx,
                     int* fft_ly, double* ms_per_step) {
  if (!d || !fft_lx || !fft_ly) return fail(MMV_EINVAL, "NULL argument");
  if (ncand < 1 || ncand > 8) return fail(MMV_EINVAL, "ncand must be in [1, 8]");
  if (nsteps < 1 || nsteps > 10000) return fail(MMV_EINVAL, "nsteps must be in [1, 10000]");
  if (!(dt > 0) || !isfinite(dt)) return fail(MMV_EINVAL, "dt must be finite and > 0");
  int rc;
  // the smallest admissible lengths: those init_mesh picks by itself
  mmv_handle h0 = nullptr;
  if ((rc = init_mesh(d, hip_stream, &h0))) return rc;
  const int lx0 = h0->Lx, ly0 = h0->Ly;
  destroy_mesh(h0);
  std::vector<int> cx{lx0}, cy{ly0};
  if (!d->fft_lx && !(d->pbc & 1))
    while ((int)cx.size() < ncand) cx.push_back(next_smooth(cx.back() + 1, true));
  if (!d->fft_ly && !(d->pbc & 2))
    while ((int)cy.size() < ncand) cy.push_back(next_smooth(cy.back() + 1, false));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = -1.0;
  int bx = lx0, by = ly0;
  rc = MMV_OK;
  for (int lx : cx)
    for (int ly : cy) {
      mmv_mesh_desc c = *d;
      c.fft_lx = lx;
      c.fft_ly = ly;
      mmv_handle h = nullptr;
      if (init_mesh(&c, hip_stream, &h)) continue;  // e.g. beyond the LDS limits
      if (h->nfilm == 2) {
        // a moving slider, so that the force and re-seat work is timed
        mmv_drive v{};
        v.mode = MMV_DRIVE_VELOCITY;
        v.v_d = 1.0;
        set_drive(h, &v);
      }
      float ms = 0.f;
      if ((rc = llg_step(h, dt, 1)) == MMV_OK && hipEventRecord(e0, h->st) == hipSuccess &&
          (rc = llg_step(h, dt, nsteps)) == MMV_OK && hipEventRecord(e1, h->st) == hipSuccess &&
          hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
        const double per = ms / nsteps;
        if (best < 0 || per < best) {
          best = per;
          bx = lx;
          by = ly;
        }
      }
      destroy_mesh(h);
      if (rc) break;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (best < 0) return fail(MMV_EHIP, "no candidate transform length could be timed");
  *fft_lx = bx;
  *fft_ly = by;
  if (ms_per_step) *ms_per_step = best;
  return MMV_OK;
}

int get_fft_lengths(mmv_handle h, int* lx, int* ly, int* lz) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (lx) *lx = h->Lx;
  if (ly) *ly = h->Ly;
  if (lz) *lz = h->cube ? h->Lz : 1;
  return MMV_OK;
}

}  // extern "C"
