// Structures shared by the host runtime and the kernels (plain data).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

struct mmv_sur;

namespace mmv {

constexpr int MAX_PASSES = 16;
constexpr int MAX_OUT = 24;

// Mixed-radix plan: L = r[0] * r[1] * ... * r[np-1], radices in {2,3,4,5,7}.
struct FftPlan {
  int L;
  int np;
  int r[MAX_PASSES];
};

// One output channel of the column pass:
//   out(kx, ky) = sum_b K_{kc[b]}(kx, ky) * mhat_{src, b}(kx, ky)
// followed by an inverse y-transform and the rows [row0, row0 + nrows)
// (cyclic in Ly) written to spec2 at element offset `off` (row stride Kx).
// Kernel spectra are stored as one real number per (kx, ky <= Ly/2):
//   fl bit0: the spectrum is imaginary (value = i * stored)
//   fl bit1: the kernel is odd in y (stored(Ly-ky) = -stored(ky))
//   fl bit2: negate (the kernel of the mirrored layer -dz)
struct OutCh {
  int src;
  int kc[3];
  int fl[3];
  int row0;
  int nrows;
  long long off;
};

struct OutTable {
  int n;
  OutCh ch[MAX_OUT];
};

// Rigid-body state of the slider, float64 on the device (Eq. 15).
struct RigidState {
  double x0, v0, t0;  // at the start of the step
  double xs, vs, ts;  // at the current RK stage
  double ax, av;      // RK accumulators
  double F[3];        // last force [N]
  long long step;
  int s_int;          // floor(x / dx), fixed within a step
  int flags;          // FLAG_* (sticky until read by the host)
  double kx[7], kv[7];  // Dormand-Prince stage derivatives of x and v
};

// Step control of the adaptive Dormand-Prince run, in device memory: every
// launch of an attempt reads the step size from here, the control kernel at
// the attempt's end decides and writes the next one.
struct DpCtrl {
  double h;         // step size of the current attempt [s]
  double t_end;     // end of the run [s]
  double tol;       // error tolerance
  double err;       // error ratio of the last attempt
  long long accepted, rejected;
  int accept;       // the last attempt was accepted (read by the commit kernel)
  int done;         // t_end reached: the field and row launches return at once
};

enum { FLAG_RANGE = 1, FLAG_NUMERIC = 2 };

struct DriveP {
  int mode;
  double v_d, k, mass, gamma_v, xa0;
};

enum { MODE_EVAL = 0, MODE_STAGE = 1, MODE_FORCE = 2 };

// The slider's stage update (Eq. 15 inside RK4) from the force partials of a
// finished row launch: applied by the first block of the next y-pass launch
// (or by a one-block kernel after the last stage of a call), so the row
// kernel needs no device-wide fence.
struct TickArgs {
  const double* partial;  // [ntask][3], F_x partial sums per row task
  RigidState* rigid;
  DriveP drive;
  double force_scale, dx;
  int ntask, travel;
  int scheme;             // 0: classic RK4 stages; 1: Dormand-Prince stages
  const DpCtrl* ctrl;     // Dormand-Prince: step size and run state
};

// Parameters of the fused row kernel (inverse row transform, spline,
// local fields, LLG stage, force partials).
struct RowParams {
  int mode;       // MODE_*
  int stage;      // RK stage 0..3
  int eval_film;  // MODE_EVAL: film written to hout
  int term_mask;
  int nfilm, nx, ny;
  int N2x, Kx;
  int halo, M, travel, kfir;
  int nbr;        // inverse row transforms per batch
  int ntask;
  int with_force;  // MODE_STAGE: accumulate F_x partials
  int full_force;  // MODE_FORCE: all three components
  double dx, dy, dz;
  double pref_ex;  // 2 A / (mu0 Ms)
  double pref_an;  // 2 Ku / (mu0 Ms)
  double u[3], hext[3];
  double gam;      // gamma0 / (1 + alpha^2)
  double alpha;
  double dt;
  double force_scale;  // mu0 Ms V
  long long off_self[2][3];
  long long off_cross[2][3];
  int cross_row0[2];      // row stored first in the cross channel
  long long off_fp[3], off_fm[3];  // G at z_s+1 and z_s-1 (force)
  // scalar-potential mode: potential of the other film on the target
  // film's layers (z_target + d, d = -3..3): channel offset and first row
  int pot;
  long long off_phi[2][7];
  int phi_row0[2][7];
  DriveP drive;
  FftPlan px;
  // learned operator: when set, film 0's cross field is read from this
  // float32 [3][ny][nx] array (times sur_scale) instead of the spline rows
  const float* hsur;
  double sur_scale;
  // MODE_STAGE: blocks only write their force partials; the slider update
  // is applied later (TickArgs) instead of by the launch's last block
  int defer_tick;
  // MODE_STAGE: when set, each cell-row task also x-transforms the three
  // components of its new magnetisation row into this spectrum array (the
  // x-pass input of the next stage), [film][comp][y][Kx]
  void* spec1_out;
  // MODE_FORCE: when set, the force [N] goes here instead of rigid->F
  double* fout;
  // the row transforms run in place (compiled lengths only): sizes the LDS
  int inplace;
  // MODE_STAGE scheme: 0 classic RK4 (acc, mnext); 1 Dormand-Prince stage
  // `stage` (0..6): writes its derivative to kdp[stage] ([7][film][3][y][x]),
  // the next stage's state to mnext (stages 0..5) or, at stage 6, the
  // block's largest |error| of m to errpart[task]; step size from ctrl
  int scheme;
  void* kdp;
  double* errpart;
  const DpCtrl* ctrl;
  // periodic in-plane axes (bit 0 = x, 1 = y): exchange wraps, and along y
  // the force's rows -1 and ny are the rows ny-1 and 0
  int pbc;
  // sampling of the other film's field along x: 0 prefiltered cubic
  // B-spline, 1 linear interpolation of the field vectors (a comparison
  // mode, Sec. IV.A)
  int interp;
  // MODE_FORCE: when set, the base field on the slider's stencil points is
  // also written here: layer z_s at rows -1..ny, i = -1..nx
  // [3][ny+2][nx+2], then layers z_s+1 and z_s-1 on the cells [3][ny][nx]
  // each (mesh precision)
  void* fieldout;
  // non-uniform applied field (mesh precision), added to the Zeeman term:
  // film 0 [3][ny][nx] on its cells; the slider's layer [3][ny][hext_w] on
  // the frame lattice, column c at lattice x c - hext_off (periodic x: the
  // period, indices modulo nx).  Null: the uniform hext only.
  const void* hext_b;
  const void* hext_s;
  int hext_w, hext_off;
};

// Per-instance descriptors of the batched launches (device memory).
struct RowFwdDesc {
  const void* src;
  void* dst;
  int nin, N2x, Kx, ny;
  FftPlan P;
  const void* tw;
  const void* twp;
};

struct ColDesc {
  const void* spec1;
  void* spec2;
  const void* kern;
  int Kx, Ly, Kyh, ny, nin_ch, ngroup, nbuf;
  FftPlan P;
  const void* twy;
  OutTable tab;
  TickArgs tick;
};

struct RowStageDesc {
  RowParams p;
  const void* spec2;
  const void* mst;
  const void* m0;
  void* mnext;
  void* acc;
  const void* tw;
  const void* twp;
  RigidState* rigid;
  double* partial;
  unsigned* counter;
};

// Records msg as the thread's last error (returned by mmv_last_error) and
// returns code.
int report_error(int code, const std::string& msg);

// Learned stray-field operator, as used inside the LLG step (mmv_fno.hip).
// sur_infer runs the network on B samples on stream st; *out points at the
// handle's own output buffer [B][3][H][W] (valid until its next call).
int sur_infer(mmv_sur* s, const float* a, int B, hipStream_t st, const float** out);
void sur_shape(const mmv_sur* s, int* H, int* W);
void sur_max_batch(const mmv_sur* s, int* Bmax);
// the operator's output buffer [max_batch][3][H][W] (written by sur_infer)
const float* sur_output(const mmv_sur* s);
// a[4][ny][nx] = (m_x, m_y, m_z of the slider, x_s / dx of the current stage)
hipError_t launch_sur_input(const float* m_slider, const RigidState* rigid, double inv_dx, int ny, int nx, float* a,
                            hipStream_t st);
// relative L2 distance between scale * pred and exact (both n floats);
// exact is overwritten; blocks on st
int sur_rel_err(mmv_sur* s, const float* pred, float* exact, long long n, double scale, hipStream_t st, double* rel);

}  // namespace mmv
