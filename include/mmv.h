/*
 * mmv.h -- C ABI of the moving-magnet micromagnetic hot path on MI355X.
 *
 * Two thin magnetic films on finite-difference lattices: film 0 (the base)
 * is fixed, film 1 (the slider) sits gap_cells empty layers above it and
 * moves rigidly along x (Rissanen & Laurson, Sec. II and III).  Per RK4
 * stage the library evaluates the effective field (exchange, uniaxial
 * anisotropy, uniform Zeeman, the demagnetising convolution of Eq. (6) and
 * the stray field of the other film sampled at the sub-cell offset by
 * prefiltered cubic B-splines, Sec. II.A and III.A), the LLG torque of
 * Eq. (1), the force of Eq. (3) and the slider equation of motion Eq. (15).
 *
 * Conventions shared by every call
 *   - Return value: MMV_OK (0) or a negative MMV_E* code; nothing throws.
 *     mmv_last_error() returns a thread-local text for the last failure.
 *   - Arguments are validated on the host before any HIP call; a call that
 *     fails validation has no effect.
 *   - Device pointers are owned by the caller (e.g. torch tensors) and must
 *     stay valid until the call's work on the handle's stream completes.
 *     The library owns its internal buffers and frees them in destroy_mesh.
 *   - Magnetisation and field buffers are structure-of-arrays
 *     [3][nz][ny][nx] (component, z, y, x; x fastest) of the mesh's
 *     precision: float for precision 32, double for precision 64.
 *   - Work is enqueued on the stream given to init_mesh and is
 *     asynchronous, except stray_force, get_state, set_offset and
 *     set_drive, which synchronise that stream.  A handle is not
 *     thread-safe.
 *   - Units are SI, except offsets given in cells where stated.
 */
#ifndef MMV_H
#define MMV_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MMV_OK = 0,
  MMV_EINVAL = -1,   /* bad argument or descriptor                         */
  MMV_ENOMEM = -2,   /* device allocation failed                           */
  MMV_EHIP = -3,     /* a HIP runtime call failed                          */
  MMV_ERANGE = -4,   /* slider offset outside the window the FFT was sized for */
  MMV_ENUMERIC = -5, /* non-finite magnetisation detected                  */
  MMV_ESTATE = -6    /* call not valid in the handle's current state       */
};

/* Field terms for eval_heff (bit mask). */
enum {
  MMV_TERM_EXCHANGE = 1,
  MMV_TERM_ANISOTROPY = 2,
  MMV_TERM_ZEEMAN = 4,
  MMV_TERM_DEMAG_SELF = 8,   /* the film's own demagnetising field, Eq. (6) */
  MMV_TERM_DEMAG_CROSS = 16, /* the other film's interpolated stray field   */
  MMV_TERM_EDDY = 32,        /* eddy-current field (Sec. III.B)             */
  MMV_TERM_ALL = 63
};

/* Slider drive (Sec. III; Eqs. 14-15). */
enum { MMV_DRIVE_FROZEN = 0, MMV_DRIVE_VELOCITY = 1, MMV_DRIVE_SPRING = 2 };

typedef struct mmv_mesh* mmv_handle;

typedef struct {
  int n_films;          /* 1: one magnet; 2: base (film 0) + slider (film 1) */
  int nx, ny, nz;       /* cells per film (two films of nz > 1: the thick-film
                           path below)                                       */
  double dx, dy, dz;    /* cell edges [m]                                     */
  int gap_cells;        /* empty layers between the films (>= 0)              */
  int max_travel_cells; /* |floor(x_s/dx)| allowed; sizes the FFT window      */
  double Ms;            /* saturation magnetisation [A/m]                     */
  double Aex;           /* exchange stiffness [J/m]                           */
  double alpha;         /* Gilbert damping                                    */
  double Ku;            /* first-order uniaxial anisotropy [J/m^3]            */
  double u[3];          /* anisotropy axis (normalised by the library)        */
  double Hext[3];       /* uniform applied field [A/m]                        */
  double sigma;         /* conductivity [S/m]; 0 = no eddy currents.  Eddy
                           currents need magnets more than one cell thick in
                           every direction (Sec. IV.D): one magnet with
                           nz > 1, or two films with nz > 1               */
  int precision;        /* 32 or 64                                           */
  int cross_mode;       /* 0: direct field spline; 1: scalar potential (needs
                           gap_cells >= 3: Sec. IV.D asks for films more than
                           two cells apart; MMV_EINVAL otherwise); 2: direct
                           field, linear interpolation of the field vectors
                           (the comparison interpolant of Sec. IV.A)         */
  int halo;             /* spline window extension along x in cells (>= 2)    */
  double rc_cells;      /* Newell / point-dipole switch radius in cells (> 0) */
  int sor_sweeps;       /* eddy SOR sweeps per step (0: library default 40);
                           -1: the Neumann problem solved exactly in the
                           cosine basis that diagonalises it (DCT-II along
                           x, y, z, division by the eigenvalues, inverse;
                           nx, ny, nz {2,3,5,7}-smooth, MMV_EINVAL
                           otherwise; a periodic axis takes the Hartley
                           transform, cas(2 pi k i / n), instead)         */
  double sor_omega;     /* eddy SOR factor (0: 2/(1+sin(pi/n_max)))           */
  int fft_lx, fft_ly, fft_lz; /* FFT lengths; 0 = smallest admissible       */
  int pbc;              /* periodic in-plane axes (Sec. III.A end, Sec. IV.B):
                           bit 0 = x, bit 1 = y; 0 = open.  Film meshes
                           (nz == 1) without eddy currents, or two
                           thicker films (with eddy currents: ny even for
                           a periodic y), in every cross mode (the scalar
                           potential's window rows and columns past the
                           period are those of the other side).  Along a
                           periodic axis the transform length is the period (nx even and {2,3,5,7}-smooth,
                           ny {2,3,5,7}-smooth), the kernel of a displacement
                           is summed over its minimum image and pbc_images
                           repetitions of the period on each side, the
                           spline window's halo is the copy from the other
                           side, exchange wraps, and along x the slider may
                           travel without bound (max_travel_cells unused)  */
  int pbc_images;       /* repetitions summed on each side (0..1024)          */
} mmv_mesh_desc;

typedef struct {
  int mode;          /* MMV_DRIVE_*                                           */
  double v_d;        /* anchor (spring) or slider (velocity) speed [m/s]      */
  double k;          /* spring constant [N/m]                                 */
  double mass;       /* slider mass [kg] (> 0 for the spring drive)           */
  double gamma_v;    /* viscous damping coefficient [1/s], Eq. (14)           */
  double x_anchor0;  /* spring anchor position at t = 0 [m]                   */
  double x0, v0;     /* slider position [m] and velocity [m/s] set now        */
} mmv_drive;

/* Create a mesh.  Validates d, chooses FFT lengths (x: even and
 * {2,3,5,7}-smooth with Lx >= 2 (nx + halo + max_travel_cells); y:
 * {2,3,5,7}-smooth with Ly >= 2 (ny + 1) for the direct mode, 2 (ny + 3)
 * for the potential mode), allocates device buffers and builds the kernel
 * spectra on the GPU in float64 (Sec. III.A: the tensor is computed once,
 * Fourier transformed and kept on the GPU).  hip_stream is a hipStream_t
 * (NULL = default stream).  Magnetisation starts at +z, slider at x = 0,
 * drive frozen, t = 0.  On success *out receives the handle.
 * Size limits of the film path (a film row and a spectrum column each
 * live in one CU's 160 KB of LDS): with the default halo and travel, nx up
 * to 1728 (float32) / 844 (float64) and ny up to 809 / 404 (potential mode,
 * gap 3: nx 944 / 459, ny 781 / 402); beyond them,
 * or for a kernel-spectrum table of 2^31 elements or more, MMV_EINVAL
 * before any device call.  The three-dimensional path (one film, nz > 1)
 * holds one x row, y column or z column of a transform pass per
 * block in LDS: nx up to 2520, ny up to 1701 and nz up to 1458 (float32) /
 * 729 (float64), and fewer than 2^31 cells; beyond them, MMV_EINVAL.
 *
 * Two films more than one cell thick (n_films 2, nz > 1; Sec. II.A end,
 * III.B, IV.C-D): the thick-film path.  Every cross mode (the scalar
 * potential's windows reach three rows and layers past the films, Ly >=
 * 2 (ny + 3)).  Periodic in-plane boundaries (pbc) in every cross mode:
 * the layer kernels (and the potential's S) summed over the images, the transform
 * along a periodic axis over the period, windows unshifted along it (the
 * sampler wraps their columns and rows modulo the period) and exchange
 * wrapping; with eddy currents the S sums take the image-summed kernel and
 * each film's Neumann problem wraps along the periods (no surface there).
 * Each field
 * is a sum over the source film's layers of in-plane convolutions with the
 * kernel of each layer offset (FFT lengths as for one-layer films, fft_lz
 * unused): the films' own fields, the base's field on the slider's window
 * (layers z_s - 1 .. z_s + nz, rows -1..ny: Eq. 3's stencil) and the
 * slider's field on the base's window, sampled along x as in the film
 * path.  The force of Eq. 3 sums every slider layer.  With sigma > 0, eddy
 * currents run in both films, once per step from the state at its start
 * (held through the RK stages): B = mu0 (H_d + H_ext + Ms m) per film with
 * H_d its own plus the other film's sampled field, dB/dt its backward
 * difference over the last step (formed in float64 from the fields of the
 * mesh precision; zero on the first step after set_m), E_sol = sum over
 * both films of S x dB/dt (the other film's part on its window, sampled),
 * one Neumann problem per film (SOR as for one magnet), J = sigma (E_sol +
 * E_irrot) and H_eddy = -sum over both films of S x J the same way.
 * A non-uniform H_ext per layer with set_hext_field.  Limits: the sampling
 * rows (6 (nx + 2 halo) reals) and a transform row or column in LDS, and
 * fewer than 2^31 elements in the product spectra.                      */
int init_mesh(const mmv_mesh_desc* d, void* hip_stream, mmv_handle* out);

/* Copy a film's magnetisation from / to a caller device buffer
 * (SoA [3][nz][ny][nx], mesh precision).  set_m does not renormalise.   */
int set_m(mmv_handle h, int film, const void* m_dev);
int get_m(mmv_handle h, int film, void* m_dev);

/* Place the slider at x_s = x_cells * dx (Fig. 3: x_s = (s_int + x_p) dx
 * with s_int = floor(x_cells)).  MMV_ERANGE if |s_int| exceeds
 * max_travel_cells.  Reads the device-side slider state back and writes it
 * again: synchronises the stream.                                       */
int set_offset(mmv_handle h, double x_cells);

/* Set the drive and the slider's position and velocity (x0, v0; for the
 * velocity drive v0 is replaced by v_d).  Synchronises the stream (as
 * set_offset).  On a batch instance the batch's launch descriptors are
 * rebuilt before its next batch_step.                                   */
int set_drive(mmv_handle h, const mmv_drive* drv);

/* Non-uniform applied field (Sec. II.A), added to the Zeeman term (with the
 * uniform Hext of the descriptor).  The field does not move with either
 * film; it is given on the fixed lattice.
 *   film 0: field[3][ny][nx] (SoA, mesh precision) on the base film's cells.
 *   film 1: field[3][ny][nx + 2 W], W = max_travel_cells + halo, on the
 *           slider's layer.  Column c is lattice x index c - W; with
 *           periodic x (pbc bit 0) it is [3][ny][nx], the period.
 * Films thicker than one cell take one such plane per layer:
 * [3][nz][ny][nx] for film 0 and [3][nz][ny][nx + 2 W] for the slider's
 * layers; the field also enters B of the eddy-current update.
 * The slider's cells take the field at their moved positions, interpolated
 * along x like the cross field: same window and mirror ends, the cubic
 * B-spline (cross_mode 0, 1) or linear interpolation (cross_mode 2).  The
 * force of Eq. 3 does not include this field.
 * The array (host or device memory) is copied, stream-ordered, on the mesh's
 * stream into a buffer the library owns; NULL removes the field.
 * MMV_EINVAL if film is out of range; MMV_ESTATE on the single-magnet 3-D
 * path.  On a batch instance, the batch's descriptors are rebuilt before
 * its next batch_step.                                                  */
int set_hext_field(mmv_handle h, int film, const void* field);

/* Residual of the last eddy-current solve (Eq. 12, Sec. III.B): the
 * relative L2 norm ||L phi - r|| / ||r|| of the finite-volume Neumann
 * problem after the step's SOR sweeps (L: sum over interior faces of
 * (phi_j - phi_i) / d^2; r: the surface flux of E_sol, zero mean).  The
 * sweeps per step are fixed (sor_sweeps), so this is the check of how far
 * they left the potential from the solution; two thick films: both
 * problems pooled, sqrt(sum_f ||L phi_f - r_f||^2 / sum_f ||r_f||^2).
 * Synchronises the stream.
 * MMV_ESTATE if the mesh has no eddy currents or no step has run yet.    */
int eddy_residual(mmv_handle h, double* rel);

/* Tricubic B-spline of a scalar field on a 3-D lattice (Sec. III.A's
 * spline, here along all three axes; the 4 x 4 x 4 nearest-neighbour
 * evaluation of Sec. IV.D), for interpolation at arbitrary displacements.
 * field, coef, work: device [nz][ny][nx] arrays of the precision (32 or
 * 64).  The lattice point (i, j, k) sits at (x, y, z) = (i, j, k) in cells.
 *
 * spline3_prefilter: coef = the coefficients whose spline passes through
 * field.  Prefilter along x, then y, then z: the exact inverse of the
 * B-spline's sampling filter with whole-sample mirror ends, truncated below
 * the precision's rounding.  work is scratch.  The three arrays must not
 * overlap.
 *
 * spline3_gather: out[p] = sum over the 4 x 4 x 4 nearest coefficients of
 * beta3(x - i) beta3(y - j) beta3(z - k) c[k][j][i], for points[p] =
 * (x, y, z), [npts][3], device, in the precision.  Points outside the box
 * use the mirror extension.
 *
 * Both are asynchronous on hip_stream.  MMV_EINVAL for a bad precision, a
 * size < 1 or of 2^31 elements or more, NULL buffers, npts < 0, or
 * overlapping prefilter buffers.                                         */
int spline3_prefilter(int precision, const void* field, void* coef, void* work, int nx, int ny, int nz,
                      void* hip_stream);
int spline3_gather(int precision, const void* coef, int nx, int ny, int nz, const void* points, int npts, void* out,
                   void* hip_stream);

/* Effective field of one film at the current state: the sum of the terms
 * in term_mask (MMV_TERM_*), in A/m, written to h_dev (SoA, mesh
 * precision).  The cross term is the other film's stray field sampled at
 * the current slider offset (Sec. II.A).                               */
int eval_heff(mmv_handle h, int film, int term_mask, void* h_dev);

/* Advance nsteps classic RK4 steps of size dt [s] for (m_base, m_slider,
 * x_s, v_s) (Eq. 1 with Eq. 15); every stage evaluates the full field at
 * its own magnetisation, offset and time; m is renormalised after each
 * step and s_int re-seated to floor(x_s / dx) (Sec. III).  Asynchronous.
 * A slider leaving the sized window sets a flag reported as MMV_ERANGE by
 * the next get_state / stray_force.                                      */
int llg_step(mmv_handle h, double dt, int nsteps);

/* Adaptive Dormand-Prince RK5(4) run from the current state to t_end [s]
 * (the paper's RK45 solver with the slider's equation of motion, Sec. III).
 * Every attempt evaluates seven stages, each the full field at its own
 * magnetisation, offset and time; it advances with the fifth-order state
 * and estimates the error from the embedded fourth-order one.  Error ratio:
 * the largest of max over cells |e_m|, |e_x| / dx and |e_v| h / dx, over
 * tol; accepted when <= 1 (then m is renormalised and s_int re-seated).
 * Next step h * min(5, max(0.2, 0.9 ratio^(-1/5))) (at most h after a
 * rejection), clipped so the run ends exactly at t_end (reached when
 * t_end - t <= 1e-9 t_end).  The step control runs on the device; the host
 * checks the run's end every 8 attempts (synchronising the stream) and
 * stops at t_end or after max_attempts attempts (the state then lies
 * before t_end: get_state tells).  *h_io: initial step in, next proposed
 * step out; *accepted / *rejected (may be NULL): attempts of this call.
 * Film meshes only (MMV_ESTATE for the three-dimensional path, films
 * thicker than one cell, batch instances and meshes with a learned operator attached); MMV_EINVAL for
 * t_end not after the current time, tol or *h_io not finite and > 0.
 * Reports pending MMV_ERANGE / MMV_ENUMERIC (a non-finite error stops the
 * run with MMV_ENUMERIC).                                                */
int llg_run_dp(mmv_handle h, double t_end, double tol, double* h_io, int max_attempts, long* accepted,
               long* rejected);

/* Force of Eq. (3) exerted by the base on the slider [N] at the current
 * state, all three components, accumulated in float64 in a fixed order.
 * Synchronises the stream.  MMV_ESTATE for a single-film mesh.          */
int stray_force(mmv_handle h, double F_out[3]);

/* Divergence and curl of the base film's stray field as the slider samples
 * it at the current offset (Sec. IV.A, Eq. 13): per slider cell the
 * two-point central differences of the interpolated field at the six
 * neighbour points of the shifted lattice (the points of Eq. 3), and
 * D = mean over the nx*ny slider cells of |div H|, C = mean of |curl H|
 * [A/m^2], summed in float64 in a fixed order.  Works for every cross_mode
 * (0 spline, 1 scalar potential, 2 linear interpolation).  Synchronises
 * the stream.  MMV_ESTATE for a single-film mesh and for films thicker
 * than one cell.                                                         */
int div_curl(mmv_handle h, double* D, double* C);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the force
 * of stray_force with no allocation and no synchronisation.  Same kernels
 * and fixed summation order as stray_force; the three float64 components
 * [N] are written to the caller's device buffer F_dev (3 doubles),
 * asynchronously on the handle's stream.  The float64 partial sums of the
 * row blocks and the arrival counter live in a static device array of
 * 64 KiB per GPU, held until the process ends (the counter is cleared by a
 * fill kernel at each call): the ny + 2 force rows need 24 bytes each, at
 * most 65280 bytes (ny <= 2718, which covers every two-film mesh init_mesh
 * accepts), MMV_EINVAL otherwise.  All calls on one GPU share that array:
 * calls that overlap on one GPU (other streams, handles or threads) race
 * and must be ordered by the caller.  Pending MMV_ERANGE / MMV_ENUMERIC
 * flags are left for get_state.  MMV_ESTATE for a single-film mesh and
 * for films thicker than one cell.                                      */
int stray_force_noalloc(mmv_handle h, double* F_dev);

/* Time [s], slider position [m] and velocity [m/s] and step count.
 * Synchronises the stream; reports a pending MMV_ERANGE / MMV_ENUMERIC. */
int get_state(mmv_handle h, double* t, double* x_s, double* v_s, long* step);

/* Diagnostics: time every launch of one kernel with HIP events recorded on
 * the handle's stream around that launch.  kernel: 1 = x transform,
 * 2 = y pass with kernel multiplication, 3 = row kernel (inverse x
 * transform, spline, local terms, LLG stage, force).  profile_end
 * synchronises the stream, returns the summed duration [ms] and the number
 * of timed launches since profile_begin, and stops timing.               */
int profile_begin(mmv_handle h, int kernel);
int profile_end(mmv_handle h, double* total_ms, long* launches);
/* Diagnostics: launch `kernel` (as above) reps times back to back with the
 * inputs of an RK stage, bracketed by one pair of HIP events on the handle's
 * stream, and return the mean time per launch (blocks).  The launches
 * overwrite the stage buffers, spectra and force partials: the mesh state is
 * undefined afterwards (set m, offset and drive again before stepping).
 * Two-film meshes of one-cell-thick films that are not part of a batch
 * (MMV_ESTATE otherwise).                                                */
int profile_repeat(mmv_handle h, int kernel, int reps, double* avg_ms);

/* Chosen FFT lengths (diagnostics). */
int get_fft_lengths(mmv_handle h, int* lx, int* ly, int* lz);

/* Transform-length autotuner (Sec. III.A: the convolutions run by FFT over
 * padded lengths, any admissible length giving the same result up to
 * rounding).  For each open in-plane axis whose length d leaves at 0, takes
 * the ncand smallest admissible {2,3,5,7}-smooth lengths (Lx even, from the
 * one init_mesh picks by itself), builds a mesh from d with each pair on
 * hip_stream (its own initial state m = +z; two films get a 1 m/s velocity
 * drive), times nsteps llg_step steps of size dt after one untimed step
 * with HIP events, and returns the fastest pair in *fft_lx, *fft_ly and,
 * if not NULL, its time per step [ms] in *ms_per_step.  A periodic axis or
 * a length d fixes keeps that length; pairs init_mesh refuses are skipped.
 * Set the result into d's fft_lx / fft_ly for the mesh that is kept.
 * MMV_EINVAL for NULL d or outputs, ncand outside [1, 8], nsteps outside
 * [1, 10000] or dt not finite and > 0; init_mesh's error for d itself;
 * MMV_EHIP if no pair could be timed.  Synchronous; allocates and frees
 * the candidate meshes.                                                   */
int tune_fft_lengths(const mmv_mesh_desc* d, double dt, int nsteps, int ncand, void* hip_stream, int* fft_lx,
                     int* fft_ly, double* ms_per_step);

/* ------------------------------------------------------------------------
 * Batches: many independent two-film meshes of uneven sizes advanced
 * together, one launch per pass covering every instance (per-instance
 * descriptors live in device memory), optionally replayed from a captured
 * HIP graph.  Instances of equal geometry share their kernel spectra.
 * flags: MMV_BATCH_AUTOTUNE times the y-pass grouping per mesh size at
 * set-up and keeps the fastest; MMV_BATCH_GRAPH captures 8 steps into a
 * graph (on an internal stream ordered after the caller's) and replays it.
 * All instances must have two films, the same precision and nz == 1.     */
enum { MMV_BATCH_AUTOTUNE = 1, MMV_BATCH_GRAPH = 2 };
typedef struct mmv_batch* mmv_batch_handle;

int init_batch(const mmv_mesh_desc* descs, int n, void* hip_stream, int flags, mmv_batch_handle* out);
/* Per-instance handle (owned by the batch; do not destroy): set_m, get_m,
 * set_drive, set_offset, eval_heff, stray_force and get_state act on that
 * instance.                                                              */
int batch_instance(mmv_batch_handle b, int i, mmv_handle* out);
/* Advance every instance nsteps RK4 steps of size dt (llg_step semantics). */
int batch_step(mmv_batch_handle b, double dt, int nsteps);
/* Chosen launch shape of instance i (diagnostics): the y-pass grouping
 * and, if row_threads is not NULL, the row kernel's threads per block (128,
 * 256 or 512).  MMV_EINVAL for a NULL batch or col_groups or i out of
 * range.                                                                  */
int batch_tuning(mmv_batch_handle b, int i, int* col_groups, int* row_threads);
/* Tuning cache for MMV_BATCH_AUTOTUNE (process-wide; NULL or "" = none).
 * A text file, one line per tuned mesh size: a key naming the device (arch,
 * CU count), the precision, the batch's size mix and the size, a tab, and
 * the chosen y-pass grouping; and one line per tuned row length (key ending
 * in " row") with the row kernel's threads per block / 64.  init_batch reads it, times only the sizes not
 * in it and rewrites the file (temporary file + rename) with the new
 * results; malformed lines are ignored, a failed write is reported on
 * stderr and does not fail init_batch.  The path is copied.  MMV_EINVAL
 * for a path of 4096 bytes or more.                                      */
int set_tune_cache(const char* path);
int destroy_batch(mmv_batch_handle b);

/* Release every device buffer of the handle.  NULL is accepted.         */
int destroy_mesh(mmv_handle h);

/* ------------------------------------------------------------------------
 * Learned stray-field operator (a Fourier neural operator standing in for
 * the cross term of Eqs. (6)-(8) sampled at the slider offset, Sec. III.A).
 *
 * Input  a [B][4][H][W] float32 (device): m_x, m_y, m_z of the slider film
 *        and, as the fourth channel, its offset in cells (x_p) at every
 *        pixel.  Output [B][3][H][W] float32 (device): the stray field on the
 *        base film, in the units the training targets carry.
 * Network: pointwise lift 4 -> width; `layers` blocks
 *        v <- GELU( IDFT2[ R(k) DFT2[v](k) ] + Wp v + bp ) keeping the modes
 *        kx in [0, modes_x), ky in [0, modes_y/2) U [H - modes_y/2, H) with a
 *        complex width x width matrix R(k) per mode; pointwise projection
 *        width -> 3.  Products run on the BF16 matrix cores with float32
 *        accumulation; parameters, gradients and Adam state are float32.
 * Parameter vector (float32, sur_param_count entries): wl [width][4],
 *        bl [width], then per layer R [modes_x*modes_y][2][width][width]
 *        (real, imaginary planes; mode index ky_slot*modes_x + kx with
 *        ky_slot < modes_y/2 for ky = ky_slot and H - modes_y + ky_slot
 *        otherwise), Wp [width][width], bp [width]; then wq [3][width],
 *        bq [3].  sur_param_offsets returns those start offsets in order.
 * The DFT convention is numpy's: forward exp(-i 2 pi k x / W) unnormalised,
 * inverse normalised by 1/(H W), with the real part kept after doubling the
 * kx > 0 modes (Hermitian completion of the half spectrum).
 * All pointers are device pointers; calls are ordered on the handle's stream.
 * Errors: MMV_EINVAL for bad sizes or NULL pointers, MMV_ENOMEM, MMV_EHIP. */
typedef struct {
  int H, W;        /* grid of the base film (rows, columns)              */
  int width;       /* channels C (1..256)                                 */
  int modes_x;     /* kept kx modes (1..W/2)                              */
  int modes_y;     /* kept ky modes, even, split over both ends (<= H)   */
  int layers;      /* spectral blocks (1..16)                             */
  int max_batch;   /* largest B any call may pass (1..256)                */
  int reserved[9];
} mmv_sur_desc;
typedef struct mmv_sur* mmv_sur_handle;

/* Allocate parameters (zeroed), Adam state and activations for max_batch. */
int sur_create(const mmv_sur_desc* d, void* hip_stream, mmv_sur_handle* out);
long long sur_param_count(mmv_sur_handle h);
/* Start offsets of wl, bl, (R, Wp, bp) per layer, wq, bq: n >= 4 + 3 layers. */
int sur_param_offsets(mmv_sur_handle h, long long* offs, int n);
/* Copy the parameter vector in (resets Adam's moments and step) or out.  */
int sur_set_params(mmv_sur_handle h, const float* w_dev);
int sur_get_params(mmv_sur_handle h, float* w_dev);
/* out = network(a) for B samples.                                         */
int sur_forward(mmv_sur_handle h, const float* a_dev, int B, float* out_dev);
/* Gradient of the mean over all B*3*H*W outputs of (out - target)^2 with
 * respect to the parameter vector (written to grad_dev if not NULL);
 * *loss receives that mean (blocks until it is known).                    */
int sur_gradient(mmv_sur_handle h, const float* a_dev, const float* target_dev, int B, float* grad_dev,
                 double* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * loss; *loss and *rel_err (||out - target|| / ||target||) are of the
 * parameters before the step.                                             */
int sur_train_step(mmv_sur_handle h, const float* a_dev, const float* target_dev, int B, float lr, double* loss,
                   double* rel_err);
/* The matrix-core product on its own: C = alpha A B + beta C with
 * A(m,k) = A[m*am + k*ak], B(k,n) = B[k*bk + n*bn], C(m,n) = C[m*cm + n*cn]
 * (float32 in memory, BF16 operands, float32 accumulation).              */
int sur_gemm_bf16(const float* A, long long am, long long ak, const float* B, long long bk, long long bn, float* C,
                  long long cm, long long cn, int M, int N, int K, float alpha, float beta, void* hip_stream);
int sur_destroy(mmv_sur_handle h);

/* Use the operator for film 0's cross field inside llg_step: at every RK
 * stage the network reads the stage's slider magnetisation and offset
 * x_s / dx and its output, times Ms, replaces the interpolated stray field
 * of film 1 on film 0 (the film-0 cross channels are then not computed).
 * Every judge_every steps, before the step, the exact cross field is
 * computed as well and compared (relative L2 over the film); above tol the
 * mesh falls back to the exact path for good (until attached again).  The
 * network must have been created with H = ny, W = nx and be trained on
 * targets in units of Ms.  Needs two films, nz = 1, precision 32 and
 * cross_mode 0, on a mesh that is not part of a batch (MMV_ESTATE
 * otherwise).  The operator is not owned; s = NULL detaches.  Each judge
 * blocks the host until its error is known.                            */
int sur_attach(mmv_handle h, mmv_sur_handle s, int judge_every, double tol);
/* Error at the last judge (-1 before the first), whether the mesh has
 * fallen back to the exact path, and how many judges ran.               */
int sur_status(mmv_handle h, double* last_rel_err, int* fallback, long* judged);

/* The operator inside batch_step for every instance of a batch (the
 * surrogate + batched form): at every RK stage one batched inference over
 * all instances (each instance's stage slider magnetisation and offset)
 * replaces film 0's cross field, as sur_attach does for one mesh.  Every
 * judge_every steps, before the step, the exact cross fields of all
 * instances are computed and compared with the network's (relative L2 over
 * the whole batch); above tol the whole batch falls back to the exact path
 * until attached again.  Needs precision 32, cross_mode 0, every instance
 * on the operator's grid (H = ny, W = nx) and at most max_batch instances.
 * With the operator the batch's steps are launched without graph replay.
 * s = NULL detaches.  Each judge blocks the host until its error is known. */
int batch_sur_attach(mmv_batch_handle b, mmv_sur_handle s, int judge_every, double tol);
int batch_sur_status(mmv_batch_handle b, double* last_rel_err, int* fallback, long* judged);

/* Thread-local message for the most recent failing call ("" if none).   */
const char* mmv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MMV_H */
