"""Python binding of libmmv (the moving-magnet micromagnetic hot path).

Argument marshalling only: every call forwards to the C ABI declared in
include/mmv.h, and every step of the computation runs in the HIP kernels of
libmmv.so.  Device buffers are torch tensors on the GPU; the library only
sees their pointers and the current HIP stream.  If libmmv.so is missing the
first call raises -- there is no fallback implementation.
"""
import ctypes
import os

__all__ = ["MMVError", "lib_path", "load", "MeshDesc", "DriveDesc", "init_mesh",
           "set_m", "get_m", "set_offset", "set_drive", "set_hext_field", "eval_heff", "llg_step", "llg_run_dp",
           "spline3_prefilter", "spline3_gather", "eddy_residual",
           "stray_force", "stray_force_noalloc", "div_curl", "get_state", "get_fft_lengths", "tune_fft_lengths", "destroy_mesh",
           "profile_begin", "profile_end", "profile_repeat", "init_batch", "batch_instance", "batch_step",
           "batch_tuning", "set_tune_cache", "destroy_batch", "Batch", "batch_sur_attach", "batch_sur_status", "SurDesc", "sur_create", "sur_param_count",
           "sur_param_offsets", "sur_set_params", "sur_get_params", "sur_forward", "sur_gradient",
           "sur_train_step", "sur_gemm_bf16", "sur_destroy", "sur_attach", "sur_status", "Surrogate",
           "last_error", "Mesh", "TERM", "EXPORTS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libmmv.so")

TERM = dict(exchange=1, anisotropy=2, zeeman=4, demag_self=8, demag_cross=16,
            eddy=32, all=63)
ERRORS = {-1: "MMV_EINVAL", -2: "MMV_ENOMEM", -3: "MMV_EHIP", -4: "MMV_ERANGE",
          -5: "MMV_ENUMERIC", -6: "MMV_ESTATE"}
EXPORTS = ("init_mesh", "set_m", "get_m", "set_offset", "set_drive", "set_hext_field", "eval_heff",
           "spline3_prefilter", "spline3_gather", "eddy_residual",
           "llg_step", "llg_run_dp", "stray_force", "stray_force_noalloc", "div_curl", "get_state", "profile_begin", "profile_end",
           "get_fft_lengths", "tune_fft_lengths", "profile_repeat", "init_batch", "batch_instance", "batch_step", "batch_tuning",
           "set_tune_cache", "destroy_batch", "destroy_mesh", "sur_create", "sur_param_count", "sur_param_offsets",
           "sur_set_params", "sur_get_params", "sur_forward", "sur_gradient", "sur_train_step",
           "sur_gemm_bf16", "sur_destroy", "sur_attach", "sur_status", "batch_sur_attach", "batch_sur_status",
           "mmv_last_error")
BATCH_AUTOTUNE, BATCH_GRAPH = 1, 2


class MMVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_films", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("gap_cells", ctypes.c_int),
                ("max_travel_cells", ctypes.c_int), ("Ms", ctypes.c_double),
                ("Aex", ctypes.c_double), ("alpha", ctypes.c_double), ("Ku", ctypes.c_double),
                ("u", ctypes.c_double * 3), ("Hext", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("precision", ctypes.c_int),
                ("cross_mode", ctypes.c_int), ("halo", ctypes.c_int),
                ("rc_cells", ctypes.c_double), ("sor_sweeps", ctypes.c_int),
                ("sor_omega", ctypes.c_double), ("fft_lx", ctypes.c_int),
                ("fft_ly", ctypes.c_int), ("fft_lz", ctypes.c_int),
                ("pbc", ctypes.c_int), ("pbc_images", ctypes.c_int)]


class DriveDesc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("v_d", ctypes.c_double), ("k", ctypes.c_double),
                ("mass", ctypes.c_double), ("gamma_v", ctypes.c_double),
                ("x_anchor0", ctypes.c_double), ("x0", ctypes.c_double),
                ("v0", ctypes.c_double)]


class SurDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("width", ctypes.c_int),
                ("modes_x", ctypes.c_int), ("modes_y", ctypes.c_int), ("layers", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("reserved", ctypes.c_int * 9)]


_LIB = None


def load():
    """Load libmmv.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is missing: build it with "
                              "`python -m paper_1801_04181_amd.build` (no fallback exists)")
        lib = ctypes.CDLL(lib_path)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        lib.init_mesh.argtypes = [ctypes.POINTER(MeshDesc), vp, ctypes.POINTER(vp)]
        lib.set_m.argtypes = [vp, i, vp]
        lib.get_m.argtypes = [vp, i, vp]
        lib.set_offset.argtypes = [vp, d]
        lib.set_drive.argtypes = [vp, ctypes.POINTER(DriveDesc)]
        lib.eval_heff.argtypes = [vp, i, i, vp]
        lib.set_hext_field.argtypes = [vp, i, vp]
        lib.spline3_prefilter.argtypes = [i, vp, vp, vp, i, i, i, vp]
        lib.eddy_residual.argtypes = [vp, pd]
        lib.spline3_gather.argtypes = [i, vp, i, i, i, vp, i, vp, vp]
        lib.llg_step.argtypes = [vp, d, i]
        lib.llg_run_dp.argtypes = [vp, d, d, pd, i, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
        lib.stray_force.argtypes = [vp, pd]
        lib.stray_force_noalloc.argtypes = [vp, vp]
        lib.div_curl.argtypes = [vp, pd, pd]
        lib.get_state.argtypes = [vp, pd, pd, pd, ctypes.POINTER(ctypes.c_long)]
        lib.get_fft_lengths.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
        lib.tune_fft_lengths.argtypes = [ctypes.POINTER(MeshDesc), d, i, i, vp, ctypes.POINTER(i), ctypes.POINTER(i),
                                         pd]
        lib.destroy_mesh.argtypes = [vp]
        lib.profile_begin.argtypes = [vp, i]
        lib.init_batch.argtypes = [ctypes.POINTER(MeshDesc), i, vp, i, ctypes.POINTER(vp)]
        lib.batch_instance.argtypes = [vp, i, ctypes.POINTER(vp)]
        lib.batch_step.argtypes = [vp, d, i]
        lib.batch_tuning.argtypes = [vp, i, ctypes.POINTER(i), ctypes.POINTER(i)]
        lib.set_tune_cache.argtypes = [ctypes.c_char_p]
        lib.destroy_batch.argtypes = [vp]
        lib.profile_end.argtypes = [vp, pd, ctypes.POINTER(ctypes.c_long)]
        lib.profile_repeat.argtypes = [vp, i, i, pd]
        ll, f = ctypes.c_longlong, ctypes.c_float
        lib.sur_create.argtypes = [ctypes.POINTER(SurDesc), vp, ctypes.POINTER(vp)]
        lib.sur_param_count.argtypes = [vp]
        lib.sur_param_offsets.argtypes = [vp, ctypes.POINTER(ll), i]
        lib.sur_set_params.argtypes = [vp, vp]
        lib.sur_get_params.argtypes = [vp, vp]
        lib.sur_forward.argtypes = [vp, vp, i, vp]
        lib.sur_gradient.argtypes = [vp, vp, vp, i, vp, pd]
        lib.sur_train_step.argtypes = [vp, vp, vp, i, f, pd, pd]
        lib.sur_gemm_bf16.argtypes = [vp, ll, ll, vp, ll, ll, vp, ll, ll, i, i, i, f, f, vp]
        lib.sur_destroy.argtypes = [vp]
        lib.sur_attach.argtypes = [vp, vp, i, d]
        lib.sur_status.argtypes = [vp, pd, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_long)]
        lib.batch_sur_attach.argtypes = [vp, vp, i, d]
        lib.batch_sur_status.argtypes = [vp, pd, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_long)]
        lib.mmv_last_error.restype = ctypes.c_char_p
        for name in EXPORTS[:-1]:
            getattr(lib, name).restype = ctypes.c_int
        lib.sur_param_count.restype = ll
        _LIB = lib
    return _LIB


def last_error():
    return load().mmv_last_error().decode()


def _check(rc):
    if rc != 0:
        raise MMVError(rc, last_error())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def to_desc(desc):
    """workloads.Desc (or any object with the same attributes) -> MeshDesc."""
    c = MeshDesc()
    for name, _ in MeshDesc._fields_:
        if name in ("u", "Hext"):
            arr = (ctypes.c_double * 3)(*[float(v) for v in getattr(desc, name)])
            setattr(c, name, arr)
        elif name in ("fft_lx", "fft_ly", "fft_lz", "pbc", "pbc_images"):
            setattr(c, name, int(getattr(desc, name, 0)))
        else:
            setattr(c, name, getattr(desc, name))
    return c


def to_drive(drv):
    c = DriveDesc()
    c.mode, c.v_d, c.k, c.mass = drv.mode, drv.v_d, drv.k, drv.mass
    c.gamma_v, c.x_anchor0, c.x0, c.v0 = drv.gamma_v, drv.x_anchor0, drv.x0, drv.v0
    return c


def init_mesh(desc, stream=None):
    h = ctypes.c_void_p()
    cd = desc if isinstance(desc, MeshDesc) else to_desc(desc)
    _check(load().init_mesh(ctypes.byref(cd), _stream(stream), ctypes.byref(h)))
    return h


def set_m(h, film, m):
    _check(load().set_m(h, film, _ptr(m)))


def get_m(h, film, out):
    _check(load().get_m(h, film, _ptr(out)))
    return out


def set_offset(h, x_cells):
    _check(load().set_offset(h, float(x_cells)))


def set_drive(h, drv):
    cd = drv if isinstance(drv, DriveDesc) else to_drive(drv)
    _check(load().set_drive(h, ctypes.byref(cd)))


def set_hext_field(h, film, field):
    """Non-uniform applied field of one film (a tensor in the mesh precision,
    [3][ny][nx] for film 0, [3][ny][nx + 2 (max_travel_cells + halo)] for the
    slider's layer, [3][ny][nx] with periodic x; films thicker than one cell
    one such plane per layer, [3][nz][ny][...]), or None to remove it."""
    _check(load().set_hext_field(h, int(film), None if field is None else _ptr(field)))


def eddy_residual(h):
    """Relative L2 residual of the last eddy-current solve (Eq. 12)."""
    r = ctypes.c_double()
    _check(load().eddy_residual(h, ctypes.byref(r)))
    return r.value


def _prec(t):
    import torch
    if t.dtype == torch.float64:
        return 64
    if t.dtype == torch.float32:
        return 32
    raise TypeError("float32 or float64 tensors")


def spline3_prefilter(field, coef, work, stream=None):
    """coef <- spline coefficients of field ([nz][ny][nx] tensors of one
    precision on the device); work is scratch."""
    nz, ny, nx = field.shape
    _check(load().spline3_prefilter(_prec(field), _ptr(field), _ptr(coef), _ptr(work), nx, ny, nz,
                                    _stream(stream)))
    return coef


def spline3_gather(coef, points, out, stream=None):
    """out[p] = tricubic spline of coef at points[p] = (x, y, z) in cells."""
    nz, ny, nx = coef.shape
    _check(load().spline3_gather(_prec(coef), _ptr(coef), nx, ny, nz, _ptr(points), int(points.shape[0]),
                                 _ptr(out), _stream(stream)))
    return out


def eval_heff(h, film, term_mask, out):
    _check(load().eval_heff(h, film, int(term_mask), _ptr(out)))
    return out


def llg_step(h, dt, nsteps=1):
    _check(load().llg_step(h, float(dt), int(nsteps)))


def llg_run_dp(h, t_end, tol, h0, max_attempts=100000):
    """Adaptive Dormand-Prince run to t_end; returns accepted and rejected
    attempts and the next proposed step."""
    hh = ctypes.c_double(float(h0))
    acc, rej = ctypes.c_long(), ctypes.c_long()
    _check(load().llg_run_dp(h, float(t_end), float(tol), ctypes.byref(hh), int(max_attempts), ctypes.byref(acc),
                             ctypes.byref(rej)))
    return dict(accepted=acc.value, rejected=rej.value, h=hh.value)


def stray_force(h):
    F = (ctypes.c_double * 3)()
    _check(load().stray_force(h, F))
    return [F[0], F[1], F[2]]


def stray_force_noalloc(h, F_dev):
    """Force [N] into the float64 device tensor F_dev (3 elements), no
    allocation, no synchronisation."""
    _check(load().stray_force_noalloc(h, _ptr(F_dev)))
    return F_dev


def div_curl(h):
    """(D, C) of Eq. 13 for the base film's field in the slider [A/m^2]."""
    D, C = ctypes.c_double(), ctypes.c_double()
    _check(load().div_curl(h, ctypes.byref(D), ctypes.byref(C)))
    return D.value, C.value


def get_state(h):
    t, x, v = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_long()
    _check(load().get_state(h, ctypes.byref(t), ctypes.byref(x), ctypes.byref(v), ctypes.byref(n)))
    return dict(t=t.value, x=x.value, v=v.value, step=n.value)


def tune_fft_lengths(desc, dt, nsteps=20, ncand=3, stream=None):
    """tune_fft_lengths of the C ABI: (fft_lx, fft_ly, ms per step) of the
    fastest candidate pair for the mesh `desc` describes."""
    c = to_desc(desc)
    a, b, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(load().tune_fft_lengths(ctypes.byref(c), float(dt), int(nsteps), int(ncand), _stream(stream),
                                   ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms)))
    return a.value, b.value, ms.value


def get_fft_lengths(h):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().get_fft_lengths(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


KERNELS = {"row_fwd": 1, "col": 2, "row_stage": 3}


def profile_begin(h, kernel):
    _check(load().profile_begin(h, KERNELS.get(kernel, kernel)))


def profile_end(h):
    ms, n = ctypes.c_double(), ctypes.c_long()
    _check(load().profile_end(h, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def profile_repeat(h, kernel, reps=200):
    """Mean ms per launch of one kernel launched reps times back to back
    (leaves the mesh state undefined)."""
    k = {"row_fwd": 1, "col": 2, "row_stage": 3}.get(kernel, kernel)
    v = ctypes.c_double()
    _check(load().profile_repeat(h, k, reps, ctypes.byref(v)))
    return v.value


def destroy_mesh(h):
    _check(load().destroy_mesh(h))


def init_batch(descs, stream=None, flags=0):
    arr = (MeshDesc * len(descs))(*[d if isinstance(d, MeshDesc) else to_desc(d) for d in descs])
    h = ctypes.c_void_p()
    _check(load().init_batch(arr, len(descs), _stream(stream), int(flags), ctypes.byref(h)))
    return h


def batch_instance(b, i):
    h = ctypes.c_void_p()
    _check(load().batch_instance(b, int(i), ctypes.byref(h)))
    return h


def batch_step(b, dt, nsteps=1):
    _check(load().batch_step(b, float(dt), int(nsteps)))


def batch_tuning(b, i, row_threads=False):
    """y-pass grouping of instance i, or (grouping, row kernel threads per
    block) with row_threads=True."""
    g = ctypes.c_int()
    r = ctypes.c_int()
    _check(load().batch_tuning(b, int(i), ctypes.byref(g), ctypes.byref(r)))
    return (g.value, r.value) if row_threads else g.value


def set_tune_cache(path):
    """Tuning cache file for MMV_BATCH_AUTOTUNE (None or "" = none)."""
    _check(load().set_tune_cache(None if not path else os.fsencode(path)))


def destroy_batch(b):
    _check(load().destroy_batch(b))


class Batch:
    """Many film pairs advanced together (torch tensors for device memory)."""

    def __init__(self, descs, drives=None, ms=None, flags=0, stream=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.descs = list(descs)
        self.dtype = torch.float64 if self.descs[0].precision == 64 else torch.float32
        self.b = init_batch(self.descs, self.stream, flags)
        self.h = [batch_instance(self.b, i) for i in range(len(self.descs))]
        for i, d in enumerate(self.descs):
            if drives is not None:
                set_drive(self.h[i], drives[i])
            if ms is not None:
                for f, mf in enumerate(ms[i]):
                    t = torch.as_tensor(mf, dtype=self.dtype).to(self.device).contiguous()
                    set_m(self.h[i], f, t)
        torch.cuda.current_stream(self.device).synchronize()

    def step(self, dt, n=1):
        batch_step(self.b, dt, n)

    def get_m(self, i, film):
        d = self.descs[i]
        out = self.torch.empty((3, d.nz, d.ny, d.nx), dtype=self.dtype, device=self.device)
        get_m(self.h[i], film, out)
        return out

    def state(self, i):
        return get_state(self.h[i])

    def tuning(self, i, row_threads=False):
        return batch_tuning(self.b, i, row_threads)

    def close(self):
        if self.b is not None:
            destroy_batch(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Owns one handle; torch tensors supply device memory and the stream."""

    def __init__(self, desc, drive=None, m=None, stream=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.desc = desc
        self.device = torch.device(device)
        self.dtype = torch.float64 if desc.precision == 64 else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = init_mesh(desc, self.stream)
        self.shape = (3, desc.nz, desc.ny, desc.nx)
        if drive is not None:
            set_drive(self.h, drive)
        if m is not None:
            for f, mf in enumerate(m):
                self.set_m(f, mf)

    def set_m(self, film, m):
        t = self.torch.as_tensor(m, dtype=self.dtype).to(self.device).contiguous()
        assert tuple(t.shape) == self.shape, (t.shape, self.shape)
        set_m(self.h, film, t)
        self.torch.cuda.current_stream(self.device).synchronize()

    def get_m(self, film):
        out = self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
        get_m(self.h, film, out)
        return out

    def set_hext_field(self, film, field):
        if field is None:
            set_hext_field(self.h, film, None)
            return
        d = self.desc
        w = d.nx if (film == 0 or getattr(d, "pbc", 0) & 1) else d.nx + 2 * (d.max_travel_cells + d.halo)
        want = (3, d.ny, w) if d.nz == 1 else (3, d.nz, d.ny, w)
        t = self.torch.as_tensor(field, dtype=self.dtype).to(self.device).contiguous()
        if tuple(t.shape) != want:
            raise ValueError(f"applied field of film {film}: shape {tuple(t.shape)}, expected {want}")
        set_hext_field(self.h, film, t)
        self.stream.synchronize()

    def eval_heff(self, film, mask=63):
        out = self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
        eval_heff(self.h, film, mask, out)
        return out

    def step(self, dt, n=1):
        llg_step(self.h, dt, n)

    def run_dp(self, t_end, tol, h0, max_attempts=100000):
        return llg_run_dp(self.h, t_end, tol, h0, max_attempts)

    def force(self):
        return stray_force(self.h)

    def state(self):
        return get_state(self.h)

    def set_offset(self, x_cells):
        set_offset(self.h, x_cells)

    def fft_lengths(self):
        return get_fft_lengths(self.h)

    def close(self):
        if self.h is not None:
            destroy_mesh(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sur_create(H, W, width=32, modes_x=16, modes_y=32, layers=4, max_batch=8, stream=None):
    d = SurDesc(H, W, width, modes_x, modes_y, layers, max_batch)
    h = ctypes.c_void_p()
    _check(load().sur_create(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
    return h


def sur_param_count(h):
    return int(load().sur_param_count(h))


def sur_param_offsets(h, layers):
    n = 4 + 3 * layers
    arr = (ctypes.c_longlong * n)()
    _check(load().sur_param_offsets(h, arr, n))
    return list(arr)


def sur_set_params(h, w):
    _check(load().sur_set_params(h, _ptr(w)))


def sur_get_params(h, out):
    _check(load().sur_get_params(h, _ptr(out)))


def sur_forward(h, a, B, out):
    _check(load().sur_forward(h, _ptr(a), B, _ptr(out)))


def sur_gradient(h, a, target, B, grad=None):
    loss = ctypes.c_double()
    g = _ptr(grad) if grad is not None else None
    _check(load().sur_gradient(h, _ptr(a), _ptr(target), B, g, ctypes.byref(loss)))
    return loss.value


def sur_train_step(h, a, target, B, lr):
    loss, rel = ctypes.c_double(), ctypes.c_double()
    _check(load().sur_train_step(h, _ptr(a), _ptr(target), B, ctypes.c_float(lr),
                                 ctypes.byref(loss), ctypes.byref(rel)))
    return loss.value, rel.value


def sur_gemm_bf16(A, am, ak, B, bk, bn, C, cm, cn, M, N, K, alpha=1.0, beta=0.0, stream=None):
    _check(load().sur_gemm_bf16(_ptr(A), am, ak, _ptr(B), bk, bn, _ptr(C), cm, cn, M, N, K,
                                ctypes.c_float(alpha), ctypes.c_float(beta), _stream(stream)))


def sur_destroy(h):
    _check(load().sur_destroy(h))


def sur_attach(h, s, judge_every=10, tol=1e-3):
    _check(load().sur_attach(h, s, judge_every, tol))


def sur_status(h):
    e, f, n = ctypes.c_double(), ctypes.c_int(), ctypes.c_long()
    _check(load().sur_status(h, ctypes.byref(e), ctypes.byref(f), ctypes.byref(n)))
    return e.value, bool(f.value), n.value


def batch_sur_attach(b, s, judge_every=10, tol=1e-3):
    _check(load().batch_sur_attach(b, s, judge_every, tol))


def batch_sur_status(b):
    e, f, n = ctypes.c_double(), ctypes.c_int(), ctypes.c_long()
    _check(load().batch_sur_status(b, ctypes.byref(e), ctypes.byref(f), ctypes.byref(n)))
    return e.value, bool(f.value), n.value


class Surrogate:
    """Learned stray-field operator; torch tensors supply device memory."""

    def __init__(self, H, W, width=32, modes_x=16, modes_y=32, layers=4, max_batch=8,
                 stream=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.H, self.W, self.layers = H, W, layers
        self.h = sur_create(H, W, width, modes_x, modes_y, layers, max_batch, self.stream)
        self.n = sur_param_count(self.h)
        self.offsets = sur_param_offsets(self.h, layers)

    def set_params(self, w):
        w = self.torch.as_tensor(w, dtype=self.torch.float32).to(self.device).contiguous()
        assert w.numel() == self.n
        sur_set_params(self.h, w)
        self.torch.cuda.current_stream(self.device).synchronize()

    def get_params(self):
        out = self.torch.empty(self.n, dtype=self.torch.float32, device=self.device)
        sur_get_params(self.h, out)
        return out

    def forward(self, a):
        B = a.shape[0]
        out = self.torch.empty((B, 3, self.H, self.W), dtype=self.torch.float32, device=self.device)
        sur_forward(self.h, a.contiguous(), B, out)
        return out

    def gradient(self, a, target):
        g = self.torch.empty(self.n, dtype=self.torch.float32, device=self.device)
        loss = sur_gradient(self.h, a.contiguous(), target.contiguous(), a.shape[0], g)
        return loss, g

    def train_step(self, a, target, lr):
        return sur_train_step(self.h, a.contiguous(), target.contiguous(), a.shape[0], lr)

    def close(self):
        if self.h is not None:
            sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
