"""Benchmark: cell-updates/s of the two-film hot path on one MI355X.

One step = one classic RK4 step of both films (4 effective-field
evaluations: x transforms, y pass with the kernel multiplication, fused row
kernel with the spline, local terms, LLG stage and force) plus the slider's
equation of motion.  Workload: the stick-slip films, 2 x 512 x 128 cells of
2 nm, float32, spring drive, seeded synthetic +/-z domain states.

Prints one JSON line: metric, value, unit, timing, roofline of the dominant
kernel and the float64 CPU reference's rate on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "cell-updates/s per LLG step; surrogate+batched vs plain at ≤1e-3 H error"

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs
# (summaries under profiles/), scaled by the same counters read on a plain
# device copy of known size, keyed by kernel and by the hash of the kernel
# sources they were taken on: a changed kernel reports null.
TRAFFIC = {
    "col": {"source": "06dd3518653b", "bytes": 16149150},
    "row_stage": {"source": "06dd3518653b", "bytes": 19418985},
    "batch_step": {"source": "06dd3518653b", "bytes": 3064962902},
}
KERNEL_SOURCES = ("paper_1801_04181_amd/csrc/mmv_kernels.hip", "paper_1801_04181_amd/csrc/mmv_device.h",
                  "paper_1801_04181_amd/csrc/mmv_internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def traffic_of(kernel):
    t = TRAFFIC.get(kernel)
    if t is None or t.get("source") != kernel_source_hash():
        return None
    return t["bytes"]


def kernel_bytes(desc, lx, ly):
    """Algorithmic bytes per launch of each kernel (float32, direct mode).

    x transform: read m, write the row spectra of the ny non-zero rows.
    y pass:      read those spectra and each kernel channel once, write every
                 output row of every channel.
    row kernel:  read every output row, m of the stage, m at the step start,
                 the RK accumulator (3 of 4 stages), write the next stage m and
                 the accumulator (3 of 4 stages), and write the next stage's
                 row spectra (the x transform runs inside the row kernel).
    """
    r = 4 if desc.precision == 32 else 8
    c = 2 * r
    nf, nx, ny = desc.n_films, desc.nx, desc.ny
    kx = lx // 2 + 1
    kyh = ly // 2 + 1
    cells = nf * nx * ny
    spec1 = 3 * nf * ny * kx * c
    rows = 3 * nf * ny
    nkern = 4
    if nf == 2:
        rows += 3 * (ny + 2) + 2 * ny + 3 * ny
        nkern += 6 + 3 + 3
    spec2 = rows * kx * c
    kern = nkern * kx * kyh * r
    return {
        "row_fwd": 3 * cells * r + spec1,
        "col": spec1 + kern + spec2,
        "row_stage": spec2 + cells * 3 * r * (1 + 1 + 0.75 + 1 + 0.75) + spec1,
    }, cells


def cpu_baseline(cfg, m, budget_s=12.0):
    """The float64 oracle, as it stands, on a bounded sample of the workload."""
    from threadpoolctl import threadpool_limits
    from oracle.sim import System
    d = cfg["desc"]
    with threadpool_limits(limits=1):
        s = System(d, cfg["drive"], m)
        s.field_terms()            # build the kernel windows outside the clock
        t0 = time.perf_counter()
        n = 0
        while n < 2 or (time.perf_counter() - t0 < budget_s and n < 50):
            s.step(cfg["dt"])
            n += 1
        dt = time.perf_counter() - t0
    return {"value": d.cells * n / dt, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} RK4 steps of the same 2x{d.nx}x{d.ny} workload, float64 "
                      f"NumPy/SciPy oracle, 1 thread, {dt:.1f} s"}


def host_info():
    """Cores this process may run on and the CPU model (the baseline's host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


class scipy_fft_backend:
    """Within the block, numpy's FFT calls (the oracle's) run on scipy.fft
    with `workers` threads; the oracle's code itself is unchanged."""
    NAMES = ("fft2", "ifft2", "rfftn", "irfftn", "fftn", "ifftn", "rfft", "irfft", "fft", "ifft")

    def __init__(self, workers):
        self.workers = workers

    def __enter__(self):
        import numpy as np
        import scipy.fft as sf
        self.saved = {k: getattr(np.fft, k) for k in self.NAMES}
        for k in self.NAMES:
            fn = getattr(sf, k)
            setattr(np.fft, k, (lambda f: lambda *a, **kw: f(*a, workers=self.workers, **kw))(fn))
        return self

    def __exit__(self, *exc):
        import numpy as np
        for k, f in self.saved.items():
            setattr(np.fft, k, f)


def cpu_baseline_variants():
    """The float64 oracle on the other workloads and with a multi-threaded FFT
    backend (bounded samples; throughput per step is constant)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.sim import System
    from workloads import get_config, initial_state
    from workloads.configs import batch_pairs
    ncore, model = host_info()
    out = {"host_cores": ncore, "cpu_model": model, "runs": []}

    def timed(name, systems, steps, dt, workers):
        cells = sum(sy.desc.cells for sy in systems)
        ctx = scipy_fft_backend(workers) if workers > 1 else None
        with threadpool_limits(limits=workers):
            if ctx:
                ctx.__enter__()
            try:
                for sy in systems:
                    sy.field_terms()            # kernel windows built outside the clock
                t0 = time.perf_counter()
                for sy in systems:
                    sy.run(dt, steps)
                el = time.perf_counter() - t0
            finally:
                if ctx:
                    ctx.__exit__(None, None, None)
        out["runs"].append({"workload": name, "value": cells * steps / el, "unit": "cell-updates/s",
                            "cores": workers, "fft": "scipy.fft workers=%d" % workers if workers > 1
                            else "numpy.fft (1 thread)", "steps": steps, "seconds": el})

    cfg = get_config("stickslip")
    timed("stickslip 2x512x128 f64 oracle", [System(cfg["desc"], cfg["drive"], initial_state(cfg))], 8,
          cfg["dt"], ncore)
    cfg = get_config("tiny")
    timed("tiny 2x32x32 (100 steps)", [System(cfg["desc"], cfg["drive"], initial_state(cfg))], 100, cfg["dt"], 1)
    cfg = get_config("cube_eddy")
    timed("cube 64^3 with eddy currents", [System(cfg["desc"], cfg["drive"], initial_state(cfg))], 2, cfg["dt"], 1)
    pairs = batch_pairs(64)[:8]          # one pair of each size class
    timed("batch: 8 of the 64 uneven pairs (one per size class)",
          [System(p["desc"], p["drive"], initial_state(p)) for p in pairs], 1, pairs[0]["dt"], 1)
    return out


def batch_step_bytes(descs, lxly):
    """Algorithmic bytes of one batched RK4 step (four stages of the y pass
    and the row kernel per instance; the x pass runs inside the row kernel)."""
    tot = 0.0
    for d, (lx, ly) in zip(descs, lxly):
        per, _ = kernel_bytes(d, lx, ly)
        tot += 4 * (per["col"] + per["row_stage"])
    return tot


def batched_vs_plain(steps_batch=200, steps_plain=50, graph=True):
    """64 uneven pairs: per-instance launches vs one batched, graph-replayed launch per pass."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import initial_state
    from workloads.configs import batch_pairs
    pairs = batch_pairs(64)
    descs = [p["desc"] for p in pairs]
    drives = [p["drive"] for p in pairs]
    ms = [initial_state(p) for p in pairs]
    dt = pairs[0]["dt"]
    cells = sum(d.cells for d in descs)
    meshes = [mmv.Mesh(d, drv, m) for d, drv, m in zip(descs, drives, ms)]
    lxly = [me.fft_lengths()[:2] for me in meshes]
    for me in meshes:
        me.step(dt, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for me in meshes:
        me.step(dt, steps_plain)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for me in meshes:
        me.close()
    B = mmv.Batch(descs, drives, ms, flags=mmv.BATCH_AUTOTUNE | (mmv.BATCH_GRAPH if graph else 0))
    B.step(dt, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(dt, steps_batch)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    groups = sorted(set(B.tuning(i) for i in range(len(descs))))
    row_threads = {}
    for i, d in enumerate(descs):
        row_threads[str(d.nx)] = B.tuning(i, row_threads=True)[1]
    B.close()
    plain = cells * steps_plain / t_plain
    batched = cells * steps_batch / t_batch
    step_bytes = batch_step_bytes(descs, lxly)
    step_s = t_batch / steps_batch
    achieved = step_bytes / step_s / 1e9
    return {"workload": "64 uneven pairs nx {64,128,256,512} x ny {64,128}, 2 nm, f32, spring drives",
            "cells": cells, "plain_cell_updates_per_s": plain,
            "batched_cell_updates_per_s": batched, "speedup": batched / plain,
            "ms_per_step_batched": step_s * 1e3, "autotuned_groups": groups,
            "autotuned_row_threads_by_nx": row_threads,
            "roofline": {"bound": "hbm", "scope": "whole batched step (every launch of the 4 stages)",
                         "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM_GBS, "bytes_per_step": step_bytes,
                         "traffic": traffic_of("batch_step"),
                         "timing": "host clock around graph-replayed steps, stream synchronised"}}


def surrogate_batched(n=16, steps=20):
    """The metric's comparison on the learned-operator workload (2 x 256 x
    256 films): n instances stepped with the width-32 operator replacing film
    0's cross field (one batched inference per RK stage), against the same
    instances exact-batched and stepped one by one.  The operator here is
    untrained (seeded initial weights): its speed does not depend on the
    weights, and its judged error is reported as measured."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state
    from workloads.fno_inputs import init_params
    cfg = get_config("learned")
    d, drv, dt = cfg["desc"], cfg["drive"], cfg["dt"]
    m = initial_state(cfg)
    C, Mx, My, L = 32, 16, 32, 4
    cells = d.cells * n
    sur = mmv.Surrogate(d.ny, d.nx, C, Mx, My, L, max_batch=n)
    sur.set_params(torch.from_numpy(init_params(C, Mx, My, L, seed=2)).float())
    B = mmv.Batch([d] * n, [drv] * n, [m] * n)
    mmv.batch_sur_attach(B.b, sur.h, 10, 1e30)      # judge every 10 steps, never falls back
    B.step(dt, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(dt, steps)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    err, fell, judged = mmv.batch_sur_status(B.b)
    B.close()
    E = mmv.Batch([d] * n, [drv] * n, [m] * n, flags=mmv.BATCH_GRAPH)
    E.step(dt, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step(dt, 2 * steps)
    torch.cuda.synchronize()
    t_exact = (time.perf_counter() - t0) / 2
    E.close()
    meshes = [mmv.Mesh(d, drv, m) for _ in range(n)]
    for me in meshes:
        me.step(dt, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for me in meshes:
        me.step(dt, steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for me in meshes:
        me.close()
    sur.close()
    return {"workload": f"{n} x (2 films 256x256), f32, spring drive; operator width {C}, "
                        f"{Mx}x{My} modes, {L} layers, BF16 matrix cores (untrained weights)",
            "instances": n, "cells": cells,
            "surrogate_batched_cell_updates_per_s": cells * steps / t_sur,
            "exact_batched_cell_updates_per_s": cells * steps / t_exact,
            "plain_cell_updates_per_s": cells * steps / t_plain,
            "surrogate_batched_vs_plain": t_plain / t_sur,
            "judged_rel_err": err, "judges": judged,
            "meets_1e-3": bool(err <= 1e-3)}


def cube_report(steps=40, warmup=4):
    """Step time of the 64^3 conducting cube (the single-magnet 3-D path),
    float32 and float64, with the eddy term (sigma = 1e7 S/m, once per step:
    dB/dt, the E_sol convolution, 40 red-black SOR sweeps, J x S), with it
    and the exact cosine-basis Neumann solve instead of the sweeps, and
    without it (sigma = 0): HIP events around `steps` RK4 steps on the mesh's
    stream."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state

    cfg = get_config("cube_eddy")
    m = initial_state(cfg)
    cells = cfg["desc"].nx * cfg["desc"].ny * cfg["desc"].nz
    out = {"workload": "64^3 cube, 2 nm cells, RK4 dt 5e-14 s, Zeeman + exchange + demag (+ eddy)",
           "cells": cells, "steps": steps}
    for prec in (32, 64):
        for eddy in (True, "exact", False):
            d = cfg["desc"].replace(precision=prec, sigma=cfg["desc"].sigma if eddy else 0.0,
                                    sor_sweeps=-1 if eddy == "exact" else cfg["desc"].sor_sweeps)
            mesh = mmv.Mesh(d, cfg["drive"], m)
            mesh.step(cfg["dt"], warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(mesh.stream)
            mesh.step(cfg["dt"], steps)
            e1.record(mesh.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            mesh.close()
            name = {True: "eddy", "exact": "eddy_exact_solve", False: "no_eddy", "periodic": "eddy_periodic"}[eddy]
            out[f"fp{prec}_{name}"] = {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3)}
    return out


def eddy_films_report(steps=20, warmup=2, cpu=True):
    """Step time of two conducting CoCrPt films, 2 x 128 x 128 x 5 cells of
    4 nm (the eddy-current friction workload), float32 and float64, with
    eddy currents in both films (sigma = 1e6 S/m: dB/dt, the E_sol sums with
    the other film's interpolated part, 40 red-black SOR sweeps per film,
    J x S), with the exact cosine-basis Neumann solve instead of the sweeps,
    without (sigma = 0), and with the sweeps in films periodic in x and y
    (one image on each side; the transform lengths are the periods, 128):
    HIP events around `steps` RK4 steps on the mesh's stream.  The oracle
    (float64 CPU) times one step."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state

    cfg = get_config("eddy_films")
    d0, drv, dt = cfg["desc"], cfg["drive"], cfg["dt"]
    m = initial_state(cfg)
    cells = d0.n_films * d0.nx * d0.ny * d0.nz
    out = {"workload": "2 films 128x128x5 cells of 4 nm, 5 cells apart, CoCrPt, sigma 1e6 S/m, "
                       "spring drive 2 m/s, RK4 dt 1e-13 s",
           "cells": cells, "steps": steps}
    for prec in (32, 64):
        for eddy in (True, "exact", False, "periodic"):
            d = d0.replace(precision=prec, sigma=d0.sigma if eddy else 0.0,
                           sor_sweeps=-1 if eddy == "exact" else d0.sor_sweeps)
            if eddy == "periodic":
                d = d.replace(pbc=3, pbc_images=1)
            mesh = mmv.Mesh(d, drv, m)
            mesh.step(dt, warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(mesh.stream)
            mesh.step(dt, steps)
            e1.record(mesh.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            name = {True: "eddy", "exact": "eddy_exact_solve", False: "no_eddy", "periodic": "eddy_periodic"}[eddy]
            out[f"fp{prec}_{name}"] = {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                                       "fft": list(mesh.fft_lengths()[:2])}
            mesh.close()
    if cpu:
        from threadpoolctl import threadpool_limits
        from oracle.slab import SlabSystem
        with threadpool_limits(limits=1):
            s = SlabSystem(d0.replace(precision=64), drv, m)
            s.step(dt)              # kernel windows and the first eddy update outside the clock
            t0 = time.perf_counter()
            s.step(dt)
            sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cells / sec, "unit": "cell-updates/s", "kind": "oracle", "cores": 1,
                               "sample": f"1 RK4 step with eddy currents of the same workload, float64 "
                                         f"NumPy/SciPy oracle, 1 thread, {sec:.1f} s"}
    return out


def variants_report(steps=400, warmup=40, dp_span_steps=400, dp_tol=1e-5):
    """The step's variants on the stick-slip films (2 x 512 x 128, float32).

    periodic: in-plane periodic boundaries along x and y (pbc = 3, one image
      on each side; the transform lengths are the periods, 512 and 128):
      HIP events around `steps` RK4 steps, and the row kernel's launch time
      against its algorithmic bytes (as the main line's roofline);
    adaptive: the Dormand-Prince RK5(4) run (llg_run_dp) over
      dp_span_steps x 1e-13 s at tol dp_tol from the state after `warmup`
      RK4 steps: attempts, accepted steps, mean accepted step, wall time
      (host clock around the call, which checks the run's end every 8
      attempts), time per attempt (seven stages) and cell-updates per second
      counted per accepted step."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state

    cfg = get_config("stickslip")
    d0, drv, dt = cfg["desc"], cfg["drive"], cfg["dt"]
    m = initial_state(cfg)
    out = {"workload": "stickslip: 2 films 512x128x1 cells of 2 nm, float32, spring drive"}
    d = d0.replace(pbc=3, pbc_images=1)
    mesh = mmv.Mesh(d, drv, m)
    mesh.step(dt, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(mesh.stream)
    mesh.step(dt, steps)
    e1.record(mesh.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lx, ly, _ = mesh.fft_lengths()
    per_launch, cells = kernel_bytes(d, lx, ly)
    kern_ms = {k: mmv.profile_repeat(mesh.h, k, 200) for k in ("col", "row_stage")}
    dom = max(kern_ms, key=kern_ms.get)
    ach = per_launch[dom] / (kern_ms[dom] * 1e-3) / 1e9
    out["periodic"] = {"pbc": 3, "pbc_images": 1, "fft": [lx, ly], "ms_per_step": ms,
                       "cell_updates_per_s": cells / (ms * 1e-3),
                       "kernel_us": {k: v * 1e3 for k, v in kern_ms.items()},
                       "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": PEAK_HBM_GBS,
                                    "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                                    "bytes_per_launch": per_launch[dom]}}
    mesh.close()
    mesh = mmv.Mesh(d0, drv, m)
    mesh.step(dt, warmup)
    torch.cuda.synchronize()
    t0s = mesh.state()["t"]
    t_end = t0s + dp_span_steps * dt
    w0 = time.perf_counter()
    r = mesh.run_dp(t_end, dp_tol, dt, max_attempts=20000)
    wall = time.perf_counter() - w0
    st = mesh.state()
    attempts = r["accepted"] + r["rejected"]
    out["adaptive"] = {"tol": dp_tol, "span_s": t_end - t0s, "reached_s": st["t"] - t0s,
                       "accepted": r["accepted"], "rejected": r["rejected"],
                       "mean_step_s": (st["t"] - t0s) / max(r["accepted"], 1), "wall_s": wall,
                       "ms_per_attempt": wall * 1e3 / max(attempts, 1),
                       "cell_updates_per_s": cells * r["accepted"] / wall,
                       "rk4_equivalent_steps_per_s": (st["t"] - t0s) / dt / wall}
    mesh.close()
    out["spline3"] = spline3_timing()
    return out


def spline3_timing(n=128, npts=1 << 20, reps=20):
    """The 64-tap tricubic spline primitives (motion off the x axis) on an
    n^3 float32 field: the prefilter along x, y, z and the gather at npts
    seeded random points, HIP events around `reps` calls each.  Algorithmic
    bytes: the prefilter reads and writes the field once per axis (6 n^3 x 4
    B); the gather reads each point (12 B) and writes its value (4 B), the
    coefficients once (n^3 x 4 B)."""
    import torch
    import paper_1801_04181_amd as mmv
    g = torch.Generator(device="cuda:0").manual_seed(5)
    f = torch.rand((n, n, n), generator=g, device="cuda:0", dtype=torch.float32)
    coef = torch.empty_like(f)
    work = torch.empty_like(f)
    pts = torch.rand((npts, 3), generator=g, device="cuda:0", dtype=torch.float32) * (n - 1)
    out = torch.empty(npts, device="cuda:0", dtype=torch.float32)
    st = torch.cuda.current_stream()
    mmv.spline3_prefilter(f, coef, work, stream=st)
    mmv.spline3_gather(coef, pts, out, stream=st)
    res = {"n": n, "points": npts}
    for name, fn, nbytes in (("prefilter", lambda: mmv.spline3_prefilter(f, coef, work, stream=st), 6 * n ** 3 * 4),
                             ("gather", lambda: mmv.spline3_gather(coef, pts, out, stream=st),
                              npts * 16 + n ** 3 * 4)):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        res[name] = {"us_per_call": us, "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / (us * 1e-6) / 1e9,
                     "frac_of_hbm": nbytes / (us * 1e-6) / 1e9 / PEAK_HBM_GBS}
    return res


def surrogate_report(train_steps=3000, B=8, steps=200, log=None):
    """Learned stray-field operator on the 2 x 256 x 256 films: train on fresh
    exact pairs, held-out error, then LLG steps with the operator attached
    (judge every 10 steps) against plain exact steps and the batched exact path."""
    import numpy as np
    import torch
    import paper_1801_04181_amd as mmv
    from paper_1801_04181_amd.surrogate import PairSource, train, held_out_error
    from workloads import get_config, initial_state
    from workloads.states import domain_state
    from workloads.fno_inputs import init_params
    log = log or (lambda msg: print(msg, file=sys.stderr, flush=True))
    cfg = get_config("learned")
    d, drv, dt = cfg["desc"], cfg["drive"], cfg["dt"]
    C, Mx, My, L = 32, 16, 32, 4
    pool = [domain_state((1, d.ny, d.nx), 1000 + k)[:, 0] for k in range(64)]
    src = PairSource(d, pool, seed=1)
    sur = mmv.Surrogate(d.ny, d.nx, C, Mx, My, L, max_batch=B)
    sur.set_params(torch.from_numpy(init_params(C, Mx, My, L, seed=2)).float())
    t0 = time.perf_counter()
    hist = train(sur, src, train_steps, B=B, log=log)
    t_train = time.perf_counter() - t0
    held = held_out_error(sur, PairSource(d, pool, seed=99), n=64, B=B)
    log(f"held-out relative error {held:.4f}")
    a = src.batch(B)[0]
    times = {}
    for nb in (1, B):
        for _ in range(3):
            sur.forward(a[:nb])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            sur.forward(a[:nb])
        torch.cuda.synchronize()
        times[nb] = (time.perf_counter() - t0) / 20 * 1e3
    m = initial_state(cfg)

    def run(attach=None):
        me = mmv.Mesh(d, drv, m)
        if attach is not None:
            mmv.sur_attach(me.h, sur.h, 10, attach)
        me.step(dt, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        me.step(dt, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = mmv.sur_status(me.h) if attach is not None else None
        me.close()
        return d.cells * steps / el, el / steps * 1e3, st

    plain, ms_plain, _ = run()
    sur_rate, ms_sur, st_free = run(1e30)          # judge runs, never falls back
    strict_rate, ms_strict, st_strict = run(1e-3)
    descs = [d] * B
    bt = mmv.Batch(descs, [drv] * B, [m] * B, flags=mmv.BATCH_AUTOTUNE | mmv.BATCH_GRAPH)
    bt.step(dt, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(dt, steps)
    torch.cuda.synchronize()
    batched = d.cells * B * steps / (time.perf_counter() - t0)
    bt.close()
    sur.close()
    return {
        "workload": f"2x{d.nx}x{d.ny} films, f32, spring drive; operator width {C}, "
                    f"{Mx}x{My} modes, {L} layers, BF16 matrix cores",
        "train_steps": train_steps, "train_batch": B, "train_s": t_train,
        "train_rel_err_last100": float(np.mean(hist[-100:])),
        "held_out_rel_err": held,
        "forward_ms": {str(k): v for k, v in times.items()},
        "plain_cell_updates_per_s": plain, "plain_ms_per_step": ms_plain,
        "surrogate_cell_updates_per_s": sur_rate, "surrogate_ms_per_step": ms_sur,
        "surrogate_judged_rel_err": st_free[0],
        "strict_tol_1e-3": {"fell_back": st_strict[1], "judged": st_strict[2],
                            "rel_err": st_strict[0], "cell_updates_per_s": strict_rate},
        "batched_exact_8_pairs_cell_updates_per_s": batched,
        "meets_1e-3": bool(held <= 1e-3),
    }


def divcurl_study(nx=256, ny=64, gaps=(3, 5), npts=21, seed=13):
    """Eq. 13 on the GPU: D(x) and C(x) of the base film's field sampled in the
    slider, relative to the stationary (lattice) position, while the slider
    moves one cell (4 nm) over a frozen random base (Sec. IV.A), for the
    spline of the direct field, the scalar potential and linear
    interpolation; float64 curves, the float32 maxima beside them, and the
    time of one div_curl call (HIP events)."""
    import numpy as np
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import Desc, Drive
    from workloads.states import random_unit

    rng = np.random.default_rng(seed)
    m = [random_unit((1, ny, nx), rng), random_unit((1, ny, nx), rng)]
    xs = [i / (npts - 1) for i in range(npts)]
    out = {"workload": f"2 films {nx}x{ny}x1, 4 nm cells, random frozen base and slider (seed {seed}), "
                       f"slider moved 0..1 cell in {npts - 1} steps",
           "x_cells": xs, "runs": []}
    for gap in gaps:
        for mode, name in ((0, "spline"), (1, "potential"), (2, "linear")):
            run = {"gap_cells": gap, "interpolant": name}
            for prec in (64, 32):
                d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=4e-9, dy=4e-9, dz=4e-9, gap_cells=gap,
                         max_travel_cells=2, Ms=8e5, Aex=1.3e-11, alpha=0.5, cross_mode=mode, precision=prec)
                mesh = mmv.Mesh(d, Drive(), m)
                rD, rC = [], []
                D0 = C0 = None
                for x in xs:
                    mesh.set_offset(x)
                    D, C = mmv.div_curl(mesh.h)
                    if D0 is None:
                        D0, C0 = D, C
                    rD.append((D - D0) / D0)
                    rC.append((C - C0) / C0)
                if prec == 64:
                    run.update(D0=D0, C0=C0, rel_D=rD, rel_C=rC)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(mesh.stream)
                    for _ in range(5):
                        mmv.div_curl(mesh.h)
                    e1.record(mesh.stream)
                    torch.cuda.synchronize()
                    run["ms_per_call_f64"] = e0.elapsed_time(e1) / 5
                run[f"max_abs_rel_D_f{prec}"] = max(abs(v) for v in rD)
                run[f"max_abs_rel_C_f{prec}"] = max(abs(v) for v in rC)
                mesh.close()
            print(f"divcurl gap {gap} {name}: max |dD/D| {run['max_abs_rel_D_f64']:.3e} "
                  f"max |dC/C| {run['max_abs_rel_C_f64']:.3e}", file=sys.stderr, flush=True)
            out["runs"].append(run)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="stickslip")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-eddy", action="store_true", help="skip the conducting cube and thick-film step times")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the periodic and adaptive variants of the stick-slip step")
    ap.add_argument("--no-graph", action="store_true", help="--report batch: eager launches (counter runs)")
    ap.add_argument("--report", choices=["surrogate", "cube", "batch", "surrogate-batched", "divcurl",
                                         "eddy-films", "variants"],
                    default=None)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, copy 256 MiB device to device 3 times (counter calibration)")
    args = ap.parse_args()
    if args.report == "cube":
        print(json.dumps({"cube_report": cube_report()}), flush=True)
        return
    if args.report == "variants":
        print(json.dumps({"variants": variants_report()}), flush=True)
        return
    if args.report == "eddy-films":
        print(json.dumps({"eddy_films_report": eddy_films_report(steps=args.steps if args.steps < 2000 else 20,
                                                                 cpu=not args.no_cpu)}), flush=True)
        return
    if args.report == "batch":
        print(json.dumps({"batched": batched_vs_plain(steps_batch=args.steps, steps_plain=2,
                                                      graph=not args.no_graph)}), flush=True)
        if args.calib_copy:
            calib_copy()
        return
    if args.report == "divcurl":
        print(json.dumps({"divcurl_study": divcurl_study()}), flush=True)
        return
    if args.report == "surrogate-batched":
        print(json.dumps({"surrogate_batched": surrogate_batched()}), flush=True)
        return
    if args.report == "surrogate":
        print(json.dumps({"surrogate_report": surrogate_report(args.train_steps)}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; sharding the films over several "
              "GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state

    cfg = get_config(args.config)
    d, drv, dt = cfg["desc"], cfg["drive"], cfg["dt"]
    m = initial_state(cfg)
    print(f"bench: {args.config} 2x{d.nx}x{d.ny} fp{d.precision}, warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    mesh = mmv.Mesh(d, drv, m)
    lx, ly, _ = mesh.fft_lengths()
    per_launch, cells = kernel_bytes(d, lx, ly)
    stream = mesh.stream

    mesh.step(dt, args.warmup)
    torch.cuda.synchronize()

    # timed region
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    mesh.step(dt, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    value = cells * args.steps / (ms_total * 1e-3)

    st = mesh.state()
    # per-kernel launch time: each hot kernel launched 200 times back to back
    # with stage inputs between one pair of HIP events (this leaves the mesh
    # state undefined, so it runs after the timed region and the state read)
    kern_ms = {k: mmv.profile_repeat(mesh.h, k, 200) for k in ("col", "row_stage")}
    dom = max(kern_ms, key=kern_ms.get)
    avg_s = kern_ms[dom] * 1e-3
    achieved = per_launch[dom] / avg_s / 1e9
    mesh.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if d.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 2 films {d.nx}x{d.ny}x1 cells of "
                               f"{d.dx*1e9:g} nm, RK4 dt {dt:g} s, spring drive, direct spline mode",
                   "cells": cells, "fft": [lx, ly], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic_of(dom), "bytes_per_launch": per_launch[dom],
                     "avg_launch_us": avg_s * 1e6, "launches": 200,
                     "timing": "HIP events around 200 back-to-back launches with stage inputs"},
        "kernel_us": {k: v * 1e3 for k, v in kern_ms.items()},
        "wall_s": wall,
        "slider_x_nm": st["x"] * 1e9,
    }
    if not args.no_batch:
        out["batched"] = batched_vs_plain()
        out["surrogate_batched"] = surrogate_batched()
    if not args.no_eddy:
        # the conducting workloads' step times (GPU only; their oracles'
        # timings are in the reports of their own)
        out["cube_eddy"] = cube_report()
        out["eddy_films"] = eddy_films_report(cpu=False)
    if not args.no_variants:
        out["variants"] = variants_report()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, m)
        out["cpu_baseline_variants"] = cpu_baseline_variants()
    print(json.dumps(out), flush=True)
    if args.calib_copy:
        calib_copy()


def calib_copy():
    """Three device copies of 256 MiB: the counters' scale for known bytes."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("calib copy: 268435456 bytes read and written per launch", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
