"""Precision split of the GPU path against the float64 oracle (a report
script beside the tests, not a test; run on one GPU).

  python tests/precision_report.py > report.json

Parts:
- the 64^3 conducting cube (eddy currents on): per-term relative L2 error
  of the float32 and float64 GPU paths after 2 steps, and max |dm| after 6;
- the same cube over 2000 steps (the precision configuration's length):
  at steps 500, 1000, 1500 and 2000, max |dm| on the 16^3 sub-lattice of
  every fourth cell and the error of the mean magnetisation against the
  oracle's run stored in tests/golden/cube_2000.npz (written by
  tests/golden/make_cube_long.py from the oracle alone), and the float32
  path's drift from the float64 path over all cells;
- the stick-slip films (2 x 512 x 128, float32): per-term errors, the force,
  and max |dm| and the slider position after 50 steps.

float64 is kept on the GPU for the tensor / potential-kernel construction
and for the slider's position, velocity and force accumulation in both
precisions.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)


def precision_report(steps_cube=6, steps_film=50):
    """Per-term error of the float32 and float64 GPU paths against the float64
    oracle: the 64^3 conducting cube (eddy currents on) and the stick-slip films.
    float64 is kept on the GPU for the tensor/S construction and for the
    slider's position, velocity and force accumulation in both precisions."""
    import numpy as np
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state
    from oracle.sim import System

    def rel(a, b):
        nb = np.linalg.norm(b)
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))

    names = (("exchange", 1), ("anisotropy", 2), ("zeeman", 4), ("demag_self", 8),
             ("demag_cross", 16), ("eddy", 32))
    out = {}
    cfg = get_config("cube_eddy")
    m = initial_state(cfg)
    ref = System(cfg["desc"], cfg["drive"], m)
    ref.run(cfg["dt"], 2)                     # two steps: dB/dt and the eddy field exist
    terms2, _ = ref.field_terms()
    m2 = [x.copy() for x in ref.m]
    ref.run(cfg["dt"], steps_cube - 2)
    for prec in (32, 64):
        d = cfg["desc"].replace(precision=prec)
        mesh = mmv.Mesh(d, cfg["drive"], m)
        mesh.step(cfg["dt"], 2)
        torch.cuda.synchronize()
        r = {"m_after_2": float(np.abs(mesh.get_m(0).cpu().numpy() - m2[0]).max())}
        for name, bit in names:
            if name == "demag_cross" or not np.any(terms2[0][name]):
                continue
            # field terms of the GPU state after 2 steps vs the oracle's
            r[name] = rel(mesh.eval_heff(0, bit).cpu().numpy(), terms2[0][name])
        r["total"] = rel(mesh.eval_heff(0, 63).cpu().numpy(), System.total(terms2[0]))
        mesh.step(cfg["dt"], steps_cube - 2)
        torch.cuda.synchronize()
        r[f"m_after_{steps_cube}"] = float(np.abs(mesh.get_m(0).cpu().numpy() - ref.m[0]).max())
        mesh.close()
        out[f"cube_eddy_fp{prec}"] = r
    cfg = get_config("stickslip")
    m = initial_state(cfg)
    ref = System(cfg["desc"], cfg["drive"], m)
    terms, F = ref.field_terms()
    mesh = mmv.Mesh(cfg["desc"], cfg["drive"], m)
    r = {}
    for f in range(2):
        for name, bit in names[:5]:
            if np.any(terms[f][name]):
                r[f"film{f}_{name}"] = rel(mesh.eval_heff(f, bit).cpu().numpy(), terms[f][name])
    Fg = np.array(mesh.force())
    r["force"] = float(np.linalg.norm(Fg - F) / np.linalg.norm(F))
    mesh.step(cfg["dt"], steps_film)
    torch.cuda.synchronize()
    ref.run(cfg["dt"], steps_film)
    r[f"m_after_{steps_film}"] = max(float(np.abs(mesh.get_m(f).cpu().numpy() - ref.m[f]).max())
                                     for f in range(2))
    st = mesh.state()
    r[f"x_after_{steps_film}_cells"] = abs(st["x"] - ref.x) / cfg["desc"].dx
    mesh.close()
    out["stickslip_fp32"] = r
    return out


def cube_long():
    """2000 steps of the cube in both precisions against the stored oracle
    samples; the float32 path's drift from the float64 path."""
    import numpy as np
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import get_config, initial_state
    g = np.load(os.path.join(HERE, "golden", "cube_2000.npz"))
    steps = [int(s) for s in g["steps"]]
    stride = int(g["stride"])
    cfg = get_config("cube_eddy")
    m = initial_state(cfg)
    meshes = {p: mmv.Mesh(cfg["desc"].replace(precision=p), cfg["drive"], m) for p in (32, 64)}
    out = {"steps": steps, "sample": f"every {stride}th cell along each axis", "fp32": [], "fp64": [],
           "fp32_vs_fp64": []}
    done = 0
    for s in steps:
        full = {}
        for p, mesh in meshes.items():
            mesh.step(cfg["dt"], s - done)
            torch.cuda.synchronize()
            mg = mesh.get_m(0).cpu().numpy().astype(np.float64)
            full[p] = mg
            samp = mg[:, ::stride, ::stride, ::stride]
            ref = g[f"m_{s}"]
            out[f"fp{p}"].append({
                "step": s,
                "max_dm_sampled": float(np.abs(samp - ref).max()),
                "mean_m_error": float(np.abs(mg.reshape(3, -1).mean(axis=1) - g[f"mean_{s}"]).max()),
                "eddy_residual": mmv.eddy_residual(mesh.h)})
        out["fp32_vs_fp64"].append({"step": s, "max_dm_all_cells": float(np.abs(full[32] - full[64]).max())})
        done = s
        print(f"cube long: step {s}: fp32 {out['fp32'][-1]['max_dm_sampled']:.3e} "
              f"fp64 {out['fp64'][-1]['max_dm_sampled']:.3e}", file=sys.stderr, flush=True)
    # per-term float32 rounding on the state 2000 steps in: the float32
    # kernels evaluated on the float64 run's state against the float64
    # kernels on it (instantaneous terms); the eddy field, which carries the
    # step history, float32 run against float64 run
    def rel(a, b):
        nb = np.linalg.norm(b)
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
    m64 = meshes[64].get_m(0).cpu().numpy()
    probe = mmv.Mesh(cfg["desc"].replace(precision=32, sigma=0.0), cfg["drive"], [m64])
    terms = {}
    for name, bit in (("exchange", 1), ("zeeman", 4), ("demag_self", 8)):
        terms[name] = rel(probe.eval_heff(0, bit).cpu().numpy().astype(np.float64),
                          meshes[64].eval_heff(0, bit).cpu().numpy())
    terms["eddy_fp32_run_vs_fp64_run"] = rel(meshes[32].eval_heff(0, 32).cpu().numpy().astype(np.float64),
                                             meshes[64].eval_heff(0, 32).cpu().numpy())
    probe.close()
    out["terms_at_2000"] = terms
    for mesh in meshes.values():
        mesh.close()
    return out


if __name__ == "__main__":
    rep = {"precision_report": precision_report()}
    if os.path.exists(os.path.join(HERE, "golden", "cube_2000.npz")):
        rep["precision_report"]["cube_eddy_2000_steps"] = cube_long()
    print(json.dumps(rep), flush=True)
