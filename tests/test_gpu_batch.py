"""Batched film pairs: one launch per pass over uneven instances, graph replay,
autotuned grouping.  Checked bitwise against the same instances stepped alone,
and against the oracle."""
import numpy as np
import pytest
from workloads import get_config, initial_state
from workloads.configs import batch_pairs
from gpu_common import oracle_system

pytestmark = pytest.mark.gpu


def small_pairs(n, shrink):
    pairs = batch_pairs(n)
    for p in pairs:
        d = p["desc"]
        p["desc"] = d.replace(nx=max(4, d.nx // shrink), ny=max(3, d.ny // shrink))
    return pairs


def state(mmv, h, d):
    import torch
    out = []
    for f in range(2):
        t = torch.empty((3, 1, d.ny, d.nx), dtype=torch.float32, device="cuda:0")
        mmv.get_m(h, f, t)
        out.append(t.cpu().numpy())
    return out, mmv.get_state(h)


def test_batch_equals_single_instances_and_oracle():
    import torch
    import paper_1801_04181_amd as mmv
    pairs = small_pairs(10, 4)
    ms = [initial_state(p) for p in pairs]
    print("batch of", len(pairs), [(p["desc"].nx, p["desc"].ny) for p in pairs], flush=True)
    B = mmv.Batch([p["desc"] for p in pairs], [p["drive"] for p in pairs], ms)
    B.step(1e-13, 12)
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        single = mmv.Mesh(p["desc"], p["drive"], ms[i])
        single.step(1e-13, 12)
        mb, sb = state(mmv, B.h[i], p["desc"])
        m1, s1 = state(mmv, single.h, p["desc"])
        for f in range(2):
            assert np.array_equal(mb[f], m1[f]), (i, f)
        assert sb == s1
        single.close()
    for i in (0, 3, 9):
        s = oracle_system(pairs[i]["desc"], pairs[i]["drive"], ms[i])
        s.run(1e-13, 12)
        mb, sb = state(mmv, B.h[i], pairs[i]["desc"])
        dm = max(np.abs(mb[f] - s.m[f]).max() for f in range(2))
        print("  oracle instance", i, "max|dm|", dm, flush=True)
        assert dm < 1e-5
        assert abs(sb["x"] - s.x) < 1e-4 * pairs[i]["desc"].dx
    B.close()


def test_graph_replay_equals_eager_every_replay():
    import torch
    import paper_1801_04181_amd as mmv
    pairs = small_pairs(6, 8)
    ms = [initial_state(p) for p in pairs]
    descs = [p["desc"] for p in pairs]
    drives = [p["drive"] for p in pairs]
    G = mmv.Batch(descs, drives, ms, flags=mmv.BATCH_GRAPH)
    E = mmv.Batch(descs, drives, ms)
    for rep in range(4):
        G.step(1e-13, 8)        # one graph replay of 8 steps
        E.step(1e-13, 8)        # the same launches, eager
        torch.cuda.synchronize()
        for i, p in enumerate(pairs):
            mg, sg = state(mmv, G.h[i], p["desc"])
            me, se = state(mmv, E.h[i], p["desc"])
            for f in range(2):
                assert np.array_equal(mg[f], me[f]), (rep, i, f)
            assert sg == se, (rep, i)
        # host-side work between replays
        _ = torch.ones(1000, device="cuda:0").sum().item()
    G.step(1e-13, 11)           # one replay + three eager steps
    E.step(1e-13, 11)
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        assert np.array_equal(state(mmv, G.h[i], p["desc"])[0][1], state(mmv, E.h[i], p["desc"])[0][1])
    G.close()
    E.close()


def test_autotune_choice_is_valid_and_harmless():
    import torch
    import paper_1801_04181_amd as mmv
    pairs = small_pairs(8, 2)
    ms = [initial_state(p) for p in pairs]
    descs = [p["desc"] for p in pairs]
    drives = [p["drive"] for p in pairs]
    T = mmv.Batch(descs, drives, ms, flags=mmv.BATCH_AUTOTUNE)
    U = mmv.Batch(descs, drives, ms)
    groups = [T.tuning(i) for i in range(len(pairs))]
    rows = [T.tuning(i, row_threads=True)[1] for i in range(len(pairs))]
    print("autotuned groups", groups, "row threads", rows, flush=True)
    assert all(1 <= g <= 4 for g in groups)
    for nt, d in zip(rows, descs):
        assert nt in (128, 256, 512) and nt >= min(d.nx, 512), (nt, d.nx)
    T.step(1e-13, 5)
    U.step(1e-13, 5)
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        for f in range(2):
            assert np.array_equal(state(mmv, T.h[i], p["desc"])[0][f], state(mmv, U.h[i], p["desc"])[0][f])
    T.close()
    U.close()


def test_tuning_cache_is_written_and_read_back(tmp_path):
    """The first autotuned batch writes one line per mesh size; a second batch
    of the same mix takes the stored groupings without timing (an edited
    entry is honoured and left in place)."""
    import paper_1801_04181_amd as mmv
    pairs = small_pairs(8, 2)
    ms = [initial_state(p) for p in pairs]
    descs = [p["desc"] for p in pairs]
    drives = [p["drive"] for p in pairs]
    path = tmp_path / "tune.txt"
    sizes = {(d.nx, d.ny) for d in descs}
    try:
        mmv.set_tune_cache(str(path))
        T = mmv.Batch(descs, drives, ms, flags=mmv.BATCH_AUTOTUNE)
        groups = [T.tuning(i) for i in range(len(pairs))]
        T.close()
        lines = path.read_text().splitlines()
        print("cache", lines, flush=True)
        stored, row_lines = {}, {}
        for ln in lines:
            key, g = ln.split("\t")
            assert "gfx" in key and " f32 " in key
            (row_lines if key.endswith(" row") else stored)[key] = int(g)
        assert len(stored) == len(sizes)
        assert set(stored.values()) <= set(groups)
        # row lengths with more than one block size to choose from: 72 and
        # 140 points (nx 64 and 128; 128, 256 or 512 threads), 270 (nx 256)
        assert len(row_lines) == 3 and set(row_lines.values()) <= {2, 4, 8}
        # edit every grouping to another valid one; keep the row entries
        edited = {k: (3 if g != 3 else 1) for k, g in stored.items()}
        edited.update(row_lines)
        path.write_text("".join(f"{k}\t{g}\n" for k, g in edited.items()) + "malformed line\n")
        U = mmv.Batch(descs, drives, ms, flags=mmv.BATCH_AUTOTUNE)
        regroup = [U.tuning(i) for i in range(len(pairs))]
        U.close()
        for i, g in enumerate(groups):
            assert regroup[i] == (3 if g != 3 else 1), (i, g, regroup[i])
        # nothing was re-timed, so the file keeps the edited entries
        kept = dict(ln.split("\t") for ln in path.read_text().splitlines() if "\t" in ln)
        assert {k: int(v) for k, v in kept.items()} == edited
    finally:
        mmv.set_tune_cache(None)


def test_batch_with_a_largest_instance_equals_single_instances():
    """A batch mixing the widest float32 mesh init_mesh accepts with small
    ones: every instance's magnetisation bitwise equal to the same instance
    stepped alone.  The slider state agrees to float64 rounding: the batch
    row kernel runs 512 threads and the single-mesh one 1024, so on rows
    wider than 512 cells each thread sums a different set of cells into
    its float64 force partial."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import slider_mass_damping
    from workloads.configs import DRIVE_SPRING
    from workloads import Drive
    base = batch_pairs(2)
    descs, drives, ms = [], [], []
    for nx, ny in [(1728, 8), (64, 64), (96, 24)]:
        d = base[0]["desc"].replace(nx=nx, ny=ny)
        mass, gv = slider_mass_damping(nx, ny, 1e-3)
        descs.append(d)
        drives.append(Drive(mode=DRIVE_SPRING, v_d=3.0, k=1e-3, mass=mass, gamma_v=gv))
        ms.append([np.asarray(x) for x in initial_state(dict(base[0], desc=d))])
    print("batch with the widest instance", [(d.nx, d.ny) for d in descs], flush=True)
    B = mmv.Batch(descs, drives, ms)
    B.step(1e-13, 4)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        single = mmv.Mesh(d, drives[i], ms[i])
        single.step(1e-13, 4)
        mb, sb = state(mmv, B.h[i], d)
        m1, s1 = state(mmv, single.h, d)
        for f in range(2):
            assert np.array_equal(mb[f], m1[f]), (i, f)
        assert sb["step"] == s1["step"] and sb["t"] == s1["t"]
        for k in ("x", "v"):
            assert abs(sb[k] - s1[k]) <= 1e-12 * max(abs(s1[k]), 1e-30), (i, k, sb[k], s1[k])
        if d.nx <= 512:
            assert sb == s1, i
        single.close()
    B.close()
