"""C-ABI checks that need no GPU: the library loads, exports every symbol of
include/mmv.h, and rejects bad arguments before touching the device."""
import ctypes
import os
import re
import pytest
import paper_1801_04181_amd as mmv
from workloads import Desc, get_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mmv.h")


def header_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|long long|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_header_lists_the_path_calls():
    fns = header_functions()
    for name in ("init_mesh", "set_offset", "eval_heff", "llg_step", "stray_force"):
        assert name in fns


def test_library_exports_every_header_symbol():
    lib = mmv.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(mmv.EXPORTS)


def test_struct_layout_matches_header():
    # offsets the C compiler assigns (x86-64 SysV): checked against ctypes
    assert ctypes.sizeof(mmv.MeshDesc) == 200
    assert ctypes.sizeof(mmv.DriveDesc) == 64
    assert ctypes.sizeof(mmv.SurDesc) == 64


@pytest.mark.parametrize("field,value,msg", [
    ("n_films", 3, "n_films"), ("nx", 0, "nx"), ("dx", 0.0, "cell edges"),
    ("dz", float("nan"), "cell edges"), ("Ms", -1.0, "Ms"), ("precision", 16, "precision"),
    ("halo", 1, "halo"), ("gap_cells", -1, "gap_cells"),
    ("sigma", 1e6, "eddy"), ("rc_cells", 0.0, "rc_cells"), ("max_travel_cells", -1, "max_travel"),
    ("fft_lx", 71, "fft_lx"), ("fft_ly", 11, "fft_ly"),
])
def test_init_rejects_bad_descriptors(field, value, msg):
    d = get_config("tiny")["desc"]
    c = mmv.to_desc(d)
    setattr(c, field, value)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(c)
    assert e.value.code == -1
    assert msg in str(e.value)


@pytest.mark.parametrize("change,msg", [
    (dict(pbc=4), "pbc must be"), (dict(pbc=1, pbc_images=-1), "pbc_images"),
    (dict(pbc=1, pbc_images=1025), "pbc_images"), (dict(pbc=1, nx=31), "nx even"),
    (dict(pbc=2, ny=11), "ny {2,3,5,7}"), (dict(pbc=1, fft_lx=72), "period"),
])
def test_periodic_descriptor_validation(change, msg):
    c = mmv.to_desc(get_config("tiny")["desc"])
    for k, v in change.items():
        setattr(c, k, v)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(c)
    assert e.value.code == -1
    assert msg in str(e.value)


def test_periodic_needs_films():
    d = get_config("cube_eddy")["desc"].replace(nx=8, ny=8, nz=8, pbc=1)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(d)
    assert "one cell thick" in str(e.value)


@pytest.mark.parametrize("gap", [0, 1, 2])
def test_potential_mode_refused_closer_than_three_cells(gap):
    # Sec. IV.D: the films must be more than two cells apart for the
    # potential's four-point difference (and the force stencil around it)
    d = get_config("tiny_potential")["desc"].replace(gap_cells=gap)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(d)
    assert e.value.code == -1
    assert "gap_cells >= 3" in str(e.value)


def test_null_handle_and_pointers():
    lib = mmv.load()
    assert lib.destroy_mesh(None) == 0
    assert lib.llg_step(None, 1e-13, 1) == -1
    assert "handle" in mmv.last_error()
    assert lib.init_mesh(None, None, None) == -1
    F = (ctypes.c_double * 3)()
    assert lib.stray_force(None, F) == -1


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library every call raises (no CPU fallback): run in
    a fresh interpreter so the loaded library of this process is untouched."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1801_04181_amd as mmv\n"
        "mmv.lib_path = %r\n"
        "from workloads import get_config\n"
        "for f in (lambda: mmv.load(), lambda: mmv.init_mesh(mmv.to_desc(get_config('tiny')['desc']))):\n"
        "    try:\n"
        "        f()\n"
        "    except ImportError as e:\n"
        "        assert 'no fallback' in str(e), e\n"
        "    else:\n"
        "        raise SystemExit('call succeeded without the library')\n"
        "print('ok')\n"
    ) % (ROOT, str(tmp_path / "absent" / "libmmv.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_tune_cache_path_checks():
    """The tuning-cache path is validated and copied; clearing it is always
    accepted (no GPU call is made)."""
    with pytest.raises(mmv.MMVError) as e:
        mmv.set_tune_cache("x" * 5000)
    assert e.value.code == -1 and "too long" in str(e.value)
    mmv.set_tune_cache("/tmp/some_cache_file")
    mmv.set_tune_cache("")
    mmv.set_tune_cache(None)


@pytest.mark.parametrize("kw,msg", [(dict(nx=1800, ny=16), "row kernel's LDS"),
                                    (dict(nx=900, ny=16, precision=64), "row kernel's LDS"),
                                    (dict(nx=64, ny=820), "y pass"),
                                    (dict(nx=64, ny=410, precision=64), "y pass")])
def test_size_limits_are_checked_before_any_device_call(kw, msg):
    """Meshes past the LDS limits of the film kernels are refused with
    MMV_EINVAL from the host checks (no GPU here: a device call would have
    returned MMV_EHIP)."""
    d = get_config("stickslip")["desc"].replace(**kw)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d))
    assert e.value.code == -1 and msg in str(e.value)


@pytest.mark.parametrize("prec,shape", [(32, (2600, 4, 4)), (32, (4, 1800, 4)), (32, (4, 4, 1500)),
                                        (64, (4, 4, 760))])
def test_cube_size_limits_are_checked_before_any_device_call(prec, shape):
    nx, ny, nz = shape
    d = get_config("cube_eddy")["desc"].replace(nx=nx, ny=ny, nz=nz, precision=prec)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d))
    assert e.value.code == -1 and "three-dimensional" in str(e.value)


def test_thick_films_descriptor_rules():
    """Thick films take the scalar potential only more than two cells apart
    (as one-layer films), periodic in-plane boundaries only as two films, and
    eddy currents in films periodic in y with an even period (red-black
    sweeps)."""
    d = get_config("tiny_potential")["desc"].replace(nz=2, gap_cells=2)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d))
    assert e.value.code == -1 and "gap_cells >= 3" in str(e.value)
    for change, msg in ((dict(nz=2, pbc=1, n_films=1), "two thicker films"),
                        (dict(nz=2, pbc=2, ny=31, sigma=1e6), "ny even")):
        d = get_config("tiny")["desc"].replace(**change)
        with pytest.raises(mmv.MMVError) as e:
            mmv.init_mesh(mmv.to_desc(d))
        assert e.value.code == -1 and msg in str(e.value), (change, str(e.value))


def test_potential_mode_needs_two_films():
    d = get_config("tiny_potential")["desc"].replace(n_films=1)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d))
    assert e.value.code == -1 and "two films" in str(e.value)


def test_exact_neumann_solve_descriptor():
    d = get_config("cube_eddy")["desc"]
    for sweeps in (-2, -100):
        with pytest.raises(mmv.MMVError) as e:
            mmv.init_mesh(mmv.to_desc(d.replace(sor_sweeps=sweeps)))
        assert "sor_sweeps" in str(e.value)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d.replace(sor_sweeps=-1, nx=37)))
    assert "smooth" in str(e.value)


def test_eddy_needs_a_thick_single_magnet():
    d = get_config("stickslip")["desc"].replace(sigma=1e6)
    with pytest.raises(mmv.MMVError) as e:
        mmv.init_mesh(mmv.to_desc(d))
    assert "eddy" in str(e.value)
    d = get_config("cube_eddy")["desc"].replace(sor_omega=2.5)
    with pytest.raises(mmv.MMVError):
        mmv.init_mesh(mmv.to_desc(d))


@pytest.mark.parametrize("kw,msg", [
    (dict(H=4), "H, W"), (dict(width=0), "width"), (dict(modes_x=200), "modes_x"),
    (dict(modes_y=3), "modes_y"), (dict(layers=0), "layers"), (dict(max_batch=0), "max_batch")])
def test_surrogate_rejects_bad_shapes(kw, msg):
    args = dict(H=64, W=64, width=8, modes_x=8, modes_y=8, layers=2, max_batch=2)
    args.update(kw)
    with pytest.raises(mmv.MMVError) as e:
        mmv.sur_create(**args)
    assert e.value.code == -1 and msg in str(e.value)


@pytest.mark.parametrize("args,msg", [
    ((16, 1, 1, 1, 1, 1, 1, 1), "precision"),
    ((32, 0, 8, 16, 0, 4, 4, 0), "NULL"),
    ((32, 8, 16, 24, 0, 4, 4, 0), "nx, ny, nz"),
    ((64, 8, 16, 24, 2048, 2048, 1024, 0), "too large"),
    ((32, 8, 8, 24, 2, 2, 2, 0), "overlap"),
])
def test_spline3_prefilter_argument_checks(args, msg):
    """Rejected before any device call (the pointers are never touched)."""
    lib = mmv.load()
    prec, f, c, w, nx, ny, nz, st = args
    vp = ctypes.c_void_p
    rc = lib.spline3_prefilter(prec, vp(f) if f else None, vp(c) if c else None, vp(w) if w else None,
                               nx, ny, nz, None)
    assert rc == -1
    assert msg in mmv.last_error()


def test_spline3_gather_argument_checks():
    lib = mmv.load()
    assert lib.spline3_gather(8, None, 2, 2, 2, None, 1, None, None) == -1
    assert lib.spline3_gather(32, None, 2, 0, 2, None, 1, None, None) == -1
    assert lib.spline3_gather(32, None, 2, 2, 2, None, -1, None, None) == -1
    assert lib.spline3_gather(32, None, 2, 2, 2, None, 3, None, None) == -1
    assert "NULL" in mmv.last_error()
    assert lib.spline3_gather(32, None, 2, 2, 2, None, 0, None, None) == 0   # empty: nothing launched


def test_tune_fft_lengths_checks_arguments_before_any_device_call():
    d = get_config("tiny")["desc"]
    for kw, msg in ((dict(ncand=0), "ncand"), (dict(ncand=9), "ncand"), (dict(nsteps=0), "nsteps"),
                    (dict(dt=-1.0), "dt")):
        args = dict(dt=1e-13, nsteps=5, ncand=3)
        args.update(kw)
        with pytest.raises(mmv.MMVError) as e:
            mmv.tune_fft_lengths(d, **args)
        assert e.value.code == -1 and msg in str(e.value), (kw, str(e.value))
