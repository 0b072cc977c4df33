"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/sph.h declares, validates arguments before
enqueueing anything, and its own constants agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2411_13992_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sph.h")).read()
    return re.findall(r"^(?:int32_t|const char \*)\s*(sph_\w+)\s*\(", text, flags=re.M)


def test_params_layout_matches_header():
    """The ctypes mirror of sph_params has the header's field order: the
    doubles start at byte 40 (after eight 32-bit and one 64-bit fields), the
    wall count and the lane count follow the sixteen doubles; sph_particles
    holds nine pointers."""
    assert _lib.SphParams.box.offset == 40
    assert _lib.SphParams.tv_mode.offset == 36
    assert _lib.SphParams.n_wall.offset == 40 + 8 * 16
    assert _lib.SphParams.lanes.offset == 40 + 8 * 16 + 8
    assert ctypes.sizeof(_lib.SphParams) == 40 + 8 * 16 + 16
    assert _lib.SphParticles.wall_vel.offset == 64
    assert ctypes.sizeof(_lib.SphParticles) == 72


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_lib.EXPORTS)


def _params(**kw):
    p = _lib.SphParams()
    p.dim, p.dtype, p.n = 2, _lib.SPH_F32, 1000
    p.ncell[0], p.ncell[1], p.ncell[2] = 10, 10, 1
    p.box[0], p.box[1], p.box[2] = 1.0, 1.0, 1.0
    p.tv_every = 1
    p.per_particle = 0
    p.rho0, p.c0, p.eta = 1.0, 10.0, 0.01
    p.h_min = p.h_max = 0.04
    p.mass = 1e-3
    p.kappa = 1.01
    p.dt, p.xi, p.lim_c, p.lim_s0, p.riemann_eta, p.band_tol = 1e-3, -0.2, 1e3, 5e-4, 3.0, 1e-5
    for k, v in kw.items():
        if k in ("ncell", "box"):
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        else:
            setattr(p, k, v)
    return p


def _status(p):
    out = ctypes.c_size_t(0)
    return _lib.load().sph_workspace_size(ctypes.byref(p), ctypes.byref(out)), out.value


def test_argument_validation():
    st, size = _status(_params())
    assert st == 0 and size > 0
    assert _status(_params(dim=4))[0] == -6
    assert _status(_params(dtype=7))[0] == -6
    assert _status(_params(n=-1))[0] == -1
    assert _status(_params(ncell=(2, 10, 1)))[0] == -4
    assert _status(_params(h_max=0.06))[0] == -4          # L = 0.1 < 2 h_max
    assert _status(_params(c0=float("nan")))[0] == -5
    assert _status(_params(dt=-1.0))[0] == -1
    assert _status(_params(h_min=0.05, h_max=0.04))[0] == -1
    assert _status(_params(per_particle=2))[0] == -1
    for mode in (_lib.TV_LIMITED, _lib.TV_SCALED, _lib.TV_BACKGROUND):
        assert _status(_params(tv_mode=mode))[0] == 0
    assert _status(_params(tv_mode=3))[0] == -1
    assert _status(_params(tv_mode=-1))[0] == -1
    assert _status(_params(n_wall=1000))[0] == 0
    assert _status(_params(n_wall=1001))[0] == -1
    assert _status(_params(n_wall=-1))[0] == -1
    assert _status(_params(n_wall=10, per_particle=1))[0] == -6    # walls: uniform resolution
    for lanes in (0, 2, 4, 8):
        assert _status(_params(lanes=lanes))[0] == 0
    assert _status(_params(lanes=3))[0] == -1
    assert _status(_params(lanes=16))[0] == -1
    L = _lib.load()
    assert L.sph_workspace_size(None, None) == -1
    assert b"cell grid" in L.sph_status_string(-4)


def test_sizes_grow_with_n_and_dtype():
    s32 = _status(_params(n=1000))[1]
    s32b = _status(_params(n=5000))[1]
    s64 = _status(_params(n=1000, dtype=_lib.SPH_F64))[1]
    assert s32b > s32 and s64 > s32
    # more lanes per particle: more diagnostic partial rows
    assert _status(_params(lanes=8))[1] > _status(_params(lanes=2))[1]
    assert _lib.tape_size(_params()) > 0


def test_null_pointers_rejected_before_launch():
    L = _lib.load()
    p = _params()
    parts = _lib.SphParticles()
    assert L.sph_density(ctypes.byref(p), ctypes.byref(parts), None, None, None) == -1
    assert L.sph_kdk_step(ctypes.byref(p), ctypes.byref(parts), None, 0, None, 0, None, None,
                          None) == -1
    st = L.sph_build_cells(ctypes.byref(p), None, None, None, None, 0, None)
    assert st == -1


def test_wall_arguments_checked_before_launch():
    """Walls need their prescribed velocities, checked before any launch."""
    L = _lib.load()
    p = _params(n_wall=100)
    parts = _lib.SphParticles()
    for name in ("cell", "id", "off", "vel", "acc", "rho"):
        setattr(parts, name, 4096)       # never dereferenced: the checks fail first
    assert L.sph_wall_state(ctypes.byref(p), ctypes.byref(parts), None, None) == -1
    assert L.sph_density(ctypes.byref(p), ctypes.byref(parts), 4096, 4096, None) == -1
    assert L.sph_kdk_step(ctypes.byref(p), ctypes.byref(parts), 4096, 0, 4096, 1 << 40,
                          None, None, None) == -1
    # walled tapes carry the particle ids: larger than wall-free ones
    assert _lib.tape_size(_params(n_wall=100)) > _lib.tape_size(_params()) + 4 * 1000


@pytest.mark.parametrize("dim", [2, 3])
def test_library_kappa_matches_oracle(dim):
    """The library's reference kernel sum (Eq. 8) agrees with the oracle's,
    two independent codes of the same lattice sum."""
    assert abs(_lib.lattice_kappa(dim, 1.3) - oracle.lattice_kappa(dim, 1.3)) < 1e-14


def test_automatic_lane_choice():
    """0 picks by size: 8 for small inputs, 2 (2-D) or 4 (3-D) for the
    benchmark workloads; the choice shows in the workspace size."""
    from paper_2411_13992_amd import _lib
    from paper_2411_13992_amd.sim import config_from_case, make_params

    def ws(case, lanes):
        p = make_params(config_from_case(case, lanes=lanes), case.n, "f32")
        return _lib.workspace_size(p)
    import cases
    small = cases.taylor_green_2d(37, jitter=0.05, seed=9)
    assert ws(small, 0) == ws(small, 8)
    big = cases.taylor_green_2d(400, jitter=0.05)
    assert ws(big, 0) == ws(big, 2)
    cube = cases.taylor_green_3d(128)
    assert ws(cube, 0) == ws(cube, 4)


def test_static_run_rejects_oversize_before_launch():
    """The allocation-free run refuses, on the host and before anything is
    enqueued, a problem whose workspace exceeds its static scratch, and checks
    its other arguments like sph_kdk_run."""
    L = _lib.load()
    parts = _lib.SphParticles()
    for name in ("cell", "id", "off", "vel", "acc", "rho"):
        setattr(parts, name, 4096)       # never dereferenced: the checks fail first
    small = _params(n=1000)
    assert _status(small)[1] <= _lib.STATIC_SCRATCH_BYTES
    big = _params(n=1_000_000, ncell=(400, 400, 1), h_min=1e-3, h_max=1e-3)
    assert _status(big)[1] > _lib.STATIC_SCRATCH_BYTES
    st = L.sph_kdk_run_static(ctypes.byref(big), ctypes.byref(parts), 4096, 0, 3, None, None,
                              None, None)
    assert st == _lib.SPH_E_TOO_LARGE
    assert b"static scratch" in L.sph_status_string(st)
    assert L.sph_kdk_run_static(ctypes.byref(small), ctypes.byref(parts), None, 0, 3, None,
                                None, None, None) == -1
    assert L.sph_kdk_run_static(ctypes.byref(small), None, 4096, 0, 3, None, None, None,
                                None) == -1
    assert L.sph_kdk_run_static(ctypes.byref(small), ctypes.byref(parts), 4096, -1, 3, None,
                                None, None, None) == -1


def test_list_entry_points_check_arguments():
    """sph_list_size is positive for an ordinary problem; the list sweeps
    reject a missing or short list buffer before enqueueing anything."""
    L = _lib.load()
    p = _params()
    size = ctypes.c_size_t(0)
    assert L.sph_list_size(ctypes.byref(p), ctypes.byref(size)) == 0
    assert size.value > 0
    parts = _lib.SphParticles()
    for name in ("cell", "id", "off", "vel", "acc", "rho"):
        setattr(parts, name, 4096)       # never dereferenced: the checks fail first
    args = (ctypes.byref(p), ctypes.byref(parts), 4096, 4096)
    assert L.sph_density_lists(*args, None, size.value, None) == -1
    assert L.sph_density_lists(*args, 4096, size.value - 1, None) == -3
    assert L.sph_forces_lists(*args, 4096, None, size.value, None) == -1
    assert L.sph_forces_lists(*args, 4096, 4096, size.value - 1, None) == -3


def test_resume_checks_arguments():
    """sph_kdk_run_resume validates its arguments like sph_kdk_run, before
    enqueueing anything."""
    L = _lib.load()
    p = _params()
    parts = _lib.SphParticles()
    for name in ("cell", "id", "off", "vel", "acc", "rho"):
        setattr(parts, name, 4096)       # never dereferenced: the checks fail first
    assert L.sph_kdk_run_resume(ctypes.byref(p), ctypes.byref(parts), None, 0, 3, 4096, 1 << 40,
                                None, None) == -1
    assert L.sph_kdk_run_resume(ctypes.byref(p), ctypes.byref(parts), 4096, 0, 3, None, 1 << 40,
                                None, None) == -1
    assert L.sph_kdk_run_resume(ctypes.byref(p), ctypes.byref(parts), 4096, 0, 3, 4096, 16,
                                None, None) == -3
    assert L.sph_kdk_run_resume(ctypes.byref(p), ctypes.byref(parts), 4096, -1, 3, 4096, 1 << 40,
                                None, None) == -1
