"""ctypes binding of libsph (include/sph.h).  Argument marshalling only: every
step of the method runs in the HIP kernels behind these calls.

Device arrays are passed as raw pointers (``tensor.data_ptr()``) and the
stream as the HIP stream handle of a ``torch.cuda.Stream``.  A missing or
unloadable library raises at once; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK = 0
SPH_E_TOO_LARGE = -7
STATIC_SCRATCH_BYTES = 64 << 20   # the static scratch of sph_kdk_run_static
SPH_F32 = 0
SPH_F64 = 1
SPH_NDIAG = 9
# transport-velocity formulations (params.tv_mode)
TV_LIMITED = 0      # Eq. 15-16
TV_SCALED = 1       # Eq. 14 without limiter
TV_BACKGROUND = 2   # Eq. 12, background pressure rho0 c0^2 in the kick-drift-kick drift
TV_MODES = {"limited": TV_LIMITED, "scaled": TV_SCALED, "background": TV_BACKGROUND}

FLAG_NONFINITE = 1
FLAG_CFL = 2
FLAG_OUT_OF_BOX = 4
FLAG_INTERNAL = 8

DIAG_NAMES = ("ke", "px", "py", "pz", "vmax", "npairs", "nbeta", "nband", "transport_vmax")

# entry points declared in include/sph.h, in declaration order
EXPORTS = (
    "sph_workspace_size", "sph_tape_size", "sph_lattice_kappa", "sph_bin_positions",
    "sph_build_cells", "sph_density", "sph_forces", "sph_list_size", "sph_density_lists",
    "sph_forces_lists", "sph_wall_state", "sph_tv_correction",
    "sph_kdk_step",
    "sph_kdk_run", "sph_kdk_run_resume", "sph_kdk_run_static", "sph_dual_run", "sph_diagnostics", "sph_adjoint_step", "sph_adjoint_init", "sph_neighbor_counts",
    "sph_get_flags", "sph_clear_flags", "sph_status_string",
)


class SphParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64),
        ("ncell", ctypes.c_int32 * 3), ("tv_every", ctypes.c_int32),
        ("per_particle", ctypes.c_int32), ("tv_mode", ctypes.c_int32),
        ("box", ctypes.c_double * 3),
        ("rho0", ctypes.c_double), ("c0", ctypes.c_double), ("eta", ctypes.c_double),
        ("h_min", ctypes.c_double), ("h_max", ctypes.c_double), ("mass", ctypes.c_double),
        ("kappa", ctypes.c_double), ("dt", ctypes.c_double), ("xi", ctypes.c_double),
        ("lim_c", ctypes.c_double), ("lim_s0", ctypes.c_double),
        ("riemann_eta", ctypes.c_double), ("band_tol", ctypes.c_double),
        ("n_wall", ctypes.c_int64), ("lanes", ctypes.c_int32),
    ]


class SphDualParams(ctypes.Structure):
    _fields_ = [("cfl_ad", ctypes.c_double), ("cfl_ac", ctypes.c_double),
                ("u_ref", ctypes.c_double), ("nu", ctypes.c_double),
                ("max_substeps", ctypes.c_int32)]


class SphParticles(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("cell", "id", "off", "vel", "acc", "rho", "mass", "h", "wall_vel")]


class SphAdjoint(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in ("r_bar", "v_bar", "a_bar", "rho_bar")]


class SphError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn} failed: {text} (status {status})")
        self.status = status


_lib = None


def load():
    """Load libsph.so from the package directory; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built: run `python -m paper_2411_13992_amd.build_lib` "
            "(the GPU path has no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    pp = P(SphParams)
    sig = {
        "sph_workspace_size": [pp, P(ctypes.c_size_t)],
        "sph_tape_size": [pp, P(ctypes.c_size_t)],
        "sph_lattice_kappa": [i32, ctypes.c_double, P(ctypes.c_double)],
        "sph_bin_positions": [pp, vp, P(SphParticles), vp, ctypes.c_size_t, vp],
        "sph_build_cells": [pp, P(SphParticles), vp, vp, vp, ctypes.c_size_t, vp],
        "sph_density": [pp, P(SphParticles), vp, vp, vp],
        "sph_forces": [pp, P(SphParticles), vp, vp, vp, vp],
        "sph_list_size": [pp, P(ctypes.c_size_t)],
        "sph_density_lists": [pp, P(SphParticles), vp, vp, vp, ctypes.c_size_t, vp],
        "sph_forces_lists": [pp, P(SphParticles), vp, vp, vp, vp, ctypes.c_size_t, vp],
        "sph_wall_state": [pp, P(SphParticles), vp, vp],
        "sph_tv_correction": [pp, P(SphParticles), vp, vp, vp, vp, vp, vp],
        "sph_kdk_step": [pp, P(SphParticles), vp, ctypes.c_int64, vp, ctypes.c_size_t, vp, vp,
                         vp],
        "sph_kdk_run": [pp, P(SphParticles), vp, ctypes.c_int64, ctypes.c_int64, vp,
                        ctypes.c_size_t, vp, vp, vp],
        "sph_kdk_run_resume": [pp, P(SphParticles), vp, ctypes.c_int64, ctypes.c_int64, vp,
                               ctypes.c_size_t, vp, vp],
        "sph_kdk_run_static": [pp, P(SphParticles), vp, ctypes.c_int64, ctypes.c_int64, vp, vp,
                               vp, vp],
        "sph_dual_run": [pp, P(SphDualParams), P(SphParticles), vp, ctypes.c_int64, vp,
                         ctypes.c_size_t, vp, vp, vp],
        "sph_diagnostics": [pp, P(SphParticles), vp, vp, ctypes.c_size_t, vp, vp],
        "sph_adjoint_step": [pp, vp, P(SphAdjoint), vp, vp, ctypes.c_size_t, vp],
        "sph_adjoint_init": [pp, P(SphParticles), vp, P(SphAdjoint), vp, ctypes.c_size_t, vp],
        "sph_neighbor_counts": [pp, P(SphParticles), vp, vp, vp],
        "sph_get_flags": [vp, vp, P(ctypes.c_uint32)],
        "sph_clear_flags": [vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    L.sph_status_string.argtypes = [i32]
    L.sph_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != SPH_OK:
        text = load().sph_status_string(status).decode()
        raise SphError(fn, status, text)


def call(fn: str, *args) -> None:
    check(fn, getattr(load(), fn)(*args))


def workspace_size(params: SphParams) -> int:
    out = ctypes.c_size_t(0)
    call("sph_workspace_size", ctypes.byref(params), ctypes.byref(out))
    return int(out.value)


def list_size(params: SphParams) -> int:
    out = ctypes.c_size_t(0)
    call("sph_list_size", ctypes.byref(params), ctypes.byref(out))
    return int(out.value)


def tape_size(params: SphParams) -> int:
    out = ctypes.c_size_t(0)
    call("sph_tape_size", ctypes.byref(params), ctypes.byref(out))
    return int(out.value)


def lattice_kappa(dim: int, h_over_dx: float = 1.3) -> float:
    out = ctypes.c_double(0.0)
    call("sph_lattice_kappa", dim, float(h_over_dx), ctypes.byref(out))
    return float(out.value)
