"""FP64 CPU oracle for the transport-velocity WCSPH step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The GPU library never imports, links or calls it, and it imports
nothing from the GPU package.  The arithmetic lives in ``sph_oracle.c`` (plain
C, FP64, index-order sums); this module loads it with ctypes and marshals NumPy
arrays.  ``brute.py`` holds an independent NumPy statement of the neighbour
set for tiny inputs.

Citations (sections and equations of arXiv 2411.13992):
  density summation Eq. (8); EOS Eq. (2); Riemann momentum Eq. (3b) with the
  limited linear solver Eq. (5)-(6); viscous term Eq. (7); transport-velocity
  correction Eq. (14)-(16); Wendland kernel with h = 1.3 dp (Sec. 4);
  kick-drift-kick integration (Sec. 3, the time integration of the original
  transport-velocity formulation); wall particles for the lid-driven cavity
  (Sec. 4.2; the wall treatment is a reading, stated in ``sph_oracle.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NDIAG = 9
DIAG_NAMES = ("ke", "px", "py", "pz", "vmax", "npairs", "nbeta", "nband", "transport_vmax")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (C11, -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("rho0", ctypes.c_double), ("c0", ctypes.c_double), ("eta", ctypes.c_double),
        ("dt", ctypes.c_double), ("xi", ctypes.c_double), ("lim_c", ctypes.c_double),
        ("lim_s0", ctypes.c_double), ("riemann_eta", ctypes.c_double),
        ("h_min", ctypes.c_double), ("kappa", ctypes.c_double), ("band_tol", ctypes.c_double),
        ("tv_every", ctypes.c_int32), ("use_grid", ctypes.c_int32),
        ("tv_mode", ctypes.c_int32), ("n_wall", ctypes.c_int64),
        ("wall_vel", ctypes.POINTER(ctypes.c_double)),
    ]


class DualParams(ctypes.Structure):
    """Dual-criteria time stepping (Sec. 2.4): CFL numbers of Eq. 9 and 11,
    the reference speed and kinematic viscosity of Eq. 10, and an optional
    cap on the acoustic substeps of one advection step."""
    _fields_ = [
        ("cfl_ad", ctypes.c_double), ("cfl_ac", ctypes.c_double), ("u_ref", ctypes.c_double),
        ("nu", ctypes.c_double), ("max_substeps", ctypes.c_int32),
        ("refresh_geometry", ctypes.c_int32),
    ]


def dual_params(case, cfl_ad: float = 0.25, cfl_ac: float = 0.6,
                max_substeps: int = 0, refresh_geometry: bool = False) -> DualParams:
    return DualParams(cfl_ad=cfl_ad, cfl_ac=cfl_ac, u_ref=case.u_ref, nu=case.eta / case.rho0,
                      max_substeps=max_substeps, refresh_geometry=int(refresh_geometry))


# Transport-velocity formulations
TV_LIMITED = 0      # h-scaled correction with the limiter, Eq. (16)
TV_SCALED = 1       # h-scaled correction without limiter, Eq. (14)
TV_BACKGROUND = 2   # background pressure rho0 c0^2 in kick-drift-kick, Eq. (12)
TV_MODES = {"limited": TV_LIMITED, "scaled": TV_SCALED, "background": TV_BACKGROUND}


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_kernel_w.restype = ctypes.c_double
        L.oracle_kernel_w.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oracle_kernel_f.restype = ctypes.c_double
        L.oracle_kernel_f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oracle_lattice_kappa.restype = ctypes.c_double
        L.oracle_lattice_kappa.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        for name in ("oracle_neighbors_brute", "oracle_neighbors_grid"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _I64, _I32]
        L.oracle_density.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _I64, _I32,
                                     ctypes.c_double, _D]
        L.oracle_tv.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _I64, _I32,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                _D, _D, _D, _D, _D]
        L.oracle_forces.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _D,
                                    _I64, _I32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_wall_bc.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _D, _D, _D,
                                     _I64, _I32, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.oracle_init.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D,
                                  ctypes.POINTER(Params), _D, _D]
        L.oracle_kdk_step.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D,
                                      ctypes.POINTER(Params), ctypes.c_int64, _D, _D, _D, _D, _D]
        L.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D,
                                 ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int64, _D]
        L.oracle_dt_advection.restype = ctypes.c_double
        L.oracle_dt_advection.argtypes = [ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(DualParams)]
        L.oracle_dt_acoustic.restype = ctypes.c_double
        L.oracle_dt_acoustic.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(DualParams)]
        L.oracle_continuity.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _D,
                                        _I64, _I32, ctypes.c_double, ctypes.c_double, _D]
        L.oracle_dual_step.restype = ctypes.c_int64
        L.oracle_dual_step.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D, _D,
                                       ctypes.POINTER(Params), ctypes.POINTER(DualParams),
                                       _D, _D, _D, _D, _D, _D]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    if a.dtype == np.float64:
        return a.ctypes.data_as(_D)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_I64)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_I32)
    raise TypeError(a.dtype)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def kernel_w(dim, r, h):
    return lib().oracle_kernel_w(dim, float(r), float(h))


def kernel_f(dim, r, h):
    return lib().oracle_kernel_f(dim, float(r), float(h))


def lattice_kappa(dim: int, h_over_dx: float = 1.3) -> float:
    """kappa_D = sum over a perfect lattice (incl. self) of W * dx^D."""
    return lib().oracle_lattice_kappa(dim, float(h_over_dx))


def params(case, band_tol: float = 1e-5, tv_every: int = 1, use_grid: bool = True,
           xi: float | None = None, kappa: float | None = None,
           tv_mode: int | str = TV_LIMITED) -> Params:
    if isinstance(tv_mode, str):
        tv_mode = TV_MODES[tv_mode]
    prm = Params(rho0=case.rho0, c0=case.c0, eta=case.eta, dt=case.dt,
                 xi=case.xi if xi is None else xi, lim_c=case.lim_c, lim_s0=case.lim_s0,
                 riemann_eta=case.riemann_eta, h_min=case.h_min,
                 kappa=lattice_kappa(case.dim) if kappa is None else kappa,
                 band_tol=band_tol, tv_every=tv_every, use_grid=1 if use_grid else 0,
                 tv_mode=int(tv_mode), n_wall=int(getattr(case, "n_wall", 0)))
    if prm.n_wall > 0:
        prm.wall_keep = _f64(case.wall_vel).copy()     # kept alive with the struct
        prm.wall_vel = _p(prm.wall_keep)
    return prm


def neighbors(pos, h, box, method: str = "grid"):
    """CSR neighbour lists (start[n+1], list[P]) with ascending j per particle."""
    pos = _f64(pos)
    h = _f64(h)
    box = _f64(box)
    dim, n = pos.shape
    start = np.zeros(n + 1, dtype=np.int64)
    f = lib().oracle_neighbors_grid if method == "grid" else lib().oracle_neighbors_brute
    total = f(dim, n, _p(pos), _p(h), _p(box), _p(start), None)
    lst = np.zeros(max(total, 1), dtype=np.int32)
    f(dim, n, _p(pos), _p(h), _p(box), _p(start), _p(lst))
    return start, lst[:total]


def density(pos, mass, h, box, nbr, kappa):
    pos, mass, h, box = map(_f64, (pos, mass, h, box))
    dim, n = pos.shape
    start, lst = nbr
    rho = np.zeros(n)
    lib().oracle_density(dim, n, _p(pos), _p(mass), _p(h), _p(box), _p(start), _p(lst),
                         float(kappa), _p(rho))
    return rho


def tv(pos, mass, rho, h, box, nbr, h_min, xi=-0.2, lim_c=1e3, lim_s0=5e-4,
       tv_mode: int | str = TV_LIMITED, bg: float = 0.0):
    """Returns dict g, s, beta, dr, gscale.  bg = rho0 c0^2 dt^2 is used by the
    background-pressure formulation only."""
    if isinstance(tv_mode, str):
        tv_mode = TV_MODES[tv_mode]
    pos, mass, rho, h, box = map(_f64, (pos, mass, rho, h, box))
    dim, n = pos.shape
    start, lst = nbr
    out = {k: np.zeros((dim, n)) for k in ("g", "dr")}
    out.update({k: np.zeros(n) for k in ("s", "beta", "gscale")})
    lib().oracle_tv(dim, n, _p(pos), _p(mass), _p(rho), _p(h), _p(box), _p(start), _p(lst),
                    float(h_min), float(xi), float(lim_c), float(lim_s0), int(tv_mode),
                    float(bg), _p(out["g"]),
                    _p(out["s"]), _p(out["beta"]), _p(out["dr"]), _p(out["gscale"]))
    return out


def wall_bc(pos, vel, rho, h, box, nbr, n_wall, wall_vel, rho0, c0):
    """Wall particles (the last n_wall) from their fluid neighbours: returns
    (rho, vel) with the wall entries replaced (Shepard-averaged pressure
    through the inverted EOS, no-slip mirror velocity); fluid entries copied."""
    pos, vel, rho, h, box, wall_vel = map(_f64, (pos, vel, rho, h, box, wall_vel))
    dim, n = pos.shape
    start, lst = nbr
    rho = rho.copy()
    vel = vel.copy()
    lib().oracle_wall_bc(dim, n, int(n_wall), _p(pos), _p(h), _p(box), _p(start), _p(lst),
                         float(rho0), float(c0), _p(wall_vel), _p(rho), _p(vel))
    return rho, vel


def forces(pos, vel, mass, rho, h, box, nbr, rho0, c0, eta, riemann_eta=3.0):
    """Returns (acc (D, N), ascale (N,))."""
    pos, vel, mass, rho, h, box = map(_f64, (pos, vel, mass, rho, h, box))
    dim, n = pos.shape
    start, lst = nbr
    acc = np.zeros((dim, n))
    ascale = np.zeros(n)
    lib().oracle_forces(dim, n, _p(pos), _p(vel), _p(mass), _p(rho), _p(h), _p(box),
                        _p(start), _p(lst), float(rho0), float(c0), float(eta),
                        float(riemann_eta), _p(acc), _p(ascale))
    return acc, ascale


def dt_advection(vmax, h_min, q: DualParams) -> float:
    """Eq. 9-10: CFL_ad h_min / max(|v|_max, max(nu / h_min, U_ref))."""
    return float(lib().oracle_dt_advection(float(vmax), float(h_min), ctypes.byref(q)))


def dt_acoustic(vmax, h_min, c0, q: DualParams) -> float:
    """Eq. 11: CFL_ac h_min / (|v|_max + c0)."""
    return float(lib().oracle_dt_acoustic(float(vmax), float(h_min), float(c0), ctypes.byref(q)))


def continuity(pos, vel, mass, rho, h, box, nbr, rho0, c0):
    """drho/dt of Eq. 3a with the U* of Eq. 5 at the given state."""
    pos, vel, mass, rho, h, box = map(_f64, (pos, vel, mass, rho, h, box))
    dim, n = pos.shape
    start, lst = nbr
    out = np.zeros(n)
    lib().oracle_continuity(dim, n, _p(pos), _p(vel), _p(mass), _p(rho), _p(h), _p(box),
                            _p(start), _p(lst), float(rho0), float(c0), _p(out))
    return out


class State:
    """FP64 particle state (absolute positions) advanced by the C oracle."""

    def __init__(self, case, pos=None, vel=None, rho=None, acc=None, prm: Params | None = None,
                 **pkw):
        self.dim = case.dim
        self.pos = _f64(case.pos if pos is None else pos).copy()
        self.vel = _f64(case.vel if vel is None else vel).copy()
        self.mass = _f64(case.mass).copy()
        self.h = _f64(case.h).copy()
        self.box = _f64(case.box).copy()
        self.n = self.pos.shape[1]
        self.prm = prm if prm is not None else params(case, **pkw)
        self.step_index = 0
        if rho is None or acc is None:
            self.rho = np.zeros(self.n)
            self.acc = np.zeros((self.dim, self.n))
            lib().oracle_init(self.dim, self.n, _p(self.pos), _p(self.vel), _p(self.mass),
                              _p(self.h), _p(self.box), ctypes.byref(self.prm), _p(self.rho),
                              _p(self.acc))
        else:
            self.rho = _f64(rho).copy()
            self.acc = _f64(acc).copy()

    def step(self, want=False):
        """One KDK step.  With want=True returns the correction at step n
        (dr, beta, s, g) and the diagnostics of the new state."""
        d, n = self.dim, self.n
        dr = np.zeros((d, n)) if want else None
        beta = np.zeros(n) if want else None
        s = np.zeros(n) if want else None
        g = np.zeros((d, n)) if want else None
        diag = np.zeros(NDIAG)
        lib().oracle_kdk_step(d, n, _p(self.pos), _p(self.vel), _p(self.acc), _p(self.rho),
                              _p(self.mass), _p(self.h), _p(self.box), ctypes.byref(self.prm),
                              self.step_index, _p(dr), _p(beta), _p(s), _p(g), _p(diag))
        self.step_index += 1
        out = dict(zip(DIAG_NAMES, diag))
        if want:
            out.update(dr=dr, beta=beta, s=s, g=g)
        return out

    def run(self, nsteps: int):
        """nsteps steps; returns the (nsteps, 9) diagnostics array."""
        diag = np.zeros((nsteps, NDIAG))
        lib().oracle_run(self.dim, self.n, _p(self.pos), _p(self.vel), _p(self.acc),
                         _p(self.rho), _p(self.mass), _p(self.h), _p(self.box),
                         ctypes.byref(self.prm), self.step_index, nsteps, _p(diag))
        self.step_index += nsteps
        return diag

    def dual_step(self, q: DualParams, want: bool = False):
        """One advection step of the dual-criteria scheme (density by
        summation, viscous force and correction at the step's start, acoustic
        substeps with the continuity equation).  Returns dict: dt_ad,
        substeps, t (time advanced), dt_sub (substep sizes), the diagnostics
        of the new state, and with want=True the correction (dr, beta, s)."""
        d, n = self.dim, self.n
        cap = q.max_substeps if q.max_substeps > 0 else 64
        info = np.zeros(3)
        dt_sub = np.zeros(cap)
        dr = np.zeros((d, n)) if want else None
        beta = np.zeros(n) if want else None
        s = np.zeros(n) if want else None
        diag = np.zeros(NDIAG)
        nsub = lib().oracle_dual_step(d, n, _p(self.pos), _p(self.vel), _p(self.rho),
                                      _p(self.mass), _p(self.h), _p(self.box),
                                      ctypes.byref(self.prm), ctypes.byref(q), _p(info),
                                      _p(dt_sub), _p(dr), _p(beta), _p(s), _p(diag))
        self.step_index += 1
        out = dict(zip(DIAG_NAMES, diag))
        out.update(dt_ad=info[0], substeps=int(nsub), t=info[2], dt_sub=dt_sub[:min(nsub, cap)])
        if want:
            out.update(dr=dr, beta=beta, s=s)
        return out

    def kinetic_energy(self) -> float:
        return float(0.5 * np.sum(self.mass * np.sum(self.vel * self.vel, axis=0)))
