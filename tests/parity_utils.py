"""Helpers for comparing the GPU path with the FP64 oracle on identical inputs.

The GPU state (cell index + cell-local offset in FP32 or FP64) is widened
exactly to FP64 absolute positions; the oracle then evaluates the same
particles.  Tolerances (stated per field, max-norm):

* positions: minimum-image difference / dx
* velocities: / U_ref
* density: / rho0
* sweep outputs with identical inputs (g, dr, a): / the particle's own sum of
  absolute pair terms (the summation-error scale of the sweep)
* accelerations after a whole step: / the particle's sum of absolute pair
  terms, with the oracle's forces evaluated at the GPU's own state after the
  step (step_acc_error), so the EOS does not amplify the density's rounding
* FP32: 1e-5, FP64: 1e-12.
"""
from __future__ import annotations

import copy

import numpy as np

import oracle

TOL = {"f32": 1e-5, "f64": 1e-12}
EPS = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}


def case_with(case, mass=None, h=None):
    c = copy.copy(case)
    if mass is not None:
        c.mass = np.asarray(mass, dtype=np.float64)
    if h is not None:
        c.h = np.asarray(h, dtype=np.float64)
    return c


def gpu_inputs(sim, case):
    """FP64 view of the GPU state in id order, plus mass/h as the GPU holds them."""
    st = sim.export()
    n = case.n
    T = np.float32 if sim.dtype == "f32" else np.float64
    if "mass" in st:
        mass, h = st["mass"], st["h"]
    else:
        mass = np.full(n, float(T(case.mass[0])))
        h = np.full(n, float(T(case.h_min)))
    return st, mass, h


def cutoff_band(pos, h, box, dtype, nb):
    """Particles with a pair whose distance lies within a few FP ulps of the
    support radius 2 h_ij (their neighbour count may legitimately differ)."""
    start, lst = nb
    i = np.repeat(np.arange(pos.shape[1]), np.diff(start))
    j = lst.astype(np.int64)
    d = pos[:, i] - pos[:, j]
    b = np.asarray(box, dtype=np.float64).reshape(-1, 1)
    d -= b * np.round(d / b)
    r = np.sqrt(np.sum(d * d, axis=0))
    sup = h[i] + h[j]
    close = np.abs(r - sup) <= 16 * EPS[dtype] * sup
    flag = np.zeros(pos.shape[1], dtype=bool)
    flag[i[close]] = True
    flag[j[close]] = True
    return flag


def widen(nb, mask, hops=1):
    """Extend a particle mask to neighbours, `hops` times."""
    start, lst = nb
    m = mask.copy()
    for _ in range(hops):
        i = np.repeat(np.arange(len(m)), np.diff(start))
        hit = m[lst]
        m2 = m.copy()
        np.logical_or.at(m2, i[hit], True)
        m = m2
    return m


def limiter_band(s, g, gscale, h_min, s0, dtype):
    """Particles whose FP64 oracle s is close enough to the threshold s0 that
    the sweep's rounding may put them on the other branch of Eq. 15:
    |s - s0| <= 2 h^2 |g| (64 eps sum|terms|) (plus a relative 1e-9 floor)."""
    gnorm = np.sqrt(np.sum(g * g, axis=0))
    ds = 2.0 * h_min * h_min * gnorm * 64.0 * EPS[dtype] * gscale
    return np.abs(s - s0) <= ds + 1e-9 * s0


def min_image(a, b, box):
    d = a - b
    bx = np.asarray(box, dtype=np.float64).reshape(-1, 1)
    return d - bx * np.round(d / bx)


def step_acc_error(out, case, mass, h, mask=None):
    """Acceleration error of a GPU step on the summation-error scale: the
    oracle's forces (Eq. 2-7) evaluated at the GPU's own state after the step
    (positions, the density rho^{n+1} and, for the fluid, the half-step
    velocity v' = v^{n+1} - dt/2 a^{n+1}; walls keep their state velocity),
    against the GPU's a^{n+1}, per particle / sum_j |pair term|.  Evaluating
    at the GPU's density keeps the EOS from amplifying the density's own
    rounding (c0^2 delta rho) into the comparison.  Fluid particles only."""
    nf = case.n - getattr(case, "n_wall", 0)
    vhalf = out["vel"].copy()
    vhalf[:, :nf] -= 0.5 * case.dt * out["acc"][:, :nf]
    nb = oracle.neighbors(out["pos"], h, case.box)
    acc, scale = oracle.forces(out["pos"], vhalf, mass, out["rho"], h, case.box, nb,
                               case.rho0, case.c0, case.eta, case.riemann_eta)
    err = np.abs(out["acc"][:, :nf] - acc[:, :nf]) / scale[:nf]
    if mask is not None:
        err = err[:, mask[:nf]]
    return float(err.max()) if err.size else 0.0
