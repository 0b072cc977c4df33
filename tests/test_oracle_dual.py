"""Pins of the oracle's dual-criteria time stepping (Sec. 2.4, Eq. 3a, 5,
9-11; CPU).

The continuity equation with the Riemann velocity U* of Eq. 5 is checked
against closed forms (a linear velocity field on a lattice, a two-particle
pressure jump, a two-particle compression, Galilean invariance); the
advection step against what it must do to states whose evolution is known
(a lattice at rest stays put, a lattice in uniform translation moves by
V dt_ad), with the acoustic substeps of Eq. 11 covering the advection step
of Eq. 9-10 exactly; and momentum is conserved.
"""
import math

import numpy as np
import pytest

import cases
import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _second_moment(c, nb, i0):
    """M = -sum_j V_j F_ij r_ij r_ij^T over particle i0's neighbours (V = m / rho0)."""
    start, lst = nb
    M = np.zeros((c.dim, c.dim))
    for j in lst[start[i0]:start[i0 + 1]]:
        r = c.pos[:, i0] - c.pos[:, j]
        M -= c.mass[j] * oracle.kernel_f(c.dim, np.linalg.norm(r), c.h[0]) * np.outer(r, r)
    return M


def test_continuity_of_a_linear_velocity_field():
    """Eq. 3a at uniform density with v = A r: the pressure term of U*
    vanishes and drho_i/dt = -rho_i tr(A M) exactly, M the lattice's discrete
    second moment (M = I within 3% at h = 1.3 dx), the SPH form of
    drho/dt = -rho div v (Eq. 1).  Interior particles (the field is not
    periodic)."""
    c = cases.taylor_green_2d(40)
    A = np.array([[0.3, -0.7], [0.2, -0.1]])
    vel = A @ c.pos
    rho = np.full(c.n, 1.3)
    nb = oracle.neighbors(c.pos, c.h, c.box)
    drho = oracle.continuity(c.pos, vel, c.mass, rho, c.h, c.box, nb, 1.0, 10.0)
    M = _second_moment(c, nb, 20 + 40 * 20)      # with V = m / rho0: M ~ I
    inner = np.all((c.pos > 3 * c.h[0]) & (c.pos < 1 - 3 * c.h[0]), axis=0)
    expect = -1.3 * np.trace(A @ (M / 1.3))      # V_j = m_j / rho_j
    assert np.max(np.abs(drho[inner] - expect)) < 1e-12 * abs(expect)
    assert abs(np.trace(A @ M) / np.trace(A) - 1.0) < 0.03


def _pair(rho_i, rho_j, u_i=0.0, u_j=0.0, sep=0.02, c0=10.0):
    pos = np.array([[0.5, 0.5 + sep], [0.5, 0.5]])
    vel = np.array([[u_i, u_j], [0.0, 0.0]])
    h = np.full(2, 0.013)
    m = np.full(2, 1e-4)
    rho = np.array([rho_i, rho_j])
    nb = oracle.neighbors(pos, h, np.ones(2), method="brute")
    return oracle.continuity(pos, vel, m, rho, h, np.ones(2), nb, 1.0, c0), m, h, sep


def _dwdr(r, h):
    e = 1e-7 * h
    return (oracle.kernel_w(2, r + e, h) - oracle.kernel_w(2, r - e, h)) / (2 * e)


def test_continuity_pressure_jump_of_a_pair_at_rest():
    """Eq. 5 with U_l = U_r = 0: U* = (p_i - p_j) / (2 rhobar c0), so
    drho_i/dt = rho_i V_j (p_i - p_j) / (rhobar c0) dW/dr: mass flows from high
    to low pressure (the higher density falls, the lower rises)."""
    c0 = 10.0
    drho, m, h, r = _pair(1.02, 0.99, c0=c0)
    p = c0 ** 2 * (np.array([1.02, 0.99]) - 1.0)
    rhobar = 0.5 * (1.02 + 0.99)
    w1 = _dwdr(r, h[0])
    expect = np.array([1.02 * m[1] / 0.99 * (p[0] - p[1]) / (rhobar * c0) * w1,
                       0.99 * m[0] / 1.02 * (p[1] - p[0]) / (rhobar * c0) * w1])
    assert np.allclose(drho, expect, rtol=1e-7, atol=0.0)
    assert drho[0] < 0.0 < drho[1]


def test_continuity_compression_of_an_approaching_pair():
    """Eq. 3a with equal pressures: U* is the mean normal velocity, and
    drho_i/dt = 2 rho_i V_j (U* - U_l) dW/dr = rho_i V_j (U_r - U_l) dW/dr > 0
    for particles approaching each other; separating pairs expand."""
    drho, m, h, r = _pair(1.0, 1.0, u_i=0.3, u_j=-0.2)
    du = 0.3 - (-0.2)                    # U_l - U_r along the axis from i to j
    expect = 1.0 * m[1] / 1.0 * (-du) * _dwdr(r, h[0])
    assert np.allclose(drho, [expect, expect], rtol=1e-7, atol=0.0)
    assert expect > 0.0
    apart, _, _, _ = _pair(1.0, 1.0, u_i=-0.3, u_j=0.2)
    assert np.all(apart < 0.0)


def test_continuity_is_galilean_invariant():
    """Only velocity differences enter Eq. 3a: a uniform velocity added to a
    disordered, non-uniform state leaves drho/dt unchanged."""
    c = cases.taylor_green_2d(16, jitter=0.2, seed=61)
    rng = np.random.default_rng(62)
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, c.n)
    nb = oracle.neighbors(c.pos, c.h, c.box)
    a = oracle.continuity(c.pos, c.vel, c.mass, rho, c.h, c.box, nb, 1.0, 10.0)
    b = oracle.continuity(c.pos, c.vel + np.array([[0.7], [-0.4]]), c.mass, rho, c.h, c.box,
                          nb, 1.0, 10.0)
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(a))
    assert np.max(np.abs(a)) > 0.0


@pytest.mark.parametrize("regime", ["u_ref", "viscous"])
def test_lattice_at_rest_stays_put(regime):
    """Eq. 9-11 on a lattice at rest: |v|_max = 0, so dt_ad = CFL_ad h /
    max(nu / h, U_ref) and every acoustic substep is CFL_ac h / c0 except a
    shorter last one; the substeps cover dt_ad exactly, nothing moves, and the
    density stays rho0."""
    c = cases.taylor_green_2d(20)
    if regime == "viscous":
        c.eta = 0.5                      # nu / h = 19 > U_ref = 1
    vad = max(c.eta / c.rho0 / c.h_min, c.u_ref)
    c.vel = np.zeros_like(c.pos)
    st = oracle.State(c)
    pos0 = st.pos.copy()
    d = st.dual_step(oracle.dual_params(c))
    dt_ad = 0.25 * c.h_min / vad
    dt_ac = 0.6 * c.h_min / c.c0
    assert abs(d["dt_ad"] / dt_ad - 1.0) < 1e-15
    k = math.ceil(dt_ad / dt_ac)
    assert d["substeps"] == k
    assert np.all(np.abs(d["dt_sub"][:-1] / dt_ac - 1.0) < 1e-15)
    assert 0.0 < d["dt_sub"][-1] <= dt_ac
    assert abs(d["t"] / dt_ad - 1.0) < 1e-14
    # (the lattice sum equals rho0 to rounding, so forces are rounding-sized)
    assert np.max(np.abs(st.pos - pos0)) < 1e-12 * c.dx
    assert np.max(np.abs(st.rho - c.rho0)) < 1e-13 and np.max(np.abs(st.vel)) < 1e-10


def test_lattice_in_uniform_translation():
    """A lattice moving at V > U_ref: no pressure, viscous or correction
    term (uniform density and velocity, g = 0), so one advection step moves
    every particle by V dt_ad with dt_ad = CFL_ad h / V (Eq. 9-10) and
    substeps CFL_ac h / (V + c0) (Eq. 11)."""
    c = cases.taylor_green_2d(20)
    V = np.array([3.0, -1.5])
    c.vel = np.tile(V[:, None], (1, c.n))
    vmax = float(np.linalg.norm(V))
    st = oracle.State(c)
    pos0 = st.pos.copy()
    d = st.dual_step(oracle.dual_params(c))
    dt_ad = 0.25 * c.h_min / vmax
    assert abs(d["dt_ad"] / dt_ad - 1.0) < 1e-15
    dt_ac = 0.6 * c.h_min / (vmax + c.c0)
    assert d["substeps"] == math.ceil(dt_ad / dt_ac)
    assert np.all(np.abs(d["dt_sub"][:-1] / dt_ac - 1.0) < 1e-13)
    moved = st.pos - pos0
    moved -= np.round(moved)
    assert np.max(np.abs(moved - V[:, None] * dt_ad)) < 1e-14
    assert np.max(np.abs(st.vel - V[:, None])) < 1e-12


def test_dual_step_conserves_momentum_and_caps_substeps():
    """Pressure (Eq. 3b, 5-6) and viscous (Eq. 7) pair terms on the frozen
    geometry are antisymmetric, so sum m v is conserved through the substeps
    of a disordered state; a substep cap ends the advection step early, with
    the same first substeps."""
    c = cases.taylor_green_2d(16, jitter=0.2, seed=63)
    a = oracle.State(c)
    p0 = np.sum(c.mass * a.vel, axis=1)
    for _ in range(3):
        d = a.dual_step(oracle.dual_params(c))
    assert np.max(np.abs(np.sum(c.mass * a.vel, axis=1) - p0)) < 1e-15
    full = oracle.State(c).dual_step(oracle.dual_params(c))
    capped = oracle.State(c).dual_step(oracle.dual_params(c, max_substeps=2))
    assert capped["substeps"] == 2 < full["substeps"]
    assert np.array_equal(capped["dt_sub"], full["dt_sub"][:2])
    assert capped["t"] < full["t"]


def test_standing_acoustic_wave_frequency():
    """The acoustic substeps integrate Eq. 2, 3a-3b as a wave equation: a
    standing wave v_x = eps c0 sin(k x) on a lattice (no viscosity, Riemann
    dissipation or correction) oscillates at omega = c0 k M_xx, M the discrete
    second moment that both the continuity and the pressure sum carry (each
    within the kernel's O((k h)^2) smoothing: 4% here), with little damping
    (the pressure jump of U* diffuses density slowly)."""
    from scipy.optimize import curve_fit
    n = 40
    c = cases.taylor_green_2d(n)
    c.eta, c.riemann_eta = 0.0, 0.0
    k, eps = 2 * math.pi, 0.01
    x = c.pos[0]
    c.vel = np.stack([eps * c.c0 * np.sin(k * x), np.zeros(c.n)])
    st = oracle.State(c, xi=0.0)
    q = oracle.dual_params(c)
    ts, amp = [0.0], [eps * c.c0]
    while ts[-1] < 0.2:
        d = st.dual_step(q)
        ts.append(ts[-1] + d["t"])
        amp.append(2 * np.mean(st.vel[0] * np.sin(k * x)))
    ts, amp = np.array(ts), np.array(amp)

    def wave(t, a, w, g):
        return a * np.cos(w * t) * np.exp(-g * t)

    (a, w, g), _ = curve_fit(wave, ts, amp, p0=[amp[0], 60.0, 1.0])
    nb = oracle.neighbors(c.pos, c.h, c.box)
    M = _second_moment(c, nb, 20 + n * 20)
    assert np.max(np.abs(wave(ts, a, w, g) - amp)) < 0.01 * amp[0]
    assert abs(w / (c.c0 * k * M[0, 0]) - 1.0) < 0.04
    assert 0.0 <= g < 2.0


def test_correction_moves_particles_once_per_advection_step():
    """Sec. 3: in the dual-criteria scheme the correction of Eq. (16) is
    applied once per advection step, at the step's start, with the density
    just reinitialised by summation.  With v = 0, no viscosity and a sound
    speed too small for pressure to move anything, one advection step moves
    each particle by exactly that correction (expected values from central
    differences of the density sum, Eq. 8)."""
    c = cases.taylor_green_2d(16, jitter=0.05, seed=64)
    c.eta = 0.0
    c.c0 = 1e-100
    c.vel = np.zeros_like(c.pos)
    st = oracle.State(c)
    pos0 = st.pos.copy()
    nb = oracle.neighbors(pos0, c.h, c.box)
    rho = oracle.density(pos0, c.mass, c.h, c.box, nb, oracle.lattice_kappa(2))
    st.dual_step(oracle.dual_params(c))
    moved = st.pos - pos0
    moved -= np.round(moved)
    kappa = oracle.lattice_kappa(2)
    tv = oracle.tv(pos0, c.mass, rho, c.h, c.box, nb, c.h_min)
    for i in (5, 77, 130, 201):
        g = np.zeros(2)
        for kk in range(2):
            e = 1e-6 * c.dx
            vals = []
            for sgn in (1, -1):
                p = pos0.copy()
                p[kk, i] += sgn * e
                nbp = oracle.neighbors(p, c.h, c.box)
                vals.append(oracle.density(p, c.mass / rho, c.h, c.box, nbp, kappa)[i])
            g[kk] = (vals[0] - vals[1]) / (2 * e) * kappa
        s = c.h_min ** 2 * float(g @ g)
        beta = min(1e3 * s, 1.0) if s > 5e-4 else 0.0
        assert beta == tv["beta"][i]          # away from the limiter threshold
        expect = -0.2 * beta * c.h_min ** 2 * g
        assert np.all(np.abs(moved[:, i] - expect) <= 1e-6 * 0.2 * c.h_min ** 2
                      * tv["gscale"][i] + 1e-15 * c.dx), i


def test_viscous_decay_of_a_shear_wave():
    """Eq. 7 held over each advection step: a slow shear wave
    u = U sin(2 pi y) on a lattice decays like exp(-nu k^2 t) (the viscous
    operator gives nu d2u/dy2 up to the discrete second moment, within 5%)."""
    n = 40
    c = cases.taylor_green_2d(n)
    U, k = 1e-3, 2 * math.pi
    y = c.pos[1]
    c.vel = np.stack([U * np.sin(k * y), np.zeros(c.n)])
    st = oracle.State(c, xi=0.0)
    q = oracle.dual_params(c)
    t = 0.0
    for _ in range(4):
        t += st.dual_step(q)["t"]
    amp = 2 * np.mean(st.vel[0] * np.sin(k * y))
    rate = -math.log(amp / U) / t
    assert abs(rate / (c.eta / c.rho0 * k * k) - 1.0) < 0.05
