"""Pins of the oracle's wall particles (the lid-driven cavity of Sec. 4.2;
the wall treatment is a reading, stated in oracle/sph_oracle.c): the wall
state reproduces constant fields and mirrors velocity about the wall value,
a resting fluid next to walls feels no force, the fluid never reaches across
the periodic seam, and plane Couette start-up follows the series solution of
the diffusion equation and settles on the exact linear profile."""
import numpy as np
import pytest

import cases
import oracle


def _brute_pairs(pos, h, box):
    """Pairs within 2h by minimum image, and whether the direct (unwrapped)
    distance is the minimum one; plain NumPy, independent of the oracle."""
    d = pos[:, :, None] - pos[:, None, :]
    b = np.asarray(box, dtype=np.float64).reshape(-1, 1, 1)
    wrapped = d - b * np.round(d / b)
    r = np.sqrt(np.sum(wrapped ** 2, axis=0))
    near = (r < 2.0 * h[:, None]) & ~np.eye(pos.shape[1], dtype=bool)
    direct = np.all(np.abs(wrapped - d) < 1e-12, axis=0)
    return near, direct


@pytest.mark.parametrize("make", [lambda: cases.lid_driven_cavity(12),
                                  lambda: cases.lid_driven_cavity(6, dim=3),
                                  lambda: cases.couette_2d(16)])
def test_fluid_never_reaches_across_the_seam(make):
    case = make()
    near, direct = _brute_pairs(case.pos, case.h, case.box)
    nf = case.n_fluid
    fluid_pairs = near[:nf, :]
    assert fluid_pairs.any()
    if case.extra.get("side") is not None:          # cavity: walls on all sides
        assert np.all(direct[:nf, :][fluid_pairs])
    else:                                           # Couette: periodic in x only
        ydirect = np.abs((case.pos[1][:nf, None] - case.pos[1][None, :])) < 0.5 * case.box[1]
        assert np.all(ydirect[fluid_pairs])


def _cavity_with(rho_f, vel_f, u_lid=0.7, dim=2):
    case = cases.lid_driven_cavity(12 if dim == 2 else 6, u_lid=u_lid, dim=dim)
    nf = case.n_fluid
    rho = np.full(case.n, case.rho0)
    rho[:nf] = rho_f
    vel = case.vel.copy()
    vel[:, :nf] = np.asarray(vel_f).reshape(dim, -1)
    return case, rho, vel


@pytest.mark.parametrize("dim", [2, 3])
def test_wall_state_reproduces_constant_fields(dim):
    """Uniform fluid pressure and velocity: every wall particle with fluid
    neighbours gets the fluid's density and 2 u_w - u; the others get rho0 and
    u_w (their own prescribed velocity)."""
    u = [[0.3], [-0.2], [0.1]][:dim]
    case, rho, vel = _cavity_with(1.013, u, dim=dim)
    nb = oracle.neighbors(case.pos, case.h, case.box)
    rho2, vel2 = oracle.wall_bc(case.pos, vel, rho, case.h, case.box, nb, case.n_wall,
                                case.wall_vel, case.rho0, case.c0)
    nf = case.n_fluid
    near, _ = _brute_pairs(case.pos, case.h, case.box)
    has_fluid = near[nf:, :nf].any(axis=1)
    assert has_fluid.any() and (~has_fluid).any()
    uw = case.wall_vel
    assert np.allclose(rho2[nf:][has_fluid], 1.013, rtol=0, atol=1e-14)
    assert np.allclose(vel2[:, nf:][:, has_fluid],
                       2 * uw[:, has_fluid] - np.array(u), rtol=0, atol=1e-14)
    assert np.all(rho2[nf:][~has_fluid] == case.rho0)
    assert np.array_equal(vel2[:, nf:][:, ~has_fluid], uw[:, ~has_fluid])
    # fluid entries untouched
    assert np.array_equal(rho2[:nf], rho[:nf]) and np.array_equal(vel2[:, :nf], vel[:, :nf])
    # the lid moves (top wall, corner blocks included); the rest is at rest
    top = case.pos[1][nf:] > case.extra["origin"] + 1.0
    assert np.all(uw[0, top] == 0.7) and np.all(uw[0, ~top] == 0.0) and np.all(uw[1:] == 0.0)


def test_wall_state_averages_with_kernel_weights():
    """A fluid pressure linear in y: a wall particle's pressure is the
    kernel-weighted mean, i.e. the field's value at the weighted mean height of
    its fluid neighbours (Shepard averages reproduce linear fields at their
    centroid), which lies inside the fluid."""
    case = cases.lid_driven_cavity(12)
    nf = case.n_fluid
    y = case.pos[1]
    rho = np.full(case.n, case.rho0)
    rho[:nf] = case.rho0 + 1e-3 * y[:nf]
    nb = oracle.neighbors(case.pos, case.h, case.box)
    rho2, _ = oracle.wall_bc(case.pos, case.vel, rho, case.h, case.box, nb, case.n_wall,
                             case.wall_vel, case.rho0, case.c0)
    start, lst = nb
    for a in range(nf, case.n, 7):
        js = lst[start[a]:start[a + 1]]
        js = js[js < nf]
        if js.size == 0:
            continue
        r = np.hypot(*(case.pos[:, js] - case.pos[:, [a]]))
        w = np.array([oracle.kernel_w(2, x, case.h[a]) for x in r])
        ybar = np.sum(w * y[js]) / np.sum(w)
        assert abs((rho2[a] - case.rho0) - 1e-3 * ybar) < 1e-15
        assert y[js].min() <= ybar <= y[js].max()


@pytest.mark.parametrize("dim", [2, 3])
def test_resting_fluid_between_walls_feels_no_force(dim):
    """Fluid at rest with uniform density 1.01 rho0 and walls at rest: the
    walls take the fluid's pressure, every fluid particle's support holds a
    complete lattice, and the pressure forces cancel to rounding."""
    case = cases.lid_driven_cavity(12 if dim == 2 else 6, dim=dim)
    case.wall_vel = np.zeros_like(case.wall_vel)
    nf = case.n_fluid
    rho = np.full(case.n, 1.01)
    vel = np.zeros_like(case.vel)
    nb = oracle.neighbors(case.pos, case.h, case.box)
    rho2, vel2 = oracle.wall_bc(case.pos, vel, rho, case.h, case.box, nb, case.n_wall,
                                case.wall_vel, case.rho0, case.c0)
    acc, scale = oracle.forces(case.pos, vel2, case.mass, rho2, case.h, case.box, nb,
                               case.rho0, case.c0, case.eta, case.riemann_eta)
    assert scale[:nf].min() > 0
    assert np.max(np.abs(acc[:, :nf]) / scale[:nf]) < 1e-13


def _couette_series(y, t, nu, u=1.0, height=1.0, terms=4000):
    """u(y, t) for a plate at y = H started impulsively at speed U over a
    fluid at rest between it and a fixed plate at y = 0 (separation of
    variables): U y / H + sum_k 2 U (-1)^k / (k pi) sin(k pi y / H) e^{-k^2 pi^2 nu t / H^2}."""
    k = np.arange(1, terms + 1)[:, None]
    return u * y / height + np.sum(2 * u * (-1.0) ** k / (k * np.pi)
                                   * np.sin(k * np.pi * y / height)
                                   * np.exp(-(k * np.pi) ** 2 * nu * t / height ** 2), axis=0)


def test_couette_series_solution_is_right():
    """The reference itself: at t = 0+ it vanishes inside, at late times it is
    linear, and it satisfies u_t = nu u_yy (finite differences)."""
    y = np.linspace(0.05, 0.95, 19)
    assert np.max(np.abs(_couette_series(y, 1e-7, 0.1))) < 2e-3
    assert np.max(np.abs(_couette_series(y, 50.0, 0.1) - y)) < 1e-12
    t, dt, dy, nu = 0.2, 1e-5, 1e-3, 0.1
    ut = (_couette_series(y, t + dt, nu) - _couette_series(y, t - dt, nu)) / (2 * dt)
    uyy = (_couette_series(y + dy, t, nu) - 2 * _couette_series(y, t, nu)
           + _couette_series(y - dy, t, nu)) / dy ** 2
    assert np.max(np.abs(ut - nu * uyy)) < 1e-4


def test_couette_startup_matches_series_and_settles_linear():
    """Re = 10 Couette start-up (20 particles across, lid speed U): the fluid
    velocity follows the series solution within 1% U during the transient (the
    weakly compressible fluid, c0 = 10 U, carries acoustic ripples of a few
    1e-3 U) and, at t = 8, every row's mean lies within 2e-3 U of the exact
    linear profile; the vertical velocity stays small."""
    case = cases.couette_2d(20, re=10.0)
    st = oracle.State(case)
    nf = case.n_fluid
    for t_end in (0.1, 0.5):
        st.run(int(round(t_end / case.dt)) - st.step_index)
        t = st.step_index * case.dt
        y = st.pos[1, :nf] - case.extra["origin"]
        err = np.abs(st.vel[0, :nf] - _couette_series(y, t, case.nu))
        assert err.max() < 1e-2, (t, err.max())
    st.run(int(round(8.0 / case.dt)) - st.step_index)
    y = st.pos[1, :nf] - case.extra["origin"]
    rows = np.floor(y * 20).astype(int)
    for r in range(20):
        sel = rows == r
        assert sel.sum() == 10
        assert abs(st.vel[0, :nf][sel].mean() - (r + 0.5) / 20) < 2e-3, r
    assert np.abs(st.vel[1, :nf]).max() < 1e-2
    # walls never move; the diagnostics count the fluid only
    assert np.array_equal(st.pos[:, nf:], case.pos[:, nf:])
    ke = 0.5 * np.sum(case.mass[:nf] * np.sum(st.vel[:, :nf] ** 2, axis=0))
    d = st.run(1)
    assert abs(d[0, 0] - 0.5 * np.sum(case.mass[:nf] * np.sum(st.vel[:, :nf] ** 2, axis=0))) \
        < 1e-12 * ke

