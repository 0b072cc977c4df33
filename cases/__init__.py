"""Seeded synthetic particle sets for the transport-velocity WCSPH step.

This module only lays out inputs: lattices, seeded jitter, the prescribed
initial velocity fields and the run parameters.  It holds none of the SPH
arithmetic (no kernel, no sum over neighbours), so that both the FP64 CPU
oracle and the GPU library can be fed from it without sharing method code.

Conventions (shared by every case):

* positions are absolute FP64 coordinates in a periodic box [0, B)^D, stored
  structure-of-arrays as an array of shape (D, N);
* particle ids are 0..N-1 in lattice order, x fastest (id = i + n*j [+ n*n*k]);
* lattice points sit at cell centres, x = (i + 1/2) dx;
* jitter is uniform per component, drawn from ``numpy.random.default_rng(seed)``
  as an (N, D) array in id order;
* reference density rho0 = 1; particle mass m = rho0 * dp^D (the particle
  volume of the variable-resolution discussion in Sec. 2.4), smoothing length
  h = 1.3 dp (Sec. 4, first paragraph);
* the fixed time step is the smaller of the two criteria of Eq. (9)-(11) with
  the maximum speed replaced by the reference speed: the acoustic
  0.6 h_min / (U_ref + c0) and the advection 0.25 h_min / max(U_ref, nu / h_min),
  whose nu / h term bounds the explicit viscous step (it decides only in the
  low-speed variable-resolution box; every Taylor-Green case takes the
  acoustic step);
* c0 = 10 U_ref (Sec. 2.1, the artificial sound speed);
* the transport-velocity constants are those of Sec. 3: xi = -0.2 (Eq. 14/16),
  limiter C = 1e3 and threshold 5e-4 (Eq. 15); the Riemann dissipation limiter
  uses eta = 3 (Eq. 6).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Case", "lattice", "taylor_green_2d", "taylor_green_3d",
    "variable_resolution_2d", "lid_driven_cavity", "couette_2d", "make", "CONFIGS",
]

H_OVER_DP = 1.3          # Sec. 4: h = 1.3 dp
CFL_AC = 0.6             # Eq. (11) constant
CFL_AD = 0.25            # Eq. (9) constant
XI = -0.2                # Eq. (14) and (16)
LIMITER_C = 1.0e3        # Eq. (15)
LIMITER_S0 = 5.0e-4      # Eq. (15) threshold
RIEMANN_ETA = 3.0        # Eq. (6)


@dataclass
class Case:
    """One synthetic workload: particle arrays plus run parameters."""
    name: str
    dim: int
    pos: np.ndarray          # (D, N) float64 absolute positions in [0, box)
    vel: np.ndarray          # (D, N) float64
    mass: np.ndarray         # (N,) float64
    h: np.ndarray            # (N,) float64 per-particle smoothing length
    box: tuple               # (D,) periodic box edges
    dx: float                # nominal (finest) lattice spacing
    rho0: float = 1.0
    c0: float = 10.0
    eta: float = 0.01        # dynamic viscosity
    u_ref: float = 1.0
    dt: float = 0.0
    xi: float = XI
    lim_c: float = LIMITER_C
    lim_s0: float = LIMITER_S0
    riemann_eta: float = RIEMANN_ETA
    steps: int = 1
    uniform: bool = True     # uniform mass and h (scalars suffice)
    extra: dict = field(default_factory=dict)
    n_wall: int = 0          # the last n_wall ids are wall particles
    wall_vel: np.ndarray | None = None   # (D, n_wall) prescribed wall velocity

    @property
    def n_fluid(self) -> int:
        return self.n - self.n_wall

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @property
    def h_min(self) -> float:
        return float(self.h.min())

    @property
    def h_max(self) -> float:
        return float(self.h.max())

    @property
    def nu(self) -> float:
        return self.eta / self.rho0

    def ncell(self):
        """Cells per axis: floor(box / (2 h_max)), the largest grid whose cell
        edge is at least the kernel support radius 2 h_max."""
        return tuple(int(math.floor(b / (2.0 * self.h_max) * (1.0 - 1e-12)))
                     for b in self.box)


def lattice(dim: int, n: int, box: float = 1.0) -> np.ndarray:
    """Cell-centred lattice of n^dim points, shape (dim, n^dim), x fastest."""
    dx = box / n
    axis = (np.arange(n, dtype=np.float64) + 0.5) * dx
    grids = np.meshgrid(*([axis] * dim), indexing="ij")
    # indexing="ij" makes the first index slowest; reverse so x is fastest
    pts = [g.transpose(tuple(reversed(range(dim)))).reshape(-1) for g in grids]
    return np.stack(pts, axis=0)


def _jitter(pos: np.ndarray, amp: np.ndarray | float, seed: int, box) -> np.ndarray:
    d, n = pos.shape
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(n, d)).T      # id order, component inner
    out = pos + u * amp
    for k in range(d):
        out[k] = np.mod(out[k], box[k])
        out[k][out[k] >= box[k]] = 0.0
    return out


def _dt(h_min: float, u_ref: float, c0: float, nu: float) -> float:
    acoustic = CFL_AC * h_min / (u_ref + c0)
    advection = CFL_AD * h_min / max(u_ref, nu / h_min)
    return min(acoustic, advection)


def taylor_green_2d(n: int, jitter: float = 0.0, seed: int = 1, re: float = 100.0,
                    u: float = 1.0, vel_perturb: float = 0.0, steps: int = 100,
                    name: str | None = None) -> Case:
    """2-D periodic Taylor-Green vortex on the unit square (Sec. 4.1, Eq. 17 at
    t = 0): u = -U cos(2 pi x) sin(2 pi y), v = U sin(2 pi x) cos(2 pi y).

    ``jitter`` is the half-width of the uniform position noise in units of dx;
    ``vel_perturb`` multiplies each velocity component by (1 + vel_perturb * w),
    w ~ U(-1, 1), drawn after the jitter from a generator seeded with seed + 1000.
    """
    box = (1.0, 1.0)
    dx = 1.0 / n
    pos = lattice(2, n)
    if jitter > 0.0:
        pos = _jitter(pos, jitter * dx, seed, box)
    x, y = pos
    vel = np.stack([-u * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y),
                    u * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)])
    if vel_perturb > 0.0:
        rng = np.random.default_rng(seed + 1000)
        w = rng.uniform(-1.0, 1.0, size=(pos.shape[1], 2)).T
        vel = vel * (1.0 + vel_perturb * w)
    rho0 = 1.0
    c0 = 10.0 * u
    eta = rho0 * u * 1.0 / re
    h = np.full(n * n, H_OVER_DP * dx)
    mass = np.full(n * n, rho0 * dx * dx)
    return Case(name=name or f"tg2d_{n}", dim=2, pos=pos, vel=vel, mass=mass, h=h,
                box=box, dx=dx, rho0=rho0, c0=c0, eta=eta, u_ref=u,
                dt=_dt(H_OVER_DP * dx, u, c0, eta / rho0), steps=steps, uniform=True,
                extra={"re": re, "jitter": jitter, "seed": seed})


def taylor_green_3d(n: int, jitter: float = 0.05, seed: int = 1, nu: float = 0.01,
                    u: float = 1.0, steps: int = 200, name: str | None = None) -> Case:
    """3-D periodic Taylor-Green initial field on the unit cube:
    u = U sin2pi x cos2pi y cos2pi z, v = -U cos2pi x sin2pi y cos2pi z, w = 0."""
    box = (1.0, 1.0, 1.0)
    dx = 1.0 / n
    pos = lattice(3, n)
    if jitter > 0.0:
        pos = _jitter(pos, jitter * dx, seed, box)
    x, y, z = pos
    s2, c2 = np.sin, np.cos
    tp = 2 * np.pi
    vel = np.stack([u * s2(tp * x) * c2(tp * y) * c2(tp * z),
                    -u * c2(tp * x) * s2(tp * y) * c2(tp * z),
                    np.zeros_like(x)])
    rho0 = 1.0
    c0 = 10.0 * u
    h = np.full(n ** 3, H_OVER_DP * dx)
    mass = np.full(n ** 3, rho0 * dx ** 3)
    return Case(name=name or f"tg3d_{n}", dim=3, pos=pos, vel=vel, mass=mass, h=h,
                box=box, dx=dx, rho0=rho0, c0=c0, eta=rho0 * nu, u_ref=u,
                dt=_dt(H_OVER_DP * dx, u, c0, nu), steps=steps, uniform=True,
                extra={"jitter": jitter, "seed": seed})


def variable_resolution_2d(dp_min: float = 1.0 / 1306, jitter: float = 0.1, seed: int = 1,
                           u: float = 1.0e-3, nu: float = 1.0e-5, width: float = 0.05,
                           kmax: int = 4, steps: int = 500, name: str | None = None) -> Case:
    """2-D periodic box whose resolution varies smoothly 2:1 across x.

    h(x) = h_min (1.5 + 0.5 tanh((|x - 1/2| - 1/4) / width)), dp = h / 1.3:
    fine (h = h_min) around x = 1/2, coarse (h ~ 2 h_min) at the periodic seam.
    Columns are marched along x with the local spacing and rescaled to close the
    seam; column k holds n_k = round(1 / w_k) particles at y = (m + 1/2) / n_k.
    Each particle's volume is w_k / n_k, its mass rho0 * volume, its smoothing
    length 1.3 sqrt(volume).  Positions get +-jitter*dp uniform noise.  The
    velocity is divergence-free, u = d psi/dy, v = -d psi/dx, from a stream
    function of random Fourier modes with 1 <= |k| <= kmax, scaled so the
    largest particle speed is U (a low-velocity flow, the regime of Sec. 3).
    """
    h_min = H_OVER_DP * dp_min

    def dp_of(x):
        return h_min * (1.5 + 0.5 * math.tanh((abs(x - 0.5) - 0.25) / width)) / H_OVER_DP

    edges = [0.0]
    while edges[-1] < 1.0:
        e = edges[-1]
        edges.append(e + dp_of(e + 0.5 * dp_of(e)))
    # choose the column count whose end lies closest to 1, then rescale
    if abs(edges[-2] - 1.0) < abs(edges[-1] - 1.0):
        edges = edges[:-1]
    edges = np.asarray(edges) / edges[-1]
    widths = np.diff(edges)
    centres = 0.5 * (edges[:-1] + edges[1:])
    nrow = np.maximum(3, np.rint(1.0 / widths).astype(np.int64))
    xs, ys, vols = [], [], []
    for xc, wk, nk in zip(centres, widths, nrow):
        dy = 1.0 / nk
        ys.append((np.arange(nk, dtype=np.float64) + 0.5) * dy)
        xs.append(np.full(nk, xc))
        vols.append(np.full(nk, wk * dy))
    # order: column-major in x (columns are the slow index here); ids follow
    pos = np.stack([np.concatenate(xs), np.concatenate(ys)])
    vol = np.concatenate(vols)
    dp = np.sqrt(vol)
    box = (1.0, 1.0)
    if jitter > 0.0:
        pos = _jitter(pos, jitter * dp[None, :], seed, box)
    rng = np.random.default_rng(seed + 2000)
    modes = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
             if 0 < kx * kx + ky * ky <= kmax * kmax]
    amp = rng.normal(size=len(modes))
    phase = rng.uniform(0.0, 2 * np.pi, size=len(modes))
    x, y = pos
    uu = np.zeros_like(x)
    vv = np.zeros_like(x)
    for (kx, ky), a, ph in zip(modes, amp, phase):
        arg = 2 * np.pi * (kx * x + ky * y) + ph
        s = np.sin(arg)
        uu += -a * 2 * np.pi * ky * s
        vv += a * 2 * np.pi * kx * s
    scale = u / np.sqrt(uu * uu + vv * vv).max()
    vel = np.stack([uu * scale, vv * scale])
    rho0 = 1.0
    c0 = 10.0 * u
    h = H_OVER_DP * dp
    mass = rho0 * vol
    return Case(name=name or "varres2d", dim=2, pos=pos, vel=vel, mass=mass, h=h,
                box=box, dx=float(dp.min()), rho0=rho0, c0=c0, eta=rho0 * nu, u_ref=u,
                dt=_dt(float(h.min()), u, c0, nu), steps=steps, uniform=False,
                extra={"jitter": jitter, "seed": seed, "columns": len(widths)})


def _walled_box(nx: int, ny: int, layers: int, dx: float, wall_x: bool, nz: int = 0):
    """Fluid on the cell-centred lattice of [0, nx dx) x [0, ny dx) (x [0, nz dx)
    in 3-D), then `layers` rows of wall particles on the same lattice below and
    above it in y (and, with wall_x, `layers` columns left and right in x and,
    in 3-D, in front and behind in z; edges and corners included).  Returns
    (fluid positions, wall positions, wall-above-the-fluid mask) in wall-box
    coordinates: the periodic box starts `layers` spacings below / left of /
    in front of the fluid on every walled axis (x fastest, then y, then z)."""
    lx = layers if wall_x else 0
    ix = np.arange(-lx, nx + lx)
    iy = np.arange(-layers, ny + layers)
    if nz:
        iz = np.arange(-layers, nz + layers)
        gz, gy, gx = np.meshgrid(iz, iy, ix, indexing="ij")     # x fastest
        gx, gy, gz = gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)
        fluid = ((gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny) & (gz >= 0) & (gz < nz))
        pts = np.stack([(gx + lx + 0.5) * dx, (gy + layers + 0.5) * dx,
                        (gz + layers + 0.5) * dx])
    else:
        gx, gy = np.meshgrid(ix, iy, indexing="xy")            # x fastest
        gx, gy = gx.reshape(-1), gy.reshape(-1)
        fluid = (gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny)
        pts = np.stack([(gx + lx + 0.5) * dx, (gy + layers + 0.5) * dx])
    return pts[:, fluid], pts[:, ~fluid], gy[~fluid] >= ny


def lid_driven_cavity(n: int, re: float | None = None, u_lid: float = 1.0, layers: int = 3,
                      dim: int = 2, jitter: float = 0.0, seed: int = 1, steps: int = 1000,
                      name: str | None = None) -> Case:
    """Lid-driven cavity of side 1: 2-D (Sec. 4.2, Re = 1000 by default) or
    3-D (the cube of the three-dimensional cavity section, Re = 100 by
    default), Re = U L / nu.

    Fluid at rest on the n^D cell-centred lattice of the unit square / cube;
    wall particles continue the lattice `layers` spacings beyond every face
    (edges and corners included).  The top wall (every wall particle above
    the fluid in y, its edge and corner blocks included) moves at (u_lid, 0[,
    0]); the other walls are at rest.  Coordinates are shifted by layers*dp so
    the box [0, 1 + 2 layers dp)^D is the periodic box of the cell grid; with
    layers*dp >= 2h (layers >= 3 at h = 1.3 dp) no fluid particle has a
    neighbour across its seams.  Ids: the fluid first (x fastest), then the
    walls (x fastest).  ``jitter`` (in units of dp, at most 0.25) moves the
    fluid particles by seeded uniform noise; the walls stay on the lattice.
    """
    if layers * 1.0 < 2 * H_OVER_DP:
        raise ValueError("layers must cover the kernel support 2h")
    if dim not in (2, 3):
        raise ValueError("dim is 2 or 3")
    re = (1000.0 if dim == 2 else 100.0) if re is None else re
    dx = 1.0 / n
    fluid, wall, top = _walled_box(n, n, layers, dx, True, nz=n if dim == 3 else 0)
    if jitter > 0.0:
        if jitter > 0.25:
            raise ValueError("jitter above 0.25 dp could bring fluid onto the walls")
        rng = np.random.default_rng(seed)
        fluid = fluid + rng.uniform(-1.0, 1.0, size=(fluid.shape[1], dim)).T * jitter * dx
    pos = np.concatenate([fluid, wall], axis=1)
    nw = wall.shape[1]
    wall_vel = np.zeros((dim, nw))
    wall_vel[0, top] = u_lid
    vel = np.zeros_like(pos)
    vel[:, fluid.shape[1]:] = wall_vel
    rho0 = 1.0
    c0 = 10.0 * u_lid
    eta = rho0 * u_lid * 1.0 / re
    npart = pos.shape[1]
    edge = (n + 2 * layers) * dx
    return Case(name=name or f"cavity{dim}d_{n}", dim=dim, pos=pos, vel=vel,
                mass=np.full(npart, rho0 * dx ** dim), h=np.full(npart, H_OVER_DP * dx),
                box=(edge,) * dim, dx=dx, rho0=rho0, c0=c0, eta=eta, u_ref=u_lid,
                dt=_dt(H_OVER_DP * dx, u_lid, c0, eta / rho0), steps=steps, uniform=True,
                extra={"re": re, "layers": layers, "origin": layers * dx, "side": 1.0},
                n_wall=nw, wall_vel=wall_vel)


def couette_2d(n: int, re: float = 10.0, u_wall: float = 1.0, layers: int = 3,
               width: int | None = None, steps: int = 1000, name: str | None = None) -> Case:
    """Plane Couette start-up between walls at y = 0 (at rest) and y = 1
    (moving at (u_wall, 0) from t = 0), periodic in x: fluid at rest on the
    width x n lattice (dp = 1/n, width n/2 columns by default), `layers` rows
    of wall particles below and above.  Coordinates are shifted by layers*dp
    in y (box [0, width dp) x [0, 1 + 2 layers dp)).  Ids: fluid, then walls."""
    width = width or max(n // 2, 8)
    dx = 1.0 / n
    fluid, wall, top = _walled_box(width, n, layers, dx, False)
    pos = np.concatenate([fluid, wall], axis=1)
    nw = wall.shape[1]
    wall_vel = np.zeros((2, nw))
    wall_vel[0, top] = u_wall
    vel = np.zeros_like(pos)
    vel[:, fluid.shape[1]:] = wall_vel
    rho0 = 1.0
    c0 = 10.0 * u_wall
    eta = rho0 * u_wall * 1.0 / re
    npart = pos.shape[1]
    return Case(name=name or f"couette2d_{n}", dim=2, pos=pos, vel=vel,
                mass=np.full(npart, rho0 * dx * dx), h=np.full(npart, H_OVER_DP * dx),
                box=(width * dx, (n + 2 * layers) * dx), dx=dx, rho0=rho0, c0=c0, eta=eta,
                u_ref=u_wall, dt=_dt(H_OVER_DP * dx, u_wall, c0, eta / rho0), steps=steps,
                uniform=True, extra={"re": re, "layers": layers, "origin": layers * dx,
                                     "height": 1.0},
                n_wall=nw, wall_vel=wall_vel)


# The five workloads of the performance/parity plan, smallest first.
CONFIGS = {
    # 50x50 lattice, FP64, 100 steps: small enough for the oracle end to end
    "tg2d_50": lambda: taylor_green_2d(50, jitter=0.0, steps=100, name="tg2d_50"),
    # 400x400 jittered lattice, 160k particles, 1000 steps: the benchmark workload
    "tg2d_400": lambda: taylor_green_2d(400, jitter=0.05, seed=1, steps=1000, name="tg2d_400"),
    # variable resolution 2:1, ~1M particles, low velocity, 500 steps
    "varres2d_1m": lambda: variable_resolution_2d(steps=500, name="varres2d_1m"),
    # 3-D 128^3 jittered lattice, 200 steps
    "tg3d_128": lambda: taylor_green_3d(128, jitter=0.05, steps=200, name="tg3d_128"),
    # differentiation workload: 200x200 lattice, +-1% velocity perturbation, 200 steps
    "adjoint_tg2d_200": lambda: taylor_green_2d(200, jitter=0.0, vel_perturb=0.01, seed=1,
                                                steps=200, name="adjoint_tg2d_200"),
    # walls: the lid-driven cavity (Sec. 4.2) at dp = 1/200, Re = 1000
    "cavity2d_200": lambda: lid_driven_cavity(200, name="cavity2d_200"),
    # the three-dimensional cavity at dp = 1/128, Re = 100 (2.4M particles)
    "cavity3d_128": lambda: lid_driven_cavity(128, dim=3, name="cavity3d_128"),
}


def make(name: str) -> Case:
    return CONFIGS[name]()
