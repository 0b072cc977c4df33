"""Wide kernel supports (h = 3 dx in 2-D, 2 dx in 3-D): every lane holds more
neighbours than its LDS neighbour list, so the force sweep flushes the list in
the middle of a cell row and, outside the position stage, tests several
batches of candidates per cell.  Neighbour counts, densities and
accelerations against the FP64 oracle, and fused runs against single steps,
for lane groups of 2 (4 in 3-D) and 8."""
import numpy as np
import pytest

import cases
import oracle
from tests import parity_utils as pu

pytestmark = pytest.mark.gpu


def _wide(dim):
    if dim == 2:
        c = cases.taylor_green_2d(36, jitter=0.1, seed=5, name="wide2d")
        c.h = np.full(c.n, 3.0 * c.dx)          # ~113 neighbours per particle
    else:
        c = cases.taylor_green_3d(18, jitter=0.05, seed=6, name="wide3d")
        c.h = np.full(c.n, 2.0 * c.dx)          # ~268 neighbours per particle
    return c


WIDE = {2: _wide(2), 3: _wide(3)}
PARAMS = [(2, 2), (2, 8), (3, 4), (3, 8)]


def _sim(case, dtype, lanes):
    import torch
    from paper_2411_13992_amd import Simulation
    sim = Simulation.from_case(case, dtype=dtype, lanes=lanes)
    torch.cuda.synchronize()
    return sim


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dim,lanes", PARAMS)
def test_wide_support_sweeps(dim, lanes, dtype):
    case = WIDE[dim]
    assert all(nc >= 3 for nc in case.ncell())
    sim = _sim(case, dtype, lanes)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = oracle.neighbors(st["pos"], h, case.box)
    ref_counts = np.diff(nb[0])
    # more neighbours per lane (per z-plane of cells in 3-D, where the list is
    # flushed after each plane) than the lane's list holds
    cap = {2: 24, 4: 16, 8: 8}[lanes]
    assert ref_counts.min() / lanes / (3 if dim == 3 else 1) > cap
    got = sim.neighbor_counts().cpu().numpy()
    got_id = np.empty_like(got)
    got_id[sim.id.cpu().numpy()] = got
    band = pu.cutoff_band(st["pos"], h * (1 + 1e-5), case.box, dtype,
                          oracle.neighbors(st["pos"], h * (1 + 1e-5), case.box))
    assert band.mean() < 0.01
    assert np.array_equal(got_id[~band], ref_counts[~band])
    rho = oracle.density(st["pos"], mass, h, case.box, nb, oracle.lattice_kappa(dim))
    assert np.abs(st["rho"] - rho).max() / case.rho0 < pu.TOL[dtype]
    acc, scale = oracle.forces(st["pos"], st["vel"], mass, st["rho"], h, case.box, nb,
                               case.rho0, case.c0, case.eta, case.riemann_eta)
    err = np.max(np.abs(st["acc"] - acc) / scale)
    assert err < pu.TOL[dtype], err
    assert sim.flags() == 0


@pytest.mark.parametrize("dim,lanes", PARAMS)
def test_wide_support_fused_equals_single(dim, lanes):
    """Fused run and single steps agree bit for bit when the lists overflow."""
    import torch
    a = _sim(WIDE[dim], "f32", lanes)
    b = _sim(WIDE[dim], "f32", lanes)
    for _ in range(3):
        a.step(1)
    b.run(3)
    torch.cuda.synchronize()
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(a, key), getattr(b, key)), key
