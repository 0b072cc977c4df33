"""Dual-criteria time stepping on the GPU (sph_dual_run) against the FP64
oracle's advection step (Sec. 2.4, Eq. 3a, 5, 9-11), element by element.

Each comparison starts the oracle from the GPU's own state widened exactly to
FP64.  Per advection step: the step size dt_ad, the number of acoustic
substeps and the time they cover; positions / dx, velocities / U, the
substeps' density / rho0 (FP32 1e-5, FP64 1e-12).  A particle whose limiter
branch (Eq. 15) differs between the two must lie in the rounding band around
s0; on the step's fixed topology its correction moves only itself, so only
it is left out of the position comparison.  Substep by substep: the same with
the substeps capped at 1, 2 and 3.
"""
import numpy as np
import pytest

import cases
import oracle
from tests import parity_utils as pu

pytestmark = pytest.mark.gpu


def _sim(case, dtype, **kw):
    import torch
    from paper_2411_13992_amd import Simulation
    sim = Simulation.from_case(case, dtype=dtype, **kw)
    torch.cuda.synchronize()
    return sim


def _cases():
    v = cases.variable_resolution_2d(dp_min=1.0 / 90, jitter=0.1, seed=3, name="varres_small")
    return {
        "jitter64": cases.taylor_green_2d(64, jitter=0.1, seed=2, name="jitter64"),
        "ragged37": cases.taylor_green_2d(37, jitter=0.05, seed=9, name="ragged37"),
        "tg3d_12": cases.taylor_green_3d(12, jitter=0.05, seed=4, name="tg3d_12"),
        "varres_small": v,
    }


CASES = _cases()
GRID = [("jitter64", "f32", "limited"), ("jitter64", "f64", "limited"),
        ("jitter64", "f64", "scaled"), ("ragged37", "f32", "scaled"),
        ("tg3d_12", "f32", "limited"), ("tg3d_12", "f64", "limited"),
        ("varres_small", "f32", "limited"), ("varres_small", "f64", "limited")]


def _compare(case, dtype, mode, cap, nsteps=1):
    sim = _sim(case, dtype, tv_mode=mode)
    st, mass, h = pu.gpu_inputs(sim, case)
    rc = pu.case_with(case, mass, h)
    rc.pos, rc.vel = st["pos"], st["vel"]
    ref = oracle.State(rc, tv_mode=mode)
    q = oracle.dual_params(rc, max_substeps=cap)
    flipped = np.zeros(case.n, dtype=bool)
    recs = []
    for _ in range(nsteps):
        # limiter-branch flips at this step's start (its summation density)
        nb = oracle.neighbors(ref.pos, h, case.box)
        rho = oracle.density(ref.pos, mass, h, case.box, nb, oracle.lattice_kappa(case.dim))
        tv = oracle.tv(ref.pos, mass, rho, h, case.box, nb, case.h_min, tv_mode=mode)
        band = pu.limiter_band(tv["s"], tv["g"], tv["gscale"], case.h_min, case.lim_s0, dtype)
        d = ref.dual_step(q)
        recs.append(d)
        flipped |= band
    _, rec = sim.dual_run(nsteps, max_substeps=cap)
    rec = rec.cpu().numpy()
    out = sim.export()
    return sim, out, ref, recs, rec, flipped


@pytest.mark.parametrize("name,dtype,mode", GRID)
def test_advection_step_parity(name, dtype, mode):
    """One advection step with all its substeps."""
    case = CASES[name]
    sim, out, ref, recs, rec, band = _compare(case, dtype, mode, 0)
    tol = pu.TOL[dtype]
    d = recs[0]
    assert rec[0, 1] == d["substeps"] and d["substeps"] >= 3
    assert abs(rec[0, 0] / d["dt_ad"] - 1.0) < tol and abs(rec[0, 2] / d["t"] - 1.0) < tol
    ok = ~band
    e_pos = np.abs(pu.min_image(out["pos"], ref.pos, case.box)[:, ok]).max() / case.dx
    e_vel = np.abs(out["vel"] - ref.vel).max() / case.u_ref
    e_rho = np.abs(out["rho"] - ref.rho).max() / case.rho0
    print(f"dual step {name} {dtype} {mode}: substeps {d['substeps']} pos {e_pos:.2e} "
          f"vel {e_vel:.2e} rho {e_rho:.2e} (band {int(band.sum())})")
    assert e_pos < tol and e_vel < tol and e_rho < tol, (e_pos, e_vel, e_rho)
    diag = sim.diagnostics()
    # pair counts: exact in FP64; FP32 distances may put a pair within
    # rounding of the support radius on the other side
    assert abs(diag["npairs"] - d["npairs"]) <= (0 if dtype == "f64" else 2)
    assert abs(diag["ke"] / d["ke"] - 1.0) < tol
    assert sim.flags() == 0


@pytest.mark.parametrize("cap", [1, 2, 3])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_acoustic_substep_parity(cap, dtype):
    """The advection step ended after `cap` substeps: the state after each
    of the first substeps (positions, velocities, density)."""
    case = CASES["jitter64"]
    sim, out, ref, recs, rec, band = _compare(case, dtype, "limited", cap)
    tol = pu.TOL[dtype]
    d = recs[0]
    assert rec[0, 1] == d["substeps"] == cap and d["t"] < d["dt_ad"]
    assert abs(rec[0, 2] / d["t"] - 1.0) < tol
    ok = ~band
    e_pos = np.abs(pu.min_image(out["pos"], ref.pos, case.box)[:, ok]).max() / case.dx
    e_vel = np.abs(out["vel"] - ref.vel).max() / case.u_ref
    e_rho = np.abs(out["rho"] - ref.rho).max() / case.rho0
    assert e_pos < tol and e_vel < tol and e_rho < tol, (e_pos, e_vel, e_rho)
    assert sim.flags() == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_several_advection_steps(dtype):
    """Five advection steps: step sizes, substep counts, energy and the
    correction's diagnostics stay on the oracle's course (FP64: the state
    to 1e-10)."""
    case = CASES["jitter64"]
    sim, out, ref, recs, rec, band = _compare(case, dtype, "limited", 0, nsteps=5)
    tol = pu.TOL[dtype]
    for s, d in enumerate(recs):
        assert rec[s, 1] == d["substeps"]
        assert abs(rec[s, 0] / d["dt_ad"] - 1.0) < 10 * tol
    diag = sim.diagnostics()
    assert abs(diag["ke"] / recs[-1]["ke"] - 1.0) < 10 * tol
    if dtype == "f64":
        e_pos = np.abs(pu.min_image(out["pos"], ref.pos, case.box)).max() / case.dx
        assert e_pos < 1e-10
    assert sim.flags() == 0


def test_dual_run_arguments():
    """Walls and the background-pressure formulation are not supported; a
    substep cap beyond 64 is an argument error."""
    from paper_2411_13992_amd import SphError
    cav = cases.lid_driven_cavity(12)
    sim = _sim(cav, "f32")
    with pytest.raises(SphError):
        sim.dual_run(1)
    sim = _sim(CASES["ragged37"], "f32", tv_mode="background")
    with pytest.raises(SphError):
        sim.dual_run(1)
    sim = _sim(CASES["ragged37"], "f32")
    with pytest.raises(SphError):
        sim.dual_run(1, max_substeps=65)


def test_dual_tg_study_matches_oracle():
    """The dual-criteria Taylor-Green study (tg_study.run_dual) on a jittered
    50 x 50 start, FP64, against the oracle's advection steps from the same
    particles: step times and the sampled kinetic-energy ratio."""
    from paper_2411_13992_amd.tg_study import run_dual
    r = run_dual(50, 0.06, "limited", dtype="f64", jitter=0.05, chunk=10, samples=10)
    assert r["flags"] == 0
    case = cases.taylor_green_2d(50, jitter=0.05, seed=1)
    st = oracle.State(case)
    ke0 = st.kinetic_energy()
    q = oracle.dual_params(case)
    t, ke = [], []
    while len(t) < r["advection_steps"]:
        d = st.dual_step(q)
        t.append((t[-1] if t else 0.0) + d["t"])
        ke.append(d["ke"] / ke0)
    t, ke = np.array(t), np.array(ke)
    idx = np.searchsorted(t, np.asarray(r["t"]) - 1e-12)
    assert np.allclose(np.asarray(r["t"]), t[idx], rtol=1e-12, atol=0)
    assert np.max(np.abs(np.asarray(r["ke_over_ke0"]) / ke[idx] - 1.0)) < 1e-9
