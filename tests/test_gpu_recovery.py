"""Checkpoints on disk and recovery from a failed run: a state saved and
loaded again continues bit for bit; a fused run that raises a device flag is
undone (the state returns to the snapshot before it) and the run continues
from there once the cause is removed."""
import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu


def _sim(case, dtype="f32", **kw):
    import torch
    from paper_2411_13992_amd import Simulation
    sim = Simulation.from_case(case, dtype=dtype, **kw)
    torch.cuda.synchronize()
    return sim


@pytest.mark.parametrize("name", ["tg", "cavity"])
def test_checkpoint_round_trip(tmp_path, name):
    import torch
    case = (cases.taylor_green_2d(40, jitter=0.05, seed=3) if name == "tg"
            else cases.lid_driven_cavity(20))
    sim = _sim(case)
    sim.run(10, diag=False)
    path = str(tmp_path / "state.npz")
    sim.save_checkpoint(path)
    sim.run(10, diag=False)
    a = sim.snapshot()
    sim.load_checkpoint(path)
    assert sim.step_index == 10
    sim.run(10, diag=False)
    torch.cuda.synchronize()
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(sim, key), a[key]), key
    # loaded with pickling off; another configuration is refused
    with np.load(path) as z:
        assert int(z["step_index"]) == 10
    other = _sim(cases.taylor_green_2d(40, jitter=0.05, seed=3), tv_mode="scaled")
    if name == "tg":
        with pytest.raises(ValueError):
            other.load_checkpoint(path)


def test_run_checked_recovers_from_a_flagged_run():
    """A time step of 0.5 (over 1000 times the stable one) moves particles over
    more than a cell in its first step (SPH_FLAG_CFL; the drift clamps, so
    the kernels stay in bounds): run_checked restores
    the state before that run and raises; with the step size back, the run
    goes on and matches an undisturbed run."""
    import torch
    from paper_2411_13992_amd import StepFlagError
    from paper_2411_13992_amd import _lib
    case = cases.taylor_green_2d(32, jitter=0.05, seed=4)
    ref = _sim(case)
    ref.run_checked(30, chunk=10)
    sim = _sim(case)
    assert sim.run_checked(20, chunk=10) == 20
    before = sim.snapshot()
    dt = sim.params.dt
    sim.params.dt = 0.5
    with pytest.raises(StepFlagError) as e:
        sim.run_checked(1, chunk=1)
    assert e.value.flags & _lib.FLAG_CFL and e.value.step_index == 20
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(sim, key), before[key]), key
    sim.params.dt = dt
    sim.run_checked(10, chunk=5)
    torch.cuda.synchronize()
    assert sim.flags() == 0
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(sim, key), getattr(ref, key)), key
