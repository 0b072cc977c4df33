"""GPU path (libsph through its C-ABI) against the FP64 oracle, element by element.

Every comparison starts the oracle from the GPU's own state widened exactly to
FP64, so the only differences are the GPU's rounding.  Tolerances and
normalisations are those of tests/parity_utils.py.
"""
import math

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


def _small_cases():
    v = cases.variable_resolution_2d(dp_min=1.0 / 90, jitter=0.1, seed=3, name="varres_small")
    return {
        "lattice10": cases.taylor_green_2d(10, name="lattice10"),           # 3 cells per axis
        "tg2d_50": cases.make("tg2d_50"),
        "ragged37": cases.taylor_green_2d(37, jitter=0.05, seed=9, name="ragged37"),
        "jitter64": cases.taylor_green_2d(64, jitter=0.1, seed=2, name="jitter64"),
        "tg3d_12": cases.taylor_green_3d(12, jitter=0.05, seed=4, name="tg3d_12"),
        "varres_small": v,
    }


SMALL = _small_cases()
CASE_DTYPES = [(name, dt) for name in SMALL for dt in ("f32", "f64")]


def _oracle_nb(pos, h, box):
    return oracle.neighbors(pos, h, box)


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_cells_sorted_and_binned(name, dtype):
    """(cell, id) order, cell_start consistent with the cells, and cell indices
    equal to floor(x / L) of the input positions (bit-exact, apart from
    particles within rounding of a face)."""
    case = SMALL[name]
    sim = _sim(case, dtype)
    cell = sim.cell.cpu().numpy().astype(np.int64)
    ids = sim.id.cpu().numpy().astype(np.int64)
    cs = sim.cs.cpu().numpy().astype(np.int64)
    key = cell * case.n + ids
    assert np.all(np.diff(key) > 0), "not in (cell, id) order"
    assert np.array_equal(np.sort(ids), np.arange(case.n))
    counts = np.bincount(cell, minlength=sim.ncells)
    assert cs[0] == 0 and np.array_equal(np.diff(cs), counts)
    # canonical binning of the input positions
    nc = sim.cfg.cells()
    pos = case.pos[:, ids]
    lin = np.zeros(case.n, dtype=np.int64)
    stride = 1
    near_face = np.zeros(case.n, dtype=bool)
    for k in range(case.dim):
        L = case.box[k] / nc[k]
        c = np.floor(pos[k] / L).astype(np.int64)
        frac = pos[k] / L - c
        near_face |= (frac < 1e-6) | (frac > 1 - 1e-6)
        lin += np.clip(c, 0, nc[k] - 1) * stride
        stride *= nc[k]
    ok = ~near_face
    assert np.array_equal(lin[ok], cell[ok])
    # offsets reproduce the positions
    back = sim.positions_fp64()
    err = np.abs(pu.min_image(back, pos, case.box)).max() / case.dx
    assert err < (1e-6 if dtype == "f32" else 1e-13)


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_neighbour_counts_exact(name, dtype):
    """|N(i)| from the GPU's cell search equals the oracle's, bit for bit, for
    every particle without a pair within rounding of the cutoff."""
    case = SMALL[name]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    ref = np.diff(nb[0])
    got = sim.neighbor_counts().cpu().numpy()
    got_id = np.empty_like(got)
    got_id[sim.id.cpu().numpy()] = got
    band = pu.cutoff_band(st["pos"], h * (1 + 1e-5), case.box, dtype,
                          _oracle_nb(st["pos"], h * (1 + 1e-5), case.box))
    assert band.mean() < 0.01
    assert np.array_equal(got_id[~band], ref[~band])


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_density_parity(name, dtype):
    """Eq. 8 on identical positions: |rho_gpu - rho_oracle| / rho0 within tolerance."""
    case = SMALL[name]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    ref = oracle.density(st["pos"], mass, h, case.box, nb, oracle.lattice_kappa(case.dim))
    err = np.abs(st["rho"] - ref).max() / case.rho0
    assert err < pu.TOL[dtype], err


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_tv_parity(name, dtype):
    """Eq. 14-16 on identical positions and densities: g and dr against the
    oracle on the summation-error scale; the limiter branch agrees outside the
    rounding band around s0; s is the FP64 test value."""
    import torch
    case = SMALL[name]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    ref = oracle.tv(st["pos"], mass, st["rho"], h, case.box, nb, case.h_min, xi=case.xi,
                    lim_c=case.lim_c, lim_s0=case.lim_s0)
    out = sim.tv_correction()
    torch.cuda.synchronize()
    order = st["order"]
    g = out["g"].cpu().double().numpy()[:, order]
    dr = out["dr"].cpu().double().numpy()[:, order]
    beta = out["beta"].cpu().double().numpy()[order]
    s = out["s"].cpu().numpy()[order]
    scale = ref["gscale"]
    tol = pu.TOL[dtype]
    assert np.max(np.abs(g - ref["g"]) / scale) < tol
    band = pu.limiter_band(ref["s"], ref["g"], scale, case.h_min, case.lim_s0, dtype)
    ok = ~band
    assert np.array_equal(beta[ok] > 0, ref["beta"][ok] > 0)
    hb = case.h_min ** 2
    assert np.max(np.abs(dr[:, ok] - ref["dr"][:, ok]) / (abs(case.xi) * hb * scale[ok])) < 4 * tol
    # s is h_min^2 |g|^2 of the GPU's own g, in FP64
    assert np.allclose(s, hb * np.sum(g * g, axis=0), rtol=1e-12, atol=0.0)
    # the ramp branch of Eq. 15
    ramp = ok & (ref["s"] > case.lim_s0) & (case.lim_c * ref["s"] < 1.0)
    if ramp.any():
        assert np.max(np.abs(beta[ramp] - case.lim_c * s[ramp])) < (1e-6 if dtype == "f32" else 1e-14)


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_forces_parity(name, dtype):
    """Eq. 2-7 on identical positions, velocities and densities: the
    acceleration error on the summation-error scale of the force sum."""
    case = SMALL[name]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    ref, scale = oracle.forces(st["pos"], st["vel"], mass, st["rho"], h, case.box, nb,
                               case.rho0, case.c0, case.eta, case.riemann_eta)
    err = np.max(np.abs(st["acc"] - ref) / scale)
    assert err < pu.TOL[dtype], err


@pytest.mark.parametrize("name,dtype", CASE_DTYPES)
def test_step_parity(name, dtype):
    """One whole kick-drift-kick step from an identical state.  A particle whose
    limiter branch (Eq. 15) differs between GPU and oracle must lie in the
    rounding band around s0; it and the particles within two neighbour hops of
    it (density, then forces) are excluded from the field comparison."""
    import torch
    case = SMALL[name]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    ref = oracle.State(pu.case_with(case, mass, h), pos=st["pos"], vel=st["vel"],
                       rho=st["rho"], acc=st["acc"])
    nb0 = _oracle_nb(st["pos"], h, case.box)
    tv0 = oracle.tv(st["pos"], mass, st["rho"], h, case.box, nb0, case.h_min)
    band = pu.limiter_band(tv0["s"], tv0["g"], tv0["gscale"], case.h_min, case.lim_s0, dtype)
    beta_gpu = sim.tv_correction()["beta"].cpu().double().numpy()[st["order"]]
    torch.cuda.synchronize()
    flipped = (beta_gpu > 0) != (tv0["beta"] > 0)
    assert not np.any(flipped & ~band)
    sim.step(1)
    ref.step()
    out = sim.export()
    nb1 = _oracle_nb(ref.pos, h, case.box)
    skip = pu.widen(nb1, flipped, 2)
    assert skip.mean() < 0.5
    ok = ~skip
    tol = pu.TOL[dtype]
    e_pos = np.abs(pu.min_image(out["pos"], ref.pos, case.box)[:, ok]).max() / case.dx
    e_vel = np.abs(out["vel"] - ref.vel)[:, ok].max() / case.u_ref
    e_rho = np.abs(out["rho"] - ref.rho)[ok].max() / case.rho0
    e_acc = pu.step_acc_error(out, case, mass, h, ok)
    assert e_pos < tol and e_vel < tol and e_rho < tol and e_acc < tol, \
        (e_pos, e_vel, e_rho, e_acc)
    assert sim.flags() == 0


def test_tg2d_50_fp64_trajectory():
    """The 50x50 Taylor-Green workload, 100 FP64 steps on the GPU and in the
    oracle from the same initial state: kinetic energy and momentum agree,
    and the decay stays on the oracle's course."""
    case = cases.make("tg2d_50")
    sim = _sim(case, "f64")
    st, mass, h = pu.gpu_inputs(sim, case)
    ref = oracle.State(case, pos=st["pos"], vel=st["vel"], rho=st["rho"], acc=st["acc"])
    ke_gpu = []
    for _ in range(case.steps):
        sim.step(1)
        ke_gpu.append(sim.diagnostics()["ke"])
    d = ref.run(case.steps)
    ke_ref = d[:, 0]
    assert np.max(np.abs(np.array(ke_gpu) / ke_ref - 1.0)) < 1e-9
    diag = sim.diagnostics()
    assert abs(diag["px"]) < 1e-13 and abs(diag["py"]) < 1e-13
    assert diag["npairs"] == d[-1, 5]
    out = sim.export()
    e = np.abs(pu.min_image(out["pos"], ref.pos, case.box)).max() / case.dx
    assert e < 1e-9


def test_tg2d_50_fp32_trajectory_reported(capsys):
    """100 FP32 steps against the FP64 oracle: per-field errors after N steps
    are reported; the gates are conservation (momentum) and the decay."""
    case = cases.make("tg2d_50")
    sim = _sim(case, "f32")
    st, mass, h = pu.gpu_inputs(sim, case)
    ref = oracle.State(case, pos=st["pos"], vel=st["vel"], rho=st["rho"], acc=st["acc"])
    sim.step(case.steps)
    d = ref.run(case.steps)
    diag = sim.diagnostics()
    out = sim.export()
    e_pos = np.abs(pu.min_image(out["pos"], ref.pos, case.box)).max() / case.dx
    e_vel = np.abs(out["vel"] - ref.vel).max() / case.u_ref
    e_rho = np.abs(out["rho"] - ref.rho).max() / case.rho0
    print(f"tg2d_50 f32 after {case.steps} steps: pos {e_pos:.2e} dx, vel {e_vel:.2e} U, "
          f"rho {e_rho:.2e} rho0, KE rel {diag['ke'] / d[-1, 0] - 1:.2e}")
    assert abs(diag["ke"] / d[-1, 0] - 1.0) < 1e-3
    assert abs(diag["px"]) < 1e-6 and abs(diag["py"]) < 1e-6


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_empty_input(dtype):
    """N = 0: every call succeeds and the diagnostics are zero."""
    import torch
    case = cases.taylor_green_2d(10)
    case.pos = case.pos[:, :0]
    case.vel = case.vel[:, :0]
    case.mass = np.full(1, case.mass[0])
    sim = _sim(case, dtype)
    sim.step(2)
    torch.cuda.synchronize()
    assert np.all(sim.diag.cpu().numpy() == 0.0)
    assert np.all(sim.cs.cpu().numpy() == 0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_coincident_particles(dtype):
    """Two particles at one point: both count as neighbours, the pressure term
    of the pair vanishes (no Riemann axis), results match the oracle."""
    case = cases.taylor_green_2d(12, jitter=0.05, seed=3)
    case.pos[:, 7] = case.pos[:, 8]
    sim = _sim(case, dtype)
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    rho = oracle.density(st["pos"], mass, h, case.box, nb, oracle.lattice_kappa(2))
    acc, scale = oracle.forces(st["pos"], st["vel"], mass, st["rho"], h, case.box, nb,
                               case.rho0, case.c0, case.eta)
    assert np.abs(st["rho"] - rho).max() < pu.TOL[dtype]
    assert np.max(np.abs(st["acc"] - acc) / scale) < pu.TOL[dtype]
    assert sim.flags() == 0


def test_flags_nonfinite_and_cfl():
    """Device error flags, forced from the host: a NaN velocity sets
    SPH_FLAG_NONFINITE; a time step that moves particles over more than one
    cell sets SPH_FLAG_CFL.  The kernels stay in bounds in both cases."""
    import torch
    from paper_2411_13992_amd import _lib
    case = cases.taylor_green_2d(16)
    sim = _sim(case, "f32")
    sim.vel[0, 3] = float("nan")
    sim.step(1)
    assert sim.flags() & _lib.FLAG_NONFINITE
    sim = _sim(case, "f32", dt=0.5)
    sim.step(1)
    torch.cuda.synchronize()
    assert sim.flags() & _lib.FLAG_CFL


@pytest.mark.parametrize("name,dtype", [("jitter64", "f32"), ("jitter64", "f64"),
                                        ("tg3d_12", "f32"), ("varres_small", "f32")])
@pytest.mark.parametrize("tv_every", [1, 3])
def test_fused_run_equals_single_steps(name, dtype, tv_every):
    """sph_kdk_run (correction and next drift fused into the force sweep) gives
    bit-identical states and diagnostics to the same number of sph_kdk_step
    calls, including runs whose correction applies only every third step."""
    import torch
    case = SMALL[name]
    a = _sim(case, dtype, tv_every=tv_every)
    b = _sim(case, dtype, tv_every=tv_every)
    rows = []
    for _ in range(7):
        a.step(1)
        rows.append(a.diag.clone())
    d = b.run(7)
    torch.cuda.synchronize()
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(a, key), getattr(b, key)), key
    assert torch.equal(torch.stack(rows), d)
    assert a.flags() == 0 and b.flags() == 0


@pytest.mark.parametrize("name,dtype,mode", [("jitter64", "f32", "limited"),
                                             ("jitter64", "f64", "limited"),
                                             ("tg3d_12", "f32", "limited"),
                                             ("varres_small", "f32", "limited"),
                                             ("jitter64", "f32", "background")])
@pytest.mark.parametrize("tv_every", [1, 3])
def test_fused_run_tapes_equal_single_step_tapes(name, dtype, mode, tv_every):
    """The tapes a fused run records (correction sums from the fused force
    sweep, states shared between consecutive steps) are byte-identical to
    those of the same number of single steps."""
    import torch
    case = SMALL[name]
    a = _sim(case, dtype, tv_every=tv_every, tv_mode=mode)
    b = _sim(case, dtype, tv_every=tv_every, tv_mode=mode)
    nsteps, tb = 5, a.tape_bytes()
    # both start zeroed, so the never-written alignment padding compares equal
    ta = torch.zeros((nsteps, tb), dtype=torch.uint8, device=a.device)
    tb_ = torch.zeros((nsteps, tb), dtype=torch.uint8, device=b.device)
    for s in range(nsteps):
        a.step(1, tape=ta[s])
    b.run(nsteps, diag=False, tapes=tb_)
    torch.cuda.synchronize()
    for s in range(nsteps):
        assert torch.equal(ta[s], tb_[s]), s
    for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
        assert torch.equal(getattr(a, key), getattr(b, key)), key


def test_deterministic_rerun():
    """No floating-point atomics: two identical runs agree bit for bit."""
    case = SMALL["jitter64"]
    outs = []
    for _ in range(2):
        sim = _sim(case, "f32")
        sim.step(5)
        outs.append((sim.off.cpu().numpy(), sim.vel.cpu().numpy(), sim.rho.cpu().numpy(),
                     sim.diag.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_benchmark_workload_sweeps(dtype):
    """The 400x400 jittered Taylor-Green workload (160k particles), in the
    launch configuration the benchmark times, after 5 steps: every sweep output
    against the oracle at the GPU's state, all particles."""
    import torch
    case = cases.make("tg2d_400")
    sim = _sim(case, dtype)
    sim.step(5)
    torch.cuda.synchronize()
    st, mass, h = pu.gpu_inputs(sim, case)
    nb = _oracle_nb(st["pos"], h, case.box)
    tol = pu.TOL[dtype]
    rho = oracle.density(st["pos"], mass, h, case.box, nb, oracle.lattice_kappa(2))
    rho_gpu = sim.density(out=torch.empty_like(sim.rho)).cpu().double().numpy()[st["order"]]
    assert np.abs(rho_gpu - rho).max() / case.rho0 < tol
    acc, scale = oracle.forces(st["pos"], st["vel"], mass, st["rho"], h, case.box, nb,
                               case.rho0, case.c0, case.eta)
    acc_gpu = sim.forces(out=torch.empty_like(sim.acc)).cpu().double().numpy()[:, st["order"]]
    assert np.max(np.abs(acc_gpu - acc) / scale) < tol
    ref = oracle.tv(st["pos"], mass, st["rho"], h, case.box, nb, case.h_min)
    out = sim.tv_correction()
    g = out["g"].cpu().double().numpy()[:, st["order"]]
    assert np.max(np.abs(g - ref["g"]) / ref["gscale"]) < tol
    counts = np.empty(case.n, dtype=np.int64)
    counts[sim.id.cpu().numpy()] = sim.neighbor_counts().cpu().numpy()
    band = pu.cutoff_band(st["pos"], h * (1 + 1e-5), case.box, dtype,
                          _oracle_nb(st["pos"], h * (1 + 1e-5), case.box))
    assert np.array_equal(counts[~band], np.diff(nb[0])[~band])
    assert sim.flags() == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rebuild_many_tiles_canonical_order(dtype):
    """A 700x700 lattice has more cell-build tiles (538) than one block per CU
    can run at once, so the runs use the cell build's plain instance.  After
    fused steps the state is in (cell, id) order: the general cell build
    (slot claims, scan, scatter, in-cell ranking by id) leaves every array
    unchanged and returns the identity permutation."""
    import torch
    case = cases.taylor_green_2d(700, jitter=0.1, seed=21, name="tg2d_700")
    sim = _sim(case, dtype)
    nc0, nc1 = int(sim.params.ncell[0]), int(sim.params.ncell[1])
    occ = sim.n / (nc0 * nc1)
    t = max(1, min(int(2048 / (1.5 * occ)), 512, nc0))
    assert -(-nc0 // t) * nc1 > 256
    sim.run(4)
    torch.cuda.synchronize()
    assert sim.flags() == 0
    keys = ("cell", "id", "off", "vel", "rho", "cs")
    before = {k: getattr(sim, k).clone() for k in keys}
    perm = torch.empty(sim.n, dtype=torch.int32, device=sim.device)
    sim.build_cells(perm)
    torch.cuda.synchronize()
    for k in keys:
        assert torch.equal(before[k], getattr(sim, k)), k
    assert torch.equal(perm.long(), torch.arange(sim.n, device=sim.device))


def _cavity_small():
    return cases.lid_driven_cavity(12, jitter=0.1, seed=31)


@pytest.mark.parametrize("name,dtype,tv_every", [("jitter64", "f32", 1), ("jitter64", "f64", 1),
                                                 ("jitter64", "f32", 3), ("tg3d_12", "f32", 1),
                                                 ("varres_small", "f32", 1), ("cavity", "f32", 1)])
def test_resumed_run_equals_one_run(name, dtype, tv_every):
    """sph_kdk_run_resume continues where the previous run or step left off
    (its first correction and drift come from that call's last force sweep):
    3 + 4 resumed steps, and 2 single steps + 5 resumed, equal one run of 7
    bit for bit, states and every diagnostics row, also when the earlier call
    kept no diagnostics."""
    import torch
    case = _cavity_small() if name == "cavity" else SMALL[name]
    ref = _sim(case, dtype, tv_every=tv_every)
    d_ref = ref.run(7)
    a = _sim(case, dtype, tv_every=tv_every)
    d1 = a.run(3)
    d2 = a.run(4, resume=True)
    b = _sim(case, dtype, tv_every=tv_every)
    b.step(2)
    d3 = b.run(5, resume=True)
    c = _sim(case, dtype, tv_every=tv_every)
    c.run(4, diag=False)
    d4 = c.run(3, resume=True)
    torch.cuda.synchronize()
    for sim in (a, b, c):
        for key in ("cell", "id", "off", "vel", "acc", "rho", "cs"):
            assert torch.equal(getattr(ref, key), getattr(sim, key)), key
        assert sim.flags() == 0
    assert torch.equal(torch.cat([d1, d2]), d_ref)
    assert torch.equal(d3, d_ref[2:])
    assert torch.equal(d4, d_ref[4:])


def test_resume_refused_after_state_changes():
    """The Python layer refuses to resume once anything but a run or step
    touched the simulation, and a resumed run records no tapes."""
    case = SMALL["jitter64"]
    sim = _sim(case, "f32")
    with pytest.raises(ValueError):
        sim.run(2, resume=True)          # nothing to resume from yet
    sim.run(2)
    sim.set_xi(sim.params.xi)
    with pytest.raises(ValueError):
        sim.run(2, resume=True)
    sim.run(2)
    sim.density()
    with pytest.raises(ValueError):
        sim.run(2, resume=True)
    sim.step(1)
    sim.run(2, resume=True)
    import torch
    tapes = torch.zeros((2, sim.tape_bytes()), dtype=torch.uint8, device=sim.device)
    with pytest.raises(ValueError):
        sim.run(2, resume=True, tapes=tapes)
