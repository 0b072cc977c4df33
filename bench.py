"""Benchmark: pair interactions per second of one transport-velocity WCSPH step.

Workload: 2-D periodic Taylor-Green vortex, 400 x 400 lattice (160,000
particles) jittered by +-0.05 dx, h = 1.3 dx, Wendland C2, Re = 100, the
h-scaled transport-velocity correction with its limiter every step.  A step
is the whole hot path: correction sweep, kick + drift + rebin, cell build,
density sweep, force sweep, kick + FP64 diagnostics.  Inputs are resident on
the GPU before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
        [--workload tg2d_400 | tg3d_128 | varres2d_1m | cavity2d_200 | cavity3d_128]

Prints one JSON line.  The default workload is the benchmark; the others
(3-D Taylor-Green cube, variable-resolution box, walled 2-D and 3-D cavities)
print the same line format.  `value` is FP32 pair interactions per second (ordered
neighbour pairs j != i with r < 2h, counted by the step itself, divided by the
step time).  Extra fields: the FP64 rate, the adjoint / forward time ratio,
the roofline of the dominant kernel (the force sweep over stored neighbour
lists, timed live with HIP events on its stream) and the FP64 CPU oracle's
rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/s per TV-WCSPH step, FP32 vs FP64; adjoint/forward time"
WORKLOAD = "tg2d_400"
WORKLOADS = {
    "tg2d_400": "2-D periodic Taylor-Green vortex, 400x400 lattice jittered +-0.05 dx "
                "(160,000 particles), h = 1.3 dx, Wendland C2, Re = 100, c0 = 10 U, "
                "transport-velocity correction with limiter every step, FP32 sweeps with "
                "FP64 reductions",
    "tg3d_128": "3-D periodic Taylor-Green vortex, 128^3 lattice jittered +-0.05 dx "
                "(2,097,152 particles), h = 1.3 dx, Wendland C2, nu = 0.01, c0 = 10 U, "
                "correction with limiter every step, FP32 sweeps with FP64 reductions",
    "varres2d_1m": "2-D periodic variable-resolution box, smooth 2:1 smoothing-length "
                   "profile, dp_min = 1/1306 (1,000,632 particles), jitter +-0.1 dp, "
                   "low-speed random divergence-free flow, correction with limiter every "
                   "step, FP32 sweeps with FP64 reductions",
    "cavity2d_200": "2-D lid-driven cavity (Sec. 4.2), dp = 1/200, Re = 1000, 200x200 fluid "
                    "particles at rest inside three layers of wall particles (42,436 "
                    "particles), lid at U = 1, correction with limiter every step, FP32 "
                    "sweeps with FP64 reductions",
    "cavity3d_128": "3-D lid-driven cavity, dp = 1/128, Re = 100, 128^3 fluid particles at "
                    "rest inside three layers of wall particles (2,406,104 particles), lid "
                    "velocity (1, 0, 0), correction with limiter every step, FP32 sweeps "
                    "with FP64 reductions",
}

# Algorithmic work per interacting pair of the force sweep, counted from the
# oracle's pair formula (Eq. 2, 3b, 5-7), one flop per add, subtract,
# multiply, divide/reciprocal, square root, min or max (an FMA counts two);
# uniform resolution, constants folded, no summation compensation, no
# candidate test (the neighbour search is overhead, not the method's work).
# Items: pair vector r_ij, r^2, r, q = r/h, 1 - q/2, F = W'/r, p_j (EOS),
# U_l - U_r (1/r, velocity difference, axis, dot), the dissipation limiter
# beta (Eq. 6), mean density, P* (Eq. 5), 2 m_j / (rho_i rho_j), and per
# component the pressure and viscous terms and the accumulation.
def force_flops_per_pair(dim: int) -> int:
    d = dim
    items = [d, 2 * d - 1, 1, 1, 2, 3, 2, 1 + d + d + (2 * d - 1), 4, 2, 6, 3, 4 + 4 * d]
    return sum(items)


FORCE_FLOPS_PER_PAIR = {2: force_flops_per_pair(2), 3: force_flops_per_pair(3)}   # 49, 60

# Compulsory HBM bytes per particle of each kernel of a 2-D FP32 step (each
# kernel reads its per-particle inputs once and writes its outputs once) and
# VALU lane-operations per interacting pair (FMA = 1): the step's attainable
# time is sum_k max(bytes_k N / HBM, ops_k P / VALU).
STEP_KERNELS_2D_F32 = {
    #  kernel: (bytes per particle, lane-ops per pair)
    "cell build (keys, scatter, in-cell order, permute)": (88, 0),
    "transport correction sweep": (20, 22),
    "density sweep": (12, 20),
    "force sweep": (28, 47),
    "kick + drift + rebin": (56, 0),
    "kick + FP64 reductions": (32, 0),
}
HBM_PEAK = 8e12                       # MI355X HBM3E, bytes/s
# Published vector FP32 peak of MI355X (packed FP32): 157.3 TFLOP/s.  This
# library is built without packed FP32 math, so the peak it can attain is
# half of it: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 flops per FMA.
VALU_FP32_PEAK_TFLOPS = 157.3
VALU_ATTAINABLE_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12       # 78.6
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9                           # 39.3e12 lane-ops/s


def force_bytes_per_particle(dim: int, dtype: str, per_particle: bool) -> int:
    """Compulsory bytes of the force sweep per particle: reads of offsets D,
    velocity D and density 1 (plus mass and h with per-particle resolution)
    and the write of the acceleration D, once each."""
    words = 3 * dim + 1 + (2 if per_particle else 0)
    return words * (8 if dtype == "f64" else 4)


def step_bounds(n: int, pairs: float, t_step: float) -> dict:
    """Whole-step fractions for the 2-D FP32 step: algorithmic HBM bytes over
    time against the HBM peak, and the attainable step time (per kernel the
    larger of its byte and its VALU time, summed) over the measured time."""
    t_bound = 0.0
    nbytes = 0
    for b, ops in STEP_KERNELS_2D_F32.values():
        nbytes += b * n
        t_bound += max(b * n / HBM_PEAK, ops * pairs / VALU_LANE_OPS)
    return {"algorithmic_bytes": nbytes, "hbm_frac": nbytes / t_step / HBM_PEAK,
            "attainable_us": t_bound * 1e6, "attainable_frac": t_bound / t_step}


PMC_SUMMARY = os.path.join(ROOT, "profiles", "forces_list_kernel_tg2d_400_f32_pmc.md")
PMC_COPY_BYTES = 64 << 20
KERNEL_SOURCES = os.path.join(ROOT, "paper_2411_13992_amd", "csrc")


def _events_time(fn, reps):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / reps


def time_steps(sim, steps, warmup):
    """Seconds per step of `steps` consecutive steps (one fused run, every
    step's diagnostics kept on the device) and the mean ordered pair count.
    The timed run continues the warm-up run (sph_kdk_run_resume): its first
    step's correction sweep was evaluated by the warm-up's last force sweep,
    and its own last force sweep evaluates the next step's, so the timed
    region holds exactly `steps` steps of work."""
    import torch
    sim.run(warmup)
    rows = sim.diag_rows(steps)
    torch.cuda.synchronize()
    resume = warmup > 0
    t = _events_time(lambda: sim.run(steps, diag=rows, resume=resume), 1) / steps
    pairs = float(rows[:, 5].mean().item())
    return t, pairs


def time_adjoint(sim, steps, every):
    """Seconds per step of the forward rollout and of its reverse sweep
    (recompute with tapes + reverse steps + the init reverse)."""
    import torch
    from paper_2411_13992_amd.adjoint import backward_run, forward_run
    v0 = sim.velocity_by_id().clone()
    xi = sim.params.xi
    forward_run(sim, v0, xi, steps, every)     # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ckpts = forward_run(sim, v0, xi, steps, every)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / steps
    vbar = v0.clone()
    final_id = sim.id.clone()
    tapes = torch.empty((every, sim.tape_bytes()), dtype=torch.uint8, device=sim.device)
    backward_run(sim, ckpts, steps, every, vbar, final_id, tapes)   # warm
    ckpts = forward_run(sim, v0, xi, steps, every)
    final_id = sim.id.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    backward_run(sim, ckpts, steps, every, vbar, final_id, tapes)
    torch.cuda.synchronize()
    t_bwd = (time.perf_counter() - t0) / steps
    return t_fwd, t_bwd


def kernel_roofline(sim, pairs, dtype, reps=200, use_pmc=True):
    """Average duration of the force sweep over stored neighbour lists
    (sph_forces_lists after sph_density_lists on the benchmark state: the
    step's force sweep without its fused correction sum and kick-drift
    epilogue, same lists, stage and launch shape), by HIP events on the
    stream it runs on; the density sweep that records the lists (the step's
    own kernel) is timed the same way."""
    import torch
    lists = sim.neighbor_lists()
    rho = torch.empty_like(sim.rho)
    out = torch.empty_like(sim.acc)
    sim.density_lists(lists, out=rho)
    sim.forces_lists(lists, out=out)
    t = _events_time(lambda: sim.forces_lists(lists, out=out), reps)
    t_density = _events_time(lambda: sim.density_lists(lists, out=rho), reps)
    flops = FORCE_FLOPS_PER_PAIR[sim.dim] * pairs
    bytes_ = force_bytes_per_particle(sim.dim, dtype, sim.var) * sim.n
    achieved = flops / t / 1e12
    traffic = _pmc_traffic() if use_pmc else None
    return {
        "kernel": "forces_list_kernel",
        "bound": "alu",
        "achieved": achieved,
        "peak": VALU_FP32_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / VALU_FP32_PEAK_TFLOPS,
        "traffic": traffic,
        "attainable_peak": VALU_ATTAINABLE_TFLOPS,
        "attainable_frac": achieved / VALU_ATTAINABLE_TFLOPS,
        "attainable_peak_note": "non-packed FP32: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2",
        "avg_launch_us": t * 1e6,
        "flops_per_pair": FORCE_FLOPS_PER_PAIR[sim.dim],
        "algorithmic_flops_per_launch": flops,
        "algorithmic_bytes_per_launch": bytes_,
        "hbm_frac": bytes_ / t / HBM_PEAK,
        "density_list_kernel_us": t_density * 1e6,
    }


def _pmc_traffic():
    """Bytes per launch of the force sweep between L2 and the memory fabric,
    from the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE,
    each scaled by what it reads for a device copy of known size), if it was
    taken on the current kernel sources."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b:
        return None
    return float(b.group(1)) if source_digest() == m.group(1) else None


# the sources the force sweep is compiled from
FORCE_SWEEP_SOURCES = ("sph_dev.hpp", "sph_internal.hpp", "sweeps.hip")


def source_digest():
    """SHA-256 over the force sweep's sources (sorted by name) with comments
    and whitespace removed: a counter summary taken on other kernel code is
    not used, one taken before a comment-only edit (or an edit of code the
    force sweep does not contain) still is."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        if name in FORCE_SWEEP_SOURCES:
            text = open(os.path.join(KERNEL_SOURCES, name)).read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(name.encode())
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def time_dual(case, nsteps=60, warmup=5):
    """The dual-criteria scheme (sph_dual_run) on the same workload, FP32:
    time per advection step and per acoustic substep (a substep is one
    pressure and one continuity sweep; an advection step adds the density,
    prologue and move sweeps and the cell build)."""
    import torch
    from paper_2411_13992_amd import Simulation
    sim = Simulation.from_case(case, dtype="f32")
    sim.dual_run(warmup)
    torch.cuda.synchronize()
    box = {}
    t = _events_time(lambda: box.update(r=sim.dual_run(nsteps)), 1)
    d, rec = box["r"]
    rec = rec.cpu().numpy()
    sub = float(rec[:, 1].mean())
    pairs = float(d[:, 5].mean().item())
    return {"ms_per_advection_step": t / nsteps * 1e3, "substeps_per_step": sub,
            "us_per_substep_amortised": t / nsteps / sub * 1e6,
            "dt_ad": float(rec[:, 0].mean()),
            "pair_interactions_per_s": pairs * (2 + 2 * sub) / (t / nsteps),
            "note": "pairs counted once per neighbour sweep: density, prologue, and a "
                    "pressure and a continuity sweep per substep"}


def decay_accuracy(case, nsteps):
    """FP32 and FP64 runs of nsteps steps from the identical start (the FP32
    state widened exactly), kinetic energy against the analytic Taylor-Green
    decay KE(0) exp(-16 pi^2 t / Re) of Eq. (17)."""
    import copy
    import math
    import numpy as np
    from paper_2411_13992_amd import Simulation
    s32 = Simulation.from_case(case, dtype="f32")
    st = s32.export()
    start = copy.copy(case)
    start.pos, start.vel = st["pos"], st["vel"]
    s64 = Simulation.from_case(start, dtype="f64")
    ke0 = float(0.5 * np.sum(case.mass * np.sum(st["vel"] ** 2, axis=0)))
    s32.run(nsteps, diag=False)
    s64.run(nsteps, diag=False)
    ke32 = s32.diagnostics(fresh=True)["ke"]
    ke64 = s64.diagnostics(fresh=True)["ke"]
    t = nsteps * case.dt
    exact = ke0 * math.exp(-16 * math.pi ** 2 * t / case.extra.get("re", 100.0))
    return {"steps": nsteps, "t": t, "ke_vs_analytic_f32": ke32 / exact - 1.0,
            "ke_vs_analytic_f64": ke64 / exact - 1.0, "ke_f32_vs_f64": ke32 / ke64 - 1.0}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_median_step(case, threads, warm, reps):
    """Median wall time of `reps` whole oracle steps after `warm` untimed
    ones, on `threads` OpenMP threads, and the mean ordered pair count."""
    import oracle
    oracle.set_threads(threads)
    st = oracle.State(case)
    for _ in range(warm):
        st.step()
    times, pairs = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        d = st.step()
        times.append(time.perf_counter() - t0)
        pairs.append(d["npairs"])
    times.sort()
    return times[len(times) // 2], sum(pairs) / len(pairs)


def cpu_baseline(case):
    """The FP64 oracle, as it stands, on the same workload: the median time of
    a whole step after two warm-up steps, once on every host thread (the
    reported value) and once single-threaded; about 10-20 s in all."""
    import oracle
    threads = os.cpu_count() or 1
    oracle.set_threads(threads)
    threads = oracle.get_threads()
    t_all, pairs = _oracle_median_step(case, threads, 2, 20)
    t_one, _ = _oracle_median_step(case, 1, 2, 5)
    oracle.set_threads(threads)
    return {"value": pairs / t_all, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"median of 20 whole FP64 steps (after 2 warm-up steps) of the "
                      f"{case.n}-particle workload on {threads} threads, neighbour search by "
                      f"cells; single-threaded: median of 5 steps",
            "s_per_step": t_all,
            "single_thread": {"value": pairs / t_one, "s_per_step": t_one, "cores": 1},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(WORKLOADS),
                    help="the 2-D benchmark workload (default) or one of the larger "
                         "parity workloads, reported on the same line format")
    ap.add_argument("--pmc", action="store_true",
                    help="counter run: 20 force-sweep launches on the benchmark state and one "
                         "64 MiB device copy of known size (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import cases
    from paper_2411_13992_amd import Simulation

    case = cases.make(args.workload)
    default = args.workload == WORKLOAD
    sim = Simulation.from_case(case, dtype="f32")
    if args.pmc:
        # 20 launches each of the list sweeps (density recording the lists,
        # forces over them), FP32 then FP64, on the benchmark state after the
        # warm-up steps, then one copy of known size to calibrate the byte
        # counters
        for dt in ("f32", "f64"):
            s = sim if dt == "f32" else Simulation.from_case(case, dtype="f64")
            s.run(args.warmup)
            lists = s.neighbor_lists()
            out = torch.empty_like(s.acc)
            rho = torch.empty_like(s.rho)
            for _ in range(20):
                s.density_lists(lists, out=rho)
            for _ in range(20):
                s.forces_lists(lists, out=out)
            torch.cuda.synchronize()
        src = torch.ones(PMC_COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_run": True, "force_launches": 20, "density_launches": 20,
                          "copy_bytes": PMC_COPY_BYTES}))
        return
    steps, warmup = args.steps, args.warmup
    if case.n > 500_000:     # 10-30x the work per step: keep the timed region short
        steps, warmup = max(steps // 10, 5), max(warmup // 10, 2)
    t32, pairs = time_steps(sim, steps, warmup)
    roof = kernel_roofline(sim, pairs, "f32", reps=200 if default else 20, use_pmc=default)
    flags32 = sim.flags()
    del sim
    sim64 = Simulation.from_case(case, dtype="f64")
    t64, pairs64 = time_steps(sim64, max(steps // 2, 1), max(warmup // 2, 1))
    del sim64
    simadj = Simulation.from_case(case, dtype="f32")
    t_fwd, t_bwd = time_adjoint(simadj, 40, 20)
    del simadj
    adjoint = {"forward_ms_per_step": t_fwd * 1e3, "reverse_ms_per_step": t_bwd * 1e3,
               "adjoint_over_forward": t_bwd / t_fwd,
               "rollout": "40 FP32 steps, checkpoints every 20, reverse includes "
                          "recomputation with tapes"}
    out = {
        "metric": METRIC,
        "value": pairs / t32,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload,
                   "particles": case.n, "pairs_per_step": pairs, "dt": case.dt},
        "fp64": {"value": pairs64 / t64, "ms_per_step": t64 * 1e3,
                 "fp32_speedup": t64 / t32},
        "adjoint": adjoint,
        "roofline": roof,
        "device_flags": flags32,
    }
    if case.dim == 2 and not case.n_wall and case.uniform:
        out["step_roofline"] = step_bounds(case.n, pairs, t32)
    if args.workload == WORKLOAD:
        out["accuracy"] = decay_accuracy(case, case.steps)
        out["dual_criteria"] = time_dual(case)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
