"""Lid-driven cavity studies on the GPU: the unit square of Sec. 4.2 (top
wall moving at U = 1, Re = U L / nu = 1000) and the unit cube of the
three-dimensional cavity section (lid velocity (1, 0, 0), Re = 100), run to
t_end at several resolutions dp = 1/n with the limited correction (Eq. 16)
and, for comparison, the unlimited h-scaled one (Eq. 14).  Reported: the
horizontal velocity u along the vertical centre line x = L/2 and the vertical
velocity v along the horizontal centre line y = L/2 (in the middle plane
z = L/2 in 3-D), and their self-convergence (the paper's reference data are
not used here: only differences between resolutions).

    python -m paper_2411_13992_amd.cavity [--dim 2] [--n 50 100 200] [--t-end 30]
        [--modes limited scaled] [--dtype f32] [--json out.json]

Every step runs through sph_kdk_run.  The centre-line values are
kernel-weighted (Shepard) averages of the fluid particles' velocities at the
probe points, evaluated on the host from the exported FP64 state
(post-processing, outside the hot path).
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

PROBES = np.linspace(0.025, 0.975, 39)


def shepard(points: np.ndarray, pos: np.ndarray, values: np.ndarray, h: float) -> np.ndarray:
    """Kernel-weighted averages of `values` (k, N) at `points` (2, P) over the
    particles within 2h (Wendland C2 weights (1 - q/2)^4 (1 + 2q), q = r/h)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(pos.T)
    out = np.zeros((values.shape[0], points.shape[1]))
    for p, nb in enumerate(tree.query_ball_point(points.T, 2.0 * h)):
        if not nb:
            out[:, p] = np.nan
            continue
        nb = np.asarray(nb)
        q = np.linalg.norm(pos[:, nb] - points[:, [p]], axis=0) / h
        w = (1.0 - 0.5 * q) ** 4 * (1.0 + 2.0 * q)
        out[:, p] = values[:, nb] @ w / w.sum()
    return out


def centre_lines(case, state: dict) -> dict:
    """u(x = 1/2, y) and v(x, y = 1/2) at PROBES (cavity coordinates; z = 1/2
    in 3-D)."""
    nf = case.n_fluid
    o = case.extra["origin"]
    pos = state["pos"][:, :nf] - o
    vel = state["vel"][:, :nf]
    h = float(case.h_min)
    half = np.full_like(PROBES, 0.5)
    vline = np.stack([half, PROBES] + [half] * (case.dim - 2))
    hline = np.stack([PROBES, half] + [half] * (case.dim - 2))
    return {"y": PROBES.tolist(), "u": shepard(vline, pos, vel[:1], h)[0].tolist(),
            "x": PROBES.tolist(), "v": shepard(hline, pos, vel[1:2], h)[0].tolist()}


def run(n: int, t_end: float, mode: str = "limited", dtype: str = "f32",
        re: float | None = None, chunk: int = 5000, dim: int = 2) -> dict:
    import torch

    import cases
    from .sim import Simulation

    case = cases.lid_driven_cavity(n, re=re, dim=dim)
    re = case.extra["re"]
    sim = Simulation.from_case(case, dtype=dtype, tv_mode=mode)
    nsteps = int(round(t_end / case.dt))
    ke = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    last = time.perf_counter()
    while done < nsteps:
        k = min(chunk, nsteps - done)
        d = sim.run(k, diag=True)
        ke.append(float(d[-1, 0]))
        done += k
        if time.perf_counter() - last > 30.0:      # progress on long runs
            last = time.perf_counter()
            print(f"  {mode} n {n}: t = {done * case.dt:.2f} of {nsteps * case.dt:.2f}, "
                  f"KE {ke[-1]:.5f}", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    state = sim.export()
    # steadiness: relative change of the kinetic energy over the last tenth of the run
    tenth = max(len(ke) // 10, 1)
    drift = abs(ke[-1] - ke[-1 - tenth]) / ke[-1] if len(ke) > tenth else float("nan")
    out = {"n": n, "dim": dim, "mode": mode, "dtype": dtype, "re": re, "particles": case.n,
           "fluid": case.n_fluid, "dt": case.dt, "steps": nsteps, "t": nsteps * case.dt,
           "wall_s": wall, "us_per_step": wall / nsteps * 1e6, "flags": sim.flags(),
           "ke_per_chunk": ke, "ke_final": ke[-1], "ke_change_last_tenth": drift}
    out.update(centre_lines(case, state))
    return out


def convergence(runs: list) -> dict:
    """RMS differences of the centre-line profiles between successive
    resolutions and the observed order log2(e_coarse / e_fine) (resolutions
    doubling)."""
    runs = sorted(runs, key=lambda r: r["n"])
    diffs = []
    for a, b in zip(runs, runs[1:]):
        du = np.asarray(b["u"]) - np.asarray(a["u"])
        dv = np.asarray(b["v"]) - np.asarray(a["v"])
        diffs.append({"from": a["n"], "to": b["n"],
                      "rms_u": float(np.sqrt(np.mean(du ** 2))),
                      "rms_v": float(np.sqrt(np.mean(dv ** 2)))})
    orders = []
    for a, b in zip(diffs, diffs[1:]):
        ratio = b["to"] / a["to"]
        orders.append({"at": b["to"],
                       "order_u": math.log(a["rms_u"] / b["rms_u"]) / math.log(ratio),
                       "order_v": math.log(a["rms_v"] / b["rms_v"]) / math.log(ratio)})
    return {"differences": diffs, "orders": orders}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[50, 100, 200],
                    help="particles per side (dp = 1/n)")
    ap.add_argument("--t-end", type=float, default=30.0)
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3))
    ap.add_argument("--re", type=float, default=None,
                    help="Reynolds number (default 1000 in 2-D, 100 in 3-D)")
    ap.add_argument("--chunk", type=int, default=5000, help="steps per fused run")
    ap.add_argument("--dtype", default="f32", choices=("f32", "f64"))
    ap.add_argument("--modes", nargs="+", default=["limited", "scaled"],
                    choices=("limited", "scaled", "background"))
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    result = {"runs": [], "convergence": {}, "formulations": []}
    for mode in args.modes:
        runs = []
        for n in args.n:
            r = run(n, args.t_end, mode, args.dtype, args.re, args.chunk, args.dim)
            runs.append(r)
            print(f"{mode:8s} n {n:4d} ({r['particles']} particles, {r['steps']} steps, "
                  f"{r['wall_s']:.1f} s, {r['us_per_step']:.1f} us/step) flags {r['flags']}; "
                  f"KE {r['ke_final']:.5f} (last tenth: {100 * r['ke_change_last_tenth']:.2f}%); "
                  f"u(0.5, y) min {np.nanmin(r['u']):+.4f}, v(x, 0.5) range "
                  f"[{np.nanmin(r['v']):+.4f}, {np.nanmax(r['v']):+.4f}]", flush=True)
        result["runs"] += runs
        if len(runs) > 1:
            c = convergence(runs)
            result["convergence"][mode] = c
            for d in c["differences"]:
                print(f"{mode:8s} dp 1/{d['from']} -> 1/{d['to']}: rms change u {d['rms_u']:.2e}, "
                      f"v {d['rms_v']:.2e}", flush=True)
            for o in c["orders"]:
                print(f"{mode:8s} observed order at 1/{o['at']}: u {o['order_u']:.2f}, "
                      f"v {o['order_v']:.2f}", flush=True)
    if len(args.modes) > 1:
        for n in args.n:
            by = {r["mode"]: r for r in result["runs"] if r["n"] == n}
            ms = list(by)
            a, b = by[ms[0]], by[ms[1]]
            du = float(np.sqrt(np.mean((np.asarray(a["u"]) - np.asarray(b["u"])) ** 2)))
            dv = float(np.sqrt(np.mean((np.asarray(a["v"]) - np.asarray(b["v"])) ** 2)))
            result["formulations"].append({"n": n, "modes": ms[:2], "rms_u": du, "rms_v": dv})
            print(f"n {n}: {ms[0]} vs {ms[1]}: rms difference u {du:.2e}, v {dv:.2e}", flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(result, f)
    return result


if __name__ == "__main__":
    main()
