"""Differentiable rollout: gradients of a loss on the final velocities with
respect to the initial velocities and the correction coefficient xi (Eq. 14/16).

Forward: N kick-drift-kick steps, keeping a state checkpoint every K steps.
Backward: for each segment, last first, restore its checkpoint, recompute its
K steps in one fused run recording a tape per step (sph_kdk_run with tapes),
then run the reverse steps (sph_adjoint_step) from the last step of the
segment back to its first.  The initial evaluation (rho^0 by summation, a^0 from v^0) is
reversed last (sph_adjoint_init).  The neighbour sets are held fixed within
a step (the C2 kernel and its first two derivatives vanish at the support
edge), and the limiter's jump at s0 contributes no derivative.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .sim import Simulation, _stream, _vp


class Adjoint:
    """Cotangent buffers of one state (sorted order), in the sweep precision."""

    def __init__(self, sim: Simulation):
        d, n, dev, T = sim.dim, sim.n, sim.device, sim.T
        self.r = torch.zeros((d, n), dtype=T, device=dev)
        self.v = torch.zeros((d, n), dtype=T, device=dev)
        self.a = torch.zeros((d, n), dtype=T, device=dev)
        self.rho = torch.zeros(n, dtype=T, device=dev)

    def abi(self) -> _lib.SphAdjoint:
        a = _lib.SphAdjoint()
        a.r_bar, a.v_bar = self.r.data_ptr(), self.v.data_ptr()
        a.a_bar, a.rho_bar = self.a.data_ptr(), self.rho.data_ptr()
        return a


def adjoint_step(sim: Simulation, tape: torch.Tensor, adj: Adjoint, xi_bar: torch.Tensor):
    _lib.call("sph_adjoint_step", ctypes.byref(sim.params), _vp(tape), ctypes.byref(adj.abi()),
              _vp(xi_bar), _vp(sim.ws), sim.ws_bytes, _stream())


def adjoint_init(sim: Simulation, adj: Adjoint):
    _lib.call("sph_adjoint_init", ctypes.byref(sim.params), ctypes.byref(sim.parts()),
              _vp(sim.cs), ctypes.byref(adj.abi()), _vp(sim.ws), sim.ws_bytes, _stream())


def forward_run(sim: Simulation, v0: torch.Tensor, xi: float, nsteps: int, every: int | None):
    """Start from the simulation's initial positions with velocities v0 (id
    order), run nsteps; returns the checkpoints (every `every` steps)."""
    sim.set_xi(xi)
    sim.restore(sim.initial)
    sim.set_velocity(v0)
    sim.init_fields()
    ckpts = []
    s = 0
    while s < nsteps:
        chunk = min(every, nsteps - s) if every else nsteps - s
        if every:
            ckpts.append(sim.snapshot())
        sim.run(chunk, diag=False)
        s += chunk
    return ckpts


def backward_run(sim: Simulation, ckpts: list, nsteps: int, every: int,
                 v_bar_final: torch.Tensor, final_id: torch.Tensor,
                 tapes: torch.Tensor | None = None):
    """Reverse sweep.  v_bar_final is id-ordered; final_id is the sorted id
    order of the rollout's final state (sim.id right after forward_run), so the
    simulation may have been stepped or restored since.  The simulation's state
    is the same on return as on entry.  Returns (v0_bar id-ordered, r0_bar
    id-ordered, xi_bar float)."""
    entry = sim.snapshot()
    adj = Adjoint(sim)
    adj.v.copy_(v_bar_final.to(sim.device, sim.T)[:, final_id.long()])
    xi_bar = torch.zeros(1, dtype=torch.float64, device=sim.device)
    if tapes is None:
        tapes = torch.empty((every, sim.tape_bytes()), dtype=torch.uint8, device=sim.device)
    nseg = (nsteps + every - 1) // every
    for seg in reversed(range(nseg)):
        start = seg * every
        stop = min(start + every, nsteps)
        sim.restore(ckpts[seg])
        sim.run(stop - start, diag=False, tapes=tapes)
        for s in reversed(range(start, stop)):
            adjoint_step(sim, tapes[s - start], adj, xi_bar)
    sim.restore(ckpts[0])
    adjoint_init(sim, adj)
    ids = sim.id.long()
    v0_bar = torch.empty_like(adj.v)
    v0_bar[:, ids] = adj.v
    r0_bar = torch.empty_like(adj.r)
    r0_bar[:, ids] = adj.r
    sim.restore(entry)
    return v0_bar, r0_bar, float(xi_bar.item())


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v0, xi, sim, nsteps, every):
        ckpts = forward_run(sim, v0.detach(), float(xi), nsteps, every)
        ctx.sim, ctx.nsteps, ctx.every, ctx.ckpts = sim, nsteps, every, ckpts
        ctx.final_id = sim.id.clone()
        ctx.xi = float(xi)
        ctx.v0_dtype, ctx.xi_dtype = v0.dtype, xi.dtype
        return sim.velocity_by_id().to(v0.dtype)

    @staticmethod
    def backward(ctx, grad_v):
        sim = ctx.sim
        xi_now = sim.params.xi
        sim.set_xi(ctx.xi)
        v0_bar, _, xi_bar = backward_run(sim, ctx.ckpts, ctx.nsteps, ctx.every, grad_v,
                                         ctx.final_id)
        sim.set_xi(xi_now)
        xi_grad = torch.tensor(xi_bar, dtype=ctx.xi_dtype, device=grad_v.device)
        return v0_bar.to(ctx.v0_dtype), xi_grad, None, None, None


def rollout(sim: Simulation, v0: torch.Tensor, xi: torch.Tensor, nsteps: int,
            every: int = 20) -> torch.Tensor:
    """Final velocities (id order) after nsteps steps from the simulation's
    initial positions with initial velocities v0 (id order) and correction
    coefficient xi; differentiable in v0 and xi."""
    if not torch.is_tensor(xi):
        xi = torch.tensor(float(xi), dtype=torch.float64, device=v0.device)
    return _Rollout.apply(v0, xi, sim, nsteps, every)


def kinetic_energy(sim: Simulation, vel_by_id: torch.Tensor) -> torch.Tensor:
    """1/2 sum m |v|^2 over the fluid particles in FP64 (a torch loss on the
    rollout output; wall particles, the last n_wall ids, carry their no-slip
    mirror velocity and are left out)."""
    if sim.var:
        m = torch.empty(sim.n, dtype=torch.float64, device=sim.device)
        m[sim.id.long()] = sim.mass.double()
    else:
        m = torch.full((sim.n,), float(sim.cfg.mass), dtype=torch.float64, device=sim.device)
    nf = sim.n - sim.n_wall
    return 0.5 * (m[:nf] * (vel_by_id[:, :nf].double() ** 2).sum(0)).sum()
