"""Device state and step driver over the libsph C-ABI.

PyTorch provides device memory and the stream; every computation runs in the
library's HIP kernels.  The state is kept in (cell, id) order as the library
leaves it; ``export()`` maps it back to particle-id order in FP64.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Config:
    """Physical and numerical parameters of a run (symbols as in the paper)."""
    dim: int
    box: tuple
    rho0: float
    c0: float
    eta: float
    dt: float
    h_min: float
    h_max: float
    mass: float               # uniform mass (ignored when per-particle masses are given)
    xi: float = -0.2          # Eq. 14/16
    lim_c: float = 1.0e3      # Eq. 15
    lim_s0: float = 5.0e-4    # Eq. 15
    riemann_eta: float = 3.0  # Eq. 6
    tv_every: int = 1
    tv_mode: str = "limited"  # "limited" (Eq. 16), "scaled" (Eq. 14), "background" (Eq. 12)
    band_tol: float = 1.0e-5
    h_over_dx: float = 1.3    # Sec. 4: h = 1.3 dp, fixes the reference kernel sum
    ncell: tuple | None = None
    lanes: int = 0            # lanes per particle in the sweeps (0: chosen by size)
    u_ref: float = 1.0        # reference speed of Eq. 10 (dual-criteria stepping)

    def cells(self):
        if self.ncell is not None:
            return tuple(self.ncell)
        return tuple(int(math.floor(b / (2.0 * self.h_max) * (1.0 - 1e-12))) for b in self.box)


def config_from_case(case, **overrides) -> Config:
    cfg = Config(dim=case.dim, box=tuple(case.box), rho0=case.rho0, c0=case.c0, eta=case.eta,
                 dt=case.dt, h_min=case.h_min, h_max=case.h_max, mass=float(case.mass[0]),
                 xi=case.xi, lim_c=case.lim_c, lim_s0=case.lim_s0,
                 riemann_eta=case.riemann_eta, u_ref=case.u_ref)
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def make_params(cfg: Config, n: int, dtype: str, per_particle: bool = False) -> _lib.SphParams:
    p = _lib.SphParams()
    p.per_particle = 1 if per_particle else 0
    p.dim = cfg.dim
    p.dtype = _lib.SPH_F64 if dtype == "f64" else _lib.SPH_F32
    p.n = n
    nc = cfg.cells()
    for k in range(3):
        p.ncell[k] = nc[k] if k < cfg.dim else 1
        p.box[k] = cfg.box[k] if k < cfg.dim else 1.0
    p.tv_every = cfg.tv_every
    p.tv_mode = _lib.TV_MODES[cfg.tv_mode]
    p.rho0, p.c0, p.eta = cfg.rho0, cfg.c0, cfg.eta
    p.h_min, p.h_max, p.mass = cfg.h_min, cfg.h_max, cfg.mass
    p.kappa = _lib.lattice_kappa(cfg.dim, cfg.h_over_dx)
    p.dt, p.xi, p.lim_c, p.lim_s0 = cfg.dt, cfg.xi, cfg.lim_c, cfg.lim_s0
    p.riemann_eta, p.band_tol = cfg.riemann_eta, cfg.band_tol
    p.lanes = cfg.lanes
    return p


class StepFlagError(RuntimeError):
    """A fused run raised a device flag; the state was restored to the
    snapshot taken before that run (step_index is where it stands now)."""

    def __init__(self, flags: int, step_index: int):
        names = [n for bit, n in ((_lib.FLAG_NONFINITE, "non-finite value"),
                                  (_lib.FLAG_CFL, "a particle moved more than one cell"),
                                  (_lib.FLAG_OUT_OF_BOX, "position outside the box"),
                                  (_lib.FLAG_INTERNAL, "internal wait gave up")) if flags & bit]
        super().__init__(f"device flags {flags:#x} ({', '.join(names)}); state restored to "
                         f"step {step_index}")
        self.flags = flags
        self.step_index = step_index


class Simulation:
    """Particles on one GPU advanced by libsph's kick-drift-kick step."""

    def __init__(self, cfg: Config, pos, vel, mass=None, h=None, dtype: str = "f32",
                 device: str = "cuda", wall_vel=None):
        """pos, vel: (D, N) FP64 in particle-id order.  wall_vel: (D, n_wall)
        prescribed velocities of wall particles, which are the last n_wall ids."""
        _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a GPU (HIP device); there is no CPU path")
        self.cfg = cfg
        self.dim = cfg.dim
        self.dtype = dtype
        self.T = torch.float64 if dtype == "f64" else torch.float32
        self.device = torch.device(device)
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.n = int(pos.shape[1])
        self.var = mass is not None
        self.params = make_params(cfg, self.n, dtype, self.var)
        self.n_wall = 0 if wall_vel is None else int(np.asarray(wall_vel).shape[1])
        self.params.n_wall = self.n_wall
        d, n, dev, T = self.dim, self.n, self.device, self.T
        self.ws_bytes = _lib.workspace_size(self.params)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.cell = torch.zeros(n, dtype=torch.int32, device=dev)
        self.id = torch.arange(n, dtype=torch.int32, device=dev)
        self.off = torch.zeros((d, n), dtype=T, device=dev)
        self.vel = torch.as_tensor(np.asarray(vel, dtype=np.float64), device=dev).to(T).contiguous()
        self.acc = torch.zeros((d, n), dtype=T, device=dev)
        self.rho = torch.zeros(n, dtype=T, device=dev)
        self.mass = (torch.as_tensor(np.asarray(mass, dtype=np.float64), device=dev).to(T)
                     .contiguous() if self.var else None)
        self.h = (torch.as_tensor(np.asarray(h, dtype=np.float64), device=dev).to(T).contiguous()
                  if self.var else None)
        self.wall_vel = (torch.as_tensor(np.asarray(wall_vel, dtype=np.float64), device=dev)
                         .to(T).contiguous() if self.n_wall else None)
        ncells = int(np.prod(cfg.cells()[:d]))
        self.ncells = ncells
        self.cs = torch.zeros(ncells + 1, dtype=torch.int32, device=dev)
        # the last step's diagnostics: this buffer after step(), a view of the
        # last row after run() (no copy launch)
        self._diag_own = torch.zeros(_lib.SPH_NDIAG, dtype=torch.float64, device=dev)
        self.diag = self._diag_own
        self.step_index = 0
        # step index at which the last run() or step() left the state (None once
        # anything else touched the state, params or workspace): run(resume=True)
        # continues only from there
        self._resume_at = None
        pos_dev = torch.as_tensor(pos, device=dev).contiguous()
        s = _stream()
        _lib.call("sph_bin_positions", ctypes.byref(self.params), _vp(pos_dev),
                  ctypes.byref(self.parts()), _vp(self.ws), self.ws_bytes, s)
        self.build_cells()
        self.init_fields()
        torch.cuda.current_stream().synchronize()
        del pos_dev
        self.initial = self.snapshot()

    @classmethod
    def from_case(cls, case, dtype: str = "f32", **overrides):
        cfg = config_from_case(case, **overrides)
        wv = case.wall_vel if getattr(case, "n_wall", 0) else None
        if case.uniform:
            return cls(cfg, case.pos, case.vel, dtype=dtype, wall_vel=wv)
        return cls(cfg, case.pos, case.vel, mass=case.mass, h=case.h, dtype=dtype, wall_vel=wv)

    # ------------------------------------------------------------ plumbing
    def parts(self) -> _lib.SphParticles:
        p = _lib.SphParticles()
        p.cell, p.id = self.cell.data_ptr(), self.id.data_ptr()
        p.off, p.vel, p.acc, p.rho = (self.off.data_ptr(), self.vel.data_ptr(),
                                      self.acc.data_ptr(), self.rho.data_ptr())
        p.mass = self.mass.data_ptr() if self.var else None
        p.h = self.h.data_ptr() if self.var else None
        p.wall_vel = self.wall_vel.data_ptr() if self.n_wall else None
        return p

    # ------------------------------------------------------------ hot path
    def build_cells(self, perm: torch.Tensor | None = None) -> None:
        self._resume_at = None
        _lib.call("sph_build_cells", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(perm), _vp(self.ws), self.ws_bytes, _stream())

    def density(self, out: torch.Tensor | None = None) -> torch.Tensor:
        self._resume_at = None
        out = self.rho if out is None else out
        _lib.call("sph_density", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(out), _stream())
        return out

    def forces(self, vel: torch.Tensor | None = None, out: torch.Tensor | None = None):
        self._resume_at = None
        vel = self.vel if vel is None else vel
        out = self.acc if out is None else out
        _lib.call("sph_forces", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(vel), _vp(out), _stream())
        return out

    def neighbor_lists(self) -> torch.Tensor:
        """A device buffer for the stored neighbour lists (sph_list_size bytes)."""
        self._resume_at = None
        nbytes = _lib.list_size(self.params)
        if nbytes == 0:
            raise RuntimeError("stored neighbour lists cannot index this many particles")
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def density_lists(self, lists: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """sph_density that also records the neighbour lists into `lists`."""
        self._resume_at = None
        out = self.rho if out is None else out
        _lib.call("sph_density_lists", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(out), _vp(lists), lists.numel(), _stream())
        return out

    def forces_lists(self, lists: torch.Tensor, vel: torch.Tensor | None = None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """sph_forces over lists recorded by density_lists at the same state."""
        self._resume_at = None
        vel = self.vel if vel is None else vel
        out = self.acc if out is None else out
        _lib.call("sph_forces_lists", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(vel), _vp(out), _vp(lists), lists.numel(), _stream())
        return out

    def tv_correction(self):
        """Eq. 14-16 at the current state: dict of dr, beta, s (FP64), g."""
        self._resume_at = None
        d, n, dev, T = self.dim, self.n, self.device, self.T
        out = {"dr": torch.zeros((d, n), dtype=T, device=dev),
               "beta": torch.zeros(n, dtype=T, device=dev),
               "s": torch.zeros(n, dtype=torch.float64, device=dev),
               "g": torch.zeros((d, n), dtype=T, device=dev)}
        _lib.call("sph_tv_correction", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(out["dr"]), _vp(out["beta"]), _vp(out["s"]), _vp(out["g"]),
                  _stream())
        return out

    def neighbor_counts(self) -> torch.Tensor:
        self._resume_at = None
        out = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        _lib.call("sph_neighbor_counts", ctypes.byref(self.params), ctypes.byref(self.parts()),
                  _vp(self.cs), _vp(out), _stream())
        return out

    def wall_state(self) -> None:
        """Wall particles' density and no-slip mirror velocity from the fluid
        (sph_wall_state); nothing without walls."""
        self._resume_at = None
        if self.n_wall:
            _lib.call("sph_wall_state", ctypes.byref(self.params), ctypes.byref(self.parts()),
                      _vp(self.cs), _stream())

    def init_fields(self) -> None:
        """rho^0 by summation (Eq. 8), the walls' state, and a^0 from the
        initial velocity."""
        self._resume_at = None
        self.density()
        self.wall_state()
        self.forces()

    def step(self, nsteps: int = 1, diag: bool = True,
             tape: torch.Tensor | None = None) -> None:
        """nsteps kick-drift-kick steps; with `tape` (sph_tape_size bytes) one
        step is recorded for the adjoint."""
        if tape is not None and nsteps != 1:
            raise ValueError("a tape records exactly one step")
        parts = self.parts()
        s = _stream()
        self.diag = self._diag_own
        for _ in range(nsteps):
            _lib.call("sph_kdk_step", ctypes.byref(self.params), ctypes.byref(parts),
                      _vp(self.cs), self.step_index, _vp(self.ws), self.ws_bytes, _vp(tape),
                      _vp(self.diag) if diag else None, s)
            self.step_index += 1
            self._resume_at = self.step_index

    def run(self, nsteps: int, diag=True, tapes: torch.Tensor | None = None,
            resume: bool = False) -> torch.Tensor | None:
        """nsteps steps in one fused call (sph_kdk_run).  diag: True keeps every
        step's diagnostics (returned as an (nsteps, 9) FP64 device tensor;
        self.diag then views its last row), False skips them, or a preallocated
        (nsteps, 9) FP64 device tensor to fill.  tapes: optional uint8 device
        tensor of at least nsteps x tape_bytes() bytes (one tape per step,
        contiguous).  resume: continue the previous run() or step()
        (sph_kdk_run_resume: its first step's correction was evaluated by that
        call's last force sweep; bit-identical results); only valid when
        nothing has changed the particle tensors since then (refused when a
        method of this class did; writes into the tensors themselves are not
        seen), without tapes."""
        if nsteps <= 0:
            return None
        if diag is True:
            d = torch.empty((nsteps, _lib.SPH_NDIAG), dtype=torch.float64, device=self.device)
        elif diag is False or diag is None:
            d = None
        else:
            d = diag
        if tapes is not None:
            if (tapes.dtype != torch.uint8 or not tapes.is_contiguous()
                    or tapes.numel() < nsteps * self.tape_bytes()):
                raise ValueError("tapes must be a contiguous uint8 tensor of nsteps x tape_bytes()")
        if resume:
            if tapes is not None:
                raise ValueError("a resumed run records no tapes")
            if self._resume_at != self.step_index:
                raise ValueError("resume needs the state a run() or step() left, untouched")
            _lib.call("sph_kdk_run_resume", ctypes.byref(self.params), ctypes.byref(self.parts()),
                      _vp(self.cs), self.step_index, nsteps, _vp(self.ws), self.ws_bytes,
                      _vp(d), _stream())
        else:
            _lib.call("sph_kdk_run", ctypes.byref(self.params), ctypes.byref(self.parts()),
                      _vp(self.cs), self.step_index, nsteps, _vp(self.ws), self.ws_bytes,
                      _vp(tapes), _vp(d), _stream())
        if d is not None:
            self.diag = d[-1]
        self.step_index += nsteps
        self._resume_at = self.step_index
        return d

    def dual_run(self, nsteps: int, cfl_ad: float = 0.25, cfl_ac: float = 0.6,
                 max_substeps: int = 0, diag: bool = True):
        """nsteps advection steps of the dual-criteria scheme (sph_dual_run):
        the correction once per advection step, acoustic substeps with the
        continuity equation, step sizes of Eq. 9-11 chosen on the device.
        Returns (diagnostics rows (nsteps, 9), step records (nsteps, 3):
        dt_ad, substeps, time covered), FP64 device tensors."""
        self._resume_at = None
        q = _lib.SphDualParams(cfl_ad=cfl_ad, cfl_ac=cfl_ac, u_ref=self.cfg.u_ref,
                               nu=self.cfg.eta / self.cfg.rho0, max_substeps=max_substeps)
        d = (torch.empty((nsteps, _lib.SPH_NDIAG), dtype=torch.float64, device=self.device)
             if diag else None)
        rec = torch.empty((nsteps, 3), dtype=torch.float64, device=self.device)
        _lib.call("sph_dual_run", ctypes.byref(self.params), ctypes.byref(q),
                  ctypes.byref(self.parts()), _vp(self.cs), nsteps, _vp(self.ws), self.ws_bytes,
                  _vp(d), _vp(rec), _stream())
        if d is not None and nsteps > 0:
            self.diag = d[-1]
        self.step_index += nsteps
        return d, rec

    def diag_rows(self, nsteps: int) -> torch.Tensor:
        """Device buffer for the per-step diagnostics of a run."""
        return torch.empty((nsteps, _lib.SPH_NDIAG), dtype=torch.float64, device=self.device)

    def tape_bytes(self) -> int:
        return _lib.tape_size(self.params)

    def set_xi(self, xi: float) -> None:
        self._resume_at = None
        self.params.xi = float(xi)

    # ------------------------------------------------------------ checkpoints
    _STATE = ("cell", "id", "off", "vel", "acc", "rho", "cs")

    def snapshot(self) -> dict:
        snap = {k: getattr(self, k).clone() for k in self._STATE}
        if self.var:
            snap["mass"] = self.mass.clone()
            snap["h"] = self.h.clone()
        snap["step_index"] = self.step_index
        return snap

    def restore(self, snap: dict) -> None:
        self._resume_at = None
        for k in self._STATE:
            getattr(self, k).copy_(snap[k])
        if self.var:
            self.mass.copy_(snap["mass"])
            self.h.copy_(snap["h"])
        self.step_index = snap["step_index"]

    def set_velocity(self, vel_by_id: torch.Tensor) -> None:
        """Replace velocities from an id-ordered (D, N) tensor."""
        self._resume_at = None
        self.vel.copy_(vel_by_id.to(self.device, self.T)[:, self.id.long()])

    def velocity_by_id(self) -> torch.Tensor:
        out = torch.empty_like(self.vel)
        out[:, self.id.long()] = self.vel
        return out

    def diagnostics(self, fresh: bool = False) -> dict:
        """FP64 diagnostics of the last step (or of the current state alone)."""
        if fresh:
            self._resume_at = None
            self.diag = self._diag_own
            _lib.call("sph_diagnostics", ctypes.byref(self.params), ctypes.byref(self.parts()),
                      _vp(self.cs), _vp(self.ws), self.ws_bytes, _vp(self.diag), _stream())
        vals = self.diag.cpu().numpy()
        return dict(zip(_lib.DIAG_NAMES, vals))

    # ------------------------------------------------------------ recovery
    def save_checkpoint(self, path: str) -> None:
        """Write the state (sorted arrays, cell_start, step index, and the
        run parameters it belongs to) to an uncompressed .npz file; no
        pickled objects, so np.load with its default allow_pickle=False reads
        it back."""
        arrays = {k: getattr(self, k).cpu().numpy() for k in self._STATE}
        if self.var:
            arrays["mass"] = self.mass.cpu().numpy()
            arrays["h"] = self.h.cpu().numpy()
        if self.n_wall:
            arrays["wall_vel"] = self.wall_vel.cpu().numpy()
        arrays["step_index"] = np.array(self.step_index, dtype=np.int64)
        arrays["params"] = np.frombuffer(bytes(self.params), dtype=np.uint8)
        np.savez(path, **arrays)

    def load_checkpoint(self, path: str) -> None:
        """Restore a state written by save_checkpoint for the same run
        parameters (checked byte for byte, xi aside)."""
        self._resume_at = None
        with np.load(path) as z:
            mine = bytearray(bytes(self.params))
            theirs = bytearray(z["params"].tobytes())
            off = _lib.SphParams.xi.offset
            mine[off:off + 8] = theirs[off:off + 8] = bytes(8)
            if mine != theirs:
                raise ValueError(f"{path}: checkpoint of a different configuration")
            for k in self._STATE:
                getattr(self, k).copy_(torch.from_numpy(z[k]))
            if self.var:
                self.mass.copy_(torch.from_numpy(z["mass"]))
                self.h.copy_(torch.from_numpy(z["h"]))
            if self.n_wall:
                self.wall_vel.copy_(torch.from_numpy(z["wall_vel"]))
            self.step_index = int(z["step_index"])

    def run_checked(self, nsteps: int, chunk: int = 500, diag=False) -> int:
        """nsteps steps in fused runs of at most `chunk`, checking the device
        flags after each; a run that raised a flag (non-finite value, a
        particle moving more than a cell in a step, ...) is undone: the state
        goes back to the snapshot taken before it and StepFlagError reports
        the flag word and the step index reached (recovery: restart from the
        last good state, e.g. with a smaller dt).  Returns the steps done."""
        done = 0
        while done < nsteps:
            k = min(chunk, nsteps - done)
            snap = self.snapshot()
            self.run(k, diag=diag)
            f = self.flags()
            if f:
                self.restore(snap)
                raise StepFlagError(f, self.step_index)
            done += k
        return done

    def flags(self) -> int:
        out = ctypes.c_uint32(0)
        _lib.call("sph_get_flags", _vp(self.ws), _stream(), ctypes.byref(out))
        return int(out.value)

    # ------------------------------------------------------------ export
    def positions_fp64(self, cell=None, off=None) -> np.ndarray:
        """Absolute FP64 positions (sorted order): cell origin + offset."""
        cell = (self.cell if cell is None else cell).cpu().numpy().astype(np.int64)
        off = (self.off if off is None else off).cpu().numpy().astype(np.float64)
        nc = self.cfg.cells()
        idx = [cell % nc[0]]
        rest = cell // nc[0]
        if self.dim == 3:
            idx += [rest % nc[1], rest // nc[1]]
        else:
            idx += [rest]
        pos = np.empty_like(off)
        for k in range(self.dim):
            L = self.cfg.box[k] / nc[k]
            pos[k] = idx[k].astype(np.float64) * L + off[k]
        return pos

    def export(self) -> dict:
        """State in particle-id order, widened exactly to FP64."""
        ids = self.id.cpu().numpy().astype(np.int64)
        order = np.argsort(ids)
        out = {
            "pos": self.positions_fp64()[:, order],
            "vel": self.vel.cpu().double().numpy()[:, order],
            "acc": self.acc.cpu().double().numpy()[:, order],
            "rho": self.rho.cpu().double().numpy()[order],
            "order": order,
        }
        if self.var:
            out["mass"] = self.mass.cpu().double().numpy()[order]
            out["h"] = self.h.cpu().double().numpy()[order]
        return out
