"""MI355X-native hot path of the transport-velocity WCSPH method
(Wang, Haidn & Hu, arXiv 2411.13992): cell-linked-list neighbour search,
density summation, Riemann pressure and viscous forces, the smoothing-length
scaled transport-velocity correction with its limiter, and kick-drift-kick
integration, as hand-written HIP kernels for gfx950 behind the C-ABI library
libsph (include/sph.h).  PyTorch supplies device memory and streams only.
"""
from ._lib import SphError, load as load_library, lattice_kappa  # noqa: F401

__all__ = ["SphError", "load_library", "lattice_kappa", "Simulation", "Config",
           "config_from_case", "StepFlagError"]


def __getattr__(name):
    # the torch-based driver is imported on first use
    if name in ("Simulation", "Config", "config_from_case", "make_params", "StepFlagError"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
