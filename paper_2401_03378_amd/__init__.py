"""MI355X-native FP64 block-structured compressible-Euler step.

One explicit SSP-RK step of a finite-volume Euler solver over a table of
guard-cell-padded blocks (guard gather, PLM-MC or WENO5 reconstruction of
primitives, HLLC fluxes, flux-difference update, ideal-gas EOS, CFL dt),
run by hand-written HIP kernels for gfx950 behind the C ABI of
include/hydro.h.  PyTorch supplies device memory and streams only.

Submodules: workloads (seeded inputs), solver (Solver), adjoint
(HydroStep autograd Function, checkpointed rollout), autotune.
"""
from . import workloads  # noqa: F401  (inputs only; no GPU needed)

__all__ = ["workloads", "Solver"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
