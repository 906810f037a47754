"""MI355X-native multigrid solver for the variable-density pressure-Poisson
equation of a volume-of-fluid flow solver (HIP kernels for gfx950 behind a
C ABI, include/mgp.h).  torch supplies device memory and streams only."""
from ._lib import MgError, load as load_library  # noqa: F401

__all__ = ["MgError", "load_library", "Solver", "SolveStats", "faces_from_vof", "divergence",
           "poisson_solve", "plan_levels"]


def __getattr__(name):
    # torch-dependent parts are imported lazily so that the C ABI can be
    # inspected without initialising torch
    if name in ("Solver", "SolveStats", "faces_from_vof", "divergence", "plan_levels"):
        from . import solver
        return getattr(solver, name)
    if name == "poisson_solve":
        from .autograd import poisson_solve
        return poisson_solve
    raise AttributeError(name)
