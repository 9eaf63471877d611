"""MI355X-native hot path of the centroidal-Taylor P1 discontinuous Galerkin scheme
(Mocz et al. 2013) for the Euler and ideal-MHD equations.

The compute path is the HIP library ``libdg.so`` behind the C ABI ``include/dg.h``;
this package holds its ctypes binding and torch-facing wrappers.
"""
from . import capi  # noqa: F401

__all__ = ["capi", "Solver", "cartesian"]


def __getattr__(name):
    if name in ("Solver", "cartesian"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
