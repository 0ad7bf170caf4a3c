"""MI355X-native V-cycle multigrid for lowest-order hexahedral Nedelec H(curl) problems.

The library ``libndmg.so`` (C ABI in ``include/ndmg.h``) holds every computation; this
package is its binding.  Importing the package does not load the library; the first
solver does, and fails loudly if it has not been built.
"""
from . import synth  # noqa: F401

__all__ = ["Solver", "BatchedSolver", "solve", "synth"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name == "BatchedSolver":
        from .solver import BatchedSolver
        return BatchedSolver
    if name == "solve":
        from .autograd import solve
        return solve
    raise AttributeError(name)
