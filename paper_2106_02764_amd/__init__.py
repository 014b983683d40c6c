"""MI355X (gfx950) aMFP-BTE hot path: C-ABI HIP library + thin Python binding.

The library (libobte.so, built from csrc/ by build.py) implements the
source iteration of the anisotropic-MFP phonon BTE; this package only
marshals arguments to it.  Importing the binding requires the built library:
there is no CPU fallback.
"""
from . import autotune, obte
from .obte import ObteError, default_opts, lib
from .solver import KappaEff, Solver, UMeshSolver, solve_batch

__all__ = ["obte", "ObteError", "default_opts", "lib", "Solver", "UMeshSolver", "KappaEff", "solve_batch"]
