"""MI355X (gfx950) two-level nonlinear Schwarz: HIP library libnls and its
Python binding.  See include/nls.h for the C ABI."""
from .nls import Solver, load, NLSError, SYMBOLS  # noqa: F401
