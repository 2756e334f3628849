"""MI355X (gfx950) explicit finite-difference wave propagation.

The solver is libfd.so (HIP kernels behind the C ABI of include/fd.h); this
package binds it (``_binding``: same entry-point names, argument marshalling
only) and wraps it for torch tensors (``solver.Solver``).  The library is
loaded on first use and its absence is an error: there is no CPU fallback.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import lib  # noqa: F401

__all__ = [n for n in dir() if n.startswith(("fd_", "FD_"))] + ["lib", "FdGrid", "FdModel",
                                                                 "FdPoints", "FdError",
                                                                 "make_grid", "EXPORTS"]
