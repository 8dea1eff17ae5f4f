"""MI355X iHDG library: Python binding of libihdg.so (see include/ihdg.h)."""
from .binding import (CD, FP64, MIXED, SHALLOW_WATER, TRANSPORT, Batch, IhdgError, Solver, footprint,
                      library_path, load, quadrature_points, sizes)

__all__ = ["Solver", "Batch", "IhdgError", "sizes", "quadrature_points", "footprint", "load", "library_path",
           "TRANSPORT", "SHALLOW_WATER", "CD", "FP64", "MIXED"]
