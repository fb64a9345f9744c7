"""BBWADG on MI355X: Bernstein-Bezier weight-adjusted DG for the 3D acoustic wave
equation on affine tetrahedra, with hand-written HIP kernels for gfx950 behind a C ABI
(include/bbwadg.h) and this thin Python binding."""
from .bbwadg import (BBWADGError, Solver, coef_index, dimp, load_library, projection_coefficients,  # noqa: F401
                     LIB_PATH, EXPORTS)

__version__ = "0.1"
