"""BBWADG on MI355X: Bernstein-Bezier weight-adjusted DG for the 3D acoustic wave
equation on affine tetrahedra, with hand-written HIP kernels for gfx950 behind a C ABI
(include/bbwadg.h) and this thin Python binding."""
from .bbwadg import (BBWADGError, Solver, bernstein_positivity, coef_index, dimp, load_library,  # noqa: F401
                     projection_coefficients,
                     LIB_PATH, EXPORTS)

__version__ = "0.1"
