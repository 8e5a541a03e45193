"""Modal and Cholesky theta-methods for eddy-current transients on MI355X.

Python front end of libmm (HIP kernels for gfx950 behind a C ABI, see
include/mm.h).  It follows Ventre et al., "Modal Decomposition in Numerical
Computation of Eddy Current Transients" (arXiv 2407.11993), Sec. 3.
"""
from .solver import Solver, kernels  # noqa: F401
