"""MI355X Laplace-EIG engine for 2-D seismic source design.

The hot path (forward solves, central-difference Jacobians, Gauss-Newton
Hessians, scaled Cholesky log-determinants, quadrature averages and design
search) runs in HIP kernels in libeigseis.so behind the C ABI declared in
include/eigseis.h; `eigseis` is its ctypes binding and `query` composes the
calls for one design query.  Importing fails loudly when the library has
not been built.
"""
from . import eigseis  # noqa: F401
from .eigseis import Context, EigError, make_prior, sparse_grid_gl  # noqa: F401
