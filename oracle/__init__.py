"""Oracle: a plain, slow, FP64 CPU implementation of the Laplace-EIG hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or run anything here.  The product
path (paper_1502_07873_amd) never imports it, and the oracle never imports
the product: the two share no code.  Inputs come from the separate
`synthetic` package, which holds no method arithmetic.

Contents and the passages they follow (Long, Motamed & Tempone, "Fast Bayesian
optimal experimental design for seismic source inversion"):
  fd_oracle.c   leapfrog solve of the 2-D elastic wave equation
                (Section 3.3.1, full-discrete scheme; operator = minus the
                gradient of the discrete elastic energy, see the file header)
  elastic.py    regularised delta / delta' source weights (Section 3.3.2),
                point moment-tensor source (Section 2.1), wavelets
                (Section 4.1), receiver traces (Section 2.2), central-
                difference Jacobian
  laplace.py    H_1 (Theorem 2), scaled Hessian and log-det (Section 3.3.3),
                D^_KL (Theorem 4), Monte Carlo / quadrature averages
                (Section 3.3.4), design sums and greedy search (Section 4.5)
  smolyak.py    Gauss-Legendre total-degree sparse grids (Sections 3.3.4, 4.3)
  pipeline.py   the per-query composition of the above

Every function is pinned by tests/test_oracle_*.py against properties the
paper and the mathematics fix; none is "parity unpinned".
"""
from . import elastic, laplace, pipeline, smolyak  # noqa: F401
from ._clib import build  # noqa: F401
