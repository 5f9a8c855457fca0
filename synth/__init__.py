"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws random numbers and fixes workload shapes; it holds none of
the orthogonalisation arithmetic.  Orthonormal factors needed to build
Stewart matrices come from numpy's LAPACK QR, not from this project's
oracle or kernels.

Recipes
-------
normal_block(n, s, seed)
    numpy.random.default_rng(seed).standard_normal((n, s)): row-major draw
    order, element (r, c) is draw r*s + c.  Start blocks of the Arnoldi
    workloads ("N(0,1), seed 0").
stewart(n, m, kappa, seed)
    Sec. 6.1: X = U diag(sigma) V^T with U (n x m) and V (m x m) Haar
    orthonormal (QR of Gaussian matrices, sign-fixed) and sigma log-spaced
    from 1 down to 1/kappa: sigma_j = kappa^(-j/(m-1)).  The paper leaves the
    random distribution and the exact spacing open; this is the reading.
"""

from .gen import normal_block, stewart, haar, column_major, from_column_major
from .workloads import WORKLOADS, Workload, grid_for

__all__ = ["normal_block", "stewart", "haar", "column_major",
           "from_column_major", "WORKLOADS", "Workload", "grid_for"]
