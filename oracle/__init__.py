"""CPU FP64 oracle for the project-and-normalize (PQR) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
directory; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path: it is plain numpy in float64, written to be read against the paper
(Dreier & Engwer, "A Hardware-aware and Stable Orthogonalization Framework",
arXiv 2204.13393), not to be fast.

Modules
-------
householder  Householder QR (Sec. 2.2 / Golub-Van Loan) with the positive
             diagonal sign fix that makes the thin QR unique.
pqr          The PQR problem, eq. (1.1): the unique reference solution
             (block CGS twice with Householder inner QR), BCGS-PIP and
             BCGS-PIP+ (Sec. 3, Sec. 3.1) and a breakdown-detecting
             Cholesky.
hhpqr        The Householder method for the PQR problem (Sec. 2.2,
             Algorithm "HH"), the basis held as unit reflectors.
deflate      Deflation of BCGS-PIP(+) by the truncated eigen decomposition
             of G - P^T P (Sec. 3.1) and the deflated PQR solution from
             the SVD of the residual.
tspqr        TreeTSPQR (Sec. 4.1) with the locally orthogonal basis
             representation, single- and multi-level trees; BCGS-PIP,
             BCGS-PIP+ or Householder leaves.
flattspqr    FlatTSPQR (Sec. 4.2): the basis as a chain of per-block
             factors, the local problems solved one after another.
krylov       Block Arnoldi (Sec. 2, Algorithm "Block Arnoldi") and the
             block-column QR driver (Sec. 2, Algorithm "Block Column-oriented
             QR-factorization").
operators    2D/3D 5/7-point Laplacians and their closed-form spectra
             (the test operator; the paper names none).
metrics      e_perp (Sec. 2), residuals, Pythagoras defect, Arnoldi relation.

Readings of the paper that the oracle adopts where the text is silent,
ambiguous or garbled are listed in the docstrings of the functions that
depend on them.  Pins that tie every function to something other than
itself live in ``tests/test_oracle_*.py``.
"""

from .householder import householder_qr, house
from .pqr import (Breakdown, cholesky_upper, triu_solve_right, pqr_reference,
                  bcgs_pip, bcgs_pip_plus, SUBALGORITHMS)
from .hhpqr import HouseholderBasis, hh_pqr
from .deflate import (truncated_sqrt, deflating_pip, deflating_pip_plus,
                      pqr_deflated_reference)
from .tspqr import TreeTSPQR, leaf_bounds
from .flattspqr import FlatTSPQR
from .krylov import block_arnoldi, block_column_qr
from . import operators, metrics

__all__ = [
    "householder_qr", "house", "Breakdown", "cholesky_upper",
    "triu_solve_right", "pqr_reference", "bcgs_pip", "bcgs_pip_plus",
    "SUBALGORITHMS", "HouseholderBasis", "hh_pqr", "truncated_sqrt",
    "deflating_pip", "deflating_pip_plus", "pqr_deflated_reference", "TreeTSPQR", "FlatTSPQR", "leaf_bounds", "block_arnoldi",
    "block_column_qr", "operators", "metrics",
]
