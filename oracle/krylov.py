"""Drivers that consume a PQR solver (oracle; test infrastructure).

block_arnoldi     Sec. 2, Algorithm "Block Arnoldi": V_0 from the QR of the
                  start block R (R = V_0 H_0), then per step X = A V_i, solve
                  the PQR problem for [V X], append U, and grow the block
                  Hessenberg matrix by the column block [P; N].
block_column_qr   Sec. 2, Algorithm "Block Column-oriented QR-factorization":
                  QR of A by solving the PQR problem on its s-column blocks.
                  Reading adopted for the listing's index typos ("U_u", the
                  loop bounds): block j is columns [s j, s (j+1)), j = 0..m/s-1,
                  the first block is factorised with an empty basis, and R
                  collects the column blocks [P; N].

Both accept either a stateless explicit-basis solver ``pqr(Q, X) -> (P, N, U)``
or a stateful object with ``step(X) -> (P, N, U)`` (e.g. ``TreeTSPQR``), whose
basis stays in its own representation.
"""

import numpy as np

from .householder import householder_qr
from .pqr import pqr_reference


class _Explicit:
    """Explicit-basis wrapper so both solver kinds share one driver loop."""

    def __init__(self, pqr, n):
        self.pqr = pqr
        self.Q = np.zeros((n, 0))

    def step(self, X):
        P, N, U = self.pqr(self.Q, X)
        self.Q = np.hstack([self.Q, U])
        return P, N, U


def _solver(pqr, n):
    if pqr is None:
        pqr = pqr_reference
    return pqr if hasattr(pqr, "step") else _Explicit(pqr, n)


def block_arnoldi(apply_A, R, steps, pqr=None):
    """Run ``steps`` block-Arnoldi steps from start block R (n x s).

    Returns (V, H, H0, blocks):
      V   explicit basis n x (steps+1)s (assembled from the returned U blocks),
      H   block Hessenberg ((steps+1)s x steps s) with A V[:, :steps s] = V H,
      H0  s x s upper factor with R = V_0 H0,
      blocks  the list of X_i = A V_{i-1} fed to the solver (for open-loop use).
    The first QR uses the solver itself with an empty basis (k = 0), which is
    the QR factorisation of Algorithm "Block Arnoldi", first line.
    """
    R = np.asarray(R, dtype=np.float64)
    n, s = R.shape
    solver = _solver(pqr, n)
    _, H0, V0 = solver.step(R)
    Vs = [V0]
    H = np.zeros(((steps + 1) * s, steps * s))
    blocks = []
    Vi = V0
    for i in range(steps):
        X = apply_A(Vi)
        blocks.append(X)
        P, N, U = solver.step(X)
        H[:(i + 1) * s, i * s:(i + 1) * s] = P
        H[(i + 1) * s:(i + 2) * s, i * s:(i + 1) * s] = N
        Vs.append(U)
        Vi = U
    return np.hstack(Vs), H, H0, blocks


def block_column_qr(A, s, pqr=None):
    """QR of A (n x m, s | m) by the PQR problem on s-column blocks.

    Returns (Q, R) with Q = the concatenated U blocks and R upper triangular.
    """
    A = np.asarray(A, dtype=np.float64)
    n, m = A.shape
    if m % s:
        raise ValueError("m must be a multiple of s")
    solver = _solver(pqr, n)
    R = np.zeros((m, m))
    Us = []
    for j in range(m // s):
        P, N, U = solver.step(A[:, j * s:(j + 1) * s])
        R[:j * s, j * s:(j + 1) * s] = P
        R[j * s:(j + 1) * s, j * s:(j + 1) * s] = N
        Us.append(U)
    return np.hstack(Us), R


def householder_arnoldi_start(R):
    """V_0, H_0 of the first Arnoldi line via Householder QR (R = V_0 H_0)."""
    return householder_qr(R)
