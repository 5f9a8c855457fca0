"""The project-and-normalize (PQR) problem in FP64 (oracle; test only).

PQR problem, eq. (1.1): given Q (n x k) with orthonormal columns and a new
block X (n x s), find U (n x s) with Q^T U = 0 and

    [Q X] = [Q U] [[I, P], [0, N]],   P = Q^T X (k x s),  N (s x s) upper.

For full rank [Q X] and diag(N) > 0 the solution is unique (it is the thin
QR of [Q X] with the known leading block): P = Q^T X, N is the Cholesky
factor of (X - QP)^T (X - QP) = X^T X - P^T P (Sec. 3), U = (X - QP) N^{-1}.

Functions
---------
pqr_reference   the unique solution computed stably: block classical
                Gram-Schmidt applied twice (Algorithms "BCGS" and "BCGS+",
                Sec. 2.1) with Householder QR as the inner factorisation.
bcgs_pip        Algorithm "BCGS-PIP" (Sec. 3): P and G = X^T X in one sweep,
                N^T N = G - P^T P, U = (X - QP) N^{-1}.  O(eps kappa^2).
bcgs_pip_plus   Algorithm "BCGS-PIP+" (Sec. 3.1): BCGS-PIP twice.  O(eps)
                while eps kappa^2 <= 1/2.

Reading adopted for the reiteration combination.  The paper prints
"P = P1 N2 + P2 and N = N2 + N1 N2" for both BCGS+ and BCGS-PIP+.  That does
not follow from the two factorisations it combines:
    [Q X]  = [Q U1] [[I, P1], [0, N1]]
    [Q U1] = [Q U ] [[I, P2], [0, N2]]
give [Q X] = [Q U] [[I, P1 + P2 N1], [0, N2 N1]], so the oracle uses
P = P1 + P2 N1 and N = N2 N1 (pinned by the residual and closed-form tests).
"""

import numpy as np

from .householder import householder_qr


class Breakdown(ArithmeticError):
    """Cholesky met a pivot that is not positive and finite.

    Sec. 3.1 notes that the textbook Cholesky factorisation is not
    rank-revealing; the oracle reports breakdown instead of deflating
    (deflation by a truncated SVD of G - P^T P is ``oracle.deflate``).
    """

    def __init__(self, index, pivot):
        super().__init__(f"Cholesky breakdown at column {index}: pivot {pivot!r}")
        self.index = index
        self.pivot = pivot


def cholesky_upper(S):
    """Upper Cholesky factor N with N^T N = S and diag(N) > 0.

    Plain column-by-column algorithm (Golub-Van Loan Sec. 4.2).  Raises
    Breakdown when a pivot (the value before the square root) is <= 0 or
    not finite; no threshold is applied.
    """
    S = np.array(S, dtype=np.float64, copy=True)
    s = S.shape[0]
    N = np.zeros((s, s), dtype=np.float64)
    for j in range(s):
        pivot = S[j, j] - np.dot(N[:j, j], N[:j, j])
        if not np.isfinite(pivot) or pivot <= 0.0:
            raise Breakdown(j, pivot)
        d = np.sqrt(pivot)
        N[j, j] = d
        for c in range(j + 1, s):
            N[j, c] = (S[j, c] - np.dot(N[:j, j], N[:j, c])) / d
    return N


def triu_solve_right(Y, N):
    """Return Y N^{-1} for upper-triangular N by forward substitution on columns.

    Column c of Z = Y N^{-1} satisfies sum_{i<=c} Z[:, i] N[i, c] = Y[:, c].
    """
    Y = np.asarray(Y, dtype=np.float64)
    s = N.shape[0]
    Z = np.zeros_like(Y)
    for c in range(s):
        acc = Y[:, c].copy()
        for i in range(c):
            acc -= Z[:, i] * N[i, c]
        Z[:, c] = acc / N[c, c]
    return Z


def _as_basis(Q, n):
    if Q is None:
        return np.zeros((n, 0), dtype=np.float64)
    return np.asarray(Q, dtype=np.float64)


def pqr_reference(Q, X):
    """Unique PQR solution (P, N, U) via BCGS2 with Householder inner QR.

    Block classical Gram-Schmidt (Sec. 2.1, Algorithm "BCGS": P = Q^T X,
    U~ = X - QP, U~ = UN by QR) applied twice (Algorithm "BCGS+"), with
    the Householder QR as the inner factorisation and the corrected
    combination P = P1 + P2 N1, N = N2 N1.  The inner QR is sign-fixed so
    diag(N) > 0.  Q may be None or have zero columns (k = 0): then the
    result is the thin QR of X.
    """
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    Q = _as_basis(Q, n)
    P1 = Q.T @ X
    U1, N1 = householder_qr(X - Q @ P1)
    P2 = Q.T @ U1
    U, N2 = householder_qr(U1 - Q @ P2)
    P = P1 + P2 @ N1
    N = N2 @ N1
    return P, N, U


def bcgs_pip(Q, X):
    """Algorithm "BCGS-PIP" (Sec. 3): CholQR applied to the PQR problem.

    P = Q^T X and G = X^T X computed from one sweep over the rows, the
    Cholesky factor N of G - P^T P (N^T N), then U = X N^{-1} - Q P N^{-1}.
    Returns (P, N, U); raises Breakdown when G - P^T P is not numerically
    positive definite.
    """
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    Q = _as_basis(Q, n)
    P = Q.T @ X
    G = X.T @ X
    N = cholesky_upper(G - P.T @ P)
    U = triu_solve_right(X - Q @ P, N)
    return P, N, U


def bcgs_pip_plus(Q, X):
    """Algorithm "BCGS-PIP+" (Sec. 3.1): BCGS-PIP applied twice.

    (P1, N1, U1) = BCGS-PIP(Q, X); (P2, N2, U) = BCGS-PIP(Q, U1);
    P = P1 + P2 N1, N = N2 N1 (corrected combination, see module notes).
    """
    P1, N1, U1 = bcgs_pip(Q, X)
    P2, N2, U = bcgs_pip(Q, U1)
    return P1 + P2 @ N1, N2 @ N1, U


# subalgorithm table used by TreeTSPQR (local and reduction choices, Sec. 4.1)
SUBALGORITHMS = {
    "pip": bcgs_pip,
    "pip+": bcgs_pip_plus,
    "ref": pqr_reference,
}
