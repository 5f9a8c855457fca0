"""Deflation of BCGS-PIP and BCGS-PIP+ (oracle; test infrastructure only).

Sec. 3.1: the textbook Cholesky factorisation cannot tell whether G - P^T P
has full rank, so the paper takes the eigen (singular value) decomposition
G - P^T P = V Lambda V^T, drops the eigenvalues below a tolerance and uses
the square root of what is left as the normalizer.  The block then has
rank t < s (the deflation case of eq. (1.1) in Sec. 1: N is t x s).

Readings adopted where the paper is silent or garbled:
* the printed square root puts the eigenvectors on the left (an s x t
  matrix); a normalizer with N^T N = G - P^T P has to be t x s, so it is
  N = Lambda~^{1/2} V~^T, the kept eigenvalues in decreasing order;
* the tolerance is relative to the block: an eigenvalue lambda is kept when
  lambda > (delta ||X||_F)^2, i.e. a direction stays when its residual
  singular value exceeds delta ||X||_F; ||X||_F^2 is the trace of G.  The
  Gram matrix carries rounding errors of about u ||X||_F^2, so directions
  below about sqrt(u) ||X||_F cannot be told from noise: delta should stay
  well above sqrt(u) (1e-6 in the tests);
* eigenvectors carry a sign: each kept one is turned so that its entry of
  largest magnitude (the first of them on a tie) is positive;
* the width stays s: rows t..s-1 of N and columns t..s-1 of U are exact
  zeros (a row-padded form of the t x s normalizer), so the basis grows by s
  columns of which s - t are zero.  A zero column of a later block stays zero
  and is deflated again;
* when nothing is dropped (t = s) the step is the plain Cholesky step, so
  deflation changes nothing for a full-rank block;
* BCGS-PIP+ deflates in its first sweep only: the second sweep runs the
  Cholesky factorisation on the t kept columns of U1 (whose other columns are
  zero), N2 = diag(L, 0), and the combination P = P1 + P2 N1, N = N2 N1 of
  the reiteration is unchanged.
"""

import numpy as np

from .pqr import bcgs_pip, cholesky_upper, pqr_reference, triu_solve_right, _as_basis


def sign_fix(v):
    """v turned so that its first entry of largest magnitude is positive."""
    i = int(np.argmax(np.abs(v)))
    return -v if v[i] < 0.0 else v


def truncated_sqrt(M, threshold):
    """Eigen decomposition of the symmetric s x s M with the small part dropped.

    Returns (t, N, W): t eigenvalues exceed ``threshold``; N (s x s) holds
    Lambda~^{1/2} V~^T in its first t rows and zeros below; W (s x s) holds
    V~ Lambda~^{-1/2} in its first t columns and zeros after, so that
    (X - QP) W is the deflated U and W N is the projector V~ V~^T.
    """
    M = np.asarray(M, dtype=np.float64)
    s = M.shape[0]
    lam, V = np.linalg.eigh(0.5 * (M + M.T))
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    t = int(np.count_nonzero(lam > threshold))
    N = np.zeros((s, s), dtype=np.float64)
    W = np.zeros((s, s), dtype=np.float64)
    for r in range(t):
        v = sign_fix(V[:, r])
        N[r, :] = np.sqrt(lam[r]) * v
        W[:, r] = v / np.sqrt(lam[r])
    return t, N, W


def deflating_pip(Q, X, delta):
    """BCGS-PIP (Sec. 3) with the deflation of Sec. 3.1.

    P = Q^T X and G = X^T X in one sweep; the eigen decomposition of
    G - P^T P decides the rank t; t = s is the plain Cholesky step, else
    N = Lambda~^{1/2} V~^T (rows padded with zeros) and U = (X - QP) W.
    Returns (P, N, U, t).
    """
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    Q = _as_basis(Q, n)
    P = Q.T @ X
    G = X.T @ X
    t, N, W = truncated_sqrt(G - P.T @ P, delta * delta * np.trace(G))
    if t == s:
        P, N, U = bcgs_pip(Q, X)
        return P, N, U, t
    U = (X - Q @ P) @ W
    return P, N, U, t


def deflating_pip_plus(Q, X, delta):
    """BCGS-PIP+ (Sec. 3.1) with deflation in the first sweep.

    The second sweep factors the t kept columns of U1 by Cholesky; the
    combination is P = P1 + P2 N1, N = N2 N1 as for the plain reiteration.
    Returns (P, N, U, t).
    """
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    Q = _as_basis(Q, n)
    P1, N1, U1, t = deflating_pip(Q, X, delta)
    P2 = Q.T @ U1
    G2 = U1.T @ U1
    N2 = np.zeros((s, s), dtype=np.float64)
    U = np.zeros((n, s), dtype=np.float64)
    if t:
        L = cholesky_upper((G2 - P2.T @ P2)[:t, :t])
        N2[:t, :t] = L
        U[:, :t] = triu_solve_right((U1 - Q @ P2)[:, :t], L)
    return P1 + P2 @ N1, N2 @ N1, U, t


def pqr_deflated_reference(Q, X, delta):
    """The deflated PQR solution from its definition (no Gram matrices).

    P = Q^T X; the residual R = X - QP (projected twice, as in BCGS2, so that
    it is orthogonal to Q to rounding); the SVD R = Y Sigma Z^T; t singular
    values exceed delta ||X||_F; U = [Y_t 0], N = [Sigma_t Z_t^T; 0] with
    each Z column turned by ``sign_fix`` and Y_t = R Z_t Sigma_t^{-1}.  With
    nothing dropped (t = s) it is the unique full-rank solution (triangular
    N, positive diagonal) of ``pqr_reference``.  Returns (P, N, U, t).
    """
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    Q = _as_basis(Q, n)
    P = Q.T @ X
    R = X - Q @ P
    R = R - Q @ (Q.T @ R)
    _, sig, Zt = np.linalg.svd(R, full_matrices=False)
    t = int(np.count_nonzero(sig > delta * np.linalg.norm(X)))
    if t == s:
        return pqr_reference(Q, X) + (s,)
    N = np.zeros((s, s), dtype=np.float64)
    U = np.zeros((n, s), dtype=np.float64)
    for r in range(t):
        z = sign_fix(Zt[r])
        N[r, :] = sig[r] * z
        U[:, r] = R @ z / sig[r]
    return P, N, U, t
