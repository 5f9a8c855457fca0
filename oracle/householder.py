"""Householder QR in FP64 (oracle; test infrastructure only).

The paper's Householder method (Sec. 2.2, eq. (2.4) and Algorithm "HH")
stores the basis as a product of reflectors H_i = I - 2 v_i v_i^T with unit
v_i, chooses the reflector sign opposite to the leading entry to avoid
cancellation, and cites Golub & Van Loan, Ch. 5 for the details.  The
oracle follows that textbook form (Householder vector with beta = 2/(v^T v),
column-by-column triangularisation, backward accumulation of the thin Q)
rather than the index-garbled listing in the paper: the listing reads the
sign from the k-th entry of u~ and takes the norm over [k:n], where the
i-th column step needs entry k+i and range [k+i:n].

Uniqueness: for full column rank A the thin QR with diag(R) > 0 is unique.
The reflector convention may leave negative diagonal entries (the paper's
N[i,i] = sigma*lambda can be negative), so the result is sign-fixed with
D = diag(sign R_jj), sign(0) = +1:  R <- D R,  Q <- Q D.
"""

import numpy as np


def house(x):
    """Householder vector for x (Golub-Van Loan Sec. 5.1.2).

    Returns (v, beta, alpha) with (I - beta v v^T) x = alpha e_1, where
    alpha = -sign(x_0) ||x||_2 and sign(0) = +1 (the sign choice of the
    paper's Householder method: the opposite sign of the leading entry).
    beta = 0 when x is the zero vector.
    """
    x = np.asarray(x, dtype=np.float64)
    nrm = np.sqrt(np.dot(x, x))
    if nrm == 0.0:
        v = np.zeros_like(x)
        v[0] = 1.0
        return v, 0.0, 0.0
    sgn = 1.0 if x[0] >= 0.0 else -1.0
    alpha = -sgn * nrm
    v = x.copy()
    v[0] = x[0] - alpha          # = x0 + sign(x0) ||x||, no cancellation
    vtv = np.dot(v, v)
    beta = 2.0 / vtv
    return v, beta, alpha


def householder_qr(A):
    """Thin QR of A (m x n, m >= n) with diag(R) >= 0.

    Returns (Q, R): Q is m x n with orthonormal columns, R is n x n upper
    triangular with non-negative diagonal (positive for full column rank).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    if A.ndim != 2:
        raise ValueError("householder_qr expects a matrix")
    m, n = A.shape
    if m < n:
        raise ValueError("householder_qr needs m >= n (tall matrix)")
    vs = []
    betas = []
    for j in range(n):
        v, beta, alpha = house(A[j:, j])
        if beta != 0.0:
            # apply H_j = I - beta v v^T to the trailing block
            w = v @ A[j:, j:]
            A[j:, j:] -= beta * np.outer(v, w)
        A[j, j] = alpha if beta != 0.0 else A[j, j]
        A[j + 1:, j] = 0.0
        vs.append(v)
        betas.append(beta)
    R = np.triu(A[:n, :n])
    # thin Q = H_0 H_1 ... H_{n-1} [I_n; 0], accumulated backwards
    Q = np.zeros((m, n), dtype=np.float64)
    Q[:n, :n] = np.eye(n)
    for j in range(n - 1, -1, -1):
        v, beta = vs[j], betas[j]
        if beta != 0.0:
            w = v @ Q[j:, :]
            Q[j:, :] -= beta * np.outer(v, w)
    # sign fix: the thin QR with positive diagonal is the unique one
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    R = d[:, None] * R
    Q = Q * d[None, :]
    return Q, R
