"""Accuracy metrics (oracle side; test infrastructure).

e_perp             Sec. 2: e_perp = ||I - Q^T Q||_F (Frobenius, as defined there).
pqr_residual       ||X - Q P - U N||_F / ||X||_F for one PQR step, eq. (1.1).
qr_residual        ||A - Q R||_F / ||A||_F (the paper's tables print ||A - QR||
                   without naming the norm; Stewart matrices have ||A||_2 = 1,
                   the relative Frobenius value is reported).
pythagoras_defect  | ||X||_F^2 - ||P||_F^2 - ||N||_F^2 | / ||X||_F^2: for
                   [Q X] = [Q U][[I,P],[0,N]] with [Q U] orthonormal,
                   ||X||^2 = ||QP + UN||^2 = ||P||^2 + ||N||^2 (Sec. 3,
                   the Pythagorean identity behind BCGS-PIP).
arnoldi_relation   ||A V_j - V_{j+1} H||_F / (||A||_2 sqrt(K)).
"""

import numpy as np


def e_perp(Q):
    Q = np.asarray(Q, dtype=np.float64)
    k = Q.shape[1]
    return float(np.linalg.norm(np.eye(k) - Q.T @ Q, "fro"))


def pqr_residual(Q, X, P, N, U):
    X = np.asarray(X, dtype=np.float64)
    R = X - U @ N
    if Q is not None and Q.shape[1]:
        R = R - Q @ P
    return float(np.linalg.norm(R, "fro") / np.linalg.norm(X, "fro"))


def qr_residual(A, Q, R):
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - Q @ R, "fro") / np.linalg.norm(A, "fro"))


def pythagoras_defect(X, P, N):
    x2 = float(np.sum(np.asarray(X, dtype=np.float64) ** 2))
    p2 = float(np.sum(np.asarray(P) ** 2)) if P is not None else 0.0
    n2 = float(np.sum(np.asarray(N) ** 2))
    return abs(x2 - p2 - n2) / x2


def arnoldi_relation(apply_A, V, H, norm_A):
    K = H.shape[1]
    AV = apply_A(V[:, :K])
    return float(np.linalg.norm(AV - V[:, :H.shape[0]] @ H, "fro") / (norm_A * np.sqrt(H.shape[0])))
