"""Seeded generators (no orthogonalisation arithmetic of this project)."""

import numpy as np


def normal_block(n, s, seed):
    """N(0,1) block, n x s float64; element (r, c) is draw r*s + c of default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((n, s))


def haar(n, m, rng):
    """n x m matrix with Haar-distributed orthonormal columns (numpy QR, sign-fixed)."""
    G = rng.standard_normal((n, m))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def stewart(n, m, kappa, seed):
    """Stewart matrix X = U diag(sigma) V^T with sigma_j = kappa^(-j/(m-1))."""
    rng = np.random.default_rng(seed)
    U = haar(n, m, rng)
    V = haar(m, m, rng)
    if m > 1:
        sigma = kappa ** (-np.arange(m) / (m - 1.0))
    else:
        sigma = np.ones(1)
    return (U * sigma[None, :]) @ V.T


def column_major(X):
    """Row-major numpy (n x s) -> contiguous (s x n) array = column-major n x s, ld = n."""
    return np.ascontiguousarray(np.asarray(X, dtype=np.float64).T)


def from_column_major(Xcm, n=None):
    """Inverse of ``column_major``: (s x ld) buffer -> n x s array."""
    Xcm = np.asarray(Xcm)
    if n is None:
        n = Xcm.shape[1]
    return np.ascontiguousarray(Xcm[:, :n].T)
