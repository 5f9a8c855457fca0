"""Pins for the oracle's Householder QR (CPU only).

* library pin: LAPACK QR (numpy.linalg.qr) after the positive-diagonal sign fix;
* brute force: exact Gram in rationals + 60-digit Cholesky on tiny integer
  matrices gives the unique R (and Q = A R^{-1});
* closed form: the Householder vector maps x to alpha e_1 with
  |alpha| = ||x|| and the sign opposite to x_0 (Sec. 2.2).
"""

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import householder_qr, house

U = 2.0 ** -53


def _lapack_unique_qr(A):
    Q, R = np.linalg.qr(A)
    d = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * d, d[:, None] * R


@pytest.mark.parametrize("shape", [(1, 1), (5, 1), (7, 7), (40, 6), (300, 17), (1000, 32)])
def test_householder_matches_lapack(shape):
    rng = np.random.default_rng(hash(shape) % 2**32)
    A = rng.standard_normal(shape)
    Q, R = householder_qr(A)
    Ql, Rl = _lapack_unique_qr(A)
    m, n = shape
    assert Q.shape == (m, n) and R.shape == (n, n)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(R, -1), 0.0)
    tol = 200 * U * np.sqrt(m * n)
    assert np.linalg.norm(R - Rl) / np.linalg.norm(Rl) < tol
    assert np.linalg.norm(Q - Ql) / np.sqrt(n) < tol * np.linalg.cond(A)
    assert np.linalg.norm(np.eye(n) - Q.T @ Q) < 50 * U * np.sqrt(m) * n


def _exact_qr(Aint, digits=60):
    """Unique R of a full-rank integer matrix from the exact Gram matrix."""
    m, n = Aint.shape
    G = [[sum(Fraction(int(Aint[r, i])) * int(Aint[r, j]) for r in range(m)) for j in range(n)]
         for i in range(n)]
    getcontext().prec = digits
    Gd = [[Decimal(g.numerator) / Decimal(g.denominator) for g in row] for row in G]
    R = [[Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        piv = Gd[j][j] - sum(R[i][j] * R[i][j] for i in range(j))
        assert piv > 0
        R[j][j] = piv.sqrt()
        for c in range(j + 1, n):
            R[j][c] = (Gd[j][c] - sum(R[i][j] * R[i][c] for i in range(j))) / R[j][j]
    return np.array([[float(x) for x in row] for row in R])


@pytest.mark.parametrize("seed", range(6))
def test_householder_brute_force_tiny_integer(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(3, 13))
    n = int(rng.integers(1, min(m, 6) + 1))
    while True:
        A = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
        if np.linalg.matrix_rank(A) == n:
            break
    R_exact = _exact_qr(A.astype(int))
    Q_exact = np.linalg.solve(R_exact.T, A.T).T
    Q, R = householder_qr(A)
    kappa = np.linalg.cond(A)
    assert np.max(np.abs(R - R_exact)) <= 100 * U * kappa * np.max(np.abs(R_exact))
    assert np.max(np.abs(Q - Q_exact)) <= 100 * U * kappa


@pytest.mark.parametrize("x", [[3.0, 4.0], [-3.0, 4.0], [0.0, 2.0, 0.0], [5.0], [-1e-300, 1.0, 1.0]])
def test_house_reflects_to_alpha_e1(x):
    x = np.array(x)
    v, beta, alpha = house(x)
    Hx = x - beta * v * (v @ x)
    assert abs(abs(alpha) - np.linalg.norm(x)) <= 4 * U * np.linalg.norm(x)
    expect_sign = -1.0 if x[0] >= 0 else 1.0
    assert np.sign(alpha) == expect_sign
    assert abs(Hx[0] - alpha) <= 8 * U * np.linalg.norm(x)
    assert np.all(np.abs(Hx[1:]) <= 8 * U * np.linalg.norm(x))


def test_householder_zero_column_keeps_shape():
    A = np.zeros((5, 2))
    A[:, 1] = 1.0
    Q, R = householder_qr(A)
    assert R[0, 0] == 0.0
    assert np.allclose(Q @ R, A)
