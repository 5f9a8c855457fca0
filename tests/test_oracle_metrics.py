"""Pins of the oracle's metrics against hand-computed values.

e_perp is the Frobenius norm ||I - Q^T Q||_F (Sec. 2).  The matrices below
are chosen so that the Frobenius value differs from the 2-norm and from
the max-abs entry, so a norm slip fails them; the residuals are checked on
cases small enough to do by hand.
"""

import math

import numpy as np

from oracle import metrics


def test_e_perp_hand_matrix_frobenius_not_two_norm():
    # Q^T Q = [[1, 1], [1, 2]], I - Q^T Q = [[0, -1], [-1, -1]]:
    # Frobenius sqrt(3); 2-norm (1 + sqrt 5) / 2; max-abs 1
    Q = np.array([[1.0, 1.0], [0.0, 1.0]])
    assert metrics.e_perp(Q) == math.sqrt(3.0)
    assert abs(metrics.e_perp(Q) - (1.0 + math.sqrt(5.0)) / 2.0) > 0.1


def test_e_perp_scaled_columns():
    # columns of norms sqrt 2 and sqrt 3, orthogonal: I - Q^T Q = diag(-1, -2),
    # Frobenius sqrt 5 (the 2-norm would be 2)
    Q = np.array([[math.sqrt(2.0), 0.0], [0.0, math.sqrt(3.0)], [0.0, 0.0]])
    assert abs(metrics.e_perp(Q) - math.sqrt(5.0)) <= 1e-15


def test_e_perp_orthonormal_is_zero_and_tall():
    # exactly orthonormal columns (a permutation of unit vectors): 0
    Q = np.zeros((5, 3))
    Q[4, 0] = Q[0, 1] = Q[2, 2] = 1.0
    assert metrics.e_perp(Q) == 0.0
    # one column doubled: I - Q^T Q has a single entry -3 on the diagonal
    Q[:, 1] *= 2.0
    assert metrics.e_perp(Q) == 3.0


def test_pqr_residual_by_hand():
    # X = Q P + U N exactly except for a known defect in one entry
    Q = np.array([[1.0], [0.0], [0.0]])
    U = np.array([[0.0], [1.0], [0.0]])
    P = np.array([[2.0]])
    N = np.array([[3.0]])
    X = np.array([[2.0], [3.0], [4.0]])      # defect (0, 0, 4); ||X||_F = sqrt(29)
    assert abs(metrics.pqr_residual(Q, X, P, N, U) - 4.0 / math.sqrt(29.0)) <= 1e-15
    # no basis: X - U N only
    assert abs(metrics.pqr_residual(None, X, None, N, U) - math.sqrt(4.0 + 16.0) / math.sqrt(29.0)) <= 1e-15


def test_qr_residual_and_pythagoras_by_hand():
    A = np.array([[3.0, 0.0], [4.0, 5.0]])
    Q = np.array([[0.6, -0.8], [0.8, 0.6]])
    R = np.array([[5.0, 4.0], [0.0, 3.0]])          # Q R = A exactly
    assert metrics.qr_residual(A, Q, R) <= 1e-15
    R2 = R.copy()
    R2[1, 1] = 4.0                                  # defect Q[:,1] * 1 -> norm 1
    assert abs(metrics.qr_residual(A, Q, R2) - 1.0 / math.sqrt(50.0)) <= 1e-15
    # ||X||^2 = 25, ||P||^2 + ||N||^2 = 9 + 16 -> defect 0; with N = 5: |25 - 34| / 25
    X = np.array([[3.0], [4.0]])
    assert metrics.pythagoras_defect(X, np.array([[3.0]]), np.array([[4.0]])) == 0.0
    assert metrics.pythagoras_defect(X, np.array([[3.0]]), np.array([[5.0]])) == 9.0 / 25.0
