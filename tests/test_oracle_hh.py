"""Pins for the oracle's Householder method (Sec. 2.2, Algorithm "HH") and
TreeTSPQR with Householder leaves (CPU only).

* hand-derived 3 x 3 cases fix the reflector sign (sigma = -sgn of the
  pivot entry, sgn(0) = +1), N's negative diagonal and U exactly;
* LAPACK's QR of the stacked [Q X] (numpy.linalg.qr, independent of the
  oracle) gives the unique PQR solution: P, D N and U D must match it;
* closed form X = Q C + U0 N0 with U0 orthogonal to Q: P = C, D N = N0;
* structure: unit reflectors, zero above their pivot rows, orthonormal
  explicit basis, apply / apply_transpose inverse to each other;
* stability: a block nearly in the span of Q (kappa ~ 1e12), where
  BCGS-PIP+ breaks down, keeps [Q U] orthonormal to rounding;
* a zero column gives N[i, i] = 0 and reflector e_{k+i} (the reading);
* TreeTSPQR with Householder leaves returns the unique PQR solution for
  any partition and fan-in, and survives a leaf whose local block is
  nearly dependent while the global block is not (BCGS-PIP+ leaves break
  down there).
"""

import numpy as np
import pytest

from oracle import Breakdown, HouseholderBasis, TreeTSPQR, bcgs_pip_plus, metrics, pqr_reference


def _lapack_pqr(Q, X):
    """Unique (P, N, U) from LAPACK QR of [Q X] with a positive diagonal."""
    k = Q.shape[1]
    Qf, Rf = np.linalg.qr(np.hstack([Q, X]))
    d = np.where(np.diag(Rf) < 0.0, -1.0, 1.0)
    Rf = d[:, None] * Rf
    Qf = Qf * d[None, :]
    return Rf[:k, k:], Rf[k:, k:], Qf[:, k:]


def _signs(N):
    return np.where(np.diag(N) < 0.0, -1.0, 1.0)


def test_hand_example_first_block():
    # x = (3, 4, 0): lambda = 5, pivot 3 >= 0 -> sigma = -1, N = -5,
    # v ~ (3 + 5, 4, 0), U = H e_0 = (-0.6, -0.8, 0)
    B = HouseholderBasis(3)
    P, N, U = B.pqr(np.array([[3.0], [4.0], [0.0]]))
    assert P.shape == (0, 1)
    assert N[0, 0] == pytest.approx(-5.0, abs=1e-15)
    assert np.allclose(U[:, 0], [-0.6, -0.8, 0.0], atol=1e-15)
    assert np.allclose(B.V[:, 0], np.array([8.0, 4.0, 0.0]) / np.sqrt(80.0), atol=1e-15)


def test_hand_example_second_block_and_zero_pivot_sign():
    # step 1: x0 = (0, 0, 2): pivot 0 -> sgn(0) = +1 -> sigma = -1, N = -2,
    # v0 = (1, 0, 1)/sqrt 2, U = (0, 0, -1)
    B = HouseholderBasis(3)
    P, N, U = B.pqr(np.array([[0.0], [0.0], [2.0]]))
    assert N[0, 0] == pytest.approx(-2.0, abs=1e-15)
    assert np.allclose(U[:, 0], [0.0, 0.0, -1.0], atol=1e-15)
    # step 2: x1 = (1, 1, 1): P = q^T x1 = -1; x1 - q P = (1, 1, 0), whose
    # norm sqrt 2 with pivot entry (row 1 of H0 x1) = +1 -> N = -sqrt 2,
    # U = (1, 1, 0) / (-sqrt 2)
    P, N, U = B.pqr(np.array([[1.0], [1.0], [1.0]]))
    assert P[0, 0] == pytest.approx(-1.0, abs=1e-15)
    assert N[0, 0] == pytest.approx(-np.sqrt(2.0), abs=1e-15)
    assert np.allclose(U[:, 0], [-1.0 / np.sqrt(2.0), -1.0 / np.sqrt(2.0), 0.0], atol=1e-15)
    assert B.V[0, 1] == 0.0          # zero above the pivot row


@pytest.mark.parametrize("n,s,steps", [(200, 1, 6), (300, 4, 5), (257, 8, 4), (100, 16, 3)])
def test_matches_lapack_qr_of_stacked_blocks(n, s, steps):
    rng = np.random.default_rng(n + s)
    B = HouseholderBasis(n)
    for _ in range(steps):
        Qe = B.explicit()
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 1e-3, s)
        P, N, U = B.pqr(X)
        Pl, Nl, Ul = _lapack_pqr(Qe, X)
        d = _signs(N)
        xn = np.linalg.norm(X)
        assert np.linalg.norm(P - Pl) <= 1e-13 * xn
        assert np.linalg.norm(d[:, None] * N - Nl) <= 1e-13 * xn
        assert np.max(np.abs(U * d[None, :] - Ul)) <= 1e-10
        # the step's own factorisation and orthogonality
        assert metrics.pqr_residual(Qe, X, P, N, U) <= 1e-14
        if Qe.shape[1]:
            assert np.max(np.abs(Qe.T @ U)) <= 1e-14


def test_closed_form_projection_and_normalizer():
    n, s = 400, 4
    rng = np.random.default_rng(7)
    B = HouseholderBasis(n)
    B.pqr(rng.standard_normal((n, 8)))
    Qe = B.explicit()
    G = rng.standard_normal((n, s))
    U0, _ = np.linalg.qr(G - Qe @ (Qe.T @ G))
    U0, _ = np.linalg.qr(U0 - Qe @ (Qe.T @ U0))
    C = rng.standard_normal((8, s))
    N0 = np.triu(rng.standard_normal((s, s)))
    N0[np.diag_indices(s)] = np.abs(N0[np.diag_indices(s)]) + 1.0
    X = Qe @ C + U0 @ N0
    P, N, U = B.pqr(X)
    d = _signs(N)
    assert np.allclose(P, C, atol=1e-13)
    assert np.allclose(d[:, None] * N, N0, atol=1e-13)
    assert np.allclose(U * d[None, :], U0, atol=1e-13)


def test_reflector_structure_and_inverse():
    n = 120
    rng = np.random.default_rng(3)
    B = HouseholderBasis(n)
    for _ in range(3):
        B.pqr(rng.standard_normal((n, 5)))
    V = B.V
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-15)
    for i in range(B.k):
        assert np.all(V[:i, i] == 0.0)
    Qe = B.explicit()
    assert metrics.e_perp(Qe) <= 1e-14
    C = rng.standard_normal((B.k, 3))
    Y = B.apply(C)
    back = B.apply_transpose(Y)
    assert np.allclose(back[:B.k], C, atol=1e-14) and np.allclose(back[B.k:], 0.0, atol=1e-14)


def test_stable_where_cholesky_qr_breaks_down():
    n, s = 500, 4
    rng = np.random.default_rng(11)
    B = HouseholderBasis(n)
    B.pqr(rng.standard_normal((n, 12)))
    Qe = B.explicit()
    G = rng.standard_normal((n, s))
    U0, _ = np.linalg.qr(G - Qe @ (Qe.T @ G))
    X = Qe @ rng.standard_normal((12, s)) + 1e-12 * U0 @ np.triu(np.ones((s, s)))
    with pytest.raises(Breakdown):
        bcgs_pip_plus(Qe, X)
    P, N, U = B.pqr(X)
    assert metrics.e_perp(np.hstack([Qe, U])) <= 1e-14
    assert metrics.pqr_residual(Qe, X, P, N, U) <= 1e-15
    d = _signs(N)
    assert np.linalg.norm(d[:, None] * N - 1e-12 * np.triu(np.ones((s, s)))) <= 1e-14 * np.linalg.norm(X)


def test_single_column_is_projection_and_scaling():
    n = 90
    rng = np.random.default_rng(5)
    B = HouseholderBasis(n)
    B.pqr(rng.standard_normal((n, 6)))
    Qe = B.explicit()
    x = rng.standard_normal((n, 1))
    r = x - Qe @ (Qe.T @ x)
    P, N, U = B.pqr(x)
    assert abs(abs(N[0, 0]) - np.linalg.norm(r)) <= 1e-14 * np.linalg.norm(x)
    assert np.allclose(U * np.sign(N[0, 0]), r / np.linalg.norm(r), atol=1e-14)


@pytest.mark.parametrize("k0", [0, 3])
def test_zero_column_reading(k0):
    n, s = 50, 4
    rng = np.random.default_rng(9)
    B = HouseholderBasis(n)
    if k0:
        B.pqr(rng.standard_normal((n, k0)))
    Qe = B.explicit()
    X = rng.standard_normal((n, s))
    X[:, 2] = 0.0
    P, N, U = B.pqr(X)
    assert N[2, 2] == 0.0
    v = B.V[:, k0 + 2]
    assert v[k0 + 2] == 1.0 and np.count_nonzero(v) == 1
    assert metrics.pqr_residual(Qe, X, P, N, U) <= 1e-15
    assert metrics.e_perp(np.hstack([Qe, U])) <= 1e-14


@pytest.mark.parametrize("n,s,leaf,fan_in", [(1000, 4, 250, None), (1037, 8, 200, None),
                                              (2048, 4, 256, 2), (999, 2, 100, 3)])
def test_tree_with_householder_leaves_is_the_unique_solution(n, s, leaf, fan_in):
    rng = np.random.default_rng(n)
    t = TreeTSPQR(n, s, leaf, "hh", "pip+", fan_in)
    Q = np.zeros((n, 0))
    for _ in range(5):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 1e-2, s)
        P, N, U = t.step(X)
        Pr, Nr, Ur = pqr_reference(Q, X)
        xn = np.linalg.norm(X)
        if Q.shape[1]:
            assert np.linalg.norm(P - Pr) <= 1e-13 * xn
        assert np.linalg.norm(N - Nr) <= 1e-13 * xn
        assert np.max(np.abs(U - Ur)) <= 1e-11
        Q = np.hstack([Q, Ur])
    Qe = t.explicit_Q()
    assert metrics.e_perp(Qe) <= 1e-14
    for B in t.leaves:
        assert metrics.e_perp(B.explicit()) <= 1e-14
    if fan_in is None:                           # single level: [R_1; ...; R_p] orthonormal
        assert metrics.e_perp(t.stacked_factor(0)) <= 1e-14


def test_householder_leaves_survive_a_locally_dependent_leaf():
    """Leaf 0's part of the second block lies in that leaf's basis up to
    1e-11, leaf 1's part is random: the global block is well conditioned,
    the local problem of leaf 0 is not.  BCGS-PIP+ leaves break down; the
    Householder leaves give the unique solution."""
    n, s, leaf = 2000, 4, 1000
    rng = np.random.default_rng(13)
    X0 = rng.standard_normal((n, s))
    X1 = rng.standard_normal((n, s))
    hh = TreeTSPQR(n, s, leaf, "hh", "pip+")
    pp = TreeTSPQR(n, s, leaf, "pip+", "pip+")
    hh.step(X0)
    pp.step(X0)
    Q0 = hh.leaves[0].explicit()                 # leaf 0's local basis (1000 x 4)
    X1[:leaf] = Q0 @ rng.standard_normal((s, s)) + 1e-11 * rng.standard_normal((leaf, s))
    with pytest.raises(Breakdown):
        pp.step(X1)
    P, N, U = hh.step(X1)
    Q = np.hstack([pqr_reference(None, X0)[2]])
    Pr, Nr, Ur = pqr_reference(Q, X1)
    xn = np.linalg.norm(X1)
    assert np.linalg.norm(P - Pr) <= 1e-13 * xn and np.linalg.norm(N - Nr) <= 1e-13 * xn
    assert np.max(np.abs(U - Ur)) <= 1e-12
    assert metrics.e_perp(hh.explicit_Q()) <= 1e-14
