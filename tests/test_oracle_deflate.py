"""Pins for the oracle's deflation (Sec. 3.1: truncated eigen decomposition
of G - P^T P) and TreeTSPQR with a deflating reduction (CPU only).

* a hand-derived diagonal case fixes the order, the sign convention, the
  zero padding of N and W;
* closed form X = Q C + Y0 Sigma0 Z0^T with Y0 orthogonal to Q: P = C, the
  rank, and (up to the sign of each direction) U = Y0, N = Sigma0 Z0^T;
* a full-rank block is the plain BCGS-PIP(+) step and the unique solution
  (LAPACK QR of [Q X]);
* exact dependence (a zero column, a repeated column) gives exact zeros in
  U and N and an orthonormal [Q U_t];
* the dropped part is the truncated SVD error (Eckart-Young, numpy's SVD);
* the Gram route (eigh of G - P^T P, then the Cholesky sweep) and the
  definition (SVD of the residual) agree;
* the tree with Householder leaves and a deflating reduction gives the
  deflated solution of the global problem for any partition, and block
  Arnoldi meeting an invariant direction deflates it and keeps the
  relation A Q = Q H on the kept columns.
"""

import numpy as np
import pytest

from oracle import (Breakdown, TreeTSPQR, bcgs_pip, bcgs_pip_plus, deflating_pip, deflating_pip_plus,
                    metrics, pqr_deflated_reference, pqr_reference, truncated_sqrt)


def _orth(rng, n, m):
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    return Q


def _complement(rng, Q, m):
    n = Q.shape[0]
    G = rng.standard_normal((n, m))
    G -= Q @ (Q.T @ G)
    G -= Q @ (Q.T @ G)
    Y, _ = np.linalg.qr(G)
    return Y


def test_truncated_sqrt_hand_case():
    # eigenvalues 9 (e2), 4 (e0), 0 (e1): kept in decreasing order
    t, N, W = truncated_sqrt(np.diag([4.0, 0.0, 9.0]), 1e-12)
    assert t == 2
    assert np.array_equal(N, np.array([[0.0, 0.0, 3.0], [2.0, 0.0, 0.0], [0.0, 0.0, 0.0]]))
    assert np.allclose(W, np.array([[0.0, 0.5, 0.0], [0.0, 0.0, 0.0], [1.0 / 3.0, 0.0, 0.0]]), atol=0)
    # sign convention: the entry of largest magnitude is positive
    t, N, W = truncated_sqrt(np.array([[1.0, -1.0], [-1.0, 1.0]]), 1e-12)    # eigen 2 on (1,-1)/sqrt2
    assert t == 1 and N[0, 0] == pytest.approx(1.0) and N[0, 1] == pytest.approx(-1.0)
    assert np.all(N[1] == 0.0) and np.all(W[:, 1] == 0.0)


def test_truncated_sqrt_is_a_square_root_of_the_kept_part():
    rng = np.random.default_rng(1)
    V = _orth(rng, 6, 6)
    lam = np.array([7.0, 3.0, 1.0, 0.5, 1e-14, 0.0])
    M = V @ np.diag(lam) @ V.T
    t, N, W = truncated_sqrt(M, 1e-10)
    assert t == 4
    Vt = V[:, :4]
    assert np.allclose(N.T @ N, Vt @ np.diag(lam[:4]) @ Vt.T, atol=1e-13)
    assert np.allclose(W @ N, Vt @ Vt.T, atol=1e-13)          # projector on the kept directions
    assert np.allclose(N @ W, np.diag([1.0, 1.0, 1.0, 1.0, 0.0, 0.0]), atol=1e-13)


@pytest.mark.parametrize("fn", [deflating_pip_plus, pqr_deflated_reference])
@pytest.mark.parametrize("k,s,t", [(0, 4, 2), (12, 8, 5), (30, 4, 3), (16, 2, 1)])
def test_closed_form_deflated_block(fn, k, s, t):
    n = 600
    rng = np.random.default_rng(100 * k + 10 * s + t)
    Q = _orth(rng, n, k) if k else np.zeros((n, 0))
    Y0 = _complement(rng, Q, t)
    Z0 = _orth(rng, s, t)
    sig = np.geomspace(3.0, 0.1, t)
    C = rng.standard_normal((k, s))
    X = Q @ C + Y0 @ np.diag(sig) @ Z0.T
    P, N, U, tt = fn(Q, X, 1e-6)
    assert tt == t
    assert np.allclose(P, C, atol=1e-13)
    assert np.all(N[t:] == 0.0) and np.all(U[:, t:] == 0.0)
    for r in range(t):
        d = 1.0 if N[r] @ Z0[:, r] > 0 else -1.0
        assert np.allclose(N[r], d * sig[r] * Z0[:, r], atol=1e-12)
        assert np.allclose(U[:, r], d * Y0[:, r], atol=1e-12)
        i = int(np.argmax(np.abs(N[r])))
        assert N[r, i] > 0.0                         # the sign convention
    assert metrics.e_perp(np.hstack([Q, U[:, :t]])) <= 1e-14
    assert np.linalg.norm(X - Q @ P - U @ N) <= 1e-13 * np.linalg.norm(X)


@pytest.mark.parametrize("k,s", [(0, 4), (20, 8)])
def test_full_rank_block_is_the_plain_step(k, s):
    n = 500
    rng = np.random.default_rng(k + s)
    Q = _orth(rng, n, k) if k else np.zeros((n, 0))
    X = rng.standard_normal((n, s))
    P, N, U, t = deflating_pip_plus(Q, X, 1e-6)
    assert t == s
    Pp, Np, Up = bcgs_pip_plus(Q, X)
    assert np.array_equal(P, Pp) and np.array_equal(N, Np) and np.array_equal(U, Up)
    Pr, Nr, Ur = pqr_reference(Q, X)
    assert np.allclose(N, Nr, atol=1e-13) and np.allclose(U, Ur, atol=1e-13)
    P1, N1, U1, t1 = deflating_pip(Q, X, 1e-6)
    Pq, Nq, Uq = bcgs_pip(Q, X)
    assert t1 == s and np.array_equal(N1, Nq) and np.array_equal(U1, Uq)


@pytest.mark.parametrize("case", ["zero", "repeat", "combination"])
def test_exact_dependence(case):
    n, k, s = 400, 10, 4
    rng = np.random.default_rng(3)
    Q = _orth(rng, n, k)
    X = rng.standard_normal((n, s))
    if case == "zero":
        X[:, 1] = 0.0
    elif case == "repeat":
        X[:, 3] = X[:, 0]
    else:
        X[:, 2] = 2.0 * X[:, 0] - X[:, 1] + Q @ rng.standard_normal(k)
    P, N, U, t = deflating_pip_plus(Q, X, 1e-6)
    assert t == s - 1
    assert np.all(U[:, t:] == 0.0) and np.all(N[t:] == 0.0)
    assert metrics.e_perp(np.hstack([Q, U[:, :t]])) <= 1e-14
    assert np.linalg.norm(X - Q @ P - U @ N) <= 1e-13 * np.linalg.norm(X)
    assert np.allclose(P, Q.T @ X, atol=1e-13)
    with pytest.raises(Breakdown):                   # the Cholesky step cannot do this
        bcgs_pip_plus(Q, X)


def test_dropped_part_is_the_truncated_svd_error():
    n, k, s = 800, 16, 6
    rng = np.random.default_rng(21)
    Q = _orth(rng, n, k)
    Y0 = _complement(rng, Q, s)
    Z0 = _orth(rng, s, s)
    sig = np.array([2.0, 1.0, 0.3, 1e-3, 1e-9, 1e-12])
    X = Q @ rng.standard_normal((k, s)) + Y0 @ np.diag(sig) @ Z0.T
    xn = np.linalg.norm(X)
    for fn in (deflating_pip_plus, pqr_deflated_reference):
        P, N, U, t = fn(Q, X, 1e-4 / xn)       # keeps sigma >= 1e-3, drops 1e-9, 1e-12
        assert t == 4
        R = X - Q @ (Q.T @ X)
        sv = np.linalg.svd(R, compute_uv=False)
        err = np.linalg.norm(R - U @ N)
        assert err == pytest.approx(np.sqrt(np.sum(sv[4:] ** 2)), rel=2e-2)


def test_gram_route_agrees_with_the_definition():
    n, k, s = 1000, 24, 8
    rng = np.random.default_rng(8)
    Q = _orth(rng, n, k)
    Y0 = _complement(rng, Q, 5)
    Z0 = _orth(rng, s, 5)
    X = Q @ rng.standard_normal((k, s)) + Y0 @ np.diag([4.0, 2.0, 1.0, 0.5, 0.25]) @ Z0.T
    X += 1e-13 * rng.standard_normal((n, s))
    a = deflating_pip_plus(Q, X, 1e-6)
    b = pqr_deflated_reference(Q, X, 1e-6)
    assert a[3] == b[3] == 5
    xn = np.linalg.norm(X)
    assert np.linalg.norm(a[0] - b[0]) <= 1e-13 * xn
    assert np.linalg.norm(a[1] - b[1]) <= 1e-12 * xn
    assert np.max(np.abs(a[2] - b[2])) <= 1e-11


@pytest.mark.parametrize("n,s,leaf,red", [(2000, 4, 250, "pip+"), (1537, 8, 300, "pip+"), (1200, 4, 400, "pip")])
def test_tree_with_deflating_reduction(n, s, leaf, red):
    rng = np.random.default_rng(n + s)
    t = TreeTSPQR(n, s, leaf, "hh", red, deflate=1e-6)
    Q = np.zeros((n, 0))
    ranks = []
    for j in range(4):
        X = rng.standard_normal((n, s))
        if j == 1:
            X[:, 1] = X[:, 0] - 3.0 * X[:, 2]          # rank s - 1
        if j == 2:
            X[:, 0] = 0.0                            # a zero column
        if j == 3 and Q.shape[1]:
            X[:, 3] = Q[:, :Q.shape[1]] @ rng.standard_normal(Q.shape[1])   # in the span of Q
        P, N, U, = t.step(X)
        Pr, Nr, Ur, tr = pqr_deflated_reference(Q, X, 1e-6)
        ranks.append(t.last_rank)
        assert t.last_rank == tr
        xn = np.linalg.norm(X)
        if Q.shape[1]:
            assert np.linalg.norm(P - Pr) <= 1e-12 * xn
        assert np.linalg.norm(N - Nr) <= 1e-11 * xn
        assert np.max(np.abs(U - Ur)) <= 1e-10
        assert np.all(U[:, tr:] == 0.0)
        Q = np.hstack([Q, Ur])
    assert ranks == [s, s - 1, s - 1, s - 1]
    Qe = t.explicit_Q()
    keep = np.linalg.norm(Qe, axis=0) > 0.5
    assert np.count_nonzero(keep) == sum(ranks)
    assert metrics.e_perp(Qe[:, keep]) <= 1e-13
    assert np.all(Qe[:, ~keep] == 0.0)


def test_block_arnoldi_deflates_an_invariant_direction():
    """The start block holds an eigenvector of A: A u_0 lies in the basis,
    the next block deflates it, its zero column stays deflated, and the
    Arnoldi relation A Q_k = Q_{k+s} H holds on the kept columns."""
    n, s, leaf, steps = 1200, 4, 300, 4
    rng = np.random.default_rng(2)
    d = np.linspace(1.0, 3.0, n)
    A = np.diag(d)
    X = rng.standard_normal((n, s))
    X[:, 0] = 0.0
    X[7, 0] = 1.0                                    # e_7, an eigenvector
    t = TreeTSPQR(n, s, leaf, "hh", "pip+", deflate=1e-6)
    H = np.zeros(((steps + 1) * s, steps * s))
    ranks = []
    _, R0, U = t.step(X)
    ranks.append(t.last_rank)
    for j in range(steps):
        W = A @ U
        P, N, U = t.step(W)
        ranks.append(t.last_rank)
        H[:(j + 1) * s, j * s:(j + 1) * s] = P
        H[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = N
    assert ranks == [s] + [s - 1] * steps
    Qe = t.explicit_Q()
    keep = np.linalg.norm(Qe, axis=0) > 0.5
    assert metrics.e_perp(Qe[:, keep]) <= 1e-13
    Qk = Qe[:, :steps * s]
    assert np.linalg.norm(A @ Qk - Qe @ H) <= 1e-12 * np.linalg.norm(A @ Qk)
