"""Pins for the oracle's PQR solvers (CPU only).

* closed form: X = Q C + U0 N0 with U0 orthonormal, Q^T U0 = 0 and N0 upper
  triangular with positive diagonal has the unique PQR solution (C, N0, U0)
  (eq. (1.1) plus uniqueness of QR);
* a different algorithm: Householder QR of the whole [Q X] yields the same
  P, N, U (leading block = identity after the sign fix);
* library pins: numpy Cholesky, scipy triangular solve;
* stated error orders (Sec. 3, Sec. 3.1, Sec. 6.1): BCGS-PIP loses
  orthogonality like eps kappa^2, BCGS-PIP+ and the reference stay O(eps)
  (BCGS-PIP+ while eps kappa^2 <= 1/2);
* ill-conditioned residuals: the reiteration's combination P = P1 + P2 N1,
  N = N2 N1 matters there (a wrong combination fails these).
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import (Breakdown, bcgs_pip, bcgs_pip_plus, cholesky_upper,
                    householder_qr, pqr_reference, triu_solve_right)
from oracle import metrics
from oracle.krylov import block_column_qr
from synth import stewart

U = 2.0 ** -53
SOLVERS = {"ref": pqr_reference, "pip": bcgs_pip, "pip+": bcgs_pip_plus}


def _closed_form_case(n, k, s, seed, cond_n0=10.0):
    rng = np.random.default_rng(seed)
    W, _ = np.linalg.qr(rng.standard_normal((n, k + s)))
    Q, U0 = W[:, :k], W[:, k:]
    C = rng.standard_normal((k, s))
    N0 = np.triu(rng.standard_normal((s, s)), 1) * 0.3
    N0[np.diag_indices(s)] = np.geomspace(1.0, 1.0 / cond_n0, s)
    X = Q @ C + U0 @ N0
    return Q, X, C, N0, U0


@pytest.mark.parametrize("name", list(SOLVERS))
@pytest.mark.parametrize("n,k,s", [(50, 0, 3), (64, 8, 4), (500, 40, 8), (200, 3, 1), (1000, 16, 16)])
def test_closed_form_solution(name, n, k, s):
    Q, X, C, N0, U0 = _closed_form_case(n, k, s, seed=n + 7 * k + s)
    P, N, Uo = SOLVERS[name](Q, X)
    scale = np.linalg.norm(X)
    assert P.shape == (k, s) and N.shape == (s, s) and Uo.shape == (n, s)
    assert np.allclose(np.tril(N, -1), 0.0)
    assert np.all(np.diag(N) > 0)
    # one CholQR sweep (BCGS-PIP) is accurate to O(eps kappa^2) only
    kappa = np.linalg.cond(N0)
    tol = max(1e-12, 100 * U * kappa ** 2) if name == "pip" else 1e-12
    if k:
        assert np.linalg.norm(P - C) / scale < tol
    assert np.linalg.norm(N - N0) / scale < tol
    assert np.max(np.abs(Uo - U0)) < tol * 100


@pytest.mark.parametrize("seed", range(4))
def test_reference_equals_householder_of_whole_matrix(seed):
    rng = np.random.default_rng(seed)
    n, k, s = 300, 12, 5
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    X = rng.standard_normal((n, s)) * np.geomspace(1, 1e-3, s)
    Qf, Rf = householder_qr(np.hstack([Q, X]))
    # leading block of the whole-matrix QR is the identity for orthonormal Q
    assert np.linalg.norm(Rf[:k, :k] - np.eye(k)) < 1e-13
    P, N, Uo = pqr_reference(Q, X)
    assert np.linalg.norm(P - Rf[:k, k:]) < 1e-13
    assert np.linalg.norm(N - Rf[k:, k:]) < 1e-13
    assert np.linalg.norm(Uo - Qf[:, k:]) < 1e-10


@pytest.mark.parametrize("s", [1, 2, 5, 8, 16])
def test_cholesky_matches_lapack(s):
    rng = np.random.default_rng(s)
    B = rng.standard_normal((3 * s + 2, s))
    S = B.T @ B
    N = cholesky_upper(S)
    L = np.linalg.cholesky(S)
    assert np.allclose(N, L.T, rtol=1e-13, atol=1e-13 * np.abs(L).max())


def test_cholesky_breakdown_cases():
    with pytest.raises(Breakdown) as e:
        cholesky_upper(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert e.value.index == 1
    with pytest.raises(Breakdown):
        cholesky_upper(np.zeros((3, 3)))
    with pytest.raises(Breakdown):
        cholesky_upper(np.array([[np.nan]]))
    with pytest.raises(Breakdown):
        cholesky_upper(np.array([[-1.0]]))


def test_triu_solve_matches_scipy():
    rng = np.random.default_rng(3)
    N = np.triu(rng.standard_normal((7, 7))) + 4 * np.eye(7)
    Y = rng.standard_normal((40, 7))
    Z = triu_solve_right(Y, N)
    Zs = scipy.linalg.solve_triangular(N.T, Y.T, lower=True).T
    assert np.allclose(Z, Zs, rtol=1e-13, atol=1e-13)


def test_breakdown_when_x_in_span_q():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((80, 6)))
    X = Q @ rng.standard_normal((6, 3))
    with pytest.raises(Breakdown):
        bcgs_pip(Q, X)
    X2 = rng.standard_normal((80, 3))
    X2[:, 2] = X2[:, 1]
    with pytest.raises(Breakdown):
        bcgs_pip(Q, X2)


def _alg2_eperp(solver, kappa, n=4000, m=32, s=4, seed=11):
    A = stewart(n, m, kappa, seed)
    Q, R = block_column_qr(A, s, solver)
    return metrics.e_perp(Q), metrics.qr_residual(A, Q, R)


def test_error_orders_kappa_sweep():
    """Sec. 6.1 error orders: PIP ~ eps kappa^2, PIP+ and reference O(eps)."""
    e_pip = {}
    for kappa in (1e2, 1e4, 1e6):
        e, res = _alg2_eperp(bcgs_pip, kappa)
        e_pip[kappa] = e
        assert res < 1e-14
    # slope ~ 2 per decade pair: e(1e6)/e(1e2) ~ 1e8 within a factor 100
    ratio = e_pip[1e6] / e_pip[1e2]
    assert 1e6 < ratio < 1e10, e_pip
    assert 1e-3 * U * 1e12 < e_pip[1e6] < 1e3 * U * 1e12
    for kappa in (1e2, 1e5, 1e7):
        e, res = _alg2_eperp(bcgs_pip_plus, kappa)
        assert e < 1e-13, (kappa, e)
        assert res < 1e-14
    for kappa in (1e4, 1e10, 1e13):
        e, res = _alg2_eperp(pqr_reference, kappa)
        assert e < 1e-13, (kappa, e)
        assert res < 1e-14


def test_pip_plus_breaks_down_beyond_stability_region():
    """eps kappa^2 >> 1/2: BCGS-PIP's Cholesky fails (Sec. 6.1, condition on kappa)."""
    with pytest.raises(Breakdown):
        _alg2_eperp(bcgs_pip_plus, 1e12)


@pytest.mark.parametrize("name", list(SOLVERS))
def test_ill_conditioned_residual_and_pythagoras(name):
    """kappa = 1e6: the reiteration combination is visible in the residual."""
    rng = np.random.default_rng(9)
    n, k, s = 2000, 24, 8
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    X = stewart(n, s, 1e6, 4) + Q @ rng.standard_normal((k, s))
    P, N, Uo = SOLVERS[name](Q, X)
    assert metrics.pqr_residual(Q, X, P, N, Uo) < 2e-15 * np.sqrt(s)
    assert metrics.pythagoras_defect(X, P, N) < 1e-14
    if name != "pip":
        assert metrics.e_perp(np.hstack([Q, Uo])) < 1e-13


def test_s1_matches_modified_gram_schmidt():
    """s = 1: the block method is CGS2 on one vector; MGS gives the same unique result."""
    rng = np.random.default_rng(21)
    Q, _ = np.linalg.qr(rng.standard_normal((100, 7)))
    x = rng.standard_normal((100, 1))
    v = x[:, 0].copy()
    coeff = np.zeros(7)
    for j in range(7):
        coeff[j] = Q[:, j] @ v
        v -= coeff[j] * Q[:, j]
    nv = np.linalg.norm(v)
    for name, f in SOLVERS.items():
        P, N, Uo = f(Q, x)
        assert np.allclose(P[:, 0], coeff, atol=1e-14)
        assert abs(N[0, 0] - nv) < 1e-14
        assert np.allclose(Uo[:, 0], v / nv, atol=1e-13)


def test_k0_is_thin_qr():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((64, 5))
    Qh, Rh = householder_qr(X)
    for f in SOLVERS.values():
        P, N, Uo = f(None, X)
        assert P.shape == (0, 5)
        assert np.allclose(N, Rh, atol=1e-13)
        assert np.allclose(Uo, Qh, atol=1e-13)
