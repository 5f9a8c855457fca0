"""Pins for the oracle's FlatTSPQR (Sec. 4.2, Algorithm "FlatTSPQR"; CPU only).

* uniqueness of the PQR solution (eq. (1.1)): for every block partition
  (one block, two, many, a ragged last block) and every local subalgorithm
  (BCGS-PIP+, the reference solution, Householder) the chain's global
  (P, N, U) equals pqr_reference's on the chain's own basis, step after
  step (the Householder form after its diagonal signs D = diag(sign N_ii)
  are fixed; its basis columns keep those signs);
* every factor of the chain has orthonormal columns, the chain's explicit
  basis is orthonormal and apply_Q(C) equals the explicit basis times C;
* the zero rows inserted for N_{i-1}'s coordinates: a factor keeps exact
  zero rows where the previous block's new coordinates enter only through
  its own new columns (checked on the second factor after the first step);
* one block reduces to the local subalgorithm itself;
* the stability statement of Sec. 4.2 (the flat variant inherits its
  subalgorithm's stability): on the Sec. 6.1 Stewart workload (kappa = 1e4,
  n = 2^16, 32 columns, s = 4, 8 and 256 blocks) BCGS-PIP local problems
  lose orthogonality O(eps kappa^2) and BCGS-PIP+ / Householder keep O(eps);
  the paper prints no value for the flat variant, so the pin is the class.
A slip in the stacking order of [P; N; X_i], in the position of the
inserted rows or in the chain's product order fails the uniqueness and
apply_Q checks.
"""

import numpy as np
import pytest

from oracle import HouseholderBasis, bcgs_pip_plus, metrics, pqr_reference
from oracle.flattspqr import FlatTSPQR
from oracle.krylov import block_column_qr
from synth import stewart

def _signfix(P, N, U):
    d = np.sign(np.diag(N))
    d[d == 0] = 1.0
    return P, d[:, None] * N, U * d[None, :]


@pytest.mark.parametrize("n,s,rows,local", [
    (300, 3, 300, "pip+"), (300, 3, 150, "pip+"), (1037, 4, 100, "pip+"), (1000, 2, 130, "ref"),
    (500, 4, 60, "hh"), (777, 1, 70, "hh"), (640, 8, 80, "pip+"),
])
def test_flat_equals_unique_solution(n, s, rows, local):
    rng = np.random.default_rng(n + s + rows)
    flat = FlatTSPQR(n, s, rows, local)
    Q = np.zeros((n, 0))
    kmax = min(rows, 48) // s * s
    for step in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.3, s)
        if step:
            X = X + Q @ rng.standard_normal((Q.shape[1], s))
        P, N, Uraw = flat.step(X)
        # the reference on the chain's own basis (Householder columns carry
        # the signs of their N's diagonal)
        Pr, Nr, Ur = pqr_reference(Q, X)
        P, N, U = _signfix(P, N, Uraw) if local == "hh" else (P, N, Uraw)
        xn = np.linalg.norm(X)
        assert np.linalg.norm(P - Pr) / xn <= 1e-12, step
        assert np.linalg.norm(N - Nr) / xn <= 1e-12, step
        assert np.max(np.abs(U - Ur)) <= 1e-11, step
        Q = np.hstack([Q, Uraw])
    # the chain's factors and its explicit basis
    for i in range(flat.p):
        F = flat.factor(i)
        assert np.max(np.abs(F.T @ F - np.eye(F.shape[1]))) <= 1e-12, i
    E = flat.explicit_Q()
    assert metrics.e_perp(E) <= 1e-12
    C = rng.standard_normal((flat.k, 5))
    assert np.max(np.abs(flat.apply_Q(C) - E @ C)) <= 1e-12 * np.abs(C).sum(0).max()


def test_flat_factor_rows():
    """Factor i >= 2 spans the chain's k coordinates then block i's rows; after
    the first step of width s its first s rows are those coordinates."""
    n, s, rows = 400, 4, 100
    rng = np.random.default_rng(5)
    flat = FlatTSPQR(n, s, rows)
    flat.step(rng.standard_normal((n, s)))
    assert flat.factor(0).shape == (100, 4)
    for i in range(1, 4):
        assert flat.factor(i).shape == (4 + 100, 4)
    flat.step(rng.standard_normal((n, s)))
    # second step: 4 old coordinates, 4 new ones, then the block's rows;
    # the old columns have exact zeros in the 4 inserted rows
    F = flat.factor(2)
    assert F.shape == (8 + 100, 8)
    assert np.all(F[4:8, :4] == 0.0)


def test_one_block_is_the_subalgorithm():
    n, s = 200, 4
    rng = np.random.default_rng(7)
    flat = FlatTSPQR(n, s, n, "pip+")
    Q = np.zeros((n, 0))
    for _ in range(4):
        X = rng.standard_normal((n, s))
        P, N, U = flat.step(X)
        P2, N2, U2 = bcgs_pip_plus(Q, X)
        assert np.array_equal(P, P2) and np.array_equal(N, N2)
        assert np.max(np.abs(U - U2)) <= 1e-14
        Q = np.hstack([Q, U2])
    hh = FlatTSPQR(n, s, n, "hh")
    basis = HouseholderBasis(n)
    rng = np.random.default_rng(8)
    for _ in range(3):
        X = rng.standard_normal((n, s))
        P, N, U = hh.step(X)
        P2, N2, U2 = basis.pqr(X)
        assert np.array_equal(P, P2) and np.array_equal(N, N2)
        assert np.max(np.abs(U - U2)) <= 1e-14


@pytest.fixture(scope="module")
def stewart_1e4():
    return stewart(2 ** 16, 32, 1e4, 0)


@pytest.mark.parametrize("p", [8, 256])
def test_flat_inherits_subalgorithm_stability(stewart_1e4, p):
    """No value is printed for the flat variant; the pin is the stability
    class.  BCGS-PIP loses orthogonality like eps kappa^2 (kappa = 1e4: about
    1e-8; measured 3-4e-8), BCGS-PIP+ and Householder stay O(eps) (measured
    5.5e-15 .. 7.7e-14, growing with the chain's length p), and A = QR holds
    to rounding for all three."""
    A = stewart_1e4
    n = A.shape[0]
    for local in ("pip", "pip+", "hh"):
        flat = FlatTSPQR(n, 4, n // p, local)
        Q, R = block_column_qr(A, 4, flat)
        e = metrics.e_perp(flat.explicit_Q())
        if local == "pip":
            assert 1e-10 <= e <= 1e-6, (local, p, e)
        else:
            assert e <= 1e-12, (local, p, e)
        assert metrics.qr_residual(A, Q, R) <= 1e-13, (local, p)
