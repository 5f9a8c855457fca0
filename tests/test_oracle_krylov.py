"""Pins for the oracle's drivers and test operators (CPU only).

* the Laplacian stencils against a brute-force dense matrix assembled entry by
  entry from the grid definition, and their extreme eigenvalues against the
  closed form and LAPACK (numpy.linalg.eigvalsh);
* block Arnoldi (Sec. 2) on a symmetric operator: the square part of the
  block Hessenberg matrix is V^T A V, so it is symmetric block tridiagonal
  with the super-diagonal block equal to the previous N^T; Ritz values lie in
  [lambda_min, lambda_max]; the Arnoldi relation A V_j = V_{j+1} H holds;
* block-column QR (Sec. 2): R equals the unique Householder R and
  R^T R = A^T A.
"""

import numpy as np
import pytest

from oracle import TreeTSPQR, block_arnoldi, block_column_qr, householder_qr, metrics
from oracle import operators as ops


def _dense_brute(dims, shift):
    n = int(np.prod(dims))
    A = np.zeros((n, n))
    diag = 2.0 * len(dims) + shift
    strides = [int(np.prod(dims[:d])) for d in range(len(dims))]
    for p in range(n):
        idx = [(p // strides[d]) % dims[d] for d in range(len(dims))]
        A[p, p] = diag
        for d in range(len(dims)):
            for delta in (-1, 1):
                j = idx[d] + delta
                if 0 <= j < dims[d]:
                    A[p, p + delta * strides[d]] = -1.0
    return A


@pytest.mark.parametrize("dims,shift", [((5, 4), 0.0), ((7, 3), 0.01), ((3, 4, 5), 0.0), ((2, 2, 2), 0.5)])
def test_laplacian_matches_brute_force_and_spectrum(dims, shift):
    A = _dense_brute(dims, shift)
    assert np.array_equal(ops.laplacian_dense(dims, shift), A)
    ev = np.linalg.eigvalsh(A)
    lo, hi = ops.laplacian_extreme_eigs(dims, shift)
    assert abs(ev[0] - lo) < 1e-12 and abs(ev[-1] - hi) < 1e-12


def test_closed_form_extremes_of_workloads():
    lo, hi = ops.laplacian_extreme_eigs((100, 100), 0.01)
    assert abs(lo - 0.0119349) < 1e-6 and abs(hi - 8.0080651) < 1e-6


@pytest.mark.parametrize("solver", ["ref", "tree"])
def test_block_arnoldi_invariants(solver):
    nx, ny, shift, s, steps = 30, 20, 0.01, 3, 8
    n = nx * ny
    apply_A = lambda X: ops.laplacian_2d_apply(X, nx, ny, shift)
    R0 = np.random.default_rng(0).standard_normal((n, s))
    pqr = None if solver == "ref" else TreeTSPQR(n, s, 100)
    V, H, H0, blocks = block_arnoldi(apply_A, R0, steps, pqr)
    K = steps * s
    assert metrics.e_perp(V) < 1e-13
    assert np.allclose(V[:, :s] @ H0, R0, atol=1e-12)
    lo, hi = ops.laplacian_extreme_eigs((nx, ny), shift)
    assert metrics.arnoldi_relation(apply_A, V, H, hi) < 1e-14
    T = H[:K, :K]
    assert np.allclose(T, T.T, atol=1e-12)
    for i in range(steps):
        for j in range(i + 2, steps):
            assert np.max(np.abs(T[i * s:(i + 1) * s, j * s:(j + 1) * s])) < 1e-12 * hi
    for j in range(1, steps):
        Nprev = H[j * s:(j + 1) * s, (j - 1) * s:j * s]
        assert np.allclose(T[(j - 1) * s:j * s, j * s:(j + 1) * s], Nprev.T, atol=1e-12)
    ritz = np.linalg.eigvalsh(T)
    assert ritz[0] >= lo - 1e-10 and ritz[-1] <= hi + 1e-10


def test_block_column_qr_unique_r():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((400, 24))
    Q, R = block_column_qr(A, 6)
    Qh, Rh = householder_qr(A)
    assert np.allclose(R, Rh, atol=1e-12)
    assert np.allclose(R.T @ R, A.T @ A, atol=1e-11)
    assert np.allclose(Q, Qh, atol=1e-12)
