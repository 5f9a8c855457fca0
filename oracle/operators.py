"""Test operators for the Arnoldi driver (oracle side; test infrastructure).

The paper runs Arnoldi on no named operator; the workloads use the standard
Dirichlet finite-difference Laplacians:

* 2D 5-point stencil on an nx x ny grid: (A x)_p = 4 x_p - sum of the (up to
  four) grid neighbours, neighbours outside the grid dropped, plus an
  optional diagonal shift;
* 3D 7-point stencil on nx x ny x nz: 6 x_p - sum of (up to six) neighbours.

Unknowns are ordered lexicographically: p = i + nx*j (+ nx*ny*l), i fastest.
Both operators are symmetric positive definite with the closed-form spectrum
lambda = sum_d (2 - 2 cos(pi i_d / (n_d + 1))), i_d = 1..n_d, plus the shift.
"""

import numpy as np


def laplacian_2d_apply(X, nx, ny, shift=0.0):
    """A X for the 2D 5-point Dirichlet Laplacian; X is (nx*ny) x s."""
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    if n != nx * ny:
        raise ValueError("size mismatch")
    G = X.reshape(ny, nx, s)                 # [j, i, :]
    Y = (4.0 + shift) * G
    Y[:, 1:, :] -= G[:, :-1, :]
    Y[:, :-1, :] -= G[:, 1:, :]
    Y[1:, :, :] -= G[:-1, :, :]
    Y[:-1, :, :] -= G[1:, :, :]
    return Y.reshape(n, s)


def laplacian_3d_apply(X, nx, ny, nz, shift=0.0):
    """A X for the 3D 7-point Dirichlet Laplacian; X is (nx*ny*nz) x s."""
    X = np.asarray(X, dtype=np.float64)
    n, s = X.shape
    if n != nx * ny * nz:
        raise ValueError("size mismatch")
    G = X.reshape(nz, ny, nx, s)             # [l, j, i, :]
    Y = (6.0 + shift) * G
    Y[:, :, 1:, :] -= G[:, :, :-1, :]
    Y[:, :, :-1, :] -= G[:, :, 1:, :]
    Y[:, 1:, :, :] -= G[:, :-1, :, :]
    Y[:, :-1, :, :] -= G[:, 1:, :, :]
    Y[1:, :, :, :] -= G[:-1, :, :, :]
    Y[:-1, :, :, :] -= G[1:, :, :, :]
    return Y.reshape(n, s)


def laplacian_dense(dims, shift=0.0):
    """Dense matrix of the Laplacian on a grid of shape ``dims`` (tiny grids only)."""
    n = int(np.prod(dims))
    if len(dims) == 2:
        return laplacian_2d_apply(np.eye(n), dims[0], dims[1], shift)
    if len(dims) == 3:
        return laplacian_3d_apply(np.eye(n), dims[0], dims[1], dims[2], shift)
    raise ValueError("2D or 3D grids only")


def laplacian_extreme_eigs(dims, shift=0.0):
    """(lambda_min, lambda_max) of the Dirichlet Laplacian on ``dims``."""
    lo = sum(2.0 - 2.0 * np.cos(np.pi / (d + 1)) for d in dims) + shift
    hi = sum(2.0 - 2.0 * np.cos(np.pi * d / (d + 1)) for d in dims) + shift
    return lo, hi
