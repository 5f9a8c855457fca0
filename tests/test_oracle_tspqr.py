"""Pins for the oracle's TreeTSPQR (CPU only).

* the paper's printed numbers (Sec. 6.1 stability table, stored in
  tests/golden/paper_stability_tables.json): Stewart kappa = 1e4,
  n = 2^16, 32 columns, s = 4.  e_perp and ||A - QR|| must fall in the band
  [min/10, 10*max] of the printed column for BCGS-PIP and BCGS-PIP+;
* uniqueness of the PQR solution: for any leaf partition and tree shape the
  global (P, N, U) equals the reference solution;
* Sec. 4.1's orthonormality of the stacked factors and the local bases;
* consistency of the representation: apply_Q(C) = explicit Q C.

Readings: "recursion level l" is a fan-in-2 tree of depth l with 2^l leaves;
"subproblems in two levels" is the single-level tree (leaves + one
reduction) with that many leaves.
"""

import json
import os

import numpy as np
import pytest

from oracle import TreeTSPQR, leaf_bounds, metrics, pqr_reference
from oracle.krylov import block_column_qr
from synth import stewart

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "paper_stability_tables.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def stewart_1e4():
    return stewart(2 ** 16, 32, 1e4, 0)


def _band(golden, table, col):
    vals = [row[col] for row in golden[table].values()]
    return min(vals) / 10.0, max(vals) * 10.0


def _run(A, p, fan_in, sub):
    n = A.shape[0]
    solver = TreeTSPQR(n, 4, n // p, sub, sub, fan_in)
    Q, R = block_column_qr(A, 4, solver)
    Qe = solver.explicit_Q()
    assert np.allclose(Qe, Q, atol=1e-12)
    return metrics.e_perp(Qe), np.linalg.norm(A - Qe @ R, "fro"), metrics.qr_residual(A, Qe, R)


@pytest.mark.parametrize("level", [0, 3, 8])
def test_recursion_levels_match_paper_table(golden, stewart_1e4, level):
    for sub, ecol, rcol in (("pip", 0, 3), ("pip+", 1, 4)):
        e, res_abs, res_rel = _run(stewart_1e4, 2 ** level, 2, sub)
        lo, hi = _band(golden, "recursion_levels", ecol)
        assert lo <= e <= hi, (sub, level, e, lo, hi)
        rlo, rhi = _band(golden, "recursion_levels", rcol)
        assert rlo <= res_abs <= rhi and rlo <= res_rel <= rhi


@pytest.mark.parametrize("p", [8, 64, 1024])
def test_subproblem_count_matches_paper_table(golden, stewart_1e4, p):
    for sub, ecol, rcol in (("pip", 0, 3), ("pip+", 1, 4)):
        e, res_abs, res_rel = _run(stewart_1e4, p, None, sub)
        lo, hi = _band(golden, "subproblems", ecol)
        assert lo <= e <= hi, (sub, p, e, lo, hi)
        rlo, rhi = _band(golden, "subproblems", rcol)
        assert rlo <= res_abs <= rhi and rlo <= res_rel <= rhi


@pytest.mark.parametrize("n,s,leaf_rows,fan_in", [(1000, 4, 100, None), (1037, 3, 128, None),
                                                    (999, 2, 64, 3), (512, 8, 512, None),
                                                    (2000, 5, 90, 4)])
def test_tree_equals_unique_reference(n, s, leaf_rows, fan_in):
    """Open loop: same X each step to the tree and to the explicit reference."""
    rng = np.random.default_rng(n + s)
    tree = TreeTSPQR(n, s, leaf_rows, "pip+", "pip+", fan_in)
    Q = np.zeros((n, 0))
    for step in range(6):
        X = rng.standard_normal((n, s)) * np.geomspace(1, 1e-2, s)
        if step:
            X += Q @ rng.standard_normal((Q.shape[1], s))
        P, N, U = tree.step(X)
        Pr, Nr, Ur = pqr_reference(Q, X)
        assert np.linalg.norm(P - Pr) / np.linalg.norm(X) < 1e-13
        assert np.linalg.norm(N - Nr) / np.linalg.norm(X) < 1e-13
        assert np.max(np.abs(U - Ur)) < 1e-11
        Q = np.hstack([Q, Ur])
    # local and stacked-factor orthonormality (Sec. 4.1)
    for Qi in tree.leaves:
        assert metrics.e_perp(Qi) < 1e-13
    for level in range(len(tree.levels)):
        for node in tree.levels[level]:
            Sv = np.vstack(node["S"])
            assert metrics.e_perp(Sv) < 1e-13
    C = rng.standard_normal((tree.k, 3))
    assert np.allclose(tree.apply_Q(C), tree.explicit_Q() @ C, atol=1e-12)
    assert np.allclose(tree.explicit_Q(), Q, atol=1e-11)


def test_leaf_bounds_ragged():
    assert leaf_bounds(10, 3) == [(0, 3), (3, 6), (6, 10)]
    assert leaf_bounds(5, 8) == [(0, 5)]
    assert leaf_bounds(16, 4) == [(0, 4), (4, 8), (8, 12), (12, 16)]


def test_refuses_rank_deficient_local_problem():
    tree = TreeTSPQR(40, 4, 8)
    rng = np.random.default_rng(0)
    tree.step(rng.standard_normal((40, 4)))
    tree.step(rng.standard_normal((40, 4)))
    with pytest.raises(ValueError):
        tree.step(rng.standard_normal((40, 4)))


# ---- Householder at the reduction (single-level tree)

def _signfix(P, N, U):
    d = np.sign(np.diag(N))
    d[d == 0] = 1.0
    return P, d[:, None] * N, U * d[None, :]


@pytest.mark.parametrize("n,s,leaf_rows,local", [(1000, 4, 100, "pip+"), (1037, 3, 128, "hh"),
                                                   (512, 8, 512, "hh"), (2000, 2, 90, "ref"),
                                                   (777, 1, 70, "pip")])
def test_householder_reduction_equals_unique_reference(n, s, leaf_rows, local):
    """Open loop with the reduction node's basis as reflectors: (P, N D, U D)
    with D = diag(sign N_ii) equals the unique solution; the basis stays
    orthonormal and apply_Q matches the explicit basis."""
    rng = np.random.default_rng(n + 7 * s)
    tree = TreeTSPQR(n, s, leaf_rows, local, "hh")
    Q = np.zeros((n, 0))
    tol = 1e-11 if local == "pip" else 1e-13
    for step in range(5):
        X = rng.standard_normal((n, s)) * np.geomspace(1, 1e-2, s)
        if step:
            X += Q @ rng.standard_normal((Q.shape[1], s))
        P, N, Uraw = tree.step(X)
        P, N, U = _signfix(P, N, Uraw)
        Pr, Nr, Ur = pqr_reference(Q, X)
        assert np.linalg.norm(P - Pr) / np.linalg.norm(X) < tol
        assert np.linalg.norm(N - Nr) / np.linalg.norm(X) < tol
        assert np.max(np.abs(U - Ur)) < 100 * tol
        Q = np.hstack([Q, Uraw])
    Sv = tree.stacked_factor(0)
    assert metrics.e_perp(Sv) < 1e-13
    C = rng.standard_normal((tree.k, 3))
    assert np.allclose(tree.apply_Q(C), tree.explicit_Q() @ C, atol=1e-12)
    assert np.allclose(tree.explicit_Q(), Q, atol=1e-11)


def test_householder_reduction_inserted_rows_are_zero():
    """After the second call every old reflector of the reduction node has
    exact zeros in the rows of each child's newest coordinates."""
    n, s, lr = 400, 4, 100
    rng = np.random.default_rng(3)
    tree = TreeTSPQR(n, s, lr, "pip+", "hh")
    tree.step(rng.standard_normal((n, s)))
    tree.step(rng.standard_normal((n, s)))
    V = tree.root_hh.V
    assert V.shape == (4 * 2 * s, 2 * s)
    for c in range(4):
        assert np.all(V[c * 2 * s + s:c * 2 * s + 2 * s, :s] == 0.0)


def test_householder_reduction_refusals():
    with pytest.raises(ValueError):
        TreeTSPQR(1000, 4, 100, "hh", "hh", deflate=1e-6)


@pytest.mark.parametrize("n,s,leaf_rows,fan_in,local", [(2000, 4, 100, 2, "hh"), (3000, 3, 150, 3, "pip+"),
                                                          (1037, 2, 64, 4, "hh"), (4096, 8, 256, 2, "ref")])
def test_householder_tree_equals_unique_reference(n, s, leaf_rows, fan_in, local):
    """Householder at every node of a reduction tree (fan-in 2..4, ragged
    groups): (P, N D, U D) equals the unique solution; every node's stacked
    factor stays orthonormal."""
    rng = np.random.default_rng(n + fan_in)
    tree = TreeTSPQR(n, s, leaf_rows, local, "hh", fan_in)
    assert len(tree.levels) > 1
    Q = np.zeros((n, 0))
    for step in range(5):
        X = rng.standard_normal((n, s)) * np.geomspace(1, 1e-2, s)
        if step:
            X += Q @ rng.standard_normal((Q.shape[1], s))
        P, N, Uraw = tree.step(X)
        P, N, U = _signfix(P, N, Uraw)
        Pr, Nr, Ur = pqr_reference(Q, X)
        assert np.linalg.norm(P - Pr) / np.linalg.norm(X) < 1e-13
        assert np.linalg.norm(N - Nr) / np.linalg.norm(X) < 1e-13
        assert np.max(np.abs(U - Ur)) < 1e-11
        Q = np.hstack([Q, Uraw])
    for level in range(len(tree.levels)):
        for node in tree.levels[level]:
            assert metrics.e_perp(np.vstack(node["S"])) < 1e-13
    C = rng.standard_normal((tree.k, 3))
    assert np.allclose(tree.apply_Q(C), tree.explicit_Q() @ C, atol=1e-12)


@pytest.mark.parametrize("level", [1, 3, 8])
def test_recursion_levels_householder_column(golden, stewart_1e4, level):
    """The Householder column of the recursion-levels table (Sec. 6.1):
    Householder at the leaves and at every node of the fan-in-2 tree."""
    e, res_abs, res_rel = _run(stewart_1e4, 2 ** level, 2, "hh")
    lo, hi = _band(golden, "recursion_levels", 2)
    assert lo <= e <= hi, (level, e, lo, hi)
    rlo, rhi = _band(golden, "recursion_levels", 5)
    assert rlo <= res_abs <= rhi and rlo <= res_rel <= rhi


@pytest.mark.parametrize("p", [8, 64, 256])
def test_subproblem_count_householder_column(golden, stewart_1e4, p):
    """The Householder column of the subproblems table (Sec. 6.1): one
    method at both levels, so Householder leaves and a Householder
    reduction; e_perp and ||A - QR|| within [min / 10, 10 max]."""
    e, res_abs, res_rel = _run(stewart_1e4, p, None, "hh")
    lo, hi = _band(golden, "subproblems", 2)
    assert lo <= e <= hi, (p, e, lo, hi)
    rlo, rhi = _band(golden, "subproblems", 5)
    assert rlo <= res_abs <= rhi and rlo <= res_rel <= rhi


def test_householder_at_both_levels_is_unconditionally_stable():
    """Sec. 2.2 / 6.1: with Householder at both levels e_perp stays O(eps)
    far past the CholeskyQR bound (kappa = 1e12, where BCGS-PIP+ at either
    level breaks down or loses orthogonality)."""
    from oracle.pqr import Breakdown
    A = stewart(2 ** 14, 32, 1e12, 1)
    n = A.shape[0]
    tree = TreeTSPQR(n, 4, 256, "hh", "hh")
    Q, R = block_column_qr(A, 4, tree)
    assert metrics.e_perp(tree.explicit_Q()) <= 1e-13
    assert metrics.qr_residual(A, Q, R) <= 1e-13
    for local, red in (("pip+", "hh"), ("hh", "pip+")):
        tree = TreeTSPQR(n, 4, 256, local, red)
        try:
            block_column_qr(A, 4, tree)
        except Breakdown:
            continue
        assert metrics.e_perp(tree.explicit_Q()) >= 1e-6, (local, red)
