"""Element-wise parity at the reduction level's wide launch shapes.

The reduction problem (Sec. 4.1: the PQR problem on the stacked leaf
coefficient blocks [[T_i, P_i], [0, N_i]]) has p (k + s) rows.  Its launch
shape grows with the number of leaves p and the width k + s:

* k + s >= 65 runs the Gram product with 2 or 4 tile groups per workgroup;
* k + s > 256 adds column groups;
* more than 16 partial slots per sweep go through fixed-order pre-sums
  (k_reduce) before the factorisation.

Every case here reaches those shapes and compares every call's H, R and U
with the oracle's unique PQR solution (open loop: both sides get the same
block, built from the oracle's basis), and the locally orthogonal factors
with the oracle's TreeTSPQR on the same leaves:

* n = 2^20, leaf 4096 (256 leaves), s = 8, k_max = 248: the headline shape
  with 256 leaves; and the same blocks with leaf 256 (4096 leaves), which
  is exactly the reduction-level geometry of the 2^24-row headline run
  (that geometry depends on p and k only);
* s = 32 with 128 leaves and k_max = 544: 4 tile groups, 3 column groups
  and pre-sums at the reduction level.

Tolerances are those of test_gpu_parity.py (FP64 form): ||dH||_F/||X||_F
<= 1e-12, ||dR||_F/||X||_F and max |dU| <= 1e-12 kappa_j, local factors
<= 1e-11 kappa.
"""

import sys

import numpy as np
import pytest

from oracle import TreeTSPQR, metrics, pqr_reference

from gpu_util import kappa_after_projection, to_dev, to_host

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_13393_amd import orth
    orth.load()
    return torch


def _open_loop(n, s, kmax, seed, tree_leaf):
    """Blocks X_j (N(0,1) columns scaled 1 .. 1/4 plus a random combination of
    the oracle's basis), the oracle's (P, N, U, kappa_j) for each, and the
    oracle TreeTSPQR with leaves of tree_leaf rows run over the same blocks."""
    rng = np.random.default_rng(seed)
    tree = TreeTSPQR(n, s, tree_leaf, "pip+", "pip+")
    Q = np.zeros((n, 0))
    steps = []
    for j in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s)
        if j:
            X = X + Q @ rng.standard_normal((Q.shape[1], s))
        P, N, U = pqr_reference(Q, X)
        tree.step(X)
        steps.append((X, P, N, U, kappa_after_projection(N, X)))
        Q = np.hstack([Q, U])
        if j % 8 == 0:
            _say(f"oracle step {j} of {kmax // s} (n={n}, s={s})")
    return steps, tree


def _check_steps(gpu, steps, label):
    kap_max = 1.0
    for j, (X, P, N, U, kap) in enumerate(steps):
        H, R, Ug = (to_host(t) for t in gpu.step(to_dev(X)))
        xn = np.linalg.norm(X)
        if j:
            assert np.linalg.norm(H - P) / xn <= 1e-12, (label, j)
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0), (label, j)
        assert np.linalg.norm(R - N) / xn <= 1e-12 * kap, (label, j)
        assert np.max(np.abs(Ug - U)) <= 1e-12 * kap, (label, j)
        kap_max = max(kap_max, kap)
    st, info = gpu.status()
    assert st == 0, (label, info)
    return kap_max


@pytest.fixture(scope="module")
def headline_rows_2m():
    return _open_loop(1 << 20, 8, 248, 2024, 4096)


def test_256_leaves_every_call(torch_cuda, headline_rows_2m):
    """n = 2^20, leaf 4096, s = 8, k_max = 248: 31 calls, k + s up to 248
    (four tile groups at the reduction level, 31 root chunks, pre-sums)."""
    from paper_2204_13393_amd import Orthogonalizer
    steps, tree = headline_rows_2m
    n, s, kmax, leaf = 1 << 20, 8, 248, 4096
    _say("reduction shapes: 256 leaves", n, s, kmax, leaf)
    gpu = Orthogonalizer(n, s, kmax, leaf)
    kap = _check_steps(gpu, steps, "256 leaves")
    Qloc, T = (to_host(t) for t in gpu.export_local())
    assert np.max(np.abs(T - tree.stacked_factor(0))) <= 1e-11 * kap
    assert np.max(np.abs(Qloc - np.vstack(tree.leaves))) <= 1e-11 * kap
    assert metrics.e_perp(T) <= 1e-12
    rng = np.random.default_rng(5)
    C = rng.standard_normal((gpu.k, 3))
    V = np.hstack([st[3] for st in steps])
    Y = to_host(gpu.apply_Q(to_dev(C)))
    assert np.max(np.abs(Y - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    gpu.close()


def test_4096_leaves_every_call(torch_cuda, headline_rows_2m):
    """The same blocks with leaf 256: 4096 leaves, i.e. the reduction-level
    geometry of the 2^24-row headline run (496 root chunks at k + s = 248).
    Global results against the oracle at every call; the local factors
    through properties (orthonormal leaves and stacked factor)."""
    from paper_2204_13393_amd import Orthogonalizer
    steps, _ = headline_rows_2m
    n, s, kmax, leaf = 1 << 20, 8, 248, 256
    _say("reduction shapes: 4096 leaves", n, s, kmax, leaf)
    gpu = Orthogonalizer(n, s, kmax, leaf)
    _check_steps(gpu, steps, "4096 leaves")
    Qloc, T = (to_host(t) for t in gpu.export_local())
    assert metrics.e_perp(T) <= 1e-12
    worst = max(metrics.e_perp(Qloc[r0:r0 + leaf]) for r0 in range(0, n, leaf))
    assert worst <= 1e-12
    gpu.close()


def test_s32_128_leaves_wide_root(torch_cuda):
    """s = 32, 128 leaves of 544 rows, k_max = 544: at k + s = 544 the
    reduction-level Gram runs 4 tile groups over 3 column groups and its 34
    partial slots are pre-summed."""
    from paper_2204_13393_amd import Orthogonalizer
    n, s, kmax, leaf = 128 * 544, 32, 544, 544
    _say("reduction shapes: s = 32, 128 leaves", n, s, kmax, leaf)
    steps, tree = _open_loop(n, s, kmax, 77, leaf)
    gpu = Orthogonalizer(n, s, kmax, leaf)
    kap = _check_steps(gpu, steps, "s32")
    Qloc, T = (to_host(t) for t in gpu.export_local())
    assert np.max(np.abs(T - tree.stacked_factor(0))) <= 1e-11 * kap
    assert np.max(np.abs(Qloc - np.vstack(tree.leaves))) <= 1e-11 * kap
    gpu.close()
