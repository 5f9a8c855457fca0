"""orth_apply_Q_noalloc against orth_apply_Q, through the C ABI (MI355X).

The allocation-free entry point runs the same kernels as orth_apply_Q with
the coefficient scratch in the library's fixed device array instead of the
handle's workspace, so its output must equal orth_apply_Q's bit for bit.
Two calls follow each other on the same array, the second with a smaller
input; a handle whose coefficient column does not fit the array is refused
with ORTH_ERR_SCRATCH before anything is enqueued.  Y is also checked
against V C with V the explicit blocks the steps returned (tolerance
1e-12 max|C| column sums, as in the parity tests).
"""

import sys

import numpy as np
import pytest

from gpu_util import to_dev, to_host

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


def _grown(n, s, kmax, leaf_rows, precision, seed):
    """A handle after kmax / s steps on Gaussian blocks, and its explicit basis."""
    from paper_2204_13393_amd import Orthogonalizer
    gpu = Orthogonalizer(n, s, kmax, leaf_rows, precision=precision)
    rng = np.random.default_rng(seed)
    V = []
    for _ in range(kmax // s):
        X = rng.standard_normal((n, s))
        _, _, U = gpu.step(to_dev(X))
        V.append(to_host(U))
    st, info = gpu.status()
    assert st == 0, info
    return gpu, np.hstack(V)


def _both(torch, gpu, C):
    """(orth_apply_Q's Y, orth_apply_Q_noalloc's Y) for C (k x m, host)."""
    from paper_2204_13393_amd import orth
    n = gpu.n
    k, m = C.shape
    Cd = to_dev(C)
    Y1 = torch.full((m, n), np.nan, dtype=torch.float64, device="cuda")
    Y2 = torch.full((m, n), np.nan, dtype=torch.float64, device="cuda")
    assert orth.orth_apply_Q(gpu.h, Cd.data_ptr(), k, m, Y1.data_ptr(), n) == orth.ORTH_OK
    assert orth.orth_apply_Q_noalloc(gpu.h, Cd.data_ptr(), k, m, Y2.data_ptr(), n) == orth.ORTH_OK
    torch.cuda.synchronize()
    return to_host(Y1), to_host(Y2)


# (n, s, k_max, leaf_rows, precision, m first, m second)
CASES = [
    (200000, 8, 64, 4096, 0, 37, 5),      # 48 leaves: blocks of 16 columns
    (300000, 4, 32, 32, 0, 20, 3),        # 9375 leaves: p k_max = 300000, blocks of 13
    (40000, 8, 48, 2000, 2, 19, 2),       # Householder leaves: two scratch regions
]


@pytest.mark.parametrize("n,s,kmax,leaf_rows,precision,m1,m2", CASES)
def test_noalloc_matches_apply_Q(torch_cuda, n, s, kmax, leaf_rows, precision, m1, m2):
    torch = torch_cuda
    _say("noalloc", n, s, kmax, leaf_rows, precision, m1, m2)
    gpu, V = _grown(n, s, kmax, leaf_rows, precision, seed=n + s)
    rng = np.random.default_rng(n)
    k = gpu.k
    for m in (m1, m2):                      # two calls in a row, the second smaller
        C = rng.standard_normal((k, m))
        Y1, Y2 = _both(torch, gpu, C)
        assert np.array_equal(Y1, Y2), (m, np.max(np.abs(Y1 - Y2)))
        assert np.max(np.abs(Y2 - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    gpu.close()


def test_noalloc_smaller_handle_after_larger(torch_cuda):
    """A call on a small handle right after one on a large handle (same array)."""
    torch = torch_cuda
    _say("noalloc large then small")
    big, Vb = _grown(300000, 4, 32, 32, 0, seed=1)
    small, Vs = _grown(5000, 2, 8, 1000, 0, seed=2)
    rng = np.random.default_rng(3)
    for gpu, V, m in ((big, Vb, 16), (small, Vs, 3)):
        C = rng.standard_normal((gpu.k, m))
        Y1, Y2 = _both(torch, gpu, C)
        assert np.array_equal(Y1, Y2)
        assert np.max(np.abs(Y2 - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    big.close()
    small.close()


def test_noalloc_refuses_oversized(torch_cuda):
    """p k_max above the array's 4 Mi doubles: ORTH_ERR_SCRATCH, nothing enqueued."""
    torch = torch_cuda
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("noalloc oversized")
    n = (4 << 20) + 1                       # leaf_rows = k_max = 1: p k_max > 4 Mi
    gpu = Orthogonalizer(n, 1, 1, 1)
    Y = torch.zeros((1, n), dtype=torch.float64, device="cuda")
    C = torch.ones((1, 1), dtype=torch.float64, device="cuda")
    code = orth.orth_apply_Q_noalloc(gpu.h, C.data_ptr(), 1, 1, Y.data_ptr(), n)
    assert code == orth.ORTH_ERR_SCRATCH
    torch.cuda.synchronize()
    assert float(Y.abs().max()) == 0.0
    gpu.close()
