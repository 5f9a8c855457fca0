"""GPU FlatTSPQR (orth_create_flat, Sec. 4.2) against the oracle's FlatTSPQR.

* every call's H, R, U against the unique PQR solution (pqr_reference, eq.
  (1.1)) and against the oracle chain with the same blocks and local
  subalgorithm, at the FP64 tolerances of the tree tests
  (||dH||_F / ||W||_F <= 1e-12, ||dR||_F / ||W||_F and max |dU| <= 1e-12
  kappa_j; BCGS-PIP local problems against the oracle chain only, 1e-10);
* Y = Q C down the chain against the explicit basis times C;
* the entry points a flat handle does not support answer UNSUPPORTED;
* the stability class of the flat variant on the Sec. 6.1 Stewart workload
  (kappa = 1e4, n = 2^16, 32 columns, s = 4; 8 and 256 blocks), the class the
  oracle's own pin fixes: BCGS-PIP local problems lose orthogonality like
  eps kappa^2, BCGS-PIP+ keeps O(eps), A = QR to rounding.
"""

import sys

import numpy as np
import pytest

from oracle import metrics, pqr_reference
from oracle.flattspqr import FlatTSPQR
from synth import stewart

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


CASES = [
    # n, s, kmax, block_rows, local subalgorithm
    (3000, 4, 24, 3000, "pip+"),      # one block: the local subalgorithm itself
    (10000, 4, 40, 2500, "pip+"),     # four blocks
    (1037, 2, 16, 128, "pip+"),       # eight blocks, the last ragged (141 rows)
    (5001, 16, 64, 1001, "pip+"),     # odd block heights, s = 16 (LDS-staged row update)
    (6000, 32, 96, 1500, "pip+"),     # s = 32
    (2000, 1, 12, 250, "pip+"),       # s = 1
    (9000, 8, 248, 3000, "pip+"),     # k + s = 256
    (4000, 8, 48, 1000, "pip"),       # BCGS-PIP local problems
]


@pytest.mark.parametrize("n,s,kmax,rows,local", CASES)
def test_flat_parity(torch_cuda, n, s, kmax, rows, local):
    torch = torch_cuda
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("flat", n, s, kmax, rows, local)
    rng = np.random.default_rng(n + 3 * s + rows)
    gpu = Orthogonalizer(n, s, kmax, rows, flat=True,
                         variant=orth.ORTH_PIP if local == "pip" else orth.ORTH_PIP_PLUS)
    chain = FlatTSPQR(n, s, rows, local)
    assert (gpu.p, gpu.leaf_rows) == (chain.p, rows)
    assert gpu.levels == 0
    tol = 1e-12 if local == "pip+" else 1e-10
    Q = np.zeros((n, 0))
    Ugpu = []
    for step in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s)
        if step:
            X = X + Q @ rng.standard_normal((Q.shape[1], s))
        Hd, Rd, Ud = gpu.step(to_dev(X))
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        P, N, Ur = pqr_reference(Q, X)
        Pc, Nc, Uc = chain.step(X)
        kap = kappa_after_projection(N, X)
        xn = np.linalg.norm(X)
        if local == "pip+":
            if step:
                assert np.linalg.norm(H - P) / xn <= tol, step
            assert np.linalg.norm(R - N) / xn <= tol * kap, step
            assert np.max(np.abs(U - Ur)) <= tol * kap, step
        if step:
            assert np.linalg.norm(H - Pc) / xn <= tol * kap, step
        assert np.linalg.norm(R - Nc) / xn <= tol * kap, step
        assert np.max(np.abs(U - Uc)) <= tol * kap, step
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)
        Ugpu.append(U)
        Q = np.hstack([Q, Ur])
    st, info = gpu.status()
    assert st == 0, info
    V = np.hstack(Ugpu)
    assert metrics.e_perp(V) <= (1e-12 if local == "pip+" else 1e-10)
    # Y = Q C down the chain (two column blocks of the apply when m > 16)
    C = rng.standard_normal((gpu.k, 19))
    Cd = to_dev(C)
    Y = to_host(gpu.apply_Q(Cd))
    assert np.max(np.abs(Y - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    Yc = chain.apply_Q(C)
    assert np.max(np.abs(Y - Yc)) <= 1e-11 * np.abs(C).sum(0).max()
    # what a flat handle does not support
    Y2 = torch.empty((19, n), dtype=torch.float64, device="cuda")
    assert orth.orth_apply_Q_noalloc(gpu.h, Cd.data_ptr(), gpu.k, 19, Y2.data_ptr(), n) == orth.ORTH_ERR_UNSUPPORTED
    assert orth.orth_export_local(gpu.h, Y2.data_ptr(), n, None, 1) == orth.ORTH_ERR_UNSUPPORTED
    assert orth.orth_export_tree_level(gpu.h, 0, Y2.data_ptr(), n) == orth.ORTH_ERR_UNSUPPORTED
    assert orth.orth_set_deflation(gpu.h, 1e-6) == orth.ORTH_ERR_UNSUPPORTED
    # a call past k_max is refused without touching the chain
    if gpu.k + s > kmax:
        W = to_dev(rng.standard_normal((n, s)))
        with pytest.raises(orth.OrthError):
            gpu.step(W)
    gpu.close()


@pytest.fixture(scope="module")
def stewart_1e4():
    return stewart(2 ** 16, 32, 1e4, 0)


@pytest.mark.parametrize("p", [8, 256])
def test_flat_stability_class(torch_cuda, stewart_1e4, p):
    torch = torch_cuda
    from paper_2204_13393_amd import Orthogonalizer, orth
    A = stewart_1e4
    n, m, s = A.shape[0], A.shape[1], 4
    for local in ("pip", "pip+"):
        _say("flat stewart", p, local)
        gpu = Orthogonalizer(n, s, m, n // p, flat=True,
                             variant=orth.ORTH_PIP if local == "pip" else orth.ORTH_PIP_PLUS)
        R = np.zeros((m, m))
        for j in range(m // s):
            Hd, Rd, _ = gpu.step(to_dev(A[:, j * s:(j + 1) * s]))
            R[:j * s, j * s:(j + 1) * s] = to_host(Hd)
            R[j * s:(j + 1) * s, j * s:(j + 1) * s] = to_host(Rd)
        st, info = gpu.status()
        assert st == 0, info
        Q = to_host(gpu.apply_Q(torch.eye(m, dtype=torch.float64, device="cuda")))
        e = metrics.e_perp(Q)
        if local == "pip":
            assert 1e-10 <= e <= 1e-6, (p, e)
        else:
            assert e <= 1e-12, (p, e)
        assert metrics.qr_residual(A, Q, R) <= 1e-13, (local, p)
        print(f"[flat stewart] p {p} {local}: e_perp {e:.2e}", flush=True)
        gpu.close()
