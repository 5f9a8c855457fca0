"""GPU tests of deflation at the reduction level (orth_set_deflation,
Sec. 3.1) with Householder leaves.

* parity with the oracle's TreeTSPQR with Householder leaves and a deflating
  BCGS-PIP+ reduction, step by step, on sequences that plant rank-deficient
  blocks (a combination of columns, a zero column, a column in the span of
  the basis, a block wholly in that span): the rank, H, R, U; the dropped
  columns of U and rows of R are exact zeros; ragged leaves, one leaf, s
  from 1 to 16, and the deflated solution's definition (SVD of the
  residual) as a second reference;
* full-rank blocks give the plain step (same results as without deflation,
  rank s, no drop counted);
* BCGS-PIP at the reduction;
* block Arnoldi with an invariant direction: the next block deflates it,
  the zero column stays deflated, A Q = Q H on the kept columns;
* argument errors, the forms that cannot deflate;
* graph capture: replays equal the eager run bitwise.
"""

import math
import sys

import numpy as np
import pytest

from oracle import TreeTSPQR, metrics, pqr_deflated_reference
from synth import normal_block

from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

DELTA = 1e-6


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


def _block(rng, n, s, Q, step):
    """Step 0 full rank; later steps mix in the basis and plant a dependence."""
    X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s)
    k = Q.shape[1]
    if k:
        X = X + Q @ rng.standard_normal((k, s))
    kind = step % 5
    if step == 0 or kind == 0:
        return X, "full"
    if kind == 1 and s >= 3:
        X[:, 1] = 0.5 * X[:, 0] - 2.0 * X[:, 2]
        return X, "combination"
    if kind == 2:
        X[:, 0] = 0.0
        return X, "zero column"
    if kind == 3 and k:
        X[:, s - 1] = Q @ rng.standard_normal(k)
        return X, "column in span Q"
    if kind == 4 and k:
        X = Q @ rng.standard_normal((k, s))
        return X, "block in span Q"
    return X, "full"


CASES = [
    # n, s, kmax, leaf_rows
    (10000, 4, 44, 1000),     # ten leaves
    (3001, 8, 64, 700),       # ragged last leaf
    (1000, 4, 28, 1000),      # one leaf
    (777, 1, 12, 100),        # s = 1
    (5000, 2, 20, 1000),
    (6000, 16, 96, 1000),     # s = 16
    (16384, 8, 80, 4096),     # two chunks per leaf
    # 256 leaves: from k + s = 72 on the reduction level has more than 16
    # partial slots per sweep, pre-summed before the deflating factorisation
    (65536, 8, 128, 256),
]


@pytest.mark.parametrize("n,s,kmax,leaf_rows", CASES)
def test_deflation_parity(torch_cuda, n, s, kmax, leaf_rows):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("deflation parity", n, s, kmax, leaf_rows)
    rng = np.random.default_rng(n * 3 + s)
    gpu = Orthogonalizer(n, s, kmax, leaf_rows, precision=orth.ORTH_FP64_HOUSEHOLDER)
    gpu.set_deflation(DELTA)
    tree = TreeTSPQR(n, s, leaf_rows, "hh", "pip+", deflate=DELTA)
    Q = np.zeros((n, 0))
    drops, dropped = 0, 0
    kinds = set()
    for step in range(kmax // s):
        X, kind = _block(rng, n, s, Q, step)
        Hd, Rd, Ud = gpu.step(to_dev(X))
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        t, steps_g, dropped_g = gpu.deflation_info()
        Pt, Nt, Ut = tree.step(X)
        Pr, Nr, Ur, tr = pqr_deflated_reference(Q, X, DELTA)
        assert t == tree.last_rank == tr, (step, kind)
        kinds.add(kind)
        if t < s:
            drops += 1
            dropped += s - t
        assert (steps_g, dropped_g) == (drops, dropped)
        xn = max(np.linalg.norm(X), 1e-300)
        if step:
            assert np.linalg.norm(H - Pt) / xn <= 1e-12, (step, kind)
            assert np.linalg.norm(H - Pr) / xn <= 1e-12, (step, kind)
        assert np.all(R[t:] == 0.0) and np.all(U[:, t:] == 0.0), (step, kind)
        if t == s:
            assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)
        assert np.linalg.norm(R - Nt) / xn <= 1e-11, (step, kind)
        assert np.linalg.norm(R - Nr) / xn <= 1e-11, (step, kind)
        assert np.max(np.abs(U - Ut)) <= 1e-10, (step, kind)
        assert np.max(np.abs(U - Ur)) <= 1e-10, (step, kind)
        Q = np.hstack([Q, Ur])
    st, info = gpu.status()
    assert st == 0, info
    assert drops > 0
    Qe = to_host(gpu.apply_Q(to_dev(np.eye(gpu.k))))
    keep = np.linalg.norm(Qe, axis=0) > 0.5
    assert np.count_nonzero(keep) == gpu.k - dropped
    assert metrics.e_perp(Qe[:, keep]) <= 1e-12
    assert np.max(np.abs(Qe[:, ~keep])) == 0.0
    gpu.close()


@pytest.mark.parametrize("n,s,kmax,leaf_rows", [(10000, 4, 44, 1000), (16384, 8, 64, 4096),
                                                 (6000, 16, 64, 1000)])
def test_full_rank_blocks_are_the_plain_step(torch_cuda, n, s, kmax, leaf_rows):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("deflation full rank", n, s, kmax, leaf_rows)
    rng = np.random.default_rng(n + 5 * s)
    a = Orthogonalizer(n, s, kmax, leaf_rows, precision=orth.ORTH_FP64_HOUSEHOLDER)
    b = Orthogonalizer(n, s, kmax, leaf_rows, precision=orth.ORTH_FP64_HOUSEHOLDER)
    b.set_deflation(DELTA)
    Q = np.zeros((n, 0))
    for step in range(kmax // s):
        X = rng.standard_normal((n, s))
        if step:
            X = X + Q @ rng.standard_normal((Q.shape[1], s))
        Ha, Ra, Ua = (to_host(x) for x in a.step(to_dev(X)))
        Hb, Rb, Ub = (to_host(x) for x in b.step(to_dev(X)))
        xn = np.linalg.norm(X)
        assert np.linalg.norm(Ha - Hb) / xn <= 1e-13
        assert np.linalg.norm(Ra - Rb) / xn <= 1e-13
        assert np.all(np.tril(Rb, -1) == 0.0)
        assert np.max(np.abs(Ua - Ub)) <= 1e-12
        Q = np.hstack([Q, Ua])
    assert b.deflation_info() == (s, 0, 0)
    assert a.deflation_info() == (s, 0, 0)
    assert a.status()[0] == 0 and b.status()[0] == 0
    a.close()
    b.close()


def test_deflation_with_pip_reduction(torch_cuda):
    from paper_2204_13393_amd import Orthogonalizer, orth
    n, s, kmax, leaf = 8000, 4, 32, 1000
    _say("deflation pip reduction", n, s, kmax, leaf)
    rng = np.random.default_rng(17)
    gpu = Orthogonalizer(n, s, kmax, leaf, precision=orth.ORTH_FP64_HOUSEHOLDER,
                         variant=orth.ORTH_PIP_PLUS, reduction_variant=orth.ORTH_PIP)
    gpu.set_deflation(DELTA)
    tree = TreeTSPQR(n, s, leaf, "hh", "pip", deflate=DELTA)
    Q = np.zeros((n, 0))
    for step in range(kmax // s):
        X, kind = _block(rng, n, s, Q, step)
        H, R, U = (to_host(x) for x in gpu.step(to_dev(X)))
        Pt, Nt, Ut = tree.step(X)
        assert gpu.deflation_info()[0] == tree.last_rank, (step, kind)
        xn = max(np.linalg.norm(X), 1e-300)
        if step:
            assert np.linalg.norm(H - Pt) / xn <= 1e-12, (step, kind)
        assert np.linalg.norm(R - Nt) / xn <= 1e-11, (step, kind)
        assert np.max(np.abs(U - Ut)) <= 1e-10, (step, kind)
        Q = np.hstack([Q, Ut])
    assert gpu.status()[0] == 0
    gpu.close()


def test_block_arnoldi_deflates_an_invariant_direction(torch_cuda):
    """A diagonal operator and a start block holding the eigenvector e_7: the
    second block drops A u_0 (already in the basis), its zero column is
    dropped again in every later block, and A Q_k = Q_{k+s} H holds."""
    import torch
    from paper_2204_13393_amd import Orthogonalizer, orth
    n, s, leaf, steps = 50000, 4, 5000, 6
    _say("deflation arnoldi", n, s, leaf, steps)
    kmax = (steps + 1) * s
    rng = np.random.default_rng(2)
    d = np.linspace(1.0, 3.0, n)
    X = rng.standard_normal((n, s))
    X[:, 0] = 0.0
    X[7, 0] = 1.0
    gpu = Orthogonalizer(n, s, kmax, leaf, precision=orth.ORTH_FP64_HOUSEHOLDER)
    gpu.set_deflation(DELTA)
    tree = TreeTSPQR(n, s, leaf, "hh", "pip+", deflate=DELTA)
    dd = torch.from_numpy(d).to("cuda")
    Hess = np.zeros((kmax, steps * s))
    _, _, Ud = gpu.step(to_dev(X))
    _, _, Ut = tree.step(X)
    ranks = [gpu.deflation_info()[0]]
    for j in range(steps):
        Wd = Ud * dd[None, :]
        Hd, Rd, Ud = gpu.step(Wd.contiguous())
        W = to_host(Wd)
        Pt, Nt, Ut = tree.step(d[:, None] * Ut)
        ranks.append(gpu.deflation_info()[0])
        assert ranks[-1] == tree.last_rank
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        wn = np.linalg.norm(W)
        assert np.linalg.norm(H - Pt) / wn <= 1e-11 and np.linalg.norm(R - Nt) / wn <= 1e-11
        assert np.max(np.abs(U - Ut)) <= 1e-10
        Hess[:(j + 1) * s, j * s:(j + 1) * s] = H
        Hess[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = R
    assert ranks == [s] + [s - 1] * steps
    Qe = to_host(gpu.apply_Q(to_dev(np.eye(gpu.k))))
    keep = np.linalg.norm(Qe, axis=0) > 0.5
    assert metrics.e_perp(Qe[:, keep]) <= 1e-12
    Qk = Qe[:, :steps * s]
    AQ = d[:, None] * Qk
    assert np.linalg.norm(AQ - Qe @ Hess) <= 1e-11 * np.linalg.norm(AQ)
    assert gpu.status()[0] == 0
    gpu.close()


def test_deflation_arguments(torch_cuda):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("deflation arguments")
    h = Orthogonalizer(4096, 4, 16, 1024, precision=orth.ORTH_FP64_HOUSEHOLDER)
    for bad in (-1e-6, 1.0, 2.0, math.nan, math.inf):
        assert orth.orth_set_deflation(h.h, bad) == orth.ORTH_ERR_ARG, bad
    assert orth.orth_set_deflation(h.h, 0.0) == 0
    assert orth.orth_set_deflation(h.h, 1e-6) == 0
    assert orth.orth_set_deflation(None, 1e-6) == orth.ORTH_ERR_ARG
    assert orth.orth_deflation_info(None)[0] == orth.ORTH_ERR_ARG
    assert h.deflation_info() == (4, 0, 0)
    h.close()
    for prec in (orth.ORTH_FP64, orth.ORTH_MIXED_SPLIT32):
        g = Orthogonalizer(4096, 4, 16, 1024, precision=prec)
        assert orth.orth_set_deflation(g.h, 1e-6) == orth.ORTH_ERR_UNSUPPORTED
        assert orth.orth_set_deflation(g.h, 0.0) == 0
        assert g.deflation_info() == (4, 0, 0)
        g.close()
    # Householder leaves at s = 32: the reduction level's eigen solver stops at s = 16
    g = Orthogonalizer(8192, 32, 64, 4096, precision=orth.ORTH_FP64_HOUSEHOLDER)
    assert orth.orth_set_deflation(g.h, 1e-6) == orth.ORTH_ERR_UNSUPPORTED
    assert orth.orth_set_deflation(g.h, 0.0) == 0
    g.close()


def test_deflation_graph_replay(torch_cuda):
    """Five steps (two of them deflating) captured in a hipGraph and replayed
    from fresh handles on the same workspace, eager work between replays:
    every replay equals the eager run bitwise, and each fresh handle's
    record counts the replay's own drops."""
    import torch
    from paper_2204_13393_amd import orth
    _say("deflation graph")
    n, s, kmax, leaf = 16384, 8, 40, 4096
    H_ = orth.ORTH_FP64_HOUSEHOLDER
    rng = np.random.default_rng(31)
    Xh = [normal_block(n, s, 90 + j) for j in range(5)]
    Xh[2][:, 3] = 0.0
    Xh[4][:, 1] = Xh[4][:, 0] + Xh[4][:, 2]
    X = [to_dev(x) for x in Xh]
    nbytes = orth.orth_workspace_bytes(n, s, kmax, leaf, H_)
    side = torch.cuda.Stream()

    def buffers():
        return (torch.zeros((kmax, kmax), dtype=torch.float64, device="cuda"),
                torch.empty((kmax, n), dtype=torch.float64, device="cuda"))

    def make():
        code, h = orth.orth_create(n, s, kmax, leaf, H_, wp, nbytes, side.cuda_stream)
        assert code == 0
        assert orth.orth_set_deflation(h, DELTA) == 0
        return h

    def run(h, H, U):
        for j in range(5):
            k = j * s
            col = H[j * s:(j + 1) * s]
            hp = col.data_ptr() if k else 0
            assert orth.orth_step(h, X[j].data_ptr(), n, hp, kmax, col[:, k:].data_ptr(), kmax,
                                  U[k:k + s].data_ptr(), n) == 0

    ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    He, Ue = buffers()
    with torch.cuda.stream(side):
        h = make()
        run(h, He, Ue)
    side.synchronize()
    assert orth.orth_status(h)[1] == 0
    assert orth.orth_deflation_info(h) == (0, s - 1, 2, 2)
    orth.orth_destroy(h)
    He_h, Ue_h = to_host(He), to_host(Ue)
    keep = np.linalg.norm(Ue_h, axis=0) > 0.5
    assert np.count_nonzero(keep) == 5 * s - 2
    assert metrics.e_perp(Ue_h[:, keep]) <= 1e-12

    Hg, Ug = buffers()
    with torch.cuda.stream(side):
        h = make()
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        run(h, Hg, Ug)
    orth.orth_destroy(h)
    for rep in range(3):
        h = make()
        side.synchronize()
        Hg.zero_()
        Ug.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        code, st, info = orth.orth_status(h)
        assert code == 0 and st == 0, info
        assert orth.orth_deflation_info(h) == (0, s - 1, 2, 2), rep
        assert np.array_equal(to_host(Hg), He_h), rep
        assert np.array_equal(to_host(Ug), Ue_h), rep
        orth.orth_destroy(h)
        x = torch.randn(1000, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())


def test_deflation_full_size_stewart(torch_cuda):
    """The precision workload at its full size (n = 2^24, s = 8, 30 calls,
    leaf height 4096, sigma from 1 to 1e-12): with deflation the run ends
    without breakdown; per call, the rank equals the number of singular
    values of the projected block (torch's SVD of W_j - Q Q^T W_j on the
    device) above delta ||W_j||_F wherever none lies within a factor 2 of
    that threshold; dropped columns of Q and rows of R are exact zeros; the
    kept columns are orthonormal; W = Q R to the dropped energy."""
    import torch
    from paper_2204_13393_amd import orth
    n, m, s, leaf = 1 << 24, 240, 8, 4096
    _say("deflation full size stewart", n, m, s, leaf)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    Gt = torch.randn((m, n), dtype=torch.float64, device="cuda", generator=gen)
    Gt /= math.sqrt(n)
    Vh, _ = torch.linalg.qr(torch.randn((m, m), dtype=torch.float64, device="cuda", generator=gen))
    sig = torch.logspace(0.0, -12.0, m, dtype=torch.float64, device="cuda")
    Wt = torch.mm(Vh * sig, Gt)
    del Gt
    Qt = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    Rt = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    H_ = orth.ORTH_FP64_HOUSEHOLDER
    nbytes = orth.orth_workspace_bytes(n, s, m, leaf, H_)
    ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    code, h = orth.orth_create(n, s, m, leaf, H_, wp, nbytes, torch.cuda.current_stream().cuda_stream)
    assert code == 0
    assert orth.orth_set_deflation(h, DELTA) == 0
    checked, total_drop = 0, 0
    for j in range(m // s):
        k = j * s
        col = Rt[k:k + s]
        assert orth.orth_step(h, Wt[k:k + s].data_ptr(), n, col.data_ptr(), m, col[:, k:].data_ptr(), m,
                              Qt[k:k + s].data_ptr(), n) == 0
        code, t, _, dropped = orth.orth_deflation_info(h)
        assert code == 0
        # Qt row c is column c of Q; Rt[c, r] = R[r, c]
        assert torch.all(Qt[k + t:k + s] == 0.0) and torch.all(Rt[k:k + s, k + t:k + s] == 0.0), j
        Wj = Wt[k:k + s]
        Rj = Wj - torch.mm(torch.mm(Wj, Qt[:k].t()), Qt[:k]) if k else Wj.clone()
        Rj -= torch.mm(torch.mm(Rj, Qt[:k].t()), Qt[:k]) if k else 0.0
        sv = torch.linalg.svdvals(torch.mm(Rj, Rj.t())).sqrt()
        thr = DELTA * float(torch.linalg.norm(Wj))
        if not bool(torch.any((sv > 0.5 * thr) & (sv < 2.0 * thr))):
            assert t == int(torch.count_nonzero(sv > thr)), j
            checked += 1
        total_drop += s - t
        del Rj
    assert dropped == total_drop > 0
    assert checked >= 10
    code, st, info = orth.orth_status(h)
    assert code == 0 and st == 0, info
    orth.orth_destroy(h)
    keep = torch.linalg.vector_norm(Qt, dim=1) > 0.5
    assert int(keep.sum()) == m - total_drop
    Qk = Qt[keep]
    Gq = torch.mm(Qk, Qk.t())
    Gq -= torch.eye(Qk.shape[0], dtype=torch.float64, device="cuda")
    assert float(torch.linalg.matrix_norm(Gq, "fro")) <= 1e-12
    del Gq, Qk
    res2 = 0.0
    for c0 in range(0, n, 1 << 21):
        D = Wt[:, c0:c0 + (1 << 21)] - torch.mm(Rt, Qt[:, c0:c0 + (1 << 21)])     # W^T = R^T Q^T
        res2 += float(torch.sum(D * D))
        del D
    assert math.sqrt(res2) / float(torch.linalg.norm(Wt)) <= 1e-5
