"""GPU tests of the batched form (many instances, one grouped launch per phase).

* the batch runs the same device code as single handles, on the same leaf
  geometry, so every instance's H, R and U must equal a single handle's
  bitwise, for uneven n (ragged leaves) and every block width;
* against the oracle, per instance, at the parity tolerances of
  test_gpu_parity.py;
* a captured hipGraph of a closed-loop Arnoldi run (operator + batch step)
  replayed several times from a freshly created batch, eager work and
  synchronisation in between, equals the eager run bitwise every time;
* breakdown in one instance is reported with its index;
* the mixed form (ORTH_MIXED_SPLIT32): every instance equals a mixed single
  handle bitwise and the FP64 oracle at the mixed form's tolerances
  (||dP||_F / ||X||_F <= 1e-10, ||dN||_F / ||X||_F and max |dU| <= 1e-10
  kappa_j); a first-sweep pivot that fails on the FP32 copy of one
  instance redoes that instance's sweep only, in a graph replay too;
* Householder leaves (ORTH_FP64_HOUSEHOLDER, s from 1 to 32): every instance
  equals a Householder single handle bitwise and the unique PQR solution at
  the FP64 tolerances; the BCGS-PIP variant is refused.
"""

import sys

import numpy as np
import pytest

from oracle import pqr_reference
from synth import normal_block

from gpu_util import kappa_after_projection, to_dev, to_host

pytestmark = pytest.mark.gpu

INSTANCES = [  # n, s, k_max, leaf_rows (0: default)
    (5000, 4, 24, 1000),
    (3001, 8, 48, 700),
    (777, 1, 6, 100),
    (6000, 16, 96, 2000),
    (4100, 32, 192, 2048),
    (2600, 32, 192, 0),
    (10000, 2, 12, 0),
    (16384, 8, 48, 4096),
]
STEPS = 6


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


def _inputs(seed):
    rng = np.random.default_rng(seed)
    out = []
    for (n, s, km, lr) in INSTANCES:
        out.append([rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s) for _ in range(STEPS)])
    return out


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_equals_single_handles_bitwise(torch_cuda, precision):
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, Orthogonalizer
    _say("batch vs single", len(INSTANCES), "precision", precision)
    X = _inputs(3)
    ns = [i[0] for i in INSTANCES]
    ss = [i[1] for i in INSTANCES]
    ks = [i[2] for i in INSTANCES]
    lrs = [i[3] for i in INSTANCES]
    tol = 1e-12 if precision == 0 else 1e-10
    b = BatchOrthogonalizer(ns, ss, ks, lrs, precision=precision)
    assert tuple(b.progress()) == (0, STEPS)
    W = [torch.empty((s, n), dtype=torch.float64, device="cuda") for (n, s, _, _) in INSTANCES]
    U = [torch.empty_like(w) for w in W]
    Hess = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
    Ub = [[] for _ in INSTANCES]
    for j in range(STEPS):
        for i, w in enumerate(W):
            w.copy_(to_dev(X[i][j]))
        b.step(W, U, Hess)
        for i, u in enumerate(U):
            Ub[i].append(to_host(u))
    st, info = b.status()
    assert st == 0, info
    assert b.mixed_fallbacks() == 0
    for i, (n, s, km, lr) in enumerate(INSTANCES):
        g = Orthogonalizer(n, s, km, lr, precision=precision)
        assert g.leaf_rows == b.leaf_rows[i]
        Hb = to_host(Hess[i])
        Q = np.zeros((n, 0))
        for j in range(STEPS):
            H, R, Uo = g.step(to_dev(X[i][j]))
            k = j * s
            assert np.array_equal(Hb[:k, j * s:(j + 1) * s], to_host(H)), (i, j)
            assert np.array_equal(Hb[k:k + s, j * s:(j + 1) * s], to_host(R)), (i, j)
            assert np.array_equal(Ub[i][j], to_host(Uo)), (i, j)
            # oracle parity of the batch result
            P, N, Ur = pqr_reference(Q, X[i][j])
            kap = kappa_after_projection(N, X[i][j])
            xn = np.linalg.norm(X[i][j])
            if k:
                assert np.linalg.norm(Hb[:k, j * s:(j + 1) * s] - P) / xn <= tol
            assert np.linalg.norm(Hb[k:k + s, j * s:(j + 1) * s] - N) / xn <= tol * kap
            assert np.max(np.abs(Ub[i][j] - Ur)) <= tol * kap
            Q = np.hstack([Q, Ur])
        g.close()
    b.close()


def _grids():
    return [(50, 60), (101, 37), (64, 64)]


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp64", "mixed", "householder"])
def test_batch_graph_replay_arnoldi(torch_cuda, precision):
    """Capture start block + 4 Arnoldi steps (operator and batch step) and replay."""
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, orth
    _say("graph replay", precision)
    grids = _grids()
    ss = [4, 8, 2]
    steps = 5
    ns = [gx * gy for gx, gy in grids]
    ks = [steps * s for s in ss]
    lrs = [1000, 1024, 0]
    R0 = [to_dev(normal_block(n, s, 40 + i)) for i, (n, s) in enumerate(zip(ns, ss))]

    def run(batch, Wb, Ub, Hb, stream):
        # start block, then W = A U_{j-1} and a step, all on `stream`
        sp = stream.cuda_stream
        for i in range(len(ns)):
            Wb[i].copy_(R0[i])
        batch.step(Wb, Ub, Hb)
        for j in range(1, steps):
            for i, (gx, gy) in enumerate(grids):
                code = orth.orth_laplacian_apply(Ub[i].data_ptr(), ns[i], Wb[i].data_ptr(), ns[i], ss[i],
                                                 gx, gy, 1, 0.0, sp)
                assert code == 0
            batch.step(Wb, Ub, Hb)

    def buffers():
        W = [torch.empty((s, n), dtype=torch.float64, device="cuda") for n, s in zip(ns, ss)]
        U = [torch.empty_like(w) for w in W]
        H = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
        return W, U, H

    side = torch.cuda.Stream()
    # eager reference
    We, Ue, He = buffers()
    with torch.cuda.stream(side):
        ref = BatchOrthogonalizer(ns, ss, ks, lrs, stream=side, precision=precision)
        run(ref, We, Ue, He, side)
    side.synchronize()
    st, info = ref.status()
    assert st == 0, info
    He_h = [to_host(h) for h in He]
    Ue_h = [to_host(u) for u in Ue]
    ref.close()

    # captured run on its own workspace
    Wg, Ug, Hg = buffers()
    with torch.cuda.stream(side):
        cap = BatchOrthogonalizer(ns, ss, ks, lrs, stream=side, precision=precision)
        ptrs = (cap.pointer_array(Wg), cap.pointer_array(Ug), cap.pointer_array(Hg))
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for i in range(len(ns)):
            Wg[i].copy_(R0[i])
        cap.step(*ptrs)
        for j in range(1, steps):
            for i, (gx, gy) in enumerate(grids):
                assert orth.orth_laplacian_apply(Ug[i].data_ptr(), ns[i], Wg[i].data_ptr(), ns[i], ss[i],
                                                 gx, gy, 1, 0.0, side.cuda_stream) == 0
            cap.step(*ptrs)
    ws = cap.workspace
    cap.close()
    for rep in range(3):
        # fresh basis state on the same workspace, eager and synchronised
        code, h = orth.orth_batch_create(ns, ss, ks, lrs, precision,
                                         (ws.data_ptr() + 255) // 256 * 256,
                                         orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, precision),
                                         side.cuda_stream)
        assert code == 0
        for t in Ug + Hg:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        code, st, info = orth.orth_batch_status(h)
        assert code == 0 and st == 0, info
        for i in range(len(ns)):
            assert np.array_equal(to_host(Hg[i]), He_h[i]), (rep, i)
            assert np.array_equal(to_host(Ug[i]), Ue_h[i]), (rep, i)
        orth.orth_batch_destroy(h)
        # some eager work of the program between replays
        x = torch.randn(1000, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())


def test_batch_breakdown_reports_instance(torch_cuda):
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, orth
    _say("batch breakdown")
    ns, ss, ks = [3000, 4000, 2500], [4, 8, 2], [8, 16, 4]
    b = BatchOrthogonalizer(ns, ss, ks, [1000, 1000, 500])
    W = [to_dev(normal_block(n, s, i)) for i, (n, s) in enumerate(zip(ns, ss))]
    U = [torch.empty_like(w) for w in W]
    H = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
    b.step(W, U, H)
    assert b.status()[0] == 0
    X = normal_block(ns[1], ss[1], 7)
    X[:, 5] = 0.0
    W = [to_dev(normal_block(ns[0], ss[0], 8)), to_dev(X), to_dev(normal_block(ns[2], ss[2], 9))]
    b.step(W, U, H)
    st, info = b.status()
    assert st == orth.ORTH_ERR_BREAKDOWN
    assert info[0] == 1 and info[1] == 0 and info[4] == 5, info
    assert orth.orth_batch_step(b.h, 0, 0, 0) == orth.ORTH_ERR_POISONED
    b.close()


def test_batch_pip_variant_equals_single(torch_cuda):
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, Orthogonalizer, orth
    _say("batch pip")
    ns, ss, ks, lrs = [4000, 1500], [4, 2], [16, 8], [1000, 500]
    b = BatchOrthogonalizer(ns, ss, ks, lrs, variant=orth.ORTH_PIP)
    singles = [Orthogonalizer(n, s, k, lr, variant=orth.ORTH_PIP) for n, s, k, lr in zip(ns, ss, ks, lrs)]
    U = [torch.empty((s, n), dtype=torch.float64, device="cuda") for n, s in zip(ns, ss)]
    H = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
    for j in range(4):
        W = [to_dev(normal_block(n, s, 100 * j + i)) for i, (n, s) in enumerate(zip(ns, ss))]
        b.step(W, U, H)
        for i, g in enumerate(singles):
            Hs, Rs, Us = g.step(W[i])
            assert np.array_equal(to_host(U[i]), to_host(Us))
            assert np.array_equal(to_host(H[i])[j * ss[i]:(j + 1) * ss[i], j * ss[i]:(j + 1) * ss[i]],
                                  to_host(Rs))
    for g in singles:
        g.close()
    b.close()


def test_batch_mixed_fallback_is_per_instance(torch_cuda):
    """Instance 1 gets a block that lies in its basis up to 1e-5 (its first
    sweep on the FP32 copy fails a pivot, as in the single-handle fallback
    test); instances 0 and 2 get well-conditioned blocks.  Exactly one redo
    is counted, and every instance equals a mixed single handle bitwise, so
    the others did not take the redo; a graph replay of the same three steps
    counts one redo per replay and equals the eager run bitwise."""
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, Orthogonalizer, orth
    _say("batch mixed fallback")
    MIX = orth.ORTH_MIXED_SPLIT32
    ns, ss, ks, lrs = [6000, 8192, 3000], [4, 8, 2], [12, 24, 6], [1500, 2048, 1000]
    rng = np.random.default_rng(21)
    n1, s1 = ns[1], ss[1]
    W0, _ = np.linalg.qr(rng.standard_normal((n1, s1)))
    X1 = W0 @ rng.standard_normal((s1, s1)) + 1e-5 * rng.standard_normal((n1, s1)) / np.sqrt(n1)
    blocks = [[normal_block(ns[0], ss[0], 50 + j) for j in range(3)],
              [W0, X1, normal_block(n1, s1, 22)],
              [normal_block(ns[2], ss[2], 60 + j) for j in range(3)]]
    Wd = [[to_dev(x) for x in bl] for bl in blocks]

    def buffers():
        U = [torch.empty((s, n), dtype=torch.float64, device="cuda") for n, s in zip(ns, ss)]
        H = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
        return U, H

    b = BatchOrthogonalizer(ns, ss, ks, lrs, precision=MIX)
    U, H = buffers()
    Ue, falls = [], []
    for j in range(3):
        b.step([Wd[i][j] for i in range(3)], U, H)
        Ue.append([to_host(u) for u in U])
        falls.append(b.mixed_fallbacks())
    st, info = b.status()
    assert st == 0, info
    assert falls == [0, 1, 1], falls
    He = [to_host(h) for h in H]
    for i in range(3):
        g = Orthogonalizer(ns[i], ss[i], ks[i], lrs[i], precision=MIX)
        s = ss[i]
        for j in range(3):
            Hs, Rs, Us = g.step(Wd[i][j])
            k = j * s
            assert np.array_equal(Ue[j][i], to_host(Us)), (i, j)
            assert np.array_equal(He[i][k:k + s, j * s:(j + 1) * s], to_host(Rs)), (i, j)
            if k:
                assert np.array_equal(He[i][:k, j * s:(j + 1) * s], to_host(Hs)), (i, j)
        assert orth.orth_mixed_fallbacks(g.h)[1] == (1 if i == 1 else 0)
        g.close()
    ws = b.workspace
    b.close()

    # the same three steps captured once and replayed on fresh batch state
    side = torch.cuda.Stream()
    nbytes = orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, MIX)
    wp = (ws.data_ptr() + 255) // 256 * 256
    Ug, Hg = buffers()
    with torch.cuda.stream(side):
        code, h = orth.orth_batch_create(ns, ss, ks, lrs, MIX, wp, nbytes, side.cuda_stream)
        assert code == 0
        parr = lambda ts: torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device="cuda")
        ptrs = [(parr([Wd[i][j] for i in range(3)]), parr(Ug), parr(Hg)) for j in range(3)]
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for j in range(3):
            assert orth.orth_batch_step(h, *(p.data_ptr() for p in ptrs[j])) == 0
    orth.orth_batch_destroy(h)
    for rep in range(3):
        code, h = orth.orth_batch_create(ns, ss, ks, lrs, MIX, wp, nbytes, side.cuda_stream)
        assert code == 0
        for t in Ug + Hg:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        code, st, info = orth.orth_batch_status(h)
        assert code == 0 and st == 0, info
        assert orth.orth_batch_mixed_fallbacks(h) == (0, 1), rep
        for i in range(3):
            assert np.array_equal(to_host(Ug[i]), Ue[2][i]), (rep, i)
            assert np.array_equal(to_host(Hg[i]), He[i]), (rep, i)
        orth.orth_batch_destroy(h)
        x = torch.randn(1000, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())


HH_INSTANCES = [  # n, s, k_max, leaf_rows (0: default): within the panel's limits
    (5000, 4, 24, 1000),
    (3001, 8, 48, 700),        # ragged last leaf
    (777, 1, 6, 100),
    (6000, 16, 96, 1000),
    (8192, 32, 192, 4096),     # s = 32: the sub-panel kernel
    (2600, 2, 12, 0),
]


def test_batch_householder_equals_single_handles_bitwise(torch_cuda):
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, Orthogonalizer, orth
    HH = orth.ORTH_FP64_HOUSEHOLDER
    _say("batch householder vs single", len(HH_INSTANCES))
    rng = np.random.default_rng(11)
    steps = min(k // s for _, s, k, _ in HH_INSTANCES)
    X = [[rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s) for _ in range(steps)]
         for (n, s, _, _) in HH_INSTANCES]
    ns = [i[0] for i in HH_INSTANCES]
    ss = [i[1] for i in HH_INSTANCES]
    ks = [i[2] for i in HH_INSTANCES]
    lrs = [i[3] for i in HH_INSTANCES]
    b = BatchOrthogonalizer(ns, ss, ks, lrs, precision=HH)
    assert orth.orth_batch_set_variant(b.h, orth.ORTH_PIP) == orth.ORTH_ERR_UNSUPPORTED
    W = [torch.empty((s, n), dtype=torch.float64, device="cuda") for (n, s, _, _) in HH_INSTANCES]
    U = [torch.empty_like(w) for w in W]
    Hess = [torch.zeros((k, k), dtype=torch.float64, device="cuda") for k in ks]
    Ub = [[] for _ in HH_INSTANCES]
    for j in range(steps):
        for i, w in enumerate(W):
            w.copy_(to_dev(X[i][j]))
        b.step(W, U, Hess)
        for i, u in enumerate(U):
            Ub[i].append(to_host(u))
    st, info = b.status()
    assert st == 0, info
    for i, (n, s, km, lr) in enumerate(HH_INSTANCES):
        g = Orthogonalizer(n, s, km, lr, precision=HH)
        assert g.leaf_rows == b.leaf_rows[i]
        Hb = to_host(Hess[i])
        Q = np.zeros((n, 0))
        for j in range(steps):
            H, R, Uo = g.step(to_dev(X[i][j]))
            k = j * s
            assert np.array_equal(Hb[:k, j * s:(j + 1) * s], to_host(H)), (i, j)
            assert np.array_equal(Hb[k:k + s, j * s:(j + 1) * s], to_host(R)), (i, j)
            assert np.array_equal(Ub[i][j], to_host(Uo)), (i, j)
            P, N, Ur = pqr_reference(Q, X[i][j])
            kap = kappa_after_projection(N, X[i][j])
            xn = np.linalg.norm(X[i][j])
            if k:
                assert np.linalg.norm(Hb[:k, j * s:(j + 1) * s] - P) / xn <= 1e-12
            assert np.linalg.norm(Hb[k:k + s, j * s:(j + 1) * s] - N) / xn <= 1e-12 * kap
            assert np.max(np.abs(Ub[i][j] - Ur)) <= 1e-12 * kap
            Q = np.hstack([Q, Ur])
        g.close()
    b.close()
