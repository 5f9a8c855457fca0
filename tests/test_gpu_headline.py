"""Parity and properties at the headline size: the block-Arnoldi workload the
bench times (2D Dirichlet Laplacian on a 4096 x 4096 grid, n = 2^24, s = 8,
leaf height 4096, k_max = 248), in the bench's launch configuration.

* open loop, three seeded N(0,1) blocks: every output of every step (H, R
  and U, all 2^24 rows) against the oracle's reference PQR solution computed
  on the host at full size; the FP64 form at the parity tolerances of
  test_gpu_parity.py, the mixed form at 1e-10, the Householder leaves at the
  FP64 ones;
* closed loop, the bench's 31 calls (start block and 30 Arnoldi steps):
  properties that hold at any size, checked with torch's own GEMM and a
  torch stencil (itself checked against the oracle's operator): e_perp of
  the 248 columns <= 1e-12, every R upper triangular with a positive
  diagonal, and the block Arnoldi relation A V_240 = V_248 H~ to 1e-12
  relative (||A||_2 <= 8);
* the batched workload (512 instances) and the large-block workload (3D
  Laplacian, s = 32) the bench times, at full size: statuses, R, and for
  the large block and twelve sampled instances the same properties (the
  sampled instances' first call also against the oracle).
"""

import sys

import numpy as np
import pytest

from oracle import operators as ops
from oracle import pqr_reference
from synth import normal_block

from gpu_util import kappa_after_projection, to_dev, to_host

pytestmark = pytest.mark.gpu

NX = NY = 4096
N = NX * NY
S, KMAX, LEAF = 8, 248, 4096


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


@pytest.fixture(scope="module")
def open_loop_reference():
    """Three N(0,1) blocks and the oracle's (P, N, U) for each step."""
    X = [normal_block(N, S, 700 + j) for j in range(3)]
    Q = np.zeros((N, 0))
    ref = []
    for Xj in X:
        P, Nn, U = pqr_reference(Q, Xj)
        ref.append((P, Nn, U, kappa_after_projection(Nn, Xj)))
        Q = np.hstack([Q, U])
    return X, ref


@pytest.mark.parametrize("form", ["fp64", "mixed", "householder"])
def test_headline_open_loop_parity(torch_cuda, open_loop_reference, form):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("headline open loop", form)
    prec = {"fp64": orth.ORTH_FP64, "mixed": orth.ORTH_MIXED_SPLIT32,
            "householder": orth.ORTH_FP64_HOUSEHOLDER}[form]
    tol = 1e-10 if form == "mixed" else 1e-12
    X, ref = open_loop_reference
    g = Orthogonalizer(N, S, KMAX, LEAF, precision=prec)
    for j, (Xj, (P, Nn, U, kap)) in enumerate(zip(X, ref)):
        H, R, Ug = (to_host(t) for t in g.step(to_dev(Xj)))
        xn = np.linalg.norm(Xj)
        if j:
            assert np.linalg.norm(H - P) / xn <= tol, (form, j)
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)
        assert np.linalg.norm(R - Nn) / xn <= tol * kap, (form, j)
        assert np.max(np.abs(Ug - U)) <= tol * kap, (form, j)
    st, info = g.status()
    assert st == 0, info
    g.close()


def _stencil(torch, U, nx=NX, ny=NY):
    """A U for the 2D 5-point Dirichlet Laplacian (unknown i + nx j), U of
    shape (m, nx ny), plain torch ops."""
    m = U.shape[0]
    G = U.view(m, ny, nx)
    Y = 4.0 * G
    Y[:, :, 1:] -= G[:, :, :-1]
    Y[:, :, :-1] -= G[:, :, 1:]
    Y[:, 1:, :] -= G[:, :-1, :]
    Y[:, :-1, :] -= G[:, 1:, :]
    return Y.view(m, -1)


def test_torch_stencil_matches_oracle_operator(torch_cuda):
    import torch
    nx, ny = 37, 23
    X = np.random.default_rng(3).standard_normal((nx * ny, 3))
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    Y = _stencil(torch, Xt, nx, ny)
    assert np.allclose(Y.cpu().numpy().T, ops.laplacian_2d_apply(X, nx, ny), atol=1e-14)


def test_headline_closed_loop_properties(torch_cuda):
    import torch
    from paper_2204_13393_amd import Orthogonalizer
    _say("headline closed loop")
    steps = 30
    g = Orthogonalizer(N, S, KMAX, LEAF)
    V = torch.empty((KMAX, N), dtype=torch.float64, device="cuda")      # rows = basis columns
    Hbar = torch.zeros((KMAX, steps * S), dtype=torch.float64, device="cuda")
    W = to_dev(normal_block(N, S, 0))
    for j in range(steps + 1):
        k = j * S
        H, R, U = g.step(W)
        Rh = R.cpu().numpy().T
        assert np.all(np.tril(Rh, -1) == 0.0) and np.all(np.diag(Rh) > 0), j
        V[k:k + S] = U
        if j:
            # column block j-1 of H~: A U_{j-1} = V[:, :k] H + U_j R
            Hbar[:k, (j - 1) * S:j * S] = H.t()
            Hbar[k:k + S, (j - 1) * S:j * S] = R.t()
        if j < steps:
            W = _stencil(torch, U.contiguous())
    st, info = g.status()
    assert st == 0, info
    g.close()
    # e_perp of the 248 columns (torch's GEMM)
    Gm = torch.mm(V, V.t())
    Gm -= torch.eye(KMAX, dtype=torch.float64, device="cuda")
    ep = float(torch.linalg.matrix_norm(Gm, "fro"))
    del Gm
    print("  e_perp", ep, flush=True)
    assert ep <= 1e-12
    # block Arnoldi relation, one column block at a time
    num2 = 0.0
    for j in range(steps):
        k1 = (j + 2) * S
        AU = _stencil(torch, V[j * S:(j + 1) * S].contiguous())
        res = AU - torch.mm(Hbar[:k1, j * S:(j + 1) * S].t(), V[:k1])
        num2 += float(torch.sum(res * res))
    rel = np.sqrt(num2) / (8.0 * np.sqrt(steps * S))
    print("  Arnoldi relation", rel, flush=True)
    assert rel <= 1e-12


def test_batched_headline_properties(torch_cuda):
    """The batched workload the bench times (512 instances, n log-uniform in
    [2^14, 2^20] on near-square grids, s in {1, 2, 4, 8, 16}, start block and
    20 Arnoldi steps, autotuned leaf heights), at full size.  Every instance:
    status ok and every R upper triangular with a positive diagonal.  Twelve
    sampled instances (every width): the first call against the oracle's QR of
    the start block, e_perp of all 21 blocks <= 1e-12 and the block Arnoldi
    relation to 1e-12 relative (torch GEMM and torch stencil)."""
    import torch
    from bench import batched_workload
    from paper_2204_13393_amd import BatchOrthogonalizer, autotune
    _say("batched headline")
    inst = batched_workload()
    steps = 20
    ns = [nx * ny for nx, ny, _ in inst]
    ss = [s for _, _, s in inst]
    ks = [(steps + 1) * s for s in ss]
    tuned = autotune.tune_batch(ns, ss, ks)
    sample = []
    for s in (1, 2, 4, 8, 16):
        idx = [i for i in range(len(inst)) if ss[i] == s]
        sample += [idx[0], idx[-1]] if s != 16 else [idx[0], idx[len(idx) // 2], idx[-1]]
    sample = sorted(set(sample))[:12]
    gen = torch.Generator(device="cuda")
    W, U, H = [], [], []
    for i, (n, s, k) in enumerate(zip(ns, ss, ks)):
        gen.manual_seed(1000 + i)
        W.append(torch.randn((s, n), dtype=torch.float64, device="cuda", generator=gen))
        U.append(torch.empty((s, n), dtype=torch.float64, device="cuda"))
        H.append(torch.zeros((k, k), dtype=torch.float64, device="cuda"))
    R0 = {i: W[i].cpu().numpy().T.copy() for i in sample}
    V = {i: torch.empty((ks[i], ns[i]), dtype=torch.float64, device="cuda") for i in sample}
    b = BatchOrthogonalizer(ns, ss, ks, tuned)
    for j in range(steps + 1):
        if j:
            for i, (nx, ny, s) in enumerate(inst):
                W[i] = _stencil(torch, U[i], nx, ny).contiguous()
        b.step(W, U, H)
        for i in sample:
            V[i][j * ss[i]:(j + 1) * ss[i]] = U[i]
    st, info = b.status()
    assert st == 0, info
    b.close()
    for i, (n, s, k) in enumerate(zip(ns, ss, ks)):
        Hh = H[i].cpu().numpy().T                 # call j: [H; R] in column block j
        for j in range(steps + 1):
            R = Hh[j * s:(j + 1) * s, j * s:(j + 1) * s]
            assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0), (i, j)
    for i in sample:
        nx, ny, s = inst[i]
        n, k = ns[i], ks[i]
        Hh = H[i].cpu().numpy().T
        # the first call: QR of the start block, against the oracle
        P, N0, U0 = pqr_reference(None, R0[i])
        kap = kappa_after_projection(N0, R0[i])
        assert np.linalg.norm(Hh[:s, :s] - N0) / np.linalg.norm(R0[i]) <= 1e-12 * kap, i
        assert np.max(np.abs(V[i][:s].cpu().numpy().T - U0)) <= 1e-12 * kap, i
        Gm = torch.mm(V[i], V[i].t()) - torch.eye(k, dtype=torch.float64, device="cuda")
        ep = float(torch.linalg.matrix_norm(Gm, "fro"))
        assert ep <= 1e-12, (i, ep)
        # A U_j (the input of call j + 1) = V[:, :(j+2) s] times column block j + 1
        Ht = torch.from_numpy(np.ascontiguousarray(Hh)).to("cuda")
        num2 = 0.0
        for j in range(steps):
            k1 = (j + 2) * s
            AU = _stencil(torch, V[i][j * s:(j + 1) * s].contiguous(), nx, ny)
            res = AU - torch.mm(Ht[:k1, (j + 1) * s:(j + 2) * s].t().contiguous(), V[i][:k1])
            num2 += float(torch.sum(res * res))
        rel = np.sqrt(num2) / (8.0 * np.sqrt(steps * s))
        assert rel <= 1e-12, (i, rel)
    print("  sampled instances", sample, flush=True)


def _stencil3(torch, U, n1):
    """A U for the 3D 7-point Dirichlet Laplacian on n1^3 (unknown i + n1 j + n1^2 l)."""
    m = U.shape[0]
    G = U.view(m, n1, n1, n1)
    Y = 6.0 * G
    for d in (1, 2, 3):
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[d], hi[d] = slice(1, None), slice(None, -1)
        Y[tuple(lo)] -= G[tuple(hi)]
        Y[tuple(hi)] -= G[tuple(lo)]
    return Y.view(m, -1)


def test_torch_stencil3_matches_oracle_operator(torch_cuda):
    import torch
    n1 = 9
    X = np.random.default_rng(4).standard_normal((n1 ** 3, 2))
    Y = _stencil3(torch, torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda"), n1)
    assert np.allclose(Y.cpu().numpy().T, ops.laplacian_3d_apply(X, n1, n1, n1), atol=1e-14)


def test_large_block_headline_properties(torch_cuda):
    """The large-block workload the bench times (3D Laplacian on 256^3,
    n = 2^24, s = 32, start block N(0,1) seed 5 and 16 Arnoldi steps, leaf
    height 4096, k_max = 544), at full size: R upper triangular with a
    positive diagonal, e_perp of the 544 columns <= 1e-12 and the block
    Arnoldi relation to 1e-12 relative (||A||_2 <= 12)."""
    import torch
    from paper_2204_13393_amd import Orthogonalizer
    _say("large block headline")
    n1, s, steps, kmax = 256, 32, 16, 544
    n = n1 ** 3
    g = Orthogonalizer(n, s, kmax, 4096)
    V = torch.empty((kmax, n), dtype=torch.float64, device="cuda")
    Hbar = torch.zeros((kmax, steps * s), dtype=torch.float64, device="cuda")
    W = to_dev(normal_block(n, s, 5))
    for j in range(steps + 1):
        k = j * s
        H, R, U = g.step(W)
        Rh = R.cpu().numpy().T
        assert np.all(np.tril(Rh, -1) == 0.0) and np.all(np.diag(Rh) > 0), j
        V[k:k + s] = U
        if j:
            Hbar[:k, (j - 1) * s:j * s] = H.t()
            Hbar[k:k + s, (j - 1) * s:j * s] = R.t()
        if j < steps:
            W = _stencil3(torch, U.contiguous(), n1)
    st, info = g.status()
    assert st == 0, info
    g.close()
    Gm = torch.mm(V, V.t())
    Gm -= torch.eye(kmax, dtype=torch.float64, device="cuda")
    ep = float(torch.linalg.matrix_norm(Gm, "fro"))
    del Gm
    print("  e_perp", ep, flush=True)
    assert ep <= 1e-12
    num2 = 0.0
    for j in range(steps):
        k1 = (j + 2) * s
        AU = _stencil3(torch, V[j * s:(j + 1) * s].contiguous(), n1)
        res = AU - torch.mm(Hbar[:k1, j * s:(j + 1) * s].t(), V[:k1])
        num2 += float(torch.sum(res * res))
    rel = np.sqrt(num2) / (12.0 * np.sqrt(steps * s))
    print("  Arnoldi relation", rel, flush=True)
    assert rel <= 1e-12
