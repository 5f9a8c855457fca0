"""GPU parity of the HIP path against the CPU oracle (MI355X, gfx950).

Tolerances (FP64 form), stated per quantity; u = 2^-53, kappa_j the condition
of the projected block (||X||_2 ||N^{-1}||_2):
  H (= P) vs oracle          ||dP||_F / ||X||_F        <= 1e-12
  R (= N) vs oracle          ||dN||_F / ||X||_F        <= 1e-12 kappa_j
  U vs oracle                max |dU|                  <= 1e-12 kappa_j
  local factors vs oracle TreeTSPQR (same leaves)      <= 1e-11 kappa
  orthogonality of the explicit blocks  e_perp         <= 1e-12
The oracle (tests-only) is the unique PQR solution for the global results and
oracle.TreeTSPQR with the same leaf partition for the locally orthogonal
factors, which are unique once the partition is fixed.

Open-loop inputs are moderately conditioned (kappa_j ~ 4): two independent
FP64 bases drift apart by rounding and the drift is amplified by ~kappa_j per
step through the projection (two correct CPU solvers already differ by 1e-11
in P after 5 steps at kappa_j = 1e3).  Ill-conditioned blocks are covered by
test_ill_conditioned_blocks with properties of the GPU's own results plus
first-step parity.
"""

import sys

import numpy as np
import pytest

from oracle import TreeTSPQR, metrics, pqr_reference
from oracle import operators as ops
from synth import normal_block, stewart

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
    # n, s, kmax, leaf_rows
    (1000, 4, 24, 1000),      # one leaf
    (10000, 4, 44, 1000),     # the small Arnoldi workload's shape, 10 leaves
    (1037, 2, 16, 128),       # ragged last leaf (141 rows)
    (3000, 8, 64, 700),       # ragged, s = 8
    (4096, 16, 96, 1024),     # s = 16
    (777, 1, 12, 100),        # s = 1 (CGS2 on vectors), ragged
    (5000, 8, 248, 2500),     # widest basis of the headline shape (k + s = 256)
    (6000, 32, 160, 2000),    # s = 32, two N tiles in the Gram products
    (5000, 16, 256, 2500),    # k + s = 272: two column groups in the Gram kernel
    (9000, 8, 504, 4500),     # k + s = 512, coefficient blocks of 64 columns
    (20000, 4, 32, 16384),    # one leaf of 10 chunks: its 40 Gram slots are pre-summed
    (4100, 32, 96, 1366),     # LDS-staged row update: even leaves, last one ragged (1368 rows)
    (5001, 16, 64, 1001),     # odd leaf height: row pairs unaligned, the register-streamed row update
    (9000, 16, 80, 4500),     # LDS-staged row update over 3 chunks per leaf (2048, 2048, 404 rows)
    (4097, 16, 64, 4097),     # one leaf of odd height: LDS-staged, its last row pair half past the end
]

# the widest basis the planner accepts (k_max + s = 2048), s = 32, one leaf,
# and two leaves with the reduction level at its widest
WIDE_CASES = [(2100, 32, 2016, 2100), (4200, 32, 2016, 2100)]


@pytest.mark.parametrize("n,s,kmax,leaf_rows", CASES)
def test_open_loop_parity(torch_cuda, n, s, kmax, leaf_rows):
    from paper_2204_13393_amd import Orthogonalizer
    _say("open-loop", n, s, kmax, leaf_rows)
    rng = np.random.default_rng(n * 31 + s)
    gpu = Orthogonalizer(n, s, kmax, leaf_rows)
    tree = TreeTSPQR(n, s, leaf_rows, "pip+", "pip+")
    Q = np.zeros((n, 0))
    Ugpu = []
    kap_max = 1.0
    for step in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s)
        if step:
            X = X + Q @ rng.standard_normal((Q.shape[1], s))
        Hd, Rd, Ud = gpu.step(to_dev(X))
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        P, N, Ur = pqr_reference(Q, X)
        Pt, Nt, Ut = tree.step(X)
        kap = kappa_after_projection(N, X)
        kap_max = max(kap_max, kap)
        xn = np.linalg.norm(X)
        assert H.shape == P.shape and R.shape == (s, s)
        if step:
            assert np.linalg.norm(H - P) / xn <= 1e-12, step
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)
        assert np.linalg.norm(R - N) / xn <= 1e-12 * kap, step
        assert np.max(np.abs(U - Ur)) <= 1e-12 * kap, step
        assert np.max(np.abs(U - Ut)) <= 1e-12 * kap, step
        Ugpu.append(U)
        Q = np.hstack([Q, Ur])
    st, info = gpu.status()
    assert st == 0, info
    V = np.hstack(Ugpu)
    assert metrics.e_perp(V) <= 1e-12
    # locally orthogonal factors against the oracle tree with the same leaves
    Qloc, T = gpu.export_local()
    Qloc, T = to_host(Qloc), to_host(T)
    assert np.max(np.abs(Qloc - np.vstack(tree.leaves))) <= 1e-11 * kap_max
    assert np.max(np.abs(T - tree.stacked_factor(0))) <= 1e-11 * kap_max
    for (r0, r1) in tree.bounds:
        assert metrics.e_perp(Qloc[r0:r1]) <= 1e-12
    assert metrics.e_perp(T) <= 1e-12
    # Y = Q C through the representation
    C = rng.standard_normal((gpu.k, 21))
    Y = to_host(gpu.apply_Q(to_dev(C)))
    assert np.max(np.abs(Y - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    gpu.close()


@pytest.mark.parametrize("n,s,kmax,leaf_rows", WIDE_CASES)
def test_widest_basis(torch_cuda, n, s, kmax, leaf_rows):
    """k_max + s = 2048: parity of every step against the oracle, e_perp of the
    explicit basis, and Y = Q C through the representation."""
    from paper_2204_13393_amd import Orthogonalizer
    _say("widest", n, s, kmax, leaf_rows)
    rng = np.random.default_rng(n + s)
    gpu = Orthogonalizer(n, s, kmax, leaf_rows)
    Q = np.zeros((n, 0))
    Ugpu = []
    for step in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 0.25, s)
        Hd, Rd, Ud = gpu.step(to_dev(X))
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        P, N, Ur = pqr_reference(Q, X)
        kap = kappa_after_projection(N, X)
        xn = np.linalg.norm(X)
        if step:
            assert np.linalg.norm(H - P) / xn <= 1e-12, step
        assert np.linalg.norm(R - N) / xn <= 1e-12 * kap, step
        assert np.max(np.abs(U - Ur)) <= 1e-12 * kap, step
        Ugpu.append(U)
        Q = np.hstack([Q, Ur])
    st, info = gpu.status()
    assert st == 0, info
    V = np.hstack(Ugpu)
    assert metrics.e_perp(V) <= 1e-12
    C = rng.standard_normal((gpu.k, 5))
    Y = to_host(gpu.apply_Q(to_dev(C)))
    assert np.max(np.abs(Y - V @ C)) <= 1e-12 * np.abs(C).sum(0).max()
    gpu.close()


@pytest.mark.parametrize("n,s,kmax,leaf_rows", [(4000, 4, 40, 800), (3000, 8, 64, 700)])
def test_ill_conditioned_blocks(torch_cuda, n, s, kmax, leaf_rows):
    """kappa_j ~ 1e3 per block: parity on the first two steps, then the GPU's own
    residual ||X - Q H - U R|| / ||X|| <= 1e-13 and e_perp <= 1e-12 at every step."""
    from paper_2204_13393_amd import Orthogonalizer
    _say("ill-conditioned", n, s, kmax, leaf_rows)
    rng = np.random.default_rng(n + 5 * s)
    gpu = Orthogonalizer(n, s, kmax, leaf_rows)
    Qo = np.zeros((n, 0))
    Vg = np.zeros((n, 0))
    for step in range(kmax // s):
        X = rng.standard_normal((n, s)) * np.geomspace(1.0, 1e-3, s)
        if step:
            X = X + Qo @ rng.standard_normal((Qo.shape[1], s))
        Hd, Rd, Ud = gpu.step(to_dev(X))
        H, R, U = to_host(Hd), to_host(Rd), to_host(Ud)
        P, N, Ur = pqr_reference(Qo, X)
        kap = kappa_after_projection(N, X)
        assert kap > 100.0
        if step <= 1:
            xn = np.linalg.norm(X)
            if step:
                assert np.linalg.norm(H - P) / xn <= 1e-12
            assert np.linalg.norm(R - N) / xn <= 1e-12 * kap
            assert np.max(np.abs(U - Ur)) <= 1e-12 * kap
        assert metrics.pqr_residual(Vg, X, H, R, U) <= 1e-13
        Vg = np.hstack([Vg, U])
        assert metrics.e_perp(Vg) <= 1e-12
        Qo = np.hstack([Qo, Ur])
    st, _ = gpu.status()
    assert st == 0
    gpu.close()


def test_c1_arnoldi_closed_loop(torch_cuda):
    """Small workload: 2D 100x100 Laplacian + 0.01 I, s = 4, 10 steps, 10 leaves."""
    import torch
    from paper_2204_13393_amd import Orthogonalizer, laplacian_apply
    _say("arnoldi lap2d-100x100-s4")
    nx, ny, shift, s, steps, leaf = 100, 100, 0.01, 4, 10, 1000
    n = nx * ny
    R0 = normal_block(n, s, 0)
    apply_A = lambda X: ops.laplacian_2d_apply(X, nx, ny, shift)
    # oracle
    from oracle import block_arnoldi
    Vo, Ho, H0o, _ = block_arnoldi(apply_A, R0, steps)
    # GPU, closed loop with the library's stencil
    gpu = Orthogonalizer(n, s, (steps + 1) * s, leaf)
    K = (steps + 1) * s
    Hd = torch.zeros((steps * s, K), dtype=torch.float64, device="cuda")   # column-major K x steps*s
    _, H0d, V = gpu.step(to_dev(R0))
    blocks = [V]
    for j in range(steps):
        X = laplacian_apply(blocks[-1], (nx, ny), shift)
        k = gpu.k
        col = Hd[j * s:(j + 1) * s]
        Hj, Rj, U = gpu.step(X)
        col[:, :k] = Hj
        col[:, k:k + s] = Rj
        blocks.append(U)
    torch.cuda.synchronize()
    st, info = gpu.status()
    assert st == 0, info
    H = to_host(Hd)
    Vg = np.hstack([to_host(b) for b in blocks])
    assert np.allclose(to_host(H0d), H0o, rtol=0, atol=1e-12 * np.abs(H0o).max())
    assert np.max(np.abs(H - Ho)) <= 1e-10
    assert metrics.e_perp(Vg) <= 1e-12
    lo, hi = ops.laplacian_extreme_eigs((nx, ny), shift)
    assert metrics.arnoldi_relation(apply_A, Vg, H, hi) <= 1e-13
    ritz = np.linalg.eigvalsh(H[:steps * s, :steps * s])
    assert lo - 1e-10 <= ritz[0] and ritz[-1] <= hi + 1e-10
    gpu.close()


@pytest.mark.parametrize("leaves,variant", [(256, "pip+"), (8, "pip+"), (256, "pip"), (1024, "pip+")])
def test_paper_stability_workload(torch_cuda, leaves, variant):
    """Sec. 6.1 table workload on the GPU: Stewart kappa = 1e4, n = 2^16, 32 columns, s = 4."""
    import json
    import os
    import torch
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("stewart-1e4", leaves, variant)
    n, m, s = 2 ** 16, 32, 4
    A = stewart(n, m, 1e4, 0)
    gpu = Orthogonalizer(n, s, m, n // leaves,
                         variant=orth.ORTH_PIP if variant == "pip" else orth.ORTH_PIP_PLUS)
    R = np.zeros((m, m))
    for j in range(m // s):
        Hd, Rd, Ud = gpu.step(to_dev(A[:, j * s:(j + 1) * s]))
        R[:j * s, j * s:(j + 1) * s] = to_host(Hd)
        R[j * s:(j + 1) * s, j * s:(j + 1) * s] = to_host(Rd)
    st, _ = gpu.status()
    assert st == 0
    Q = to_host(gpu.apply_Q(torch.eye(m, dtype=torch.float64, device="cuda")))
    e = metrics.e_perp(Q)
    res = np.linalg.norm(A - Q @ R, "fro")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_stability_tables.json")))
    col = 1 if variant == "pip+" else 0
    vals = [row[col] for row in gold["subproblems"].values()]
    assert min(vals) / 10 <= e <= max(vals) * 10, e
    rvals = [row[col + 3] for row in gold["subproblems"].values()]
    assert min(rvals) / 10 <= res <= max(rvals) * 10, res
    # the oracle tree on the same partition lands in the same band
    tree = TreeTSPQR(n, s, n // leaves, variant, variant)
    from oracle.krylov import block_column_qr
    Qo, Ro = block_column_qr(A, s, tree)
    eo = metrics.e_perp(tree.explicit_Q())
    assert 0.1 <= e / eo <= 10.0
    if variant == "pip+":
        assert np.max(np.abs(R - Ro)) <= 1e-11
    gpu.close()


def test_breakdown_poisons_handle(torch_cuda):
    """A zero column makes the pivot exactly 0: breakdown is certain (no threshold)."""
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("breakdown")
    n, s = 2000, 4
    gpu = Orthogonalizer(n, s, 16, 500)
    X = normal_block(n, s, 3)
    gpu.step(to_dev(X))
    st, _ = gpu.status()
    assert st == 0
    Y = normal_block(n, s, 4)
    Y[:, 3] = 0.0
    gpu.step(to_dev(Y))
    st, info = gpu.status()
    assert st == orth.ORTH_ERR_BREAKDOWN
    assert info[0] == 0 and info[2] == 1 and info[3] == 3, info
    code = orth.orth_step(gpu.h, 0, n, 0, 4, 0, s, 0, n)
    assert code == orth.ORTH_ERR_POISONED
    assert orth.orth_apply_Q(gpu.h, 0, 8, 1, 0, n) == orth.ORTH_ERR_POISONED
    assert orth.orth_destroy(gpu.h) == orth.ORTH_OK
    gpu.h = None


@pytest.mark.parametrize("s,col", [(16, 11), (32, 19), (32, 0)])
def test_breakdown_wide_blocks(torch_cuda, s, col):
    """Zero column at s = 16, 32 (the wide Cholesky): the pivot of that column is 0."""
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("breakdown wide", s, col)
    n = 4096
    gpu = Orthogonalizer(n, s, 4 * s, 1024)
    gpu.step(to_dev(normal_block(n, s, 5)))
    assert gpu.status()[0] == 0
    Y = normal_block(n, s, 6)
    Y[:, col] = 0.0
    gpu.step(to_dev(Y))
    st, info = gpu.status()
    assert st == orth.ORTH_ERR_BREAKDOWN
    assert info[0] == 0 and info[2] == 1 and info[3] == col, info
    gpu.close()


def test_nan_input_breaks_down_wide(torch_cuda):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("nan breakdown wide")
    n, s = 3000, 32
    gpu = Orthogonalizer(n, s, 64, 1000)
    W = normal_block(n, s, 2)
    W[1700, 5] = np.nan
    gpu.step(to_dev(W))
    st, info = gpu.status()
    assert st == orth.ORTH_ERR_BREAKDOWN, (st, info)
    gpu.close()


def test_nan_input_breaks_down(torch_cuda):
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("nan breakdown")
    n, s = 1500, 2
    gpu = Orthogonalizer(n, s, 8, 500)
    W = normal_block(n, s, 1)
    W[700, 1] = np.nan
    gpu.step(to_dev(W))
    st, info = gpu.status()
    assert st == orth.ORTH_ERR_BREAKDOWN
    gpu.close()


def test_capacity_and_argument_errors(torch_cuda):
    import torch
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("capacity/args")
    n, s = 800, 4
    gpu = Orthogonalizer(n, s, 8, 400)
    W = to_dev(normal_block(n, s, 0))
    H = torch.zeros((s, 8), dtype=torch.float64, device="cuda")
    R = torch.zeros((s, s), dtype=torch.float64, device="cuda")
    U = torch.zeros((s, n), dtype=torch.float64, device="cuda")
    assert orth.orth_step(gpu.h, W.data_ptr(), n - 1, H.data_ptr(), 8, R.data_ptr(), s, U.data_ptr(), n) == orth.ORTH_ERR_ARG
    assert orth.orth_step(gpu.h, W.data_ptr(), n, H.data_ptr(), 8, R.data_ptr(), s - 1, U.data_ptr(), n) == orth.ORTH_ERR_ARG
    assert orth.orth_apply_Q(gpu.h, H.data_ptr(), 8, 1, U.data_ptr(), n) == orth.ORTH_ERR_ARG  # k = 0
    W2 = to_dev(normal_block(n, s, 1))     # a fresh block: the first one is in span(Q) now
    assert orth.orth_step(gpu.h, W.data_ptr(), n, 0, 1, R.data_ptr(), s, U.data_ptr(), n) == 0
    assert orth.orth_step(gpu.h, W2.data_ptr(), n, 0, 1, R.data_ptr(), s, U.data_ptr(), n) == orth.ORTH_ERR_ARG  # H needed
    assert orth.orth_step(gpu.h, W2.data_ptr(), n, H.data_ptr(), 4, R.data_ptr(), s, U.data_ptr(), n) == 0
    assert gpu.k == 8
    assert orth.orth_step(gpu.h, W.data_ptr(), n, H.data_ptr(), 8, R.data_ptr(), s, U.data_ptr(), n) == orth.ORTH_ERR_CAPACITY
    assert gpu.k == 8
    st, _ = gpu.status()
    assert st == 0
    gpu.close()


@pytest.mark.parametrize("form", [0, 1, 2])
def test_w_may_alias_u(torch_cuda, form):
    """W and U may be the same buffer, in every storage form."""
    from paper_2204_13393_amd import Orthogonalizer
    _say("alias", form)
    n, s = 3000, 4
    a = Orthogonalizer(n, s, 12, 1000, precision=form)
    b = Orthogonalizer(n, s, 12, 1000, precision=form)
    for j in range(3):
        X = normal_block(n, s, 10 + j)
        _, Ra, Ua = a.step(to_dev(X))
        buf = to_dev(X)
        _, Rb, Ub = b.step(buf, U=buf)
        assert np.array_equal(to_host(Ua), to_host(buf))
        assert np.array_equal(to_host(Ra), to_host(Rb))
    a.close()
    b.close()


def test_determinism_bitwise(torch_cuda):
    from paper_2204_13393_amd import Orthogonalizer
    _say("determinism")
    n, s, kmax = 20000, 8, 64
    outs = []
    for rep in range(2):
        g = Orthogonalizer(n, s, kmax, 2048)
        rng = np.random.default_rng(77)
        res = []
        for j in range(kmax // s):
            H, R, U = g.step(to_dev(rng.standard_normal((n, s))))
            res += [to_host(H), to_host(R), to_host(U)]
        outs.append(res)
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("grid,shift", [((100, 100), 0.01), ((37, 53), 0.0), ((16, 12, 9), 0.0)])
def test_laplacian_operator_parity(torch_cuda, grid, shift):
    from paper_2204_13393_amd import laplacian_apply
    _say("laplacian", grid)
    n = int(np.prod(grid))
    X = normal_block(n, 3, 5)
    Y = to_host(laplacian_apply(to_dev(X), grid, shift))
    if len(grid) == 2:
        Yo = ops.laplacian_2d_apply(X, grid[0], grid[1], shift)
    else:
        Yo = ops.laplacian_3d_apply(X, grid[0], grid[1], grid[2], shift)
    assert np.max(np.abs(Y - Yo)) <= 1e-14 * np.abs(X).max()


def test_probe_copy(torch_cuda):
    import torch
    from paper_2204_13393_amd import orth
    _say("probe copy")
    src = torch.randn(1001, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    assert orth.orth_probe_copy(src.data_ptr(), dst.data_ptr(), 1001, torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("n,s,kmax,leaf", [
    (6000, 4, 24, 1000),
    # s >= 16: the one-sweep finalize skips the products of its zero
    # coefficient tiles
    (6000, 16, 64, 1000),
    (8192, 32, 128, 2048),
])
def test_pip_variant_matches_oracle_tree(torch_cuda, n, s, kmax, leaf):
    """BCGS-PIP leaves and reduction (one CholQR sweep) on a well-conditioned input."""
    from paper_2204_13393_amd import Orthogonalizer, orth
    _say("pip variant", n, s, kmax, leaf)
    gpu = Orthogonalizer(n, s, kmax, leaf, variant=orth.ORTH_PIP)
    tree = TreeTSPQR(n, s, leaf, "pip", "pip")
    rng = np.random.default_rng(8)
    for j in range(kmax // s):
        X = rng.standard_normal((n, s))
        H, R, U = gpu.step(to_dev(X))
        P, N, Ut = tree.step(X)
        assert np.max(np.abs(to_host(R) - N)) <= 1e-11
        assert np.max(np.abs(to_host(U) - Ut)) <= 1e-11
        if j:
            assert np.max(np.abs(to_host(H) - P)) <= 1e-11
    gpu.close()


def test_graph_replay_wide_blocks(torch_cuda):
    """Three s = 32 steps (LDS-staged row updates, wide Cholesky) captured in a
    hipGraph and replayed from freshly created handles on the same workspace,
    eager work and synchronisation between replays: every replay equals the
    eager run bitwise."""
    import torch
    from paper_2204_13393_amd import orth
    _say("graph wide")
    n, s, kmax, leaf = 4096, 32, 96, 1024
    X = [to_dev(normal_block(n, s, 60 + j)) for j in range(3)]
    nbytes = orth.orth_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64)
    side = torch.cuda.Stream()

    def buffers():
        H = torch.zeros((kmax, kmax), dtype=torch.float64, device="cuda")
        U = torch.empty((kmax, n), dtype=torch.float64, device="cuda")
        return H, U

    def run(h, H, U):
        for j in range(3):
            k = j * s
            col = H[j * s:(j + 1) * s]
            hp = col.data_ptr() if k else 0
            assert orth.orth_step(h, X[j].data_ptr(), n, hp, kmax, col[:, k:].data_ptr(), kmax,
                                  U[k:k + s].data_ptr(), n) == 0

    ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    He, Ue = buffers()
    with torch.cuda.stream(side):
        code, h = orth.orth_create(n, s, kmax, leaf, orth.ORTH_FP64, wp, nbytes, side.cuda_stream)
        assert code == 0
        run(h, He, Ue)
    side.synchronize()
    assert orth.orth_status(h)[1] == 0
    orth.orth_destroy(h)
    He_h, Ue_h = to_host(He), to_host(Ue)

    Hg, Ug = buffers()
    with torch.cuda.stream(side):
        code, h = orth.orth_create(n, s, kmax, leaf, orth.ORTH_FP64, wp, nbytes, side.cuda_stream)
        assert code == 0
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        run(h, Hg, Ug)
    orth.orth_destroy(h)
    for rep in range(3):
        code, h = orth.orth_create(n, s, kmax, leaf, orth.ORTH_FP64, wp, nbytes, side.cuda_stream)
        assert code == 0
        Hg.zero_()
        Ug.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        code, st, info = orth.orth_status(h)
        assert code == 0 and st == 0, info
        assert np.array_equal(to_host(Hg), He_h), rep
        assert np.array_equal(to_host(Ug), Ue_h), rep
        orth.orth_destroy(h)
        x = torch.randn(1000, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())
