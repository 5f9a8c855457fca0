"""Host-side checks of the C ABI (CPU): the library loads, exports every symbol
that include/orth.h and include/orth_measure.h declare, sizes workspaces by
pure arithmetic, and rejects bad arguments before touching the GPU."""

import os
import re

import pytest

from paper_2204_13393_amd import orth

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
HEADERS = [os.path.join(INCLUDE, "orth.h"), os.path.join(INCLUDE, "orth_measure.h")]


def _declared(headers=HEADERS):
    names = set()
    for path in headers:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names.update(re.findall(r"\b(orth_[a-zA-Z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = orth.load()
    names = _declared()
    assert "orth_step" in names and "orth_create" in names and "orth_apply_Q" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared set
    assert sorted(n for n, _, _ in orth.SIGNATURES) == names
    # the measurement helpers stay out of the method's header
    product = _declared(HEADERS[:1])
    for helper in ("orth_laplacian_apply", "orth_probe_copy", "orth_profile_read"):
        assert helper in names and helper not in product


def test_workspace_bytes_arithmetic():
    b = orth.orth_workspace_bytes(10000, 4, 44, 1000, 0)
    assert b > 0 and b % 256 == 0
    # the basis storage alone is n*kmax doubles; the total must cover it
    assert b >= 10000 * 44 * 8
    big = orth.orth_workspace_bytes(2 ** 24, 8, 248, 4096, 0)
    assert 2 ** 24 * 248 * 8 < big < 2 ** 24 * 248 * 8 * 1.25
    # default leaf height equals an explicit 4096
    assert orth.orth_workspace_bytes(2 ** 24, 8, 248, 0, 0) == big


@pytest.mark.parametrize("args", [
    (0, 4, 44, 0, 0),        # n < 1
    (1000, 3, 12, 0, 0),     # s not in {1,2,4,8,16,32}
    (1000, 4, 2, 0, 0),      # k_max < s
    (1000, 4, 10, 0, 0),     # k_max not a multiple of s
    (1000, 4, 40, 20, 0),    # leaf_rows < k_max
    (1000, 4, 40, 2000, 0),  # leaf_rows > n
    (1000, 4, 40, 0, 3),     # unknown storage form
    (100000, 16, 2048, 0, 0),  # wider than the planner accepts (k_max + s > 2048)
])
def test_workspace_rejects_bad_arguments(args):
    assert orth.orth_workspace_bytes(*args) == 0


def _basis_ld(rows):
    """Leading dimension of a stored basis: rows rounded up to an odd
    multiple of 32 doubles (256 bytes)."""
    ld = -(-rows // 32) * 32
    return ld + 32 if (ld // 32) % 2 == 0 else ld


def test_householder_form_workspace_and_limits():
    H = orth.ORTH_FP64_HOUSEHOLDER
    # adds three k_max x k_max blocks per leaf (T in both orders, the
    # reflectors' top rows), a second apply_Q coefficient scratch and the
    # deflation state (64 bytes and an s x s matrix); its reflectors are one
    # column-major matrix where the other forms store each leaf's block
    # on its own
    for (n, s, k, lr) in ((10000, 4, 44, 1000), (2 ** 24, 8, 248, 4096), (777, 1, 12, 100)):
        f64 = orth.orth_workspace_bytes(n, s, k, lr, 0)
        hh = orth.orth_workspace_bytes(n, s, k, lr, H)
        p = max(1, n // lr)
        last = n - (p - 1) * lr
        qdiff = (_basis_ld(n) - (p - 1) * _basis_ld(lr) - _basis_ld(last)) * k * 8
        extra = 3 * p * k * k * 8 + (p * k + 64) * 16 * 8 + 64 + s * s * 8 + 256
        assert 3 * p * k * k * 8 - 512 <= hh - f64 - qdiff <= extra + 512
    # limits: the panel kernel's register capacity (s = 32 in 8-column
    # sub-panels, 4096 rows) and the small products' LDS staging, at most
    # 160 KB: ((k_max) s + s^2) doubles for the T update
    assert orth.orth_workspace_bytes(2 ** 20, 8, 64, 4096, H) > 0
    assert orth.orth_workspace_bytes(2 ** 20, 8, 64, 8192, H) == 0        # leaf rows > 4096 at s = 8
    assert orth.orth_workspace_bytes(4096 + 4095, 8, 64, 4096, H) == 0    # the last leaf takes 8191 rows
    assert orth.orth_workspace_bytes(2 ** 20, 4, 64, 8192, H) > 0
    assert orth.orth_workspace_bytes(2 ** 20, 16, 64, 1024, H) > 0
    assert orth.orth_workspace_bytes(2 ** 20, 16, 64, 2048, H) == 0
    assert orth.orth_workspace_bytes(2 ** 20, 32, 64, 512, H) > 0
    assert orth.orth_workspace_bytes(2 ** 20, 32, 64, 8192, H) == 0       # leaf rows > 4096 at s = 32
    assert orth.orth_workspace_bytes(2 ** 24, 32, 544, 4096, H) > 0       # the 3D large-block shape
    assert orth.orth_workspace_bytes(2 ** 20, 32, 608, 4096, H) > 0       # (608 * 32 + 1024) * 8 <= 160 KB
    assert orth.orth_workspace_bytes(2 ** 20, 32, 640, 4096, H) == 0      # (640 * 32 + 1024) * 8 > 160 KB
    assert orth.orth_workspace_bytes(2 ** 20, 8, 1024, 4096, H) > 0       # past the former k_max s <= 4096
    code, h = orth.orth_create(2 ** 20, 8, 64, 8192, H, 4096, 1 << 40, 0)
    assert code == orth.ORTH_ERR_UNSUPPORTED


def test_mixed_form_workspace_adds_the_fp32_copy():
    # the FP32 copy of the leaf bases: 4 bytes per stored entry on top (each
    # leaf's block padded to its own leading dimension)
    for (n, s, k, lr) in ((10000, 4, 44, 1000), (2 ** 24, 8, 248, 4096), (777, 1, 12, 100)):
        f64 = orth.orth_workspace_bytes(n, s, k, lr, 0)
        mixed = orth.orth_workspace_bytes(n, s, k, lr, orth.ORTH_MIXED_SPLIT32)
        assert f64 > 0 and mixed % 256 == 0
        p = max(1, n // lr)
        stored = ((p - 1) * _basis_ld(lr) + _basis_ld(n - (p - 1) * lr)) * k
        assert stored * 4 <= mixed - f64 <= stored * 4 + 256


def test_householder_batch_workspace_and_limits():
    # a Householder batch adds each instance's compact-WY factors (three
    # k_max x k_max blocks per leaf) and its apply scratch; an instance past
    # the panel's limits (s = 16, 2048-row leaves) makes the batch invalid
    f = orth.ORTH_FP64_HOUSEHOLDER
    ns, ss, ks, lrs = [5000, 3000], [4, 8], [16, 32], [1000, 1000]
    f64 = orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, orth.ORTH_FP64)
    hh = orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, f)
    factors = sum(3 * (n // lr) * k * k * 8 for n, k, lr in zip(ns, ks, lrs))
    assert f64 > 0 and hh >= f64 + factors
    assert orth.orth_batch_workspace_bytes([8192, 3000], [16, 8], [32, 32], [2048, 1000], f) == 0
    code, h = orth.orth_batch_create([8192, 3000], [16, 8], [32, 32], [2048, 1000], f, 4096, 1 << 30, None)
    assert code == orth.ORTH_ERR_UNSUPPORTED
    code, h = orth.orth_batch_create([5000, 3000], [4, 8], [16, 32], None, 7, 4096, 1 << 30, None)
    assert code == orth.ORTH_ERR_ARG


def test_mixed_batch_workspace():
    # the mixed batch adds each instance's FP32 copy of its leaf bases (a
    # single column-major n x k_max matrix per instance, padded ld)
    ns, ss, ks, lrs = [5000, 3000, 777], [4, 8, 1], [16, 32, 12], [1000, 0, 100]
    f64 = orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, orth.ORTH_FP64)
    mixed = orth.orth_batch_workspace_bytes(ns, ss, ks, lrs, orth.ORTH_MIXED_SPLIT32)
    assert f64 > 0 and mixed % 8 == 0
    copy = sum(n * k * 4 for n, k in zip(ns, ks))
    assert copy <= mixed - f64 <= copy + sum(ks) * 256 * 4 + 3 * 512


def test_wide_blocks_are_planned():
    # s = 32 and bases wider than 256 columns (the 3D large-block workload)
    assert orth.orth_workspace_bytes(2 ** 24, 32, 544, 4096, 0) > 2 ** 24 * 544 * 8
    assert orth.orth_workspace_bytes(4096, 32, 128, 0, 0) > 0


def test_create_validates_before_any_device_call():
    code, h = orth.orth_create(0, 4, 44, 0, 0, 0, 0, 0)
    assert code == orth.ORTH_ERR_ARG and not h.value
    code, h = orth.orth_create(10000, 4, 44, 1000, 0, 0, 0, 0)
    assert code == orth.ORTH_ERR_WORKSPACE
    code, h = orth.orth_create(10000, 4, 44, 1000, 0, 256 * 3 + 8, 1 << 30, 0)
    assert code == orth.ORTH_ERR_WORKSPACE          # misaligned
    need = orth.orth_workspace_bytes(10000, 4, 44, 1000, 0)
    code, h = orth.orth_create(10000, 4, 44, 1000, 0, 4096, need - 8, 0)
    assert code == orth.ORTH_ERR_WORKSPACE          # too small
    code, h = orth.orth_create(100000, 16, 2048, 0, 0, 4096, 1 << 40, 0)
    assert code == orth.ORTH_ERR_UNSUPPORTED


def test_null_handle_calls():
    assert orth.orth_step(None, 0, 1, 0, 1, 0, 1, 0, 1) == orth.ORTH_ERR_ARG
    assert orth.orth_apply_Q(None, 0, 1, 1, 0, 1) == orth.ORTH_ERR_ARG
    assert orth.orth_apply_Q_noalloc(None, 0, 1, 1, 0, 1) == orth.ORTH_ERR_ARG
    assert orth.orth_set_variant(None, 0) == orth.ORTH_ERR_ARG
    assert orth.orth_set_level_variants(None, 0, 1) == orth.ORTH_ERR_ARG
    assert orth.orth_mixed_fallbacks(None)[0] == orth.ORTH_ERR_ARG
    assert orth.orth_set_deflation(None, 1e-6) == orth.ORTH_ERR_ARG
    assert orth.orth_deflation_info(None)[0] == orth.ORTH_ERR_ARG
    assert orth.orth_destroy(None) == orth.ORTH_OK
    assert orth.orth_laplacian_apply(0, 1, 0, 1, 1, 1, 1, 1, 0.0, None) == orth.ORTH_ERR_ARG
    assert orth.orth_probe_copy(0, 0, 1, None) == orth.ORTH_ERR_ARG


def test_product_path_has_no_oracle_import():
    """The product package never imports the oracle (which is test-only)."""
    pkg = os.path.join(INCLUDE, "..", "paper_2204_13393_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(root, f)).read()
                assert "oracle" not in re.findall(r"^\s*(?:from|import)\s+(\w+)", src, flags=re.M), f


def test_tune_workspace_and_argument_checks():
    # the tuner's workspace holds the largest candidate plan plus W, U, H, R
    n, s, k = 20000, 4, 32
    need = orth.orth_tune_workspace_bytes(n, s, k, 1)
    assert need % 256 == 0
    heights = (256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536)
    plan_max = max(orth.orth_workspace_bytes(n, s, k, lr, 0) for lr in heights)
    assert need >= plan_max + 2 * n * s * 8 + k * s * 8
    # batches of copies: the largest batch workspace plus per-copy U and Hess
    need4 = orth.orth_tune_workspace_bytes(n, s, k, 4)
    batch_max = max(orth.orth_batch_workspace_bytes([n] * 4, [s] * 4, [k] * 4, [lr] * 4) for lr in heights)
    assert need4 >= batch_max + n * s * 8 + 4 * (n * s * 8 + k * k * 8)
    assert orth.orth_tune_workspace_bytes(0, 4, 32, 1) == 0
    assert orth.orth_tune_workspace_bytes(100, 4, 200, 1) == 0       # k_max > n: no candidate
    assert orth.orth_tune_workspace_bytes(n, s, k, 0) == 0           # copies out of range
    # rejected before any device call
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k, 0, 1, 4096, need, None)
    assert code == orth.ORTH_ERR_ARG                                  # steps < 1
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k, k // s + 1, 1, 4096, need, None)
    assert code == orth.ORTH_ERR_ARG                                  # steps > k_max / s
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k, 2, 1, 4096, need - 8, None)
    assert code == orth.ORTH_ERR_WORKSPACE
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k, 2, 1, 4096 + 8, need, None)
    assert code == orth.ORTH_ERR_WORKSPACE                            # misaligned
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k, 2, 4, 4096, need4 - 8, None)
    assert code == orth.ORTH_ERR_WORKSPACE


def test_autotune_batch_buckets(monkeypatch, tmp_path):
    from paper_2204_13393_amd import autotune
    calls = []

    def fake(n, s, k_max, steps=None, copies=1, cache=None, stream=None):
        calls.append((n, s, k_max, copies))
        return 8192
    monkeypatch.setattr(autotune, "tune_leaf_rows", fake)
    ns = [20000, 17000, 1 << 20, 3000, 5000]
    ss = [4, 4, 8, 2, 2]
    ks = [84, 84, 168, 42, 42]
    rows = autotune.tune_batch(ns, ss, ks)
    # 20000 and 17000 share the 2^14 bucket; 3000 rounds to 2^12 and 5000 to 2^12
    assert calls == [(16384, 4, 84, 64), (1 << 20, 8, 168, 8), (4096, 2, 42, 64)]
    # results are clipped to each instance's [k_max, n]
    assert rows == [8192, 8192, 8192, 3000, 5000]


def test_tree_workspace_arguments():
    """Reduction trees: fan-in 1 and negative fan-ins are refused, Householder
    leaves take trees too, a fan-in at or above the leaf count is the
    single level, and the upper levels add storage (host arithmetic only)."""
    one = orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, 0)
    assert one == orth.orth_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64) > 0
    assert orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, 1) == 0
    assert orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, -2) == 0
    # Householder leaves under a tree (their compact-WY factors and a third
    # apply region on top)
    assert orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64_HOUSEHOLDER, 2) > \
        orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, 2) > 0
    assert orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, 20) == one
    assert orth.orth_tree_workspace_bytes(10000, 4, 16, 500, orth.ORTH_FP64, 2) > one
    assert orth.orth_tree_levels(None)[0] == orth.ORTH_ERR_ARG
    assert orth.orth_export_tree_level(None, 0, 0, 1) == orth.ORTH_ERR_ARG
    code, h = orth.orth_create_tree(10000, 4, 16, 500, orth.ORTH_FP64, 1, 0, 0, None)
    assert code == orth.ORTH_ERR_ARG and not h.value


def test_flat_workspace_arguments():
    """FlatTSPQR handles (orth_create_flat): block_rows in [k_max, n] with no
    default, the usual width rules, and a workspace that holds one factor of
    (block rows + k_max) x k_max per block (host arithmetic only)."""
    n, s, kmax = 10000, 4, 16
    one = orth.orth_flat_workspace_bytes(n, s, kmax, n)
    four = orth.orth_flat_workspace_bytes(n, s, kmax, 2500)
    assert one >= 8 * (n + kmax) * kmax                    # the one factor
    assert four >= 8 * ((n + 4 * kmax) * kmax + (n - 2500 + 3 * kmax) * s)   # factors, staging
    assert orth.orth_flat_workspace_bytes(n, s, kmax, 0) == 0             # no default
    assert orth.orth_flat_workspace_bytes(n, s, kmax, kmax - 1) == 0
    assert orth.orth_flat_workspace_bytes(n, s, kmax, n + 1) == 0
    assert orth.orth_flat_workspace_bytes(n, 3, 15, 100) == 0
    assert orth.orth_flat_workspace_bytes(n, s, 18, 100) == 0            # k_max not a multiple of s
    assert orth.orth_flat_workspace_bytes(0, s, kmax, 100) == 0
    assert orth.orth_flat_workspace_bytes(100000, 32, 2048, 4096) == 0   # k_max + s above 2048
    code, h = orth.orth_create_flat(n, s, kmax, 0, 0, 0, None)
    assert code == orth.ORTH_ERR_ARG and not h.value
    code, h = orth.orth_create_flat(100000, 32, 2048, 4096, 0, 0, None)
    assert code == orth.ORTH_ERR_UNSUPPORTED and not h.value
    code, h = orth.orth_create_flat(n, s, kmax, 2500, 0, four, None)
    assert code == orth.ORTH_ERR_WORKSPACE and not h.value
    code, h = orth.orth_create_flat(n, s, kmax, 2500, 256, four - 8, None)
    assert code == orth.ORTH_ERR_WORKSPACE and not h.value


def test_variant_constants_match_the_header():
    """The binding's variant codes are the header's enum values, and the
    level-variant setter checks its handle before anything else."""
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "orth.h")).read()
    for name in ("ORTH_PIP_PLUS", "ORTH_PIP", "ORTH_HOUSEHOLDER"):
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, hdr)
        assert m and int(m.group(1)) == getattr(orth, name), name
    assert orth.orth_set_level_variants(None, orth.ORTH_PIP_PLUS, orth.ORTH_HOUSEHOLDER) == orth.ORTH_ERR_ARG
    assert orth.orth_set_level_variants(None, orth.ORTH_HOUSEHOLDER, orth.ORTH_PIP_PLUS) == orth.ORTH_ERR_ARG


def test_tune_tree_workspace_arguments():
    """The fan-in tuner's workspace holds the largest candidate handle plus
    one block of W, U, H, R; invalid sizes give 0 and ARG (host only)."""
    n, s, kmax, lr = 1 << 16, 8, 64, 1024
    ws = orth.orth_tune_tree_workspace_bytes(n, s, kmax, lr)
    assert ws >= orth.orth_tree_workspace_bytes(n, s, kmax, lr, orth.ORTH_FP64, 2) + 2 * 8 * n * s
    assert orth.orth_tune_tree_workspace_bytes(n, s, kmax, 0) == 0
    assert orth.orth_tune_tree_workspace_bytes(n, s, kmax, kmax - 1) == 0
    assert orth.orth_tune_tree_workspace_bytes(n, 3, kmax, lr) == 0
    code, best, cand = orth.orth_tune_tree(n, s, kmax, lr, 2, 0, 0, None)
    assert code == orth.ORTH_ERR_WORKSPACE
    code, best, cand = orth.orth_tune_tree(n, s, kmax, lr, 0, 256, ws, None)
    assert code == orth.ORTH_ERR_ARG


def test_tile_shapes_workspace_and_arguments():
    """orth_tiles: the plan's own tiles size the workspace like
    orth_tree_workspace_bytes; smaller leaf-Gram tiles mean more partial-sum
    slots and never a smaller workspace; row-update heights and the kernel
    choice do not change it; values off the power-of-two ranges are refused
    (host only)."""
    n, s, kmax, lr = 1 << 20, 8, 64, 4096
    F = orth.ORTH_FP64
    base = orth.orth_tree_workspace_bytes(n, s, kmax, lr, F, 0)
    assert orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, None) == base
    assert orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, (0, 0, 0)) == base
    small = orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, (128, 0, 0))
    big = orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, (8192, 0, 0))
    assert small > base >= big > 0
    for upd, kern in ((64, 0), (8192, 1), (512, 1)):
        assert orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, (0, upd, kern)) == base
    for bad in ((100, 0, 0), (64, 0, 0), (16384, 0, 0), (0, 32, 0), (0, 16384, 0), (0, 100, 0), (0, 0, 2),
                (0, 0, -1)):
        assert orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, bad) == 0, bad
        code, h = orth.orth_create_tiles(n, s, kmax, lr, F, 0, bad, 4096, 1 << 40, None)
        assert code == orth.ORTH_ERR_ARG, bad
    # the tuner's workspace holds its largest candidate handle plus W, U, H, R
    ws = orth.orth_tune_tiles_workspace_bytes(n, s, kmax, lr)
    assert ws >= orth.orth_tiles_workspace_bytes(n, s, kmax, lr, F, 0, (1024, 0, 0)) + 2 * 8 * n * s
    assert orth.orth_tune_tiles_workspace_bytes(n, s, kmax, 0) == 0
    code, best, cand = orth.orth_tune_tiles(n, s, kmax, lr, 2, 0, 0, None)
    assert code == orth.ORTH_ERR_WORKSPACE
    code, best, cand = orth.orth_tune_tiles(n, s, kmax, lr, 0, 256, ws, None)
    assert code == orth.ORTH_ERR_ARG
    assert orth.orth_tiles_in_use(None)[0] == orth.ORTH_ERR_ARG
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "orth.h")).read()
    import re
    for name in ("ORTH_TILE_AUTO", "ORTH_TILE_REGISTER"):
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, hdr)
        assert m and int(m.group(1)) == getattr(orth, name), name


def test_large_plan_sizes_are_sane():
    """Plans far past one GPU's memory still size consistently (64-bit row
    counts throughout): the workspace holds at least the leaf bases and stays
    within a small multiple of them (host arithmetic only)."""
    n, s, kmax = 1 << 34, 8, 248
    for lr in (kmax, 4096, 1 << 16):
        b = orth.orth_workspace_bytes(n, s, kmax, lr, orth.ORTH_FP64)
        assert 8 * n * kmax <= b <= 4 * 8 * n * kmax, (lr, b)
        t = orth.orth_tree_workspace_bytes(n, s, kmax, lr, orth.ORTH_FP64, 16)
        assert b <= t <= 4 * 8 * n * kmax, (lr, t)
