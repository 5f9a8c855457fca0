"""Host-side checks of the C ABI (CPU): the library loads, exports every symbol
that include/orth.h declares, sizes workspaces by pure arithmetic, and rejects
bad arguments before touching the GPU."""

import os
import re

import pytest

from paper_2204_13393_amd import orth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "orth.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(orth_[a-zA-Z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = orth.load()
    names = _declared()
    assert "orth_step" in names and "orth_create" in names and "orth_apply_Q" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared set
    assert sorted(n for n, _, _ in orth.SIGNATURES) == names


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
    (1000, 4, 40, 0, 1),     # unknown precision
    (100000, 16, 2048, 0, 0),  # wider than the planner accepts (k_max + s > 2048)
])
def test_workspace_rejects_bad_arguments(args):
    assert orth.orth_workspace_bytes(*args) == 0


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
    assert orth.orth_set_variant(None, 0) == orth.ORTH_ERR_ARG
    assert orth.orth_destroy(None) == orth.ORTH_OK
    assert orth.orth_laplacian_apply(0, 1, 0, 1, 1, 1, 1, 1, 0.0, None) == orth.ORTH_ERR_ARG
    assert orth.orth_probe_copy(0, 0, 1, None) == orth.ORTH_ERR_ARG


def test_product_path_has_no_oracle_import():
    """The product package never imports the oracle (which is test-only)."""
    pkg = os.path.join(os.path.dirname(HEADER), "..", "paper_2204_13393_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(root, f)).read()
                assert "oracle" not in re.findall(r"^\s*(?:from|import)\s+(\w+)", src, flags=re.M), f
