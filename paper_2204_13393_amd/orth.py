"""Thin Python binding of liborth.so (the C ABI declared in include/orth.h).

Every function here only marshals arguments: each step of the method runs
in the library's HIP kernels.  There is no fallback: if the shared library is
missing or cannot be loaded, ``load()`` raises and nothing runs.

Raw calls keep the C names and argument order (pointers are ints, streams are
ints holding a hipStream_t).  ``Orthogonalizer`` is a convenience wrapper that
owns a torch-allocated workspace and takes torch device tensors; a
column-major n x s matrix is a contiguous torch tensor of shape (s, n).
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborth.so")

ORTH_OK = 0
ORTH_ERR_ARG = 1
ORTH_ERR_CAPACITY = 2
ORTH_ERR_BREAKDOWN = 3
ORTH_ERR_HIP = 4
ORTH_ERR_POISONED = 5
ORTH_ERR_WORKSPACE = 6
ORTH_ERR_UNSUPPORTED = 7
ORTH_ERR_SCRATCH = 8
ORTH_FP64 = 0
ORTH_MIXED_SPLIT32 = 1
ORTH_FP64_HOUSEHOLDER = 2
ORTH_PIP_PLUS = 0
ORTH_PIP = 1
ORTH_HOUSEHOLDER = 2      # reduction variant only
ORTH_TILE_AUTO = 0
ORTH_TILE_REGISTER = 1


class OrthTiles(ctypes.Structure):
    """orth_tiles: rows per workgroup of the leaf Grams and row updates, row-update kernel."""
    _fields_ = [("gram_rows", ctypes.c_int32), ("update_rows", ctypes.c_int32), ("update_kernel", ctypes.c_int32)]

    def as_tuple(self):
        return (self.gram_rows, self.update_rows, self.update_kernel)



CODE_NAMES = {0: "OK", 1: "ARG", 2: "CAPACITY", 3: "BREAKDOWN", 4: "HIP", 5: "POISONED",
              6: "WORKSPACE", 7: "UNSUPPORTED", 8: "SCRATCH"}

# (name, restype, argtypes) for every symbol in include/orth.h and include/orth_measure.h
_i32, _i64, _sz, _vp, _dp = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p
SIGNATURES = [
    ("orth_workspace_bytes", _sz, [_i64, _i32, _i32, _i32, _i32]),
    ("orth_create", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    ("orth_tree_workspace_bytes", _sz, [_i64, _i32, _i32, _i32, _i32, _i32]),
    ("orth_create_tree", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    ("orth_tree_levels", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("orth_export_tree_level", ctypes.c_int, [_vp, _i32, _dp, _i64]),
    ("orth_flat_workspace_bytes", _sz, [_i64, _i32, _i32, _i32]),
    ("orth_tiles_workspace_bytes", _sz, [_i64, _i32, _i32, _i32, _i32, _i32, _vp]),
    ("orth_create_tiles", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _sz, _vp,
                                         ctypes.POINTER(_vp)]),
    ("orth_tiles_in_use", ctypes.c_int, [_vp, _vp]),
    ("orth_tune_tiles_workspace_bytes", _sz, [_i64, _i32, _i32, _i32]),
    ("orth_tune_tiles", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _vp, _sz, _vp, _vp, _vp,
                                       ctypes.POINTER(ctypes.c_double), _i32, ctypes.POINTER(_i32)]),
    ("orth_tune_tree_workspace_bytes", _sz, [_i64, _i32, _i32, _i32]),
    ("orth_tune_tree", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double), _i32,
                                      ctypes.POINTER(_i32)]),
    ("orth_create_flat", ctypes.c_int, [_i64, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    ("orth_set_variant", ctypes.c_int, [_vp, _i32]),
    ("orth_set_level_variants", ctypes.c_int, [_vp, _i32, _i32]),
    ("orth_mixed_fallbacks", ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    ("orth_set_deflation", ctypes.c_int, [_vp, ctypes.c_double]),
    ("orth_deflation_info", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    ("orth_step", ctypes.c_int, [_vp, _dp, _i64, _dp, _i64, _dp, _i64, _dp, _i64]),
    ("orth_apply_Q", ctypes.c_int, [_vp, _dp, _i64, _i32, _dp, _i64]),
    ("orth_apply_Q_noalloc", ctypes.c_int, [_vp, _dp, _i64, _i32, _dp, _i64]),
    ("orth_status", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("orth_basis_width", ctypes.c_int, [_vp, ctypes.POINTER(_i32)]),
    ("orth_leaf_count", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("orth_export_local", ctypes.c_int, [_vp, _dp, _i64, _dp, _i64]),
    ("orth_profile_enable", ctypes.c_int, [_vp, _i32]),
    ("orth_profile_select", ctypes.c_int, [_vp, ctypes.c_uint32]),
    ("orth_profile_read", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
    ("orth_profile_reset", ctypes.c_int, [_vp]),
    ("orth_destroy", ctypes.c_int, [_vp]),
    ("orth_batch_workspace_bytes", _sz, [_i32, _vp, _vp, _vp, _vp, _i32]),
    ("orth_batch_create", ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp,
                                         ctypes.POINTER(_vp)]),
    ("orth_batch_set_variant", ctypes.c_int, [_vp, _i32]),
    ("orth_batch_step", ctypes.c_int, [_vp, _dp, _dp, _dp]),
    ("orth_batch_status", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("orth_batch_mixed_fallbacks", ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    ("orth_batch_progress", ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("orth_batch_leaf_rows", ctypes.c_int, [_vp, _vp]),
    ("orth_batch_destroy", ctypes.c_int, [_vp]),
    ("orth_laplacian_apply", ctypes.c_int, [_dp, _i64, _dp, _i64, _i32, _i32, _i32, _i32,
                                            ctypes.c_double, _vp]),
    ("orth_probe_copy", ctypes.c_int, [_dp, _dp, _i64, _vp]),
    ("orth_tune_workspace_bytes", _sz, [_i64, _i32, _i32, _i32]),
    ("orth_tune_leaf_rows", ctypes.c_int, [_i64, _i32, _i32, _i32, _i32, _vp, _sz, _vp,
                                           ctypes.POINTER(_i32), _vp, _vp, _i32, ctypes.POINTER(_i32)]),
]

_lib = None


class OrthError(RuntimeError):
    def __init__(self, func, code):
        super().__init__(f"{func} failed: ORTH_ERR_{CODE_NAMES.get(code, code)} ({code})")
        self.code = code


def load(path=LIB_PATH):
    """Load liborth.so once; raises if it is not built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2204_13393_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(func, code):
    if code != ORTH_OK:
        raise OrthError(func, code)


# ---- raw calls (same names as the C ABI) --------------------------------

def orth_workspace_bytes(n, s, k_max, leaf_rows=0, precision=ORTH_FP64):
    return load().orth_workspace_bytes(n, s, k_max, leaf_rows, precision)


def orth_create(n, s, k_max, leaf_rows, precision, d_workspace, workspace_bytes, stream):
    h = ctypes.c_void_p()
    code = load().orth_create(n, s, k_max, leaf_rows, precision, d_workspace, workspace_bytes,
                              stream, ctypes.byref(h))
    return code, h


def orth_tree_workspace_bytes(n, s, k_max, leaf_rows=0, precision=ORTH_FP64, fan_in=0):
    return load().orth_tree_workspace_bytes(n, s, k_max, leaf_rows, precision, fan_in)


def orth_create_tree(n, s, k_max, leaf_rows, precision, fan_in, d_workspace, workspace_bytes, stream):
    h = ctypes.c_void_p()
    code = load().orth_create_tree(n, s, k_max, leaf_rows, precision, fan_in, d_workspace, workspace_bytes,
                                   stream, ctypes.byref(h))
    return code, h


def orth_tree_levels(h):
    lv, fi = ctypes.c_int32(), ctypes.c_int32()
    code = load().orth_tree_levels(h, ctypes.byref(lv), ctypes.byref(fi))
    return code, lv.value, fi.value


def orth_export_tree_level(h, level, d_T, ldt):
    return load().orth_export_tree_level(h, level, d_T, ldt)


def orth_flat_workspace_bytes(n, s, k_max, block_rows):
    return load().orth_flat_workspace_bytes(n, s, k_max, block_rows)


def orth_create_flat(n, s, k_max, block_rows, d_workspace, workspace_bytes, stream):
    h = ctypes.c_void_p()
    code = load().orth_create_flat(n, s, k_max, block_rows, d_workspace, workspace_bytes, stream,
                                   ctypes.byref(h))
    return code, h


def _tiles_arg(tiles):
    if tiles is None:
        return None, None
    t = tiles if isinstance(tiles, OrthTiles) else OrthTiles(*tiles)
    return t, ctypes.cast(ctypes.byref(t), _vp)


def orth_tiles_workspace_bytes(n, s, k_max, leaf_rows, precision, fan_in, tiles):
    t, ptr = _tiles_arg(tiles)
    return load().orth_tiles_workspace_bytes(n, s, k_max, leaf_rows, precision, fan_in, ptr)


def orth_create_tiles(n, s, k_max, leaf_rows, precision, fan_in, tiles, d_workspace, workspace_bytes, stream):
    h = ctypes.c_void_p()
    t, ptr = _tiles_arg(tiles)
    code = load().orth_create_tiles(n, s, k_max, leaf_rows, precision, fan_in, ptr, d_workspace,
                                    workspace_bytes, stream, ctypes.byref(h))
    return code, h


def orth_tiles_in_use(h):
    t = OrthTiles()
    code = load().orth_tiles_in_use(h, ctypes.cast(ctypes.byref(t), _vp))
    return code, t.as_tuple()


def orth_tune_tiles_workspace_bytes(n, s, k_max, leaf_rows):
    return load().orth_tune_tiles_workspace_bytes(n, s, k_max, leaf_rows)


def orth_tune_tiles(n, s, k_max, leaf_rows, steps, d_workspace, workspace_bytes, stream, max_cand=32):
    """(code, best (gram_rows, update_rows, update_kernel), [(tiles, ms), ...])"""
    best = OrthTiles()
    cand = (OrthTiles * max(max_cand, 1))()
    ms = (ctypes.c_double * max(max_cand, 1))()
    nc = ctypes.c_int32()
    code = load().orth_tune_tiles(n, s, k_max, leaf_rows, steps, d_workspace, workspace_bytes, stream,
                                  ctypes.cast(ctypes.byref(best), _vp), ctypes.cast(cand, _vp), ms, max_cand,
                                  ctypes.byref(nc))
    return code, best.as_tuple(), [(cand[i].as_tuple(), ms[i]) for i in range(min(nc.value, max_cand))]


def orth_tune_tree_workspace_bytes(n, s, k_max, leaf_rows):
    return load().orth_tune_tree_workspace_bytes(n, s, k_max, leaf_rows)


def orth_tune_tree(n, s, k_max, leaf_rows, steps, d_workspace, workspace_bytes, stream, max_cand=16):
    """(code, best fan-in, [(fan_in, ms), ...])"""
    best = ctypes.c_int32()
    fans = (ctypes.c_int32 * max(max_cand, 1))()
    ms = (ctypes.c_double * max(max_cand, 1))()
    nc = ctypes.c_int32()
    code = load().orth_tune_tree(n, s, k_max, leaf_rows, steps, d_workspace, workspace_bytes, stream,
                                 ctypes.byref(best), fans, ms, max_cand, ctypes.byref(nc))
    return code, best.value, [(fans[i], ms[i]) for i in range(min(nc.value, max_cand))]


def orth_set_variant(h, variant):
    return load().orth_set_variant(h, variant)


def orth_set_level_variants(h, leaf_variant, reduction_variant):
    return load().orth_set_level_variants(h, leaf_variant, reduction_variant)


def orth_mixed_fallbacks(h):
    n = _i64(0)
    code = load().orth_mixed_fallbacks(h, ctypes.byref(n))
    return code, n.value


def orth_set_deflation(h, delta):
    return load().orth_set_deflation(h, float(delta))


def orth_deflation_info(h):
    """(code, rank of the latest step, steps with a drop, columns dropped)."""
    t, st, dr = _i32(0), _i64(0), _i64(0)
    code = load().orth_deflation_info(h, ctypes.byref(t), ctypes.byref(st), ctypes.byref(dr))
    return code, t.value, st.value, dr.value


def orth_step(h, d_W, ldw, d_H, ldh, d_R, ldr, d_U, ldu):
    return load().orth_step(h, d_W, ldw, d_H, ldh, d_R, ldr, d_U, ldu)


def orth_apply_Q(h, d_C, ldc, m, d_Y, ldy):
    return load().orth_apply_Q(h, d_C, ldc, m, d_Y, ldy)


def orth_apply_Q_noalloc(h, d_C, ldc, m, d_Y, ldy):
    return load().orth_apply_Q_noalloc(h, d_C, ldc, m, d_Y, ldy)


def orth_status(h):
    st = ctypes.c_int32()
    info = (ctypes.c_int32 * 4)()
    code = load().orth_status(h, ctypes.byref(st), info)
    return code, st.value, list(info)


def orth_basis_width(h):
    k = ctypes.c_int32()
    code = load().orth_basis_width(h, ctypes.byref(k))
    return code, k.value


def orth_leaf_count(h):
    p, lr = ctypes.c_int32(), ctypes.c_int32()
    code = load().orth_leaf_count(h, ctypes.byref(p), ctypes.byref(lr))
    return code, p.value, lr.value


def orth_export_local(h, d_Qloc, ldq, d_T, ldt):
    return load().orth_export_local(h, d_Qloc, ldq, d_T, ldt)


KERNEL_CLASSES = ["leaf_gram", "leaf_chol", "leaf_correct", "root_gram", "root_chol",
                  "root_correct", "root_finalize", "leaf_finalize", "apply", "leaf_gram2",
                  "root_gram2", "leaf_fallback", "leaf_hh_panel", "leaf_hh_small"]


def orth_profile_enable(h, on):
    return load().orth_profile_enable(h, int(on))


def orth_profile_select(h, class_mask):
    return load().orth_profile_select(h, int(class_mask) & 0xFFFFFFFF)


def orth_profile_read(h):
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    code = load().orth_profile_read(h, ms, cnt)
    return code, {KERNEL_CLASSES[i]: (ms[i], cnt[i]) for i in range(n)}


def orth_profile_reset(h):
    return load().orth_profile_reset(h)


def orth_destroy(h):
    return load().orth_destroy(h)


def orth_laplacian_apply(d_X, ldx, d_Y, ldy, s, nx, ny, nz, shift, stream):
    return load().orth_laplacian_apply(d_X, ldx, d_Y, ldy, s, nx, ny, nz, shift, stream)


def orth_probe_copy(d_src, d_dst, count, stream):
    return load().orth_probe_copy(d_src, d_dst, count, stream)


def orth_tune_workspace_bytes(n, s, k_max, copies=1):
    return load().orth_tune_workspace_bytes(n, s, k_max, copies)


def orth_tune_leaf_rows(n, s, k_max, steps, copies, d_workspace, workspace_bytes, stream, max_cand=16):
    """Returns (code, best leaf height, [(candidate, ms), ...])."""
    best, count = ctypes.c_int32(), ctypes.c_int32()
    rows = (_i32 * max_cand)()
    ms = (ctypes.c_double * max_cand)()
    code = load().orth_tune_leaf_rows(n, s, k_max, steps, copies, d_workspace, workspace_bytes, stream,
                                      ctypes.byref(best), ctypes.cast(rows, _vp), ctypes.cast(ms, _vp),
                                      max_cand, ctypes.byref(count))
    cand = [(rows[i], ms[i]) for i in range(min(count.value, max_cand))] if code == ORTH_OK else []
    return code, best.value, cand


def _arr(ctype, values):
    if values is None:
        return None
    return (ctype * len(values))(*values)


def orth_batch_workspace_bytes(n, s, k_max, leaf_rows=None, precision=ORTH_FP64):
    count = len(n)
    return load().orth_batch_workspace_bytes(
        count, ctypes.cast(_arr(ctypes.c_int64, n), _vp), ctypes.cast(_arr(_i32, s), _vp),
        ctypes.cast(_arr(_i32, k_max), _vp),
        ctypes.cast(_arr(_i32, leaf_rows), _vp) if leaf_rows is not None else None, precision)


def orth_batch_create(n, s, k_max, leaf_rows, precision, d_workspace, workspace_bytes, stream):
    h = ctypes.c_void_p()
    count = len(n)
    code = load().orth_batch_create(
        count, ctypes.cast(_arr(ctypes.c_int64, n), _vp), ctypes.cast(_arr(_i32, s), _vp),
        ctypes.cast(_arr(_i32, k_max), _vp),
        ctypes.cast(_arr(_i32, leaf_rows), _vp) if leaf_rows is not None else None,
        precision, d_workspace, workspace_bytes, stream, ctypes.byref(h))
    return code, h


def orth_batch_set_variant(b, variant):
    return load().orth_batch_set_variant(b, variant)


def orth_batch_step(b, d_W, d_U, d_Hess):
    return load().orth_batch_step(b, d_W, d_U, d_Hess)


def orth_batch_status(b):
    st = ctypes.c_int32()
    info = (ctypes.c_int32 * 5)()
    code = load().orth_batch_status(b, ctypes.byref(st), info)
    return code, st.value, list(info)


def orth_batch_mixed_fallbacks(b):
    n = _i64(0)
    code = load().orth_batch_mixed_fallbacks(b, ctypes.byref(n))
    return code, n.value


def orth_batch_progress(b):
    done, mx = ctypes.c_int32(), ctypes.c_int32()
    code = load().orth_batch_progress(b, ctypes.byref(done), ctypes.byref(mx))
    return code, done.value, mx.value


def orth_batch_leaf_rows(b, count):
    out = (_i32 * count)()
    code = load().orth_batch_leaf_rows(b, ctypes.cast(out, _vp))
    return code, list(out)


def orth_batch_destroy(b):
    return load().orth_batch_destroy(b)


# ---- torch convenience wrapper ------------------------------------------

def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Orthogonalizer:
    """One TreeTSPQR basis on one GPU, with a torch-owned workspace.

    Tensors are column-major: an n x s matrix is a contiguous float64 tensor
    of shape (s, n) on the device.  flat=True: FlatTSPQR over blocks of
    leaf_rows rows instead (orth_create_flat; FP64, no reduction tree).
    tiles: None or (gram_rows, update_rows, update_kernel) for orth_create_tiles.
    """

    def __init__(self, n, s, k_max, leaf_rows=0, device="cuda", stream=None, variant=ORTH_PIP_PLUS,
                 precision=ORTH_FP64, reduction_variant=None, fan_in=0, flat=False, tiles=None):
        import torch
        load()
        self.n, self.s, self.k_max = int(n), int(s), int(k_max)
        self.precision = precision
        self.device = torch.device(device)
        self.flat = bool(flat)
        if self.flat:
            if precision != ORTH_FP64 or fan_in or tiles is not None:
                raise OrthError("orth_create_flat", ORTH_ERR_UNSUPPORTED)
            nbytes = orth_flat_workspace_bytes(self.n, self.s, self.k_max, leaf_rows)
        else:
            nbytes = orth_tiles_workspace_bytes(self.n, self.s, self.k_max, leaf_rows, precision, fan_in, tiles)
        if nbytes == 0:
            raise OrthError("orth_workspace_bytes", ORTH_ERR_ARG)
        self.stream = stream
        self.workspace = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        if self.flat:
            code, h = orth_create_flat(self.n, self.s, self.k_max, leaf_rows, aligned, nbytes, _stream_ptr(stream))
        else:
            code, h = orth_create_tiles(self.n, self.s, self.k_max, leaf_rows, precision, fan_in, tiles, aligned,
                                        nbytes, _stream_ptr(stream))
        _check("orth_create", code)
        self.h = h
        red = variant if reduction_variant is None else reduction_variant
        _check("orth_set_level_variants", orth_set_level_variants(self.h, variant, red))
        _, self.p, self.leaf_rows = orth_leaf_count(self.h)
        _, self.levels, self.fan_in = orth_tree_levels(self.h)

    @property
    def k(self):
        return orth_basis_width(self.h)[1]

    @property
    def tiles(self):
        """(gram_rows, update_rows, update_kernel) the plan resolved."""
        code, t = orth_tiles_in_use(self.h)
        _check("orth_tiles_in_use", code)
        return t

    def step(self, W, H=None, R=None, U=None):
        """Solve eq. (1.1) for W ((s, n) tensor); returns (H (s,k), R (s,s), U (s,n))."""
        import torch
        k, s, n = self.k, self.s, self.n
        assert W.dtype == torch.float64 and W.is_contiguous() and W.shape == (s, n)
        if H is None:
            H = torch.empty((s, max(k, 1)), dtype=torch.float64, device=self.device)
        if R is None:
            R = torch.empty((s, s), dtype=torch.float64, device=self.device)
        if U is None:
            U = torch.empty((s, n), dtype=torch.float64, device=self.device)
        code = orth_step(self.h, W.data_ptr(), n, H.data_ptr(), max(k, 1), R.data_ptr(), s,
                         U.data_ptr(), n)
        _check("orth_step", code)
        return H[:, :k], R, U

    def apply_Q(self, C, Y=None):
        """Y = Q C for C ((m, k) tensor, column-major k x m); returns (m, n)."""
        import torch
        m, k = C.shape
        assert k == self.k and C.is_contiguous()
        if Y is None:
            Y = torch.empty((m, self.n), dtype=torch.float64, device=self.device)
        _check("orth_apply_Q", orth_apply_Q(self.h, C.data_ptr(), k, m, Y.data_ptr(), self.n))
        return Y

    def status(self):
        code, st, info = orth_status(self.h)
        _check("orth_status", code)
        return st, info

    def set_deflation(self, delta):
        """Deflate at the reduction level with relative tolerance delta (0: off)."""
        _check("orth_set_deflation", orth_set_deflation(self.h, delta))

    def deflation_info(self):
        """(rank of the latest step, steps with a drop, columns dropped)."""
        code, t, steps, dropped = orth_deflation_info(self.h)
        _check("orth_deflation_info", code)
        return t, steps, dropped

    def export_local(self):
        """(Qloc (k, n) column-major n x k, T (k, p*k) column-major (p k) x k)."""
        import torch
        k = self.k
        Qloc = torch.empty((k, self.n), dtype=torch.float64, device=self.device)
        T = torch.empty((k, self.p * k), dtype=torch.float64, device=self.device)
        _check("orth_export_local",
               orth_export_local(self.h, Qloc.data_ptr(), self.n, T.data_ptr(), self.p * k))
        return Qloc, T

    def export_tree_level(self, level):
        """Level `level`'s stacked node factors: (k, children*k), column-major (children k) x k."""
        import torch
        k = self.k
        children = self.p
        for _ in range(level):
            children = (children + self.fan_in - 1) // self.fan_in
        T = torch.empty((k, children * k), dtype=torch.float64, device=self.device)
        _check("orth_export_tree_level", orth_export_tree_level(self.h, level, T.data_ptr(), children * k))
        return T

    def close(self):
        if getattr(self, "h", None) is not None:
            orth_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def laplacian_apply(X, grid, shift=0.0, Y=None, stream=None):
    """Y = A X with the library's test Laplacian; X is (s, n) float64 on the device."""
    import torch
    s, n = X.shape
    nx, ny = grid[0], grid[1]
    nz = grid[2] if len(grid) > 2 else 1
    if Y is None:
        Y = torch.empty_like(X)
    _check("orth_laplacian_apply", orth_laplacian_apply(X.data_ptr(), n, Y.data_ptr(), n, s, nx, ny,
                                                        nz, float(shift), _stream_ptr(stream)))
    return Y


class BatchOrthogonalizer:
    """Many independent TreeTSPQR bases advancing one step per call.

    n, s, k_max, leaf_rows: per-instance lists (leaf_rows None or 0 entries:
    default height).  Tensors are column-major as in ``Orthogonalizer``:
    instance i's block is a (s_i, n_i) float64 tensor, its Hessenberg buffer a
    (K_i, K_i) tensor (column j of the K_i x K_i matrix is row j of the tensor).
    precision: ORTH_FP64, ORTH_MIXED_SPLIT32 or ORTH_FP64_HOUSEHOLDER (every instance).
    """

    def __init__(self, n, s, k_max, leaf_rows=None, device="cuda", stream=None, variant=ORTH_PIP_PLUS,
                 precision=ORTH_FP64):
        import torch
        load()
        self.n, self.s, self.k_max = list(map(int, n)), list(map(int, s)), list(map(int, k_max))
        self.count = len(self.n)
        self.device = torch.device(device)
        self.precision = precision
        nbytes = orth_batch_workspace_bytes(self.n, self.s, self.k_max, leaf_rows, precision)
        if nbytes == 0:
            raise OrthError("orth_batch_workspace_bytes", ORTH_ERR_ARG)
        self.workspace = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream
        code, h = orth_batch_create(self.n, self.s, self.k_max, leaf_rows, precision, aligned, nbytes,
                                    _stream_ptr(stream))
        _check("orth_batch_create", code)
        self.h = h
        _check("orth_batch_set_variant", orth_batch_set_variant(self.h, variant))
        self.leaf_rows = orth_batch_leaf_rows(self.h, self.count)[1]
        self._ptrs = {}

    def pointer_array(self, tensors):
        """Device int64 array of the tensors' data pointers (cached by identity)."""
        import torch
        key = tuple(t.data_ptr() for t in tensors)
        arr = self._ptrs.get(key)
        if arr is None:
            arr = torch.tensor(list(key), dtype=torch.int64, device=self.device)
            self._ptrs[key] = arr
        return arr

    def step(self, W, U, Hess):
        """One step for every instance; W, U, Hess are lists of tensors (or device pointer arrays)."""
        pw = W if not isinstance(W, (list, tuple)) else self.pointer_array(W)
        pu = U if not isinstance(U, (list, tuple)) else self.pointer_array(U)
        ph = Hess if not isinstance(Hess, (list, tuple)) else self.pointer_array(Hess)
        _check("orth_batch_step", orth_batch_step(self.h, pw.data_ptr(), pu.data_ptr(), ph.data_ptr()))

    def progress(self):
        return orth_batch_progress(self.h)[1:]

    def mixed_fallbacks(self):
        code, n = orth_batch_mixed_fallbacks(self.h)
        _check("orth_batch_mixed_fallbacks", code)
        return n

    def status(self):
        code, st, info = orth_batch_status(self.h)
        _check("orth_batch_status", code)
        return st, info

    def close(self):
        if getattr(self, "h", None) is not None:
            orth_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
