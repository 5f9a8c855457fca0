"""Leaf-height autotuner: the local problem size chosen by measurement.

The leaf height (local problem size, Sec. 4.1) trades the leaves' streaming
work against the reduction level, which holds p (k+s) rows for p leaves; its
best value depends on the machine (the local problem size study of Sec. 6.2).
The measurement runs in the library (``orth_tune_leaf_rows`` times whole
step sequences on synthetic blocks for every candidate height, through one
handle or through a batch of identical copies); this module owns the device
workspace for it, caches results per device and shape in a JSON file, and
buckets the instances of a batch so that a batch of hundreds of uneven
instances needs only a few dozen measurements.  Batch buckets are measured
as batches of copies of the bucket's shape, so that the GPU is as busy as in
the real batch (one small instance alone only measures launch latency).
"""

import json
import math
import os

from . import orth

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2204_13393_amd", "leaf_rows.json")


def _cache_path(cache):
    return cache or os.environ.get("ORTH_TUNE_CACHE") or DEFAULT_CACHE


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure_leaf_rows(n, s, k_max, steps=None, copies=1, stream=None):
    """Run the library's tuner once (no cache): (best, [(candidate, ms), ...])."""
    import torch
    steps = steps or min(k_max // s, 32)
    nbytes = orth.orth_tune_workspace_bytes(n, s, k_max, copies)
    if nbytes == 0:
        raise orth.OrthError("orth_tune_workspace_bytes", orth.ORTH_ERR_ARG)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    sp = (stream or torch.cuda.current_stream()).cuda_stream
    code, best, cand = orth.orth_tune_leaf_rows(n, s, k_max, steps, copies, base, nbytes, sp)
    del ws
    if code != orth.ORTH_OK:
        raise orth.OrthError("orth_tune_leaf_rows", code)
    return best, cand


def measure_fan_in(n, s, k_max, leaf_rows, steps=None, stream=None):
    """Run the library's fan-in tuner for single handles once:
    (best fan-in, [(candidate, ms), ...]); 0 is the single reduction level."""
    import torch
    steps = steps or min(k_max // s, 32)
    nbytes = orth.orth_tune_tree_workspace_bytes(n, s, k_max, leaf_rows)
    if nbytes == 0:
        raise orth.OrthError("orth_tune_tree_workspace_bytes", orth.ORTH_ERR_ARG)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    sp = (stream or torch.cuda.current_stream()).cuda_stream
    code, best, cand = orth.orth_tune_tree(n, s, k_max, leaf_rows, steps, base, nbytes, sp)
    del ws
    if code != orth.ORTH_OK:
        raise orth.OrthError("orth_tune_tree", code)
    return best, cand


def measure_tiles(n, s, k_max, leaf_rows, steps=None, stream=None):
    """Run the library's tile tuner once: (best (gram_rows, update_rows,
    update_kernel), [(candidate, ms), ...]); (0, 0, 0) is the plan's own."""
    import torch
    steps = steps or min(k_max // s, 32)
    nbytes = orth.orth_tune_tiles_workspace_bytes(n, s, k_max, leaf_rows)
    if nbytes == 0:
        raise orth.OrthError("orth_tune_tiles_workspace_bytes", orth.ORTH_ERR_ARG)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    sp = (stream or torch.cuda.current_stream()).cuda_stream
    code, best, cand = orth.orth_tune_tiles(n, s, k_max, leaf_rows, steps, base, nbytes, sp)
    del ws
    if code != orth.ORTH_OK:
        raise orth.OrthError("orth_tune_tiles", code)
    return best, cand


def tune_leaf_rows(n, s, k_max, steps=None, copies=1, cache=None, stream=None):
    """Measured leaf height for one shape, cached per device and shape."""
    import torch
    steps = steps or min(k_max // s, 32)
    path = _cache_path(cache)
    key = f"{torch.cuda.get_device_name()}|n={n}|s={s}|k_max={k_max}|steps={steps}|copies={copies}"
    table = _load(path)
    if key in table:
        return int(table[key]["leaf_rows"])
    best, cand = measure_leaf_rows(n, s, k_max, steps, copies, stream)
    table[key] = {"leaf_rows": best, "candidates_ms": {str(r): m for r, m in cand}}
    _store(path, table)
    return best


def bucket_of(n, s, k_max):
    """Instances share a measurement when s and k_max agree and n rounds to the
    same power of two; the bucket is measured at that power of two."""
    nb = 2 ** int(round(math.log2(n)))
    return (max(nb, k_max), s, k_max)


BATCH_ROWS = 1 << 23    # rows a bucket's measurement batch aims for (copies of its shape)


def batch_copies(n):
    return int(min(64, max(1, BATCH_ROWS // n)))


def tune_batch(ns, ss, ks, steps=None, cache=None, stream=None):
    """Leaf heights for a batch: one measurement per bucket (a batch of copies
    of the bucket's shape), each result clipped to the instance's own
    admissible range [k_max, n]."""
    chosen = {}
    out = []
    for n, s, k in zip(ns, ss, ks):
        b = bucket_of(n, s, k)
        if b not in chosen:
            chosen[b] = tune_leaf_rows(b[0], s, k, steps, batch_copies(b[0]), cache, stream)
        out.append(int(min(max(chosen[b], k), n)))
    return out
