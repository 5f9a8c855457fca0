#!/usr/bin/env python3
"""Benchmark of the block-Arnoldi orthogonalisation hot path on one MI355X.

Workload (one "step" of this benchmark): orthogonalise every block of a
30-step block-Arnoldi run on the 2D Dirichlet 5-point Laplacian on a
4096 x 4096 grid (n = 2^24 rows), block width s = 8, TSQR leaf height 4096
(4096 leaves), basis kept in locally orthogonal form: orth_create on the
workspace, then 31 orth_step calls (the start block, k = 0, and 30 Krylov
blocks, k = 8 .. 240).  The 31 input blocks (the seeded N(0,1) start block
and the A U_j blocks of the Arnoldi run) are generated on the GPU before
timing and stay resident in HBM; the operator is not part of the timed work.

Reported value: algorithmic HBM throughput of the whole sequence (GB/s,
higher is better): sum over the 31 calls of
    B(k) = 16 n (k + 2s) + 8 p (2 k^2 + 3 s (k + s))
bytes (two reads of the basis and the block, writes of U_i and U, and the
tree-factor traffic), divided by the measured time.  ``ms_per_step`` is the
time of one whole 31-call sequence.  The roofline object refers to the
dominant kernel class, timed live in the timed region with HIP events on the
handle's stream around that class's launches only (each event pair adds a
gap on the stream); one untimed sequence with every launch bracketed gives
the per-class breakdown (``kernels``) and picks the class.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "block-Arnoldi orth step time + HBM GB/s, mixed vs FP64 at \u2016I\u2212Q\u1d40Q\u2016\u22641e-10"
HBM_PEAK_GBS = 8000.0
DEFL_DELTA = 1e-6       # relative tolerance of the deflating runs
WORKLOAD = dict(name="lap2d-4096x4096-s8", nx=4096, ny=4096, s=8, steps=30, leaf_rows=4096, seed=0)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2204_13393_amd", "csrc", "orth_kernels.hip")
KERNEL_HDR = os.path.join(ROOT, "paper_2204_13393_amd", "csrc", "orth_internal.h")


def step_bytes(n, s, p, k):
    """Algorithmic bytes of one orth_step at basis width k."""
    return 16.0 * n * (k + 2 * s) + 8.0 * p * (2.0 * k * k + 3.0 * s * (k + s))


def kernel_bytes(cls, n, s, p, k):
    """Algorithmic bytes one launch of a kernel class must move at width k."""
    if cls in ("leaf_gram", "leaf_gram2"):
        return 8.0 * n * (k + s)                      # read Q_i and W_i (or u1)
    if cls == "leaf_correct":
        return 8.0 * n * (k + s) + 8.0 * n * s        # read Q_i, W_i; write u1
    if cls == "leaf_finalize":
        return 8.0 * n * (k + s) + 16.0 * n * s       # read Q_i, u1; write U_i, U
    if cls == "leaf_hh_panel":
        return 16.0 * n * s                           # read w~, write the s reflectors
    tri = k * (k + 1) / 2.0
    if cls in ("root_gram", "root_gram2"):
        return 8.0 * p * (tri + (k + s) * s)
    if cls == "root_correct":
        return 8.0 * p * (tri + 2.0 * (k + s) * s)
    if cls == "root_finalize":
        return 8.0 * p * (tri + 2.0 * (k + s) * s)
    return 0.0


class TimingEvent:
    """A HIP timing event without the system-scope fence
    (hipEventDisableSystemFence): the default fence writes back and
    invalidates caches when the event is recorded, which slows the work
    around it.  Uses the HIP runtime already loaded in the process."""

    _hip = None

    def __init__(self):
        import ctypes
        if TimingEvent._hip is None:
            TimingEvent._hip = ctypes.CDLL("libamdhip64.so.7")
        self._c = ctypes
        self.ev = ctypes.c_void_p()
        if TimingEvent._hip.hipEventCreateWithFlags(ctypes.byref(self.ev), ctypes.c_uint(0x20000000)):
            raise RuntimeError("hipEventCreateWithFlags failed")

    def record(self, stream):
        if TimingEvent._hip.hipEventRecord(self.ev, self._c.c_void_p(stream.cuda_stream)):
            raise RuntimeError("hipEventRecord failed")

    def elapsed_time(self, end):
        """Milliseconds from this event to `end`; the stream must have been synchronised."""
        ms = self._c.c_float()
        if TimingEvent._hip.hipEventElapsedTime(self._c.byref(ms), self.ev, end.ev):
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def __del__(self):
        # dropped events are destroyed at once (reference counting); at
        # interpreter exit the runtime may already be gone, so leave them
        if TimingEvent._hip is not None and self.ev and not sys.is_finalizing():
            TimingEvent._hip.hipEventDestroy(self.ev)


def source_sha():
    """sha256 over the kernel source and the shared header (launch geometry,
    chunk heights): counters taken on other sources are not used."""
    h = hashlib.sha256()
    for path in (KERNEL_SRC, KERNEL_HDR):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic(kernel_cls):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except Exception:
        return None
    if t.get("kernel_source_sha256") != source_sha():
        return None
    ent = t.get("kernels", {}).get(kernel_cls)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def cpu_baseline(rows_nx=4096, rows_ny=128, s=8, steps=30):
    """The oracle, untuned, on a bounded sample of the same workload."""
    import numpy as np
    from oracle import block_arnoldi, pqr_reference
    from oracle import operators as ops
    from synth import normal_block
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n = rows_nx * rows_ny
    spent = [0.0]
    widths = []

    def timed(Q, X):
        widths.append(Q.shape[1] if Q is not None else 0)
        t0 = time.perf_counter()
        r = pqr_reference(Q, X)
        spent[0] += time.perf_counter() - t0
        return r

    R0 = normal_block(n, s, 0)
    block_arnoldi(lambda X: ops.laplacian_2d_apply(X, rows_nx, rows_ny, 0.0), R0, steps, timed)
    p = max(1, n // 4096)
    total = sum(step_bytes(n, s, p, k) for k in widths)
    return {
        "value": total / spent[0] / 1e9,
        "unit": "GB/s",
        "cores": int(threads),
        "kind": "oracle",
        "seconds": spent[0],
        "sample": (f"2D {rows_nx}x{rows_ny} Laplacian (n = {n}, 1/{(4096 * 4096) // n} of the rows), "
                   f"s = {s}, start block + {steps} block-Arnoldi steps through the oracle's "
                   "unique-PQR reference (BCGS2 + Householder, numpy FP64); operator time "
                   "excluded; same algorithmic-byte formula as the GPU value"),
    }


def batched_workload(count=512, seed=4):
    """Instances of the batched workload: n log-uniform in [2^14, 2^20] as a
    near-square 2D grid, s uniform in {1, 2, 4, 8, 16}, start block + 20 steps."""
    import numpy as np
    rng = np.random.default_rng(seed)
    e = rng.uniform(14, 20, count)
    nx = np.round(2 ** (e / 2)).astype(int)
    ny = np.round(2 ** e / nx).astype(int)
    s = rng.choice([1, 2, 4, 8, 16], count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(nx, ny, s)]


def bench_batched(args):
    """Batched form: all instances advance together, one grouped launch per
    phase; closed-loop Arnoldi with the stencil between steps.  Reports the
    orthogonalisation time (HIP events around every batch step, stencils
    excluded), the same run in the mixed form, the same run replayed from
    one captured hipGraph, and the same instances run one after another
    through single handles."""
    import torch
    from paper_2204_13393_amd import BatchOrthogonalizer, Orthogonalizer, autotune, orth
    inst = batched_workload()
    steps = 20
    ns = [nx * ny for nx, ny, _ in inst]
    ss = [s for _, _, s in inst]
    ks = [(steps + 1) * s for s in ss]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # leaf heights from the autotuner (one measurement per (s, k_max, n rounded
    # to a power of two) bucket), and the library default for comparison
    t0 = time.perf_counter()
    tuned = autotune.tune_batch(ns, ss, ks)
    tune_s = time.perf_counter() - t0
    buckets = len({autotune.bucket_of(n, s, k) for n, s, k in zip(ns, ss, ks)})
    print(f"[bench] batched: autotuned leaf heights in {tune_s:.1f} s ({buckets} buckets)",
          file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    gen = torch.Generator(device="cuda")
    R0 = []
    for i, (n, s) in enumerate(zip(ns, ss)):
        gen.manual_seed(1000 + i)
        R0.append(torch.randn((s, n), dtype=torch.float64, device=dev, generator=gen))
    W = [torch.empty_like(r) for r in R0]
    U = [torch.empty_like(r) for r in R0]
    H = [torch.zeros((k, k), dtype=torch.float64, device=dev) for k in ks]
    print(f"[bench] batched: {len(inst)} instances, sum n = {sum(ns)}", file=sys.stderr, flush=True)

    def stencils():
        for i, (nx, ny, s) in enumerate(inst):
            if orth.orth_laplacian_apply(U[i].data_ptr(), ns[i], W[i].data_ptr(), ns[i], s, nx, ny, 1, 0.0, sp):
                raise RuntimeError("stencil failed")

    def one_run(b, timed, ptrs):
        evs = []
        for j in range(steps + 1):
            if j == 0:
                for i in range(len(ns)):
                    W[i].copy_(R0[i])
            else:
                stencils()
            if timed:
                e0, e1 = TimingEvent(), TimingEvent()
                e0.record(stream)
            b.step(*ptrs)
            if timed:
                e1.record(stream)
                evs.append((e0, e1))
        return evs

    def eager_runs(leaf_rows, precision=orth.ORTH_FP64):
        falls = 0
        with torch.cuda.stream(stream):
            bb = BatchOrthogonalizer(ns, ss, ks, leaf_rows, stream=stream, precision=precision)
            bptrs = (bb.pointer_array(W), bb.pointer_array(U), bb.pointer_array(H))
            base, nbytes = (bb.workspace.data_ptr() + 255) // 256 * 256, bb.workspace.numel() * 8 - 256
            bb.close()
            times = []
            for rep in range(args.warmup + args.steps):
                code, h = orth.orth_batch_create(ns, ss, ks, leaf_rows, precision, base, nbytes, sp)
                if code:
                    raise orth.OrthError("orth_batch_create", code)
                bb.h = h
                evs = one_run(bb, rep >= args.warmup, bptrs)
                stream.synchronize()
                st, info = bb.status()
                if st:
                    raise RuntimeError(f"batched breakdown {info}")
                falls = max(falls, bb.mixed_fallbacks())
                if evs:
                    times.append(sum(e0.elapsed_time(e1) for e0, e1 in evs))
                orth.orth_batch_destroy(h)
                bb.h = None
        bb.fallbacks = falls
        return bb, bptrs, base, nbytes, times

    b, _, _, _, default_runs = eager_runs(None)
    default_leaf = b.leaf_rows
    del b
    torch.cuda.empty_cache()
    with torch.cuda.stream(stream):
        b, ptrs, ws_ptr, ws_bytes, runs = eager_runs(tuned)
        # one hipGraph holding the whole run (stencils + batch steps), and one of the stencils alone
        code, h = orth.orth_batch_create(ns, ss, ks, tuned, orth.ORTH_FP64, ws_ptr, ws_bytes, sp)
        b.h = h
        stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        one_run(b, False, ptrs)
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gs, stream=stream):
        for j in range(steps):
            stencils()
    graph_ms = []
    for rep in range(2):
        orth.orth_batch_destroy(b.h)
        code, h = orth.orth_batch_create(ns, ss, ks, tuned, orth.ORTH_FP64, ws_ptr, ws_bytes, sp)
        b.h = h
        torch.cuda.synchronize()
        e0, e1 = TimingEvent(), TimingEvent()
        with torch.cuda.stream(stream):          # replay on the timed stream
            e0.record(stream)
            g.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        t_all = e0.elapsed_time(e1)
        with torch.cuda.stream(stream):
            e0.record(stream)
            gs.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        graph_ms.append(t_all - e0.elapsed_time(e1))
    st, info = b.status()
    if st:
        raise RuntimeError(f"graph replay breakdown {info}")
    orth.orth_batch_destroy(b.h)
    b.h = None
    leaf = b.leaf_rows
    del b, g, gs
    torch.cuda.empty_cache()

    # the mixed form (FP32 copies of the leaf bases read by the first leaf
    # Gram) on the same instances and leaf heights
    print("[bench] batched mixed form", file=sys.stderr, flush=True)
    bm, _, _, _, mixed_runs = eager_runs(tuned, orth.ORTH_MIXED_SPLIT32)
    mixed_falls = bm.fallbacks
    del bm
    torch.cuda.empty_cache()

    # the same instances through single handles, one after another
    print("[bench] single handles, sequential", file=sys.stderr, flush=True)
    single = []
    torch.cuda.synchronize()
    t_single = 0.0
    for i, (nx, ny, s) in enumerate(inst):
        with torch.cuda.stream(stream):
            o = Orthogonalizer(ns[i], s, ks[i], tuned[i], stream=stream)
            Wi, Ui = W[i], U[i]
            Wi.copy_(R0[i])
            e0, e1 = TimingEvent(), TimingEvent()
            tot = 0.0
            for j in range(steps + 1):
                if j:
                    orth.orth_laplacian_apply(Ui.data_ptr(), ns[i], Wi.data_ptr(), ns[i], s, nx, ny, 1, 0.0, sp)
                e0.record(stream)
                o.step(Wi, U=Ui)
                e1.record(stream)
                stream.synchronize()
                tot += e0.elapsed_time(e1)
            t_single += tot
            o.close()
            del o
    p_of = lambda n, lr: max(1, n // lr)
    total_bytes = 0.0
    for (n, s, lr) in zip(ns, ss, leaf):
        for j in range(steps + 1):
            total_bytes += step_bytes(n, s, p_of(n, lr), j * s)
    best = min(runs)
    hist = {}
    for lr in leaf:
        hist[str(lr)] = hist.get(str(lr), 0) + 1
    out = {
        "metric": METRIC,
        "workload": "batched-512-lap2d",
        "value": total_bytes / (best / 1e3) / 1e9,
        "unit": "GB/s",
        "ms_per_run_batched": best,
        "ms_per_run_batched_default_leaf": min(default_runs),
        "leaf_rows": {"source": "autotuned", "tuning_s": tune_s, "buckets": buckets, "histogram": hist,
                      "default_histogram": {str(v): default_leaf.count(v) for v in sorted(set(default_leaf))}},
        "ms_per_run_batched_mixed": min(mixed_runs),
        "mixed_speedup": best / min(mixed_runs),
        "mixed_fallbacks": mixed_falls,
        "ms_per_run_graph": min(graph_ms),
        "graph_note": "one hipGraph of the whole run minus a graph of its stencils alone",
        "ms_per_run_single_sequential": t_single,
        "speedup_vs_single": t_single / best,
        "instances": len(inst),
        "steps": steps,
        "sum_n": sum(ns),
        "alg_bytes_per_run": total_bytes,
        "dtype": "f64",
        "data": "synthetic: per-instance seeded N(0,1) start blocks on the GPU, 2D Dirichlet Laplacians",
    }
    print(json.dumps(out), flush=True)


def bench_c1(args):
    """Small plain-FP64 block Arnoldi (latency): 2D 5-point Dirichlet Laplacian
    on 100 x 100 (n = 10,000) shifted by 0.01 I, start block
    default_rng(0).standard_normal((10000, 4)), s = 4, start block + 10 block
    steps (k up to 40), leaf height 1000 (10 leaves).  Closed loop with the
    library's stencil between steps.  Reports microseconds per orth_step:
    eager (HIP events around each call, and host wall time of the call
    itself), and the whole closed loop captured once in a hipGraph and
    replayed (per step, stencil included; a graph of the stencils alone is
    timed beside it).  Median and min over 5 sequences (args.steps if
    larger)."""
    import numpy as np
    import torch
    from paper_2204_13393_amd import orth
    nx = ny = 100
    n, s, steps, leaf, shift = nx * ny, 4, 10, 1000, 0.01
    kmax = (steps + 1) * s
    runs = max(5, args.steps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    side = torch.cuda.Stream()
    sp = side.cuda_stream
    R0 = torch.from_numpy(np.ascontiguousarray(np.random.default_rng(0).standard_normal((n, s)).T)).to(dev)
    V = torch.empty((kmax, n), dtype=torch.float64, device=dev)
    W = torch.empty((s, n), dtype=torch.float64, device=dev)
    H = torch.zeros((kmax, kmax), dtype=torch.float64, device=dev)
    nbytes = orth.orth_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64)
    ws = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=dev)
    wp = (ws.data_ptr() + 255) // 256 * 256

    def create():
        code, h = orth.orth_create(n, s, kmax, leaf, orth.ORTH_FP64, wp, nbytes, sp)
        if code:
            raise orth.OrthError("orth_create", code)
        return h

    def stencil(j):
        if j == 0:
            W.copy_(R0)
        elif orth.orth_laplacian_apply(V[(j - 1) * s:j * s].data_ptr(), n, W.data_ptr(), n, s, nx, ny, 1,
                                       shift, sp):
            raise RuntimeError("stencil failed")

    def step(h, j):
        k = j * s
        col = H[j * s:(j + 1) * s]
        code = orth.orth_step(h, W.data_ptr(), n, col.data_ptr() if k else 0, kmax, col[:, k:].data_ptr(),
                              kmax, V[k:k + s].data_ptr(), n)
        if code:
            raise orth.OrthError("orth_step", code)

    def eager():
        h = create()
        ev, host_us = [], []
        with torch.cuda.stream(side):
            for j in range(steps + 1):
                stencil(j)
                e0, e1 = TimingEvent(), TimingEvent()
                e0.record(side)
                t0 = time.perf_counter()
                step(h, j)
                host_us.append((time.perf_counter() - t0) * 1e6)
                e1.record(side)
                ev.append((e0, e1))
        side.synchronize()
        code, st, info = orth.orth_status(h)
        orth.orth_destroy(h)
        if st:
            raise RuntimeError(f"breakdown {info}")
        return [a.elapsed_time(b) * 1e3 for a, b in ev], host_us

    for _ in range(max(1, args.warmup)):
        eager()
    dev_us, host_us = [], []
    for _ in range(runs):
        d, hst = eager()
        dev_us.append(float(np.mean(d)))
        host_us.append(float(np.mean(hst)))
    G = torch.mm(V, V.t()) - torch.eye(kmax, dtype=torch.float64, device=dev)
    e_perp = float(torch.linalg.matrix_norm(G, "fro"))

    # the closed loop captured once (its launches carry their own k) and replayed
    def capture(with_orth):
        h = create()
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for j in range(steps + 1):
                stencil(j)
                if with_orth:
                    step(h, j)
        return g, h

    out_graph = {}
    for name, with_orth in (("closed_loop", True), ("stencils_only", False)):
        g, h = capture(with_orth)
        times = []
        for r in range(runs + 1):
            e0, e1 = TimingEvent(), TimingEvent()
            e0.record(side)
            with torch.cuda.stream(side):
                g.replay()
            e1.record(side)
            side.synchronize()
            if r:
                times.append(e0.elapsed_time(e1) * 1e3 / (steps + 1))
        orth.orth_destroy(h)
        out_graph[name] = {"median_us_per_step": float(np.median(times)), "min_us_per_step": float(min(times))}
    out = {
        "metric": METRIC,
        "workload": "lap2d-100x100-s4",
        "unit": "us per orth_step",
        "orth_calls": steps + 1,
        "eager": {"median_us_per_step": float(np.median(dev_us)), "min_us_per_step": float(min(dev_us)),
                  "host_call_us_median": float(np.median(host_us))},
        "graph": {
            **out_graph,
            "orth_us_per_step_median": out_graph["closed_loop"]["median_us_per_step"]
            - out_graph["stencils_only"]["median_us_per_step"],
        },
        "algorithmic_floor_us": step_bytes(n, s, n // leaf, kmax - s) / (HBM_PEAK_GBS * 1e3),
        "e_perp": e_perp,
        "runs": runs,
        "dtype": "f64",
        "data": "synthetic: default_rng(0) N(0,1) start block, 2D Dirichlet Laplacian 100x100 + 0.01 I",
    }
    print(json.dumps(out), flush=True)


def bench_lap3d(args):
    """Large block: 3D 7-point Laplacian on 256^3 (n = 2^24), s = 32, start
    block + 16 block-Arnoldi steps (k up to 512), leaf height 4096.  The
    start block is W0 = G M with singular values sigma_j = 10^(-8 j / 31)
    (G Gaussian from default_rng(5), M = R_G^{-1} diag(sigma) V^T, V the QR
    factor of a Gaussian from default_rng(6); kappa = 1e8, eps kappa^2 ~ 1.1).
    FP64 and mixed forms on that block (the timed line), FP64 from an N(0,1)
    start block (default_rng(5)) as a second, labelled line, and the
    Householder leaves on the configured block.  Closed
    loop; HIP events around every orth_step (stencils excluded)."""
    import numpy as np
    import torch
    from paper_2204_13393_amd import orth
    from synth import normal_block
    nx = ny = nz = 256
    n, s, steps, leaf = nx * ny * nz, 32, 16, 4096
    kmax = (steps + 1) * s
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    if args.tune_tiles:
        # (before the bench's own buffers: the tuner holds a workspace of its own)
        from paper_2204_13393_amd import autotune
        t0 = time.perf_counter()
        best_t, cand_t = autotune.measure_tiles(n, s, kmax, leaf, steps=kmax // s)
        tune_s = time.perf_counter() - t0
        torch.cuda.empty_cache()
        print(f"[bench] lap3d: tile tuner picked {best_t} in {tune_s:.1f} s", file=sys.stderr, flush=True)
    print("[bench] lap3d: generating the start blocks", file=sys.stderr, flush=True)
    R0_normal = torch.from_numpy(np.ascontiguousarray(normal_block(n, s, 5).T)).to(dev)
    # the configured start block: sigma_j = 10^(-8 j / 31)
    rng = np.random.default_rng(5)
    Gm = rng.standard_normal((n, s))
    Rg = np.linalg.cholesky(Gm.T @ Gm).T
    Vh = np.linalg.qr(np.random.default_rng(6).standard_normal((s, s)))[0]
    sig = 10.0 ** (-8.0 * np.arange(s) / (s - 1))
    M = np.linalg.solve(Rg, np.diag(sig) @ Vh.T)
    R0_sigma = torch.from_numpy(np.ascontiguousarray((Gm @ M).T)).to(dev)
    del Gm
    start = {"sigma": R0_sigma, "normal": R0_normal}
    V = torch.empty((kmax, n), dtype=torch.float64, device=dev)
    W = torch.empty((s, n), dtype=torch.float64, device=dev)
    H = torch.zeros((kmax, kmax), dtype=torch.float64, device=dev)
    # one workspace for every form (the mixed form adds the FP32 copy, the
    # Householder form the per-leaf compact-WY factors)
    nbytes = max(orth.orth_workspace_bytes(n, s, kmax, leaf, p_)
                 for p_ in (orth.ORTH_MIXED_SPLIT32, orth.ORTH_FP64_HOUSEHOLDER))
    ws = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256

    fallbacks = {}      # steps whose first sweep was redone in FP64, per form

    def run(profiled, precision=orth.ORTH_FP64, block="sigma", tiles=None):
        R0 = start[block]
        code, h = orth.orth_create_tiles(n, s, kmax, leaf, precision, 0, tiles, ws_ptr, nbytes, sp)
        if code:
            raise orth.OrthError("orth_create", code)
        if profiled:
            orth.orth_profile_enable(h, 1)
        ms = 0.0
        for j in range(steps + 1):
            k = j * s
            if j == 0:
                W.copy_(R0)
            elif orth.orth_laplacian_apply(V[k - s:k].data_ptr(), n, W.data_ptr(), n, s, nx, ny, nz, 0.0, sp):
                raise RuntimeError("stencil failed")
            col = H[j * s:(j + 1) * s]
            e0, e1 = TimingEvent(), TimingEvent()
            e0.record(stream)
            code = orth.orth_step(h, W.data_ptr(), n, col.data_ptr(), kmax, col[:, k:].data_ptr(), kmax,
                                  V[k:k + s].data_ptr(), n)
            e1.record(stream)
            if code:
                raise orth.OrthError("orth_step", code)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
        code, st, info = orth.orth_status(h)
        prof = orth.orth_profile_read(h)[1] if profiled else None
        fallbacks[precision] = fallbacks.get(precision, 0) + orth.orth_mixed_fallbacks(h)[1]
        orth.orth_destroy(h)
        if st:
            raise RuntimeError(f"breakdown {info}")
        return ms, prof

    def timed(precision, block="sigma", profile=True, tiles=None):
        """Warmup, args.steps unprofiled runs (the time), then one run with
        every launch bracketed by events (the per-class breakdown)."""
        for _ in range(args.warmup):
            run(False, precision, block, tiles)
        times = []
        for _ in range(args.steps):
            ms, _ = run(False, precision, block, tiles)
            times.append(ms)
        G = torch.mm(V, V.t())
        G -= torch.eye(kmax, dtype=torch.float64, device=dev)
        ep = float(torch.linalg.matrix_norm(G, "fro"))
        del G
        pr = run(True, precision, block)[1] if profile else None
        return min(times), pr, ep

    best, prof, e_perp = timed(orth.ORTH_FP64)
    best_mixed, prof_mixed, e_perp_mixed = timed(orth.ORTH_MIXED_SPLIT32)
    best_normal, _, e_perp_normal = timed(orth.ORTH_FP64, "normal", profile=False)
    print("[bench] lap3d: householder leaves", file=sys.stderr, flush=True)
    best_hh, prof_hh, e_perp_hh = timed(orth.ORTH_FP64_HOUSEHOLDER)
    tiles = None
    if args.tune_tiles:
        if orth.orth_tiles_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64, 0, best_t) > nbytes:
            raise RuntimeError("the pick needs a larger workspace than the bench holds")
        ms_t, _, ep_t = timed(orth.ORTH_FP64, profile=False, tiles=best_t)
        tiles = {"pick": list(best_t), "tuning_s": tune_s,
                 "candidates_ms": {str(tuple(c)): m for c, m in cand_t},
                 "ms_per_sequence_pick": ms_t, "pick_vs_plan": ms_t / best, "e_perp": ep_t}
        print(f"[bench] lap3d tiles {best_t}: {ms_t:.2f} ms against {best:.2f} ms (tuned in {tune_s:.1f} s)",
              file=sys.stderr, flush=True)
    p = n // leaf
    widths = [j * s for j in range(steps + 1)]
    total_bytes = sum(step_bytes(n, s, p, k) for k in widths)
    total_flops = sum((10.0 * s * k + 14.0 * s * s) * n for k in widths)
    kernels = {name: {"ms_total": ms, "launches": cnt, "avg_us": ms / cnt * 1e3}
               for name, (ms, cnt) in prof.items() if cnt}
    out = {
        "metric": METRIC,
        "workload": "lap3d-256-s32",
        "value": total_bytes / (best / 1e3) / 1e9,
        "unit": "GB/s",
        "ms_per_sequence": best,
        "tflops_paper_count": total_flops / (best / 1e3) / 1e12,
        "orth_calls": len(widths),
        "e_perp": e_perp,
        "kernels": kernels,
        "mixed": {
            "precision": "mixed_split32: leaf bases FP32 copy for the sweep-1 Gram, FP64 arithmetic",
            "ms_per_sequence": best_mixed,
            "value_effective": total_bytes / (best_mixed / 1e3) / 1e9,
            "speedup_vs_fp64": best / best_mixed,
            "e_perp": e_perp_mixed,
            "fp64_redo_steps": fallbacks[orth.ORTH_MIXED_SPLIT32],
            "kernels": {name: {"ms_total": ms, "launches": cnt, "avg_us": ms / cnt * 1e3}
                        for name, (ms, cnt) in prof_mixed.items() if cnt},
        },
        "householder": {
            "precision": "fp64_householder: Algorithm HH at the leaves (s = 32 in 8-column sub-panels), "
                         "BCGS-PIP+ reduction",
            "ms_per_sequence": best_hh,
            "speedup_vs_fp64": best / best_hh,
            "e_perp": e_perp_hh,
            "kernels": {name: {"ms_total": ms, "launches": cnt, "avg_us": ms / cnt * 1e3}
                        for name, (ms, cnt) in prof_hh.items() if cnt},
        },
        "tile_tuner": tiles,
        "normal_start_block": {
            "start": "N(0,1), default_rng(5)",
            "ms_per_sequence": best_normal,
            "value": total_bytes / (best_normal / 1e3) / 1e9,
            "e_perp": e_perp_normal,
        },
        "dtype": "f64",
        "data": "synthetic: start block with singular values 10^(-8j/31) (kappa 1e8; G from default_rng(5), "
                "V from default_rng(6)), 3D Dirichlet Laplacian 256^3",
    }
    print(json.dumps(out), flush=True)


def bench_kappa_sweep(args):
    """Subalgorithm sweep (Sec. 6.1, the kappa sweep and the local x reduction
    combinations): QR of Stewart matrices X = U diag(sigma) V^T,
    sigma_j = kappa^(-j/31), n = 2^16, 32 columns in blocks of s = 4 (eight
    orth_step calls), leaves of 256 rows, for kappa = 10^0 .. 10^12 and the
    four combinations of BCGS-PIP / BCGS-PIP+ at the leaves and at the
    reduction, plus Householder leaves (Sec. 2.2) with either reduction, a
    Householder reduction with each kind of leaves (the full local x
    reduction map), and Householder leaves with a deflating BCGS-PIP+
    reduction (Sec. 3.1,
    delta = 1e-6).  Per case: status (breakdown or not) and e_perp of the
    explicit basis (of its kept columns, with the count dropped, for the
    deflating case).  The matrices come from synth.stewart (seed 11)."""
    import numpy as np
    import torch
    from paper_2204_13393_amd import Orthogonalizer, orth
    from synth import stewart
    n, m, s, leaf = 1 << 16, 32, 4, 256
    v = {"pip+": orth.ORTH_PIP_PLUS, "pip": orth.ORTH_PIP, "hh": orth.ORTH_HOUSEHOLDER}
    combos = [("pip+", "pip+"), ("pip+", "pip"), ("pip", "pip+"), ("pip", "pip"), ("hh", "pip+"), ("hh", "pip"),
              ("pip+", "hh"), ("pip", "hh"), ("hh", "hh"), ("hh", "pip+/deflation")]
    rows = []
    print("[bench] kappa sweep: Stewart n = 2^16, 32 columns, s = 4, leaves of 256 rows", file=sys.stderr, flush=True)
    for e in range(13):
        kappa = 10.0 ** e
        A = stewart(n, m, kappa, 11)
        At = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")
        row = {"kappa": kappa}
        for local, red in combos:
            defl = red.endswith("/deflation")
            if local == "hh":
                g = Orthogonalizer(n, s, m, leaf, precision=orth.ORTH_FP64_HOUSEHOLDER,
                                   reduction_variant=v[red.split("/")[0]])
                if defl:
                    g.set_deflation(DEFL_DELTA)
            else:
                g = Orthogonalizer(n, s, m, leaf, variant=v[local], reduction_variant=v[red])
            blocks = []
            for j in range(m // s):
                blocks.append(g.step(At[j * s:(j + 1) * s].contiguous())[2].clone())
                if g.status()[0]:
                    break
            st, info = g.status()
            if st == 0:
                # e_perp on the host (FP64 BLAS): a 32 x 32 Gram of 2^16 rows of
                # the explicit blocks U the calls returned
                Q = torch.cat(blocks).cpu().numpy()
                if defl:
                    keep = np.linalg.norm(Q, axis=1) > 0.5          # dropped columns are zero
                    Qk = Q[keep]
                    row[f"{local}/{red}"] = {"e_perp": float(np.linalg.norm(Qk @ Qk.T - np.eye(len(Qk)), "fro")),
                                             "dropped": int(m - keep.sum())}
                else:
                    row[f"{local}/{red}"] = float(np.linalg.norm(Q @ Q.T - np.eye(m), "fro"))
            else:
                row[f"{local}/{red}"] = {"breakdown": {"level": info[0], "sweep": info[2], "column": info[3]}}
            g.close()
        rows.append(row)
        print(f"[bench] kappa 1e{e}: " + ", ".join(f"{c}: {row[c] if isinstance(row[c], dict) else f'{row[c]:.2e}'}"
                                                  for c in row if c != "kappa"), file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "workload": "subalgorithm-sweep-stewart-2^16x32-s4",
        "results": rows,
        "columns": "local/reduction subalgorithm; value = e_perp of the explicit Q, or the breakdown record",
        "dtype": "f64",
        "data": "synthetic: Stewart matrices from synth.stewart(2^16, 32, kappa, 11)",
    }
    print(json.dumps(out), flush=True)


def bench_stewart(args):
    """Precision workload: block-column QR (Sec. 2, the block-column QR
    algorithm) of one n x 240 matrix W = G diag(sigma) V^T with n = 2^24,
    s = 8 (30 calls), leaf height 4096; sigma log-spaced from 1 to 1e-6 and
    from 1 to 1e-12 (kappa 1e6 and 1e12); V Haar (QR of a Gaussian), G
    Gaussian / sqrt(n), orthonormal to about 2 sqrt(240/n) = 0.008 at this n, so
    the singular values of W are sigma to within 1%.  FP64, mixed and
    Householder-leaf forms, and the Householder leaves with deflation at the
    reduction level (Sec. 3.1, delta = 1e-6): a call drops the directions
    whose residual singular value is below delta ||W_j||_F, so the kappa =
    1e12 run goes on where the other forms break down, with a smaller basis.
    Per form and range: status (and the call after which a breakdown was
    reported), the calls in which the mixed form redid its first sweep in
    FP64, time of the calls (HIP events around each), e_perp of the explicit Q
    and ||W - Q R||_F / ||W||_F."""
    import math
    import torch
    from paper_2204_13393_amd import Orthogonalizer, orth
    n, m, s, leaf = 1 << 24, 240, 8, 4096
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    print("[bench] stewart: generating W (n = 2^24, 240 columns)", file=sys.stderr, flush=True)
    Gt = torch.randn((m, n), dtype=torch.float64, device=dev, generator=gen)
    Gt /= math.sqrt(n)
    Vh, _ = torch.linalg.qr(torch.randn((m, m), dtype=torch.float64, device=dev, generator=gen))
    Qt = torch.empty((m, n), dtype=torch.float64, device=dev)          # explicit Q, column-major n x m
    Rt = torch.zeros((m, m), dtype=torch.float64, device=dev)          # R, column-major m x m
    forms = (("fp64", orth.ORTH_FP64), ("mixed", orth.ORTH_MIXED_SPLIT32),
             ("householder", orth.ORTH_FP64_HOUSEHOLDER),
             ("householder+deflation", orth.ORTH_FP64_HOUSEHOLDER))
    nbytes = max(orth.orth_workspace_bytes(n, s, m, leaf, f) for _, f in forms)
    wsbuf = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=dev)
    ws_ptr = (wsbuf.data_ptr() + 255) // 256 * 256
    results = []
    for smin in (1e-6, 1e-12):
        sig = torch.logspace(0.0, math.log10(smin), m, dtype=torch.float64, device=dev)
        Wt = torch.mm(Vh * sig, Gt)            # W^T = V diag(sigma) G^T
        wnorm = float(torch.linalg.norm(Wt))
        for name, prec in forms:
            for rep in range(args.warmup + 1):
                Rt.zero_()
                code, h = orth.orth_create(n, s, m, leaf, prec, ws_ptr, nbytes, sp)
                if code:
                    raise orth.OrthError("orth_create", code)
                if name.endswith("deflation"):
                    code = orth.orth_set_deflation(h, DEFL_DELTA)
                    if code:
                        raise orth.OrthError("orth_set_deflation", code)
                ms, failed = 0.0, None
                for j in range(m // s):
                    k = j * s
                    col = Rt[k:k + s]
                    e0, e1 = TimingEvent(), TimingEvent()
                    e0.record(stream)
                    code = orth.orth_step(h, Wt[k:k + s].data_ptr(), n, col.data_ptr(), m,
                                          col[:, k:].data_ptr(), m, Qt[k:k + s].data_ptr(), n)
                    e1.record(stream)
                    if code:
                        raise orth.OrthError("orth_step", code)
                    code, st, info = orth.orth_status(h)
                    if st:
                        failed = {"call": j, "info": info}
                        break
                    ms += e0.elapsed_time(e1)
                code, nfall = orth.orth_mixed_fallbacks(h)
                _, _, dsteps, dcols = orth.orth_deflation_info(h)
                orth.orth_destroy(h)
            row = {"form": name, "sigma_min": smin, "status": "breakdown" if failed else "ok",
                   "breakdown": failed, "fallback_steps": nfall}
            if name.endswith("deflation"):
                row.update({"delta": DEFL_DELTA, "deflated_calls": dsteps, "columns_dropped": dcols})
            if not failed:
                # e_perp over the kept columns (a dropped column of Q is exactly zero)
                keep = torch.linalg.vector_norm(Qt, dim=1) > 0.5
                Qk = Qt[keep]
                row["columns_kept"] = int(Qk.shape[0])
                Gq = torch.mm(Qk, Qk.t())
                Gq -= torch.eye(Qk.shape[0], dtype=torch.float64, device=dev)
                del Qk
                row["e_perp"] = float(torch.linalg.matrix_norm(Gq, "fro"))
                del Gq
                res2 = 0.0
                for c0 in range(0, n, 1 << 21):       # ||W^T - R^T Q^T|| in column chunks
                    D = Wt[:, c0:c0 + (1 << 21)] - torch.mm(Rt, Qt[:, c0:c0 + (1 << 21)])
                    res2 += float(torch.sum(D * D))
                    del D
                row["residual"] = math.sqrt(res2) / wnorm
                row["ms_30_calls"] = ms
                row["e_perp_gate_1e-10"] = row["e_perp"] <= 1e-10
            print(f"[bench] stewart {name} sigma_min {smin}: {row['status']}", file=sys.stderr, flush=True)
            results.append(row)
        del Wt
    fp = {r["sigma_min"]: r for r in results if r["form"] == "fp64"}
    mx = {r["sigma_min"]: r for r in results if r["form"] == "mixed"}
    speed = {str(k): fp[k]["ms_30_calls"] / mx[k]["ms_30_calls"]
             for k in fp if fp[k]["status"] == "ok" and mx[k]["status"] == "ok"}
    hx = {r["sigma_min"]: r for r in results if r["form"] == "householder"}
    hd = {r["sigma_min"]: r for r in results if r["form"] == "householder+deflation"}
    speed_hh = {str(k): fp[k]["ms_30_calls"] / hx[k]["ms_30_calls"]
                for k in fp if fp[k]["status"] == "ok" and hx[k]["status"] == "ok"}
    out = {
        "metric": METRIC,
        "workload": "stewart-2^24x240-s8",
        "results": results,
        "mixed_speedup_vs_fp64": speed,
        "householder_speedup_vs_fp64": speed_hh,
        "deflation_overhead_vs_householder": {str(k): hd[k]["ms_30_calls"] / hx[k]["ms_30_calls"]
                                              for k in hx if hx[k]["status"] == "ok" and hd[k]["status"] == "ok"},
        "dtype": "f64",
        "data": "synthetic: W = G diag(sigma) V^T, G Gaussian/sqrt(n), V Haar (torch, seed 7)",
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel HIP-event timing")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="after timing, run one plain copy of this many GiB (counter calibration)")
    ap.add_argument("--tree-fan-ins", default="",
                    help="default workload: also time the FP64 sequence with reduction trees of these "
                         "fan-ins (comma-separated)")
    ap.add_argument("--flat-blocks", default="",
                    help="default workload: also time the FP64 sequence with FlatTSPQR over this many "
                         "row blocks (comma-separated counts)")
    ap.add_argument("--tune-tiles", action="store_true",
                    help="default and lap3d workloads: run the tile tuner (orth_tune_tiles) at the shape and "
                         "time the FP64 sequence with its pick")
    ap.add_argument("--householder-tree", type=int, default=0,
                    help="default workload: also time Householder at every level (Householder leaves and a "
                         "Householder reduction tree of this fan-in)")
    ap.add_argument("--workload", default="lap2d-4096x4096-s8",
                    choices=["lap2d-4096x4096-s8", "batched", "lap3d-256-s32", "stewart", "kappa-sweep",
                             "lap2d-100x100-s4"],
                    help="the default single-basis run, the batched form (512 instances), "
                         "the large-block 3D run, the precision workload (Stewart matrices), "
                         "the subalgorithm sweep, or the small latency run (C1)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on exactly one GPU (one MI355X); "
              "sharding the basis across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "lap2d-100x100-s4":
        return bench_c1(args)
    if args.workload == "lap3d-256-s32":
        return bench_lap3d(args)
    if args.workload == "kappa-sweep":
        return bench_kappa_sweep(args)
    if args.workload == "stewart":
        return bench_stewart(args)

    import numpy as np
    import torch
    from paper_2204_13393_amd import orth, laplacian_apply
    from synth import normal_block

    orth.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = WORKLOAD
    nx, ny, s, steps, leaf = W["nx"], W["ny"], W["s"], W["steps"], W["leaf_rows"]
    n = nx * ny
    kmax = (steps + 1) * s
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    print(f"[bench] generating inputs: n={n} s={s} steps={steps}", file=sys.stderr, flush=True)
    # --- inputs: start block + 30 Krylov blocks, resident in HBM
    R0 = torch.from_numpy(np.ascontiguousarray(normal_block(n, s, W["seed"]).T)).to(dev)
    # one workspace for both forms (the mixed form's is the larger: it adds the FP32 copy)
    # (and the Householder form, when this shape is within its limits, adds the T factors)
    nbytes = max(orth.orth_workspace_bytes(n, s, kmax, leaf, p_)
                 for p_ in (orth.ORTH_FP64, orth.ORTH_MIXED_SPLIT32, orth.ORTH_FP64_HOUSEHOLDER))
    hh_ok = orth.orth_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64_HOUSEHOLDER) > 0
    ws = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    Xs = [R0]
    V = torch.empty((kmax, n), dtype=torch.float64, device=dev)          # explicit U blocks
    Hm = torch.zeros((steps * s, kmax), dtype=torch.float64, device=dev)  # column-major K x 30s
    R0out = torch.empty((s, s), dtype=torch.float64, device=dev)

    def run_sequence(blocks, h):
        for j, X in enumerate(blocks):
            k = j * s
            U = V[k:k + s]
            if j == 0:
                code = orth.orth_step(h, X.data_ptr(), n, 0, 1, R0out.data_ptr(), s, U.data_ptr(), n)
            else:
                col = Hm[(j - 1) * s:j * s]
                code = orth.orth_step(h, X.data_ptr(), n, col.data_ptr(), kmax,
                                      col[:, k:].data_ptr(), kmax, U.data_ptr(), n)
            if code:
                raise orth.OrthError("orth_step", code)

    defl_delta = [0.0]      # > 0: Householder handles deflate at the reduction level

    def make_handle(precision=orth.ORTH_FP64):
        code, h = orth.orth_create(n, s, kmax, leaf, precision, ws_ptr, nbytes, sptr)
        if code:
            raise orth.OrthError("orth_create", code)
        if defl_delta[0] > 0.0:
            code = orth.orth_set_deflation(h, defl_delta[0])
            if code:
                raise orth.OrthError("orth_set_deflation", code)
        return h

    # closed-loop Arnoldi once, to produce the Krylov blocks (not timed)
    h = make_handle()
    for j in range(steps + 1):
        k = j * s
        U = V[k:k + s]
        if j == 0:
            code = orth.orth_step(h, Xs[0].data_ptr(), n, 0, 1, R0out.data_ptr(), s, U.data_ptr(), n)
        else:
            col = Hm[(j - 1) * s:j * s]
            code = orth.orth_step(h, Xs[j].data_ptr(), n, col.data_ptr(), kmax,
                                  col[:, k:].data_ptr(), kmax, U.data_ptr(), n)
        if code:
            raise orth.OrthError("orth_step", code)
        if j < steps:
            Xs.append(laplacian_apply(U, (nx, ny), 0.0))
    code, st, info = orth.orth_status(h)
    if code or st:
        raise RuntimeError(f"Arnoldi input generation failed: status {st} info {info}")
    orth.orth_destroy(h)
    torch.cuda.synchronize()
    print("[bench] inputs ready", file=sys.stderr, flush=True)

    p = max(1, n // leaf)
    widths = [j * s for j in range(steps + 1)]

    def profiled_sequence(precision):
        """One untimed sequence with every launch bracketed by events: the
        per-class breakdown, and the dominant class for the timed region."""
        h = make_handle(precision)
        orth.orth_profile_enable(h, 1)
        run_sequence(Xs, h)
        code, pr = orth.orth_profile_read(h)
        orth.orth_destroy(h)
        if code:
            raise orth.OrthError("orth_profile_read", code)
        with_bytes = [c for c, (ms, cnt) in pr.items() if cnt and kernel_bytes(c, n, s, p, 8) > 0]
        return pr, max(with_bytes, key=lambda c: pr[c][0])

    fallbacks = {}      # steps whose first sweep was redone in FP64, per form
    drops = {}          # columns dropped by deflation, per form

    def timed_runs(precision, dom):
        """Warmup, then args.steps timed sequences over the resident inputs,
        events around the launches of class `dom` only; returns (ms per
        sequence, (ms, launches) of `dom`, e_perp of the explicit basis)."""
        for _ in range(args.warmup):
            h = make_handle(precision)
            run_sequence(Xs, h)
            orth.orth_destroy(h)
        torch.cuda.synchronize()
        handles = []
        ev0 = TimingEvent()
        ev1 = TimingEvent()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            h = make_handle(precision)
            if dom is not None:
                orth.orth_profile_select(h, 1 << orth.KERNEL_CLASSES.index(dom))
                orth.orth_profile_enable(h, 1)
            run_sequence(Xs, h)
            handles.append(h)
        ev1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        wall_ms = (t1 - t0) * 1e3 / args.steps
        gpu_ms = ev0.elapsed_time(ev1) / args.steps
        dom_ms, dom_n = 0.0, 0
        fallbacks[precision] = 0
        drops[precision] = 0
        for h in handles:
            code, st, info = orth.orth_status(h)
            if code or st:
                raise RuntimeError(f"orth_step breakdown: {info}")
            fallbacks[precision] += orth.orth_mixed_fallbacks(h)[1]
            drops[precision] += orth.orth_deflation_info(h)[3]
            if dom is not None:
                code, pr = orth.orth_profile_read(h)
                dom_ms += pr[dom][0]
                dom_n += pr[dom][1]
            orth.orth_destroy(h)
        # accuracy gate: e_perp of the explicit basis (torch GEMM, independent of the kernels)
        G = torch.mm(V, V.t())
        G -= torch.eye(kmax, dtype=torch.float64, device=dev)
        ep = float(torch.linalg.matrix_norm(G, "fro"))
        del G
        return max(wall_ms, gpu_ms), (dom_ms, dom_n), ep

    prof, dom = (None, None) if args.no_profile else profiled_sequence(orth.ORTH_FP64)
    prof_mixed, dom_mixed = (None, None) if args.no_profile else profiled_sequence(orth.ORTH_MIXED_SPLIT32)
    ms_per_step, dom_timed, e_perp = timed_runs(orth.ORTH_FP64, dom)
    print(f"[bench] timed {args.steps} sequences: {ms_per_step:.2f} ms each", file=sys.stderr, flush=True)
    # the mixed form (FP64 leaf bases plus an FP32 copy read by the sweep-1 Gram) on the same inputs
    ms_mixed, dom_mixed_timed, e_perp_mixed = timed_runs(orth.ORTH_MIXED_SPLIT32, dom_mixed)
    print(f"[bench] mixed form: {ms_mixed:.2f} ms per sequence, e_perp {e_perp_mixed:.2e}",
          file=sys.stderr, flush=True)
    # the Householder leaves (Algorithm HH at the leaves, BCGS-PIP+ reduction) on the same inputs
    hh = None
    if hh_ok:
        prof_hh, dom_hh = (None, None) if args.no_profile else profiled_sequence(orth.ORTH_FP64_HOUSEHOLDER)
        ms_hh, _, e_perp_hh = timed_runs(orth.ORTH_FP64_HOUSEHOLDER, dom_hh)
        print(f"[bench] householder leaves: {ms_hh:.2f} ms per sequence, e_perp {e_perp_hh:.2e}",
              file=sys.stderr, flush=True)
        hh = (ms_hh, e_perp_hh, prof_hh)
        # the same with deflation switched on (Sec. 3.1): the reduction level's
        # first sweep takes the Jacobi eigen decomposition in place of the
        # Cholesky factorisation; these full-rank blocks drop nothing
        defl_delta[0] = DEFL_DELTA
        prof_hd = None if args.no_profile else profiled_sequence(orth.ORTH_FP64_HOUSEHOLDER)[0]
        ms_hd, _, e_perp_hd = timed_runs(orth.ORTH_FP64_HOUSEHOLDER, None)
        defl_delta[0] = 0.0
        print(f"[bench] householder leaves with deflation: {ms_hd:.2f} ms per sequence, "
              f"{drops[orth.ORTH_FP64_HOUSEHOLDER]} columns dropped", file=sys.stderr, flush=True)
        hh_defl = (ms_hd, e_perp_hd, prof_hd, drops[orth.ORTH_FP64_HOUSEHOLDER])

    total_bytes = sum(step_bytes(n, s, p, k) for k in widths)
    value = total_bytes / (ms_per_step / 1e3) / 1e9

    def per_class(pr, first_step_skips=()):
        out = {}
        for name, (ms, cnt) in pr.items():
            if cnt == 0:
                continue
            ks = widths[1:] if name in first_step_skips else widths
            byts = sum(kernel_bytes(name, n, s, p, k) for k in ks)
            out[name] = {"ms_total": ms, "launches": cnt, "avg_us": ms / cnt * 1e3,
                         "gbs": (byts / (ms / 1e3) / 1e9) if byts else None}
        return out

    roofline = None
    kernels = {}
    if prof:
        kernels = per_class(prof)
        dom_ms, dom_n = dom_timed
        avg_us = dom_ms / dom_n * 1e3
        byts_per_launch = sum(kernel_bytes(dom, n, s, p, k) for k in widths) / len(widths)
        achieved = byts_per_launch / (avg_us / 1e6) / 1e9
        traffic = load_traffic(dom)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                    "avg_launch_us": avg_us, "launches_timed": dom_n,
                    "alg_bytes_per_launch": byts_per_launch}

    # other arrangements of the same FP64 sequence, on request, each in its
    # own workspace: reduction trees (Sec. 4.1 applied recursively; level-1
    # nodes of g leaves, level-2 nodes of g level-1 nodes, ...) and FlatTSPQR
    # over P row blocks (Sec. 4.2)
    fan_ins = [int(g) for g in args.tree_fan_ins.split(",") if g] if args.tree_fan_ins else []
    flat_ps = [int(q) for q in args.flat_blocks.split(",") if q] if args.flat_blocks else []
    if fan_ins or flat_ps or args.householder_tree or args.tune_tiles:
        del ws
        torch.cuda.empty_cache()

    def time_arrangement(nbytes_alt, create, label):
        if nbytes_alt == 0:
            raise RuntimeError(f"{label} refused")
        aws = torch.empty(nbytes_alt // 8 + 32, dtype=torch.float64, device=dev)
        aptr = (aws.data_ptr() + 255) // 256 * 256

        def handle():
            code, ah = create(aptr, nbytes_alt)
            if code:
                raise orth.OrthError(label, code)
            return ah
        for _ in range(args.warmup):
            ah = handle()
            run_sequence(Xs, ah)
            orth.orth_destroy(ah)
        times = []
        for _ in range(args.steps):
            ah = handle()
            e0, e1 = TimingEvent(), TimingEvent()
            e0.record(stream)
            run_sequence(Xs, ah)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            code, st, info = orth.orth_status(ah)
            levels = orth.orth_tree_levels(ah)[1]
            orth.orth_destroy(ah)
            if code or st:
                raise RuntimeError(f"{label}: breakdown {info}")
        G = torch.mm(V, V.t()) - torch.eye(kmax, dtype=torch.float64, device=dev)
        ep = float(torch.linalg.matrix_norm(G, "fro"))
        del G, aws
        torch.cuda.empty_cache()
        return levels, min(times), ep

    trees = {}
    for g in fan_ins:
        levels, ms, ep = time_arrangement(
            orth.orth_tree_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64, g),
            lambda ptr, nb: orth.orth_create_tree(n, s, kmax, leaf, orth.ORTH_FP64, g, ptr, nb, sptr),
            f"tree fan-in {g}")
        trees[str(g)] = {"levels": levels, "ms_per_step": ms, "e_perp": ep, "vs_single_level": ms / ms_per_step}
        print(f"[bench] tree fan-in {g}: {levels} levels, {ms:.2f} ms per sequence, e_perp {ep:.2e}",
              file=sys.stderr, flush=True)
    hh_tree = None
    if args.householder_tree:
        g = args.householder_tree

        def create_hh_tree(ptr, nb):
            code, th = orth.orth_create_tree(n, s, kmax, leaf, orth.ORTH_FP64_HOUSEHOLDER, g, ptr, nb, sptr)
            if code == 0:
                code = orth.orth_set_level_variants(th, orth.ORTH_PIP_PLUS, orth.ORTH_HOUSEHOLDER)
            return code, th
        levels, ms, ep = time_arrangement(
            orth.orth_tree_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64_HOUSEHOLDER, g), create_hh_tree,
            f"householder tree fan-in {g}")
        hh_tree = {"fan_in": g, "levels": levels, "ms_per_step": ms, "e_perp": ep, "vs_fp64": ms / ms_per_step}
        print(f"[bench] householder leaves and householder tree, fan-in {g}: {levels} levels, {ms:.2f} ms per "
              f"sequence, e_perp {ep:.2e}", file=sys.stderr, flush=True)
    tiles = None
    if args.tune_tiles:
        from paper_2204_13393_amd import autotune
        t0 = time.perf_counter()
        best_t, cand_t = autotune.measure_tiles(n, s, kmax, leaf, steps=kmax // s)
        tune_s = time.perf_counter() - t0
        print(f"[bench] tile tuner: {len(cand_t)} candidates in {tune_s:.1f} s, pick {best_t}",
              file=sys.stderr, flush=True)
        _, ms_def, _ = time_arrangement(
            orth.orth_tiles_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64, 0, None),
            lambda ptr, nb: orth.orth_create_tiles(n, s, kmax, leaf, orth.ORTH_FP64, 0, None, ptr, nb, sptr),
            "plan's own tiles")
        _, ms_t, ep_t = time_arrangement(
            orth.orth_tiles_workspace_bytes(n, s, kmax, leaf, orth.ORTH_FP64, 0, best_t),
            lambda ptr, nb: orth.orth_create_tiles(n, s, kmax, leaf, orth.ORTH_FP64, 0, best_t, ptr, nb, sptr),
            f"tiles {best_t}")
        tiles = {"pick": list(best_t), "tuning_s": tune_s,
                 "candidates_ms": {str(tuple(c)): m for c, m in cand_t},
                 "ms_per_step_plan_tiles": ms_def, "ms_per_step_pick": ms_t, "pick_vs_plan": ms_t / ms_def,
                 "e_perp": ep_t}
        print(f"[bench] tiles {best_t}: {ms_t:.2f} ms per sequence against {ms_def:.2f} ms with the plan's own",
              file=sys.stderr, flush=True)
    flats = {}
    for q in flat_ps:
        rows = n // q
        _, ms, ep = time_arrangement(
            orth.orth_flat_workspace_bytes(n, s, kmax, rows),
            lambda ptr, nb: orth.orth_create_flat(n, s, kmax, rows, ptr, nb, sptr),
            f"flat {q} blocks")
        flats[str(q)] = {"block_rows": rows, "ms_per_step": ms, "e_perp": ep, "vs_tree": ms / ms_per_step}
        print(f"[bench] flat {q} blocks of {rows} rows: {ms:.2f} ms per sequence, e_perp {ep:.2e}",
              file=sys.stderr, flush=True)

    if args.copy_probe_gib > 0:
        cnt = int(args.copy_probe_gib * (1 << 30)) // 8
        src = torch.ones(cnt, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        if orth.orth_probe_copy(src.data_ptr(), dst.data_ptr(), cnt, sptr):
            raise RuntimeError("copy probe failed")
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_orth_call": ms_per_step / len(widths),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: N(0,1) start block (seed 0) and the A U_j Krylov blocks of a block-Arnoldi "
                "run on the 2D Dirichlet Laplacian, generated on the GPU before timing",
        "config": {"workload": W["name"], "n": n, "s": s, "arnoldi_steps": steps,
                   "orth_calls_per_step": len(widths), "leaf_rows": leaf, "leaves": p,
                   "k_max": kmax, "precision": "fp64", "variant": "BCGS-PIP+ leaves and reduction"},
        "e_perp": e_perp,
        "e_perp_gate_1e-10": e_perp <= 1e-10,
        "mixed": {
            "precision": "mixed_split32: leaf bases FP32 copy for the sweep-1 Gram, FP64 arithmetic",
            "ms_per_step": ms_mixed,
            "value_effective": total_bytes / (ms_mixed / 1e3) / 1e9,
            "unit": "GB/s (FP64 algorithmic bytes)",
            "speedup_vs_fp64": ms_per_step / ms_mixed,
            "e_perp": e_perp_mixed,
            "e_perp_gate_1e-10": e_perp_mixed <= 1e-10,
            "fp64_redo_steps": fallbacks[orth.ORTH_MIXED_SPLIT32],
            "kernels": per_class(prof_mixed) if prof_mixed else {},
        },
        "householder_leaves": None if hh is None else {
            "form": "fp64_householder: Algorithm HH at the leaves (reflectors + compact-WY T), "
                    "BCGS-PIP+ reduction",
            "ms_per_step": hh[0],
            "value_effective": total_bytes / (hh[0] / 1e3) / 1e9,
            "unit": "GB/s (BCGS-PIP+ algorithmic bytes)",
            "speedup_vs_fp64": ms_per_step / hh[0],
            "e_perp": hh[1],
            "e_perp_gate_1e-10": hh[1] <= 1e-10,
            # the first call (k = 0) has no Q_k^T w passes
            "kernels": per_class(hh[2], ("leaf_gram", "leaf_correct")) if hh[2] else {},
            "with_deflation": {
                "delta": DEFL_DELTA,
                "ms_per_step": hh_defl[0],
                "overhead_vs_householder": hh_defl[0] / hh[0],
                "columns_dropped": hh_defl[3],
                "e_perp": hh_defl[1],
                # root_chol holds the Jacobi eigen solver, root_correct the u1 W pass
                "kernels": {c: v for c, v in per_class(hh_defl[2]).items()
                            if c in ("root_chol", "root_correct")} if hh_defl[2] else {},
            },
        },
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    if trees:
        out["reduction_trees"] = trees
    if flats:
        out["flat_tspqr"] = flats
    if hh_tree:
        out["householder_every_level"] = hh_tree
    if tiles:
        out["tile_tuner"] = tiles
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
