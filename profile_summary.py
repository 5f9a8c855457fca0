"""Summaries of rocprofv3 output for this library's kernels.

Kernel instantiations carry their launch site's profiler class as the last
template argument (k_gram<S, CLS>, k_rowmfma<S, EXPL, CLS>, k_rowlds<S, EXPL, CLS>); k_gram_hi<S>
is the leaf first-sweep Gram of the mixed form, which reads the FP32 copy
of the basis. So every dispatch in a kernel trace maps to one class of
orth_kernel_class (k_gram_hi to leaf_gram, reported as leaf_gram_hi).

    python profile_summary.py trace  <kernel_trace.csv>
    python profile_summary.py counters <fetch.csv> <write.csv> \
            --copy-gib G --sha <sha256 of orth_kernels.hip followed by orth_internal.h> --out traffic.json

`trace` prints per-class dispatch counts, total and average durations.
`mfma` reads one --pmc pass of SQ_INSTS_VALU_MFMA_MOPS_F64,
SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE and prints per class the FP64
matrix-core work per dispatch (MOPS x 512 flops), the achieved TFLOP/s over
the dispatch's own timestamps, its fraction of the 78.6 TFLOP/s FP64 matrix
peak, and the busy fraction of the matrix cores (busy SIMD-cycles over
active cycles x CUs x 4 SIMDs; GRBM_GUI_ACTIVE is summed over the XCDs).
`--until-first CLASS` keeps only dispatches issued before the first one of
CLASS (by Dispatch_Id), and the copy probe wherever it ran: with bench.py's default run, `--until-first
leaf_gram_hi` keeps the FP64 sequences and drops the mixed-precision one.
`--window CLASS:L:i0-i1` keeps the dispatches of runs i0 to i1, where a
run ends with every L-th dispatch of CLASS: with bench.py's default order
(generation, profiled FP64, profiled mixed, FP64 warmup, the timed FP64
sequences, ...) `--window leaf_finalize:31:4-6` is the timed FP64 region of
`--steps 3 --warmup 1`.
`counters` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per class
and scales them by what the same counters read for the copy probe of
G GiB (a plain streaming copy: G GiB read, G GiB written).
"""

import argparse
import csv
import json
import re
import sys
from collections import defaultdict

GRAM = {0: "leaf_gram", 3: "root_gram", 9: "leaf_gram2", 10: "root_gram2", 11: "leaf_fallback"}
ROWUPD = {2: "leaf_correct", 5: "root_correct", 6: "root_finalize", 7: "leaf_finalize"}


def classify(name):
    if re.search(r"k_gram_hi<\d+>", name):
        return "leaf_gram_hi"
    m = re.search(r"k_gram<(\d+), (\d+)>", name)
    if m:
        return GRAM.get(int(m.group(2)), "gram?")
    m = re.search(r"k_row(?:mfma|lds)<(\d+), (?:true|false), (\d+)>", name)
    if m:
        return ROWUPD.get(int(m.group(2)), "rowupdate?")
    if "k_hh_panel" in name:
        return "leaf_hh_panel"
    if re.search(r"k_hh_(?:prep|tupd|coef|addec)", name):
        return "leaf_hh_small"
    for key, cls in (("k_chol", "chol"), ("k_reduce", "reduce"), ("k_apply", "apply"),
                     ("k_copy(", "copy_probe"), ("k_laplacian", "operator"), ("k_fill", "fill"),
                     ("k_copy_cols", "export")):
        if key in name:
            return cls
    return "other"


def _rows(path, until_first=None, counter=None, window=None):
    with open(path, newline="") as f:
        rows = [r for r in csv.DictReader(f)
                if counter is None or r.get("Counter_Name") == counter]
    if window:
        # CLASS:L:i0-i1 -- the dispatches of runs i0..i1, a run ending with
        # every L-th dispatch of CLASS (e.g. one 31-call sequence)
        cls, length, span = window.split(":")
        length = int(length)
        i0, i1 = (int(x) for x in span.split("-"))
        ids = sorted({int(r["Dispatch_Id"]) for r in rows if classify(r["Kernel_Name"]) == cls})
        lo = ids[i0 * length - 1] if i0 > 0 else -1
        hi = ids[(i1 + 1) * length - 1]
        rows = [r for r in rows if lo < int(r["Dispatch_Id"]) <= hi]
    if until_first:
        ids = [int(r["Dispatch_Id"]) for r in rows if classify(r["Kernel_Name"]) == until_first]
        if ids:
            cut = min(ids)
            rows = [r for r in rows if int(r["Dispatch_Id"]) < cut
                    or classify(r["Kernel_Name"]) == "copy_probe"]
    return rows


def trace_summary(path, until_first=None, window=None):
    stats = defaultdict(lambda: [0, 0])
    for row in _rows(path, until_first, window=window):
        cls = classify(row["Kernel_Name"])
        dur = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
        stats[cls][0] += 1
        stats[cls][1] += dur
    return stats


def counter_avgs(path, counter, until_first=None):
    acc = defaultdict(lambda: [0, 0.0])
    for row in _rows(path, until_first, counter):
        cls = classify(row["Kernel_Name"])
        acc[cls][0] += 1
        acc[cls][1] += float(row["Counter_Value"])
    return {k: v[1] / v[0] for k, v in acc.items() if v[0]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--until-first")
    t.add_argument("--window")
    c = sub.add_parser("counters")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--copy-gib", type=float, required=True)
    c.add_argument("--sha", required=True)
    c.add_argument("--out")
    c.add_argument("--until-first")
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("--until-first")
    m.add_argument("--xcds", type=int, default=8)
    m.add_argument("--cus", type=int, default=256)
    m.add_argument("--peak-tflops", type=float, default=78.6)
    args = ap.parse_args(argv)
    if args.cmd == "mfma":
        per = defaultdict(dict)      # (class, dispatch) -> counters and duration
        for r in _rows(args.csv, args.until_first):
            key = (classify(r["Kernel_Name"]), int(r["Dispatch_Id"]))
            per[key][r["Counter_Name"]] = float(r["Counter_Value"])
            per[key]["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        acc = defaultdict(lambda: [0, 0.0, 0.0, 0.0, 0.0])
        for (cls, _), d in per.items():
            a = acc[cls]
            a[0] += 1
            a[1] += d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512.0
            a[2] += d["ns"]
            a[3] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
            a[4] += d.get("GRBM_GUI_ACTIVE", 0.0) / args.xcds * args.cus * 4
        print("| class | dispatches | FP64 MFMA GFLOP/dispatch | TFLOP/s | of FP64 peak | MFMA busy |")
        print("|---|---:|---:|---:|---:|---:|")
        for cls, (n, fl, ns, busy, cap) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
            if fl == 0.0:
                continue
            tf = fl / ns / 1e3
            print(f"| {cls} | {n} | {fl / n / 1e9:.1f} | {tf:.1f} | {tf / args.peak_tflops:.2f} | "
                  f"{(busy / cap if cap else 0.0):.2f} |")
        return 0
    if args.cmd == "trace":
        stats = trace_summary(args.csv, args.until_first, args.window)
        print("| class | dispatches | total ms | avg us |")
        print("|---|---:|---:|---:|")
        for cls, (n, ns) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
            print(f"| {cls} | {n} | {ns / 1e6:.3f} | {ns / n / 1e3:.2f} |")
        return 0
    fetch = counter_avgs(args.fetch_csv, "FETCH_SIZE", args.until_first)
    write = counter_avgs(args.write_csv, "WRITE_SIZE", args.until_first)
    copy_bytes = args.copy_gib * (1 << 30)
    sf = copy_bytes / (fetch["copy_probe"] * 1024.0)
    sw = copy_bytes / (write["copy_probe"] * 1024.0)
    out = {"kernel_source_sha256": args.sha, "copy_probe_gib": args.copy_gib,
           "until_first": args.until_first,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    print(f"copy probe: FETCH_SIZE scale {sf:.4f}, WRITE_SIZE scale {sw:.4f}")
    print("| class | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM bytes/dispatch (scaled) |")
    print("|---|---:|---:|---:|")
    for cls in sorted(set(fetch) | set(write)):
        fb = fetch.get(cls, 0.0) * 1024.0 * sf
        wb = write.get(cls, 0.0) * 1024.0 * sw
        out["kernels"][cls] = {"fetch_kib": fetch.get(cls), "write_kib": write.get(cls),
                               "hbm_bytes_per_launch": fb + wb}
        print(f"| {cls} | {fetch.get(cls, 0.0):.0f} | {write.get(cls, 0.0):.0f} | {fb + wb:.4g} |")
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
