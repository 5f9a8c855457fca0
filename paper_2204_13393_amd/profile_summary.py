"""Summaries of rocprofv3 output for this library's kernels.

Kernel instantiations carry their launch site's profiler class as the last
template argument after the block width (k_gram<S, CLS, QM>,
k_rowmfma<S, EXPL, CLS, QM>), so every
dispatch in a kernel trace maps to one class of orth_kernel_class.

    python -m paper_2204_13393_amd.profile_summary trace  <kernel_trace.csv>
    python -m paper_2204_13393_amd.profile_summary counters <fetch.csv> <write.csv> \
            --copy-gib G --sha <sha256 of orth_kernels.hip> --out traffic.json

`trace` prints per-class dispatch counts, total and average durations.
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

GRAM = {0: "leaf_gram", 3: "root_gram", 9: "leaf_gram2", 10: "root_gram2"}
ROWUPD = {2: "leaf_correct", 5: "root_correct", 6: "root_finalize", 7: "leaf_finalize"}


def classify(name):
    m = re.search(r"k_gram<(\d+), (\d+), (\d+)>", name)
    if m:
        return GRAM.get(int(m.group(2)), "gram?")
    m = re.search(r"k_rowmfma<(\d+), (?:true|false), (\d+), (\d+)>", name)
    if m:
        return ROWUPD.get(int(m.group(2)), "rowupdate?")
    for key, cls in (("k_chol", "chol"), ("k_reduce", "reduce"), ("k_apply", "apply"),
                     ("k_copy(", "copy_probe"), ("k_laplacian", "operator"), ("k_fill", "fill"),
                     ("k_copy_cols", "export")):
        if key in name:
            return cls
    return "other"


def trace_summary(path):
    stats = defaultdict(lambda: [0, 0])
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            cls = classify(row["Kernel_Name"])
            dur = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
            stats[cls][0] += 1
            stats[cls][1] += dur
    return stats


def counter_avgs(path, counter):
    acc = defaultdict(lambda: [0, 0.0])
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            cls = classify(row["Kernel_Name"])
            acc[cls][0] += 1
            acc[cls][1] += float(row["Counter_Value"])
    return {k: v[1] / v[0] for k, v in acc.items() if v[0]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    c = sub.add_parser("counters")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--copy-gib", type=float, required=True)
    c.add_argument("--sha", required=True)
    c.add_argument("--out")
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        stats = trace_summary(args.csv)
        print("| class | dispatches | total ms | avg us |")
        print("|---|---:|---:|---:|")
        for cls, (n, ns) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
            print(f"| {cls} | {n} | {ns / 1e6:.3f} | {ns / n / 1e3:.2f} |")
        return 0
    fetch = counter_avgs(args.fetch_csv, "FETCH_SIZE")
    write = counter_avgs(args.write_csv, "WRITE_SIZE")
    copy_bytes = args.copy_gib * (1 << 30)
    sf = copy_bytes / (fetch["copy_probe"] * 1024.0)
    sw = copy_bytes / (write["copy_probe"] * 1024.0)
    out = {"kernel_source_sha256": args.sha, "copy_probe_gib": args.copy_gib,
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
