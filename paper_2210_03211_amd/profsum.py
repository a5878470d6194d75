"""Summaries of rocprofv3 CSV output, as kept under profiles/.

    python3 -m paper_2210_03211_amd.profsum trace <dir> [min_total_ms]
        per kernel: dispatches, total / mean / min / max duration (kernel trace)
    python3 -m paper_2210_03211_amd.profsum pmc <dir> [kernel_regex]
        per kernel: dispatches and the mean of every collected counter per dispatch; for
        rocclr copy kernels also the largest value (the calibration copy's own dispatch)

<dir> is the rocprofv3 output directory (-d); every *kernel_trace.csv or
*counter_collection.csv below it is read.
"""
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def short(name):
    n = name.split("(")[0]
    return n.replace("void ", "")[:60]


def kernel_trace(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), short(r["Kernel_Name"]),
                             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0))
    rows.sort()
    return rows


def counters(d):
    per = defaultdict(lambda: defaultdict(list))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                per[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return per


def trace_summary(d, min_total_ms=5.0):
    agg = defaultdict(list)
    for _, k, us in kernel_trace(d):
        agg[k].append(us)
    out = ["%-48s %9s %11s %9s %9s %10s" % ("kernel", "calls", "total_ms", "avg_us", "min_us", "max_us")]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) < 1000.0 * min_total_ms:
            continue
        out.append("%-48s %9d %11.1f %9.2f %9.2f %10.2f" % (k, len(v), sum(v) / 1000, sum(v) / len(v), min(v), max(v)))
    return out


def pmc_summary(d, pattern=None):
    out = []
    per = counters(d)
    for k in sorted(per):
        if pattern and not re.search(pattern, k):
            continue
        cs = per[k]
        line = ["%-40s" % k, "n=%d" % len(next(iter(cs.values())))]
        for c, v in sorted(cs.items()):
            line.append("%s=%.6g" % (c, sum(v) / len(v)))
            if k.startswith("__amd_rocclr_copyBuffer"):
                line.append("%s_max=%.6g" % (c, max(v)))
        out.append(" ".join(line))
    return out


def main(argv):
    if len(argv) < 3 or argv[1] not in ("trace", "pmc"):
        print(__doc__, file=sys.stderr)
        return 2
    if argv[1] == "trace":
        lines = trace_summary(argv[2], float(argv[3]) if len(argv) > 3 else 5.0)
    else:
        lines = pmc_summary(argv[2], argv[3] if len(argv) > 3 else None)
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
