"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1107_4192_amd.profiling stats <run_kernel_stats.csv> [top]
    python -m paper_1107_4192_amd.profiling traffic <fetch counter csv> <write counter csv> <kernel> <out.json> \
        [bench log of the counter run]

``traffic`` scales the per-dispatch FETCH_SIZE and WRITE_SIZE of `kernel` by what
the same counters read for the plain 256 MiB device copy that ``bench.py
--calib-copy`` runs first (rocclr's copyBuffer), and records the SHA-256 of the
GEMM source so that a stale figure is recognised. Given the counter run's bench log
(its JSON line carries the algorithmic flops of the same dispatches), it also records
HBM bytes per algorithmic flop, which ``bench.py`` scales to the flops per launch of
its own run (whose mix of launches differs from the short counter run's).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 256 * 1024 * 1024
HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_stats_summary(path: str, top: int = 15) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = [f"{'kernel':78s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{r['Name'][:78]:78s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.1f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.1f} {float(r['Percentage']):6.2f}")
    return "\n".join(lines)


def _per_kernel(path: str, counter: str):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def _bench_flops(log_path: str) -> float:
    for line in open(log_path):
        if line.startswith("{"):
            r = json.loads(line)["roofline"]
            return float(r["flops_per_launch"]) * int(r["launches"])
    raise ValueError(f"no bench JSON line in {log_path}")


def traffic(fetch_csv: str, write_csv: str, kernel: str, bench_log: str | None = None) -> dict:
    f, w = _per_kernel(fetch_csv, "FETCH_SIZE"), _per_kernel(write_csv, "WRITE_SIZE")
    # the copy reads and writes COPY_BYTES: the largest dispatches of the copy kernel are the calibration
    fcopy = max(f[COPY_KERNEL]) * 1024.0
    wcopy = max(w[COPY_KERNEL]) * 1024.0
    ffac, wfac = COPY_BYTES / fcopy, COPY_BYTES / wcopy
    name = next(k for k in f if kernel in k)
    fk = [v * 1024.0 * ffac for v in f[name]]
    wk = [v * 1024.0 * wfac for v in w[name]]
    n = min(len(fk), len(wk))
    per = [fk[i] + wk[i] for i in range(n)]
    src = os.path.join(HERE, "csrc", "gemm.hip")
    return {
        "kernel": name,
        "dispatches": n,
        "fetch_scale": ffac,
        "write_scale": wfac,
        "fetch_bytes_per_launch": sum(fk[:n]) / n,
        "write_bytes_per_launch": sum(wk[:n]) / n,
        "bytes_per_launch": sum(per) / n,
        "per_dispatch_bytes": per,
        "gemm_source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
        "bytes_per_flop": (sum(per) / _bench_flops(bench_log)) if bench_log else None,
    }


def main(argv):
    if argv[1] == "stats":
        print(kernel_stats_summary(argv[2], int(argv[3]) if len(argv) > 3 else 15))
    elif argv[1] == "traffic":
        d = traffic(argv[2], argv[3], argv[4], argv[6] if len(argv) > 6 else None)
        with open(argv[5], "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps({k: v for k, v in d.items() if k != "per_dispatch_bytes"}, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
