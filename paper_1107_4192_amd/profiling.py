"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1107_4192_amd.profiling stats <run_kernel_stats.csv> [top]
    python -m paper_1107_4192_amd.profiling traffic <fetch counter csv> <write counter csv> <kernel> <out.json> \
        [bench log of the counter run]
    python -m paper_1107_4192_amd.profiling mfma <counter csv> <kernel trace csv> [min_ms]
    python -m paper_1107_4192_amd.profiling isolated <kernel trace csv> [steps]

``traffic`` scales the per-dispatch FETCH_SIZE and WRITE_SIZE of `kernel` by what
the same counters read for the plain 256 MiB device copy that ``bench.py
--calib-copy`` runs first (rocclr's copyBuffer), and records the SHA-256 of the
GEMM source so that a stale figure is recognised. Given the counter run's bench log
(its JSON line carries the algorithmic flops of the same dispatches), it also records
HBM bytes per algorithmic flop, which ``bench.py`` scales to the flops per launch of
its own run (whose mix of launches differs from the short counter run's).

``mfma`` reads a run with SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE and the MFMA op counts
(SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32, 512 flops each) per kernel: the fraction of SIMD cycles
the matrix cores were busy (busy cycles over 1024 SIMDs, GRBM_GUI_ACTIVE summed over the 8
XCDs), the shader clock that GRBM_GUI_ACTIVE implies over the kernel's duration, and the
MFMA flops it executed per second (padding of partial tiles included).
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
    # every instantiation whose name contains `kernel` (e.g. one per operand layout)
    names = sorted(k for k in f if kernel in k)
    fk = [v * 1024.0 * ffac for k in names for v in f[k]]
    wk = [v * 1024.0 * wfac for k in names for v in w.get(k, [])]
    n = min(len(fk), len(wk))
    per = [fk[i] + wk[i] for i in range(n)]
    src = os.path.join(HERE, "csrc", "gemm.hip")
    return {
        "kernel": " + ".join(names),
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


def mfma_busy(counter_csv: str, trace_csv: str, min_ms: float = 1.0) -> str:
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in csv.DictReader(open(counter_csv)):
        per[r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in csv.DictReader(open(trace_csv)):
        c = per.get(r["Dispatch_Id"])
        if c is None:
            continue
        a = agg[r["Kernel_Name"]]
        a["n"] += 1
        a["dur"] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        for k, v in c.items():
            a[k] += v
    lines = [f"{'kernel':60s} {'launches':>8s} {'total_ms':>9s} {'clock_GHz':>9s} {'mfma_busy':>9s} "
             f"{'exec_TFLOP/s':>12s}"]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["dur"]):
        if a["dur"] * 1e3 < min_ms:
            continue
        cyc = a["GRBM_GUI_ACTIVE"] / 8.0
        busy = a["SQ_VALU_MFMA_BUSY_CYCLES"] / 1024.0 / cyc if cyc else 0.0
        flops = 512.0 * (a["SQ_INSTS_VALU_MFMA_MOPS_F64"] + a["SQ_INSTS_VALU_MFMA_MOPS_F32"])
        short = name.replace("kfmeg::", "").replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"{short[:60]:60s} {int(a['n']):8d} {a['dur'] * 1e3:9.2f} {cyc / a['dur'] / 1e9:9.2f} "
                     f"{busy:9.3f} {flops / a['dur'] / 1e12:12.1f}")
    return "\n".join(lines)


def isolated_pass(trace_csv: str, steps: int = 199) -> str:
    """Kernel time of the smoother pass that ``bench.py`` serialises onto one stream (the pass whose
    eqn13 products run as gemm_kernel<double, 3, *>): per kernel, summed over the pass and per step.
    The pass starts at the first kernel after the preceding filter's last covariance update."""
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if "gemm_kernel<double, 3," in r["Kernel_Name"]]
    if not marks:
        raise ValueError("no serialised smoother pass in this trace")
    t1 = int(rows[marks[-1]]["End_Timestamp"])
    i0 = marks[0]
    # walk back to the end of the filter pass before it: the last float64 TN launch (the downdate)
    while i0 > 0 and "gemm_kernel<double, 0, 2>" not in rows[i0 - 1]["Kernel_Name"]:
        i0 -= 1
    win = [r for r in rows[i0:] if int(r["End_Timestamp"]) <= t1]
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in win:
        n = r["Kernel_Name"].replace("kfmeg::", "").replace("(anonymous namespace)::", "").split("(")[0]
        agg[n][0] += 1
        agg[n][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    wall = (t1 - int(win[0]["Start_Timestamp"])) * 1e-6
    tot = sum(v[1] for v in agg.values())
    lines = [f"pass {wall:.1f} ms, summed kernel time {tot:.1f} ms, gaps {wall - tot:.1f} ms",
             f"{'kernel':60s} {'launches':>8s} {'total_ms':>9s} {'ms/step':>8s}"]
    for n, (c, ms) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{n[:60]:60s} {c:8d} {ms:9.1f} {ms / steps:8.3f}")
    return "\n".join(lines)


def main(argv):
    if argv[1] == "stats":
        print(kernel_stats_summary(argv[2], int(argv[3]) if len(argv) > 3 else 15))
    elif argv[1] == "traffic":
        d = traffic(argv[2], argv[3], argv[4], argv[6] if len(argv) > 6 else None)
        with open(argv[5], "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps({k: v for k, v in d.items() if k != "per_dispatch_bytes"}, indent=1))
    elif argv[1] == "mfma":
        print(mfma_busy(argv[2], argv[3], float(argv[4]) if len(argv) > 4 else 1.0))
    elif argv[1] == "isolated":
        print(isolated_pass(argv[2], int(argv[3]) if len(argv) > 3 else 199))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
