"""Benchmark: Kalman filter + fixed-interval smoother time-steps/s at N=5124, m=306 on one MI355X.

One benchmark "step" is one pass of the whole hot path -- kf_filter over T time
steps followed by kf_smooth -- over the paper-scale synthetic workload (N=5124
fixed-orientation sources, m=306 sensors, T=200 steps, float64 throughout),
with all inputs resident in HBM before the timed region. The reported value is
time-steps per second: T * steps / elapsed; ms_per_step is the time of one time
step (ms_per_pass / T), ms_per_pass that of one whole pass.

Besides the contract's JSON fields the line carries:
  roofline      the smoother's float64 N x N x N products (the dominant kernel,
                gemm_kernel<double, 1, *>), event-timed live during the timed region on the
                streams they run on, one event pair per dispatch; `isolated` is the same
                products in one extra pass serialised onto one stream (each runs alone,
                gemm_kernel<double, 3, *>); `path` is the whole pass against the FP64 peak;
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample (the first 16 steps of
                the same workload at full N: filter 16 steps + smoother 15 steps);
  accuracy      the float64 and mixed-precision GPU paths against that same oracle run (same
                inputs, same 16-step horizon): normwise and element-wise errors per result;
  mixed         the same workload in mixed precision (FP32 MFMA bulk, FP64 factorisations,
                FP32 store): its rate, speedup over FP64, its error against the oracle (from
                `accuracy`) and against the FP64 path at T=200, and its pass against the bound of
                its FP64 work at the FP64 peak plus its FP32 work at the FP32 peak;
  mean_only     kf_filter + kf_smooth_means (smoothed means without P_{t|T}) on the same
                workload, and its difference from the full smoother's means;
  batched       eight data sets of the same model through one covariance pass
                (kf_filter_batch + kf_smooth_batch), in data-set time-steps/s;
  assoc         kf_smooth_assoc (the smoother as an associative scan over time) against
                kf_smooth: smoother seconds on the tiny workload at two horizons and on this
                workload, and its difference from the step-by-step smoother;
  transfers     host <-> device time of one job's inputs and outputs (outside the timed region);
  free_orientation  N=15372 (5124 sites x 3), m=306, T=100, mixed precision, float32 store: the
                whole store in HBM and again under a budget that forces checkpoint-and-recompute
                (outputs must agree bit for bit);
  serving       p50/p99 job latency and throughput of the continuous-batching server on a
                Poisson stream of jobs of mixed N, m, T, against the same jobs run one at a
                time in FP64; `constrained` runs a second stream under a 40 GiB budget that an
                N=8196, T=150 job cannot fit without checkpointing.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--T 200] [--no-cpu] [--no-mixed] [--no-serving]
                       [--no-extra] [--no-free] [--workload paper|tiny|free|serving|serving5] [--jobs J]
                       [--config 1-5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_F64 = 78.6e12     # MI355X dense FP64 MFMA, FLOP/s
PEAK_F32 = 157.3e12    # MI355X dense FP32 MFMA, FLOP/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL = "gemm_kernel<double, 1, *>"    # the smoother's N x N x N products, float64 path (NT and NN layouts)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_nxn_f64_paper_N5124_traffic.json")
GEMM_SOURCE = os.path.join(ROOT, "paper_1107_4192_amd", "csrc", "gemm.hip")


def measured_traffic(flops_per_launch):
    """HBM bytes per launch of the dominant kernel: bytes per algorithmic flop from the committed
    counter runs times this run's flops per launch; None if the kernel source changed since."""
    import hashlib
    try:
        d = json.load(open(TRAFFIC_FILE))
        h = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if d.get("gemm_source_sha256") != h or not d.get("bytes_per_flop"):
        return None
    return d["bytes_per_flop"] * flops_per_launch


def calibration_copy():
    """A plain device copy of known size (256 MiB read + 256 MiB written) for scaling the HBM counters."""
    import torch
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("calibration copy: 3 x 256 MiB device-to-device")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def truncated(p, T):
    """The same workload cut to its first T steps (same X, Q, R, x0, P0 and data)."""
    import copy
    q = copy.copy(p)
    q.Y = p.Y[:T].copy()
    return q


def cpu_baseline(p, T_sample=16):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same workload; its outputs
    also serve as the reference of the accuracy leg."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max((i.get("num_threads", 1) for i in threadpool_info()), default=os.cpu_count())
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    q = truncated(p, T_sample)
    t0 = time.perf_counter()
    xf, Pf, dPf = oracle.kf_filter(q.X, q.Q, q.R, q.x0, q.P0, q.Y)
    xs, _, dPs = oracle.rts_smooth(xf, Pf, q.Q)
    dt = time.perf_counter() - t0
    base = {"value": T_sample / dt, "unit": "time-steps/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "sample": f"first {T_sample} steps of the N={p.N}, m={p.m} workload at full size: "
                      f"filter {T_sample} steps + smoother {T_sample - 1} steps, {dt:.1f} s"}
    return base, (q, xf, dPf, xs, dPs)


def accuracy(ref):
    """Float64 and mixed-precision GPU runs on the oracle's own inputs and horizon: normwise per step
    (max over steps: ||x^ - x|| / max ||x||, ||d^ - d||_inf / ||d||_inf) and element-wise
    (|g - w| / (|w| + 1e-3 max_i |w_t,i|)) errors of x_{t|t}, diag P_{t|t}, x_{t|T}, diag P_{t|T}."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg

    q, xf, dPf, xs, dPs = ref
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    def nx(g, w):
        return float(np.linalg.norm(g - w, axis=1).max() / np.linalg.norm(w, axis=1).max())

    def nd(g, w):
        return float((np.abs(g - w).max(axis=1) / np.abs(w).max(axis=1)).max())

    def el(g, w):
        return float((np.abs(g - w) / (np.abs(w) + 1e-3 * np.abs(w).max(axis=1, keepdims=True))).max())

    out = {"horizon": q.T, "what": f"GPU against the FP64 oracle on the first {q.T} steps of the workload "
                                   "(both sides run the same truncated problem)"}
    for label, opt in (("fp64", {}), ("mixed_fp32_store", {"precision": kfmeg.KF_MIXED, "store_fp32": True})):
        ks = kfmeg.KalmanSmoother(dev(q.X), dev(q.Q), dev(q.R), dev(q.x0), dev(q.P0), T_max=q.T, **opt)
        try:
            r = ks.run(dev(q.Y))
        finally:
            ks.close()
        g = {k: getattr(r, k).cpu().numpy() for k in ("x_filt", "Pdiag_filt", "x_smooth", "Pdiag_smooth")}
        out[label] = {"eps_x_filt": nx(g["x_filt"], xf), "eps_diagP_filt": nd(g["Pdiag_filt"], dPf),
                      "eps_x_smooth": nx(g["x_smooth"], xs), "eps_diagP_smooth": nd(g["Pdiag_smooth"], dPs),
                      "elem_x_smooth": el(g["x_smooth"], xs), "elem_diagP_smooth": el(g["Pdiag_smooth"], dPs),
                      "elem_diagP_filt": el(g["Pdiag_filt"], dPf)}
        log(f"accuracy {label}: " + ", ".join(f"{k} {v:.1e}" for k, v in out[label].items()))
    return out


def run_gpu(p, precision, steps, warmup, store_fp32=False, profile=False, isolated=False):
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    X, Q, R, x0, P0, Y = (dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y))
    ks = kfmeg.KalmanSmoother(X, Q, R, x0, P0, T_max=p.T, precision=precision, store_fp32=store_fp32)
    T, N = p.T, p.N
    xf = torch.empty((T, N), dtype=torch.float64, device="cuda")
    df = torch.empty_like(xf)
    xs = torch.empty_like(xf)
    ds = torch.empty_like(xf)

    def one_pass():
        kfmeg.kf_filter(ks.plan, Y, xf, df)
        kfmeg.kf_smooth(ks.plan, xs, ds, None)

    for w in range(warmup):
        one_pass()
        log(f"warmup pass {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    if profile:
        kfmeg.kf_set_profiling(ks.plan, True)
    t_filter = t_smooth = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        a = time.perf_counter()
        kfmeg.kf_filter(ks.plan, Y, xf, df)
        b = time.perf_counter()
        kfmeg.kf_smooth(ks.plan, xs, ds, None)
        c = time.perf_counter()
        t_filter += b - a
        t_smooth += c - b
        log(f"timed pass {k + 1}/{steps}: filter {b - a:.3f} s, smoother {c - b:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = kfmeg.kf_get_profile(ks.plan) if profile else None
    out = {"elapsed": elapsed, "t_filter": t_filter / steps, "t_smooth": t_smooth / steps, "prof": prof,
           "x_smooth": xs.clone(), "d_smooth": ds.clone()}
    if isolated:
        # one more pass, outside the timed region, with the smoother serialised onto one stream:
        # each product runs alone (a separately named kernel instantiation)
        kfmeg.kf_set_profiling(ks.plan, 2)
        kfmeg.kf_filter(ks.plan, Y, xf, df)
        a = time.perf_counter()
        kfmeg.kf_smooth(ks.plan, xs, ds, None)
        torch.cuda.synchronize()
        out["isolated_smoother_s"] = time.perf_counter() - a
        out["isolated_prof"] = kfmeg.kf_get_profile(ks.plan)
        kfmeg.kf_set_profiling(ks.plan, 0)
        log(f"isolated (serialised) smoother pass: {out['isolated_smoother_s']:.3f} s")
    ks.close()
    return out


def path_roofline(p, ms_pass):
    N, m, T = p.N, p.m, p.T
    kf = 2.0 * m * N * N + 2.0 * m * m * N + m ** 3 / 3.0 + m * m * N + m * N * N
    fis = N ** 3 / 3.0 + 2.0 * N ** 3 + 3.0 * N ** 3
    flops = T * kf + (T - 1) * fis
    achieved = flops / (ms_pass * 1e-3)
    return {"flops_per_pass": flops, "achieved": achieved / 1e12, "frac": achieved / PEAK_F64,
            "unit": "TFLOP/s"}


def mixed_roofline(p, ms_pass):
    """Mixed-precision bound of one pass: the float64 work (X P, S, the Cholesky of S, C = L^{-1} B;
    the Cholesky of P_{t+1|t} and the two gain solves) at the FP64 peak plus the float32 work (the
    downdate C^T C; eqn13's M = A_t D and P_t + M A_t^T) at the FP32 peak, against the measured
    pass."""
    N, m, T = p.N, p.m, p.T
    f64 = T * (2.0 * m * N * N + 2.0 * m * m * N + m ** 3 / 3.0 + m * m * N) + (T - 1) * (N ** 3 / 3.0 + 2.0 * N ** 3)
    f32 = T * m * N * N + (T - 1) * 3.0 * N ** 3
    bound_ms = (f64 / PEAK_F64 + f32 / PEAK_F32) * 1e3
    return {"f64_flops_per_pass": f64, "f32_flops_per_pass": f32, "bound_ms_per_pass": bound_ms,
            "measured_ms_per_pass": ms_pass, "frac": bound_ms / ms_pass}


def transfer_times(p):
    """Host <-> device time of one job's inputs (X, Q, R, x0, P0, Y) and outputs (x_{t|T} and the
    diagonals of P_{t|T}) through pinned host buffers; outside the timed region of `value`."""
    import numpy as np
    import torch

    host = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y)]
    nbytes_in = sum(h.numel() * h.element_size() for h in host)
    out_dev = [torch.empty((p.T, p.N), dtype=torch.float64, device="cuda") for _ in range(2)]
    out_host = [torch.empty((p.T, p.N), dtype=torch.float64).pin_memory() for _ in range(2)]
    nbytes_out = sum(h.numel() * h.element_size() for h in out_host)
    best_in = best_out = 1e30
    for _ in range(3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        dev = [h.to("cuda", non_blocking=True) for h in host]
        torch.cuda.synchronize()
        b = time.perf_counter()
        for d, h in zip(out_dev, out_host):
            h.copy_(d, non_blocking=True)
        torch.cuda.synchronize()
        c = time.perf_counter()
        best_in, best_out = min(best_in, b - a), min(best_out, c - b)
        del dev
    return {"h2d_s": best_in, "h2d_bytes": nbytes_in, "d2h_s": best_out, "d2h_bytes": nbytes_out,
            "what": "pinned host buffers; inputs X, Q, R, x0, P0, Y and outputs x_{t|T}, diag P_{t|T} of one "
                    "job; not part of the timed region"}


def run_mean_only(p, steps, xs_ref):
    """kf_filter + kf_smooth_means (backward information recursion) on the same workload."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    X, Q, R, x0, P0, Y = (dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y))
    ks = kfmeg.KalmanSmoother(X, Q, R, x0, P0, T_max=p.T, keep_gain_factors=True)
    xf = torch.empty((p.T, p.N), dtype=torch.float64, device="cuda")
    xs = torch.empty_like(xf)
    kfmeg.kf_filter(ks.plan, Y, xf)
    kfmeg.kf_smooth_means(ks.plan, xs)
    torch.cuda.synchronize()
    t_f = t_s = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        kfmeg.kf_filter(ks.plan, Y, xf)
        b = time.perf_counter()
        kfmeg.kf_smooth_means(ks.plan, xs)
        c = time.perf_counter()
        t_f += b - a
        t_s += c - b
    elapsed = time.perf_counter() - t0
    ref = xs_ref.cpu().numpy()
    err = float(np.linalg.norm(xs.cpu().numpy() - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())
    ks.close()
    log(f"mean-only: {p.T * steps / elapsed:.1f} steps/s")
    return {"value": p.T * steps / elapsed, "unit": "time-steps/s", "filter_s_per_pass": t_f / steps,
            "smoother_s_per_pass": t_s / steps, "eps_x_smooth_vs_rts_path": err,
            "what": "kf_filter + kf_smooth_means: smoothed means only, no P_{t|T}"}


def run_assoc(p, t_rts, xs_ref, ds_ref):
    """kf_smooth_assoc (time-parallel scan) against kf_smooth: on the tiny workload (N=500, m=60) at
    two horizons, where one step's products are too small to fill the GPU, and on the workload above."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg, synth

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    def smoother_times(q, reps):
        X, Q, R, x0, P0, Y = (dev(a) for a in (q.X, q.Q, q.R, q.x0, q.P0, q.Y))
        ks = kfmeg.KalmanSmoother(X, Q, R, x0, P0, T_max=q.T)
        xs = torch.empty((q.T, q.N), dtype=torch.float64, device="cuda")
        ds = torch.empty_like(xs)
        best = {"rts": 1e30, "assoc": 1e30}
        for _ in range(reps):
            for form in ("rts", "assoc"):
                r = ks.filter(Y)
                torch.cuda.synchronize()
                a = time.perf_counter()
                (kfmeg.kf_smooth if form == "rts" else kfmeg.kf_smooth_assoc)(ks.plan, xs, ds, None)
                torch.cuda.synchronize()
                best[form] = min(best[form], time.perf_counter() - a)
        ks.close()
        return best, xs, ds

    out = {"what": "kf_smooth_assoc: smoother as a blocked associative scan over time (about 2x the "
                   "products of kf_smooth, depth about 3 sqrt(T) launch groups); smoother seconds only"}
    for T in (50, 400):
        q = synth.tiny(T=T)
        best, _, _ = smoother_times(q, 3)
        out[f"tiny_N500_T{T}"] = {"rts_s": best["rts"], "assoc_s": best["assoc"],
                                  "speedup": best["rts"] / best["assoc"]}
        log(f"assoc tiny T={T}: rts {best['rts'] * 1e3:.1f} ms, assoc {best['assoc'] * 1e3:.1f} ms")
    X, Q, R, x0, P0, Y = (dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y))
    ks = kfmeg.KalmanSmoother(X, Q, R, x0, P0, T_max=p.T)
    xs = torch.empty((p.T, p.N), dtype=torch.float64, device="cuda")
    ds = torch.empty_like(xs)
    ks.filter(Y)
    torch.cuda.synchronize()
    a = time.perf_counter()
    kfmeg.kf_smooth_assoc(ks.plan, xs, ds, None)
    torch.cuda.synchronize()
    t_assoc = time.perf_counter() - a
    ks.close()
    ref, dref = xs_ref.cpu().numpy(), ds_ref.cpu().numpy()
    ex = float(np.linalg.norm(xs.cpu().numpy() - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())
    ed = float((np.abs(ds.cpu().numpy() - dref).max(axis=1) / np.abs(dref).max(axis=1)).max())
    out["paper"] = {"rts_s": t_rts, "assoc_s": t_assoc, "speedup": t_rts / t_assoc,
                    "eps_x_smooth_vs_rts_path": ex, "eps_diagP_smooth_vs_rts_path": ed,
                    "alloc_gib": kfmeg.kf_smooth_assoc_bytes(p.N, p.T) / 2**30}
    log(f"assoc paper: rts {t_rts:.2f} s, assoc {t_assoc:.2f} s")
    return out


def run_batched(p, B, steps):
    """B data sets through one covariance pass (kf_filter_batch + kf_smooth_batch)."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(11)
    Ys = np.stack([p.Y] + [p.Y + np.std(p.Y) * rng.normal(size=p.Y.shape) for _ in range(B - 1)])
    X, Q, R, x0, P0, Yd = (dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, Ys))
    ks = kfmeg.KalmanSmoother(X, Q, R, x0, P0, T_max=p.T)
    ks.run_batch(Yd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ks.run_batch(Yd)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ks.close()
    log(f"batched B={B}: {B * p.T * steps / elapsed:.1f} data-set steps/s")
    return {"B": B, "value": B * p.T * steps / elapsed, "unit": "data-set time-steps/s",
            "s_per_pass": elapsed / steps}


def fp64_step_times(shapes, T_probe=8):
    """Seconds per time step (filter + smoother) of a plain FP64 job of each (N, m) shape, from a
    short job run twice (the second run timed)."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg, synth

    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = {}
    for (N, m) in shapes:
        p = synth.custom(4242, N, m, T_probe)
        arrs = tuple(dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y))
        ks = kfmeg.KalmanSmoother(*arrs[:5], T_max=T_probe)
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ks.run(arrs[5])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        ks.close()
        del arrs
        out[(N, m)] = dt / T_probe
        log(f"FP64 probe N={N} m={m}: {dt / T_probe * 1e3:.1f} ms per step")
    return out


def run_serving(n_jobs=16, seed=5, rate=4.0, N_choices=(2000, 5124), m_choices=(102, 204, 306),
                T_range=(20, 60), max_active=4, budget_gib=0.0, plan=None, estimate_baseline=False):
    """Serving form: Poisson arrivals of filter+smoother jobs of mixed shapes, mixed precision
    with float32 stores, continuously batched; against the same jobs one at a time in FP64.
    `plan` replaces the drawn stream with an explicit job list (arrival_s, N, m, T, seed).
    `estimate_baseline`: instead of running the jobs one at a time in FP64, time a short FP64 job
    of each shape and sum T x seconds per step over the jobs (for streams whose sequential FP64 run
    would take tens of minutes)."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg, synth

    if plan is None:
        plan = synth.serving_jobs(seed=seed, n_jobs=n_jobs, rate_per_s=rate, N_choices=N_choices,
                                  m_choices=m_choices, T_range=T_range)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    jobs = []
    for j in plan:
        p = synth.custom(j["seed"], j["N"], j["m"], j["T"])
        jobs.append((j, tuple(dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y))))
    log(f"serving: {len(jobs)} jobs generated in {time.perf_counter() - t0:.1f} s")
    # continuous batching, mixed precision + float32 store
    srv = kfmeg.Server(hbm_budget_bytes=int(budget_gib * 2 ** 30), max_active=max_active,
                       precision=kfmeg.KF_MIXED, store_fp32=True)
    ids = []
    start = time.perf_counter()
    for j, arrs in jobs:
        delay = start + j["arrival_s"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(*arrs))
    # collect each job as it completes (a line per job: long streams stay visibly alive)
    lat, pending = {}, list(ids)
    while pending:
        for i in [i for i in pending if srv.info(i)["done"]]:
            lat[i] = srv.wait(i)[2]
            pending.remove(i)
            log(f"serving: job {ids.index(i)} done, latency {lat[i]:.0f} ms ({len(ids) - len(pending)}/{len(ids)})")
        if pending:
            time.sleep(0.05)
    lats = [lat[i] for i in ids]
    st = srv.stats()
    infos = [srv.info(i) for i in ids]
    srv.close()
    log(f"serving: {st['completed']} jobs, p50 {st['p50_ms']:.0f} ms, p99 {st['p99_ms']:.0f} ms, "
        f"{st['checkpointed']} checkpointed")
    shapes = sorted({(j["N"], j["m"]) for j in plan})
    steps = sum(j["T"] for j, _ in jobs)
    if estimate_baseline:
        del jobs[:]
        torch.cuda.empty_cache()
        per_step = fp64_step_times(shapes)
        seq = sum(j["T"] * per_step[(j["N"], j["m"])] for j in plan)
        log(f"serving: sequential FP64 estimated at {seq:.1f} s")
    else:
        # baseline: the same jobs one at a time in plain FP64
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j, arrs in jobs:
            ks = kfmeg.KalmanSmoother(*arrs[:5], T_max=j["T"])
            ks.run(arrs[5])
            ks.close()
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        log(f"serving: sequential FP64 {seq:.1f} s")
    return {"workload": f"{len(plan)} jobs, N x m in {shapes}, T in [{min(j['T'] for j in plan)}, "
                        f"{max(j['T'] for j in plan)}], arrivals over {plan[-1]['arrival_s']:.1f} s; mixed "
                        "precision, float32 store" + (f", HBM budget {budget_gib:g} GiB" if budget_gib else ""),
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "jobs_per_s": st["jobs_per_s"],
            "steps_per_s": st["steps_per_s"], "max_concurrent": st["max_concurrent"],
            "checkpointed": st["checkpointed"], "peak_gib": st["peak_bytes"] / 2 ** 30,
            "sequential_fp64_steps_per_s": steps / seq,
            "sequential_fp64": "estimated from a short FP64 job per shape" if estimate_baseline else "measured",
            "jobs": [(j["N"], j["m"], j["T"], round(j["arrival_s"], 3)) for j in plan],
            "latency_ms": [round(v, 1) for v in lats],
            "throughput_speedup_vs_sequential_fp64": st["steps_per_s"] / (steps / seq),
            "mean_queue_ms": float(np.mean([i["queued_ms"] for i in infos])),
            "checkpoint_strides": [i["checkpoint_stride"] for i in infos]}


# A stream that a 40 GiB server cannot hold without checkpointing: the N=8196, T=150 job alone needs
# 40 GB of float32 covariance store plus its workspace, so it is admitted with a checkpointed store.
CONSTRAINED_JOBS = [
    {"job": 0, "arrival_s": 0.0, "N": 8196, "m": 306, "T": 150, "seed": 9100},
    {"job": 1, "arrival_s": 0.4, "N": 2000, "m": 102, "T": 60, "seed": 9101},
    {"job": 2, "arrival_s": 0.8, "N": 5124, "m": 204, "T": 40, "seed": 9102},
    {"job": 3, "arrival_s": 1.2, "N": 2000, "m": 306, "T": 50, "seed": 9103},
]


def run_free(T=100, budget_gib=64.0):
    """Free-orientation workload (N = 15372 = 5124 sites x 3, m = 306): mixed precision, float32
    store; once with the whole store in HBM and once under an HBM budget that forces
    checkpoint-and-recompute. Results must agree bit for bit."""
    import numpy as np
    import torch
    from paper_1107_4192_amd import kfmeg, synth

    t0 = time.perf_counter()
    p = synth.free(T=T)
    log(f"free-orientation workload N={p.N} m={p.m} T={p.T} generated in {time.perf_counter() - t0:.1f} s")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    arrs = [dev(a) for a in (p.X, p.Q, p.R, p.x0, p.P0, p.Y)]
    out = {"workload": f"free orientation: N={p.N} (5124 sites x 3), m={p.m}, T={p.T}, mixed precision, "
                       "float32 store"}
    ref = None
    for label, budget in (("full_store", 0), ("checkpointed", int(budget_gib * 2 ** 30))):
        ks = kfmeg.KalmanSmoother(*arrs[:5], T_max=p.T, precision=kfmeg.KF_MIXED, store_fp32=True,
                                  hbm_budget_bytes=budget)
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = ks.filter(arrs[5])
        b = time.perf_counter()
        ks.smooth(res)
        torch.cuda.synchronize()
        c = time.perf_counter()
        ks.close()
        log(f"free ({label}): filter {b - a:.1f} s, smoother {c - b:.1f} s")
        out[label] = {"steps_per_s": p.T / (c - a), "filter_s": b - a, "smoother_s": c - b,
                      "hbm_budget_gib": budget / 2 ** 30 if budget else None,
                      "plan_gib": kfmeg.kf_plan_bytes(p.N, p.m, p.T, kfmeg.options(kfmeg.KF_MIXED, True)) / 2 ** 30}
        if ref is None:
            ref = (res.x_smooth.clone(), res.Pdiag_smooth.clone())
        else:
            out["checkpointed_equals_full_store"] = bool(torch.equal(ref[0], res.x_smooth) and
                                                         torch.equal(ref[1], res.Pdiag_smooth))
        del res
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--T", type=int, default=200)
    ap.add_argument("--N", type=int, default=5124)
    ap.add_argument("--m", type=int, default=306)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing and the accuracy leg")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="run a 256 MiB copy first (HBM counter scale)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-free", action="store_true", help="skip the free-orientation leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the mean-only, batched and associative-scan legs")
    ap.add_argument("--jobs", type=int, default=64, help="jobs of the 64-job stream run by --workload serving5")
    ap.add_argument("--first", type=int, default=0, help="first job of the 64-job stream run by --workload serving5")
    ap.add_argument("--config", type=int, choices=(1, 2, 3, 4, 5),
                    help="1 tiny FP64 (N=500, m=60, T=50); 2 paper scale FP64 (the default line); 3 paper scale "
                         "FP64 and mixed only; 4 free orientation; 5 the 64-job serving stream")
    ap.add_argument("--workload", choices=("paper", "tiny", "free", "serving", "serving5"), default="paper",
                    help="free: the free-orientation N=15372 workload only (full store and checkpointed); "
                         "serving: a larger serving run only (48 jobs up to N=8196 under a 96 GiB budget)")
    args = ap.parse_args()
    if args.config == 1:
        args.workload, args.T = "tiny", 50
        args.no_free = args.no_serving = True
    elif args.config == 3:
        args.no_extra = args.no_free = args.no_serving = True
    elif args.config == 4:
        args.workload = "free"
    elif args.config == 5:
        args.workload = "serving5"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the multi-GPU sharding "
              "of this path is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1107_4192_amd import kfmeg, synth
    kfmeg.load_library()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.workload == "free":
        print(json.dumps({"free_orientation": run_free(T=min(args.T, 100))}), flush=True)
        return
    if args.workload == "serving5":
        # the 64-job stream of mixed N (2000 to 15372), m and T (50 to 400) at 4 arrivals/s; --jobs
        # of it from job --first on, in arrival order
        plan = synth.serving_jobs(seed=5, n_jobs=64)[args.first:args.first + args.jobs]
        t_first = plan[0]["arrival_s"]
        plan = [dict(j, arrival_s=j["arrival_s"] - t_first) for j in plan]   # arrivals from 0
        print(json.dumps({"serving_stream64": run_serving(plan=plan, max_active=4, estimate_baseline=True)}),
              flush=True)
        return
    if args.workload == "serving":
        print(json.dumps({"serving_large": run_serving(n_jobs=48, seed=7, rate=2.0, N_choices=(2000, 5124, 8196),
                                                       T_range=(50, 150), max_active=4, budget_gib=96.0)}),
              flush=True)
        return
    if args.calib_copy:
        calibration_copy()
    t0 = time.perf_counter()
    if args.workload == "tiny":
        p = synth.tiny(T=args.T)
        what = f"tiny fixed orientation: N={p.N} sources, m={p.m} sensors, T={p.T}, float64"
    else:
        p = synth.paper(T=args.T, N=args.N, m=args.m)
        what = f"paper-scale fixed orientation: N={p.N} sources, m={p.m} sensors, T={p.T}, float64"
    log(f"workload N={p.N} m={p.m} T={p.T} generated in {time.perf_counter() - t0:.1f} s")

    r64 = run_gpu(p, kfmeg.KF_FP64, args.steps, args.warmup, profile=True, isolated=True)
    value = p.T * args.steps / r64["elapsed"]
    ms_pass = r64["elapsed"] / args.steps * 1e3
    kms, kflops, launches = r64["prof"]
    achieved = kflops / (kms * 1e-3) if kms > 0 else 0.0
    ims, iflops, ilaunches = r64["isolated_prof"]
    iachieved = iflops / (ims * 1e-3) if ims > 0 else 0.0
    line = {
        "metric": "KF+FIS time-steps/sec at N=5124, m=306 (FP64 vs mixed); p50/p99 job latency",
        "value": value,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_pass / p.T,
        "ms_per_pass": ms_pass,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded dipole lead field on a spherical shell, Gaussian-kernel Q, 3 sinusoidal patches, 5 dB)",
        "config": {"workload": what,
                   "N": p.N, "m": p.m, "T": p.T, "precision": "fp64", "store": "fp64",
                   "step": "one benchmark step = one pass of kf_filter over T time steps + kf_smooth",
                   "filter_s_per_pass": r64["t_filter"], "smoother_s_per_pass": r64["t_smooth"]},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_F64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_F64, "traffic": measured_traffic(kflops / max(launches, 1)),
                     "kernel": KERNEL + " (the smoother's eqn13 products M = A_t D and P_t + M A_t^T), "
                               "overlapped with the gain streams as in the timed passes",
                     "launches": launches, "avg_launch_ms": kms / max(launches, 1),
                     "flops_per_launch": kflops / max(launches, 1),
                     # the same products in one extra smoother pass serialised onto one stream
                     "isolated": {"kernel": "gemm_kernel<double, 3, *>", "launches": ilaunches,
                                  "avg_launch_ms": ims / max(ilaunches, 1),
                                  "flops_per_launch": iflops / max(ilaunches, 1),
                                  "achieved": iachieved / 1e12, "frac": iachieved / PEAK_F64,
                                  "smoother_s": r64["isolated_smoother_s"]},
                     # the whole filter + smoother pass against the same peak: algorithmic flops
                     # (rank-m filter, N^3/3 Cholesky, 2 N^3 gain, 3 N^3 eqn13; no explicit inverse)
                     # over the timed wall clock
                     "path": path_roofline(p, ms_pass)},
    }
    ref = None
    if not args.no_cpu:
        line["cpu_baseline"], ref = cpu_baseline(p)
        log(f"cpu baseline: {line['cpu_baseline']['value']:.3f} time-steps/s on {line['cpu_baseline']['cores']} threads")
        line["accuracy"] = accuracy(ref)
    if not args.no_mixed:
        import numpy as np
        rmx = run_gpu(p, kfmeg.KF_MIXED, max(1, args.steps), 1, store_fp32=True, profile=True)
        vmx = p.T * max(1, args.steps) / rmx["elapsed"]
        xs64, xsm = r64["x_smooth"].cpu().numpy(), rmx["x_smooth"].cpu().numpy()
        d64, dm = r64["d_smooth"].cpu().numpy(), rmx["d_smooth"].cpu().numpy()
        ex = float(np.linalg.norm(xsm - xs64, axis=1).max() / np.linalg.norm(xs64, axis=1).max())
        ed = float((np.abs(dm - d64).max(axis=1) / np.abs(d64).max(axis=1)).max())
        line["mixed"] = {"value": vmx, "unit": "time-steps/s", "speedup_vs_fp64": vmx / value,
                         "eps_x_smooth_vs_fp64_path": ex, "eps_diagP_smooth_vs_fp64_path": ed,
                         "store": "fp32", "filter_s_per_pass": rmx["t_filter"],
                         "smoother_s_per_pass": rmx["t_smooth"],
                         "roofline": mixed_roofline(p, rmx["elapsed"] / max(1, args.steps) * 1e3)}
        if "accuracy" in line:
            acc = line["accuracy"]["mixed_fp32_store"]
            line["mixed"].update({"eps_x_smooth_vs_oracle": acc["eps_x_smooth"],
                                  "eps_diagP_smooth_vs_oracle": acc["eps_diagP_smooth"],
                                  "oracle_horizon": line["accuracy"]["horizon"]})
    line["transfers"] = transfer_times(p)
    if not args.no_extra:
        line["mean_only"] = run_mean_only(p, max(1, args.steps), r64["x_smooth"])
        line["batched"] = run_batched(p, 8, 1)
        line["assoc"] = run_assoc(p, r64["t_smooth"], r64["x_smooth"], r64["d_smooth"])
    if not args.no_free:
        line["free_orientation"] = run_free()
    if not args.no_serving:
        line["serving"] = run_serving()
        line["serving"]["constrained"] = run_serving(plan=CONSTRAINED_JOBS, max_active=4, budget_gib=40.0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
