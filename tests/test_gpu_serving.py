"""Serving loop (kfs_* entry points): continuous batching of filter + smoother jobs.

Every job's result in the mix must equal the same job run alone (bitwise: each job
has its own buffers and the kernels are deterministic), admission must keep the
arena within its budget, and jobs whose full covariance store does not fit must run
checkpointed rather than fail.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1107_4192_amd import kfmeg, synth
from _helpers import dev, eps_d, eps_x

pytestmark = pytest.mark.gpu

SHAPES = [(200, 30, 6), (300, 60, 10), (500, 100, 14), (260, 45, 9), (400, 60, 7), (350, 90, 12)]


def make_jobs(shapes=SHAPES, seed0=100):
    return [synth.custom(seed0 + k, N, m, T) for k, (N, m, T) in enumerate(shapes)]


def alone(p, **opt):
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T, **opt)
    try:
        r = ks.run(dev(p.Y))
    finally:
        ks.close()
    return r.x_smooth, r.Pdiag_smooth


def serve(jobs, budget=0, max_active=3, gap_s=0.002, **opt):
    srv = kfmeg.Server(hbm_budget_bytes=budget, max_active=max_active, **opt)
    try:
        ids = []
        for p in jobs:
            ids.append(srv.submit(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), dev(p.Y)))
            time.sleep(gap_s)
        outs = [srv.wait(i) for i in ids]
        infos = [srv.info(i) for i in ids]
        stats = srv.stats()
    finally:
        srv.close()
    return outs, infos, stats


def test_each_job_same_alone_and_in_the_mix():
    jobs = make_jobs()
    outs, infos, stats = serve(jobs)
    assert stats["completed"] == len(jobs) and stats["failed"] == 0
    assert stats["max_concurrent"] >= 2            # jobs did overlap on the device
    assert stats["peak_bytes"] <= stats["budget_bytes"]
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    for p, (xs, ds, lat) in zip(jobs, outs):
        xa, da = alone(p)
        assert torch.equal(xs, xa) and torch.equal(ds, da)
    # and the mix agrees with the oracle
    p = jobs[2]
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    xs_ref, _, dPs_ref = oracle.rts_smooth(xf, Pf, p.Q)
    assert eps_x(outs[2][0], xs_ref) <= 1e-10 and eps_d(outs[2][1], dPs_ref) <= 1e-10


def test_mixed_precision_jobs_same_alone_and_in_the_mix():
    jobs = make_jobs(SHAPES[:4], seed0=200)
    outs, _, stats = serve(jobs, precision=kfmeg.KF_MIXED, store_fp32=True)
    assert stats["completed"] == len(jobs)
    for p, (xs, ds, _) in zip(jobs, outs):
        xa, da = alone(p, precision=kfmeg.KF_MIXED, store_fp32=True)
        assert torch.equal(xs, xa) and torch.equal(ds, da)


def test_budget_limits_admission_and_forces_checkpointing():
    # a long job whose store of T covariances dominates, next to three short ones
    jobs = make_jobs([(300, 40, 60), (200, 30, 6), (260, 45, 9), (250, 30, 8)], seed0=300)
    full = kfmeg.kf_plan_bytes(300, 40, 60) + 60 * 300 * 8 + (64 << 10)
    # half the long job's full footprint: its store (60 x 0.73 MB) cannot be kept whole,
    # a checkpointed one (about 16 slots) fits
    budget = full // 2
    outs, infos, stats = serve(jobs, budget=budget, max_active=4)
    assert stats["completed"] == len(jobs)
    assert stats["peak_bytes"] <= budget
    assert stats["checkpointed"] >= 1
    assert infos[0]["checkpoint_stride"] > 1
    for p, (xs, ds, _) in zip(jobs, outs):
        xa, da = alone(p)
        assert torch.equal(xs, xa) and torch.equal(ds, da)


def test_job_that_never_fits_is_rejected():
    p = make_jobs([(300, 40, 8)], seed0=400)[0]
    srv = kfmeg.Server(hbm_budget_bytes=1 << 20, max_active=2)
    try:
        jid = srv.submit(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), dev(p.Y))
        with pytest.raises(kfmeg.KFError) as ei:
            srv.wait(jid)
        assert ei.value.status == kfmeg.KF_ENOMEM
    finally:
        srv.close()


def test_cancel_queued_job():
    # one slot: the long first job keeps the others queued while the last one is cancelled
    jobs = make_jobs([(1500, 100, 20), (200, 30, 6), (260, 45, 9), (250, 30, 8)], seed0=500)
    srv = kfmeg.Server(max_active=1)
    try:
        ids = [srv.submit(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), dev(p.Y)) for p in jobs]
        assert srv.cancel(ids[3]) is True
        with pytest.raises(kfmeg.KFError) as ei:
            srv.wait(ids[3])
        assert ei.value.status == kfmeg.KF_ECANCELED
        outs = [srv.wait(i) for i in ids[:3]]
        assert srv.cancel(ids[0]) is False              # already done
        st = srv.stats()
        assert st["completed"] == 3 and st["canceled"] == 1
        xa, _ = alone(jobs[1])
        assert torch.equal(outs[1][0], xa)
    finally:
        srv.close()


def test_inputs_written_asynchronously_on_the_submitters_stream():
    """Inputs produced by GPU work still in flight on the caller's stream: the job must wait for it."""
    p = make_jobs([(300, 60, 8)], seed0=300)[0]
    xa, da = alone(p)
    srv = kfmeg.Server(max_active=2)
    side = torch.cuda.Stream()
    try:
        with torch.cuda.stream(side):
            busy = torch.ones((4096, 4096), dtype=torch.float64, device="cuda")
            for _ in range(20):                      # keep the stream busy before Y is written
                busy = busy @ busy * (1.0 / 4096)
            Y = torch.zeros((p.T, p.m), dtype=torch.float64, device="cuda")
            Y.copy_(torch.as_tensor(p.Y), non_blocking=False)
            Y.mul_(1.0)
            jid = srv.submit(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), Y, stream=side)
        xs, ds, _ = srv.wait(jid)
    finally:
        srv.close()
    assert torch.equal(xs, xa) and torch.equal(ds, da)
