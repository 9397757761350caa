"""Time-parallel (associative scan) smoother, kf_smooth_assoc, through the C ABI.

The scan regroups eqn11-eqn13 (RTS reading) and reaches the same posterior, so it is
checked against the same FP64 oracle as kf_smooth: 1e-10 normwise per step on means,
diagonals and full covariances, for horizons that exercise every phase of the blocked
scan (T = 1, 2, a full last block, ragged blocks), ragged tile sizes, a sparse F, and
the paper's shape on a short horizon. Error paths: mixed precision, a float32 or
checkpointed store, batched data sets, and the consumed store after the call.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1107_4192_amd import kfmeg, synth
from _helpers import dev, eps_P, eps_d, eps_x

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def assoc_run(p, F=None, full=True, **opt):
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T, F=F, **opt)
    try:
        res = ks.smooth_assoc(ks.filter(dev(p.Y)), want_full=full)
    finally:
        ks.close()
    return res


def check(res, p, Fd=None, full=True):
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=Fd)
    xs, Ps, dPs = oracle.rts_smooth(xf, Pf, p.Q, F=Fd)
    errs = {"x_smooth": eps_x(res.x_smooth, xs), "d_smooth": eps_d(res.Pdiag_smooth, dPs)}
    if full:
        errs["P_smooth"] = eps_P(res.P_smooth, Ps)
        assert torch.equal(res.P_smooth, res.P_smooth.transpose(1, 2))
    assert max(errs.values()) <= TOL64, errs
    return errs


@pytest.mark.parametrize("seed,N,m,T", [(1, 1, 1, 1), (2, 5, 3, 2), (3, 20, 6, 9), (4, 130, 7, 10),
                                        (5, 257, 130, 7), (6, 64, 64, 23), (7, 40, 130, 5)])
def test_assoc_vs_oracle(seed, N, m, T):
    p = synth.small_random(seed, N, m, T)
    check(assoc_run(p), p)


def test_assoc_tiny_workload_matches_oracle_and_kf_smooth():
    p = synth.tiny(T=50)
    a = assoc_run(p, full=False)
    check(a, p, full=False)
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T)
    try:
        b = ks.run(dev(p.Y))
    finally:
        ks.close()
    assert eps_x(a.x_smooth, b.x_smooth) <= 1e-11 and eps_d(a.Pdiag_smooth, b.Pdiag_smooth) <= 1e-11


@pytest.mark.parametrize("seed,N,m,T,density", [(11, 20, 6, 8, 0.3), (12, 130, 7, 11, 0.05)])
def test_assoc_with_transition(seed, N, m, T, density):
    p = synth.small_random_F(seed, N, m, T, density)
    check(assoc_run(p, F=p.F), p, Fd=p.F_dense())


def test_assoc_paper_scale_short_horizon():
    """N=5124, m=306 on T=5 (two scan blocks): every output of the oracle."""
    p = synth.paper(T=5)
    errs = check(assoc_run(p, full=True), p)
    print("paper-scale assoc errors", errs)


def test_assoc_preconditions_and_consumed_store():
    p = synth.small_random(31, 30, 5, 6)
    # mixed precision: rejected before anything runs
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T,
                              precision=kfmeg.KF_MIXED)
    try:
        r = ks.filter(dev(p.Y))
        with pytest.raises(kfmeg.KFError, match="KF_EINVAL"):
            ks.smooth_assoc(r)
    finally:
        ks.close()
    # float32 store and checkpointed store: state errors
    for opt in ({"store_fp32": True}, {"checkpoint_stride": 3}):
        ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T, **opt)
        try:
            r = ks.filter(dev(p.Y))
            with pytest.raises(kfmeg.KFError, match="KF_ESTATE"):
                ks.smooth_assoc(r)
        finally:
            ks.close()
    # batched data sets: state error
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T)
    try:
        Y2 = dev(np.stack([p.Y, 2.0 * p.Y]))
        xb = torch.empty((2, p.T, p.N), dtype=torch.float64, device="cuda")
        kfmeg.kf_filter_batch(ks.plan, Y2, xb, None)
        with pytest.raises(kfmeg.KFError, match="KF_ESTATE"):
            ks.smooth_assoc(kfmeg.Result(xb[0], None))
        # one data set again: works; the store is then consumed until the next filter call
        r = ks.filter(dev(p.Y))
        a = ks.smooth_assoc(r, want_full=True)
        check(a, p)
        Pa = a.P_smooth.clone()
        with pytest.raises(kfmeg.KFError, match="KF_ESTATE"):
            ks.smooth(r)
        with pytest.raises(kfmeg.KFError, match="KF_ESTATE"):
            ks.smooth_assoc(r)
        b = ks.run(dev(p.Y), want_full=True)
        assert eps_P(Pa, b.P_smooth) <= 1e-11
    finally:
        ks.close()
