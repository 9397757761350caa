"""Mean-only smoother (backward information recursion) through the C ABI.

Its means must equal the oracle's -- both its own mean-only recursion and the RTS
means of eqn12 -- at 1e-10 normwise on the float64 path (1e-4 mixed), for single
and batched data sets, with a full or checkpointed covariance store.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1107_4192_amd import kfmeg, synth
from _helpers import dev, eps_x

pytestmark = pytest.mark.gpu


def _means(p, Y=None, **opt):
    Y = p.Y if Y is None else Y
    T = Y.shape[-2]
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=T, keep_gain_factors=True,
                              **opt)
    try:
        if Y.ndim == 2:
            res = ks.filter(dev(Y))
            ks.smooth_means(res)
            return res.x_smooth
        xf = torch.empty((Y.shape[0], T, p.N), dtype=torch.float64, device="cuda")
        kfmeg.kf_filter_batch(ks.plan, dev(Y), xf)
        xs = torch.empty_like(xf)
        kfmeg.kf_smooth_means(ks.plan, xs)
        return xs
    finally:
        ks.close()


@pytest.mark.parametrize("seed,N,m,T", [(1, 1, 1, 5), (2, 5, 3, 4), (3, 20, 6, 10), (4, 130, 7, 5),
                                        (5, 257, 130, 4), (6, 64, 64, 3), (7, 40, 9, 1)])
def test_means_vs_oracle(seed, N, m, T):
    p = synth.small_random(seed, N, m, T)
    xs = _means(p)
    assert eps_x(xs, oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)) <= 1e-10
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    assert eps_x(xs, oracle.rts_smooth(xf, Pf, p.Q)[0]) <= 1e-10


def test_means_tiny_workload_precisions_and_checkpointing():
    p = synth.tiny(T=16)
    ref = oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    full = _means(p)
    assert eps_x(full, ref) <= 1e-10
    ck = _means(p, checkpoint_stride=4)
    assert torch.equal(ck, full)                       # recomputed P_{t|t} are the stored ones bit for bit
    mixed = _means(p, precision=kfmeg.KF_MIXED, store_fp32=True)
    assert eps_x(mixed, ref) <= 1e-4
    mixed_ck = _means(p, precision=kfmeg.KF_MIXED, store_fp32=True, checkpoint_stride=5)
    assert torch.equal(mixed_ck, mixed)


def test_means_batched_data_sets():
    p = synth.small_random(31, 150, 20, 6)
    rng = np.random.default_rng(4)
    Ys = np.stack([p.Y] + [p.Y + rng.normal(size=p.Y.shape) for _ in range(2)])
    xs = _means(p, Y=Ys)
    for b in range(3):
        assert eps_x(xs[b], oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, Ys[b])) <= 1e-10, b
    ck = _means(p, Y=Ys, checkpoint_stride=2)
    for b in range(3):
        assert eps_x(ck[b], xs[b].cpu().numpy()) <= 1e-12, b
    one = _means(p)                                    # batch row 0 and the single-data-set path agree
    assert eps_x(xs[0], one.cpu().numpy()) <= 1e-12


def test_means_paper_scale_short_horizon():
    p = synth.paper(T=3)
    xs = _means(p)
    ref = oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    err = eps_x(xs, ref)
    print("paper-scale mean-only error", err)
    assert err <= 1e-10


def test_means_need_kept_factors():
    p = synth.small_random(41, 30, 5, 4)
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T)
    try:
        res = ks.filter(dev(p.Y))
        with pytest.raises(kfmeg.KFError) as ei:
            ks.smooth_means(res)
        assert ei.value.status == kfmeg.KF_ESTATE
    finally:
        ks.close()
