"""Free-orientation workload at full size (N = 15372 = 5124 sites x 3, m = 306).

The oracle cannot run the whole smoother at this size in seconds, so the test
checks every filtered output against the oracle and the first smoother step
(x_{t|T} in full, eight columns of P_{t|T}) against the oracle's single-step,
sampled-column form of eqn11-eqn13. Both the float64 path and the configuration of
the free-orientation workload (mixed precision, float32 store) are run.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import kalman as K
from paper_1107_4192_amd import kfmeg, synth
from _helpers import dev, eps_d, eps_x, to_np

pytestmark = pytest.mark.gpu

COLS = [0, 1, 2, 777, 5000, 9001, 15000, 15371]


@pytest.fixture(scope="module")
def workload():
    p = synth.free(T=3)
    xf, Pf, dPf = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    T = p.T
    # first smoother step: t = T-2 from x_{T|T}, P_{T|T} = filter
    xs_t, Pcols = K.rts_step_columns(xf[T - 2], Pf[T - 2], xf[T - 1], Pf[T - 1], p.Q, COLS)
    return p, xf, dPf, xs_t, Pcols


def run(p, **opt):
    ks = kfmeg.KalmanSmoother(dev(p.X), dev(p.Q), dev(p.R), dev(p.x0), dev(p.P0), T_max=p.T, **opt)
    try:
        res = ks.run(dev(p.Y), want_full=True)
    finally:
        ks.close()
    return res


@pytest.mark.parametrize("opt,tol", [({}, 1e-10),
                                     ({"precision": kfmeg.KF_MIXED, "store_fp32": True}, 1e-4)])
def test_free_orientation_full_size(workload, opt, tol):
    p, xf, dPf, xs_t, Pcols = workload
    res = run(p, **opt)
    T = p.T
    assert eps_x(res.x_filt, xf) <= tol
    assert eps_d(res.Pdiag_filt, dPf) <= tol
    assert eps_x(res.x_smooth[T - 2:T - 1], xs_t[None]) <= tol
    got = to_np(res.P_smooth[T - 2])[:, COLS]
    assert np.abs(got - Pcols).max() / np.abs(Pcols).max() <= tol
    # the smoothed covariance is exactly symmetric
    Ps = res.P_smooth[T - 2]
    assert torch.equal(Ps, Ps.T)


def test_free_orientation_checkpointed_full_size(workload):
    """Checkpoint-and-recompute at N=15372 (the store a budget would not hold): stride 3 over
    T=3 keeps only P_{3|3}, so the smoother step checked against the oracle reads a recomputed
    P_{2|2}; mixed precision, float32 store, as in the free-orientation workload."""
    p, xf, dPf, xs_t, Pcols = workload
    opt = {"precision": kfmeg.KF_MIXED, "store_fp32": True}
    full = run(p, **opt)
    ck = run(p, checkpoint_stride=3, **opt)
    T = p.T
    assert torch.equal(ck.x_smooth, full.x_smooth) and torch.equal(ck.Pdiag_smooth, full.Pdiag_smooth)
    assert torch.equal(ck.P_smooth, full.P_smooth)
    assert eps_x(ck.x_smooth[T - 2:T - 1], xs_t[None]) <= 1e-4
    got = to_np(ck.P_smooth[T - 2])[:, COLS]
    assert np.abs(got - Pcols).max() / np.abs(Pcols).max() <= 1e-4
