"""mne_solve_noalloc (the entry point for callers that cannot allocate) against mne_solve.

Both run the same launches, so the results must agree bit for bit, and both must meet the
float64 bar against the oracle. Calls follow each other on the one fixed workspace: a large
call, a failing call (X C X^T + R not positive definite), then a smaller call, which must not
see anything the earlier calls left behind. A shape whose workspace exceeds the fixed array
is rejected before any launch.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1107_4192_amd import kfmeg, synth
from _helpers import dev, eps_x

pytestmark = pytest.mark.gpu


def both(X, C, R, Y):
    T, N = Y.shape[0], X.shape[1]
    J_ref = kfmeg.mne_solve(X, C, R, Y)
    J = torch.full((T, N), np.nan, dtype=torch.float64, device="cuda")
    kfmeg.mne_solve_noalloc(X, C, R, Y, J)
    return J, J_ref


def test_noalloc_matches_mne_solve_on_calls_in_a_row():
    big = synth.small_random(41, 700, 130, 37)
    small = synth.small_random(42, 300, 50, 9)
    for q in (big, small):
        q_args = (dev(q.X), dev(q.P0), dev(q.R), dev(q.Y))
        if q is small:
            # a failing call in between: X C X^T + R = -I is not positive definite
            bad = synth.small_random(43, 200, 40, 5)
            J = torch.empty((5, 200), dtype=torch.float64, device="cuda")
            with pytest.raises(kfmeg.KFError) as ei:
                kfmeg.mne_solve_noalloc(dev(bad.X), dev(np.zeros((200, 200))), dev(-np.eye(40)), dev(bad.Y), J)
            assert ei.value.status == kfmeg.KF_ENOTPD
        J, J_ref = both(*q_args)
        assert torch.equal(J, J_ref)
        assert eps_x(J, oracle.mne_solve(q.X, q.P0, q.R, q.Y)) <= 1e-10


def test_noalloc_paper_scale():
    p = synth.paper(T=64)
    C = 0.5 * np.eye(p.N)
    J, J_ref = both(dev(p.X), dev(C), dev(p.R), dev(p.Y))
    assert torch.equal(J, J_ref)
    assert eps_x(J, oracle.mne_solve(p.X, C, p.R, p.Y)) <= 1e-10


def test_noalloc_rejects_shapes_beyond_the_fixed_workspace():
    N, m, T = 1000, 2000, 4            # S and its inverse factor alone need 64 MB
    rng = np.random.default_rng(5)
    X, C, R, Y = (dev(a) for a in (rng.normal(size=(m, N)), np.eye(N), np.eye(m), rng.normal(size=(T, m))))
    J = torch.zeros((T, N), dtype=torch.float64, device="cuda")
    with pytest.raises(kfmeg.KFError) as ei:
        kfmeg.mne_solve_noalloc(X, C, R, Y, J)
    assert ei.value.status == kfmeg.KF_EINVAL
    assert "fixed device array" in str(ei.value)
    assert torch.count_nonzero(J) == 0                 # nothing was launched
