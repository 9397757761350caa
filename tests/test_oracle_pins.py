"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

The paper prints no worked example and no recoverable value (its figures are
absent), so every pin is mathematical:

P1  brute-force joint Gaussian posterior over all time steps (filter and smoother);
P2  the MNE closed form (eqn5) and its equivalence with one Kalman update
    (the matrix-inversion-lemma remark that follows eqn10);
P3  the information form of the covariance update;
P4  the scalar Riccati steady state and the scalar smoother steady state;
P5  Q = 0: the smoother gain is the identity (recursive least squares);
P6  X = 0: no data, so P_{t|t} = P0 + t Q and smoother = filter;
P7  invariants: symmetry, P_{t|t} <= P_{t|t-1}, P_{t|T} <= P_{t|t};
P8  covariances do not depend on Y;
P9  means are linear in (x0, Y);
P10 calibration: normalised smoother errors on data drawn from the model are chi^2_N.

The last block plants mistakes in copies of the oracle and checks that the pins
catch them.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

import oracle
from oracle import kalman as K
from paper_1107_4192_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run(p):
    xf, Pf, dPf = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    xs, Ps, dPs = oracle.rts_smooth(xf, Pf, p.Q)
    return xf, Pf, dPf, xs, Ps, dPs


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("seed,N,m,T", [(1, 1, 1, 5), (2, 3, 2, 4), (3, 5, 3, 6), (4, 8, 4, 6),
                                        (5, 4, 6, 3), (6, 20, 6, 10)])
def test_p1_brute_force_joint_posterior(seed, N, m, T):
    p = synth.small_random(seed, N, m, T)
    xf, Pf, dPf, xs, Ps, dPs = run(p)
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    for got, want in zip((xf, Pf, xs, Ps), bf):
        assert rel(got, want) < 1e-11
    np.testing.assert_allclose(dPf, np.diagonal(Pf, axis1=1, axis2=2), rtol=0, atol=0)
    np.testing.assert_allclose(dPs, np.diagonal(Ps, axis1=1, axis2=2), rtol=0, atol=0)


def test_p1_brute_force_two_conditioning_forms_agree():
    p = synth.small_random(11, 6, 3, 5)
    a = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    b = oracle.joint_posterior_information(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-11


def test_p1_brute_force_prior_is_random_walk():
    # Cov(x_s, x_t) = P0 + min(s, t) Q, checked by Monte Carlo on a scalar walk.
    rng = np.random.default_rng(0)
    q, p0, T, n = 0.3, 0.7, 4, 400000
    x = rng.normal(scale=math.sqrt(p0), size=n)[:, None] + np.cumsum(
        rng.normal(scale=math.sqrt(q), size=(n, T)), axis=1)
    emp = np.cov(x.T)
    _, Sig = oracle.joint.joint_prior(np.array([[q]]), np.zeros(1), np.array([[p0]]), T)
    assert np.abs(emp - Sig).max() < 0.02


# ---------------------------------------------------------------- P2
def test_p2_mne_equals_one_kalman_step():
    p = synth.small_random(21, 12, 5, 1)
    C = p.P0 + p.Q
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, np.zeros(12), p.P0, p.Y)
    J = oracle.mne_solve(p.X, C, p.R, p.Y)
    assert rel(xf[0], J[0]) < 1e-12


def test_p2_mne_is_minimiser_of_eqn4():
    # Normal equations of ||y - X J||^2_R + ||J||^2_C: (X^T R^-1 X + C^-1) J = X^T R^-1 y.
    rng = np.random.default_rng(22)
    N, m, T = 15, 7, 4
    X = rng.normal(size=(m, N))
    C = np.diag(rng.uniform(0.5, 2.0, size=N)) * 3.0          # lambda R, R diagonal
    R = synth.random_spd(rng, m, 5.0, 0.2)
    Y = rng.normal(size=(T, m))
    J = oracle.mne_solve(X, C, R, Y)
    Rinv = np.linalg.inv(R)
    J2 = np.linalg.solve(X.T @ Rinv @ X + np.linalg.inv(C), X.T @ Rinv @ Y.T).T
    assert rel(J, J2) < 1e-11
    # and the gradient of the criterion vanishes there
    g = -X.T @ Rinv @ (Y.T - X @ J.T) + np.linalg.inv(C) @ J.T
    assert np.abs(g).max() < 1e-9 * np.abs(X.T @ Rinv @ Y.T).max()


def test_p2_kalman_update_is_mne_with_prior_mean():
    # The update equals eqn4's minimiser with mu = predicted mean, C = P_{t|t-1}.
    p = synth.small_random(23, 9, 4, 3)
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    t = 2
    mu, C = xf[t - 1], Pf[t - 1] + p.Q
    Rinv = np.linalg.inv(p.R)
    J = np.linalg.solve(p.X.T @ Rinv @ p.X + np.linalg.inv(C),
                        p.X.T @ Rinv @ p.Y[t] + np.linalg.solve(C, mu))
    assert rel(xf[t], J) < 1e-11


# ---------------------------------------------------------------- P3
def test_p3_information_form():
    p = synth.small_random(31, 10, 4, 5)
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    prev = p.P0
    info = p.X.T @ np.linalg.inv(p.R) @ p.X
    for t in range(5):
        Pp = prev + p.Q
        lhs = np.linalg.inv(Pf[t])
        rhs = np.linalg.inv(Pp) + info
        assert rel(lhs, rhs) < 1e-10
        prev = Pf[t]


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("q,r", [(0.1, 1.0), (2.0, 0.05), (1e-3, 1e-2)])
def test_p4_scalar_riccati(q, r):
    T = 400
    rng = np.random.default_rng(41)
    Y = rng.normal(size=(T, 1))
    xf, Pf, dPf, xs, Ps, dPs = run(synth.Problem("s", np.ones((1, 1)), np.array([[q]]),
                                                  np.array([[r]]), np.zeros(1),
                                                  np.array([[1.0]]), Y))
    Pinf = (-q + math.sqrt(q * q + 4 * q * r)) / 2.0
    assert abs(dPf[-1, 0] - Pinf) < 1e-13 * max(1.0, Pinf) + 1e-15
    A = Pinf / (Pinf + q)
    Psinf = Pinf / (1.0 + A)
    assert abs(dPs[T // 2, 0] - Psinf) < 1e-13 * max(1.0, Psinf) + 1e-15
    # steady-state gain on the mean: x_t = x_{t-1} + k (y_t - x_{t-1}), k = (Pinf+q)/(Pinf+q+r)
    k = (Pinf + q) / (Pinf + q + r)
    t = T - 1
    assert abs(xf[t, 0] - (xf[t - 1, 0] + k * (Y[t, 0] - xf[t - 1, 0]))) < 1e-12


# ---------------------------------------------------------------- P5
def test_p5_zero_process_noise_is_least_squares():
    p = synth.small_random(51, 6, 3, 7)
    p.Q = np.zeros_like(p.Q)
    xf, Pf, dPf, xs, Ps, dPs = run(p)
    for t in range(p.T):
        assert rel(xs[t], xf[-1]) < 1e-12
        assert rel(Ps[t], Pf[-1]) < 1e-12
    # static parameter: P_{T|T}^-1 = P0^-1 + T X^T R^-1 X
    info = np.linalg.inv(p.P0) + p.T * p.X.T @ np.linalg.inv(p.R) @ p.X
    assert rel(np.linalg.inv(Pf[-1]), info) < 1e-10


# ---------------------------------------------------------------- P6
def test_p6_no_data():
    p = synth.small_random(61, 7, 3, 6)
    p.X = np.zeros_like(p.X)
    xf, Pf, dPf, xs, Ps, dPs = run(p)
    for t in range(p.T):
        assert np.array_equal(xf[t], p.x0)
        assert rel(Pf[t], p.P0 + (t + 1) * p.Q) < 1e-15
        assert rel(xs[t], xf[t]) < 1e-15
        assert rel(Ps[t], Pf[t]) < 1e-14


# ---------------------------------------------------------------- P7
def test_p7_invariants_tiny_workload():
    p = synth.tiny(seed=1, N=120, m=30, T=12)
    xf, Pf, dPf, xs, Ps, dPs = run(p)
    prev = p.P0
    for t in range(p.T):
        Pt = Pf[t]
        assert np.array_equal(Pt, Pt.T)
        scale = np.abs(Pt).max()
        sla.cholesky(Pt, lower=True)
        assert np.linalg.eigvalsh((prev + p.Q) - Pt).min() > -1e-12 * scale
        assert np.linalg.eigvalsh(Pt - Ps[t]).min() > -1e-12 * scale
        assert np.array_equal(Ps[t], Ps[t].T)
        prev = Pt
    assert np.array_equal(xs[-1], xf[-1]) and np.array_equal(Ps[-1], Pf[-1])


# ---------------------------------------------------------------- P8
def test_p8_covariances_do_not_depend_on_data():
    p = synth.small_random(81, 9, 4, 5)
    a = run(p)
    p.Y = np.random.default_rng(82).normal(size=p.Y.shape) * 100.0
    b = run(p)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[4], b[4])


# ---------------------------------------------------------------- P9
def test_p9_means_linear_in_data():
    p = synth.small_random(91, 8, 3, 6)
    p.x0 = np.zeros(8)
    Y1, Y2 = p.Y.copy(), np.random.default_rng(92).normal(size=p.Y.shape)
    al, be = 0.7, -1.9
    p.Y = Y1; r1 = run(p)
    p.Y = Y2; r2 = run(p)
    p.Y = al * Y1 + be * Y2; r3 = run(p)
    assert rel(r3[0], al * r1[0] + be * r2[0]) < 1e-12
    assert rel(r3[3], al * r1[3] + be * r2[3]) < 1e-12


# ---------------------------------------------------------------- P10
def _simulate(seed, N, m, T):
    p = synth.small_random(seed, N, m, T)
    rng = np.random.default_rng(seed + 10_000)
    x = rng.multivariate_normal(p.x0, p.P0)
    truth = np.empty((T, N))
    for t in range(T):
        x = x + rng.multivariate_normal(np.zeros(N), p.Q)
        truth[t] = x
    p.Y = truth @ p.X.T + rng.multivariate_normal(np.zeros(m), p.R, size=T)
    return p, truth


@pytest.mark.slow
def test_p10_calibration_chi_square():
    N, m, T = 4, 2, 6
    zs, zf = [], []
    for seed in range(300):
        p, truth = _simulate(seed, N, m, T)
        xf, Pf, dPf, xs, Ps, dPs = run(p)
        t = seed % T
        e = truth[t] - xs[t]
        zs.append(e @ np.linalg.solve(Ps[t], e))
        e = truth[t] - xf[t]
        zf.append(e @ np.linalg.solve(Pf[t], e))
    assert stats.kstest(zs, stats.chi2(N).cdf).pvalue > 1e-3
    assert stats.kstest(zf, stats.chi2(N).cdf).pvalue > 1e-3


# ---------------------------------------------------------------- Section 2.4 set-up
def test_init_from_mne_closed_form():
    # X = I, C = c I, R = r I: the MNE estimate of eqn5 is exactly c / (c + r) times the data.
    # Data whose differences alternate a, b, a, b have mean (a + b) / 2 and centred differences
    # +-(a - b) / 2, so their sample covariance (divisor: differences - 1 = 3) is
    # (a - b)(a - b)^T / 3, scaled by (c / (c + r))^2, plus reg I.
    c, r, reg = 2.0, 0.5, 1e-3
    s = c / (c + r)
    a, b = np.array([1.0, 0.0]), np.array([-1.0, 2.0])
    y0 = np.array([0.5, -1.0])
    Y = np.array([y0, y0 + a, y0 + a + b, y0 + 2 * a + b, y0 + 2 * a + 2 * b])
    x0, Q = oracle.init_from_mne(np.eye(2), c * np.eye(2), r * np.eye(2), Y, reg=reg)
    assert np.allclose(x0, s * y0, rtol=0, atol=1e-15)
    expect = s * s * np.outer(a - b, a - b) / 3.0 + reg * np.eye(2)
    assert np.allclose(Q, expect, rtol=0, atol=1e-14)


def test_init_from_mne_recovers_random_walk_covariance():
    # With X = I and tiny sensor noise, MNE estimates are the states, and the differences are
    # the process noise: the estimate converges to Q.
    rng = np.random.default_rng(82)
    N, T = 3, 20000
    Qt = np.array([[0.5, 0.1, 0.0], [0.1, 0.3, 0.05], [0.0, 0.05, 0.2]])
    w = rng.multivariate_normal(np.zeros(N), Qt, size=T)
    Y = np.cumsum(w, axis=0)
    x0, Q = oracle.init_from_mne(np.eye(N), 1e6 * np.eye(N), 1e-9 * np.eye(N), Y)
    assert np.abs(Q - Qt).max() < 0.02


# ---------------------------------------------------------------- sampled smoother step
def test_rts_step_columns_matches_full_smoother():
    p = synth.small_random(71, 30, 7, 5)
    xf, Pf, dPf, xs, Ps, dPs = run(p)
    cols = [0, 3, 17, 29]
    for t in range(p.T - 1):
        x_t, Pc = K.rts_step_columns(xf[t], Pf[t], xs[t + 1], Ps[t + 1], p.Q, cols)
        assert rel(x_t, xs[t]) < 1e-12
        assert rel(Pc, Ps[t][:, cols]) < 1e-12


# ---------------------------------------------------------------- planted mistakes
def _smooth_literal_eqn12(xf, Pf, Q):
    # The misprinted eqn12 taken literally: x_{t|T} = x_{t|t} + A (x_{t|t} - x_{t+1|t}) == x_{t|t}.
    xs, Ps, dPs = K.rts_smooth(xf, Pf, Q)
    return xf.copy(), Ps, dPs


def _smooth_transposed_gain(xf, Pf, Q):
    T, N = xf.shape
    xs = xf.copy(); Ps = Pf.copy()
    for t in range(T - 2, -1, -1):
        A = K.smoother_gain(Pf[t], Q).T                     # planted: A^T instead of A
        xs[t] = xf[t] + A @ (xs[t + 1] - xf[t])
        Ps[t] = Pf[t] + A @ (Ps[t + 1] - Pf[t] - Q) @ A.T
    return xs, Ps, None


def _filter_dropped_q(X, Q, R, x0, P0, Y):
    return K.kf_filter(X, np.zeros_like(Q), R, x0, P0, Y)    # planted: predict without Q


def _filter_wrong_sign(X, Q, R, x0, P0, Y):
    T, N = Y.shape[0], X.shape[1]
    x, P = np.array(x0, float), np.array(P0, float)
    xf = np.empty((T, N)); Pf = np.empty((T, N, N))
    for t in range(T):
        Pp = P + Q
        S = X @ Pp @ X.T + R
        Kg = np.linalg.solve(S, X @ Pp).T
        x = x - Kg @ (Y[t] - X @ x)                          # planted: wrong sign
        P = Pp - Kg @ X @ Pp
        xf[t], Pf[t] = x, P
    return xf, Pf, None


@pytest.mark.parametrize("mutant", ["literal_eqn12", "transposed_gain", "dropped_q", "wrong_sign"])
def test_pins_catch_planted_mistakes(mutant):
    p = synth.small_random(7, 5, 3, 5)
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    filt = {"dropped_q": _filter_dropped_q, "wrong_sign": _filter_wrong_sign}.get(mutant, oracle.kf_filter)
    smooth = {"literal_eqn12": _smooth_literal_eqn12,
              "transposed_gain": _smooth_transposed_gain}.get(mutant, oracle.rts_smooth)
    xf, Pf, _ = filt(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    xs, Ps, _ = smooth(xf, Pf, p.Q)
    errs = [rel(a, b) for a, b in zip((xf, Pf, xs, Ps), bf)]
    assert max(errs) > 1e-6, errs


# ---------------------------------------------------------------- smoothed means without A_t
@pytest.mark.parametrize("seed,N,m,T", [(1, 1, 1, 5), (3, 5, 3, 6), (4, 8, 4, 6), (5, 4, 6, 3), (6, 20, 6, 10)])
def test_bf_means_match_brute_force(seed, N, m, T):
    p = synth.small_random(seed, N, m, T)
    xs = oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    assert rel(xs, bf[2]) < 1e-11


def test_bf_means_match_rts_on_tiny_workload():
    p = synth.tiny(T=15)
    xs = oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    assert rel(xs, run(p)[3]) < 1e-10


def test_bf_last_step_is_filter_and_zero_q_is_least_squares():
    p = synth.small_random(13, 6, 4, 5)
    xs = oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    xf = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y)[0]
    assert rel(xs[-1], xf[-1]) == 0.0                     # lambda_{T+1} = 0
    xs0 = oracle.bf_smooth_means(p.X, np.zeros_like(p.Q), p.R, p.x0, p.P0, p.Y)
    xf0 = oracle.kf_filter(p.X, np.zeros_like(p.Q), p.R, p.x0, p.P0, p.Y)[0]
    assert rel(xs0, np.broadcast_to(xf0[-1], xs0.shape)) < 1e-11   # static state: every x_{t|T} = x_{T|T}


def _bf_transposed(X, Q, R, x0, P0, Y):
    # planted: (I - K X) instead of its transpose in the lambda recursion
    T, N = Y.shape[0], X.shape[1]
    x, P = np.array(x0, float), np.array(P0, float)
    xf, Pf, e, Sf, Kg = np.empty((T, N)), [], [], [], []
    for t in range(T):
        Pp = P + Q
        S = X @ Pp @ X.T + R
        Kt = np.linalg.solve(S, X @ Pp).T
        e.append(Y[t] - X @ x); Sf.append(S); Kg.append(Kt)
        x = x + Kt @ e[-1]
        P = Pp - Kt @ X @ Pp
        xf[t] = x; Pf.append(P)
    xs, lam = np.empty((T, N)), np.zeros(N)
    for t in range(T - 1, -1, -1):
        xs[t] = xf[t] + Pf[t] @ lam
        lam = X.T @ np.linalg.solve(Sf[t], e[t]) + (np.eye(N) - Kg[t] @ X) @ lam
    return xs


def test_bf_pin_catches_planted_transpose():
    p = synth.small_random(17, 5, 3, 6)
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y)
    assert rel(_bf_transposed(p.X, p.Q, p.R, p.x0, p.P0, p.Y), bf[2]) > 1e-6


# ---------------------------------------------------------------- a transition F (eqn3)
@pytest.mark.parametrize("seed,N,m,T,density", [(21, 3, 2, 4, 1.0), (22, 5, 3, 6, 1.0), (23, 8, 4, 5, 0.4),
                                                (24, 12, 5, 6, 0.3)])
def test_transition_brute_force(seed, N, m, T, density):
    p = synth.small_random_F(seed, N, m, T, density)
    F = p.F_dense()
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    xs, Ps, _ = oracle.rts_smooth(xf, Pf, p.Q, F=F)
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    for got, want in zip((xf, Pf, xs, Ps), bf):
        assert rel(got, want) < 1e-10
    assert rel(oracle.bf_smooth_means(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F), bf[2]) < 1e-10
    bi = oracle.joint_posterior_information(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    assert rel(bi[2], bf[2]) < 1e-9


def test_transition_prior_is_lyapunov_recursion():
    p = synth.small_random_F(25, 4, 2, 5)
    F, T, N = p.F_dense(), 5, 4
    from oracle.joint import joint_prior
    mu, Sig = joint_prior(p.Q, p.x0, p.P0, T, F)
    C, x = p.P0.copy(), p.x0.copy()
    for t in range(T):
        C = F @ C @ F.T + p.Q                  # Cov(x_t, x_t) by the one-step recursion
        x = F @ x
        blk = slice(t * N, (t + 1) * N)
        assert rel(Sig[blk, blk], C) < 1e-13 and rel(mu[blk], x) < 1e-13
        if t + 1 < T:                          # Cov(x_{t+1}, x_t) = F Cov(x_t, x_t)
            assert rel(Sig[(t + 1) * N:(t + 2) * N, blk], F @ C) < 1e-13


def test_identity_transition_reproduces_random_walk():
    p = synth.small_random(26, 6, 3, 5)
    I = np.eye(6)
    a = run(p)
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=I)
    xs, Ps, _ = oracle.rts_smooth(xf, Pf, p.Q, F=I)
    assert rel(xf, a[0]) < 1e-14 and rel(xs, a[3]) < 1e-14 and rel(Ps, a[4]) < 1e-14


def test_neighbourhood_transition_is_row_stochastic_six_neighbours():
    pts = np.random.default_rng(3).normal(size=(200, 3))
    rp, ci, v = synth.neighbourhood_transition(pts, 6, 0.5)
    F = synth.csr_to_dense(rp, ci, v, 200)
    assert np.allclose(F.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(np.diff(rp) == 7) and np.allclose(np.diag(F), 0.5)
    d = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d, np.inf)
    for i in (0, 17, 199):
        assert set(np.nonzero(F[i])[0]) - {i} == set(np.argsort(d[i])[:6])


def test_transition_pin_catches_missing_ft_in_gain():
    p = synth.small_random_F(27, 5, 3, 5)
    F = p.F_dense()
    bf = oracle.joint_posterior(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    T = xf.shape[0]
    xs = xf.copy()
    for t in range(T - 2, -1, -1):              # planted: A_t = P_t P_{t+1|t}^-1 (F^T dropped)
        Pn = F @ Pf[t] @ F.T + p.Q
        A = np.linalg.solve(Pn, Pf[t]).T
        xs[t] = xf[t] + A @ (xs[t + 1] - F @ xf[t])
    assert rel(xs, bf[2]) > 1e-6


# --- Associative form of the smoother (the algebra behind kf_smooth_assoc) -----------------

def _assoc_elements(xf, Pf, Q, F=None):
    T, N = xf.shape
    Fm = np.eye(N) if F is None else F
    els = []
    for t in range(T - 1):
        A = K.smoother_gain(Pf[t], Q, F)
        els.append((A, xf[t] - A @ Fm @ xf[t], Pf[t] - A @ Fm @ Pf[t]))
    els.append((np.zeros((N, N)), xf[T - 1], Pf[T - 1]))
    return els


def _op(a, b):
    E, g, L = a
    E2, g2, L2 = b
    return (E @ E2, E @ g2 + g, E @ L2 @ E.T + L)


@pytest.mark.parametrize("with_F", [False, True])
def test_associative_scan_reproduces_rts(with_F):
    # Any bracketing of the suffix products gives the RTS smoother: right to left (the
    # sequential recursion), left to right, and the blocked scan kf_smooth_assoc runs.
    p = synth.small_random_F(21, 7, 3, 11) if with_F else synth.small_random(21, 7, 3, 11)
    F = p.F_dense() if with_F else None
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    xs, Ps, _ = oracle.rts_smooth(xf, Pf, p.Q, F)
    els = _assoc_elements(xf, Pf, p.Q, F)
    T = len(els)
    for t in range(T):
        acc = els[t]                                  # left to right: ((a_t o a_t+1) o a_t+2) ...
        for u in range(t + 1, T):
            acc = _op(acc, els[u])
        assert np.abs(acc[0]).max() == 0.0
        assert np.allclose(acc[1], xs[t], rtol=1e-11, atol=1e-12)
        assert np.allclose(acc[2], Ps[t], rtol=1e-10, atol=1e-12)
    # blocked: suffixes inside blocks, block totals from the back, then the rest of each block
    ln = math.ceil(math.sqrt(T))
    s = list(els)
    starts = list(range(0, T, ln))
    ends = [min(T, b + ln) - 1 for b in starts]
    for b0, b1 in zip(starts, ends):
        for t in range(b1 - 1, b0 - 1, -1):
            s[t] = _op(s[t], s[t + 1])
    for k in range(len(starts) - 2, -1, -1):
        s[starts[k]] = _op(s[starts[k]], s[starts[k + 1]])
    for k in range(len(starts) - 1):
        for t in range(starts[k] + 1, ends[k] + 1):
            s[t] = _op(s[t], s[starts[k + 1]])
    for t in range(T):
        assert np.allclose(s[t][1], xs[t], rtol=1e-11, atol=1e-12)
        assert np.allclose(s[t][2], Ps[t], rtol=1e-10, atol=1e-12)


def test_associative_pin_catches_planted_mistakes():
    # The same check with a transpose dropped from the operator, or F dropped from the
    # elements, must fail.
    p = synth.small_random_F(22, 6, 3, 8)
    F = p.F_dense()
    xf, Pf, _ = oracle.kf_filter(p.X, p.Q, p.R, p.x0, p.P0, p.Y, F=F)
    xs, Ps, _ = oracle.rts_smooth(xf, Pf, p.Q, F)

    def suffix(els, op):
        acc = els[-1]
        out = [acc]
        for e in reversed(els[:-1]):
            acc = op(e, acc)
            out.append(acc)
        return out[::-1]

    good = suffix(_assoc_elements(xf, Pf, p.Q, F), _op)
    assert max(np.abs(g[2] - P).max() for g, P in zip(good, Ps)) < 1e-10
    bad_op = suffix(_assoc_elements(xf, Pf, p.Q, F), lambda a, b: (a[0] @ b[0], a[0] @ b[1] + a[1],
                                                                     a[0] @ b[2] @ a[0] + a[2]))
    assert max(np.abs(g[2] - P).max() for g, P in zip(bad_op, Ps)) > 1e-6
    bad_el = suffix(_assoc_elements(xf, Pf, p.Q, None), _op)     # gains and elements without F
    assert max(np.abs(g[1] - x).max() for g, x in zip(bad_el, xs)) > 1e-6
