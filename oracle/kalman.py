"""Kalman filter, fixed-interval smoother and MNE in float64 (test infrastructure only).

Plain NumPy/SciPy, written for a reader to check against the paper by eye:
no blocking, fusion or reordering beyond what the equations state. Library
routines serve as steps: ``@`` (a matrix product) and SciPy's Cholesky
factorisation and solve.

Notation maps the paper's letters onto the build's: state J_k -> x_t,
lead field H -> X (m x N), Sigma_w -> Q, Sigma_epsilon -> R, covariances
W_{k|k}, W_{k|k-1}, W_{k|N} -> P_{t|t}, P_{t|t-1}, P_{t|T}; the transition F is
the identity (the random-walk model that follows eqn3).

Readings taken where the paper is silent or garbled:

* The smoother equations eqn12 and eqn13 carry misprints (eqn12 starts from
  x_{k|k} and its bracket vanishes identically for F = I; eqn13 puts W_{k|N}
  inside its own bracket). They are read as the standard Rauch-Tung-Striebel
  form x_{t|T} = x_{t|t} + A_t (x_{t+1|T} - x_{t+1|t}) and
  P_{t|T} = P_{t|t} + A_t (P_{t+1|T} - P_{t+1|t}) A_t^T, the form of the
  textbook the paper cites for the smoother. The brute-force joint posterior
  in ``joint`` pins this reading.
* x0 and P0 are inputs; step t = 1 first predicts from them (P_{1|0} = P0 + Q)
  and then updates, so outputs cover t = 1..T.
* The covariance update after eqn10 is applied as (I - K X) P_{t|t-1} and the
  result is symmetrised, 1/2 (P + P^T); the paper does not say how symmetry is
  kept.
* Inverses in eqn8 and eqn11 are applied through Cholesky solves: identical in
  exact arithmetic, and a failed factorisation (a matrix not positive
  definite) raises ``numpy.linalg.LinAlgError``.
* The smoother re-forms P_{t+1|t} = P_{t|t} + Q from the stored filtered
  covariance (eqn7 again) rather than storing predicted covariances too.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["kf_update", "kf_filter", "smoother_gain", "rts_smooth", "rts_step_columns", "mne_solve",
           "init_from_mne", "bf_smooth_means"]


def _chol(A: np.ndarray):
    return sla.cho_factor(A, lower=True, check_finite=True)


def kf_update(x_pred: np.ndarray, P_pred: np.ndarray, X: np.ndarray, R: np.ndarray,
              y: np.ndarray):
    """One measurement update: eqn8 (gain), eqn10 (mean) and the covariance update after it.

    K = P_pred X^T (X P_pred X^T + R)^-1, x = x_pred + K (y - X x_pred),
    P = (I - K X) P_pred, symmetrised.
    """
    S = X @ P_pred @ X.T + R                       # bracket of eqn8
    cS = _chol(S)
    K = sla.cho_solve(cS, X @ P_pred).T            # P_pred X^T S^-1 (P_pred, S symmetric)
    x = x_pred + K @ (y - X @ x_pred)              # eqn10
    P = P_pred - K @ X @ P_pred                    # [I - K X] W_{k|k-1}
    P = (P + P.T) / 2.0
    return x, P


def kf_filter(X, Q, R, x0, P0, Y, keep_cov: bool = True, F=None):
    """Kalman filter for x_t = F x_{t-1} + w_t, y_t = X x_t + v_t (eqn1, eqn3; eqn6-eqn10).

    F = None is the random walk (F = I) and skips the products with F. Returns
    (xf, Pf, dPf): xf is T x N with xf[t-1] = x_{t|t}; Pf is a T x N x N array of
    P_{t|t} (None when ``keep_cov`` is false); dPf is T x N with the diagonals of P_{t|t}.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    T, N = Y.shape[0], X.shape[1]
    x = np.array(x0, dtype=np.float64)
    P = np.array(P0, dtype=np.float64)
    xf = np.empty((T, N))
    dPf = np.empty((T, N))
    Pf = np.empty((T, N, N)) if keep_cov else None
    for t in range(T):
        if F is None:
            x_pred = x                               # eqn6, F = I
            P_pred = P + Q                           # eqn7
        else:
            x_pred = F @ x                           # eqn6
            P_pred = F @ P @ F.T + Q                 # eqn7
        x, P = kf_update(x_pred, P_pred, X, R, Y[t])
        xf[t] = x
        dPf[t] = np.diag(P)
        if keep_cov:
            Pf[t] = P
    return xf, Pf, dPf


def smoother_gain(P_filt: np.ndarray, Q: np.ndarray, F=None) -> np.ndarray:
    """eqn11: A_t = P_{t|t} F^T P_{t+1|t}^-1 with P_{t+1|t} = F P_{t|t} F^T + Q, via a Cholesky solve."""
    if F is None:
        P_next_pred = P_filt + Q
        c = _chol(P_next_pred)
        return sla.cho_solve(c, P_filt).T            # (P_{t+1|t}^-1 P_{t|t})^T
    P_next_pred = F @ P_filt @ F.T + Q
    c = _chol(P_next_pred)
    return sla.cho_solve(c, F @ P_filt).T            # (P_{t+1|t}^-1 F P_{t|t})^T


def rts_smooth(xf: np.ndarray, Pf: np.ndarray, Q: np.ndarray, F=None):
    """Fixed-interval smoother (eqn11-eqn13 in the standard RTS reading), t = T-1 .. 1.

    Starts from x_{T|T}, P_{T|T} of the filter. Returns (xs, Ps, dPs) shaped like
    the filter's outputs. F = None is the random walk.
    """
    T, N = xf.shape
    xs = np.empty((T, N))
    Ps = np.empty((T, N, N))
    dPs = np.empty((T, N))
    xs[T - 1] = xf[T - 1]
    Ps[T - 1] = Pf[T - 1]
    dPs[T - 1] = np.diag(Pf[T - 1])
    for t in range(T - 2, -1, -1):
        A = smoother_gain(Pf[t], Q, F)                           # eqn11
        if F is None:
            x_next_pred = xf[t]                                  # eqn6, F = I
            P_next_pred = Pf[t] + Q                              # eqn7
        else:
            x_next_pred = F @ xf[t]                              # eqn6
            P_next_pred = F @ Pf[t] @ F.T + Q                    # eqn7
        xs[t] = xf[t] + A @ (xs[t + 1] - x_next_pred)            # eqn12 (RTS reading)
        Pst = Pf[t] + A @ (Ps[t + 1] - P_next_pred) @ A.T        # eqn13 (RTS reading)
        Ps[t] = (Pst + Pst.T) / 2.0
        dPs[t] = np.diag(Ps[t])
    return xs, Ps, dPs


def rts_step_columns(x_filt: np.ndarray, P_filt: np.ndarray, x_next_smooth: np.ndarray,
                     P_next_smooth: np.ndarray, Q: np.ndarray, cols):
    """One smoother step (eqn11-eqn13, RTS reading) at selected columns only.

    Returns x_{t|T} in full and the columns `cols` of P_{t|T}, from one Cholesky factorisation
    of P_{t+1|t} = P_{t|t} + Q and solves with single right-hand sides, so that large N is
    affordable: A_t v = P_{t|t} (P_{t+1|t}^{-1} v) and A_t^T e_i = P_{t+1|t}^{-1} P_{t|t} e_i.
    """
    P_next_pred = P_filt + Q                                     # eqn7
    c = _chol(P_next_pred)
    d = x_next_smooth - x_filt                                   # x_{t+1|T} - x_{t+1|t}, F = I
    xs = x_filt + P_filt @ sla.cho_solve(c, d)                   # eqn12 (RTS reading)
    D = P_next_smooth - P_next_pred
    cols = list(cols)
    At_e = sla.cho_solve(c, P_filt[:, cols])                     # A_t^T e_i, one column per i
    Pcols = P_filt[:, cols] + P_filt @ sla.cho_solve(c, D @ At_e)   # eqn13 (RTS reading)
    return xs, Pcols


def mne_solve(X, C, R, Y) -> np.ndarray:
    """eqn5 with the prior covariance C in place of lambda R: J_t = C X^T (X C X^T + R)^-1 y_t.

    Y is T x m; returns J as T x N.
    """
    X = np.asarray(X, dtype=np.float64)
    G = C @ X.T                                      # lambda R H^T
    S = X @ G + R                                    # lambda H R H^T + Sigma_eps
    Z = sla.cho_solve(_chol(S), np.asarray(Y, dtype=np.float64).T)
    return (G @ Z).T


def init_from_mne(X, C, R, Y, reg: float = 0.0):
    """Initial state and process-noise covariance from MNE estimates (Section 2.4).

    Reading: the initial state is the MNE estimate of the first data sample, and Sigma_w is
    the sample covariance (divisor T-2) of the differenced sequence J_k - J_{k-1}, k = 2..T,
    plus reg * I (the sample covariance has rank at most T-2). Returns (x0, Q).
    """
    J = mne_solve(X, C, R, Y)                        # eqn5 at every sample
    D = J[1:] - J[:-1]
    Dc = D - D.mean(axis=0)
    Q = Dc.T @ Dc / (D.shape[0] - 1)
    Q = (Q + Q.T) / 2.0
    Q = Q + reg * np.eye(Q.shape[0])
    return J[0].copy(), Q


def bf_smooth_means(X, Q, R, x0, P0, Y, F=None):
    """Smoothed means only, by the backward information recursion (modified Bryson-Frazier).

    Not in the paper: an alternative to eqn12 that reaches the same x_{t|T} without the
    smoother gain A_t, so without inverting P_{t+1|t}. With lambda_{T+1} = 0 and, going back,
        x_{t|T}  = x_{t|t} + P_{t|t} F^T lambda_{t+1}
        lambda_t = X^T S_t^-1 e_t + (I - K_t X)^T F^T lambda_{t+1}
    where e_t = y_t - X x_{t|t-1}, S_t and K_t are the innovation, its covariance and the
    gain of eqn8 at step t. (Substituting A_t P_{t+1|t} = P_{t|t} F^T into eqn12 gives the
    first line; the second follows from P_{t|t} = (I - K_t X) P_{t|t-1}.) The forward pass
    is the filter above, written out again so that e_t, S_t and K_t are at hand. F = None is
    the random walk. Returns (T, N).
    """
    X = np.asarray(X, dtype=np.float64)
    T = Y.shape[0]
    N = X.shape[1]
    Fm = np.eye(N) if F is None else np.asarray(F, dtype=np.float64)
    x = np.asarray(x0, dtype=np.float64).copy()
    P = np.asarray(P0, dtype=np.float64).copy()
    xf = np.empty((T, N))
    Pf, e, Sf, K = [], [], [], []
    for t in range(T):
        x_pred = Fm @ x                                # eqn6
        P_pred = Fm @ P @ Fm.T + Q                     # eqn7
        S = X @ P_pred @ X.T + R                       # bracket of eqn8
        cS = _chol(S)
        Kt = sla.cho_solve(cS, X @ P_pred).T           # eqn8
        et = Y[t] - X @ x_pred                         # innovation of eqn10
        x = x_pred + Kt @ et                           # eqn10
        P = P_pred - Kt @ X @ P_pred
        P = (P + P.T) / 2.0
        xf[t] = x
        Pf.append(P)
        e.append(et)
        Sf.append(cS)
        K.append(Kt)
    xs = np.empty((T, N))
    lam = np.zeros(N)
    for t in range(T - 1, -1, -1):
        mu = Fm.T @ lam
        xs[t] = xf[t] + Pf[t] @ mu
        lam = X.T @ sla.cho_solve(Sf[t], e[t]) + (np.eye(N) - K[t] @ X).T @ mu
    return xs
