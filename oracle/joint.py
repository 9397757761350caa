"""Brute-force posteriors of the whole state sequence (test infrastructure only).

The filter and smoother of the paper compute the Gaussian posteriors
p(x_t | y_1..y_t) and p(x_t | y_1..y_T) (stated after eqn10 and after eqn13).
Here those posteriors are formed directly, with no recursion: stack
z = (x_1, ..., x_T), write down its Gaussian prior under the state model
(eqn3: x_t = F x_{t-1} + w_t, x_0 ~ N(x0, P0); for the random walk F = I,
E z_t = x0 and Cov(x_s, x_t) = P0 + min(s, t) Q), observe y = blockdiag(X) z + v
(eqn1, v ~ N(0, blockdiag(R))) and condition with dense linear algebra.

Two independent conditioning formulae are given (covariance form through an
LU solve, information form through explicit precisions) so that each pins the
other. Sizes: joint dimension T*N up to a few hundred.
"""
from __future__ import annotations

import numpy as np

__all__ = ["joint_prior", "joint_posterior", "joint_posterior_information"]


def joint_prior(Q, x0, P0, T, F=None):
    """Mean (T*N) and covariance (T*N x T*N) of the stacked state x_1..x_T.

    Random walk (F = None): E x_t = x0, Cov(x_s, x_t) = P0 + min(s, t) Q. With a
    transition F (eqn3, x_t = F x_{t-1} + w_t): E x_t = F^t x0 and
    Cov(x_s, x_t) = F^s P0 (F^t)^T + sum_{k=1..min(s,t)} F^(s-k) Q (F^(t-k))^T.
    """
    N = Q.shape[0]
    if F is None:
        mu = np.tile(np.asarray(x0, dtype=np.float64), T)
        Sig = np.empty((T * N, T * N))
        for s in range(T):
            for t in range(T):
                Sig[s * N:(s + 1) * N, t * N:(t + 1) * N] = P0 + (min(s, t) + 1) * Q
        return mu, Sig
    F = np.asarray(F, dtype=np.float64)
    Fp = [np.eye(N)]
    for _ in range(T):
        Fp.append(F @ Fp[-1])                      # Fp[k] = F^k
    mu = np.concatenate([Fp[t] @ np.asarray(x0, dtype=np.float64) for t in range(1, T + 1)])
    Sig = np.empty((T * N, T * N))
    for s in range(1, T + 1):
        for t in range(1, T + 1):
            C = Fp[s] @ P0 @ Fp[t].T
            for k in range(1, min(s, t) + 1):
                C = C + Fp[s - k] @ Q @ Fp[t - k].T
            Sig[(s - 1) * N:s * N, (t - 1) * N:t * N] = C
    return mu, Sig


def _blockdiag(B, T):
    r, c = B.shape
    out = np.zeros((T * r, T * c))
    for t in range(T):
        out[t * r:(t + 1) * r, t * c:(t + 1) * c] = B
    return out


def _condition_cov(mu, Sig, H, Rb, y):
    """Gaussian conditioning in covariance form: mean and covariance of z | y."""
    S = H @ Sig @ H.T + Rb
    G = np.linalg.solve(S, H @ Sig)           # S^-1 H Sig
    mean = mu + G.T @ (y - H @ mu)
    cov = Sig - Sig @ H.T @ np.linalg.solve(S, H @ Sig)
    return mean, cov


def _condition_info(mu, Sig, H, Rb, y):
    """Gaussian conditioning in information form: precision Sig^-1 + H^T Rb^-1 H."""
    Sinv = np.linalg.inv(Sig)
    Rinv = np.linalg.inv(Rb)
    Lam = Sinv + H.T @ Rinv @ H
    cov = np.linalg.inv(Lam)
    mean = cov @ (Sinv @ mu + H.T @ Rinv @ y)
    return mean, cov


def _posteriors(cond, X, Q, R, x0, P0, Y, F=None):
    X, Q, R = (np.asarray(a, dtype=np.float64) for a in (X, Q, R))
    Y = np.asarray(Y, dtype=np.float64)
    T, N = Y.shape[0], X.shape[1]
    mu, Sig = joint_prior(Q, x0, P0, T, F)
    Hfull = _blockdiag(X, T)
    Rfull = _blockdiag(R, T)
    xs = np.empty((T, N)); Ps = np.empty((T, N, N))
    xf = np.empty((T, N)); Pf = np.empty((T, N, N))
    mean, cov = cond(mu, Sig, Hfull, Rfull, Y.reshape(-1))
    for t in range(T):
        sl = slice(t * N, (t + 1) * N)
        xs[t] = mean[sl]
        Ps[t] = cov[sl, sl]
    for t in range(T):
        k = t + 1                                 # data y_1..y_k
        mean_k, cov_k = cond(mu, Sig, Hfull[:k * X.shape[0]], Rfull[:k * X.shape[0], :k * X.shape[0]],
                             Y[:k].reshape(-1))
        sl = slice(t * N, (t + 1) * N)
        xf[t] = mean_k[sl]
        Pf[t] = cov_k[sl, sl]
    return xf, Pf, xs, Ps


def joint_posterior(X, Q, R, x0, P0, Y, F=None):
    """(xf, Pf, xs, Ps): filtered and smoothed marginals by covariance-form conditioning."""
    return _posteriors(_condition_cov, X, Q, R, x0, P0, Y, F)


def joint_posterior_information(X, Q, R, x0, P0, Y, F=None):
    """Same marginals by information-form conditioning (explicit precision matrices)."""
    return _posteriors(_condition_info, X, Q, R, x0, P0, Y, F)
