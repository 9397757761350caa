"""Error measures shared by the GPU parity tests (normwise, per time step, max over steps)."""
import numpy as np
import torch


def to_np(t):
    return t.detach().cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t)


def eps_x(got, want):
    """max_t ||x^_t - x_t||_2 / max_s ||x_s||_2."""
    got, want = to_np(got), to_np(want)
    return float(np.linalg.norm(got - want, axis=1).max() / max(np.linalg.norm(want, axis=1).max(), 1e-300))


def eps_d(got, want):
    """max_t ||d^_t - d_t||_inf / ||d_t||_inf for the covariance diagonals."""
    got, want = to_np(got), to_np(want)
    return float((np.abs(got - want).max(axis=1) / np.maximum(np.abs(want).max(axis=1), 1e-300)).max())


def eps_P(got, want):
    """max_t ||P^_t - P_t||_F / ||P_t||_F."""
    got, want = to_np(got), to_np(want)
    if got.ndim == 2:
        got, want = got[None], want[None]
    num = np.sqrt(((got - want) ** 2).sum(axis=(1, 2)))
    den = np.sqrt((want ** 2).sum(axis=(1, 2)))
    return float((num / np.maximum(den, 1e-300)).max())


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def elem_rel(got, want, floor=1e-3):
    """Element-wise relative error, max over every element: |g - w| / (|w| + floor * max_i |w_t,i|),
    with the floor taken per time step (row) so that near-zero entries of a step are compared
    against that step's scale."""
    got, want = to_np(got), to_np(want)
    if got.ndim == 1:
        got, want = got[None], want[None]
    scale = np.abs(want).reshape(want.shape[0], -1).max(axis=1)
    scale = scale.reshape((-1,) + (1,) * (want.ndim - 1))
    return float((np.abs(got - want) / (np.abs(want) + floor * np.maximum(scale, 1e-300))).max())
