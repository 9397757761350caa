"""Seeded synthetic inputs shaped like the paper's MEG workloads.

This module holds no part of the filter or smoother arithmetic: it only draws
geometry, the lead field, the noise covariances and data from the state-space
model (eqn1, eqn3 with F = I), so that the HIP path and the CPU oracle consume
the very same arrays.

The paper's own inputs (a subject MRI, a BEM lead field, Vectorview
recordings, empty-room noise; Sections 4.1 and 5) are not available, so every
workload here is synthetic with the paper's shapes: about 5,120 normal-oriented
cortical sources, 306 sensors (102 sites x 3 channels), 600 Hz sampling and
about 125 active sources in three regions (Section 4.1).

Recipes (the sizes and distributions of the five workloads):

* ``tiny`` (N=500, m=60, T=50): sources uniform in a ball of radius 0.07,
  sensors uniform on the upper hemisphere of radius 0.11, seeded unit source
  normals; a dipole-style lead field ``X[i, j] = n_j . (r_i - s_j) /
  |r_i - s_j|^3`` (sensor i at r_i, source j at s_j), scaled to unit Frobenius
  norm. Q = 1e-2 I, R = 1e-4 I, x0 = 0, P0 = I. Truth: five active sources
  doing a random walk with N(0, 1e-2) increments.
* ``paper`` (N=5124, m=306, T=200): sources on a spherical shell (uniform
  direction, radius U[0.06, 0.07]), the same lead field, a spatial Gaussian
  process covariance Q_jk = 1e-2 exp(-d_jk^2 / (2 * 0.01^2)); truth is three
  patches of the 42 sources nearest to three seeded centres with z > 0, each
  patch carrying sin(2 pi f t / 600 + phi) with f ~ U[10, 40] Hz; sensor noise
  R = sigma^2 I at an SNR of 5 dB (sigma^2 = mean (X x_t)^2 / 10^(5/10)).
* ``free`` (N=15372 = 5124 sites x 3 orientations): the ``paper`` sites, three
  lead-field columns per site (unit x, y, z dipoles, site-major column 3j+a, as
  J_{k,i} is a 3-vector in eqn1), Q = K (x) I_3 with the same Gaussian kernel
  K; each patch has one seeded orientation.
* ``serving``: a seeded stream of jobs with Poisson arrivals, each built like
  ``paper`` at its own N, m and T.
* ``neighbourhood``: the ``paper`` workload with the first-order neighbourhood
  model of eqn2 as the transition F of eqn3: each source keeps (1 - beta) of its
  own previous value and takes beta/6 of each of its six nearest sources
  (beta = 0.5). Reading: eqn2 as printed adds the neighbour mean to the full
  previous value, which makes F's spectral radius about 2 (an exploding
  process); its mask weights are read as this normalisation, so that F is row
  stochastic (a stable averaging process; F = I at beta = 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "tiny", "paper", "free", "custom", "serving_jobs", "random_spd",
    "small_random",
]


@dataclass
class Problem:
    """One filter/smoother workload: float64 arrays, row-major."""

    name: str
    X: np.ndarray          # m x N lead field
    Q: np.ndarray          # N x N process-noise covariance
    R: np.ndarray          # m x m sensor-noise covariance
    x0: np.ndarray         # N initial mean
    P0: np.ndarray         # N x N initial covariance
    Y: np.ndarray          # T x m data
    truth: np.ndarray | None = None   # T x N simulated sources (not used by the path)
    meta: dict = field(default_factory=dict)
    F: tuple | None = None            # transition of eqn3 as CSR (row_ptr, col_idx, val); None = identity

    def F_dense(self) -> np.ndarray | None:
        return None if self.F is None else csr_to_dense(*self.F, self.N)

    @property
    def N(self) -> int:
        return self.X.shape[1]

    @property
    def m(self) -> int:
        return self.X.shape[0]

    @property
    def T(self) -> int:
        return self.Y.shape[0]


def _rngs(seed: int, n: int) -> list[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def _unit(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _hemisphere(rng: np.random.Generator, m: int, radius: float = 0.11) -> np.ndarray:
    v = _unit(rng, m)
    v[:, 2] = np.abs(v[:, 2])
    return radius * v


def _ball(rng: np.random.Generator, n: int, radius: float = 0.07) -> np.ndarray:
    return _unit(rng, n) * (radius * rng.uniform(size=n) ** (1.0 / 3.0))[:, None]


def _shell(rng: np.random.Generator, n: int, r0: float = 0.06, r1: float = 0.07) -> np.ndarray:
    return _unit(rng, n) * rng.uniform(r0, r1, size=n)[:, None]


def _lead_field(sensors: np.ndarray, sources: np.ndarray, normals: np.ndarray) -> np.ndarray:
    """Dipole-style lead field, one column per (source, normal) pair, unit Frobenius norm."""
    diff = sensors[:, None, :] - sources[None, :, :]          # m x N x 3
    dist3 = np.linalg.norm(diff, axis=2) ** 3
    X = np.einsum("mnk,nk->mn", diff, normals) / dist3
    return np.ascontiguousarray(X / np.linalg.norm(X))


def gaussian_kernel(points: np.ndarray, q: float = 1e-2, length: float = 0.01,
                    chunk: int = 1024) -> np.ndarray:
    """q * exp(-d^2 / (2 length^2)); built from explicit differences so it is exactly symmetric."""
    n = points.shape[0]
    K = np.empty((n, n))
    for a in range(0, n, chunk):
        d = points[a:a + chunk, None, :] - points[None, :, :]
        K[a:a + chunk] = np.exp(-np.einsum("ijk,ijk->ij", d, d) / (2.0 * length * length))
    K *= q
    return K


def _observe(rng: np.random.Generator, X: np.ndarray, truth: np.ndarray, sigma2: float) -> np.ndarray:
    T, m = truth.shape[0], X.shape[0]
    return truth @ X.T + math.sqrt(sigma2) * rng.normal(size=(T, m))


def _patch_truth(rng: np.random.Generator, sites: np.ndarray, T: int, n_patches: int = 3,
                 per_patch: int = 42, fs: float = 600.0):
    """Three patches of nearest sources with sinusoidal 10-40 Hz time courses."""
    upper = np.flatnonzero(sites[:, 2] > 0)
    centres = rng.choice(upper, size=n_patches, replace=False)
    t = np.arange(1, T + 1)
    members, courses = [], []
    for c in centres:
        d = np.linalg.norm(sites - sites[c], axis=1)
        members.append(np.argsort(d, kind="stable")[:per_patch])
        f = rng.uniform(10.0, 40.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        courses.append(np.sin(2.0 * math.pi * f * t / fs + phi))
    return members, courses


def _sigma2_at_snr(X: np.ndarray, truth: np.ndarray, snr_db: float) -> float:
    signal = truth @ X.T
    return float(np.mean(signal * signal) / 10.0 ** (snr_db / 10.0))


def tiny(seed: int = 1, N: int = 500, m: int = 60, T: int = 50) -> Problem:
    """N=500 sources in a ball, m=60 sensors, T=50; random-walk truth with 5 active sources."""
    g_src, g_nrm, g_sen, g_act, g_walk, g_noise = _rngs(seed, 6)
    sources = _ball(g_src, N)
    normals = _unit(g_nrm, N)
    sensors = _hemisphere(g_sen, m)
    X = _lead_field(sensors, sources, normals)
    q, r = 1e-2, 1e-4
    active = g_act.choice(N, size=min(5, N), replace=False)
    truth = np.zeros((T, N))
    truth[:, active] = np.cumsum(g_walk.normal(scale=math.sqrt(q), size=(T, active.size)), axis=0)
    Y = _observe(g_noise, X, truth, r)
    return Problem("tiny", X, q * np.eye(N), r * np.eye(m), np.zeros(N), np.eye(N), Y, truth,
                   {"seed": seed, "active": active})


def paper(seed: int = 2, N: int = 5124, m: int = 306, T: int = 200, snr_db: float = 5.0) -> Problem:
    """Paper-scale fixed-orientation workload (N=5124 shell sources, m=306, T=200, 5 dB)."""
    g_src, g_nrm, g_sen, g_patch, g_noise = _rngs(seed, 5)
    sites = _shell(g_src, N)
    normals = _unit(g_nrm, N)
    sensors = _hemisphere(g_sen, m)
    X = _lead_field(sensors, sites, normals)
    Q = gaussian_kernel(sites)
    members, courses = _patch_truth(g_patch, sites, T)
    truth = np.zeros((T, N))
    for idx, course in zip(members, courses):
        truth[:, idx] = course[:, None]
    sigma2 = _sigma2_at_snr(X, truth, snr_db)
    Y = _observe(g_noise, X, truth, sigma2)
    return Problem("paper", X, Q, sigma2 * np.eye(m), np.zeros(N), np.eye(N), Y, truth,
                   {"seed": seed, "sigma2": sigma2, "snr_db": snr_db})


def free(seed: int = 4, sites_n: int = 5124, m: int = 306, T: int = 100,
         snr_db: float = 5.0) -> Problem:
    """Free-orientation workload: 3 dipole columns per site (N = 3 * sites_n), Q = K (x) I3."""
    g_src, g_sen, g_patch, g_orient, g_noise = _rngs(seed, 5)
    sites = _shell(g_src, sites_n)
    sensors = _hemisphere(g_sen, m)
    N = 3 * sites_n
    src3 = np.repeat(sites, 3, axis=0)                       # column 3j + a -> site j
    nrm3 = np.tile(np.eye(3), (sites_n, 1))                  # orientation e_a
    X = _lead_field(sensors, src3, nrm3)
    K = gaussian_kernel(sites)
    Q = np.zeros((N, N))
    for a in range(3):
        Q[a::3, a::3] = K
    members, courses = _patch_truth(g_patch, sites, T)
    truth = np.zeros((T, N))
    for idx, course in zip(members, courses):
        o = _unit(g_orient, 1)[0]
        for a in range(3):
            truth[:, 3 * idx + a] = course[:, None] * o[a]
    sigma2 = _sigma2_at_snr(X, truth, snr_db)
    Y = _observe(g_noise, X, truth, sigma2)
    return Problem("free", X, Q, sigma2 * np.eye(m), np.zeros(N), np.eye(N), Y, truth,
                   {"seed": seed, "sigma2": sigma2, "snr_db": snr_db})


def custom(seed: int, N: int, m: int, T: int, snr_db: float = 5.0) -> Problem:
    """``paper`` construction at an arbitrary (N, m, T) (used for serving jobs and sweeps)."""
    p = paper(seed=seed, N=N, m=m, T=T, snr_db=snr_db)
    p.name = f"custom_N{N}_m{m}_T{T}"
    return p


def random_spd(rng: np.random.Generator, n: int, cond: float = 10.0, scale: float = 1.0) -> np.ndarray:
    """Random symmetric positive definite matrix with eigenvalues log-spaced in [scale/cond, scale]."""
    U, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = scale * np.logspace(-math.log10(cond), 0.0, n)
    A = (U * ev) @ U.T
    return (A + A.T) / 2.0


def small_random(seed: int, N: int, m: int, T: int, cond: float = 10.0) -> Problem:
    """Dense random SPD Q, R, P0 and a random X (tiny sizes for brute-force checks)."""
    g = _rngs(seed, 7)
    X = g[0].normal(size=(m, N))
    Q = random_spd(g[1], N, cond, 0.5)
    R = random_spd(g[2], m, cond, 0.3)
    P0 = random_spd(g[3], N, cond, 1.0)
    x0 = g[4].normal(size=N)
    Y = g[5].normal(size=(T, m))
    return Problem(f"small_N{N}_m{m}_T{T}", X, Q, R, x0, P0, Y, None, {"seed": seed})


def serving_jobs(seed: int = 5, n_jobs: int = 64, rate_per_s: float = 4.0,
                 N_choices=(2000, 5124, 8196, 15372), m_choices=(102, 204, 306),
                 T_range=(50, 400)) -> list[dict]:
    """Arrival times (Poisson, mean inter-arrival 1/rate) and (N, m, T, seed) per job.

    Arrays are built lazily with ``custom(**job_shape)`` since the full stream
    is far larger than host memory.
    """
    g_arr, g_shape = _rngs(seed, 2)
    gaps = g_arr.exponential(1.0 / rate_per_s, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for j in range(n_jobs):
        jobs.append({
            "job": j,
            "arrival_s": float(arrivals[j]),
            "N": int(g_shape.choice(N_choices)),
            "m": int(g_shape.choice(m_choices)),
            "T": int(g_shape.integers(T_range[0], T_range[1] + 1)),
            "seed": int(seed * 1000 + j),
        })
    return jobs


def neighbourhood_transition(points: np.ndarray, k: int = 6, beta: float = 0.5, chunk: int = 1024):
    """CSR (row_ptr int32, col_idx int32, val float64) of F = (1 - beta) I + beta/k A_k, where row p of
    A_k has ones at the k sources nearest to source p (eqn2 with its mask read as a normalisation)."""
    n = points.shape[0]
    nbr = np.empty((n, k), dtype=np.int64)
    sq = (points ** 2).sum(axis=1)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        d2 = sq[a:b, None] + sq[None, :] - 2.0 * points[a:b] @ points.T
        d2[np.arange(b - a), np.arange(a, b)] = np.inf          # not its own neighbour
        idx = np.argpartition(d2, k, axis=1)[:, :k]
        nbr[a:b] = np.sort(idx, axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for p in range(n):
        entries = {p: 1.0 - beta}
        for q in nbr[p]:
            entries[int(q)] = entries.get(int(q), 0.0) + beta / k
        cs = sorted(entries)
        cols.extend(cs)
        vals.extend(entries[c] for c in cs)
        row_ptr[p + 1] = len(cols)
    return row_ptr, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64)


def dense_to_csr(F: np.ndarray):
    """CSR of a dense matrix (explicit zeros dropped)."""
    n = F.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(F[i])[0]
        cols.extend(nz.tolist())
        vals.extend(F[i, nz].tolist())
        row_ptr[i + 1] = len(cols)
    return row_ptr, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64)


def csr_to_dense(row_ptr, col_idx, val, n: int) -> np.ndarray:
    F = np.zeros((n, n))
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            F[i, col_idx[e]] += val[e]
    return F


def neighbourhood(seed: int = 2, N: int = 5124, m: int = 306, T: int = 200, beta: float = 0.5,
                  snr_db: float = 5.0) -> Problem:
    """``paper`` workload with the six-neighbour transition of eqn2 (see the module notes)."""
    p = paper(seed=seed, N=N, m=m, T=T, snr_db=snr_db)
    g_src = _rngs(seed, 5)[0]
    sites = _shell(g_src, N)                     # the same draw as in ``paper``
    p.F = neighbourhood_transition(sites, 6, beta)
    p.name = f"neighbourhood_N{N}_m{m}_T{T}"
    p.meta["beta"] = beta
    return p


def small_random_F(seed: int, N: int, m: int, T: int, density: float = 1.0, radius: float = 0.9) -> Problem:
    """``small_random`` with a random transition F (spectral radius ``radius``; a fraction
    ``density`` of off-diagonal entries kept)."""
    p = small_random(seed, N, m, T)
    g = _rngs(seed + 1000, 2)
    F = g[0].normal(size=(N, N))
    if density < 1.0:
        keep = g[1].random(size=(N, N)) < density
        np.fill_diagonal(keep, True)
        F = F * keep
    rho = max(abs(np.linalg.eigvals(F))) if N > 0 else 1.0
    F = F * (radius / rho)
    p.F = dense_to_csr(F)
    p.name = f"smallF_N{N}_m{m}_T{T}"
    return p
