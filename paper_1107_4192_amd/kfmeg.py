"""Thin ctypes binding of the kfmeg C ABI (``include/kfmeg.h``).

Argument marshalling only: every step of the filter, smoother and MNE runs in
the HIP library. torch supplies device memory and the stream. There is no CPU
fallback: if the library is not built, or no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfmeg.so")

KF_OK, KF_EINVAL, KF_ENOTPD, KF_ENOMEM, KF_EHIP, KF_ESTATE, KF_ECANCELED = range(7)
KF_FP64, KF_MIXED = 0, 1
_STATUS = {0: "KF_OK", 1: "KF_EINVAL", 2: "KF_ENOTPD", 3: "KF_ENOMEM", 4: "KF_EHIP", 5: "KF_ESTATE",
           6: "KF_ECANCELED"}

# Every function the header declares; a CPU test checks the library exports them all.
EXPORTS = ("kf_default_options", "kf_create", "kf_filter", "kf_smooth", "kf_get_filtered_cov",
           "mne_solve", "kf_destroy", "kf_last_error", "kf_plan_bytes", "kfd_gemm", "kfd_chol_inv", "kf_set_profiling", "kf_get_profile",
           "kfs_create", "kfs_submit", "kfs_wait", "kfs_job_info", "kfs_get_stats", "kfs_last_error",
           "kfs_destroy", "kf_init_from_mne", "kf_filter_batch", "kf_smooth_batch", "kfd_gemm_tail", "kf_smooth_means",
           "kf_smooth_means_batch", "kfs_cancel",
           "kf_set_transition", "kf_smooth_assoc", "kf_smooth_assoc_bytes", "mne_solve_noalloc", "kfd_spd_solve")


class KFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class kfs_stats(ctypes.Structure):
    _fields_ = [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("jobs_per_s", ctypes.c_double), ("steps_per_s", ctypes.c_double),
                ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("checkpointed", ctypes.c_int64), ("peak_bytes", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t), ("max_concurrent", ctypes.c_int), ("canceled", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class kf_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("store_fp32", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t), ("checkpoint_stride", ctypes.c_int),
                ("keep_gain_factors", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libkfmeg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1107_4192_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    lib.kf_default_options.argtypes = [ctypes.POINTER(kf_options)]
    lib.kf_default_options.restype = None
    lib.kf_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, dp, dp, dp, dp, dp,
                              ctypes.POINTER(kf_options), vp]
    lib.kf_create.restype = ctypes.c_int
    lib.kf_filter.argtypes = [vp, i64, dp, dp, dp]
    lib.kf_filter.restype = ctypes.c_int
    lib.kf_smooth.argtypes = [vp, dp, dp, dp]
    lib.kf_smooth.restype = ctypes.c_int
    lib.kf_smooth_assoc.argtypes = [vp, dp, dp, dp]
    lib.kf_smooth_assoc.restype = ctypes.c_int
    lib.kf_set_transition.argtypes = [vp, i64, dp, dp, dp]
    lib.kf_set_transition.restype = ctypes.c_int
    lib.kf_smooth_means.argtypes = [vp, dp]
    lib.kf_smooth_means.restype = ctypes.c_int
    lib.kf_smooth_means_batch.argtypes = [vp, i64, dp]
    lib.kf_smooth_means_batch.restype = ctypes.c_int
    lib.kf_filter_batch.argtypes = [vp, i64, i64, dp, dp, dp]
    lib.kf_filter_batch.restype = ctypes.c_int
    lib.kf_smooth_batch.argtypes = [vp, i64, dp, dp, dp]
    lib.kf_smooth_batch.restype = ctypes.c_int
    lib.kf_get_filtered_cov.argtypes = [vp, i64, dp]
    lib.kf_get_filtered_cov.restype = ctypes.c_int
    lib.mne_solve.argtypes = [i64, i64, i64, dp, dp, dp, dp, dp, vp]
    lib.mne_solve.restype = ctypes.c_int
    lib.mne_solve_noalloc.argtypes = [i64, i64, i64, dp, dp, dp, dp, dp, vp]
    lib.mne_solve_noalloc.restype = ctypes.c_int
    lib.kf_destroy.argtypes = [vp]
    lib.kf_destroy.restype = None
    lib.kf_last_error.argtypes = [vp]
    lib.kf_last_error.restype = ctypes.c_char_p
    lib.kf_plan_bytes.argtypes = [i64, i64, i64, ctypes.POINTER(kf_options)]
    lib.kf_plan_bytes.restype = ctypes.c_size_t
    lib.kf_smooth_assoc_bytes.argtypes = [i64, i64]
    lib.kf_smooth_assoc_bytes.restype = ctypes.c_size_t
    lib.kf_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.kf_set_profiling.restype = ctypes.c_int
    lib.kf_get_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    lib.kf_get_profile.restype = ctypes.c_int
    lib.kf_init_from_mne.argtypes = [i64, i64, i64, dp, dp, dp, dp, ctypes.c_double, dp, dp, vp]
    lib.kf_init_from_mne.restype = ctypes.c_int
    lib.kfs_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(kf_options)]
    lib.kfs_create.restype = ctypes.c_int
    lib.kfs_submit.argtypes = [vp, i64, i64, i64, dp, dp, dp, dp, dp, dp, dp, dp, vp, ctypes.POINTER(i64)]
    lib.kfs_submit.restype = ctypes.c_int
    lib.kfs_wait.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    lib.kfs_wait.restype = ctypes.c_int
    lib.kfs_cancel.argtypes = [vp, i64]
    lib.kfs_cancel.restype = ctypes.c_int
    lib.kfs_job_info.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.kfs_job_info.restype = ctypes.c_int
    lib.kfs_get_stats.argtypes = [vp, ctypes.POINTER(kfs_stats)]
    lib.kfs_get_stats.restype = ctypes.c_int
    lib.kfs_last_error.argtypes = [vp]
    lib.kfs_last_error.restype = ctypes.c_char_p
    lib.kfs_destroy.argtypes = [vp]
    lib.kfs_destroy.restype = None
    lib.kfd_gemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, i64, dp,
                             i64, ctypes.c_double, ctypes.c_double, dp, i64, dp, i64, ctypes.c_int, vp]
    lib.kfd_gemm.restype = ctypes.c_int
    lib.kfd_gemm_tail.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, i64, dp,
                                  i64, ctypes.c_double, ctypes.c_double, dp, i64, dp, i64, ctypes.c_int, ctypes.c_int,
                                  vp]
    lib.kfd_gemm_tail.restype = ctypes.c_int
    lib.kfd_chol_inv.argtypes = [ctypes.c_int, dp, i64, dp, i64, ctypes.POINTER(ctypes.c_int), vp]
    lib.kfd_chol_inv.restype = ctypes.c_int
    lib.kfd_spd_solve.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, dp, i64, dp, i64, ctypes.POINTER(ctypes.c_int),
                                  vp]
    lib.kfd_spd_solve.restype = ctypes.c_int
    _lib = lib
    return lib


def _need_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("kfmeg needs a ROCm GPU (gfx950); none is visible")


def _dev(t: torch.Tensor, name: str, shape) -> int:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(lib, st: int, plan=None):
    if st != KF_OK:
        msg = lib.kf_last_error(plan)
        raise KFError(st, msg.decode() if msg else "")


def options(precision: int = KF_FP64, store_fp32: bool = False, hbm_budget_bytes: int = 0,
            checkpoint_stride: int = 0, keep_gain_factors: bool = False) -> kf_options:
    return kf_options(int(precision), int(bool(store_fp32)), int(hbm_budget_bytes), int(checkpoint_stride),
                      int(bool(keep_gain_factors)))


def kf_plan_bytes(N: int, m: int, T: int, opt: kf_options | None = None) -> int:
    lib = load_library()
    return int(lib.kf_plan_bytes(N, m, T, ctypes.byref(opt) if opt is not None else None))


def kf_smooth_assoc_bytes(N: int, T: int) -> int:
    """Device bytes kf_smooth_assoc allocates for one call after a filter run over T steps."""
    return int(load_library().kf_smooth_assoc_bytes(N, T))


def kf_create(N, m, T_max, X, Q, R, x0, P0, opt: kf_options | None = None, stream=None) -> int:
    """Returns an opaque plan handle (int)."""
    lib = load_library()
    _need_gpu()
    ptrs = [_dev(X, "X", (m, N)), _dev(Q, "Q", (N, N)), _dev(R, "R", (m, m)), _dev(x0, "x0", (N,)),
            _dev(P0, "P0", (N, N))]
    h = ctypes.c_void_p()
    st = lib.kf_create(ctypes.byref(h), N, m, T_max, *ptrs,
                       ctypes.byref(opt) if opt is not None else None, _stream_ptr(stream))
    _check(lib, st, None)
    return h.value


def kf_filter(plan: int, Y, x_filt, Pdiag_filt=None) -> None:
    lib = load_library()
    T, m = Y.shape
    N = x_filt.shape[1]
    st = lib.kf_filter(plan, T, _dev(Y, "Y", (T, m)), _dev(x_filt, "x_filt", (T, N)),
                       _dev(Pdiag_filt, "Pdiag_filt", (T, N)) if Pdiag_filt is not None else None)
    _check(lib, st, plan)


def kf_smooth(plan: int, x_smooth, Pdiag_smooth=None, P_smooth=None) -> None:
    lib = load_library()
    T, N = x_smooth.shape
    st = lib.kf_smooth(plan, _dev(x_smooth, "x_smooth", (T, N)),
                       _dev(Pdiag_smooth, "Pdiag_smooth", (T, N)) if Pdiag_smooth is not None else None,
                       _dev(P_smooth, "P_smooth", (T, N, N)) if P_smooth is not None else None)
    _check(lib, st, plan)


def kf_filter_batch(plan: int, Y, x_filt, Pdiag_filt=None) -> None:
    """Y: (B, T, m), x_filt: (B, T, N); the covariance pass is shared by the B data sets."""
    lib = load_library()
    B, T, m = Y.shape
    N = x_filt.shape[2]
    st = lib.kf_filter_batch(plan, B, T, _dev(Y, "Y", (B, T, m)), _dev(x_filt, "x_filt", (B, T, N)),
                             _dev(Pdiag_filt, "Pdiag_filt", (T, N)) if Pdiag_filt is not None else None)
    _check(lib, st, plan)


def kf_smooth_batch(plan: int, x_smooth, Pdiag_smooth=None, P_smooth=None) -> None:
    lib = load_library()
    B, T, N = x_smooth.shape
    st = lib.kf_smooth_batch(plan, B, _dev(x_smooth, "x_smooth", (B, T, N)),
                             _dev(Pdiag_smooth, "Pdiag_smooth", (T, N)) if Pdiag_smooth is not None else None,
                             _dev(P_smooth, "P_smooth", (T, N, N)) if P_smooth is not None else None)
    _check(lib, st, plan)


def kf_set_transition(plan: int, F) -> None:
    """F: None (random walk) or a CSR triple (row_ptr int32, col_idx int32, val float64), numpy or device."""
    lib = load_library()
    if F is None:
        _check(lib, lib.kf_set_transition(plan, 0, None, None, None), plan)
        return
    rp, ci, v = (torch.as_tensor(a).to("cuda").contiguous() for a in F)
    if rp.dtype != torch.int32 or ci.dtype != torch.int32 or v.dtype != torch.float64:
        raise TypeError("F: row_ptr and col_idx must be int32, val float64")
    _check(lib, lib.kf_set_transition(plan, int(ci.numel()), rp.data_ptr(), ci.data_ptr(), v.data_ptr()), plan)


def kf_smooth_assoc(plan: int, x_smooth, Pdiag_smooth=None, P_smooth=None) -> None:
    """Smoother as an associative scan over time (same outputs as kf_smooth; consumes the stored P_{t|t})."""
    lib = load_library()
    T, N = x_smooth.shape
    st = lib.kf_smooth_assoc(plan, _dev(x_smooth, "x_smooth", (T, N)),
                             _dev(Pdiag_smooth, "Pdiag_smooth", (T, N)) if Pdiag_smooth is not None else None,
                             _dev(P_smooth, "P_smooth", (T, N, N)) if P_smooth is not None else None)
    _check(lib, st, plan)


def kf_smooth_means(plan: int, x_smooth) -> None:
    """Smoothed means only (backward information recursion); x_smooth (T, N) or (B, T, N)."""
    lib = load_library()
    if x_smooth.dim() == 2:
        st = lib.kf_smooth_means(plan, _dev(x_smooth, "x_smooth", tuple(x_smooth.shape)))
    else:
        st = lib.kf_smooth_means_batch(plan, x_smooth.shape[0], _dev(x_smooth, "x_smooth", tuple(x_smooth.shape)))
    _check(lib, st, plan)


def kf_get_filtered_cov(plan: int, t: int, P_out) -> None:
    lib = load_library()
    N = P_out.shape[0]
    st = lib.kf_get_filtered_cov(plan, t, _dev(P_out, "P_out", (N, N)))
    _check(lib, st, plan)


def kf_set_profiling(plan: int, on) -> None:
    """on: False/0 off, True/1 event-time the smoother's N x N x N products, 2 the same with the
    smoother serialised onto the plan's stream (each product runs alone)."""
    lib = load_library()
    _check(lib, lib.kf_set_profiling(plan, int(on)), plan)


def kf_get_profile(plan: int):
    """(kernel_ms, kernel_flops, launches) of the smoother's N x N x N products since profiling was enabled."""
    lib = load_library()
    ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib, lib.kf_get_profile(plan, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)), plan)
    return ms.value, fl.value, n.value


def kf_destroy(plan: int) -> None:
    if plan:
        load_library().kf_destroy(plan)


def mne_solve(X, C, R, Y, J=None, stream=None):
    """J_t = C X^T (X C X^T + R)^-1 y_t for every row of Y (eqn5). Returns J (T x N)."""
    lib = load_library()
    _need_gpu()
    m, N = X.shape
    T = Y.shape[0]
    if J is None:
        J = torch.empty((T, N), dtype=torch.float64, device=X.device)
    st = lib.mne_solve(N, m, T, _dev(X, "X", (m, N)), _dev(C, "C", (N, N)), _dev(R, "R", (m, m)),
                       _dev(Y, "Y", (T, m)), _dev(J, "J", (T, N)), _stream_ptr(stream))
    _check(lib, st, None)
    return J


def mne_solve_noalloc(X, C, R, Y, J, stream=None):
    """mne_solve without device allocation: the workspace is the library's fixed 64 MiB array.
    J (T x N) must be given; calls that overlap on one GPU race (see kfmeg.h)."""
    lib = load_library()
    _need_gpu()
    m, N = X.shape
    T = Y.shape[0]
    st = lib.mne_solve_noalloc(N, m, T, _dev(X, "X", (m, N)), _dev(C, "C", (N, N)), _dev(R, "R", (m, m)),
                               _dev(Y, "Y", (T, m)), _dev(J, "J", (T, N)), _stream_ptr(stream))
    _check(lib, st, None)
    return J


def kf_init_from_mne(X, C, R, Y, reg: float = 0.0, stream=None):
    """Section 2.4 set-up: (x0, Q) from MNE estimates of every sample of Y."""
    lib = load_library()
    _need_gpu()
    m, N = X.shape
    T = Y.shape[0]
    x0 = torch.empty(N, dtype=torch.float64, device=X.device)
    Q = torch.empty((N, N), dtype=torch.float64, device=X.device)
    st = lib.kf_init_from_mne(N, m, T, _dev(X, "X", (m, N)), _dev(C, "C", (N, N)), _dev(R, "R", (m, m)),
                              _dev(Y, "Y", (T, m)), float(reg), x0.data_ptr(), Q.data_ptr(), _stream_ptr(stream))
    _check(lib, st, None)
    return x0, Q


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching server (kfs_* in kfmeg.h). submit() returns a job id; the
    tensors handed to a job must stay alive until wait() for it returns."""

    def __init__(self, hbm_budget_bytes: int = 0, max_active: int = 4, precision: int = KF_FP64,
                 store_fp32: bool = False):
        lib = load_library()
        _need_gpu()
        self._lib = lib
        self._keep = {}
        h = ctypes.c_void_p()
        opt = options(precision, store_fp32)
        st = lib.kfs_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_active), ctypes.byref(opt))
        if st != KF_OK:
            raise KFError(st, "kfs_create failed")
        self.h = h.value

    def submit(self, X, Q, R, x0, P0, Y, want_diag: bool = True, stream=None):
        """Queue one filter + smoother job. Its work is ordered after everything already enqueued
        on `stream` (default: the current torch stream), where the inputs may still be produced."""
        m, N = X.shape
        T = Y.shape[0]
        xs = torch.empty((T, N), dtype=torch.float64, device=X.device)
        ds = torch.empty((T, N), dtype=torch.float64, device=X.device) if want_diag else None
        jid = ctypes.c_int64()
        st = self._lib.kfs_submit(self.h, N, m, T, _dev(X, "X", (m, N)), _dev(Q, "Q", (N, N)),
                                  _dev(R, "R", (m, m)), _dev(x0, "x0", (N,)), _dev(P0, "P0", (N, N)),
                                  _dev(Y, "Y", (T, m)), xs.data_ptr(), ds.data_ptr() if ds is not None else None,
                                  _stream_ptr(stream), ctypes.byref(jid))
        if st != KF_OK:
            raise KFError(st, "kfs_submit failed")
        self._keep[jid.value] = (X, Q, R, x0, P0, Y, xs, ds)
        return jid.value

    def wait(self, job_id: int):
        """Block until the job is done: returns (x_smooth, Pdiag_smooth, latency_ms)."""
        lat = ctypes.c_double()
        st = self._lib.kfs_wait(self.h, job_id, ctypes.byref(lat))
        bufs = self._keep.pop(job_id)
        if st != KF_OK:
            msg = self._lib.kfs_last_error(self.h)
            raise KFError(st, msg.decode() if msg else "")
        return bufs[6], bufs[7], lat.value

    def cancel(self, job_id: int) -> bool:
        """Remove a job that has not started; False if it is already running or done."""
        st = self._lib.kfs_cancel(self.h, job_id)
        if st == KF_ESTATE:
            return False
        _check(self._lib, st)
        return True

    def info(self, job_id: int) -> dict:
        d, s, q, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib, self._lib.kfs_job_info(self.h, job_id, ctypes.byref(d), ctypes.byref(s), ctypes.byref(q),
                                                 ctypes.byref(r)))
        return {"done": bool(d.value), "checkpoint_stride": s.value, "queued_ms": q.value, "run_ms": r.value}

    def stats(self) -> dict:
        out = kfs_stats()
        _check(self._lib, self._lib.kfs_get_stats(self.h, ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self._lib.kfs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- kernel-level hooks (tests)
G_TA, G_TB, G_LOWER, G_MIRROR, G_ALOWER, G_BLOWER, G_BUPPER = 1, 2, 4, 8, 16, 32, 64
G_AUPPER = 8192


def kfd_gemm(A, B, M, N, K, flags=0, alpha=1.0, beta=0.0, Cin=None, C=None, ksplit=1, stream=None):
    """C = alpha op(A) op(B) + beta Cin on the MFMA path (A, B float64 or float32; C float64)."""
    lib = load_library()
    dtype = 0 if A.dtype == torch.float64 else 1
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float64, device=A.device)
    st = lib.kfd_gemm(dtype, M, N, K, flags, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), alpha, beta,
                      Cin.data_ptr() if Cin is not None else None, Cin.stride(0) if Cin is not None else 0,
                      C.data_ptr(), C.stride(0), ksplit, _stream_ptr(stream))
    if st != 0:
        raise KFError(st, "kfd_gemm failed")
    return C


def kfd_gemm_tail(A, B, M, N, K, flags=0, alpha=1.0, beta=0.0, Cin=None, C=None, full=0, k=2, stream=None):
    """kfd_gemm with the first `full` tiles whole and the rest split k ways along K."""
    lib = load_library()
    dtype = 0 if A.dtype == torch.float64 else 1
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float64, device=A.device)
    st = lib.kfd_gemm_tail(dtype, M, N, K, flags, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), alpha, beta,
                           Cin.data_ptr() if Cin is not None else None, Cin.stride(0) if Cin is not None else 0,
                           C.data_ptr(), C.stride(0), full, k, _stream_ptr(stream))
    if st != 0:
        raise KFError(st, "kfd_gemm_tail failed")
    return C


def kfd_chol_inv(W, Z=None, stream=None):
    """In place: W <- L (lower), returns Z = L^-1. Raises KFError(KF_ENOTPD) with the pivot row."""
    lib = load_library()
    n = W.shape[0]
    if Z is None:
        Z = torch.empty_like(W)
    piv = ctypes.c_int(-1)
    st = lib.kfd_chol_inv(n, W.data_ptr(), W.stride(0), Z.data_ptr(), Z.stride(0), ctypes.byref(piv),
                          _stream_ptr(stream))
    if st != 0:
        raise KFError(st, f"kfd_chol_inv failed (pivot row {piv.value})")
    return Z


def kfd_spd_solve(W, B, nb: int, X=None, stream=None):
    """X = A^-1 B with A in the lower triangle of W (overwritten by its factor L) by the smoother gain's
    outer-blocked Cholesky (block width nb) and blocked solves. Raises KFError(KF_ENOTPD) with the pivot row."""
    lib = load_library()
    n = W.shape[0]
    if X is None:
        X = torch.empty((n, n), dtype=torch.float64, device=W.device)
    piv = ctypes.c_int(-1)
    st = lib.kfd_spd_solve(n, nb, W.data_ptr(), W.stride(0), B.data_ptr(), B.stride(0), X.data_ptr(), X.stride(0),
                           ctypes.byref(piv), _stream_ptr(stream))
    if st != 0:
        raise KFError(st, f"kfd_spd_solve failed (pivot row {piv.value})")
    return X


@dataclass
class Result:
    x_filt: torch.Tensor
    Pdiag_filt: torch.Tensor | None
    x_smooth: torch.Tensor | None = None
    Pdiag_smooth: torch.Tensor | None = None
    P_smooth: torch.Tensor | None = None


class KalmanSmoother:
    """Convenience wrapper owning one plan: ``run(Y)`` = kf_filter + kf_smooth."""

    def __init__(self, X, Q, R, x0, P0, T_max: int, precision: int = KF_FP64, store_fp32: bool = False,
                 hbm_budget_bytes: int = 0, checkpoint_stride: int = 0, keep_gain_factors: bool = False,
                 F=None, stream=None):
        self.m, self.N = X.shape
        self.T_max = T_max
        self.opt = options(precision, store_fp32, hbm_budget_bytes, checkpoint_stride, keep_gain_factors)
        self.plan = kf_create(self.N, self.m, T_max, X, Q, R, x0, P0, self.opt, stream)
        if F is not None:
            try:
                kf_set_transition(self.plan, F)
            except Exception:
                self.close()
                raise

    def filter(self, Y, want_diag: bool = True) -> Result:
        T = Y.shape[0]
        xf = torch.empty((T, self.N), dtype=torch.float64, device=Y.device)
        df = torch.empty((T, self.N), dtype=torch.float64, device=Y.device) if want_diag else None
        kf_filter(self.plan, Y, xf, df)
        return Result(xf, df)

    def smooth(self, res: Result, want_diag: bool = True, want_full: bool = False) -> Result:
        T = res.x_filt.shape[0]
        dev = res.x_filt.device
        res.x_smooth = torch.empty((T, self.N), dtype=torch.float64, device=dev)
        res.Pdiag_smooth = torch.empty((T, self.N), dtype=torch.float64, device=dev) if want_diag else None
        res.P_smooth = torch.empty((T, self.N, self.N), dtype=torch.float64, device=dev) if want_full else None
        kf_smooth(self.plan, res.x_smooth, res.Pdiag_smooth, res.P_smooth)
        return res

    def run(self, Y, want_full: bool = False) -> Result:
        return self.smooth(self.filter(Y), want_full=want_full)

    def smooth_assoc(self, res: Result, want_diag: bool = True, want_full: bool = False) -> Result:
        """kf_smooth_assoc on the last filter call: same outputs as smooth(); the plan then needs a new filter call."""
        T = res.x_filt.shape[0]
        dev = res.x_filt.device
        res.x_smooth = torch.empty((T, self.N), dtype=torch.float64, device=dev)
        res.Pdiag_smooth = torch.empty((T, self.N), dtype=torch.float64, device=dev) if want_diag else None
        res.P_smooth = torch.empty((T, self.N, self.N), dtype=torch.float64, device=dev) if want_full else None
        kf_smooth_assoc(self.plan, res.x_smooth, res.Pdiag_smooth, res.P_smooth)
        return res

    def smooth_means(self, res: Result) -> Result:
        """x_{t|T} only (needs keep_gain_factors); res.x_filt from the last filter call."""
        res.x_smooth = torch.empty_like(res.x_filt)
        kf_smooth_means(self.plan, res.x_smooth)
        return res

    def run_batch(self, Y, want_diag: bool = True) -> Result:
        """Filter and smooth B data sets, Y: (B, T, m); means come back as (B, T, N)."""
        B, T, _ = Y.shape
        dev = Y.device
        res = Result(torch.empty((B, T, self.N), dtype=torch.float64, device=dev),
                     torch.empty((T, self.N), dtype=torch.float64, device=dev) if want_diag else None)
        kf_filter_batch(self.plan, Y, res.x_filt, res.Pdiag_filt)
        res.x_smooth = torch.empty((B, T, self.N), dtype=torch.float64, device=dev)
        res.Pdiag_smooth = torch.empty((T, self.N), dtype=torch.float64, device=dev) if want_diag else None
        kf_smooth_batch(self.plan, res.x_smooth, res.Pdiag_smooth)
        return res

    def filtered_cov(self, t: int) -> torch.Tensor:
        P = torch.empty((self.N, self.N), dtype=torch.float64, device="cuda")
        kf_get_filtered_cov(self.plan, t, P)
        return P

    def close(self):
        if getattr(self, "plan", None):
            kf_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
