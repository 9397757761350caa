// Kernel-level test entry points (include/kfmeg_debug.h).
#include "kf_internal.h"
#include "../../include/kfmeg_debug.h"

using namespace kfmeg;

extern "C" {

int kfd_gemm(int dtype, int M, int N, int K, int flags, const void* A, int64_t lda, const void* B, int64_t ldb,
             double alpha, double beta, const double* Cin, int64_t ldcin, double* C, int64_t ldc, int ksplit,
             void* stream) {
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C || (dtype != 0 && dtype != 1) || ksplit < 1 ||
        (flags & ~(127 | G_AUPPER)))
        return 1;
    if ((flags & G_LOWER) && M != N) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GemmProblem g;
    g.M = M; g.N = N; g.K = K; g.flags = flags;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
    g.alpha = alpha; g.beta = beta; g.Cin = Cin; g.ldcin = ldcin;
    g.C = C; g.ldc = ldc;
    void* part = nullptr;
    if (ksplit > 1) {
        if (hipMalloc(&part, (size_t)ksplit * M * N * (dtype == 0 ? 8 : 4)) != hipSuccess) return 4;
        g.ksplit = ksplit;
        g.partial = part;
    }
    hipError_t e = gemm1(dtype == 0 ? Dt::F64 : Dt::F32, g, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (part) (void)hipFree(part);
    return e == hipSuccess ? 0 : 4;
}

int kfd_gemm_tail(int dtype, int M, int N, int K, int flags, const void* A, int64_t lda, const void* B,
                  int64_t ldb, double alpha, double beta, const double* Cin, int64_t ldcin, double* C, int64_t ldc,
                  int full, int k, void* stream) {
    if (M <= 0 || N <= 0 || K < 0 || !A || !B || !C || (dtype != 0 && dtype != 1) || (flags & ~(127 | G_AUPPER)) || k < 2 ||
        k > 8 || full < 0)
        return 1;
    if ((flags & G_LOWER) && M != N) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GemmProblem g;
    g.M = M; g.N = N; g.K = K; g.flags = flags;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
    g.alpha = alpha; g.beta = beta; g.Cin = Cin; g.ldcin = ldcin;
    g.C = C; g.ldc = ldc;
    const int tiles = gemm_tiles(g);
    if (full > tiles) return 1;
    TailSplit ts;
    ts.full = full;
    ts.k = k;
    void* ws = nullptr;
    if (hipMalloc(&ws, (size_t)(tiles - full) * k * kTileElems * (dtype == 0 ? 8 : 4) + 256) != hipSuccess) return 4;
    hipError_t e = gemm_launch_tail(dtype == 0 ? Dt::F64 : Dt::F32, g, ts, ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    return e == hipSuccess ? 0 : 4;
}

int kfd_chol_inv(int n, double* W, int64_t ldw, double* Z, int64_t ldz, int* pivot_row, void* stream) {
    if (n <= 0 || !W || !Z || ldw < n || ldz < n) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevStatus* dst = nullptr;
    if (hipMalloc(&dst, sizeof(DevStatus)) != hipSuccess) return 4;
    DevStatus h{};
    hipError_t e = status_clear(dst, s);
    if (e == hipSuccess) e = chol_inv(W, ldw, Z, ldz, n, dst, W_MNE, 0, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, dst, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dst);
    if (e != hipSuccess) return 4;
    if (h.key != kStatusClear) {
        if (pivot_row) *pivot_row = status_row(h.key);
        return 2;
    }
    return 0;
}

int kfd_spd_solve(int n, int nb, double* W, int64_t ldw, const double* B, int64_t ldb, double* X, int64_t ldx,
                  int* pivot_row, void* stream) {
    if (n <= 0 || nb <= 0 || !W || !B || !X || ldw < n || ldb < n || ldx < n) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t ldd = (gain_block_width(n, nb) + 15) / 16 * 16, ld = (n + 15) / 16 * 16;
    double *D = nullptr, *Tb = nullptr, *Y = nullptr;
    DevStatus* dst = nullptr;
    auto cleanup = [&](int r) {
        for (void* a : {(void*)D, (void*)Tb, (void*)Y, (void*)dst})
            if (a) (void)hipFree(a);
        return r;
    };
    if (hipMalloc(&D, (size_t)n * ldd * 8) != hipSuccess || hipMalloc(&Tb, (size_t)ldd * ld * 8) != hipSuccess ||
        hipMalloc(&Y, (size_t)n * ld * 8) != hipSuccess || hipMalloc(&dst, sizeof(DevStatus)) != hipSuccess)
        return cleanup(4);
    int step = 0;
    DevStatus h{};
    hipError_t e = status_clear(dst, s);
    if (e == hipSuccess) e = chol_blocked_batch(n, nb, &W, ldw, &D, ldd, &Tb, ld, 1, dst, W_MNE, &step, s);
    if (e == hipSuccess) e = trsm_lower_batch(n, nb, &W, ldw, &D, ldd, &Tb, ld, &B, ldb, &Y, ld, 1, s);
    if (e == hipSuccess) e = trsm_upper_t_batch(n, nb, &W, ldw, &D, ldd, &Tb, ld, &Y, ld, &X, ldx, 1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, dst, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    else (void)hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(4);
    if (h.key != kStatusClear) {
        if (pivot_row) *pivot_row = status_row(h.key);
        return cleanup(2);
    }
    return cleanup(0);
}

}  // extern "C"
