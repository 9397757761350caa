// Vector and elementwise kernels of the filter/smoother (float64).
//
// The mean recursions are O(mN) or O(N^2) per step and bound by HBM reads of
// one matrix, so they are plain coalesced sweeps: one 64-wide wave per output
// row with a fixed-order shuffle reduction (deterministic), or one thread per
// output column.
#include "kf_internal.h"

#include <algorithm>

namespace kfmeg {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// e_i = y_i - sum_k X[i][k] x_k   (residual of eqn10)
__global__ void resid_kernel(const double* X, int64_t ldx, const double* x, const double* y, double* e, int m,
                             int N) {
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double* xr = X + (int64_t)row * ldx;
    double s = 0.0;
    for (int k = lane; k < N; k += 64) s += xr[k] * x[k];
    s = wave_sum(s);
    if (lane == 0) e[row] = y[row] - s;
}

// w_i = sum_{k <= i} L[i][k] e_k
__global__ void trmv_lower_kernel(const double* L, int64_t ldl, const double* e, double* w, int m) {
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double* lr = L + (int64_t)row * ldl;
    double s = 0.0;
    for (int k = lane; k <= row; k += 64) s += lr[k] * e[k];
    s = wave_sum(s);
    if (lane == 0) w[row] = s;
}

// x_out_j = x_in_j + sum_i C[i][j] w_i
__global__ void gemv_t_add_kernel(const double* C, int64_t ldc, const double* w, const double* x_in,
                                  double* x_out, double* x_copy, int m, int N) {
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += C[(int64_t)i * ldc + j] * w[i];
    const double v = x_in[j] + s;
    x_out[j] = v;
    if (x_copy) x_copy[j] = v;
}

// out_i = x_i + sum_k A[i][k] (v_k - x_k)
__global__ void gemv_smooth_kernel(const double* A, int64_t lda, const double* x, const double* v, double* out,
                                   int N) {
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const double* ar = A + (int64_t)row * lda;
    double s = 0.0;
    for (int k = lane; k < N; k += 64) s += ar[k] * (v[k] - x[k]);
    s = wave_sum(s);
    if (lane == 0) out[row] = x[row] + s;
}

__device__ __forceinline__ double ld_any(const void* p, bool f32, int64_t idx) {
    return f32 ? (double)static_cast<const float*>(p)[idx] : static_cast<const double*>(p)[idx];
}
__device__ __forceinline__ void st_any(void* p, bool f32, int64_t idx, double v) {
    if (f32) static_cast<float*>(p)[idx] = (float)v;
    else static_cast<double*>(p)[idx] = v;
}

__global__ void axpby3_kernel(int rows, int cols, void* D, bool d32, int64_t ldd, const void* a, bool a32,
                              int64_t lda, const void* b, bool b32, int64_t ldb, double cb, const void* c,
                              bool c32, int64_t ldc, double cc) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB) {
        const int i = (int)(idx / cols), j = (int)(idx - (int64_t)i * cols);
        double v = ld_any(a, a32, (int64_t)i * lda + j);
        if (b) v += cb * ld_any(b, b32, (int64_t)i * ldb + j);
        if (c) v += cc * ld_any(c, c32, (int64_t)i * ldc + j);
        st_any(D, d32, (int64_t)i * ldd + j, v);
    }
}

__global__ void copy2d_kernel(int rows, int cols, void* dst, bool d32, int64_t ldd, const void* src, bool s32,
                              int64_t lds) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB) {
        const int i = (int)(idx / cols), j = (int)(idx - (int64_t)i * cols);
        st_any(dst, d32, (int64_t)i * ldd + j, ld_any(src, s32, (int64_t)i * lds + j));
    }
}

__global__ void copy2d_r32_kernel(int rows, int cols, double* dst, int64_t ldd, const void* src, bool s32,
                                  int64_t lds) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB) {
        const int i = (int)(idx / cols), j = (int)(idx - (int64_t)i * cols);
        dst[(int64_t)i * ldd + j] = (double)(float)ld_any(src, s32, (int64_t)i * lds + j);
    }
}

// Dc[k][j] = (J[k+1][j] - J[k][j]) - mean_k(J[k+1][j] - J[k][j]), k < T-1; one thread per column.
__global__ void diff_center_kernel(const double* J, int64_t ldj, int T, int N, double* Dc, int64_t ldd) {
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int k = 0; k + 1 < T; ++k) s += J[(int64_t)(k + 1) * ldj + j] - J[(int64_t)k * ldj + j];
    const double mean = s / (double)(T - 1);
    for (int k = 0; k + 1 < T; ++k) Dc[(int64_t)k * ldd + j] = (J[(int64_t)(k + 1) * ldj + j] - J[(int64_t)k * ldj + j]) - mean;
}

__global__ void add_diag_kernel(double* A, int64_t lda, int n, double v) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) A[(int64_t)i * lda + i] += v;
}

__global__ void zero2d_kernel(int rows, int cols, double* dst, int64_t ldd) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB) {
        const int i = (int)(idx / cols), j = (int)(idx - (int64_t)i * cols);
        dst[(int64_t)i * ldd + j] = 0.0;
    }
}

__global__ void nonfinite_kernel(const double* v, int64_t n, int* flag) {
    bool badv = false;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB)
        badv |= !isfinite(v[idx]);
    if (badv) atomicOr(flag, 1);
}

__global__ void diag_kernel(const double* A, int64_t lda, int n, double* out) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) out[i] = A[(int64_t)i * lda + i];
}

// In-place transpose of a square n x n matrix: one workgroup per 64 x 64 tile pair
// (bi >= bj), both tiles staged through LDS and written back swapped.
constexpr int TT = 64;
__global__ __launch_bounds__(256) void transpose_inplace_kernel(double* A, int64_t lda, int n, int tiles) {
    __shared__ double t0[TT][TT + 1];
    __shared__ double t1[TT][TT + 1];
    int bi = (int)((sqrtf(8.0f * blockIdx.x + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= (int)blockIdx.x) ++bi;
    while (bi * (bi + 1) / 2 > (int)blockIdx.x) --bi;
    const int bj = blockIdx.x - bi * (bi + 1) / 2;
    const int i0 = bi * TT, j0 = bj * TT;
    for (int idx = threadIdx.x; idx < TT * TT; idx += 256) {
        const int r = idx / TT, c = idx % TT;
        if (i0 + r < n && j0 + c < n) t0[r][c] = A[(int64_t)(i0 + r) * lda + j0 + c];
        if (j0 + r < n && i0 + c < n) t1[r][c] = A[(int64_t)(j0 + r) * lda + i0 + c];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TT * TT; idx += 256) {
        const int r = idx / TT, c = idx % TT;
        if (i0 + r < n && j0 + c < n) A[(int64_t)(i0 + r) * lda + j0 + c] = t1[c][r];
        if (bi != bj && j0 + r < n && i0 + c < n) A[(int64_t)(j0 + r) * lda + i0 + c] = t0[c][r];
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 65536)); }

}  // namespace

hipError_t resid(const double* X, int64_t ldx, const double* x, const double* y, double* e, int m, int N,
                 hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3((m + 3) / 4), dim3(TPB), 0, s, X, ldx, x, y, e, m, N);
    return hipGetLastError();
}

hipError_t trmv_lower(const double* L, int64_t ldl, const double* e, double* w, int m, hipStream_t s) {
    hipLaunchKernelGGL(trmv_lower_kernel, dim3((m + 3) / 4), dim3(TPB), 0, s, L, ldl, e, w, m);
    return hipGetLastError();
}

hipError_t gemv_t_add(const double* C, int64_t ldc, const double* w, const double* x_in, double* x_out,
                      double* x_copy, int m, int N, hipStream_t s) {
    hipLaunchKernelGGL(gemv_t_add_kernel, dim3((N + TPB - 1) / TPB), dim3(TPB), 0, s, C, ldc, w, x_in, x_out,
                       x_copy, m, N);
    return hipGetLastError();
}

hipError_t gemv_smooth(const double* A, int64_t lda, const double* x, const double* v, double* out, int N,
                       hipStream_t s) {
    hipLaunchKernelGGL(gemv_smooth_kernel, dim3((N + 3) / 4), dim3(TPB), 0, s, A, lda, x, v, out, N);
    return hipGetLastError();
}

hipError_t axpby3(int rows, int cols, void* D, bool d32, int64_t ldd, const void* a, bool a32, int64_t lda,
                  const void* b, bool b32, int64_t ldb, double cb, const void* c, bool c32, int64_t ldc,
                  double cc, hipStream_t s) {
    hipLaunchKernelGGL(axpby3_kernel, dim3(grid_for((int64_t)rows * cols)), dim3(TPB), 0, s, rows, cols, D, d32,
                       ldd, a, a32, lda, b, b32, ldb, cb, c, c32, ldc, cc);
    return hipGetLastError();
}

hipError_t copy2d(int rows, int cols, void* dst, bool d32, int64_t ldd, const void* src, bool s32, int64_t lds,
                  hipStream_t s) {
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((int64_t)rows * cols)), dim3(TPB), 0, s, rows, cols, dst, d32,
                       ldd, src, s32, lds);
    return hipGetLastError();
}

hipError_t copy2d_r32(int rows, int cols, double* dst, int64_t ldd, const void* src, bool s32, int64_t lds,
                      hipStream_t s) {
    hipLaunchKernelGGL(copy2d_r32_kernel, dim3(grid_for((int64_t)rows * cols)), dim3(TPB), 0, s, rows, cols, dst, ldd,
                       src, s32, lds);
    return hipGetLastError();
}

hipError_t diff_center(const double* J, int64_t ldj, int T, int N, double* Dc, int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(diff_center_kernel, dim3((N + TPB - 1) / TPB), dim3(TPB), 0, s, J, ldj, T, N, Dc, ldd);
    return hipGetLastError();
}

hipError_t add_diag(double* A, int64_t lda, int n, double v, hipStream_t s) {
    hipLaunchKernelGGL(add_diag_kernel, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, A, lda, n, v);
    return hipGetLastError();
}

hipError_t zero2d(int rows, int cols, double* dst, int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(zero2d_kernel, dim3(grid_for((int64_t)rows * cols)), dim3(TPB), 0, s, rows, cols, dst, ldd);
    return hipGetLastError();
}

hipError_t nonfinite_scan(const double* v, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n)), dim3(TPB), 0, s, v, n, flag);
    return hipGetLastError();
}

hipError_t transpose_inplace(double* A, int64_t lda, int n, hipStream_t s) {
    const int t = (n + TT - 1) / TT;
    hipLaunchKernelGGL(transpose_inplace_kernel, dim3(t * (t + 1) / 2), dim3(256), 0, s, A, lda, n, t);
    return hipGetLastError();
}

hipError_t diag_copy(const double* A, int64_t lda, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(diag_kernel, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, A, lda, n, out);
    return hipGetLastError();
}

}  // namespace kfmeg
