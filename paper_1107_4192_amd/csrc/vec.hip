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

// x_out_j = x_in_j + sum_i C[i][j] w_i. A block covers 32 columns with 8 row groups
// (rows g, g+8, ...); the 8 partial sums are added in a fixed order (deterministic).
constexpr int GT_COLS = 32, GT_GROUPS = TPB / GT_COLS;
__global__ __launch_bounds__(TPB) void gemv_t_add_kernel(const double* C, int64_t ldc, const double* w,
                                                         const double* x_in, double* x_out, double* x_copy, int m,
                                                         int N) {
    __shared__ double part[GT_GROUPS][GT_COLS];
    const int c = threadIdx.x % GT_COLS, g = threadIdx.x / GT_COLS;
    const int j = blockIdx.x * GT_COLS + c;
    double s = 0.0;
    if (j < N)
        for (int i = g; i < m; i += GT_GROUPS) s += C[(int64_t)i * ldc + j] * w[i];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < N) {
        double t = part[0][c];
#pragma unroll
        for (int q = 1; q < GT_GROUPS; ++q) t += part[q][c];
        const double v = x_in[j] + t;
        x_out[j] = v;
        if (x_copy) x_copy[j] = v;
    }
}

// out_i = x_i + sum_k A[i][k] (v_k - u_k); one wave per row, four interleaved partial sums
// per lane so that four loads are in flight, combined in a fixed order.
__global__ void gemv_smooth_kernel(const double* A, int64_t lda, const double* x, const double* u, const double* v,
                                   double* out, int N) {
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const double* ar = A + (int64_t)row * lda;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = lane;
    for (; k + 192 < N; k += 256) {
        s0 += ar[k] * (v[k] - u[k]);
        s1 += ar[k + 64] * (v[k + 64] - u[k + 64]);
        s2 += ar[k + 128] * (v[k + 128] - u[k + 128]);
        s3 += ar[k + 192] * (v[k + 192] - u[k + 192]);
    }
    for (; k < N; k += 64) s0 += ar[k] * (v[k] - u[k]);
    double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) out[row] = x[row] + s;
}

// out_i = x_i + sum_k P[i][k] lam_k (P float or double); one wave per row, four partial sums
// per lane combined in a fixed order.
template <typename TP>
__global__ void gemv_add_kernel(const TP* P, int64_t ldp, const double* lam, const double* x, double* out, int N) {
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const TP* pr = P + (int64_t)row * ldp;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = lane;
    for (; k + 192 < N; k += 256) {
        s0 += (double)pr[k] * lam[k];
        s1 += (double)pr[k + 64] * lam[k + 64];
        s2 += (double)pr[k + 128] * lam[k + 128];
        s3 += (double)pr[k + 192] * lam[k + 192];
    }
    for (; k < N; k += 64) s0 += (double)pr[k] * lam[k];
    const double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) out[row] = x[row] + s;
}

// y_q += A_q x_q for the problems q = blockIdx.y of a batch (float64), with the row sums of
// gemv_add_kernel; y_q may be read only by its own rows, so it may not alias another x.
__global__ void gemv_add_batch_kernel(GemvAddBatch G, int64_t lda, int N) {
    const int q = blockIdx.y;
    const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const double* ar = G.A[q] + (int64_t)row * lda;
    const double* x = G.x[q];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = lane;
    for (; k + 192 < N; k += 256) {
        s0 += ar[k] * x[k];
        s1 += ar[k + 64] * x[k + 64];
        s2 += ar[k + 128] * x[k + 128];
        s3 += ar[k + 192] * x[k + 192];
    }
    for (; k < N; k += 64) s0 += ar[k] * x[k];
    const double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) G.y[q][row] += s;
}

// u_i = sum_{k >= i} L[k][i] v_k  (L lower, m x m): u = L^T v, one thread per i.
__global__ void trmv_lower_t_kernel(const double* L, int64_t ldl, const double* v, double* u, int m) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int k = i; k < m; ++k) s += L[(int64_t)k * ldl + i] * v[k];
    u[i] = s;
}

// Elementwise sweeps over a rows x cols block: blockIdx.y walks the rows, the x dimension
// the columns, so consecutive lanes touch consecutive elements and no index is divided.
template <typename TD, typename TA, typename TB, typename TC>
__global__ void axpby3_kernel(int rows, int cols, TD* D, int64_t ldd, const TA* a, int64_t lda, const TB* b,
                              int64_t ldb, double cb, const TC* c, int64_t ldc, double cc) {
    for (int i = blockIdx.y; i < rows; i += gridDim.y)
        for (int j = blockIdx.x * TPB + threadIdx.x; j < cols; j += gridDim.x * TPB) {
            double v = (double)a[(int64_t)i * lda + j];
            if (b) v += cb * (double)b[(int64_t)i * ldb + j];
            if (c) v += cc * (double)c[(int64_t)i * ldc + j];
            D[(int64_t)i * ldd + j] = (TD)v;
        }
}

template <typename TD, typename TS>
__global__ void copy2d_kernel(int rows, int cols, TD* dst, int64_t ldd, const TS* src, int64_t lds) {
    for (int i = blockIdx.y; i < rows; i += gridDim.y)
        for (int j = blockIdx.x * TPB + threadIdx.x; j < cols; j += gridDim.x * TPB)
            dst[(int64_t)i * ldd + j] = (TD)src[(int64_t)i * lds + j];
}

template <typename TS>
__global__ void copy2d_r32_kernel(int rows, int cols, double* dst, int64_t ldd, const TS* src, int64_t lds) {
    for (int i = blockIdx.y; i < rows; i += gridDim.y)
        for (int j = blockIdx.x * TPB + threadIdx.x; j < cols; j += gridDim.x * TPB)
            dst[(int64_t)i * ldd + j] = (double)(float)src[(int64_t)i * lds + j];
}

__global__ void zero2d_kernel(int rows, int cols, double* dst, int64_t ldd) {
    for (int i = blockIdx.y; i < rows; i += gridDim.y)
        for (int j = blockIdx.x * TPB + threadIdx.x; j < cols; j += gridDim.x * TPB) dst[(int64_t)i * ldd + j] = 0.0;
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

__global__ void nonfinite_kernel(const double* v, int64_t n, int* flag) {
    bool badv = false;
    for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * TPB)
        badv |= !isfinite(v[idx]);
    if (badv) atomicOr(flag, 1);
}

// dst = src^T through a 32 x 33 LDS tile (both sides coalesced); blockIdx.z picks the matrix.
constexpr int TT = 32, TR = 8;
__global__ __launch_bounds__(TT * TR) void transpose_kernel(TransposeBatch T, int rows, int cols, int64_t lds,
                                                            int64_t ldd) {
    __shared__ double tile[TT][TT + 1];
    const double* src = T.src[blockIdx.z];
    double* dst = T.dst[blockIdx.z];
    float* dst32 = T.dst32[blockIdx.z];
    const int c0 = blockIdx.x * TT, r0 = blockIdx.y * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
#pragma unroll
    for (int k = 0; k < TT; k += TR) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < rows && c < cols) tile[ty + k][tx] = src[(int64_t)r * lds + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TT; k += TR) {
        const int c = c0 + ty + k, r = r0 + tx;       // dst[c][r] = src[r][c]
        if (r < rows && c < cols) {
            const double v = tile[tx][ty + k];
            dst[(int64_t)c * ldd + r] = v;
            if (dst32) dst32[(int64_t)c * ldd + r] = (float)v;
        }
    }
}

// In-place transpose of square matrices: block (pair t, matrix z) swaps tiles (I, J) and (J, I),
// I <= J, through LDS; every element belongs to exactly one pair, so blocks never overlap.
__global__ __launch_bounds__(TT * TR) void transpose_square_kernel(TransposeInPlace T, int n, int64_t lda) {
    __shared__ double ta[TT][TT + 1], tb[TT][TT + 1];
    double* A = T.A[blockIdx.y];
    float* A32 = T.A32[blockIdx.y];
    // pair index -> (J >= I) on the lower triangle of tile indices
    const int t = blockIdx.x;
    int J = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    while (J * (J + 1) / 2 > t) --J;
    const int I = t - J * (J + 1) / 2;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    const int i0 = I * TT, j0 = J * TT;
#pragma unroll
    for (int k = 0; k < TT; k += TR) {
        const int r = ty + k;
        if (i0 + r < n && j0 + tx < n) ta[r][tx] = A[(int64_t)(i0 + r) * lda + j0 + tx];   // tile (I, J)
        if (j0 + r < n && i0 + tx < n) tb[r][tx] = A[(int64_t)(j0 + r) * lda + i0 + tx];   // tile (J, I)
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TT; k += TR) {
        const int r = ty + k;
        if (i0 + r < n && j0 + tx < n) {          // (I, J) <- (J, I)^T
            const double v = tb[tx][r];
            A[(int64_t)(i0 + r) * lda + j0 + tx] = v;
            if (A32) A32[(int64_t)(i0 + r) * lda + j0 + tx] = (float)v;
        }
        if (I != J && j0 + r < n && i0 + tx < n) {   // (J, I) <- (I, J)^T
            const double v = ta[tx][r];
            A[(int64_t)(j0 + r) * lda + i0 + tx] = v;
            if (A32) A32[(int64_t)(j0 + r) * lda + i0 + tx] = (float)v;
        }
    }
}

__global__ void status_clear_kernel(DevStatus* st) {
    st->key = kStatusClear;
    st->flag = 0;
    st->pad = 0;
}

__global__ void diag_kernel(const double* A, int64_t lda, int n, double* out) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) out[i] = A[(int64_t)i * lda + i];
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 65536)); }

dim3 grid2d(int rows, int cols) {
    return dim3((unsigned)std::max(1, std::min((cols + TPB - 1) / TPB, 64)), (unsigned)std::max(1, std::min(rows, 65535)));
}

template <typename TD, typename TA, typename TB>
hipError_t axpby3_c(int rows, int cols, TD* D, int64_t ldd, const TA* a, int64_t lda, const TB* b, int64_t ldb,
                    double cb, const void* c, bool c32, int64_t ldc, double cc, hipStream_t s) {
    if (c32)
        hipLaunchKernelGGL((axpby3_kernel<TD, TA, TB, float>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, D, ldd,
                           a, lda, b, ldb, cb, static_cast<const float*>(c), ldc, cc);
    else
        hipLaunchKernelGGL((axpby3_kernel<TD, TA, TB, double>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, D,
                           ldd, a, lda, b, ldb, cb, static_cast<const double*>(c), ldc, cc);
    return hipGetLastError();
}

template <typename TD, typename TA>
hipError_t axpby3_b(int rows, int cols, TD* D, int64_t ldd, const TA* a, int64_t lda, const void* b, bool b32,
                    int64_t ldb, double cb, const void* c, bool c32, int64_t ldc, double cc, hipStream_t s) {
    if (b32) return axpby3_c(rows, cols, D, ldd, a, lda, static_cast<const float*>(b), ldb, cb, c, c32, ldc, cc, s);
    return axpby3_c(rows, cols, D, ldd, a, lda, static_cast<const double*>(b), ldb, cb, c, c32, ldc, cc, s);
}

template <typename TD>
hipError_t axpby3_a(int rows, int cols, TD* D, int64_t ldd, const void* a, bool a32, int64_t lda, const void* b,
                    bool b32, int64_t ldb, double cb, const void* c, bool c32, int64_t ldc, double cc, hipStream_t s) {
    if (a32)
        return axpby3_b(rows, cols, D, ldd, static_cast<const float*>(a), lda, b, b32, ldb, cb, c, c32, ldc, cc, s);
    return axpby3_b(rows, cols, D, ldd, static_cast<const double*>(a), lda, b, b32, ldb, cb, c, c32, ldc, cc, s);
}

template <typename TD>
hipError_t copy2d_t(int rows, int cols, TD* dst, int64_t ldd, const void* src, bool s32, int64_t lds, hipStream_t s) {
    if (s32)
        hipLaunchKernelGGL((copy2d_kernel<TD, float>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, dst, ldd,
                           static_cast<const float*>(src), lds);
    else
        hipLaunchKernelGGL((copy2d_kernel<TD, double>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, dst, ldd,
                           static_cast<const double*>(src), lds);
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(gemv_t_add_kernel, dim3((N + GT_COLS - 1) / GT_COLS), dim3(TPB), 0, s, C, ldc, w, x_in, x_out,
                       x_copy, m, N);
    return hipGetLastError();
}

hipError_t gemv_smooth(const double* A, int64_t lda, const double* x, const double* u, const double* v, double* out,
                       int N, hipStream_t s) {
    hipLaunchKernelGGL(gemv_smooth_kernel, dim3((N + 3) / 4), dim3(TPB), 0, s, A, lda, x, u, v, out, N);
    return hipGetLastError();
}

hipError_t gemv_add(const void* P, bool p32, int64_t ldp, const double* lam, const double* x, double* out, int N,
                    hipStream_t s) {
    if (p32)
        hipLaunchKernelGGL(gemv_add_kernel<float>, dim3((N + 3) / 4), dim3(TPB), 0, s, static_cast<const float*>(P), ldp,
                           lam, x, out, N);
    else
        hipLaunchKernelGGL(gemv_add_kernel<double>, dim3((N + 3) / 4), dim3(TPB), 0, s, static_cast<const double*>(P),
                           ldp, lam, x, out, N);
    return hipGetLastError();
}

hipError_t gemv_add_batch(const GemvAddBatch& G, int count, int64_t lda, int N, hipStream_t s) {
    if (count < 1 || count > kMaxGroup) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemv_add_batch_kernel, dim3((N + 3) / 4, count), dim3(TPB), 0, s, G, lda, N);
    return hipGetLastError();
}

hipError_t trmv_lower_t(const double* L, int64_t ldl, const double* v, double* u, int m, hipStream_t s) {
    hipLaunchKernelGGL(trmv_lower_t_kernel, dim3((m + TPB - 1) / TPB), dim3(TPB), 0, s, L, ldl, v, u, m);
    return hipGetLastError();
}

hipError_t axpby3(int rows, int cols, void* D, bool d32, int64_t ldd, const void* a, bool a32, int64_t lda,
                  const void* b, bool b32, int64_t ldb, double cb, const void* c, bool c32, int64_t ldc,
                  double cc, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (d32) return axpby3_a(rows, cols, static_cast<float*>(D), ldd, a, a32, lda, b, b32, ldb, cb, c, c32, ldc, cc, s);
    return axpby3_a(rows, cols, static_cast<double*>(D), ldd, a, a32, lda, b, b32, ldb, cb, c, c32, ldc, cc, s);
}

hipError_t copy2d(int rows, int cols, void* dst, bool d32, int64_t ldd, const void* src, bool s32, int64_t lds,
                  hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (d32) return copy2d_t(rows, cols, static_cast<float*>(dst), ldd, src, s32, lds, s);
    return copy2d_t(rows, cols, static_cast<double*>(dst), ldd, src, s32, lds, s);
}

hipError_t copy2d_r32(int rows, int cols, double* dst, int64_t ldd, const void* src, bool s32, int64_t lds,
                      hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (s32)
        hipLaunchKernelGGL((copy2d_r32_kernel<float>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, dst, ldd,
                           static_cast<const float*>(src), lds);
    else
        hipLaunchKernelGGL((copy2d_r32_kernel<double>), grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, dst, ldd,
                           static_cast<const double*>(src), lds);
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
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero2d_kernel, grid2d(rows, cols), dim3(TPB), 0, s, rows, cols, dst, ldd);
    return hipGetLastError();
}

hipError_t nonfinite_scan(const double* v, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n)), dim3(TPB), 0, s, v, n, flag);
    return hipGetLastError();
}


hipError_t transpose_batch(const TransposeBatch& T, int count, int rows, int cols, int64_t lds, int64_t ldd,
                           hipStream_t s) {
    if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid((cols + TT - 1) / TT, (rows + TT - 1) / TT, count);
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(TT * TR), 0, s, T, rows, cols, lds, ldd);
    return hipGetLastError();
}

hipError_t transpose_square_inplace(const TransposeInPlace& T, int count, int n, int64_t lda, hipStream_t s) {
    if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    const int nt = (n + TT - 1) / TT;
    hipLaunchKernelGGL(transpose_square_kernel, dim3(nt * (nt + 1) / 2, count), dim3(TT * TR), 0, s, T, n, lda);
    return hipGetLastError();
}

hipError_t status_clear(DevStatus* st, hipStream_t s) {
    hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}

hipError_t diag_copy(const double* A, int64_t lda, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(diag_kernel, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s, A, lda, n, out);
    return hipGetLastError();
}

}  // namespace kfmeg
