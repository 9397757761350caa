// Products with a sparse transition matrix F (eqn3; the six-neighbour model of eqn2 has
// seven entries per row), stored in CSR (row_ptr, col_idx, val). Every product is bound by
// the dense operand's HBM traffic, so each is one coalesced sweep over dense rows:
//   spmm_rows:       Y = alpha F A + beta1 C1 + beta2 C2       (row i of Y from the rows of A
//                                                               that F's row i names)
//   dense_sparse_t:  G = P F^T                                  (row k of P staged in LDS, each
//                                                               output G[k][j] gathers from it
//                                                               with F's row j)
//   spmv_rows:       y_b = F x_b for the rows x_b of a block
// With G = P F^T and then F G, F P F^T is formed without transposing anything.
#include "kf_internal.h"

#include <algorithm>

namespace kfmeg {

namespace {

constexpr int TPB = 256;

template <typename TY>
__global__ void spmm_rows_kernel(int n, int ncols, const int* rp, const int* ci, const double* v, const double* A,
                                 int64_t lda, double alpha, const double* C1, int64_t ldc1, double beta1,
                                 const double* C2, int64_t ldc2, double beta2, TY* Y, int64_t ldy) {
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        const int e0 = rp[i], e1 = rp[i + 1];
        for (int j = blockIdx.x * TPB + threadIdx.x; j < ncols; j += gridDim.x * TPB) {
            double s = 0.0;
            for (int e = e0; e < e1; ++e) s += v[e] * A[(int64_t)ci[e] * lda + j];
            double y = alpha * s;
            if (C1) y += beta1 * C1[(int64_t)i * ldc1 + j];
            if (C2) y += beta2 * C2[(int64_t)i * ldc2 + j];
            Y[(int64_t)i * ldy + j] = (TY)y;
        }
    }
}

// One workgroup per row k of P (grid-stride over rows); with STAGE the row sits in dynamic LDS,
// otherwise it is gathered from global memory (rows longer than the LDS budget).
template <bool STAGE>
__global__ void dense_sparse_t_kernel(int n, const double* P, int64_t ldp, const int* rp, const int* ci,
                                      const double* v, double* G, int64_t ldg) {
    extern __shared__ double prow[];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const double* src = P + (int64_t)k * ldp;
        if constexpr (STAGE) {
            __syncthreads();
            for (int l = threadIdx.x; l < n; l += TPB) prow[l] = src[l];
            __syncthreads();
        }
        for (int j = threadIdx.x; j < n; j += TPB) {
            double s = 0.0;
            for (int e = rp[j]; e < rp[j + 1]; ++e) s += v[e] * (STAGE ? prow[ci[e]] : src[ci[e]]);
            G[(int64_t)k * ldg + j] = s;
        }
    }
}

__global__ void spmv_rows_kernel(int n, int rows, const int* rp, const int* ci, const double* v, const double* X,
                                 int64_t ldx, double* Y, int64_t ldy) {
    for (int b = blockIdx.y; b < rows; b += gridDim.y)
        for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
            double s = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * X[(int64_t)b * ldx + ci[e]];
            Y[(int64_t)b * ldy + i] = s;
        }
}

}  // namespace

hipError_t spmm_rows(const Csr& F, const double* A, int64_t lda, double alpha, const double* C1, int64_t ldc1,
                     double beta1, const double* C2, int64_t ldc2, double beta2, void* Y, bool y32, int64_t ldy,
                     hipStream_t s) {
    const int n = F.n;
    const dim3 grid((unsigned)std::max(1, std::min((n + TPB - 1) / TPB, 64)), (unsigned)std::max(1, std::min(n, 65535)));
    if (y32)
        hipLaunchKernelGGL(spmm_rows_kernel<float>, grid, dim3(TPB), 0, s, n, n, F.rp, F.ci, F.v, A, lda, alpha, C1,
                           ldc1, beta1, C2, ldc2, beta2, static_cast<float*>(Y), ldy);
    else
        hipLaunchKernelGGL(spmm_rows_kernel<double>, grid, dim3(TPB), 0, s, n, n, F.rp, F.ci, F.v, A, lda, alpha, C1,
                           ldc1, beta1, C2, ldc2, beta2, static_cast<double*>(Y), ldy);
    return hipGetLastError();
}

hipError_t dense_sparse_t(const Csr& F, const double* P, int64_t ldp, double* G, int64_t ldg, hipStream_t s) {
    const int n = F.n;
    const size_t lds = (size_t)n * sizeof(double);
    const dim3 grid((unsigned)std::min(n, 65535));
    if (lds <= kMaxTransitionLds)
        hipLaunchKernelGGL(dense_sparse_t_kernel<true>, grid, dim3(TPB), lds, s, n, P, ldp, F.rp, F.ci, F.v, G, ldg);
    else
        hipLaunchKernelGGL(dense_sparse_t_kernel<false>, grid, dim3(TPB), 0, s, n, P, ldp, F.rp, F.ci, F.v, G, ldg);
    return hipGetLastError();
}

hipError_t spmv_rows(const Csr& F, const double* X, int64_t ldx, int rows, double* Y, int64_t ldy, hipStream_t s) {
    const int n = F.n;
    const dim3 grid((unsigned)std::max(1, (n + TPB - 1) / TPB), (unsigned)std::max(1, std::min(rows, 65535)));
    hipLaunchKernelGGL(spmv_rows_kernel, grid, dim3(TPB), 0, s, n, rows, F.rp, F.ci, F.v, X, ldx, Y, ldy);
    return hipGetLastError();
}

}  // namespace kfmeg
