/*
 * kfmeg_debug.h -- kernel-level entry points of the kfmeg library, for tests.
 *
 * They expose the two building blocks every step of the filter and smoother
 * is made of, so each can be checked on its own against a plain reference:
 * the grouped MFMA GEMM and the blocked Cholesky fused with the inverse of
 * its factor. Conventions as in kfmeg.h: device pointers, row-major, caller
 * owns the buffers, the call synchronises `stream` before it returns.
 */
#ifndef KFMEG_DEBUG_H
#define KFMEG_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * C = alpha * op(A) op(B) + beta * Cin on the MFMA path.
 *   dtype: 0 = float64 operands (f64 MFMA), 1 = float32 operands (f32 MFMA);
 *          Cin and C are float64 in both cases.
 *   flags: bit 0 A transposed (A(i,k) = A[k*lda+i]), bit 1 B transposed
 *          (B(k,j) = B[j*ldb+k]), bit 2 lower triangle only (square C),
 *          bit 3 mirror the lower triangle into the upper, bit 4 A lower
 *          triangular, bit 5 B lower triangular, bit 6 B upper triangular
 *          (triangular operands must hold explicit zeros).
 *   ksplit: number of K slices (>1 adds a fixed-order reduction pass).
 * Returns 0 on success, 1 on bad arguments, 4 on a HIP error.
 */
int kfd_gemm(int dtype, int M, int N, int K, int flags, const void* A, int64_t lda, const void* B,
             int64_t ldb, double alpha, double beta, const double* Cin, int64_t ldcin, double* C,
             int64_t ldc, int ksplit, void* stream);

/*
 * kfd_gemm with tail splitting (flags and other arguments as for kfd_gemm,
 * ksplit = 1): the first `full` tiles of the problem's tile order are
 * computed whole and the remaining ones split `k` ways along K (2 <= k <= 8),
 * each split tile reduced by its own workgroup. The library uses this for the
 * smoother's largest products so that the last wave of workgroups is not left
 * mostly idle. Returns 0, 1 on bad arguments, 4 on a HIP error.
 */
int kfd_gemm_tail(int dtype, int M, int N, int K, int flags, const void* A, int64_t lda, const void* B,
                  int64_t ldb, double alpha, double beta, const double* Cin, int64_t ldcin, double* C,
                  int64_t ldc, int full, int k, void* stream);

/*
 * Cholesky factor and its inverse of the SPD matrix in the lower triangle of
 * W (n x n, ld ldw): on return the lower triangle of W holds L (the strict
 * upper triangle is not part of the result) and Z (n x n, ld ldz) holds
 * L^{-1}, lower triangular with explicit zeros above the diagonal. Returns 0, or 2 with *pivot_row set if a pivot is not
 * positive (or not finite), 1 on bad arguments, 4 on a HIP error.
 */
int kfd_chol_inv(int n, double* W, int64_t ldw, double* Z, int64_t ldz, int* pivot_row, void* stream);

/*
 * X = A^{-1} B for the SPD matrix A in the lower triangle of W (n x n, ld ldw)
 * and B (n x n, ld ldb), the way the smoother forms its gain (eqn11): an
 * outer-blocked Cholesky A = L L^T with diagonal blocks of width nb (the last
 * one ragged; only the diagonal blocks are inverted), then the blocked solves
 * Y = L^{-1} B and X = L^{-T} Y. On return W's lower triangle holds L (the
 * strict upper triangle is scratch); X (n x n, ld ldx) must not overlap W or B.
 * Returns 0, 2 with *pivot_row set if a pivot is not positive (or not finite),
 * 1 on bad arguments, 4 on a HIP error (workspace is allocated per call).
 */
int kfd_spd_solve(int n, int nb, double* W, int64_t ldw, const double* B, int64_t ldb, double* X, int64_t ldx,
                  int* pivot_row, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KFMEG_DEBUG_H */
