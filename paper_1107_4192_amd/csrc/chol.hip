// Blocked Cholesky factorisation fused with the inverse of the factor (float64).
//
// The filter needs S^{-1} in eqn8/eqn9 and the smoother needs P_{t+1|t}^{-1}
// in eqn11. Both are applied through the lower Cholesky factor L and its
// inverse Li = L^{-1}: S^{-1} B = Li^T (Li B), and the smoother gain
// A_t = P_{t|t} P_{t+1|t}^{-1} = (Li P_{t|t})^T Li. Li is obtained by solving
// L Z = I in the same right-looking sweep as the factorisation, so every
// O(n^3) part is a large MFMA product:
//
//   for each 64-column block k:
//     1. one workgroup factors the diagonal block in LDS and inverts it
//        (L_kk, Li_kk), flagging a non-positive or non-finite pivot;
//     2. panel:    L_{>k,k} = A_{>k,k} Li_kk^T        and  Z_{k,<k} = Li_kk Z_{k,<k}
//     3. trailing: A_{>k,>k} -= L_{>k,k} L_{>k,k}^T   and  Z_{>k,<=k} -= L_{>k,k} Z_{k,<=k}
//   (2 and 3 are each one grouped GEMM launch.)
#include "kf_internal.h"

namespace kfmeg {

namespace {

constexpr int NB = 64;
constexpr int NTD = 256;

__global__ __launch_bounds__(NTD) void potrf_inv_diag(double* W, int64_t ldw, double* Z, int64_t ldz, int nb,
                                                      int* status, int which, int step, int row0) {
    __shared__ double A[NB][NB + 1];
    __shared__ double Zs[NB][NB + 1];
    __shared__ double Ld[NB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < NB * NB; idx += NTD) {
        const int i = idx / NB, c = idx - i * NB;
        A[i][c] = (i < nb && c <= i) ? W[(int64_t)i * ldw + c] : 0.0;
        Zs[i][c] = (i == c) ? 1.0 : 0.0;
    }
    if (tid == 0) bad = -1;
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const double d = A[j][j];
        if (!(d > 0.0) || !isfinite(d)) {       // same value in every thread: uniform exit
            if (tid == 0) bad = j;
            break;
        }
        const double sq = sqrt(d), inv = 1.0 / sq;
        for (int i = j + 1 + tid; i < nb; i += NTD) A[i][j] *= inv;
        for (int c = tid; c <= j; c += NTD) Zs[j][c] *= inv;
        if (tid == 0) Ld[j] = sq;
        __syncthreads();
        const int rows = nb - j - 1;
        for (int idx = tid; idx < rows * nb; idx += NTD) {
            const int i = j + 1 + idx / nb, c = idx % nb;
            const double lij = A[i][j];
            if (c <= j) Zs[i][c] -= lij * Zs[j][c];
            else if (c <= i) A[i][c] -= lij * A[c][j];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += NTD) {
        const int i = idx / nb, c = idx - i * nb;
        W[(int64_t)i * ldw + c] = c < i ? A[i][c] : (c == i ? Ld[i] : 0.0);
        Z[(int64_t)i * ldz + c] = c <= i ? Zs[i][c] : 0.0;
    }
    if (tid == 0 && bad >= 0 && status) {
        if (atomicCAS(&status[0], 0, 1) == 0) {
            status[1] = which;
            status[2] = step;
            status[3] = row0 + bad;
        }
    }
}

}  // namespace

hipError_t chol_inv(double* W, int64_t ldw, double* Z, int64_t ldz, int n, int* status, int which, int step,
                    hipStream_t s) {
    hipError_t e = zero2d(n, n, Z, ldz, s);
    if (e != hipSuccess) return e;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int kb = n - k0 < NB ? n - k0 : NB;
        const int r0 = k0 + kb, rem = n - r0;
        double* Wkk = W + (int64_t)k0 * ldw + k0;
        double* Zkk = Z + (int64_t)k0 * ldz + k0;
        hipLaunchKernelGGL(potrf_inv_diag, dim3(1), dim3(NTD), 0, s, Wkk, ldw, Zkk, ldz, kb, status, which, step,
                           k0);
        if ((e = hipGetLastError()) != hipSuccess) return e;

        GemmProblem pr[2];
        int np = 0;
        if (rem > 0) {                    // L_{>k,k} = A_{>k,k} Li_kk^T   (in place)
            GemmProblem p;
            p.M = rem; p.N = kb; p.K = kb;
            p.A = W + (int64_t)r0 * ldw + k0; p.lda = ldw;
            p.B = Zkk; p.ldb = ldz; p.flags = G_TB | G_BUPPER;
            p.C = W + (int64_t)r0 * ldw + k0; p.ldc = ldw;
            pr[np++] = p;
        }
        if (k0 > 0) {                     // Z_{k,<k} = Li_kk Z_{k,<k}   (in place)
            GemmProblem p;
            p.M = kb; p.N = k0; p.K = kb;
            p.A = Zkk; p.lda = ldz; p.flags = G_ALOWER;
            p.B = Z + (int64_t)k0 * ldz; p.ldb = ldz;
            p.C = Z + (int64_t)k0 * ldz; p.ldc = ldz;
            pr[np++] = p;
        }
        if (np && (e = gemm_launch(Dt::F64, pr, np, s)) != hipSuccess) return e;
        if (rem > 0) {
            GemmProblem t1, t2;           // trailing Schur complement and right-hand side
            t1.M = rem; t1.N = rem; t1.K = kb;
            t1.A = W + (int64_t)r0 * ldw + k0; t1.lda = ldw;
            t1.B = W + (int64_t)r0 * ldw + k0; t1.ldb = ldw;
            t1.flags = G_TB | G_LOWER;
            t1.alpha = -1.0; t1.beta = 1.0;
            t1.Cin = W + (int64_t)r0 * ldw + r0; t1.ldcin = ldw;
            t1.C = W + (int64_t)r0 * ldw + r0; t1.ldc = ldw;

            t2.M = rem; t2.N = r0; t2.K = kb;
            t2.A = W + (int64_t)r0 * ldw + k0; t2.lda = ldw;
            t2.B = Z + (int64_t)k0 * ldz; t2.ldb = ldz;
            t2.alpha = -1.0; t2.beta = 1.0;
            t2.Cin = Z + (int64_t)r0 * ldz; t2.ldcin = ldz;
            t2.C = Z + (int64_t)r0 * ldz; t2.ldc = ldz;
            GemmProblem tr[2] = {t1, t2};
            if ((e = gemm_launch(Dt::F64, tr, 2, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace kfmeg
