// Blocked Cholesky factorisation fused with the inverse of the factor (float64),
// for a batch of independent matrices.
//
// The filter needs S^{-1} in eqn8/eqn9, applied through the lower Cholesky
// factor L and its inverse Li = L^{-1}: S^{-1} B = Li^T (Li B). Li is obtained
// by solving L Z = I in the same right-looking sweep as the factorisation. The
// smoother's P_{t+1|t}^{-1} in eqn11 uses the same sweep only for the diagonal
// blocks of an outer-blocked factorisation (second half of this file).
//
// Two-level blocking keeps the O(n^3) work in large MFMA products with a long
// K dimension:
//   for each 256-column panel K:
//     for each 64-column block k of the panel:
//       1. one workgroup per matrix factors the diagonal block in LDS and inverts
//          it (L_kk, Li_kk), flagging a non-positive or non-finite pivot;
//       2. L_{>k,k} = A_{>k,k} Li_kk^T  and  Z_{k,<k} = Li_kk Z_{k,<k}
//       3. inside the panel only: A_{>k,(k,K]} -= L_{>k,k} L_{(k,K],k}^T and
//          Z_{(k,K],<=k} -= L_{(k,K],k} Z_{k,<=k}
//     4. trailing, K = 256:  A_{>K,>K} -= L_{>K,K} L_{>K,K}^T  and
//        Z_{>K,<=K} -= L_{>K,K} Z_{K,<=K}
// Steps 2-4 are each one grouped GEMM launch over the whole batch, so the
// latency of the sequential sweep is shared by every matrix of the batch.
#include "kf_internal.h"

#include <algorithm>

namespace kfmeg {

namespace {

constexpr int NB = 64;      // diagonal block
constexpr int NB2 = 256;    // panel (K of the trailing update)
constexpr int NTD = 256;

struct DiagBatch {
    double* W[kMaxBatch];
    double* Z[kMaxBatch];
    int step[kMaxBatch];
};

// One workgroup per matrix factors a diagonal block of at most NB columns (rows past
// nb are padded with the identity) and inverts the factor, in registers.
//
// Thread t owns column c = t % 64 at rows g, g+4, ..., g+60 (g = t / 64) of both the
// matrix being factored (a) and U, the inverse of its factor with the row scaling
// deferred (L^{-1}[i][c] = U[i][c] / L[i][i], U starts as the identity). Step j
// publishes column j from the pivot d_j down (colbuf, zero above it) and row j of U
// through LDS, double buffered so that one barrier per step suffices; then, with
// colbuf read as zero at and above the pivot,
//     a[i] -= colbuf[i] colbuf[c] / d_j   (c > j: the Schur complement)
//     u[i] -= colbuf[i] U[j][c] / d_j     (c <= j: forward substitution)
// one FMA each. Column j of L (colbuf / sqrt(d_j)) is collected in LDS and written
// out at the end. 1/sqrt(d_j) comes from the hardware estimate refined by two
// Newton steps (accurate to a few ulp).
__global__ __launch_bounds__(NTD) void potrf_inv_diag(DiagBatch B, int64_t ldw, int64_t ldz, int nb,
                                                      DevStatus* status, int which, int row0) {
    __shared__ double colbuf[2][NB];
    __shared__ double urow[2][NB];
    __shared__ double invs[NB];
    __shared__ double Ls[NB][NB + 1];
    double* W = B.W[blockIdx.x];
    double* Z = B.Z[blockIdx.x];
    const int tid = threadIdx.x;
    const int c = tid & (NB - 1), g = tid >> 6;
    double a[NB / 4], u[NB / 4];
#pragma unroll
    for (int r = 0; r < NB / 4; ++r) {
        const int i = g + 4 * r;
        a[r] = (i < nb && c <= i) ? W[(int64_t)i * ldw + c] : (i == c ? 1.0 : 0.0);
        u[r] = i == c ? 1.0 : 0.0;
    }
    int bad = -1;
#pragma unroll 1
    for (int j = 0; j < NB; ++j) {
        const int buf = j & 1, rj = j >> 2;
        // column j from the diagonal down (the pivot included), and row j of U
        if (c == j) {
#pragma unroll
            for (int r = 0; r < NB / 4; ++r) colbuf[buf][g + 4 * r] = (g + 4 * r >= j) ? a[r] : 0.0;
        }
        if (g == (j & 3)) urow[buf][c] = u[rj];
        __syncthreads();
        // every LDS read of the step is issued at once, ahead of the pivot's arithmetic
        const double d = colbuf[buf][j];
        const double cbc = colbuf[buf][c];
        const double urc = urow[buf][c];
        double cb[NB / 4];
#pragma unroll
        for (int r = 0; r < NB / 4; ++r) cb[r] = colbuf[buf][g + 4 * r];
        const bool ok = d > 0.0 && isfinite(d);  // the same in every thread: a uniform exit below
        double y = __builtin_amdgcn_rsq(d);
        y = y * (1.5 - 0.5 * d * y * y);
        y = y * (1.5 - 0.5 * d * y * y);
        const double inv2 = y * y;
        const double ma = c > j ? cbc * inv2 : 0.0;
        const double mu = c <= j ? urc * inv2 : 0.0;
#pragma unroll
        for (int r = 0; r < NB / 4; ++r) {
            const double v = (g + 4 * r > j) ? cb[r] : 0.0;     // rows below the pivot only
            a[r] = fma(-v, ma, a[r]);
            u[r] = fma(-v, mu, u[r]);
        }
        if (g == 0) Ls[c][j] = c > j ? cbc * y : (c == j ? d * y : 0.0);
        if (tid == 0) invs[j] = y;
        if (!ok) {                               // checked after the step so that its reads issue together
            bad = j;
            break;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NB / 4; ++r) {
        const int i = g + 4 * r;
        if (i < nb && c < nb) {
            W[(int64_t)i * ldw + c] = c <= i ? Ls[i][c] : 0.0;
            Z[(int64_t)i * ldz + c] = c <= i ? u[r] * invs[i] : 0.0;
        }
    }
    if (tid == 0 && bad >= 0 && bad < nb && status)
        atomicMin(&status->key, status_key(B.step[blockIdx.x], row0 + bad, which));
}

}  // namespace

hipError_t chol_inv_batch(int n, double* const* W, int64_t ldw, double* const* Z, int64_t ldz, int count,
                          DevStatus* status, int which, const int* steps, hipStream_t s, int row_base) {
    if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
    hipError_t e;
    for (int b = 0; b < count; ++b)
        if ((e = zero2d(n, n, Z[b], ldz, s)) != hipSuccess) return e;
    auto w = [&](int b, int i, int j) { return W[b] + (int64_t)i * ldw + j; };
    auto z = [&](int b, int i, int j) { return Z[b] + (int64_t)i * ldz + j; };
    for (int c0 = 0; c0 < n; c0 += NB2) {
        const int r2 = c0 + (n - c0 < NB2 ? n - c0 : NB2);
        for (int k0 = c0; k0 < r2; k0 += NB) {
            const int kb = r2 - k0 < NB ? r2 - k0 : NB;
            const int r = k0 + kb;
            DiagBatch db;
            for (int b = 0; b < count; ++b) {
                db.W[b] = w(b, k0, k0);
                db.Z[b] = z(b, k0, k0);
                db.step[b] = steps ? steps[b] : 0;
            }
            hipLaunchKernelGGL(potrf_inv_diag, dim3(count), dim3(NTD), 0, s, db, ldw, ldz, kb, status, which,
                               row_base + k0);
            if ((e = hipGetLastError()) != hipSuccess) return e;

            GemmProblem pr[kMaxGroup];
            int np = 0;
            for (int b = 0; b < count; ++b) {
                if (r < n) {              // L_{>k,k} = A_{>k,k} Li_kk^T   (in place, one column tile)
                    GemmProblem p;
                    p.M = n - r; p.N = kb; p.K = kb;
                    p.A = w(b, r, k0); p.lda = ldw;
                    p.B = z(b, k0, k0); p.ldb = ldz; p.flags = G_TB | G_BUPPER;
                    p.C = w(b, r, k0); p.ldc = ldw;
                    pr[np++] = p;
                }
                if (k0 > 0) {             // Z_{k,<k} = Li_kk Z_{k,<k}   (in place, one row tile)
                    GemmProblem p;
                    p.M = kb; p.N = k0; p.K = kb;
                    p.A = z(b, k0, k0); p.lda = ldz; p.flags = G_ALOWER;
                    p.B = z(b, k0, 0); p.ldb = ldz;
                    p.C = z(b, k0, 0); p.ldc = ldz;
                    pr[np++] = p;
                }
            }
            if (np && (e = gemm_launch(Dt::F64, pr, np, s)) != hipSuccess) return e;
            if (r < r2) {                 // updates inside the panel
                np = 0;
                for (int b = 0; b < count; ++b) {
                    GemmProblem t1, t2;
                    t1.M = n - r; t1.N = r2 - r; t1.K = kb;
                    t1.A = w(b, r, k0); t1.lda = ldw;
                    t1.B = w(b, r, k0); t1.ldb = ldw; t1.flags = G_TB;
                    t1.alpha = -1.0; t1.beta = 1.0;
                    t1.Cin = w(b, r, r); t1.ldcin = ldw;
                    t1.C = w(b, r, r); t1.ldc = ldw;
                    t2.M = r2 - r; t2.N = r; t2.K = kb;
                    t2.A = w(b, r, k0); t2.lda = ldw;
                    t2.B = z(b, k0, 0); t2.ldb = ldz;
                    t2.alpha = -1.0; t2.beta = 1.0;
                    t2.Cin = z(b, r, 0); t2.ldcin = ldz;
                    t2.C = z(b, r, 0); t2.ldc = ldz;
                    pr[np++] = t1;
                    pr[np++] = t2;
                }
                if ((e = gemm_launch(Dt::F64, pr, np, s)) != hipSuccess) return e;
            }
        }
        if (r2 < n) {                     // trailing update with K = the panel width
            GemmProblem pr[kMaxGroup];
            int np = 0;
            for (int b = 0; b < count; ++b) {
                GemmProblem t1, t2;
                t1.M = n - r2; t1.N = n - r2; t1.K = r2 - c0;
                t1.A = w(b, r2, c0); t1.lda = ldw;
                t1.B = w(b, r2, c0); t1.ldb = ldw;
                t1.flags = G_TB | G_LOWER;
                t1.alpha = -1.0; t1.beta = 1.0;
                t1.Cin = w(b, r2, r2); t1.ldcin = ldw;
                t1.C = w(b, r2, r2); t1.ldc = ldw;
                t2.M = n - r2; t2.N = r2; t2.K = r2 - c0;
                t2.A = w(b, r2, c0); t2.lda = ldw;
                t2.B = z(b, c0, 0); t2.ldb = ldz;
                t2.alpha = -1.0; t2.beta = 1.0;
                t2.Cin = z(b, r2, 0); t2.ldcin = ldz;
                t2.C = z(b, r2, 0); t2.ldc = ldz;
                pr[np++] = t1;
                pr[np++] = t2;
            }
            if ((e = gemm_launch(Dt::F64, pr, np, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t chol_inv(double* W, int64_t ldw, double* Z, int64_t ldz, int n, DevStatus* status, int which,
                    int step, hipStream_t s) {
    return chol_inv_batch(n, &W, ldw, &Z, ldz, 1, status, which, &step, s, 0);
}

// ------------------------------------------------------------------ outer-blocked factorisation and solves
// For the smoother gain (eqn11) the inverse of the whole factor is not needed: with L from an
// outer-blocked Cholesky of P_{t+1|t} (diagonal blocks of width nb factored and inverted by
// chol_inv_batch above), A_t^T = L^{-T} (L^{-1} F P_{t|t}) is two blocked triangular solves whose
// off-diagonal work is products with K up to n, and whose diagonal blocks are applied as products
// with the small inverses Li_kk. Every launch covers the whole batch.

namespace {

// The gain's products run as their own named kernel instantiation (profiling).
hipError_t gain_launch(GemmProblem* pr, int count, hipStream_t s) {
    for (int u = 0; u < count; ++u) pr[u].flags |= G_GAIN;
    return gemm_launch(Dt::F64, pr, count, s);
}

// Outer blocks of width nb; a remainder narrower than nb / 4 joins the last full block (so the
// last block is up to gain_block_width(n, nb) wide) rather than costing a sweep of its own.
struct Blocks {
    int n, nb;
    int count() const {
        const int full = n / nb, rem = n - full * nb;
        if (full == 0) return 1;
        return (rem == 0 || rem < nb / 4) ? full : full + 1;
    }
    int lo(int k) const { return k * nb; }
    int hi(int k) const { return k == count() - 1 ? n : (k + 1) * nb; }
};

}  // namespace

int gain_block_width(int n, int nb) {
    const Blocks bl{n, nb};
    return bl.hi(bl.count() - 1) - bl.lo(bl.count() - 1) > nb ? bl.hi(bl.count() - 1) - bl.lo(bl.count() - 1)
                                                               : std::min(n, nb);
}

hipError_t chol_blocked_batch(int n, int nb, double* const* W, int64_t ldw, double* const* D, int64_t ldd,
                              double* const* Tb, int64_t ldt, int count, DevStatus* status, int which,
                              const int* steps, hipStream_t s, const double* const* Pa, const double* Qa) {
    if (count < 1 || count > kMaxBatch || nb < 1 || ldd < gain_block_width(n, nb) || ldt < n || (!Pa != !Qa))
        return hipErrorInvalidValue;
    const Blocks bl{n, nb};
    hipError_t e;
    if (Pa) {   // the first block column of Pa + Qa (diagonal block and panel); the rest comes in below
        for (int b = 0; b < count; ++b)
            if ((e = axpby3(n, bl.hi(0), W[b], false, ldw, Pa[b], false, ldw, Qa, false, ldw, 1.0, nullptr, false,
                            0, 0.0, s)) != hipSuccess)
                return e;
    }
    for (int k = 0; k < bl.count(); ++k) {
        const int r0 = bl.lo(k), r1 = bl.hi(k), nbk = r1 - r0, nr = n - r1;
        double* Wd[kMaxBatch];
        double* Dd[kMaxBatch];
        for (int b = 0; b < count; ++b) {
            Wd[b] = W[b] + (int64_t)r0 * ldw + r0;
            Dd[b] = D[b] + (int64_t)r0 * ldd;
        }
        // L_kk and Li_kk of the diagonal block (its trailing part already updated)
        if ((e = chol_inv_batch(nbk, Wd, ldw, Dd, ldd, count, status, which, steps, s, r0)) != hipSuccess) return e;
        if (nr == 0) break;
        GemmProblem pr[kMaxGroup];
        for (int b = 0; b < count; ++b) {     // panel, transposed: Tb = Li_kk A_{>k,k}^T = L_{>k,k}^T
            GemmProblem& g = pr[b];
            g.M = nbk; g.N = nr; g.K = nbk;
            g.A = Dd[b]; g.lda = ldd; g.flags = G_ALOWER | G_TB;
            g.B = W[b] + (int64_t)r1 * ldw + r0; g.ldb = ldw;
            g.C = Tb[b]; g.ldc = ldt;
        }
        if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
        for (int b = 0; b < count; ++b) {     // trailing: A_{>k,>k} -= L_{>k,k} L_{>k,k}^T  (lower tiles)
            GemmProblem& g = pr[b];
            g = GemmProblem();
            g.M = nr; g.N = nr; g.K = nbk;
            g.A = Tb[b]; g.lda = ldt; g.flags = G_TA | G_LOWER;
            g.B = Tb[b]; g.ldb = ldt;
            g.alpha = -1.0; g.beta = 1.0;
            if (Pa && k == 0) {   // (Pa + Qa)_{>0,>0} - L L^T
                g.Cin = Pa[b] + (int64_t)r1 * ldw + r1; g.ldcin = ldw;
                g.Cin2 = Qa + (int64_t)r1 * ldw + r1; g.ldcin2 = ldw; g.gamma = 1.0;
            } else {
                g.Cin = W[b] + (int64_t)r1 * ldw + r1; g.ldcin = ldw;
            }
            g.C = W[b] + (int64_t)r1 * ldw + r1; g.ldc = ldw;
        }
        if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
        TransposeBatch tb;                    // the panel into place: W[r1 + i][r0 + c] = Tb[c][i]
        for (int b = 0; b < count; ++b) {
            tb.src[b] = Tb[b];
            tb.dst[b] = W[b] + (int64_t)r1 * ldw + r0;
            tb.dst32[b] = nullptr;
        }
        if ((e = transpose_batch(tb, count, nbk, nr, ldt, ldw, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t trsm_lower_batch(int n, int nb, const double* const* W, int64_t ldw, const double* const* D, int64_t ldd,
                            double* const* Tb, int64_t ldt, const double* const* B, int64_t ldb, double* const* Y,
                            int64_t ldy, int count, hipStream_t s) {
    if (count < 1 || count > kMaxBatch || ldt < n) return hipErrorInvalidValue;
    const Blocks bl{n, nb};
    hipError_t e;
    GemmProblem pr[kMaxGroup];
    for (int k = 0; k < bl.count(); ++k) {
        const int r0 = bl.lo(k), nbk = bl.hi(k) - r0;
        if (k > 0) {                          // Tb = B_k - L_{k,<k} Y_{<k}
            for (int b = 0; b < count; ++b) {
                GemmProblem& g = pr[b];
                g = GemmProblem();
                g.M = nbk; g.N = n; g.K = r0;
                g.A = W[b] + (int64_t)r0 * ldw; g.lda = ldw;
                g.B = Y[b]; g.ldb = ldy;
                g.alpha = -1.0; g.beta = 1.0;
                g.Cin = B[b] + (int64_t)r0 * ldb; g.ldcin = ldb;
                g.C = Tb[b]; g.ldc = ldt;
            }
            if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
        }
        for (int b = 0; b < count; ++b) {     // Y_k = Li_kk (B_k - ...)
            GemmProblem& g = pr[b];
            g = GemmProblem();
            g.M = nbk; g.N = n; g.K = nbk;
            g.A = D[b] + (int64_t)r0 * ldd; g.lda = ldd; g.flags = G_ALOWER;
            if (k > 0) { g.B = Tb[b]; g.ldb = ldt; }
            else { g.B = B[b]; g.ldb = ldb; }
            g.C = Y[b] + (int64_t)r0 * ldy; g.ldc = ldy;
        }
        if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t trsm_upper_t_batch(int n, int nb, const double* const* W, int64_t ldw, const double* const* D,
                              int64_t ldd, double* const* Tb, int64_t ldt, const double* const* Y, int64_t ldy,
                              double* const* Z, int64_t ldz, int count, hipStream_t s) {
    if (count < 1 || count > kMaxBatch || ldt < n) return hipErrorInvalidValue;
    const Blocks bl{n, nb};
    hipError_t e;
    GemmProblem pr[kMaxGroup];
    for (int k = bl.count() - 1; k >= 0; --k) {
        const int r0 = bl.lo(k), r1 = bl.hi(k), nbk = r1 - r0;
        if (r1 < n) {                         // Tb = Y_k - L_{>k,k}^T Z_{>k}
            for (int b = 0; b < count; ++b) {
                GemmProblem& g = pr[b];
                g = GemmProblem();
                g.M = nbk; g.N = n; g.K = n - r1;
                g.A = W[b] + (int64_t)r1 * ldw + r0; g.lda = ldw; g.flags = G_TA;
                g.B = Z[b] + (int64_t)r1 * ldz; g.ldb = ldz;
                g.alpha = -1.0; g.beta = 1.0;
                g.Cin = Y[b] + (int64_t)r0 * ldy; g.ldcin = ldy;
                g.C = Tb[b]; g.ldc = ldt;
            }
            if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
        }
        for (int b = 0; b < count; ++b) {     // Z_k = Li_kk^T (Y_k - ...)
            GemmProblem& g = pr[b];
            g = GemmProblem();
            g.M = nbk; g.N = n; g.K = nbk;
            g.A = D[b] + (int64_t)r0 * ldd; g.lda = ldd; g.flags = G_TA | G_AUPPER;
            if (r1 < n) { g.B = Tb[b]; g.ldb = ldt; }
            else { g.B = Y[b] + (int64_t)r0 * ldy; g.ldb = ldy; }
            g.C = Z[b] + (int64_t)r0 * ldz; g.ldc = ldz;
        }
        if ((e = gain_launch(pr, count, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kfmeg
