// Internal interfaces of the kfmeg library: GEMM problem descriptors, the
// blocked Cholesky-with-inverse driver and the small vector kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

namespace kfmeg {

// ---------------------------------------------------------------- GEMM
// C = alpha * op(A) op(B) + beta * Cin + gamma * Cin2 (gamma = 1 when Cin2 is given).
// Operands are of the kernel's compute type (double or float); the epilogue is float64.
enum GemmFlags : int {
    G_TA = 1,          // A(i,k) = A[k*lda + i]   (else A[i*lda + k])
    G_TB = 2,          // B(k,j) = B[j*ldb + k]   (else B[k*ldb + j])
    G_LOWER = 4,       // square C: compute tiles on/below the diagonal, store i >= j only
    G_MIRROR = 8,      // with G_LOWER: also store C(j,i) = C(i,j) (exactly symmetric result)
    G_ALOWER = 16,     // A(i,k) = 0 for k > i (stored zeros): K range trimmed per tile
    G_BLOWER = 32,     // B(k,j) = 0 for k < j
    G_BUPPER = 64,     // B(k,j) = 0 for k > j
    G_CIN32 = 128,     // Cin is float (else double)
    G_CIN2_32 = 256,   // Cin2 is float (else double)
    G_NXN = 512,       // separately named instantiation: smoother N x N x N products, float64 path
    G_NXN_MIXED = 1024,// separately named instantiation: the same products in the mixed-precision path
    G_TILEPART = 2048, // with ksplit > 1: partial sums in one compact slice per tile (tile-wise reduction)
    G_NXN_SERIAL = 4096,// separately named instantiation: the smoother's float64 products in a pass run on
                        // one stream (an isolated measurement of the kernel, without concurrent work)
    G_AUPPER = 8192,   // A(i,k) = 0 for k < i (stored zeros): K range starts at the tile's first row
    G_GAIN = 16384,    // separately named instantiation: the smoother gain's blocked Cholesky and solves
};

struct GemmProblem {
    int M = 0, N = 0, K = 0, flags = 0;
    const void* A = nullptr; int64_t lda = 0;
    const void* B = nullptr; int64_t ldb = 0;
    double alpha = 1.0, beta = 0.0, gamma = 0.0;
    const void* Cin = nullptr; int64_t ldcin = 0;
    const void* Cin2 = nullptr; int64_t ldcin2 = 0;
    double* C = nullptr; int64_t ldc = 0;       // float64 output (may be null)
    float* C32 = nullptr; int64_t ldc32 = 0;    // float32 output (may be null; same ld as C when both)
    double* diag = nullptr;                     // C(i,i) for i < min(M,N) (may be null)
    int ksplit = 1;                             // >1: raw partial sums to `partial`, epilogue by gemm_reduce
    void* partial = nullptr;                    // [ksplit][M][N], or [tile][ksplit][BM*BN] with G_TILEPART
    int tile_off = 0, tile_cnt = -1;            // run only tiles [tile_off, tile_off + tile_cnt) of the
                                                // problem's tile order (-1: to the end)
};

constexpr int kMaxGroup = 16;
constexpr int kMaxBatch = 8;   // matrices per batched factorisation (two problems each per group)
constexpr int kMaxProd = 2;    // smoother gain batches in flight at once (side streams)
constexpr int kGainBlock = 1024;  // outer block of the smoother gain's Cholesky and triangular solves

enum class Dt { F64, F32 };

// Enqueue a group of up to kMaxGroup problems sharing one launch (compute type `dt`).
// Problems with ksplit > 1 are followed by their reduction launch. `main_done`, if given, is
// recorded on s right after the main kernel (before any reduction launch).
hipError_t gemm_launch(Dt dt, GemmProblem* probs, int count, hipStream_t s, hipEvent_t main_done = nullptr);
inline hipError_t gemm1(Dt dt, GemmProblem p, hipStream_t s) { return gemm_launch(dt, &p, 1, s); }

// Tail splitting of one large product: the first `full` tiles (in the problem's tile order)
// run whole, the remaining ones split k ways along K with a tile-wise reduction, so that the
// last wave of workgroups is not left mostly idle. `k == 1`: no split.
struct TailSplit {
    int full = 0, k = 1;
};
constexpr int kTileElems = 128 * 128;      // elements of one output tile
int gemm_tiles(const GemmProblem& p);      // tiles of the problem's tile order
int gemm_slots();                          // workgroups resident at once on the current device
// Best split for `tiles` equal-cost tiles with `kiters` k-steps each, at most max_units split units.
TailSplit choose_tail_split(int tiles, int kiters, int slots, int max_units);
// Launch p with split ts; ws holds (tiles - full) * k tile slices of the compute type.
hipError_t gemm_launch_tail(Dt dt, const GemmProblem& p, TailSplit ts, void* ws, hipStream_t s,
                            hipEvent_t main_done = nullptr);

// ---------------------------------------------------------------- Cholesky + inverse
// Device status record. `key` holds the failure of smallest (step, row, matrix) seen so far,
// packed as status_key(); kStatusClear (all ones) means no failure. Failures are merged with a
// 64-bit atomicMin, so the reported step is the lowest failing one whatever order the batched
// factorisations finish in. `flag` is set by the non-finite scan of the data.
enum Which : int { W_S = 1, W_PPRED = 2, W_MNE = 3 };
struct DevStatus {
    unsigned long long key;
    int flag;
    int pad;
};
constexpr unsigned long long kStatusClear = ~0ull;
__host__ __device__ constexpr unsigned long long status_key(int step, int row, int which) {
    return ((unsigned long long)(unsigned)step << 32) | ((unsigned long long)(row & 0xFFFFFF) << 8) |
           (unsigned long long)(which & 0xFF);
}
inline int status_step(unsigned long long k) { return (int)(k >> 32); }
inline int status_row(unsigned long long k) { return (int)((k >> 8) & 0xFFFFFF); }
inline int status_which(unsigned long long k) { return (int)(k & 0xFF); }
// Reset a status record on stream s (a kernel, not a memset).
hipError_t status_clear(DevStatus* st, hipStream_t s);

// Blocked right-looking Cholesky of the SPD matrix held in the lower triangle of W (n x n, ld ldw),
// fused with the inverse of the factor: on return W's lower triangle holds L (its strict upper
// triangle is scratch) and Z holds L^{-1} (lower, explicit zeros above the diagonal). Z must not
// alias W.
hipError_t chol_inv(double* W, int64_t ldw, double* Z, int64_t ldz, int n, DevStatus* status,
                    int which, int step, hipStream_t s);
// The same for `count` <= kMaxBatch independent matrices of one size, sharing every launch.
// `row_base` is added to the pivot row reported in the status record.
hipError_t chol_inv_batch(int n, double* const* W, int64_t ldw, double* const* Z, int64_t ldz, int count,
                          DevStatus* status, int which, const int* steps, hipStream_t s, int row_base = 0);

// Widest outer block of the blocked factorisation below for order n and block nb: nb, except that
// a remainder narrower than nb / 4 joins the last block (and n itself when n <= nb).
int gain_block_width(int n, int nb);
// Outer-blocked Cholesky of `count` SPD matrices held in the lower triangles of W (n x n, ld ldw):
// diagonal blocks of width nb (the last one ragged) are factored and inverted by chol_inv_batch,
// each panel is formed transposed in Tb, L_{>k,k}^T = Li_kk A_{>k,k}^T, and the trailing matrix
// is updated with K = nb. On return W's lower triangle holds L (its strict upper triangle is
// scratch) and D (n x nb, ld ldd >= nb) holds the inverse of diagonal block k in rows
// [k nb, k nb + nb_k), lower triangular with explicit zeros (ldd >= gain_block_width(n, nb)).
// Tb: gain_block_width(n, nb) x n scratch, ld ldt >= n.
// With Pa (count matrices) and Qa (one, both ld ldw) the matrices factored are Pa[b] + Qa and W
// holds nothing on entry: the sum is formed only for the first block column, and the first
// trailing update reads Pa and Qa in its epilogue (one N x N pass per matrix less).
hipError_t chol_blocked_batch(int n, int nb, double* const* W, int64_t ldw, double* const* D, int64_t ldd,
                              double* const* Tb, int64_t ldt, int count, DevStatus* status, int which,
                              const int* steps, hipStream_t s, const double* const* Pa = nullptr,
                              const double* Qa = nullptr);
// Y = L^{-1} B (B, Y: n x n) with L, D from chol_blocked_batch; block row k is
// Y_k = Li_kk (B_k - L_{k,<k} Y_{<k}). Y must not alias B, W or D; Tb is scratch.
hipError_t trsm_lower_batch(int n, int nb, const double* const* W, int64_t ldw, const double* const* D, int64_t ldd,
                            double* const* Tb, int64_t ldt, const double* const* B, int64_t ldb, double* const* Y,
                            int64_t ldy, int count, hipStream_t s);
// Z = L^{-T} Y (n x n); block row k is Z_k = Li_kk^T (Y_k - L_{>k,k}^T Z_{>k}), last block first.
// Z must not alias Y, W or D; Tb is scratch.
hipError_t trsm_upper_t_batch(int n, int nb, const double* const* W, int64_t ldw, const double* const* D,
                              int64_t ldd, double* const* Tb, int64_t ldt, const double* const* Y, int64_t ldy,
                              double* const* Z, int64_t ldz, int count, hipStream_t s);

// ---------------------------------------------------------------- vector / elementwise kernels
// e = y - X x  (X: m x N, ld ldx)
hipError_t resid(const double* X, int64_t ldx, const double* x, const double* y, double* e,
                 int m, int N, hipStream_t s);
// w = Lower(L) e  (L: m x m, ld ldl; only the lower triangle is read)
hipError_t trmv_lower(const double* L, int64_t ldl, const double* e, double* w, int m, hipStream_t s);
// x_out = x_in + C^T w  (C: m x N, ld ldc); optional copy to x_copy
hipError_t gemv_t_add(const double* C, int64_t ldc, const double* w, const double* x_in,
                      double* x_out, double* x_copy, int m, int N, hipStream_t s);
// out = x + A (v - u)   (A: N x N, ld lda)   -- smoothed mean (eqn12; u = F x, or x when F = I)
hipError_t gemv_smooth(const double* A, int64_t lda, const double* x, const double* u, const double* v,
                       double* out, int N, hipStream_t s);
// out = x + P lam  (P: N x N float or double, ld ldp)   -- mean-only smoother
hipError_t gemv_add(const void* P, bool p32, int64_t ldp, const double* lam, const double* x, double* out, int N,
                    hipStream_t s);
// y_q += A_q x_q for q < count (count <= kMaxGroup), all A_q N x N with leading dimension lda.
struct GemvAddBatch {
    const double* A[kMaxGroup];
    const double* x[kMaxGroup];
    double* y[kMaxGroup];
};
hipError_t gemv_add_batch(const GemvAddBatch& G, int count, int64_t lda, int N, hipStream_t s);
// u = Lower(L)^T v  (L: m x m, ld ldl)
hipError_t trmv_lower_t(const double* L, int64_t ldl, const double* v, double* u, int m, hipStream_t s);
// D = a + ca*b + cb*c for matrices (rows x cols); each source may be float or double
hipError_t axpby3(int rows, int cols, void* D, bool d32, int64_t ldd,
                  const void* a, bool a32, int64_t lda,
                  const void* b, bool b32, int64_t ldb, double cb,
                  const void* c, bool c32, int64_t ldc, double cc, hipStream_t s);
// copy rows x cols between (possibly) different precisions and leading dimensions
hipError_t copy2d(int rows, int cols, void* dst, bool d32, int64_t ldd,
                  const void* src, bool s32, int64_t lds, hipStream_t s);
// dst (float64) = src rounded to float32 (src float or double): what a float32 store would hold
hipError_t copy2d_r32(int rows, int cols, double* dst, int64_t ldd, const void* src, bool s32, int64_t lds,
                      hipStream_t s);
// centred first differences of the rows of J (T x N) into Dc ((T-1) x N)
hipError_t diff_center(const double* J, int64_t ldj, int T, int N, double* Dc, int64_t ldd, hipStream_t s);
// A[i][i] += v
hipError_t add_diag(double* A, int64_t lda, int n, double v, hipStream_t s);
// dst_q = src_q^T for q < count: src rows x cols (ld lds), dst cols x rows (ld ldd); with dst32_q
// also a float32 copy of dst_q (same ld). Out of place: dst must not overlap src.
struct TransposeBatch {
    const double* src[kMaxBatch];
    double* dst[kMaxBatch];
    float* dst32[kMaxBatch];
};
hipError_t transpose_batch(const TransposeBatch& T, int count, int rows, int cols, int64_t lds, int64_t ldd,
                           hipStream_t s);
// A_q = A_q^T in place for square n x n matrices (ld lda); with A32_q also a float32 copy.
struct TransposeInPlace {
    double* A[kMaxBatch];
    float* A32[kMaxBatch];
};
hipError_t transpose_square_inplace(const TransposeInPlace& T, int count, int n, int64_t lda, hipStream_t s);
// set a rows x cols block to zero
hipError_t zero2d(int rows, int cols, double* dst, int64_t ldd, hipStream_t s);
// scan n values for NaN / Inf; sets *flag = 1 if any
hipError_t nonfinite_scan(const double* v, int64_t n, int* flag, hipStream_t s);
// store diag of a square double matrix to out
hipError_t diag_copy(const double* A, int64_t lda, int n, double* out, hipStream_t s);

// Message returned by kf_last_error(NULL) for the calling thread (calls without a plan).
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------- sparse transition (eqn3)
struct Csr {
    int n = 0;                    // square n x n
    const int* rp = nullptr;      // row_ptr[n + 1] (device)
    const int* ci = nullptr;      // col_idx[nnz] (device)
    const double* v = nullptr;    // values[nnz] (device)
};
constexpr size_t kMaxTransitionLds = 64 * 1024;    // one dense row of P staged in LDS for P F^T
// Y = alpha F A + beta1 C1 + beta2 C2 (A, C1, C2: n x n float64; C1/C2 may be null; Y float or double)
hipError_t spmm_rows(const Csr& F, const double* A, int64_t lda, double alpha, const double* C1, int64_t ldc1,
                     double beta1, const double* C2, int64_t ldc2, double beta2, void* Y, bool y32, int64_t ldy,
                     hipStream_t s);
// G = P F^T (P, G: n x n float64)
hipError_t dense_sparse_t(const Csr& F, const double* P, int64_t ldp, double* G, int64_t ldg, hipStream_t s);
// Y[b] = F X[b] for `rows` vectors (rows of X and Y, leading dimensions ldx, ldy)
hipError_t spmv_rows(const Csr& F, const double* X, int64_t ldx, int rows, double* Y, int64_t ldy, hipStream_t s);

}  // namespace kfmeg
