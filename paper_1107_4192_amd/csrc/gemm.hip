// Grouped MFMA GEMM for gfx950 (CDNA4), float64 or float32 operands.
//
// One launch runs up to kMaxGroup independent problems; each workgroup owns a
// 128 x 128 output tile of one problem. Four 64-wide waves each hold a 64 x 64
// sub-tile as 4 x 4 blocks of the 16x16x4 MFMA (f64 or f32), so every operand
// fragment read from LDS feeds four MFMAs. Operand tiles of 16 k-steps are
// staged through double-buffered LDS in a fixed [k][row] layout whatever the
// global layout (transposing loads are done on the way in). Tiles go from global
// memory straight into LDS (global_load_lds_dwordx4, one k-tile ahead), with no
// staging registers and no LDS store instructions; the one barrier per k-tile sits
// before its last k-step, so the next tile's first fragments are read from LDS while
// that step's MFMAs run. A partial last k-tile, which must read zeros past K, takes
// the register path after the others.
//
// Used for every dense product of the filter and smoother: X P_{t|t-1} and
// X P X^T (eqn8), the rank-m downdate of the covariance update after eqn10,
// the trailing updates of the blocked Cholesky, the triangular products that
// form the smoother gain A_t (eqn11), A_t (P_{t+1|T} - P_{t+1|t}) and its
// product with A_t^T (eqn13).
#include "kf_internal.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <functional>
#include <queue>
#include <vector>

namespace kfmeg {

namespace {

constexpr int BM = 128, BN = 128, BK = 16, NT = 256;

// Device-side problem descriptor: what the kernels read of a GemmProblem, packed into 128
// bytes so that a group of kMaxGroup problems stays a small kernel argument (the whole group
// is passed by value; launches with larger argument blocks ran measurably slower).
struct GemmDesc {
    const void *A, *B, *Cin, *Cin2;
    double* C;
    float* C32;          // shares C's leading dimension
    double* diag;
    void* partial;
    double alpha, beta;  // Cin2 enters with coefficient 1
    int M, N, K, flags;
    int lda, ldb, ldcin, ldcin2, ldc;
    int ksplit, tile_off, tile_begin;
    __device__ __forceinline__ int tiles_m() const { return (M + 127) / 128; }
    __device__ __forceinline__ int tiles_n() const { return (N + 127) / 128; }
};
static_assert(sizeof(GemmDesc) == 128, "GemmDesc layout");

struct GemmGroup {
    GemmDesc p[kMaxGroup];
    int count = 0;
    int total_tiles = 0;
    int remap = 1;     // group equal-cost tiles per XCD (off when K ranges vary per tile)
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Result layout of the 16x16x4 MFMA: lane (lk = lane/16, lr = lane%16) holds C(row, lr) in
// register r, with row = lk + 4 r for f64 and row = 4 lk + r for f32.
template <typename T> struct Acc;
template <> struct Acc<double> {
    using V = d4;
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
    static __device__ __forceinline__ V mfma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Acc<float> {
    using V = f4;
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
    static __device__ __forceinline__ V mfma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

enum : int { G_SCALAR = 1 << 20 };   // internal: operands not 16-byte aligned -> scalar loads

// Load 8 consecutive elements p[0..7]; element q is valid iff q < nvalid.
template <typename T>
__device__ __forceinline__ void load8(T (&r)[8], const T* p, int nvalid, bool vec_ok) {
    if (nvalid >= 8 && vec_ok) {
        if constexpr (sizeof(T) == 8) {
            const d2* v = reinterpret_cast<const d2*>(p);
#pragma unroll
            for (int q = 0; q < 4; ++q) { d2 t = v[q]; r[2 * q] = t.x; r[2 * q + 1] = t.y; }
        } else {
            const f4* v = reinterpret_cast<const f4*>(p);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                f4 t = v[q];
                r[4 * q] = t.x; r[4 * q + 1] = t.y; r[4 * q + 2] = t.z; r[4 * q + 3] = t.w;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = (q < nvalid) ? p[q] : T(0);
    }
}

// Operand A tile: rows i0..i0+BM, k in [k0, k0+BK) clipped to [.., khi); into regs.
template <typename T>
__device__ __forceinline__ void fetch_a(T (&r)[8], const GemmDesc& P, int i0, int k0, int khi, int tid) {
    const T* A = static_cast<const T*>(P.A);
    const bool vec = !(P.flags & G_SCALAR);
    if (!(P.flags & G_TA)) {            // A[i*lda + k]: row r, 8 consecutive k
        const int rr = tid & (BM - 1), ks = (tid >> 7) * 8;
        const int gi = i0 + rr, gk = k0 + ks;
        const int nv = (gi < P.M) ? min(8, khi - gk) : 0;
        if (nv > 0) load8<T>(r, A + (int64_t)gi * P.lda + gk, nv, vec);
        else {
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = T(0);
        }
    } else {                            // A[k*lda + i]: k row, 8 consecutive i
        const int kr = tid >> 4, is = (tid & 15) * 8;
        const int gk = k0 + kr, gi = i0 + is;
        const int nv = (gk < khi) ? min(8, P.M - gi) : 0;
        if (nv > 0) load8<T>(r, A + (int64_t)gk * P.lda + gi, nv, vec);
        else {
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = T(0);
        }
    }
}

template <typename T>
__device__ __forceinline__ void fetch_b_one(T (&r)[8], const T* B, int64_t ldb, bool tb, const GemmDesc& P,
                                            int j0, int k0, int khi, int tid, bool vec) {
    if (!tb) {                          // B[k*ldb + j]: k row, 8 consecutive j
        const int kr = tid >> 4, js = (tid & 15) * 8;
        const int gk = k0 + kr, gj = j0 + js;
        const int nv = (gk < khi) ? min(8, P.N - gj) : 0;
        if (nv > 0) load8<T>(r, B + (int64_t)gk * ldb + gj, nv, vec);
        else {
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = T(0);
        }
    } else {                            // B[j*ldb + k]: row j, 8 consecutive k
        const int rr = tid & (BN - 1), ks = (tid >> 7) * 8;
        const int gj = j0 + rr, gk = k0 + ks;
        const int nv = (gj < P.N) ? min(8, khi - gk) : 0;
        if (nv > 0) load8<T>(r, B + (int64_t)gj * ldb + gk, nv, vec);
        else {
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = T(0);
        }
    }
}

template <typename T>
__device__ __forceinline__ void fetch_b(T (&r)[8], const GemmDesc& P, int j0, int k0, int khi, int tid) {
    const bool tb = P.flags & G_TB;
    const bool vec = !(P.flags & G_SCALAR);
    fetch_b_one<T>(r, static_cast<const T*>(P.B), P.ldb, tb, P, j0, k0, khi, tid, vec);
}

// Write the staged registers into the [k][row] LDS tile.
template <typename T>
__device__ __forceinline__ void stash(T* S, const T (&r)[8], bool transposing, int tid) {
    if (transposing) {                  // regs hold 8 consecutive k of one row
        const int rr = tid & 127, ks = (tid >> 7) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) S[(ks + q) * BM + rr] = r[q];
    } else {                            // regs hold 8 consecutive rows of one k
        const int kr = tid >> 4, is = (tid & 15) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) S[kr * BM + is + q] = r[q];
    }
}

__device__ __forceinline__ double load_any(const void* p, bool f32, int64_t idx) {
    return f32 ? (double)static_cast<const float*>(p)[idx] : static_cast<const double*>(p)[idx];
}

// Map a linear tile index onto (bm, bn) of the lower triangle bm >= bn.
__device__ __forceinline__ void tri_decode(int t, int& bm, int& bn) {
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    bm = r;
    bn = t - r * (r + 1) / 2;
}

// Tile (bm, bn) of linear index `local` in the problem's tile order.
__device__ __forceinline__ void decode_tile(const GemmDesc& P, int local, int& bm, int& bn) {
    if (P.flags & G_LOWER) tri_decode(local, bm, bn);
    else if (P.flags & G_ALOWER) {            // longest tiles (largest K range) first
        bm = P.tiles_m() - 1 - local / P.tiles_n(); bn = local % P.tiles_n();
    } else if (P.flags & G_AUPPER) {
        bm = local / P.tiles_n(); bn = local % P.tiles_n();
    } else if (P.flags & G_BLOWER) {
        bn = local / P.tiles_m(); bm = local % P.tiles_m();
    } else if (P.flags & G_BUPPER) {
        bn = P.tiles_n() - 1 - local / P.tiles_m(); bm = local % P.tiles_m();
    } else {
        // Groups of 8 tile rows, column-major inside a group: the 64 workgroups an XCD runs
        // at once cover about an 8 x 8 block of tiles and share their operand panels in L2.
        constexpr int GM = 8;
        const int per_group = GM * P.tiles_n();
        const int group = local / per_group, first = group * GM;
        const int gsize = min(P.tiles_m() - first, GM);
        const int in = local - group * per_group;
        bm = first + in % gsize;
        bn = in / gsize;
    }
}

// c[b][r] = src(ii, jj) as float64 for the 16 elements of one strip (element 0 where !ok).
__device__ __forceinline__ void gather_strip(double (&c)[4][4], const void* src, bool f32, int64_t ld,
                                             const int (&ii)[4][4], const int (&jj)[4][4], const bool (&ok)[4][4]) {
    if (f32) {
        const float* p = static_cast<const float*>(src);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) c[b][r] = (double)p[ok[b][r] ? (int64_t)ii[b][r] * ld + jj[b][r] : 0];
    } else {
        const double* p = static_cast<const double*>(src);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) c[b][r] = p[ok[b][r] ? (int64_t)ii[b][r] * ld + jj[b][r] : 0];
    }
}

// Result of one tile: raw partial sums (split-K), or C = alpha acc + beta Cin + Cin2
// with the lower / mirror / diagonal / float32 options. Lane (lk, lr) of wave (wm, wn) holds
// acc[a][b][r] = C(i0 + wm + 16a + row(lk, r), j0 + wn + 16b + lr).
// `slot` is the tile's index within a G_TILEPART range; `final` forces the result path (the
// tile-wise reduction calls it with the summed partials).
template <typename T>
__device__ __forceinline__ void epilogue(const GemmDesc& P, const typename Acc<T>::V (&acc)[4][4], int i0,
                                         int j0, int split, int slot, int tid, bool final = false) {
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;
    if (P.ksplit > 1 && !final && (P.flags & G_TILEPART)) {
        T* part = static_cast<T*>(P.partial) + ((int64_t)slot * P.ksplit + split) * kTileElems;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) part[((a * 4 + b) * 4 + r) * NT + tid] = acc[a][b][r];
        return;
    }
    if (P.ksplit > 1 && !final) {
        T* part = static_cast<T*>(P.partial) + (int64_t)split * P.M * P.N;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wm + 16 * a + Acc<T>::row(lk, r), j = j0 + wn + 16 * b + lr;
                    if (i < P.M && j < P.N) part[(int64_t)i * P.N + j] = acc[a][b][r];
                }
        return;
    }
    const bool lower = P.flags & G_LOWER, mirror = P.flags & G_MIRROR;
    const bool cin32 = P.flags & G_CIN32, cin2_32 = P.flags & G_CIN2_32;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        // The strip's Cin / Cin2 values are all loaded before any store: C may alias Cin
        // (in-place updates), so a load that follows a store in program order could not be
        // hoisted above it, and every element would pay a full memory round trip in turn.
        int ii[4][4], jj[4][4];
        bool ok[4][4];
        double c1[4][4], c2[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ii[b][r] = i0 + wm + 16 * a + Acc<T>::row(lk, r);
                jj[b][r] = j0 + wn + 16 * b + lr;
                ok[b][r] = ii[b][r] < P.M && jj[b][r] < P.N && !(lower && jj[b][r] > ii[b][r]);
            }
        if (P.Cin) gather_strip(c1, P.Cin, cin32, P.ldcin, ii, jj, ok);
        if (P.Cin2) gather_strip(c2, P.Cin2, cin2_32, P.ldcin2, ii, jj, ok);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!ok[b][r]) continue;
                const int i = ii[b][r], j = jj[b][r];
                double v = P.alpha * (double)acc[a][b][r];
                if (P.Cin) v += P.beta * c1[b][r];
                if (P.Cin2) v += c2[b][r];
                if (P.C) P.C[(int64_t)i * P.ldc + j] = v;
                if (P.C32) P.C32[(int64_t)i * P.ldc + j] = (float)v;
                if (P.diag && i == j) P.diag[i] = v;
                if (mirror && i > j) {
                    if (P.C) P.C[(int64_t)j * P.ldc + i] = v;
                    if (P.C32) P.C32[(int64_t)j * P.ldc + i] = (float)v;
                }
            }
    }
}

// Generic path: any alignment or leading dimension; branchy loads.
template <typename T>
__global__ __launch_bounds__(NT) void gemm_generic_kernel(GemmGroup G) {
    __shared__ T As[2][BK * BM];
    __shared__ T Bs[2][BK * BN];
    using AV = typename Acc<T>::V;

    const int tid = threadIdx.x;
    const int bid = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int u = 1; u < kMaxGroup; ++u)
        if (u < G.count && bid >= G.p[u].tile_begin) q = u;
    const GemmDesc& P = G.p[q];

    int local = bid - P.tile_begin;
    const int split = local % P.ksplit;
    local /= P.ksplit;
    const int slot = local;
    local += P.tile_off;
    int bm, bn;
    decode_tile(P, local, bm, bn);
    const int i0 = bm * BM, j0 = bn * BN;

    // K range of this tile (triangular operands hold explicit zeros, so trimming is exact).
    int klo = 0, khi = P.K;
    if (P.flags & G_ALOWER) khi = min(khi, i0 + BM);
    if (P.flags & G_BUPPER) khi = min(khi, j0 + BN);
    if (P.flags & G_BLOWER) klo = max(klo, j0);
    if (P.flags & G_AUPPER) klo = max(klo, i0);
    if (P.ksplit > 1) {
        const int span = max(khi - klo, 0);
        const int chunk = ((span + P.ksplit - 1) / P.ksplit + BK - 1) / BK * BK;
        const int a = klo + split * chunk;
        klo = a;
        khi = min(khi, a + chunk);
    }
    const int nk = khi > klo ? (khi - klo + BK - 1) / BK : 0;

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;

    AV acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = AV{0, 0, 0, 0};

    const bool ta_transposing = !(P.flags & G_TA);
    const bool tb_transposing = (P.flags & G_TB);

    if (nk > 0) {
        T ra[8], rb[8];
        fetch_a<T>(ra, P, i0, klo, khi, tid);
        fetch_b<T>(rb, P, j0, klo, khi, tid);
        stash<T>(As[0], ra, ta_transposing, tid);
        stash<T>(Bs[0], rb, tb_transposing, tid);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            const bool more = kt + 1 < nk;
            if (more) {
                const int k0 = klo + (kt + 1) * BK;
                fetch_a<T>(ra, P, i0, k0, khi, tid);
                fetch_b<T>(rb, P, j0, k0, khi, tid);
            }
            const T* as = As[cur];
            const T* bs = Bs[cur];
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T fa[4], fb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) fa[a] = as[(kk + lk) * BM + wm + a * 16 + lr];
#pragma unroll
                for (int b = 0; b < 4; ++b) fb[b] = bs[(kk + lk) * BN + wn + b * 16 + lr];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = Acc<T>::mfma(fa[a], fb[b], acc[a][b]);
            }
            if (more) {
                stash<T>(As[cur ^ 1], ra, ta_transposing, tid);
                stash<T>(Bs[cur ^ 1], rb, tb_transposing, tid);
            }
            __syncthreads();
        }
    }

    epilogue<T>(P, acc, i0, j0, split, slot, tid);
}

// Split-K reduction in fixed split order (deterministic), then the epilogue.
template <typename T>
__global__ void gemm_reduce_kernel(GemmDesc P) {
    const int64_t n = (int64_t)P.M * P.N;
    const T* part = static_cast<const T*>(P.partial);
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / P.N), j = (int)(idx - (int64_t)i * P.N);
        if ((P.flags & G_LOWER) && j > i) continue;
        double s = 0.0;
        for (int sp = 0; sp < P.ksplit; ++sp) s += (double)part[sp * n + idx];
        double v = P.alpha * s;
        if (P.Cin) v += P.beta * load_any(P.Cin, P.flags & G_CIN32, (int64_t)i * P.ldcin + j);
        if (P.Cin2) v += load_any(P.Cin2, P.flags & G_CIN2_32, (int64_t)i * P.ldcin2 + j);
        if (P.C) P.C[(int64_t)i * P.ldc + j] = v;
        if (P.C32) P.C32[(int64_t)i * P.ldc + j] = (float)v;
        if (P.diag && i == j) P.diag[i] = v;
        if ((P.flags & G_MIRROR) && i > j) {
            if (P.C) P.C[(int64_t)j * P.ldc + i] = v;
            if (P.C32) P.C32[(int64_t)j * P.ldc + i] = (float)v;
        }
    }
}


// ------------------------------------------------------------------ fast path
// For operands whose leading dimensions are multiples of 8 elements with 16-byte
// aligned bases (all plan-owned buffers). Out-of-range rows read clamped, in-bounds
// addresses; the register path of a partial last k-tile also zeroes them and k past
// the tile's range with selects, so the loop has no divergent control flow and the
// accumulators stay in the accumulation registers. Layouts are compile-time (bit 0:
// A transposed, bit 1: B transposed); the MASK of a kernel names the layouts it holds,
// and each problem of a group picks its own.

__device__ __forceinline__ int round8(int v) { return (v + 7) & ~7; }

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each XCD
// works on a contiguous run of tiles (which share operand panels in its L2).
__device__ __forceinline__ int xcd_remap(int id, int total) {
    const int xcd = id & 7, local = id >> 3;
    const int per = total >> 3, rem = total & 7;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + local;
}

template <typename T>
__device__ __forceinline__ void vload8(T (&r)[8], const T* p) {
    if constexpr (sizeof(T) == 8) {
        const d2* v = reinterpret_cast<const d2*>(p);
#pragma unroll
        for (int q = 0; q < 4; ++q) { d2 t = v[q]; r[2 * q] = t.x; r[2 * q + 1] = t.y; }
    } else {
        const f4* v = reinterpret_cast<const f4*>(p);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            f4 t = v[q];
            r[4 * q] = t.x; r[4 * q + 1] = t.y; r[4 * q + 2] = t.z; r[4 * q + 3] = t.w;
        }
    }
}

// One operand of the fast path. "Row-contiguous" (A not transposed / B transposed):
// the thread owns one row (of the 128) and 8 consecutive k. "K-major" (A transposed /
// B not transposed): the thread owns one k-row and 8 consecutive rows.
template <typename T, bool KCONTIG>
struct Operand {
    const T* base;      // row base (row-contiguous) or matrix base (k-major)
    int64_t ld;
    int rows;           // extent of the 128-dimension (M or N)
    int K, kcap;        // K extent; last in-bounds 8-segment start along k (row-contiguous)
    int r0, seg;        // this thread's row (row-contiguous) / k-row (k-major) and segment
    bool rowok;
    int segc;           // clamped segment start along the rows (k-major)

    __device__ __forceinline__ void init(const T* M, int64_t ld_, int rows_, int K_, int t0, int tid) {
        ld = ld_; rows = rows_; K = K_;
        if constexpr (KCONTIG) {
            r0 = tid & 127; seg = (tid >> 7) * 8;
            const int row = t0 + r0;
            rowok = row < rows;
            base = M + (int64_t)min(row, rows - 1) * ld;
            kcap = max(round8(K) - 8, 0);
        } else {
            r0 = tid >> 4; seg = (tid & 15) * 8;
            const int col = t0 + seg;
            segc = min(col, max(round8(rows) - 8, 0));
            base = M + segc;
            rowok = true;
            kcap = col;        // first row element of this segment (unclamped)
        }
    }
    __device__ __forceinline__ void fetch(T (&r)[8], int k0, int khi) const {
        T v[8];
        if constexpr (KCONTIG) {
            const int gk = k0 + seg;
            vload8<T>(v, base + min(gk, kcap));
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = (rowok && gk + q < khi) ? v[q] : T(0);
        } else {
            const int gk = k0 + r0;
            vload8<T>(v, base + (int64_t)min(gk, K - 1) * ld);
            const bool kok = gk < khi;
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = (kok && kcap + q < rows) ? v[q] : T(0);
        }
    }
};

// 16 x 16 blocks of this wave's 64 x 64 sub-tile that hold part of C: bit 4 a + b is set unless
// block (a, b) lies wholly below row M, right of column N, or (lower tiles only) above the diagonal.
__device__ __forceinline__ unsigned live_blocks(const GemmDesc& P, int i0, int j0, int wm, int wn) {
    const bool lower = P.flags & G_LOWER;
    unsigned m = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = i0 + wm + 16 * a, c = j0 + wn + 16 * b;
            if (r < P.M && c < P.N && !(lower && c > r + 15)) m |= 1u << (4 * a + b);
        }
    return m;
}

// ---- tiles loaded straight into LDS (global_load_lds_dwordx4: each lane's 16 bytes land at the
// instruction's LDS base + 16 x lane). Each wave issues 4 (float64) or 2 (float32) such loads per
// operand and k-tile. A row-contiguous operand is staged as [k group][row][E] (a lane loads E
// consecutive k of one row), a k-major one as [k][column]. Rows and columns past the matrix read clamped, in-bounds
// addresses (their products only reach outputs outside C); k never runs past the tile's range
// here, since a partial last k-tile takes the register path, which zeroes k >= khi.
typedef __attribute__((address_space(3))) void lds_void;

// E = elements per 16-byte chunk (2 float64 or 4 float32); a row-contiguous operand is staged as
// [k group of E][row][E], a k-major one as [k][column].
template <typename T, bool RC>
struct DmaOp {
    static constexpr int E = 16 / sizeof(T);
    const T* p0;   // row-contiguous: row i0 + lane; k-major: matrix base + this lane's E columns
    const T* p1;   // row-contiguous: row i0 + 64 + lane
    int64_t ld;
    __device__ __forceinline__ void init(const T* M, int64_t ld_, int rows, int t0, int lane) {
        ld = ld_;
        if constexpr (RC) {
            p0 = M + (int64_t)min(t0 + lane, rows - 1) * ld;
            p1 = M + (int64_t)min(t0 + 64 + lane, rows - 1) * ld;
        } else {   // float64: 64 lanes x 2 columns per k-row; float32: 32 lanes x 4 columns, two k-rows
            const int col = sizeof(T) == 8 ? 2 * lane : 4 * (lane & 31);
            p0 = M + min(t0 + col, max(round8(rows) - E, 0));
            p1 = p0;
        }
    }
    // tile k0..k0+15 into S
    __device__ __forceinline__ void issue(int k0, T* S, int wave, int lane) const {
        constexpr int NI = sizeof(T) == 8 ? 4 : 2;   // loads per wave and operand
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            if constexpr (RC) {
                const int c = sizeof(T) == 8 ? wave * 2 + (i >> 1) : wave, h = i & 1;
                const T* src = (h ? p1 : p0) + k0 + E * c;
                __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(S + (c * 128 + h * 64) * E), 16, 0, 0);
            } else if constexpr (sizeof(T) == 8) {
                const int kr = wave * 4 + i;
                const T* src = p0 + (int64_t)(k0 + kr) * ld;
                __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(S + kr * 128), 16, 0, 0);
            } else {
                const int kr = (wave * 2 + i) * 2;          // k-rows kr (lanes 0-31) and kr + 1 (32-63)
                const T* src = p0 + (int64_t)(k0 + kr + (lane >> 5)) * ld;
                __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(S + kr * 128), 16, 0, 0);
            }
        }
    }
};

// register-path store of a row-contiguous operand in the [k group][row][E] layout
template <typename T>
__device__ __forceinline__ void stash_groups(T* S, const T (&r)[8], int tid) {
    const int rr = tid & 127;
    if constexpr (sizeof(T) == 8) {
        const int p0 = (tid >> 7) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) reinterpret_cast<d2*>(S)[(p0 + q) * 128 + rr] = d2{r[2 * q], r[2 * q + 1]};
    } else {
        const int p0 = (tid >> 7) * 2;
#pragma unroll
        for (int q = 0; q < 2; ++q)
            reinterpret_cast<f4*>(S)[(p0 + q) * 128 + rr] = f4{r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]};
    }
}

template <typename T, bool TA, bool TB, bool EDGE>
__device__ __forceinline__ void fast_tile_dma(const GemmDesc& P, int bm, int bn, int split, int slot, T* As0,
                                              T* As1, T* Bs0, T* Bs1) {
    using AV = typename Acc<T>::V;
    constexpr int E = 16 / sizeof(T);
    const int tid = threadIdx.x;
    const int i0 = bm * BM, j0 = bn * BN;
    int klo = 0, khi = P.K;
    if (P.flags & G_ALOWER) khi = min(khi, i0 + BM);
    if (P.flags & G_BUPPER) khi = min(khi, j0 + BN);
    if (P.flags & G_BLOWER) klo = max(klo, j0);
    if (P.flags & G_AUPPER) klo = max(klo, i0);
    if (P.ksplit > 1) {
        const int span = max(khi - klo, 0);
        const int chunk = ((span + P.ksplit - 1) / P.ksplit + BK - 1) / BK * BK;
        klo = klo + split * chunk;
        khi = min(khi, klo + chunk);
    }
    const int nk = khi > klo ? (khi - klo + BK - 1) / BK : 0;
    const bool tail = nk > 0 && ((khi - klo) & (BK - 1)) != 0;   // the last k-tile is partial
    constexpr bool RA = !TA, RB = TB;

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const unsigned live = EDGE ? live_blocks(P, i0, j0, __builtin_amdgcn_readfirstlane(wm),
                                             __builtin_amdgcn_readfirstlane(wn)) : 0xFFFFu;
    DmaOp<T, RA> da;
    DmaOp<T, RB> db;
    da.init(static_cast<const T*>(P.A), P.lda, P.M, i0, lane);
    db.init(static_cast<const T*>(P.B), P.ldb, P.N, j0, lane);

    AV acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = AV{0, 0, 0, 0};

    auto put = [&](T* Sa, T* Sb, const T (&ra)[8], const T (&rb)[8]) {
        if constexpr (RA) stash_groups<T>(Sa, ra, tid); else stash<T>(Sa, ra, false, tid);
        if constexpr (RB) stash_groups<T>(Sb, rb, tid); else stash<T>(Sb, rb, false, tid);
    };
    auto rd = [&](const T* S, bool rc, int k, int row) -> T {
        return rc ? S[((k / E) * 128 + row) * E + (k % E)] : S[k * 128 + row];
    };
    auto tile = [&](const T* as, const T* bs) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = rd(as, RA, kk + lk, wm + a * 16 + lr);
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = rd(bs, RB, kk + lk, wn + b * 16 + lr);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (!EDGE || (live >> (4 * a + b)) & 1u) acc[a][b] = Acc<T>::mfma(fa[a], fb[b], acc[a][b]);
        }
    };
    const int nfull = tail ? nk - 1 : nk;    // k-tiles loaded straight into LDS
    if (nfull > 0) {
        // One barrier per k-tile, between its third and fourth k-steps: by then tile k + 1 has
        // landed (its loads were issued as tile k began) and every wave has read all of tile k
        // (the fourth k-step's fragments are read before it), so after it the next tile's first
        // fragments are read while the fourth k-step's MFMAs run.
        auto frag = [&](const T* as, const T* bs, int kk, T (&fa)[4], T (&fb)[4]) {
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = rd(as, RA, kk + lk, wm + a * 16 + lr);
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = rd(bs, RB, kk + lk, wn + b * 16 + lr);
        };
        auto mfmas = [&](const T (&fa)[4], const T (&fb)[4]) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (!EDGE || (live >> (4 * a + b)) & 1u) acc[a][b] = Acc<T>::mfma(fa[a], fb[b], acc[a][b]);
        };
        da.issue(klo, As0, wv, lane);
        db.issue(klo, Bs0, wv, lane);
        __syncthreads();
        T fa0[4], fb0[4];
        frag(As0, Bs0, 0, fa0, fb0);
        for (int kt = 0; kt < nfull; kt += 2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = kt + h;
                if (k >= nfull) break;
                const T* as = h ? As1 : As0;
                const T* bs = h ? Bs1 : Bs0;
                T* na = h ? As0 : As1;
                T* nb = h ? Bs0 : Bs1;
                const bool next = k + 1 < nfull;
                if (next) {
                    da.issue(klo + (k + 1) * BK, na, wv, lane);
                    db.issue(klo + (k + 1) * BK, nb, wv, lane);
                }
                T fa1[4], fb1[4], fa2[4], fb2[4], fa3[4], fb3[4];
                frag(as, bs, 4, fa1, fb1);
                mfmas(fa0, fb0);
                frag(as, bs, 8, fa2, fb2);
                mfmas(fa1, fb1);
                frag(as, bs, 12, fa3, fb3);
                mfmas(fa2, fb2);
                __syncthreads();
                if (next) frag(na, nb, 0, fa0, fb0);
                mfmas(fa3, fb3);
            }
        }
    }
    if (tail) {   // the partial last k-tile through registers (k >= khi read as zero)
        Operand<T, RA> oa;
        Operand<T, RB> ob;
        oa.init(static_cast<const T*>(P.A), P.lda, P.M, P.K, i0, tid);
        ob.init(static_cast<const T*>(P.B), P.ldb, P.N, P.K, j0, tid);
        T ra[8], rb[8];
        const int k0 = klo + nfull * BK;
        oa.fetch(ra, k0, khi);
        ob.fetch(rb, k0, khi);
        T* sa = (nfull & 1) ? As1 : As0;   // last read by tile nfull - 2, before the previous barrier
        T* sb = (nfull & 1) ? Bs1 : Bs0;
        put(sa, sb, ra, rb);
        __syncthreads();
        tile(sa, sb);
    }
    epilogue<T>(P, acc, i0, j0, split, slot, tid);
}

// V selects a separately named instantiation: 1 for the smoother's N x N x N
// products of the float64 path, 2 for those of the mixed path, 3 for the float64
// products of a smoother pass serialised onto one stream for measurement, 4 for the
// smoother gain's blocked Cholesky and triangular solves, so that profilers report
// them on their own. MASK is the set of operand
// layouts compiled in (bit L for layout L); each problem of the group picks its own.
template <typename T, int V, int MASK>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmGroup G) {
    __shared__ T Ad0[BK * BM], Ad1[BK * BM], Bd0[BK * BN], Bd1[BK * BN];
    int q = 0;
#pragma unroll
    for (int u = 1; u < kMaxGroup; ++u)
        if (u < G.count && (int)blockIdx.x >= G.p[u].tile_begin) q = u;
    const GemmDesc& P = G.p[q];
    int local = (int)blockIdx.x - P.tile_begin;
    // Tiles of equal cost are grouped per XCD (each problem's range on its own, so that the
    // problems of a group keep their dispatch order); tiles whose K range varies (triangular
    // operands) keep the round-robin spread so that every XCD gets a fair share.
    if (G.remap) {
        const int end = q + 1 < G.count ? G.p[q + 1].tile_begin : (int)gridDim.x;
        local = xcd_remap(local, end - P.tile_begin);
    }
    const int split = local % P.ksplit;
    local /= P.ksplit;
    const int slot = local;
    local += P.tile_off;
    int bm, bn;
    decode_tile(P, local, bm, bn);
    const int lay = (P.flags & G_TA ? 1 : 0) | (P.flags & G_TB ? 2 : 0);
    // Tiles with at most 48 rows or columns left inside C (the 4-wide edge of N = 5124, for
    // instance) skip the MFMAs of their empty 16 x 16 blocks, which shortens every wave of the
    // tile; they run a separate instantiation, so interior tiles are unchanged. (Wider edges and
    // the diagonal tiles of lower outputs would only idle some waves while the others set the pace.)
    const bool edge = P.M - bm * BM <= 48 || P.N - bn * BN <= 48;
#define KF_T(ta, tb)                                                                    \
    do {                                                                                \
        if (edge) fast_tile_dma<T, ta, tb, true>(P, bm, bn, split, slot, Ad0, Ad1, Bd0, Bd1); \
        else fast_tile_dma<T, ta, tb, false>(P, bm, bn, split, slot, Ad0, Ad1, Bd0, Bd1);     \
    } while (0)
    if ((MASK & 1) && lay == 0) KF_T(false, false);
    else if ((MASK & 2) && lay == 1) KF_T(true, false);
    else if ((MASK & 4) && lay == 2) KF_T(false, true);
    else if ((MASK & 8) && lay == 3) KF_T(true, true);
#undef KF_T
}

// Tile-wise reduction of a G_TILEPART range: one workgroup per tile sums the k slices in a
// fixed order (deterministic) and applies the epilogue.
template <typename T>
__global__ __launch_bounds__(NT) void gemm_tile_reduce_kernel(GemmDesc P) {
    using AV = typename Acc<T>::V;
    const int slot = blockIdx.x, tid = threadIdx.x;
    int bm, bn;
    decode_tile(P, P.tile_off + slot, bm, bn);
    const T* part = static_cast<const T*>(P.partial) + (int64_t)slot * P.ksplit * kTileElems;
    AV acc[4][4];
    // slice by slice, so that each slice's 64 loads are in flight together
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] = part[((a * 4 + b) * 4 + r) * NT + tid];
    for (int sp = 1; sp < P.ksplit; ++sp) {
        const T* sl = part + (int64_t)sp * kTileElems;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[a][b][r] += sl[((a * 4 + b) * 4 + r) * NT + tid];
    }
    epilogue<T>(P, acc, bm * BM, bn * BN, 0, slot, tid, true);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Fast path requirements for one operand stored with leading dimension ld whose
// contiguous extent is `contig`: ld a multiple of 8, 16-byte aligned base.
bool fast_ok(const void* p, int64_t ld, int contig) {
    return p && aligned16(p) && ld % 8 == 0 && ld >= ((contig + 7) & ~7);
}

// Only the layout masks a variant is used with are compiled for it (the eqn13 products are all
// NT; the gain's launches NN, TN or NT); any other mask runs the unnamed variant's kernel, which
// computes the same thing. This keeps the library's build time and size in check.
template <typename T, int V>
hipError_t launch_fast(const GemmGroup& G, int mask, hipStream_t s) {
    const dim3 grid(G.total_tiles), block(NT);
#define KF_L(m) hipLaunchKernelGGL((gemm_kernel<T, V, m>), grid, block, 0, s, G)
    if constexpr (V == 0) {
        switch (mask) {
            case 1: KF_L(1); break;
            case 2: KF_L(2); break;
            case 4: KF_L(4); break;
            case 8: KF_L(8); break;
            case 5: KF_L(5); break;
            default: KF_L(15); break;
        }
    } else if constexpr (V == 4) {
        switch (mask) {
            case 1: KF_L(1); break;
            case 2: KF_L(2); break;
            case 4: KF_L(4); break;
            default: return launch_fast<T, 0>(G, mask, s);
        }
    } else {
        if (mask != 4) return launch_fast<T, 0>(G, mask, s);
        KF_L(4);
    }
#undef KF_L
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_launch(Dt dt, GemmProblem* probs, int count, hipStream_t s, hipEvent_t main_done) {
    GemmGroup G;
    int total = 0;
    const int esz = dt == Dt::F64 ? 8 : 4;
    const int vec_elems = 16 / esz;
    bool fast = true;
    int layouts[kMaxGroup] = {};
    int tile_cnt[kMaxGroup] = {};
    auto fits = [](int64_t v) { return v >= 0 && v <= INT32_MAX; };
    for (int u = 0; u < count; ++u) {
        const GemmProblem& p = probs[u];
        if (p.M <= 0 || p.N <= 0) continue;
        const int ks = p.ksplit < 1 ? 1 : p.ksplit;
        const int tm = (p.M + BM - 1) / BM, tn = (p.N + BN - 1) / BN;
        if ((p.flags & G_LOWER) && p.M != p.N) return hipErrorInvalidValue;
        if (p.Cin2 && p.gamma != 1.0) return hipErrorInvalidValue;
        if (p.C && p.C32 && p.ldc32 != p.ldc) return hipErrorInvalidValue;
        if (!fits(p.lda) || !fits(p.ldb) || !fits(p.ldcin) || !fits(p.ldcin2) || !fits(p.ldc) || !fits(p.ldc32))
            return hipErrorInvalidValue;
        const bool ta = p.flags & G_TA, tb = p.flags & G_TB;
        int flags = p.flags;
        bool vec = aligned16(p.A) && aligned16(p.B) && p.lda % vec_elems == 0 && p.ldb % vec_elems == 0;
        if (!vec) flags |= G_SCALAR;
        const int all = (p.flags & G_LOWER) ? tm * (tm + 1) / 2 : tm * tn;
        if (p.tile_off < 0 || p.tile_off > all) return hipErrorInvalidValue;
        const int tiles = p.tile_cnt < 0 ? all - p.tile_off : std::min(p.tile_cnt, all - p.tile_off);
        if ((p.flags & G_TILEPART) && (ks < 2 || !p.partial)) return hipErrorInvalidValue;
        if (tiles == 0) continue;
        if (G.count >= kMaxGroup) return hipErrorInvalidValue;
        fast = fast && p.K > 0 && fast_ok(p.A, p.lda, ta ? p.M : p.K) && fast_ok(p.B, p.ldb, tb ? p.K : p.N);
        GemmDesc d;
        d.A = p.A; d.B = p.B; d.Cin = p.Cin; d.Cin2 = p.Cin2;
        d.C = p.C; d.C32 = p.C32; d.diag = p.diag; d.partial = p.partial;
        d.alpha = p.alpha; d.beta = p.beta;
        d.M = p.M; d.N = p.N; d.K = p.K; d.flags = flags;
        d.lda = (int)p.lda; d.ldb = (int)p.ldb; d.ldcin = (int)p.ldcin; d.ldcin2 = (int)p.ldcin2;
        d.ldc = (int)(p.C ? p.ldc : p.ldc32);
        d.ksplit = ks; d.tile_off = p.tile_off; d.tile_begin = total;
        total += tiles * ks;
        layouts[G.count] = (ta ? 1 : 0) | (tb ? 2 : 0);
        tile_cnt[G.count] = tiles;
        G.p[G.count++] = d;
    }
    if (G.count == 0) return hipSuccess;
    G.total_tiles = total;
    int mask = 0;
    G.remap = 1;
    for (int u = 0; u < G.count; ++u) {
        mask |= 1 << layouts[u];
        if (G.p[u].flags & (G_ALOWER | G_AUPPER | G_BLOWER | G_BUPPER)) G.remap = 0;
    }
    const int variant = (G.p[0].flags & G_NXN) ? 1 : (G.p[0].flags & G_NXN_MIXED) ? 2
                      : (G.p[0].flags & G_NXN_SERIAL) ? 3 : (G.p[0].flags & G_GAIN) ? 4 : 0;
    hipError_t e;
    if (fast) {
        if (dt == Dt::F64)
            e = variant == 1 ? launch_fast<double, 1>(G, mask, s)
              : variant == 2 ? launch_fast<double, 2>(G, mask, s)
              : variant == 3 ? launch_fast<double, 3>(G, mask, s)
              : variant == 4 ? launch_fast<double, 4>(G, mask, s) : launch_fast<double, 0>(G, mask, s);
        else
            e = variant == 2 ? launch_fast<float, 2>(G, mask, s) : launch_fast<float, 0>(G, mask, s);
    } else {
        if (dt == Dt::F64) hipLaunchKernelGGL(gemm_generic_kernel<double>, dim3(total), dim3(NT), 0, s, G);
        else hipLaunchKernelGGL(gemm_generic_kernel<float>, dim3(total), dim3(NT), 0, s, G);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (main_done && (e = hipEventRecord(main_done, s)) != hipSuccess) return e;
    for (int u = 0; u < G.count; ++u) {
        const GemmDesc& p = G.p[u];
        if (p.ksplit <= 1) continue;
        if (p.flags & G_TILEPART) {
            if (dt == Dt::F64) hipLaunchKernelGGL(gemm_tile_reduce_kernel<double>, dim3(tile_cnt[u]), dim3(NT), 0, s, p);
            else hipLaunchKernelGGL(gemm_tile_reduce_kernel<float>, dim3(tile_cnt[u]), dim3(NT), 0, s, p);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            continue;
        }
        const int64_t n = (int64_t)p.M * p.N;
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
        if (dt == Dt::F64) hipLaunchKernelGGL(gemm_reduce_kernel<double>, dim3(blocks), dim3(256), 0, s, p);
        else hipLaunchKernelGGL(gemm_reduce_kernel<float>, dim3(blocks), dim3(256), 0, s, p);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int gemm_tiles(const GemmProblem& p) {
    const int tm = (p.M + BM - 1) / BM, tn = (p.N + BN - 1) / BN;
    return (p.flags & G_LOWER) ? tm * (tm + 1) / 2 : tm * tn;
}

int gemm_slots() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    return 2 * cus;   // the fast path runs two workgroups per compute unit
}

namespace {

// Makespan, in units of one whole tile's time, of `full` whole tiles followed by
// (tiles - full) * k pieces of 1/k each, greedily placed on `slots` equal workers in
// dispatch order (how the hardware hands out workgroups).
double makespan(int tiles, int full, int k, int slots) {
    std::vector<double> busy(slots, 0.0);
    std::priority_queue<double, std::vector<double>, std::greater<double>> q(std::greater<double>(), busy);
    double mk = 0.0;
    auto place = [&](double d) {
        const double t = q.top() + d;
        q.pop();
        q.push(t);
        mk = std::max(mk, t);
    };
    for (int u = 0; u < full; ++u) place(1.0);
    for (int u = 0; u < (tiles - full) * k; ++u) place(1.0 / k);
    return mk;
}

}  // namespace

TailSplit choose_tail_split(int tiles, int kiters, int slots, int max_units) {
    TailSplit best;
    if (tiles <= 0 || slots <= 0 || kiters < 8) return best;
    best.full = tiles;
    double best_cost = makespan(tiles, tiles, 1, slots);
    // A split piece writes and re-reads one tile of partial sums: priced at 2/kiters of a
    // whole tile's time per piece (the tile's own operand traffic is about kiters tile loads).
    const double piece = 2.0 / kiters;
    for (int full = (tiles / slots) * slots; full >= 0; full -= slots) {
        for (int k = 2; k <= 4; ++k) {
            const int units = (tiles - full) * k;
            if (units <= 0 || units > max_units) continue;
            const double cost = makespan(tiles, full, k, slots) + piece * units / slots;
            if (cost < 0.97 * best_cost) {
                best_cost = cost;
                best.full = full;
                best.k = k;
            }
        }
        if (full == 0) break;
    }
    if (best.k == 1) best.full = tiles;
    return best;
}

hipError_t gemm_launch_tail(Dt dt, const GemmProblem& p, TailSplit ts, void* ws, hipStream_t s,
                            hipEvent_t main_done) {
    GemmProblem g[2] = {p, p};
    if (ts.k <= 1 || !ws || p.ksplit > 1 || p.tile_off != 0 || p.tile_cnt >= 0)
        return gemm_launch(dt, g, 1, s, main_done);
    g[0].tile_cnt = ts.full;
    g[1].tile_off = ts.full;
    g[1].ksplit = ts.k;
    g[1].flags |= G_TILEPART;
    g[1].partial = ws;
    return gemm_launch(dt, g, 2, s, main_done);
}

}  // namespace kfmeg
