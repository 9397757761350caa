// Plan, filter, smoother and MNE entry points (the C ABI of include/kfmeg.h).
//
// Filter step t (eqn6-eqn10 and the covariance update after eqn10), with
// P_prev = P_{t-1|t-1} and P_pred = P_prev + Q (F = I) or F P_prev F^T + Q:
//   B   = X P_pred                       m x N   MFMA GEMM, split-K (F = I: X P_prev + X Q, X Q formed once)
//   S   = B X^T + R                      m x m   MFMA GEMM, split-K (fixed-order reduction)
//   L Li = chol(S)                        m x m   blocked Cholesky fused with L^{-1}
//   C   = Li B                           m x N   triangular MFMA product (K range trimmed)
//   x  += C^T (Li (y_t - X x_pred))               three wave-reduction kernels (B-row products
//                                                 for several data sets)
//   P_t = P_pred - C^T C                 N x N   lower tiles only, mirrored store (exact symmetry),
//                                                diagonal out, written straight into store slot t
// since K = P_pred X^T S^{-1} = C^T Li and K X P_pred = C^T C.
//
// Smoother step t (eqn11-eqn13, RTS reading), P_t = P_{t|t}, Pn = P_{t+1|t}:
//   L = chol(Pn)                         N x N   outer-blocked Cholesky (diagonal blocks inverted),
//                                                eight steps per batch, batches on side streams
//   Y = L^{-1} F P_t ; A_t^T = L^{-T} Y  N x N   two blocked triangular solves, then A_t^T is
//                                                transposed in place: A_t = P_t F^T Pn^{-1}
//   x_{t|T} = x_{t|t} + A_t (x_{t+1|T} - F x_{t|t})
//   D   = P_{t+1|T} - Pn ;  M = A_t D    N x N   elementwise pass, MFMA GEMM (last wave split along K)
//   P_{t|T} = P_t + M A_t^T              N x N   lower tiles + mirror, diagonal out
//
// Mixed precision runs the downdate C^T C and the eqn13 products M and M A^T on FP32 MFMA with
// FP32 accumulation, keeps X P_pred, the Cholesky of S and of P_{t+1|t}, the gain A_t and every
// epilogue in FP64, and may store P_{t|t} in FP32. The mean-only smoother (kf_smooth_means)
// replaces the smoother step by one N x N matrix-vector product per step over kept gain factors;
// kf_smooth_assoc regroups the smoother as an associative scan over time.
#include "kf_internal.h"
#include "arena.h"
#include "../../include/kfmeg.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace kfmeg;

struct kf_plan {
    int64_t N = 0, m = 0, Tmax = 0;
    kf_options opt{};
    hipStream_t stream = nullptr;
    int64_t ldN = 0, ldm = 0;
    std::vector<void*> allocs;
    DeviceArena* arena = nullptr;           // serving: buffers come from the server's arena

    // model
    double *X = nullptr, *Q = nullptr, *R = nullptr, *x0 = nullptr, *P0 = nullptr;
    double* XQ = nullptr;                   // X Q (m x N): X (P + Q) = X P + X Q
    // filter workspace
    double *Bm = nullptr, *e = nullptr, *w = nullptr, *xw = nullptr;
    // Innovation covariance without the noise, St = X P_{t|t-1} X^T (m x m), kept from step to step,
    // Sw = St + R its factorisation workspace, XQX = X Q X^T, Hm = L_t^{-1} R; the inverse factor
    // L_t^{-1} of the last two steps (step t in slot t & 1)
    double *St = nullptr, *Sw = nullptr, *XQX = nullptr, *Hm = nullptr;
    double* Li2[2] = {nullptr, nullptr};
    double* Gm = nullptr;                   // G_t = X C_t^T (m x m) for the recursion of B
    double* Sck = nullptr;                  // checkpointed store: St at every segment start
    // C_t = L_t^{-1} B_t of the last two steps (step t in slot t & 1): the downdate of step t may
    // still be reading C_t while step t + 1 forms C_{t+1}
    double* Cm2[2] = {nullptr, nullptr};
    float* Cm32x[2] = {nullptr, nullptr};
    double* Bck = nullptr;                  // checkpointed store: B_t at every segment start (t % stride == 0)
    double* partial = nullptr;
    size_t partial_elems = 0;
    double* Pw[2] = {nullptr, nullptr};     // float64 working pair (store in float32 or checkpointed)
    // covariance store
    bool store32 = false;
    int stride = 1;                         // keep slots t with (t+1) % stride == 0 and t = T-1
    void* store = nullptr;
    int64_t nslots = 0;
    // segment buffer for recomputation (checkpointed mode)
    void* seg = nullptr;
    // smoother workspace
    // Smoother gains are formed for up to `gbatch` time steps at once (they are independent
    // given the stored P_{t|t}) on `nprod` side streams, ahead of the back-recursion; the
    // gains, and the upcast P_{t|t} they came from, rotate through nprod + 1 sets.
    int gbatch = 1;
    int nprod = 1;                          // gain batches in flight at once, one side stream each
    // per side stream and batch slot: W (P_{t+1|t}, then its factor L), Li (L^{-1} F P_{t|t}) and Dg
    // (inverses of L's diagonal blocks, gnb columns wide, then an gnb x N solve panel)
    double *W[kMaxProd][kMaxBatch] = {}, *Li[kMaxProd][kMaxBatch] = {}, *Dg[kMaxProd][kMaxBatch] = {};
    int gnb = kGainBlock;                   // outer block of the gain's factorisation and solves
    int64_t gld = 0;                        // leading dimension of the diagonal-block inverses
    double* Ab[kMaxProd + 1][kMaxBatch] = {};   // gain sets: nprod + 1 in rotation
    double* Pt64[kMaxProd + 1][kMaxBatch] = {};
    float* A32[kMaxProd + 1][kMaxBatch] = {};
    double* Ps[2] = {nullptr, nullptr};
    double *Dm = nullptr, *Mm = nullptr;    // D = P_{t+1|T} - P_{t+1|t} and M = A_t D (float64 path)
    float *D32 = nullptr, *M32 = nullptr;   // the same in float32 (mixed path)
    // tail splitting of the two N x N x N products of the back-recursion (M = A_t D, whole;
    // P_t + M A_t^T, lower tiles), chosen once per plan
    TailSplit ts_m, ts_low;
    void* tail_ws = nullptr;
    void* tail_ws64 = nullptr;              // mixed plan with a transition F: eqn13 runs in float64
    hipStream_t s2[kMaxProd] = {};
    // filter: the m x m chain on a few compute units of their own (its small, latency-bound
    // launches then never wait behind downdate workgroups), the downdates on the others
    hipStream_t sc = nullptr, sdm = nullptr;
    hipEvent_t ev_start = nullptr, ev_gain[kMaxProd + 1] = {}, ev_chain[kMaxProd + 1] = {};
    // filter: L_t^{-1} formed, G_t formed, B_t refreshed (t % kBRefresh == 0), N-side of step t done,
    // C_t formed, downdate t done; slot t & 1
    hipEvent_t ev_fl[2] = {}, ev_fg[2] = {}, ev_fr[2] = {}, ev_fa[2] = {}, ev_cc[2] = {}, ev_dd[2] = {};
    // status
    DevStatus* dstatus = nullptr;
    DevStatus* hstatus = nullptr;
    int64_t T_done = 0;
    int64_t B_done = 1;           // data sets of the last filter call
    double* xf_last = nullptr;    // caller's x_filt of the last filter call (for the smoother)
    // several data sets through one covariance pass: the means of all data sets advance
    // together as B-row products (buffers sized for bcap data sets, grown on demand)
    int64_t bcap = 0;
    double *Eb = nullptr, *Wb = nullptr, *Xb0 = nullptr, *Vb = nullptr;
    // gain factors of every filter step for the mean-only smoother: C_t (m x ldN),
    // L_t^-1 (m x ldm) and L_t^-1 e_t (wcap rows of ldm per step)
    bool keep = false;
    double *fac_C = nullptr, *fac_L = nullptr, *fac_w = nullptr;
    int64_t wcap = 0;
    std::vector<double*> bfac_w;            // per-data-set factor buffers grown past one data set
    // transition matrix F of eqn3 (CSR on the device) and its transpose; absent: F = I
    bool hasF = false;
    Csr F, Ft;
    std::vector<void*> fallocs;
    double *Fg = nullptr, *Fp = nullptr, *xp = nullptr;   // P F^T, F P F^T + Q, F x
    double* Ub = nullptr;                   // B x ldN: F applied to B means
    std::string err;
    // profiling of the smoother's N x N x N products (event pairs around each launch); `serial`
    // runs the smoother's gain batches on the plan's stream too, so that each product runs alone
    bool prof = false;
    bool serial = false;
    std::vector<hipEvent_t> ev;
    std::vector<double> ev_flops;
    size_t ev_used = 0;
    double prof_ms = 0.0, prof_flops = 0.0;
    int64_t prof_launches = 0;
};

namespace {

thread_local std::string g_err;

// roctx range around the host-side enqueue of one step or batch (visible in a marker trace;
// a no-op without a profiler).
struct Range {
    Range(const char* fmt, long long a, long long b = -1) {
        char buf[96];
        snprintf(buf, sizeof buf, fmt, a, b);
        roctxRangePushA(buf);
    }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Fail {
    kf_status st;
};

#define HIPCK(expr)                                                                      \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) {                                                          \
            p->err = std::string(#expr) + ": " + hipGetErrorString(_e);                  \
            return KF_EHIP;                                                              \
        }                                                                                \
    } while (0)

bool mixed(const kf_plan* p) { return p->opt.precision == KF_MIXED; }

kf_status alloc_bytes(kf_plan* p, void** out, size_t bytes) {
    void* ptr = nullptr;
    if (bytes == 0) bytes = 1;
    if (p->arena) {
        ptr = p->arena->alloc(bytes);
    } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    if (!ptr) {
        p->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
        return KF_ENOMEM;
    }
    p->allocs.push_back(ptr);
    *out = ptr;
    return KF_OK;
}

template <typename T>
kf_status alloc(kf_plan* p, T** out, size_t elems) {
    void* ptr = nullptr;
    kf_status st = alloc_bytes(p, &ptr, (elems ? elems : 1) * sizeof(T));
    if (st == KF_OK) *out = static_cast<T*>(ptr);
    return st;
}

#define TRY(expr)                           \
    do {                                    \
        kf_status _s = (expr);              \
        if (_s != KF_OK) return _s;         \
    } while (0)

size_t slot_elems(const kf_plan* p) { return (size_t)p->N * p->ldN; }

// Kept slots are float64 unless the whole store is float32 (stride 1): checkpoints stay
// float64 so that recomputed covariances match the full store bit for bit (a float32
// store is emulated by rounding wherever the smoother reads a covariance).
bool slot64(const kf_plan* p) { return !p->store32 || p->stride > 1; }

void* slot_ptr(const kf_plan* p, int64_t idx) {
    const size_t esz = slot64(p) ? 8 : 4;
    return static_cast<char*>(p->store) + (size_t)idx * slot_elems(p) * esz;
}

// Is filtered covariance t (0-based) kept in the store?  Which slot holds it?
bool kept(const kf_plan* p, int64_t t, int64_t T) { return p->stride == 1 || (t + 1) % p->stride == 0 || t == T - 1; }
int64_t slot_of(const kf_plan* p, int64_t t, int64_t T) {
    if (p->stride == 1) return t;
    if (t == T - 1) return (T - 1) / p->stride;   // after the last full checkpoint
    return (t + 1) / p->stride - 1;
}
int64_t slots_needed(int64_t T, int stride) { return stride == 1 ? T : T / stride + 1; }

size_t store_bytes(int64_t N, int64_t ldN, int64_t T, bool s32, int stride) {
    return (size_t)slots_needed(T, stride) * (size_t)N * ldN * (s32 && stride == 1 ? 4 : 8);
}

// Device bytes kf_smooth_assoc allocates for one call over T steps: the T - 1 scan elements E_t,
// the scratch of one launch group of combines with an E E' product and of one without (kMaxGroup
// / 2 and kMaxGroup matrices), and two N-vectors.
size_t assoc_bytes(int64_t N, int64_t ldN, int64_t T) {
    const size_t mats = (size_t)std::max<int64_t>(T - 1, 0) + kMaxGroup / 2 + kMaxGroup;
    return mats * (size_t)N * ldN * 8 + 2 * (size_t)N * 8;
}

// Tail splits of the back-recursion's M = A_t D (whole) and P_t + M A_t^T (lower) products.
constexpr int kTailUnits = 2048;
void tail_splits(int64_t N, TailSplit& ts_m, TailSplit& ts_low) {
    GemmProblem g;
    g.M = g.N = g.K = (int)N;
    const int slots = gemm_slots(), kiters = (int)((N + 15) / 16);
    ts_m = choose_tail_split(gemm_tiles(g), kiters, slots, kTailUnits);
    g.flags = G_LOWER;
    ts_low = choose_tail_split(gemm_tiles(g), kiters, slots, kTailUnits);
}

size_t tail_bytes(int64_t N, bool mix) {
    TailSplit a, b;
    tail_splits(N, a, b);
    GemmProblem g;
    g.M = g.N = g.K = (int)N;
    const int full = gemm_tiles(g);
    g.flags = G_LOWER;
    const int low = gemm_tiles(g);
    const size_t units = std::max<size_t>(a.k > 1 ? (size_t)(full - a.full) * a.k : 0,
                                          b.k > 1 ? (size_t)(low - b.full) * b.k : 0);
    return units * kTileElems * (mix ? 4 : 8);
}

// Gain factors kept for the mean-only smoother (one data set).
size_t factor_bytes(int64_t N, int64_t m, int64_t T) {
    const int64_t ldN = round_up(N, 16), ldm = round_up(m, 16);
    return 8 * (size_t)T * ((size_t)m * ldN + (size_t)m * ldm + (size_t)ldm);
}

// B_t (m x N) and St (m x m) kept at every segment start of a checkpointed store.
size_t bck_bytes(int64_t N, int64_t m, int64_t T, int stride) {
    return stride > 1 ? 8 * (size_t)(T / stride + 1) * (size_t)m * (round_up(N, 16) + round_up(m, 16)) : 0;
}

// Outer block width of the gain's factorisation for order N, and the leading dimension of the
// stacked diagonal-block inverses (the widest block, rounded up).
int gain_block(int64_t N) { return (int)std::min<int64_t>(kGainBlock, N); }
int64_t gain_ld(int64_t N) { return round_up(gain_block_width((int)N, gain_block(N)), 16); }
// Elements of one Dg buffer: N x gld inverses, then a (widest block) x ldN solve panel.
size_t gain_scratch_elems(int64_t N) { return (size_t)gain_ld(N) * (size_t)(N + round_up(N, 16)); }

// np: gain batches in flight (np scratch sets W, Li, Dg and np + 1 gain sets).
size_t workspace_bytes(int64_t N, int64_t m, bool mix, bool s32, int stride, int gb, int np = 1) {
    const int64_t ldN = round_up(N, 16), ldm = round_up(m, 16);
    const size_t NN = (size_t)N * ldN;
    size_t b = 0;
    b += 8 * (size_t)np * gb * gain_scratch_elems(N);
    b += 8 * (2 * NN + 2 * (size_t)m * ldN + (size_t)m * ldm + 2 * (size_t)N);   // Q, P0, X, XQ, R, x0
    b += 8 * (3 * (size_t)m * ldN + 7 * (size_t)m * ldm + 3 * (size_t)N + 64);   // B, two C, St, Sw, XQX, H, two Li, G
    b += 8 * (size_t)std::max<int64_t>(4 * m * N, 32 * m * m);                 // split-K partials
    const size_t sets = (size_t)np + 1;
    b += 8 * ((2 * (size_t)np + sets) * (size_t)gb + 2) * NN;                // W, Li per stream, A per set; Ps x2
    if (!mix) b += 8 * 2 * NN;                                                   // D, M
    if (s32) b += 8 * sets * (size_t)gb * NN;                                    // upcast P_{t|t}
    if (mix) b += 4 * (sets * (size_t)gb * NN + 2 * NN + 2 * (size_t)m * ldN);  // A32, D32, M32, two C32
    if (s32 || stride > 1) b += 8 * 2 * NN;
    if (mix) b += 4 * NN;
    if (stride > 1) b += (size_t)stride * NN * (s32 ? 4 : 8);
    b += tail_bytes(N, mix);
    return b;
}

kf_status status_check(kf_plan* p, const char* phase) {
    const unsigned long long k = p->hstatus->key;
    if (k != kStatusClear) {
        const int w = status_which(k);
        const char* which = w == W_S ? "S_t = X P_{t|t-1} X^T + R"
                          : w == W_PPRED ? (p->hasF ? "P_{t+1|t} = F P_{t|t} F^T + Q" : "P_{t+1|t} = P_{t|t} + Q")
                                         : "X C X^T + R";
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s is not positive definite at step t=%d (pivot row %d)", phase, which,
                 status_step(k), status_row(k));
        p->err = buf;
        return KF_ENOTPD;
    }
    return KF_OK;
}

// Filter step t (eqn8-eqn10 and the covariance update after eqn10) in four parts. With F = I,
// P_{t+1|t} = P_{t|t-1} - C_t^T C_t + Q, and with St = X P_{t|t-1} X^T, S_t = St + R = L_t L_t^T,
// C_t = L_t^{-1} X P_{t|t-1} and G_t = X C_t^T = St L_t^{-T}:
//     St_{t+1} = St - G_t G_t^T + X Q X^T = R - R S_t^{-1} R + X Q X^T
//              = X Q X^T + R - (L_t^{-1} R)^T (L_t^{-1} R),
//     B_{t+1}  = B_t + X Q - G_t C_t,
// (using St - St S_t^{-1} St = R - R S_t^{-1} R). So the chain from step to step is m x m work
// only -- factor St + R, form H = L_t^{-1} R, St <- X Q X^T + R - H^T H -- and the Riccati form
// does not accumulate rounding from step to step the way St - G G^T + X Q X^T would. The N-sized
// work of step t -- C_t = L_t^{-1} B_t, the mean of eqn10, G_t = X C_t^T and B_{t+1}, and the
// downdate P_t = P_pred - C_t^T C_t -- hangs off the chain and runs on side streams. B_t (whose
// recursion does accumulate rounding) and St are formed in full every kBRefresh steps, and at
// every step with a transition F, where the recursions do not hold; a checkpointed store keeps B_t
// and St at every segment start, so that recomputed segments reproduce the forward pass bit for bit.
constexpr int64_t kBRefresh = 16;

bool refresh_step(const kf_plan* p, int64_t t) { return p->hasF || t % kBRefresh == 0; }

// B_t = X P_{t|t-1} and St = B_t X^T in full from Pprev64 = P_{t-1|t-1} (or P0), on stream s.
kf_status filter_refresh(kf_plan* p, const double* Pprev64, hipStream_t s) {
    const int N = (int)p->N, m = (int)p->m;
    const double* Ppred = nullptr;
    if (p->hasF) {   // P_pred = F P_prev F^T + Q, formed as F (P_prev F^T) + Q
        HIPCK(dense_sparse_t(p->F, Pprev64, p->ldN, p->Fg, p->ldN, s));
        HIPCK(spmm_rows(p->F, p->Fg, p->ldN, 1.0, p->Q, p->ldN, 1.0, nullptr, 0, 0.0, p->Fp, false, p->ldN, s));
        Ppred = p->Fp;
    }
    {   // B = X P_pred; with F = I, X P_prev + X Q (float64 in both precisions: the gain and the mean
        // depend on it through S^{-1}, where rounding is amplified by cond(S))
        GemmProblem g;
        g.M = m; g.N = N; g.K = N;
        g.ksplit = 4;
        g.partial = p->partial;
        if (!Ppred) { g.Cin = p->XQ; g.ldcin = p->ldN; g.beta = 1.0; }
        g.C = p->Bm; g.ldc = p->ldN;
        g.A = p->X; g.lda = p->ldN;
        g.B = Ppred ? Ppred : Pprev64; g.ldb = p->ldN; g.flags = G_TB;   // P symmetric: read row-contiguous
        HIPCK(gemm1(Dt::F64, g, s));
    }
    {   // St = B X^T
        GemmProblem g;
        g.M = m; g.N = m; g.K = N;
        g.A = p->Bm; g.lda = p->ldN;
        g.B = p->X; g.ldb = p->ldN; g.flags = G_TB;
        g.C = p->St; g.ldc = p->ldm;
        g.ksplit = std::max(1, std::min(32, N / 128));
        g.partial = p->partial;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    return KF_OK;
}

// The m x m chain of step t on stream s: factor S_t = St + R (eqn8), L_t^{-1} into slot t & 1;
// then, unless step t + 1 forms St in full, St <- X Q X^T + R - H^T H with H = L_t^{-1} R.
kf_status filter_mchain(kf_plan* p, int64_t t, int64_t T, hipStream_t s) {
    const int m = (int)p->m;
    HIPCK(axpby3(m, m, p->Sw, false, p->ldm, p->St, false, p->ldm, p->R, false, p->ldm, 1.0, nullptr, false, 0, 0.0,
                 s));
    HIPCK(chol_inv(p->Sw, p->ldm, p->Li2[t & 1], p->ldm, m, p->dstatus, W_S, (int)t + 1, s));
    if (t + 1 >= T || refresh_step(p, t + 1)) return KF_OK;
    {   // H = L_t^{-1} R
        GemmProblem g;
        g.M = m; g.N = m; g.K = m;
        g.A = p->Li2[t & 1]; g.lda = p->ldm; g.flags = G_ALOWER;
        g.B = p->R; g.ldb = p->ldm;
        g.C = p->Hm; g.ldc = p->ldm;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    {   // St <- X Q X^T + R - H^T H   (lower tiles + mirror)
        GemmProblem g;
        g.M = m; g.N = m; g.K = m;
        g.A = p->Hm; g.lda = p->ldm; g.flags = G_TA | G_LOWER | G_MIRROR;
        g.B = p->Hm; g.ldb = p->ldm;
        g.alpha = -1.0;
        g.Cin = p->XQX; g.ldcin = p->ldm; g.beta = 1.0;
        g.Cin2 = p->R; g.ldcin2 = p->ldm; g.gamma = 1.0;
        g.C = p->St; g.ldc = p->ldm;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    return KF_OK;
}

// C_t = L_t^{-1} B_t into slot t & 1 (and its float32 copy for the mixed downdate), then, with `y`,
// the mean of eqn10: x_t = x_pred + C_t^T (L_t^{-1} (y_t - X x_pred)).
kf_status filter_gain_mean(kf_plan* p, int64_t t, const double* y, double* x_out_row, hipStream_t s) {
    const int N = (int)p->N, m = (int)p->m;
    {
        GemmProblem g;
        g.M = m; g.N = N; g.K = m;
        g.A = p->Li2[t & 1]; g.lda = p->ldm; g.flags = G_ALOWER;
        g.B = p->Bm; g.ldb = p->ldN;
        g.C = p->Cm2[t & 1]; g.ldc = p->ldN;
        if (mixed(p)) { g.C32 = p->Cm32x[t & 1]; g.ldc32 = p->ldN; }
        HIPCK(gemm1(Dt::F64, g, s));
    }
    if (y) {
        const double* xpred = p->xw;                                     // eqn6
        if (p->hasF) {
            HIPCK(spmv_rows(p->F, p->xw, p->ldN, 1, p->xp, p->ldN, s));
            xpred = p->xp;
        }
        HIPCK(resid(p->X, p->ldN, xpred, y, p->e, m, N, s));
        HIPCK(trmv_lower(p->Li2[t & 1], p->ldm, p->e, p->w, m, s));
        HIPCK(gemv_t_add(p->Cm2[t & 1], p->ldN, p->w, xpred, p->xw, x_out_row, m, N, s));
    }
    return KF_OK;
}

// G_t = X C_t^T, then B_{t+1} = B_t + X Q - G_t C_t in place (a recursive step t + 1 only).
kf_status filter_b_update(kf_plan* p, int64_t t, hipStream_t s) {
    const int N = (int)p->N, m = (int)p->m;
    {
        GemmProblem g;
        g.M = m; g.N = m; g.K = N;
        g.A = p->X; g.lda = p->ldN;
        g.B = p->Cm2[t & 1]; g.ldb = p->ldN; g.flags = G_TB;
        g.C = p->Gm; g.ldc = p->ldm;
        g.ksplit = std::max(1, std::min(32, N / 128));
        g.partial = p->partial;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    GemmProblem g;
    g.M = m; g.N = N; g.K = m;
    g.A = p->Gm; g.lda = p->ldm;
    g.B = p->Cm2[t & 1]; g.ldb = p->ldN;
    g.alpha = -1.0;
    g.Cin = p->Bm; g.ldcin = p->ldN; g.beta = 1.0;
    g.Cin2 = p->XQ; g.ldcin2 = p->ldN; g.gamma = 1.0;
    g.C = p->Bm; g.ldc = p->ldN;
    HIPCK(gemm1(Dt::F64, g, s));
    return KF_OK;
}

// B_t and St at a segment start of a checkpointed store: keep them (forward pass) or restore them.
kf_status filter_keep_state(kf_plan* p, int64_t t, bool restore, hipStream_t sb, hipStream_t ss) {
    const size_t mN = (size_t)p->m * p->ldN, mm = (size_t)p->m * p->ldm;
    const int64_t k = t / p->stride;
    double* bk = p->Bck + (size_t)k * mN;
    double* sk = p->Sck + (size_t)k * mm;
    HIPCK(hipMemcpyAsync(restore ? p->Bm : bk, restore ? bk : p->Bm, mN * 8, hipMemcpyDeviceToDevice, sb));
    HIPCK(hipMemcpyAsync(restore ? p->St : sk, restore ? sk : p->St, mm * 8, hipMemcpyDeviceToDevice, ss));
    return KF_OK;
}

// Lower tiles of the downdate run in launches of at most this many workgroups when it overlaps
// other work, leaving compute units free for the filter's small kernels.
constexpr int kDowndateChunk = 288;

// The covariance update after eqn10 for step t on stream `s`: P_t = P_pred - C_t^T C_t with
// P_pred = P_prev + Q (F = I) or the F P_prev F^T + Q that filter_refresh formed; lower tiles
// with a mirrored store (exact symmetry), the diagonal to diag_out, float64 to Pout64 and
// (optional) float32 to Pout32. `chunked`: in launches of at most kDowndateChunk workgroups (the
// tiles, and so the result, are the same either way).
kf_status filter_downdate(kf_plan* p, int64_t t, const double* Pprev64, double* Pout64, float* Pout32,
                          double* diag_out, hipStream_t s, bool chunked) {
    const int N = (int)p->N, m = (int)p->m;
    const double* Ppred = p->hasF ? p->Fp : nullptr;
    GemmProblem g;
    g.M = N; g.N = N; g.K = m;
    g.flags = G_TA | G_LOWER | G_MIRROR;
    g.alpha = -1.0;
    g.Cin = Ppred ? Ppred : Pprev64; g.ldcin = p->ldN; g.beta = 1.0;
    if (!Ppred) { g.Cin2 = p->Q; g.ldcin2 = p->ldN; g.gamma = 1.0; }
    g.C = Pout64; g.ldc = p->ldN;
    g.C32 = Pout32; g.ldc32 = p->ldN;
    g.diag = diag_out;
    const Dt dt = mixed(p) ? Dt::F32 : Dt::F64;
    if (mixed(p)) { g.A = p->Cm32x[t & 1]; g.B = p->Cm32x[t & 1]; }
    else { g.A = p->Cm2[t & 1]; g.B = p->Cm2[t & 1]; }
    g.lda = g.ldb = p->ldN;
    const int tiles = gemm_tiles(g);
    const int chunk = chunked ? kDowndateChunk : tiles;
    for (int off = 0; off < tiles; off += chunk) {
        GemmProblem h = g;
        h.tile_off = off;
        h.tile_cnt = std::min(chunk, tiles - off);
        HIPCK(gemm1(dt, h, s));
    }
    return KF_OK;
}

// One covariance step of the filter, everything on the plan's stream (recomputation of a
// checkpointed segment; no mean). `restore`: step t starts a recomputed segment whose B_t and
// St were kept by the forward pass.
kf_status filter_cov_step(kf_plan* p, int64_t t, int64_t T, const double* Pprev64, double* Pout64, float* Pout32,
                          bool restore) {
    hipStream_t s = p->stream;
    if (refresh_step(p, t)) TRY(filter_refresh(p, Pprev64, s));
    else if (restore) TRY(filter_keep_state(p, t, true, s, s));
    TRY(filter_mchain(p, t, T, s));
    TRY(filter_gain_mean(p, t, nullptr, nullptr, s));
    if (t + 1 < T && !refresh_step(p, t + 1)) TRY(filter_b_update(p, t, s));
    return filter_downdate(p, t, Pprev64, Pout64, Pout32, nullptr, s, false);
}

// Buffers for the means of B data sets (E, W: B x m residuals; Xb0: B copies of x0; Vb: B x N).
kf_status ensure_batch(kf_plan* p, int64_t B) {
    if (B <= p->bcap) return KF_OK;
    if (p->arena) {
        p->err = "several data sets per call are not available on a serving plan";
        return KF_EINVAL;
    }
    for (double* b : {p->Eb, p->Wb, p->Xb0, p->Vb, p->Ub})
        if (b) (void)hipFree(b);
    p->Eb = p->Wb = p->Xb0 = p->Vb = p->Ub = nullptr;
    p->bcap = 0;
    const size_t bm = (size_t)B * p->ldm * 8, bn = (size_t)B * p->ldN * 8;
    if (hipMalloc(&p->Eb, bm) != hipSuccess || hipMalloc(&p->Wb, bm) != hipSuccess ||
        hipMalloc(&p->Xb0, bn) != hipSuccess || hipMalloc(&p->Vb, bn) != hipSuccess ||
        hipMalloc(&p->Ub, bn) != hipSuccess) {
        (void)hipGetLastError();
        p->err = "device allocation for " + std::to_string(B) + " data sets failed";
        return KF_ENOMEM;
    }
    p->bcap = B;
    return KF_OK;
}

// Split-K factor for a B-row product with K = N whose partial sums share the plan's buffer.
int batch_ksplit(const kf_plan* p, int64_t rows, int64_t cols, int want) {
    int k = want;
    while (k > 1 && (size_t)k * rows * cols > p->partial_elems) k /= 2;
    return k;
}

// Mean update of eqn10 for B data sets at once, after filter_chain_step(t) has left Li = L^{-1}
// (of S_t) and C_t = Li X P_{t|t-1} in the plan: with E = Y_t - X_prev X^T (B x m),
// X_t = X_prev + (E Li^T) C. Row b of X_prev / X_t is data set b's mean (leading dimension ldx).
kf_status filter_mean_batch(kf_plan* p, int64_t t, int64_t B, const double* Xprev, int64_t ldprev, const double* Yt,
                            int64_t ldy, double* Xt, int64_t ldx, hipStream_t s) {
    const int N = (int)p->N, m = (int)p->m;
    if (p->hasF) {                           // predicted means F x (eqn6)
        HIPCK(spmv_rows(p->F, Xprev, ldprev, (int)B, p->Ub, p->ldN, s));
        Xprev = p->Ub;
        ldprev = p->ldN;
    }
    {
        GemmProblem g;                       // E = Y_t - X_prev X^T
        g.M = (int)B; g.N = m; g.K = N;
        g.A = Xprev; g.lda = ldprev;
        g.B = p->X; g.ldb = p->ldN; g.flags = G_TB;
        g.alpha = -1.0;
        g.Cin = Yt; g.ldcin = ldy; g.beta = 1.0;
        g.C = p->Eb; g.ldc = p->ldm;
        g.ksplit = batch_ksplit(p, B, m, std::max(1, std::min(16, N / 256)));
        g.partial = p->partial;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    {
        GemmProblem g;                       // W = E Li^T  (Li lower: W_b = Li e_b)
        g.M = (int)B; g.N = m; g.K = m;
        g.A = p->Eb; g.lda = p->ldm;
        g.B = p->Li2[t & 1]; g.ldb = p->ldm; g.flags = G_TB;
        g.C = p->Wb; g.ldc = p->ldm;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    {
        GemmProblem g;                       // X_t = X_prev + W C
        g.M = (int)B; g.N = N; g.K = m;
        g.A = p->Wb; g.lda = p->ldm;
        g.B = p->Cm2[t & 1]; g.ldb = p->ldN;
        g.Cin = Xprev; g.ldcin = ldprev; g.beta = 1.0;
        g.C = Xt; g.ldc = ldx;
        HIPCK(gemm1(Dt::F64, g, s));
    }
    return KF_OK;
}

// Smoothed means of eqn12 for B data sets: X_{t|T} = X_{t|t} + (X_{t+1|T} - X_{t|t}) A_t^T,
// rows of the B x T x N arrays xf / xs (leading dimension T N).
kf_status smooth_mean_batch(kf_plan* p, int64_t B, const double* A, int64_t t, const double* xf, double* xs) {
    hipStream_t s = p->stream;
    const int N = (int)p->N;
    const int64_t ldx = p->T_done * N;
    const double* xpred = xf + t * N;        // x_{t+1|t} rows: F x_{t|t}, or x_{t|t} with F = I
    int64_t ldp = ldx;
    if (p->hasF) {
        HIPCK(spmv_rows(p->F, xf + t * N, ldx, (int)B, p->Ub, p->ldN, s));
        xpred = p->Ub;
        ldp = p->ldN;
    }
    HIPCK(axpby3((int)B, N, p->Vb, false, p->ldN, xs + (t + 1) * N, false, ldx, xpred, false, ldp, -1.0, nullptr,
                 false, 0, 0.0, s));
    GemmProblem g;
    g.M = (int)B; g.N = N; g.K = N;
    g.A = p->Vb; g.lda = p->ldN;
    g.B = A; g.ldb = p->ldN; g.flags = G_TB;
    g.Cin = xf + t * N; g.ldcin = ldx; g.beta = 1.0;
    g.C = xs + t * N; g.ldc = ldx;
    g.ksplit = batch_ksplit(p, B, N, 4);
    g.partial = p->partial;
    HIPCK(gemm1(Dt::F64, g, s));
    return KF_OK;
}

kf_status sync_and_check(kf_plan* p, const char* phase) {
    HIPCK(hipMemcpyAsync(p->hstatus, p->dstatus, sizeof(DevStatus), hipMemcpyDeviceToHost, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
    return status_check(p, phase);
}

// Launch a group of the smoother's N x N x N products (named instantiation), timed when profiling.
kf_status big_group(kf_plan* p, Dt dt, GemmProblem* g, int count, double flops, hipStream_t st,
                    const TailSplit* ts = nullptr) {
    const int name = p->serial && dt == Dt::F64 ? G_NXN_SERIAL : mixed(p) ? G_NXN_MIXED : G_NXN;
    for (int u = 0; u < count; ++u) g[u].flags |= name;
    if (p->prof) {
        while (p->ev.size() < p->ev_used + 2) {
            hipEvent_t e;
            HIPCK(hipEventCreate(&e));
            p->ev.push_back(e);
        }
        HIPCK(hipEventRecord(p->ev[p->ev_used], st));
    }
    // The closing event is recorded right after the product kernel itself, before any split
    // reduction, so that each event pair spans exactly one dispatch of the named kernel.
    hipEvent_t done = p->prof ? p->ev[p->ev_used + 1] : nullptr;
    void* ws = (dt == Dt::F64 && mixed(p)) ? p->tail_ws64 : p->tail_ws;
    if (ts && ts->k > 1 && ws && count == 1) HIPCK(gemm_launch_tail(dt, g[0], *ts, ws, st, done));
    else HIPCK(gemm_launch(dt, g, count, st, done));
    if (p->prof) {
        p->ev_flops.push_back(flops);
        p->ev_used += 2;
    }
    return KF_OK;
}

kf_status big_gemm(kf_plan* p, Dt dt, GemmProblem g, double flops, hipStream_t st, const TailSplit* ts = nullptr) {
    return big_group(p, dt, &g, 1, flops, st, ts);
}

// After the stream has been synchronised: fold the recorded event pairs into the totals.
kf_status collect_profile(kf_plan* p) {
    for (size_t k = 0; k + 1 < p->ev_used; k += 2) {
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, p->ev[k], p->ev[k + 1]));
        p->prof_ms += ms;
        p->prof_flops += p->ev_flops[k / 2];
        p->prof_launches += 1;
    }
    p->ev_used = 0;
    p->ev_flops.clear();
    return KF_OK;
}

}  // namespace

extern "C" {

void kf_default_options(kf_options* opt) {
    if (!opt) return;
    opt->precision = KF_FP64;
    opt->store_fp32 = 0;
    opt->hbm_budget_bytes = 0;
    opt->checkpoint_stride = 0;
    opt->keep_gain_factors = 0;
}

size_t kf_plan_bytes(int64_t N, int64_t m, int64_t T, const kf_options* opt) {
    kf_options o;
    kf_default_options(&o);
    if (opt) o = *opt;
    if (N <= 0 || m <= 0 || T <= 0) return 0;
    const int64_t ldN = round_up(N, 16);
    const int stride = o.checkpoint_stride > 0 ? o.checkpoint_stride : 1;
    return workspace_bytes(N, m, o.precision == KF_MIXED, o.store_fp32, stride, kMaxBatch) +
           store_bytes(N, ldN, T, o.store_fp32, stride) + bck_bytes(N, m, T, stride) +
           (o.keep_gain_factors ? factor_bytes(N, m, T) : 0);
}

size_t kf_smooth_assoc_bytes(int64_t N, int64_t T) {
    if (N <= 0 || T <= 0) return 0;
    return assoc_bytes(N, round_up(N, 16), T);
}

}  // extern "C"

namespace kfmeg {

// Compute units given to the filter's m x m chain (the first ones of the device).
constexpr int kChainCUs = 32;

// Streams for the filter: the chain on the first kChainCUs compute units, the downdates on the
// rest. Left null (the filter then uses the plan's and the side streams) if the device has too
// few compute units or a CU-masked stream cannot be created.
void split_filter_streams(kf_plan* p) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 4 * kChainCUs) {
        (void)hipGetLastError();
        return;
    }
    std::vector<uint32_t> mc((cus + 31) / 32, 0u), md(mc.size(), 0u);
    for (int c = 0; c < cus; ++c) (c < kChainCUs ? mc : md)[c / 32] |= 1u << (c % 32);
    const uint32_t n = (uint32_t)mc.size();
    if (hipExtStreamCreateWithCUMask(&p->sc, n, mc.data()) != hipSuccess ||
        hipExtStreamCreateWithCUMask(&p->sdm, n, md.data()) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t* q : {&p->sc, &p->sdm})
            if (*q) (void)hipStreamDestroy(*q);
        p->sc = p->sdm = nullptr;
    }
}

// kf_create with an optional arena for every device buffer of the plan (serving).
kf_status create_plan(kf_plan** out, int64_t N, int64_t m, int64_t T_max, const double* X, const double* Q,
                      const double* R, const double* x0, const double* P0, const kf_options* opt, void* stream,
                      DeviceArena* arena) {
    if (!out) return KF_EINVAL;
    *out = nullptr;
    if (N <= 0 || m <= 0 || T_max <= 0 || N > (1 << 20) || m > (1 << 16)) {
        g_err = "kf_create: sizes must be positive (N <= 2^20, m <= 2^16)";
        return KF_EINVAL;
    }
    if (!X || !Q || !R || !x0 || !P0) {
        g_err = "kf_create: null model pointer";
        return KF_EINVAL;
    }
    kf_plan* p = new kf_plan();
    p->arena = arena;
    p->N = N; p->m = m; p->Tmax = T_max;
    kf_default_options(&p->opt);
    if (opt) p->opt = *opt;
    if (p->opt.precision != KF_FP64 && p->opt.precision != KF_MIXED) {
        g_err = "kf_create: unknown precision";
        delete p;
        return KF_EINVAL;
    }
    p->stream = static_cast<hipStream_t>(stream);
    p->ldN = round_up(N, 16);
    p->ldm = round_up(m, 16);
    p->store32 = p->opt.store_fp32 != 0;

    // Store layout: all T_max slots, or every k-th slot when over budget.
    size_t budget = p->opt.hbm_budget_bytes;
    if (budget == 0 && arena) budget = arena->largest_free();
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = fr > ((size_t)1 << 30) ? fr - ((size_t)1 << 30) : 0;
    }
    int stride = p->opt.checkpoint_stride > 0 ? p->opt.checkpoint_stride : 1;
    const bool mix = mixed(p);
    p->keep = p->opt.keep_gain_factors != 0;
    const size_t fac = p->keep ? factor_bytes(N, m, T_max) : 0;
    int np = arena ? 1 : kMaxProd;          // serving plans keep one gain batch in flight
    auto need = [&](int st, int gb) {
        return workspace_bytes(N, m, mix, p->store32, st, gb, np) + store_bytes(N, p->ldN, T_max, p->store32, st) +
               bck_bytes(N, m, T_max, st) +
               fac;
    };
    // Prefer storing every P_{t|t}; give up the second gain batch in flight, then gain
    // batching, before checkpointing. A short horizon needs no wider batch than its T - 1
    // smoother steps, and a single batch (a 2-step first batch, then gb steps) no second stream.
    int gb = kMaxBatch;
    while (gb > 1 && gb / 2 >= T_max - 1) gb /= 2;
    if (T_max - 1 <= 2) np = 1;
    while (np > 1 && need(stride, gb) > budget) --np;
    while (gb > 1 && need(stride, gb) > budget) gb /= 2;
    if (p->opt.checkpoint_stride <= 0) {
        while (stride < T_max && need(stride, gb) > budget)
            stride = stride == 1 ? std::max<int>(2, (int)std::ceil(std::sqrt((double)T_max))) : stride + 1;
    }
    if (need(stride, gb) > budget) {
        g_err = "kf_create: the covariance store does not fit the HBM budget even with checkpointing";
        delete p;
        return KF_ENOMEM;
    }
    p->gbatch = gb;
    p->nprod = np;
    p->stride = stride;
    p->nslots = slots_needed(T_max, stride);

    kf_status st = KF_OK;
    auto fail = [&](kf_status s) {
        g_err = p->err;
        kf_destroy(p);
        return s;
    };
    const size_t NN = slot_elems(p);
    const size_t mN = (size_t)m * p->ldN, mm = (size_t)m * p->ldm;
#define ALLOC(ptr, n)                        \
    if ((st = alloc(p, &(ptr), (n))) != KF_OK) return fail(st);
    ALLOC(p->X, mN); ALLOC(p->XQ, mN); ALLOC(p->Q, NN); ALLOC(p->R, mm); ALLOC(p->x0, (size_t)N); ALLOC(p->P0, NN);
    ALLOC(p->Bm, mN); ALLOC(p->Cm2[0], mN); ALLOC(p->Cm2[1], mN);
    ALLOC(p->St, mm); ALLOC(p->Sw, mm); ALLOC(p->XQX, mm); ALLOC(p->Hm, mm);
    ALLOC(p->Li2[0], mm); ALLOC(p->Li2[1], mm); ALLOC(p->Gm, mm);
    if (stride > 1) {
        ALLOC(p->Bck, (size_t)(T_max / stride + 1) * mN);
        ALLOC(p->Sck, (size_t)(T_max / stride + 1) * mm);
    }
    ALLOC(p->e, (size_t)m); ALLOC(p->w, (size_t)m); ALLOC(p->xw, (size_t)N);
    p->partial_elems = (size_t)std::max<int64_t>(4 * m * N, 32 * m * m);
    ALLOC(p->partial, p->partial_elems);
    ALLOC(p->dstatus, 1);
    p->gnb = gain_block(N);
    p->gld = gain_ld(N);
    for (int b = 0; b < p->gbatch; ++b) {
        for (int q = 0; q < p->nprod; ++q) {
            ALLOC(p->W[q][b], NN); ALLOC(p->Li[q][b], NN); ALLOC(p->Dg[q][b], gain_scratch_elems(N));
        }
        for (int set = 0; set <= p->nprod; ++set) {
            ALLOC(p->Ab[set][b], NN);
            if (p->store32) ALLOC(p->Pt64[set][b], NN);
            if (mix) ALLOC(p->A32[set][b], NN);
        }
    }
    ALLOC(p->Ps[0], NN); ALLOC(p->Ps[1], NN);
    if (p->keep) {
        ALLOC(p->fac_C, (size_t)T_max * mN);
        ALLOC(p->fac_L, (size_t)T_max * mm);
        ALLOC(p->fac_w, (size_t)T_max * p->ldm);
        p->wcap = 1;
    }
    tail_splits(N, p->ts_m, p->ts_low);
    if (const size_t tb = tail_bytes(N, mix)) {
        if ((st = alloc_bytes(p, &p->tail_ws, tb)) != KF_OK) return fail(st);
    }
    if (!mix) { ALLOC(p->Dm, NN); ALLOC(p->Mm, NN); }
    if (mix) {
        ALLOC(p->Cm32x[0], mN); ALLOC(p->Cm32x[1], mN);
        ALLOC(p->D32, NN); ALLOC(p->M32, NN);
    }
    if (p->store32 || stride > 1) { ALLOC(p->Pw[0], NN); ALLOC(p->Pw[1], NN); }
    {
        void* sp = nullptr;
        const size_t bytes = (size_t)p->nslots * NN * (slot64(p) ? 8 : 4);
        if ((st = alloc_bytes(p, &sp, bytes)) != KF_OK) {
            p->err = "device allocation of the covariance store (" + std::to_string(bytes) + " bytes) failed";
            return fail(st);
        }
        p->store = sp;
        if (stride > 1) {
            if ((st = alloc_bytes(p, &sp, (size_t)stride * NN * (p->store32 ? 4 : 8))) != KF_OK) {
                p->err = "device allocation of the recompute segment failed";
                return fail(st);
            }
            p->seg = sp;
        }
    }
#undef ALLOC
    if (hipHostMalloc(reinterpret_cast<void**>(&p->hstatus), sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        p->err = "pinned host allocation failed";
        return fail(KF_ENOMEM);
    }
    {
        bool ok = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming) == hipSuccess;
        for (int q = 0; ok && q < p->nprod; ++q) ok = hipStreamCreateWithFlags(&p->s2[q], hipStreamNonBlocking) == hipSuccess;
        if (ok && !arena) split_filter_streams(p);
        for (int k = 0; ok && k <= p->nprod; ++k)
            ok = hipEventCreateWithFlags(&p->ev_gain[k], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&p->ev_chain[k], hipEventDisableTiming) == hipSuccess;
        for (int k = 0; ok && k < 2; ++k)
            for (hipEvent_t* e : {&p->ev_fl[k], &p->ev_fg[k], &p->ev_fr[k], &p->ev_fa[k], &p->ev_cc[k], &p->ev_dd[k]})
                ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            p->err = "kf_create: creating the side streams or their events failed";
            return fail(KF_EHIP);
        }
    }
    hipStream_t s = p->stream;
    auto cp = [&](void* dst, bool d32, int64_t ldd, const double* src, int64_t rows, int64_t cols) {
        return copy2d((int)rows, (int)cols, dst, d32, ldd, src, false, cols, s);
    };
    if (cp(p->X, false, p->ldN, X, m, N) != hipSuccess || cp(p->Q, false, p->ldN, Q, N, N) != hipSuccess ||
        cp(p->R, false, p->ldm, R, m, m) != hipSuccess || cp(p->x0, false, N, x0, 1, N) != hipSuccess ||
        cp(p->P0, false, p->ldN, P0, N, N) != hipSuccess) {
        p->err = "kf_create: copying the model failed";
        return fail(KF_EHIP);
    }
    {
        GemmProblem g;                           // X Q, used by every filter step
        g.M = (int)m; g.N = (int)N; g.K = (int)N;
        g.A = p->X; g.lda = p->ldN; g.B = p->Q; g.ldb = p->ldN;
        g.C = p->XQ; g.ldc = p->ldN;
        GemmProblem h;                           // X Q X^T, used by the recursion of St
        h.M = (int)m; h.N = (int)m; h.K = (int)N;
        h.A = p->XQ; h.lda = p->ldN; h.B = p->X; h.ldb = p->ldN; h.flags = G_TB;
        h.C = p->XQX; h.ldc = p->ldm;
        if (gemm1(Dt::F64, g, s) != hipSuccess || gemm1(Dt::F64, h, s) != hipSuccess) {
            p->err = "kf_create: forming X Q and X Q X^T failed";
            return fail(KF_EHIP);
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        p->err = "kf_create: stream synchronisation failed";
        return fail(KF_EHIP);
    }
    *out = p;
    return KF_OK;
}

// Device bytes of a plan with gain-batch width gb (kf_plan_bytes uses the widest).
size_t plan_bytes_ex(int64_t N, int64_t m, int64_t T, const kf_options* opt, int gb) {
    kf_options o;
    kf_default_options(&o);
    if (opt) o = *opt;
    if (N <= 0 || m <= 0 || T <= 0) return 0;
    const int64_t ldN = round_up(N, 16);
    const int stride = o.checkpoint_stride > 0 ? o.checkpoint_stride : 1;
    return workspace_bytes(N, m, o.precision == KF_MIXED, o.store_fp32, stride, gb) +
           store_bytes(N, ldN, T, o.store_fp32, stride) + bck_bytes(N, m, T, stride) +
           (o.keep_gain_factors ? factor_bytes(N, m, T) : 0);
}

}  // namespace kfmeg

extern "C" {

kf_status kf_create(kf_plan** out, int64_t N, int64_t m, int64_t T_max, const double* X, const double* Q,
                    const double* R, const double* x0, const double* P0, const kf_options* opt, void* stream) {
    return create_plan(out, N, m, T_max, X, Q, R, x0, P0, opt, stream, nullptr);
}

static kf_status filter_impl(kf_plan* p, int64_t B, int64_t T, const double* Y, double* x_filt, double* Pdiag) {
    hipStream_t s = p->stream;
    const int64_t N = p->N, m = p->m;
    HIPCK(status_clear(p->dstatus, s));
    HIPCK(nonfinite_scan(Y, B * T * m, &p->dstatus->flag, s));
    HIPCK(hipMemcpyAsync(p->hstatus, p->dstatus, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (p->hstatus->flag) {
        p->err = "kf_filter: Y holds a non-finite value";
        return KF_EINVAL;
    }
    if (p->keep && B > p->wcap) {
        if (p->arena) {
            p->err = "several data sets per call are not available on a serving plan";
            return KF_EINVAL;
        }
        double* w = nullptr;
        if (hipMalloc(&w, (size_t)p->Tmax * B * p->ldm * 8) != hipSuccess) {
            (void)hipGetLastError();
            p->err = "device allocation of the gain factors for " + std::to_string(B) + " data sets failed";
            return KF_ENOMEM;
        }
        p->bfac_w.push_back(w);    // freed with the plan
        p->fac_w = w;
        p->wcap = B;
    }
    if (B == 1) {
        HIPCK(hipMemcpyAsync(p->xw, p->x0, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        TRY(ensure_batch(p, B));
        HIPCK(copy2d((int)B, (int)N, p->Xb0, false, p->ldN, p->x0, false, 0, s));   // x0 in every row
    }
    const bool direct = !p->store32 && p->stride == 1;   // store slot t is the working P
    // Streams: the m x m chain on s (the plan's stream, or the chain's CU-masked stream); the
    // N-sized work of each step (C_t, the mean, B's recursion and refreshes) on sa; the downdates on
    // sd. With the CU split both sa and sd are the other CU-masked stream; otherwise sa is the first
    // side stream and sd the second (= sa with one side stream). Slot t & 1 of L^{-1} and C is
    // reused at step t + 2, after the streams that read it at step t.
    hipStream_t sa = p->s2[0], sd = p->nprod > 1 ? p->s2[1] : p->s2[0];
    HIPCK(hipEventRecord(p->ev_start, s));
    const hipStream_t s0 = s;
    if (p->sc) {   // the chain on its CU-partitioned stream, the N-sized work and downdates on the other
        s = p->sc;
        sd = p->sdm;
        sa = p->sdm;
        HIPCK(hipStreamWaitEvent(s, p->ev_start, 0));
    }
    HIPCK(hipStreamWaitEvent(sa, p->ev_start, 0));
    if (sd != sa) HIPCK(hipStreamWaitEvent(sd, p->ev_start, 0));
    const double* prev64 = p->P0;
    for (int64_t t = 0; t < T; ++t) {
        Range r("kf_filter step t=%lld", (long long)t + 1);
        const int k = (int)(t & 1);
        double* out64 = direct ? static_cast<double*>(slot_ptr(p, t)) : p->Pw[k];
        float* out32 = nullptr;
        if (!slot64(p) && kept(p, t, T)) out32 = static_cast<float*>(slot_ptr(p, slot_of(p, t, T)));
        double* diag = Pdiag ? Pdiag + t * N : nullptr;
        const bool full = refresh_step(p, t);
        const bool seg = p->stride > 1 && t % p->stride == 0;
        // N side: refresh B_t and St from P_{t-1|t-1} (after downdate t - 1)
        if (full) {
            if (t >= 1) HIPCK(hipStreamWaitEvent(sa, p->ev_dd[k ^ 1], 0));
            TRY(filter_refresh(p, prev64, sa));
        }
        if (seg) {                                        // segment start: keep B_t and St
            if (!full) HIPCK(hipStreamWaitEvent(sa, p->ev_fg[k ^ 1], 0));   // St_t was formed on s
            TRY(filter_keep_state(p, t, false, sa, sa));
        }
        if (full || seg) {                                // s reads (and later overwrites) St after these
            HIPCK(hipEventRecord(p->ev_fr[k], sa));
            HIPCK(hipStreamWaitEvent(s, p->ev_fr[k], 0));
        }
        // m x m chain: L_t^{-1}, G_t, St_{t+1}
        if (t >= 2) HIPCK(hipStreamWaitEvent(s, p->ev_fa[k], 0));            // step t - 2 done with slot k
        TRY(filter_mchain(p, t, T, s));
        HIPCK(hipEventRecord(p->ev_fg[k], s));
        // N side of step t: C_t (slot k, read by downdate t - 2 before), the mean, B_{t+1}
        HIPCK(hipStreamWaitEvent(sa, p->ev_fg[k], 0));
        if (t >= 2) HIPCK(hipStreamWaitEvent(sa, p->ev_dd[k], 0));
        if (B == 1) {
            TRY(filter_gain_mean(p, t, Y + t * m, x_filt + t * N, sa));
        } else {
            TRY(filter_gain_mean(p, t, nullptr, nullptr, sa));
            const double* xprev = t == 0 ? p->Xb0 : x_filt + (t - 1) * N;
            TRY(filter_mean_batch(p, t, B, xprev, t == 0 ? p->ldN : T * N, Y + t * m, T * m, x_filt + t * N,
                                  T * N, sa));
        }
        HIPCK(hipEventRecord(p->ev_cc[k], sa));
        if (p->keep) {   // C_t, L_t^-1 and L_t^-1 e_t (one row per data set) for the mean-only smoother
            HIPCK(hipMemcpyAsync(p->fac_C + t * m * p->ldN, p->Cm2[k], (size_t)m * p->ldN * 8,
                                 hipMemcpyDeviceToDevice, sa));
            HIPCK(hipMemcpyAsync(p->fac_L + t * m * p->ldm, p->Li2[k], (size_t)m * p->ldm * 8,
                                 hipMemcpyDeviceToDevice, sa));
            HIPCK(hipMemcpyAsync(p->fac_w + t * p->wcap * p->ldm, B == 1 ? p->w : p->Wb,
                                 (B == 1 ? (size_t)m : (size_t)B * p->ldm) * 8, hipMemcpyDeviceToDevice, sa));
        }
        if (t + 1 < T && !refresh_step(p, t + 1)) TRY(filter_b_update(p, t, sa));
        HIPCK(hipEventRecord(p->ev_fa[k], sa));
        // downdate of step t
        if (sd != sa) HIPCK(hipStreamWaitEvent(sd, p->ev_cc[k], 0));
        TRY(filter_downdate(p, t, prev64, out64, out32, diag, sd, true));
        if (!direct && slot64(p) && kept(p, t, T)) {
            HIPCK(hipMemcpyAsync(slot_ptr(p, slot_of(p, t, T)), out64, slot_elems(p) * 8, hipMemcpyDeviceToDevice,
                                 sd));
        }
        HIPCK(hipEventRecord(p->ev_dd[k], sd));
        prev64 = out64;
    }
    HIPCK(hipStreamWaitEvent(s0, p->ev_fg[(T - 1) & 1], 0));
    HIPCK(hipStreamWaitEvent(s0, p->ev_fa[(T - 1) & 1], 0));
    HIPCK(hipStreamWaitEvent(s0, p->ev_dd[(T - 1) & 1], 0));
    return sync_and_check(p, "kf_filter");
}

kf_status kf_filter_batch(kf_plan* p, int64_t B, int64_t T, const double* Y, double* x_filt, double* Pdiag_filt) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    p->T_done = 0;
    if (B < 1 || T <= 0 || T > p->Tmax || !Y || !x_filt) {
        p->err = "kf_filter: need B >= 1, 1 <= T <= T_max and non-null Y, x_filt";
        return KF_EINVAL;
    }
    kf_status st = filter_impl(p, B, T, Y, x_filt, Pdiag_filt);
    if (st == KF_OK) {
        p->T_done = T;
        p->B_done = B;
        p->xf_last = x_filt;
    }
    return st;
}

kf_status kf_filter(kf_plan* p, int64_t T, const double* Y, double* x_filt, double* Pdiag_filt) {
    return kf_filter_batch(p, 1, T, Y, x_filt, Pdiag_filt);
}

}  // extern "C"

namespace {

// Recompute the filtered covariances of steps [t0, t1] (0-based) from the checkpoint before t0 into
// the segment buffer; seg slot (t - t0) holds P_t afterwards.
kf_status recompute_segment(kf_plan* p, int64_t t0, int64_t t1, int64_t T) {
    hipStream_t s = p->stream;
    const bool s32 = p->store32;
    const size_t esz = s32 ? 4 : 8;
    // starting covariance: P_{t0-1} from its checkpoint (or P0)
    const double* prev64;
    if (t0 == 0) {
        prev64 = p->P0;
    } else {
        const void* src = slot_ptr(p, slot_of(p, t0 - 1, T));   // float64 checkpoint
        HIPCK(copy2d((int)p->N, (int)p->N, p->Pw[0], false, p->ldN, src, false, p->ldN, s));
        prev64 = p->Pw[0];
    }
    for (int64_t t = t0; t <= t1; ++t) {
        double* out64 = p->Pw[(t - t0 + 1) & 1];
        void* segslot = static_cast<char*>(p->seg) + (size_t)(t - t0) * slot_elems(p) * esz;
        float* out32 = s32 ? static_cast<float*>(segslot) : nullptr;
        TRY(filter_cov_step(p, t, T, prev64, out64, out32, t == t0));
        if (!s32) HIPCK(hipMemcpyAsync(segslot, out64, slot_elems(p) * 8, hipMemcpyDeviceToDevice, s));
        prev64 = out64;
    }
    return KF_OK;
}

// Smoother gains for a batch of steps (eqn11): A_t = P_{t|t} F^T P_{t+1|t}^{-1} for each
// t = ts[b], into gain set `set`. With L the Cholesky factor of P_{t+1|t} (outer-blocked; only
// its diagonal blocks are inverted),
//     Y = L^{-1} F P_{t|t},   A_t^T = L^{-T} Y,
// two blocked triangular solves; A_t^T is then transposed in place (and rounded to float32 for
// the mixed path). Y = H^T with H = P_{t|t} F^T L^{-T} stays in the stream's Li buffers (the
// associative smoother uses H H^T). The steps are independent given the stored P_{t|t}, so
// every launch covers the whole batch.
kf_status gain_batch(kf_plan* p, int set, int q, int count, const int64_t* ts, const void* const* Pt,
                     const bool* is32, hipStream_t s) {
    double* const* Wq = p->W[q];
    double* const* Yq = p->Li[q];
    const int N = (int)p->N;
    const int64_t ld = p->ldN;
    const double* P64[kMaxBatch];
    const double* rhs[kMaxBatch];
    double *Db[kMaxBatch], *Tb[kMaxBatch];
    int steps[kMaxBatch];
    for (int b = 0; b < count; ++b) {
        P64[b] = static_cast<const double*>(Pt[b]);
        if (p->store32) {        // the float32 store's value, whether read from it or from a checkpoint
            HIPCK(copy2d_r32(N, N, p->Pt64[set][b], ld, Pt[b], is32[b], ld, s));
            P64[b] = p->Pt64[set][b];
        }
        if (p->hasF) {
            // G_t = P_t F^T (in Y's buffer until the solves need it); W = F G_t + Q (eqn7);
            // right-hand side F P_t in A_t's buffer (read by the first solve only)
            HIPCK(dense_sparse_t(p->F, P64[b], ld, Yq[b], ld, s));
            HIPCK(spmm_rows(p->F, Yq[b], ld, 1.0, p->Q, ld, 1.0, nullptr, 0, 0.0, Wq[b], false, ld, s));
            HIPCK(spmm_rows(p->F, P64[b], ld, 1.0, nullptr, 0, 0.0, nullptr, 0, 0.0, p->Ab[set][b], false, ld, s));
            rhs[b] = p->Ab[set][b];
        } else {
            rhs[b] = P64[b];      // W = P_t + Q (= P_{t+1|t}, eqn7) is formed inside the factorisation
        }
        Db[b] = p->Dg[q][b];
        Tb[b] = p->Dg[q][b] + (size_t)N * p->gld;
        steps[b] = (int)ts[b] + 1;
    }
    HIPCK(chol_blocked_batch(N, p->gnb, Wq, ld, Db, p->gld, Tb, ld, count, p->dstatus, W_PPRED, steps, s,
                             p->hasF ? nullptr : P64, p->hasF ? nullptr : p->Q));
    HIPCK(trsm_lower_batch(N, p->gnb, Wq, ld, Db, p->gld, Tb, ld, rhs, ld, Yq, ld, count, s));
    HIPCK(trsm_upper_t_batch(N, p->gnb, Wq, ld, Db, p->gld, Tb, ld, Yq, ld, p->Ab[set], ld, count, s));
    TransposeInPlace tr;
    for (int b = 0; b < count; ++b) {
        tr.A[b] = p->Ab[set][b];
        tr.A32[b] = mixed(p) ? p->A32[set][b] : nullptr;
    }
    HIPCK(transpose_square_inplace(tr, count, N, ld, s));
    return KF_OK;
}

// The sequential part of smoother step t given A_t (slot b of gain set `set`):
// eqn12 for the mean and eqn13 for the covariance.
kf_status chain_step(kf_plan* p, int set, int b, int64_t t, const void* Pt, const double* Ps_next,
                     double* Ps_out, const double* xf, double* xs, double* Pdiag) {
    hipStream_t s = p->stream;
    const int N = (int)p->N;
    const int64_t ld = p->ldN;
    const double* Pt64 = p->store32 ? p->Pt64[set][b] : static_cast<const double*>(Pt);
    const double* A = p->Ab[set][b];
    // x_{t|T} = x_{t|t} + A_t (x_{t+1|T} - x_{t|t})   (eqn12, RTS reading)
    if (p->B_done == 1) {
        const double* xpred = xf + t * N;    // x_{t+1|t} = F x_{t|t} (eqn6)
        if (p->hasF) {
            HIPCK(spmv_rows(p->F, xf + t * N, N, 1, p->xp, N, s));
            xpred = p->xp;
        }
        HIPCK(gemv_smooth(A, ld, xf + t * N, xpred, xs + (t + 1) * N, xs + t * N, N, s));
    }
    else TRY(smooth_mean_batch(p, p->B_done, A, t, xf, xs));
    // With a transition F the gain A_t has a large norm (F P_{t|t} F^T + Q is far worse
    // conditioned than P_{t|t} + Q), so A_t D A_t^T forms a small result from large terms and
    // float32 accumulation loses the stated accuracy: eqn13 then runs in float64 in both precisions.
    if (mixed(p) && !p->hasF) {
        // D = P_{t+1|T} - P_t - Q in float32; M = A D; P_{t|T} = P_t + M A^T   (eqn13)
        HIPCK(axpby3(N, N, p->D32, true, ld, Ps_next, false, ld, Pt64, false, ld, -1.0, p->Q, false, ld, -1.0, s));
        GemmProblem g;
        g.M = N; g.N = N; g.K = N;
        g.A = p->A32[set][b]; g.lda = ld; g.B = p->D32; g.ldb = ld; g.flags = G_TB;   // D symmetric
        g.C32 = p->M32; g.ldc32 = ld;
        TRY(big_gemm(p, Dt::F32, g, 2.0 * N * N * N, s, &p->ts_m));
        GemmProblem h;
        h.M = N; h.N = N; h.K = N;
        h.A = p->M32; h.lda = ld; h.B = p->A32[set][b]; h.ldb = ld; h.flags = G_TB | G_LOWER | G_MIRROR;
        h.Cin = Pt64; h.ldcin = ld; h.beta = 1.0;
        h.C = Ps_out; h.ldc = ld; h.diag = Pdiag;
        TRY(big_gemm(p, Dt::F32, h, (double)N * N * N, s, &p->ts_low));
    } else {
        // D = P_{t+1|T} - P_t - Q;  M = A_t D;  P_{t|T} = P_t + M A_t^T   (eqn13)
        if (p->hasF) {                      // D = P_{t+1|T} - F (P_t F^T) - Q   (M's buffer holds P_t F^T)
            HIPCK(dense_sparse_t(p->F, Pt64, ld, p->Mm, ld, s));
            HIPCK(spmm_rows(p->F, p->Mm, ld, -1.0, Ps_next, ld, 1.0, p->Q, ld, -1.0, p->Dm, false, ld, s));
        } else {
            HIPCK(axpby3(N, N, p->Dm, false, ld, Ps_next, false, ld, Pt64, false, ld, -1.0, p->Q, false, ld, -1.0, s));
        }
        GemmProblem g;
        g.M = N; g.N = N; g.K = N;
        g.A = A; g.lda = ld;
        g.B = p->Dm; g.ldb = ld; g.flags = G_TB;   // D symmetric: read row-contiguous
        g.C = p->Mm; g.ldc = ld;
        TRY(big_gemm(p, Dt::F64, g, 2.0 * N * N * N, s, &p->ts_m));
        GemmProblem h;
        h.M = N; h.N = N; h.K = N;
        h.A = p->Mm; h.lda = ld; h.B = A; h.ldb = ld; h.flags = G_TB | G_LOWER | G_MIRROR;
        h.Cin = Pt64; h.ldcin = ld; h.beta = 1.0;
        h.C = Ps_out; h.ldc = ld; h.diag = Pdiag;
        TRY(big_gemm(p, Dt::F64, h, (double)N * N * N, s, &p->ts_low));
    }
    return KF_OK;
}

kf_status smooth_impl(kf_plan* p, double* xs, double* Pdiag, double* Pfull) {
    hipStream_t s = p->stream;
    const int64_t T = p->T_done, N = p->N;
    const int64_t ld = p->ldN;
    const bool s32 = p->store32;
    const size_t esz = s32 ? 4 : 8;
    const double* xf = p->xf_last;
    HIPCK(status_clear(p->dstatus, s));
    // t = T-1: smoother = filter
    const void* PT = slot_ptr(p, slot_of(p, T - 1, T));
    if (s32) HIPCK(copy2d_r32((int)N, (int)N, p->Ps[(T - 1) & 1], ld, PT, !slot64(p), ld, s));
    else HIPCK(copy2d((int)N, (int)N, p->Ps[(T - 1) & 1], false, ld, PT, false, ld, s));
    HIPCK(hipMemcpy2DAsync(xs + (T - 1) * N, T * N * 8, xf + (T - 1) * N, T * N * 8, N * 8, p->B_done,
                           hipMemcpyDeviceToDevice, s));
    if (Pdiag) HIPCK(diag_copy(p->Ps[(T - 1) & 1], ld, (int)N, Pdiag + (T - 1) * N, s));
    if (Pfull)
        HIPCK(hipMemcpy2DAsync(Pfull + (T - 1) * N * N, N * 8, p->Ps[(T - 1) & 1], ld * 8, N * 8, N,
                               hipMemcpyDeviceToDevice, s));
    auto run_chain = [&](int set, int count, const int64_t* ts, const void* const* Pt) -> kf_status {
        for (int b = 0; b < count; ++b) {
            const int64_t u = ts[b];
            Range r("kf_smooth step t=%lld", (long long)u + 1);
            double* Ps_out = p->Ps[u & 1];
            TRY(chain_step(p, set, b, u, Pt[b], p->Ps[(u + 1) & 1], Ps_out, xf, xs, Pdiag ? Pdiag + u * N : nullptr));
            if (Pfull)
                HIPCK(hipMemcpy2DAsync(Pfull + u * N * N, N * 8, Ps_out, ld * 8, N * 8, N, hipMemcpyDeviceToDevice,
                                       s));
        }
        return KF_OK;
    };
    if (p->stride == 1 && !p->serial) {
        // Every P_{t|t} is stored: gains run one batch ahead on the side stream.
        struct Batch { int count; int64_t ts[kMaxBatch]; const void* Pt[kMaxBatch]; bool is32[kMaxBatch]; };
        std::vector<Batch> batches;
        for (int64_t t = T - 2; t >= 0;) {
            Batch bt;
            bt.count = 0;
            // a short first batch lets the back-recursion start early; later batches are full
            const int cap = batches.empty() ? std::min(p->gbatch, 2) : p->gbatch;
            while (bt.count < cap && t - bt.count >= 0) {
                bt.ts[bt.count] = t - bt.count;
                bt.Pt[bt.count] = slot_ptr(p, t - bt.count);
                bt.is32[bt.count] = !slot64(p);
                ++bt.count;
            }
            batches.push_back(bt);
            t -= bt.count;
        }
        // Batch k is formed on side stream k % nprod into gain set k % (nprod + 1); the
        // back-recursion consumes the sets in order, and a set is formed again only after the
        // chain that read it has been enqueued and has recorded its event.
        HIPCK(hipEventRecord(p->ev_start, s));
        for (int q = 0; q < p->nprod; ++q) HIPCK(hipStreamWaitEvent(p->s2[q], p->ev_start, 0));
        const size_t nb = batches.size();
        const int np = p->nprod, ns = p->nprod + 1;
        auto produce = [&](size_t k) -> kf_status {
            const int q = (int)(k % np), set = (int)(k % ns);
            Range r("kf_smooth gain batch t=%lld..%lld", (long long)batches[k].ts[batches[k].count - 1] + 1,
                    (long long)batches[k].ts[0] + 1);
            if (k >= (size_t)ns) HIPCK(hipStreamWaitEvent(p->s2[q], p->ev_chain[set], 0));   // chain k - ns done
            TRY(gain_batch(p, set, q, batches[k].count, batches[k].ts, batches[k].Pt, batches[k].is32, p->s2[q]));
            HIPCK(hipEventRecord(p->ev_gain[set], p->s2[q]));
            return KF_OK;
        };
        for (size_t k = 0; k < nb && k < (size_t)np; ++k) TRY(produce(k));
        for (size_t k = 0; k < nb; ++k) {
            if (k + np < nb) TRY(produce(k + np));
            const int set = (int)(k % ns);
            HIPCK(hipStreamWaitEvent(s, p->ev_gain[set], 0));
            TRY(run_chain(set, batches[k].count, batches[k].ts, batches[k].Pt));
            HIPCK(hipEventRecord(p->ev_chain[set], s));
        }
    } else {
        // Checkpointed store (segments are recomputed into one buffer) or a serialised
        // measurement pass: everything stays on the plan's stream.
        int64_t seg_lo = -1, seg_hi = -2;
        auto stored = [&](int64_t u) -> const void* {
            if (kept(p, u, T)) return slot_ptr(p, slot_of(p, u, T));
            if (u < seg_lo || u > seg_hi) return nullptr;
            return static_cast<char*>(p->seg) + (size_t)(u - seg_lo) * slot_elems(p) * esz;
        };
        int64_t t = T - 2;
        while (t >= 0) {
            if (!stored(t)) {
                // segment of non-kept steps containing t: (previous checkpoint, t]
                seg_lo = (t + 1) / p->stride * p->stride;
                seg_hi = t;
                Range r("kf_smooth recompute t=%lld..%lld", (long long)seg_lo + 1, (long long)seg_hi + 1);
                TRY(recompute_segment(p, seg_lo, seg_hi, T));
            }
            int64_t ts[kMaxBatch];
            const void* Pt[kMaxBatch];
            bool is32[kMaxBatch];
            int count = 0;
            while (count < p->gbatch && t - count >= 0 && stored(t - count)) {
                ts[count] = t - count;
                Pt[count] = stored(t - count);
                is32[count] = kept(p, t - count, T) ? !slot64(p) : s32;   // checkpoints float64, segment as stored
                ++count;
            }
            {
                Range r("kf_smooth gain batch t=%lld..%lld", (long long)ts[count - 1] + 1, (long long)ts[0] + 1);
                TRY(gain_batch(p, 0, 0, count, ts, Pt, is32, s));
            }
            TRY(run_chain(0, count, ts, Pt));
            t -= count;
        }
    }
    kf_status st = sync_and_check(p, "kf_smooth");
    if (st == KF_OK && p->prof) TRY(collect_profile(p));
    return st;
}

// Smoothed means alone for the B data sets of the last filter call (backward information
// recursion): with mu = F^T lambda_{t+1} (lambda_{t+1} itself when F = I),
// x_{t|T} = x_{t|t} + P_{t|t} mu, lambda_t = mu + X^T L_t^-T (L_t^-1 e_t - C_t mu), lambda_T = 0.
kf_status smooth_means_impl(kf_plan* p, int64_t B, double* xs) {
    hipStream_t s = p->stream;
    const int64_t T = p->T_done, N = p->N, m = p->m;
    const int64_t ld = p->ldN, ldx = T * N;
    const double* xf = p->xf_last;
    TRY(ensure_batch(p, B));                       // Xb0 / Vb: lambda double buffer; Eb, Wb: m-vectors
    double* lam[2] = {p->Xb0, p->Vb};
    HIPCK(zero2d((int)B, (int)N, lam[T & 1], ld, s));
    HIPCK(hipMemcpy2DAsync(xs + (T - 1) * N, ldx * 8, xf + (T - 1) * N, ldx * 8, N * 8, B, hipMemcpyDeviceToDevice,
                           s));
    const bool s32 = p->store32;
    int64_t seg_lo = -1, seg_hi = -2;
    for (int64_t t = T - 1; t >= 0; --t) {
        const double* ln = lam[(t + 1) & 1];       // lambda_{t+1}
        double* lc = lam[t & 1];                   // lambda_t
        if (p->hasF) {                             // everything below uses F^T lambda_{t+1}
            double* mu = B == 1 ? p->xp : p->Ub;
            HIPCK(spmv_rows(p->Ft, ln, ld, (int)B, mu, ld, s));
            ln = mu;
        }
        if (t < T - 1) {
            // P_{t|t}: a stored slot, or recomputed from the checkpoint before it
            const void* Pt;
            bool p32;
            if (kept(p, t, T)) {
                Pt = slot_ptr(p, slot_of(p, t, T));
                p32 = !slot64(p);
            } else {
                if (t < seg_lo || t > seg_hi) {
                    seg_lo = (t + 1) / p->stride * p->stride;
                    seg_hi = t;
                    TRY(recompute_segment(p, seg_lo, seg_hi, T));
                }
                Pt = static_cast<char*>(p->seg) + (size_t)(t - seg_lo) * slot_elems(p) * (s32 ? 4 : 8);
                p32 = s32;
            }
            // A float32 store holds P_{t|t} rounded to float32 (a float64 checkpoint too)
            if (s32 && (!p32 || B > 1)) {
                HIPCK(copy2d_r32((int)N, (int)N, p->Pw[0], ld, Pt, p32, ld, s));
                Pt = p->Pw[0];
                p32 = false;
            }
            if (B == 1) {
                HIPCK(gemv_add(Pt, p32, ld, ln, xf + t * N, xs + t * N, (int)N, s));
            } else {
                GemmProblem g;                     // X_{t|T} = X_{t|t} + Lambda_{t+1} P_{t|t}  (P symmetric)
                g.M = (int)B; g.N = (int)N; g.K = (int)N;
                g.A = ln; g.lda = ld; g.B = Pt; g.ldb = ld; g.flags = G_TB;
                g.Cin = xf + t * N; g.ldcin = ldx; g.beta = 1.0;
                g.C = xs + t * N; g.ldc = ldx;
                g.ksplit = batch_ksplit(p, B, N, 4);
                g.partial = p->partial;
                HIPCK(gemm1(Dt::F64, g, s));
            }
        }
        if (t == 0) break;                         // lambda_0 is not needed
        const double* C = p->fac_C + t * m * p->ldN;
        const double* L = p->fac_L + t * m * p->ldm;
        const double* w = p->fac_w + t * p->wcap * p->ldm;
        if (B == 1) {
            HIPCK(resid(C, p->ldN, ln, w, p->e, (int)m, (int)N, s));           // v = L^-1 e - C lambda
            HIPCK(trmv_lower_t(L, p->ldm, p->e, p->w, (int)m, s));            // u = L^-T v
            HIPCK(gemv_t_add(p->X, p->ldN, p->w, ln, lc, nullptr, (int)m, (int)N, s));   // lambda += X^T u
        } else {
            GemmProblem g;                         // V = W_t - Lambda C_t^T
            g.M = (int)B; g.N = (int)m; g.K = (int)N;
            g.A = ln; g.lda = ld; g.B = C; g.ldb = p->ldN; g.flags = G_TB;
            g.alpha = -1.0;
            g.Cin = w; g.ldcin = p->ldm; g.beta = 1.0;
            g.C = p->Eb; g.ldc = p->ldm;
            g.ksplit = batch_ksplit(p, B, m, std::max(1, std::min(16, (int)N / 256)));
            g.partial = p->partial;
            HIPCK(gemm1(Dt::F64, g, s));
            GemmProblem h;                         // U = V L^-1  (rows: L^-T v_b)
            h.M = (int)B; h.N = (int)m; h.K = (int)m;
            h.A = p->Eb; h.lda = p->ldm; h.B = L; h.ldb = p->ldm; h.flags = G_BLOWER;
            h.C = p->Wb; h.ldc = p->ldm;
            HIPCK(gemm1(Dt::F64, h, s));
            GemmProblem u;                         // Lambda_t = Lambda_{t+1} + U X
            u.M = (int)B; u.N = (int)N; u.K = (int)m;
            u.A = p->Wb; u.lda = p->ldm; u.B = p->X; u.ldb = p->ldN;
            u.Cin = ln; u.ldcin = ld; u.beta = 1.0;
            u.C = lc; u.ldc = ld;
            HIPCK(gemm1(Dt::F64, u, s));
        }
    }
    return sync_and_check(p, "kf_smooth_means");
}

// Time-parallel smoother: eqn12 and eqn13 regrouped as a suffix scan with an associative
// operator. Each step t < T-1 contributes the element
//     E_t = A_t,   g_t = x_{t|t} - A_t F x_{t|t},   L_t = P_{t|t} - H_t H_t^T
// with H_t = P_{t|t} F^T C_t^{-T} the first factor of the gain, C_t the Cholesky factor of
// P_{t+1|t} (A_t = H_t C_t^{-1}), so that
// H_t H_t^T = A_t F P_{t|t} = A_t P_{t+1|t} A_t^T; step T-1 contributes (0, x_{T|T}, P_{T|T}).
// With
//     (E, g, L) o (E', g', L') = (E E', E g' + g, E L' E^T + L)
// the suffix product from t to T-1 is (0, x_{t|T}, P_{t|T}): one RTS step is the action of an
// element on (x_{t+1|T}, P_{t+1|T}), and composing two steps is the operator above.
//
// Blocks of length l = ceil(sqrt(T)): (1) suffix products inside every block, one launch group
// per position over all blocks; (2) the block totals combined from the last block back;
// (3) every element of a block combined with the total of the blocks after it, all at once.
// The depth is about 3 sqrt(T) launch groups instead of T dependent steps, for about twice
// the products of the step-by-step smoother (E E' inside blocks, E L' E^T everywhere).
// The elements overwrite the stored P_{t|t}; E_t lives in a separate allocation of T - 1
// matrices made for the call.
kf_status smooth_assoc_impl(kf_plan* p, double* xs, double* Pdiag, double* Pfull) {
    hipStream_t s = p->stream;
    const int64_t T = p->T_done, N = p->N, ld = p->ldN;
    const int n = (int)N;
    const size_t mat = slot_elems(p);
    const double* xf = p->xf_last;
    constexpr int GE = kMaxGroup / 2;            // combines per launch group with an E E' product
    constexpr int G = kMaxGroup;                 // combines per launch group without one
    const int64_t nE = T - 1;
    const size_t need = assoc_bytes(N, ld, T);
    void* block = nullptr;
    if (hipMalloc(&block, need) != hipSuccess) {
        (void)hipGetLastError();
        p->err = "kf_smooth_assoc: could not allocate " + std::to_string(need >> 20) + " MiB for the scan elements";
        return KF_ENOMEM;
    }
    struct Free {
        void* b;
        ~Free() { if (b) (void)hipFree(b); }
    } guard{block};
    double* base = static_cast<double*>(block);
    std::vector<double*> E(nE), Et(GE), Wt(G);
    for (int64_t t = 0; t < nE; ++t) E[t] = base + t * mat;
    for (int k = 0; k < GE; ++k) Et[k] = base + (nE + k) * mat;
    for (int k = 0; k < G; ++k) Wt[k] = base + (nE + GE + k) * mat;
    double* zero = base + (nE + GE + G) * mat;
    double* u = zero + N;
    std::vector<double*> L(T);
    for (int64_t t = 0; t < T; ++t) L[t] = static_cast<double*>(slot_ptr(p, t));
    std::vector<char> ezero(T, 0);               // suffix already contains step T-1: E = 0
    ezero[T - 1] = 1;

    p->T_done = 0;                                       // the stored P_{t|t} are overwritten below
    HIPCK(status_clear(p->dstatus, s));
    HIPCK(zero2d(1, n, zero, N, s));
    HIPCK(hipMemcpyAsync(xs + (T - 1) * N, xf + (T - 1) * N, N * 8, hipMemcpyDeviceToDevice, s));

    // Elements, gbatch steps at a time: A_t straight into E_t, then g_t and L_t (over P_{t|t}).
    for (int64_t t0 = T - 2; t0 >= 0;) {
        const int cnt = (int)std::min<int64_t>(p->gbatch, t0 + 1);
        int64_t ts[kMaxBatch];
        const void* Pt[kMaxBatch];
        bool is32[kMaxBatch];
        double* saved[kMaxBatch];
        for (int b = 0; b < cnt; ++b) {
            ts[b] = t0 - b;
            Pt[b] = L[t0 - b];
            is32[b] = false;
            saved[b] = p->Ab[0][b];
            p->Ab[0][b] = E[t0 - b];
        }
        const kf_status st = gain_batch(p, 0, 0, cnt, ts, Pt, is32, s);
        for (int b = 0; b < cnt; ++b) p->Ab[0][b] = saved[b];
        if (st != KF_OK) return st;
        GemmProblem g[kMaxBatch];
        for (int b = 0; b < cnt; ++b) {
            const int64_t t = ts[b];
            const double* Fx = xf + t * N;
            if (p->hasF) {
                HIPCK(spmv_rows(p->F, xf + t * N, N, 1, u, N, s));
                Fx = u;
            }
            HIPCK(gemv_smooth(E[t], ld, xf + t * N, Fx, zero, xs + t * N, n, s));    // g_t = x - A F x
            // L_t = P_t - H_t H_t^T (lower tiles + mirror) over the slot; H_t^T is still in Li
            g[b].M = n; g[b].N = n; g[b].K = n;
            g[b].A = p->Li[0][b]; g[b].lda = ld; g[b].B = p->Li[0][b]; g[b].ldb = ld;
            g[b].flags = G_TA | G_LOWER | G_MIRROR;
            g[b].alpha = -1.0; g[b].beta = 1.0; g[b].Cin = L[t]; g[b].ldcin = ld;
            g[b].C = L[t]; g[b].ldc = ld;
        }
        TRY(big_group(p, Dt::F64, g, cnt, (double)cnt * N * N * N, s));
        t0 -= cnt;
    }

    // s_t <- a_t o s_r for a list of independent pairs (no r is a t of the same list), GE at a
    // time while E E' products are needed, else G at a time.
    auto combine = [&](const std::vector<std::pair<int64_t, int64_t>>& pairs) -> kf_status {
        for (size_t c0 = 0; c0 < pairs.size();) {
            bool withE = false;
            for (size_t k = c0; k < pairs.size() && k < c0 + G; ++k) withE = withE || !ezero[pairs[k].second];
            const int cnt = (int)std::min<size_t>(withE ? GE : G, pairs.size() - c0);
            GemmProblem g1[kMaxGroup], g2[kMaxGroup];
            GemvAddBatch gv;
            int n1 = 0;
            for (int k = 0; k < cnt; ++k) {
                const int64_t t = pairs[c0 + k].first, r = pairs[c0 + k].second;
                if (!ezero[r]) {                 // E_t E_r
                    GemmProblem e;
                    e.M = n; e.N = n; e.K = n;
                    e.A = E[t]; e.lda = ld; e.B = E[r]; e.ldb = ld;
                    e.C = Et[k]; e.ldc = ld;
                    g1[n1++] = e;
                }
                GemmProblem w;                   // W = E_t L_r   (L_r symmetric: read row-contiguous)
                w.M = n; w.N = n; w.K = n;
                w.A = E[t]; w.lda = ld; w.B = L[r]; w.ldb = ld; w.flags = G_TB;
                w.C = Wt[k]; w.ldc = ld;
                g1[n1++] = w;
                gv.A[k] = E[t]; gv.x[k] = xs + r * N; gv.y[k] = xs + t * N;          // g_t += E_t g_r
                GemmProblem l;                   // L_t = W E_t^T + L_t
                l.M = n; l.N = n; l.K = n;
                l.A = Wt[k]; l.lda = ld; l.B = E[t]; l.ldb = ld; l.flags = G_TB | G_LOWER | G_MIRROR;
                l.beta = 1.0; l.Cin = L[t]; l.ldcin = ld;
                l.C = L[t]; l.ldc = ld;
                g2[k] = l;
            }
            TRY(big_group(p, Dt::F64, g1, n1, 2.0 * N * N * N * n1, s));
            HIPCK(gemv_add_batch(gv, cnt, ld, n, s));
            TRY(big_group(p, Dt::F64, g2, cnt, (double)cnt * N * N * N, s));
            for (int k = 0; k < cnt; ++k) {
                const int64_t t = pairs[c0 + k].first, r = pairs[c0 + k].second;
                if (ezero[r]) ezero[t] = 1;
                else std::swap(E[t], Et[k]);     // the product becomes E_t; the old buffer is free
            }
            c0 += cnt;
        }
        return KF_OK;
    };
    const int64_t len = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)T)));
    const int64_t nb = (T + len - 1) / len;
    auto first = [&](int64_t b) { return b * len; };
    auto last = [&](int64_t b) { return std::min(T, (b + 1) * len) - 1; };
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int64_t i = len - 2; i >= 0; --i) {             // (1) inside every block
        pairs.clear();
        for (int64_t b = 0; b < nb; ++b)
            if (first(b) + i + 1 <= last(b)) pairs.emplace_back(first(b) + i, first(b) + i + 1);
        TRY(combine(pairs));
    }
    for (int64_t b = nb - 2; b >= 0; --b) {              // (2) block totals, last block first
        pairs.assign(1, {first(b), first(b + 1)});
        TRY(combine(pairs));
    }
    pairs.clear();                                       // (3) the rest of every block
    for (int64_t b = 0; b + 1 < nb; ++b)
        for (int64_t t = first(b) + 1; t <= last(b); ++t) pairs.emplace_back(t, first(b + 1));
    TRY(combine(pairs));

    for (int64_t t = 0; t < T; ++t) {
        if (Pdiag) HIPCK(diag_copy(L[t], ld, n, Pdiag + t * N, s));
        if (Pfull)
            HIPCK(hipMemcpy2DAsync(Pfull + t * N * N, N * 8, L[t], ld * 8, N * 8, N, hipMemcpyDeviceToDevice, s));
    }
    const kf_status st = sync_and_check(p, "kf_smooth_assoc");
    if (st == KF_OK && p->prof) TRY(collect_profile(p));
    return st;
}

}  // namespace

extern "C" {

kf_status kf_smooth_batch(kf_plan* p, int64_t B, double* x_smooth, double* Pdiag_smooth, double* P_smooth) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    if (p->T_done <= 0 || !p->xf_last) {
        p->err = "kf_smooth: no completed kf_filter on this plan";
        return KF_ESTATE;
    }
    if (B != p->B_done) {
        p->err = "kf_smooth: the last filter call ran " + std::to_string(p->B_done) + " data set(s), not " +
                 std::to_string(B);
        return KF_ESTATE;
    }
    if (!x_smooth) {
        p->err = "kf_smooth: x_smooth is null";
        return KF_EINVAL;
    }
    return smooth_impl(p, x_smooth, Pdiag_smooth, P_smooth);
}

kf_status kf_smooth(kf_plan* p, double* x_smooth, double* Pdiag_smooth, double* P_smooth) {
    return kf_smooth_batch(p, 1, x_smooth, Pdiag_smooth, P_smooth);
}

kf_status kf_smooth_assoc(kf_plan* p, double* x_smooth, double* Pdiag_smooth, double* P_smooth) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    if (p->arena) {
        p->err = "kf_smooth_assoc: not available on plans owned by a serving context";
        return KF_EINVAL;
    }
    if (mixed(p)) {
        p->err = "kf_smooth_assoc: needs a float64 plan (precision KF_FP64)";
        return KF_EINVAL;
    }
    if (!x_smooth) {
        p->err = "kf_smooth_assoc: x_smooth is null";
        return KF_EINVAL;
    }
    if (p->T_done <= 0 || !p->xf_last) {
        p->err = "kf_smooth_assoc: no completed kf_filter on this plan (the previous kf_smooth_assoc consumed it)";
        return KF_ESTATE;
    }
    if (p->B_done != 1) {
        p->err = "kf_smooth_assoc: the last filter call ran several data sets";
        return KF_ESTATE;
    }
    if (p->store32 || p->stride != 1) {
        p->err = "kf_smooth_assoc: needs every P_{t|t} stored in float64 (no float32 store, no checkpointing)";
        return KF_ESTATE;
    }
    return smooth_assoc_impl(p, x_smooth, Pdiag_smooth, P_smooth);
}

kf_status kf_smooth_means_batch(kf_plan* p, int64_t B, double* x_smooth) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    if (!p->keep) {
        p->err = "kf_smooth_means: the plan was created without keep_gain_factors";
        return KF_ESTATE;
    }
    if (p->T_done <= 0 || !p->xf_last) {
        p->err = "kf_smooth_means: no completed kf_filter on this plan";
        return KF_ESTATE;
    }
    if (B != p->B_done) {
        p->err = "kf_smooth_means: the last filter call ran " + std::to_string(p->B_done) + " data set(s), not " +
                 std::to_string(B);
        return KF_ESTATE;
    }
    if (!x_smooth) {
        p->err = "kf_smooth_means: x_smooth is null";
        return KF_EINVAL;
    }
    return smooth_means_impl(p, B, x_smooth);
}

kf_status kf_smooth_means(kf_plan* p, double* x_smooth) { return kf_smooth_means_batch(p, 1, x_smooth); }

kf_status kf_set_transition(kf_plan* p, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* val) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    const int64_t N = p->N;
    p->T_done = 0;                                  // a new model: the last filter call no longer applies
    if (nnz == 0 && !row_ptr && !col_idx && !val) {
        p->hasF = false;
        return KF_OK;
    }
    if (p->arena) {
        p->err = "kf_set_transition: not available on a serving plan";
        return KF_EINVAL;
    }
    if (nnz <= 0 || nnz > ((int64_t)1 << 31) - 1 || !row_ptr || !col_idx || !val) {
        p->err = "kf_set_transition: need 0 < nnz < 2^31 and non-null row_ptr, col_idx, val";
        return KF_EINVAL;
    }
    // Validate on the host: row_ptr non-decreasing from 0 to nnz, column indices in range.
    std::vector<int32_t> rp(N + 1), ci(nnz);
    std::vector<double> v(nnz);
    HIPCK(hipMemcpy(rp.data(), row_ptr, (N + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(ci.data(), col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(v.data(), val, nnz * sizeof(double), hipMemcpyDeviceToHost));
    bool ok = rp[0] == 0 && rp[N] == nnz;
    for (int64_t i = 0; ok && i < N; ++i) ok = rp[i] <= rp[i + 1];
    for (int64_t e = 0; ok && e < nnz; ++e) ok = ci[e] >= 0 && ci[e] < N && std::isfinite(v[e]);
    if (!ok) {
        p->err = "kf_set_transition: row_ptr must rise from 0 to nnz, col_idx lie in [0, N), values be finite";
        return KF_EINVAL;
    }
    // The transpose (for F^T in the mean-only smoother), by a counting sort on the host.
    std::vector<int32_t> trp(N + 1, 0), tci(nnz);
    std::vector<double> tv(nnz);
    for (int64_t e = 0; e < nnz; ++e) ++trp[ci[e] + 1];
    for (int64_t i = 0; i < N; ++i) trp[i + 1] += trp[i];
    std::vector<int32_t> fill(trp.begin(), trp.end() - 1);
    for (int64_t i = 0; i < N; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t d = fill[ci[e]]++;
            tci[d] = (int32_t)i;
            tv[d] = v[e];
        }
    for (void* a : p->fallocs) (void)hipFree(a);
    p->fallocs.clear();
    p->hasF = false;
    if (mixed(p)) {                                 // the float64 eqn13 buffers lived in fallocs
        p->Dm = p->Mm = nullptr;
        p->tail_ws64 = nullptr;
    }
    auto dev = [&](const void* src, size_t bytes) -> void* {
        void* d = nullptr;
        if (hipMalloc(&d, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        p->fallocs.push_back(d);
        if (src && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        return d;
    };
    const size_t NN = (size_t)N * p->ldN * 8;
    void *a = dev(rp.data(), (N + 1) * 4), *b = dev(ci.data(), nnz * 4), *c = dev(v.data(), nnz * 8);
    void *d = dev(trp.data(), (N + 1) * 4), *e = dev(tci.data(), nnz * 4), *f = dev(tv.data(), nnz * 8);
    void *g = dev(nullptr, NN), *h = dev(nullptr, NN), *x = dev(nullptr, (size_t)p->ldN * 8);
    bool more = true;
    if (mixed(p)) {                                 // eqn13 in float64 under F (see chain_step)
        void *dm = dev(nullptr, NN), *mm = dev(nullptr, NN);
        const size_t tb = tail_bytes(N, false);
        void* tw = tb ? dev(nullptr, tb) : nullptr;
        more = dm && mm && (tw || !tb);
        p->Dm = static_cast<double*>(dm);
        p->Mm = static_cast<double*>(mm);
        p->tail_ws64 = tw;
    }
    if (!a || !b || !c || !d || !e || !f || !g || !h || !x || !more) {
        p->err = "kf_set_transition: device allocation failed";
        return KF_ENOMEM;
    }
    p->F.n = p->Ft.n = (int)N;
    p->F.rp = static_cast<int*>(a); p->F.ci = static_cast<int*>(b); p->F.v = static_cast<double*>(c);
    p->Ft.rp = static_cast<int*>(d); p->Ft.ci = static_cast<int*>(e); p->Ft.v = static_cast<double*>(f);
    p->Fg = static_cast<double*>(g);
    p->Fp = static_cast<double*>(h);
    p->xp = static_cast<double*>(x);
    p->hasF = true;
    return KF_OK;
}

kf_status kf_get_filtered_cov(kf_plan* p, int64_t t, double* P_out) {
    if (!p) return KF_EINVAL;
    p->err.clear();
    if (p->T_done <= 0) {
        p->err = "kf_get_filtered_cov: no completed kf_filter";
        return KF_ESTATE;
    }
    if (t < 1 || t > p->T_done || !P_out) {
        p->err = "kf_get_filtered_cov: need 1 <= t <= T and non-null P_out";
        return KF_EINVAL;
    }
    const int64_t T = p->T_done, i = t - 1;
    if (!kept(p, i, T)) {
        const int64_t lo = (i + 1) / p->stride * p->stride;
        TRY(recompute_segment(p, lo, i, T));
        const size_t esz = p->store32 ? 4 : 8;
        const void* src = static_cast<char*>(p->seg) + (size_t)(i - lo) * slot_elems(p) * esz;
        HIPCK(copy2d((int)p->N, (int)p->N, P_out, false, p->N, src, p->store32, p->ldN, p->stream));
    } else if (p->store32) {       // the float32 store's value (a checkpoint is kept in float64)
        HIPCK(copy2d_r32((int)p->N, (int)p->N, P_out, p->N, slot_ptr(p, slot_of(p, i, T)), !slot64(p), p->ldN,
                         p->stream));
    } else {
        HIPCK(copy2d((int)p->N, (int)p->N, P_out, false, p->N, slot_ptr(p, slot_of(p, i, T)), false, p->ldN,
                     p->stream));
    }
    HIPCK(hipStreamSynchronize(p->stream));
    return KF_OK;
}

kf_status kf_set_profiling(kf_plan* p, int on) {
    if (!p) return KF_EINVAL;
    if (on < 0 || on > 2) {
        p->err = "kf_set_profiling: on must be 0, 1 or 2";
        return KF_EINVAL;
    }
    p->prof = on != 0;
    p->serial = on == 2;
    p->prof_ms = 0.0;
    p->prof_flops = 0.0;
    p->prof_launches = 0;
    p->ev_used = 0;
    p->ev_flops.clear();
    return KF_OK;
}

kf_status kf_get_profile(const kf_plan* p, double* kernel_ms, double* kernel_flops, int64_t* launches) {
    if (!p) return KF_EINVAL;
    if (kernel_ms) *kernel_ms = p->prof_ms;
    if (kernel_flops) *kernel_flops = p->prof_flops;
    if (launches) *launches = p->prof_launches;
    return KF_OK;
}

void kf_destroy(kf_plan* p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    for (hipStream_t q : p->s2)
        if (q) (void)hipStreamSynchronize(q);
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    for (int k = 0; k <= kMaxProd; ++k) {
        if (p->ev_gain[k]) (void)hipEventDestroy(p->ev_gain[k]);
        if (p->ev_chain[k]) (void)hipEventDestroy(p->ev_chain[k]);
    }
    for (int k = 0; k < 2; ++k)
        for (hipEvent_t e : {p->ev_fl[k], p->ev_fg[k], p->ev_fr[k], p->ev_fa[k], p->ev_cc[k], p->ev_dd[k]})
            if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : p->s2)
        if (q) (void)hipStreamDestroy(q);
    for (hipStream_t q : {p->sc, p->sdm})
        if (q) (void)hipStreamDestroy(q);
    for (double* b : {p->Eb, p->Wb, p->Xb0, p->Vb, p->Ub})
        if (b) (void)hipFree(b);
    for (double* b : p->bfac_w) (void)hipFree(b);
    for (void* a : p->fallocs) (void)hipFree(a);
    for (void* a : p->allocs) {
        if (p->arena) p->arena->release(a);
        else (void)hipFree(a);
    }
    if (p->hstatus) (void)hipHostFree(p->hstatus);
    delete p;
}

const char* kf_last_error(const kf_plan* p) { return p ? p->err.c_str() : g_err.c_str(); }

}  // extern "C"

namespace kfmeg {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace kfmeg

extern "C" {

kf_status kf_init_from_mne(int64_t N, int64_t m, int64_t T, const double* X, const double* C, const double* R,
                           const double* Y, double reg, double* x0_out, double* Q_out, void* stream) {
    g_err.clear();
    if (N <= 0 || m <= 0 || T < 3 || !X || !C || !R || !Y || !x0_out || !Q_out || !(reg >= 0.0)) {
        g_err = "kf_init_from_mne: need N, m > 0, T >= 3, reg >= 0 and non-null pointers";
        return KF_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    kf_plan tmp;
    kf_plan* p = &tmp;
    const int64_t ld = round_up(N, 16);
    double *J = nullptr, *Dc = nullptr;
    kf_status st = alloc(p, &J, (size_t)T * N);
    if (st == KF_OK) st = alloc(p, &Dc, (size_t)(T - 1) * ld);
    auto run = [&]() -> kf_status {
        kf_status r = mne_solve(N, m, T, X, C, R, Y, J, stream);           // eqn5 at every sample
        if (r != KF_OK) return r;
        HIPCK(diff_center(J, N, (int)T, (int)N, Dc, ld, s));               // J_k - J_{k-1}, centred
        GemmProblem g;                                                      // Dc^T Dc / (T - 2)
        g.M = (int)N; g.N = (int)N; g.K = (int)(T - 1);
        g.A = Dc; g.lda = ld; g.B = Dc; g.ldb = ld; g.flags = G_TA | G_LOWER | G_MIRROR;
        g.alpha = 1.0 / (double)(T - 2);
        g.C = Q_out; g.ldc = N;
        HIPCK(gemm1(Dt::F64, g, s));
        if (reg > 0.0) HIPCK(add_diag(Q_out, N, (int)N, reg, s));
        HIPCK(hipMemcpyAsync(x0_out, J, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCK(hipStreamSynchronize(s));
        return KF_OK;
    };
    if (st == KF_OK) st = run();
    if (st != KF_OK && g_err.empty()) g_err = tmp.err;
    for (void* a : tmp.allocs) (void)hipFree(a);
    tmp.allocs.clear();
    return st;
}

}  // extern "C"
