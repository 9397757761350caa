// Minimum-norm estimate of eqn5 for every sample of the data:
//   G = C X^T (N x m),  S = X G + R,  L Li = chol(S),  J^T = G (Li^T (Li Y^T)),
// two entry points over the same launches: mne_solve allocates its workspace for the call,
// mne_solve_noalloc takes it from a fixed device array (for callers that cannot allocate).
#include "kf_internal.h"
#include "../../include/kfmeg.h"

#include <mutex>
#include <string>

using namespace kfmeg;

namespace {

// Workspace of the allocation-free entry point: one array per device, held until the process
// ends. Host code never passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in); it uses the device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct MneWork {
    double *G = nullptr, *S = nullptr, *Lis = nullptr, *U = nullptr, *V = nullptr, *part = nullptr;
    DevStatus* status = nullptr;
};

struct MneShape {
    int64_t ldm, ldT;
    int ksplit;
    size_t off[7];     // byte offsets of G, S, Lis, U, V, part, status (256-byte aligned)
    size_t total;
};

MneShape mne_shape(int64_t N, int64_t m, int64_t T) {
    MneShape sh;
    sh.ldm = round_up(m, 16);
    sh.ldT = round_up(T, 16);
    sh.ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(32, N / 128));
    const size_t bytes[7] = {8 * (size_t)N * sh.ldm, 8 * (size_t)m * sh.ldm, 8 * (size_t)m * sh.ldm,
                             8 * (size_t)m * sh.ldT, 8 * (size_t)m * sh.ldT,
                             8 * (size_t)sh.ksplit * m * m, sizeof(DevStatus)};
    size_t o = 0;
    for (int k = 0; k < 7; ++k) {
        sh.off[k] = o;
        o += (bytes[k] + 255) / 256 * 256;
    }
    sh.total = o;
    return sh;
}

MneWork carve(void* base, const MneShape& sh) {
    char* b = static_cast<char*>(base);
    MneWork w;
    w.G = reinterpret_cast<double*>(b + sh.off[0]);
    w.S = reinterpret_cast<double*>(b + sh.off[1]);
    w.Lis = reinterpret_cast<double*>(b + sh.off[2]);
    w.U = reinterpret_cast<double*>(b + sh.off[3]);
    w.V = reinterpret_cast<double*>(b + sh.off[4]);
    w.part = reinterpret_cast<double*>(b + sh.off[5]);
    w.status = reinterpret_cast<DevStatus*>(b + sh.off[6]);
    return w;
}

#define MCK(expr)                                                                   \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess) {                                                     \
            err = std::string(#expr) + ": " + hipGetErrorString(_e);                \
            return KF_EHIP;                                                         \
        }                                                                           \
    } while (0)

// eqn5 for every row of Y on `s` with workspace w, then wait for the stream and read the status.
kf_status mne_run(int64_t N, int64_t m, int64_t T, const double* X, const double* C, const double* R,
                  const double* Y, double* J, hipStream_t s, const MneShape& sh, const MneWork& w,
                  std::string& err) {
    MCK(status_clear(w.status, s));
    GemmProblem g;                       // G = C X^T   (N x m)
    g.M = (int)N; g.N = (int)m; g.K = (int)N;
    g.A = C; g.lda = N; g.B = X; g.ldb = N; g.flags = G_TB;
    g.C = w.G; g.ldc = sh.ldm;
    MCK(gemm1(Dt::F64, g, s));
    GemmProblem h;                       // S = X G + R
    h.M = (int)m; h.N = (int)m; h.K = (int)N;
    h.A = X; h.lda = N; h.B = w.G; h.ldb = sh.ldm;
    h.Cin = R; h.ldcin = m; h.beta = 1.0;
    h.C = w.S; h.ldc = sh.ldm;
    h.ksplit = sh.ksplit;
    h.partial = w.part;
    MCK(gemm1(Dt::F64, h, s));
    MCK(chol_inv(w.S, sh.ldm, w.Lis, sh.ldm, (int)m, w.status, W_MNE, 0, s));
    GemmProblem u;                       // U = Li Y^T   (m x T)
    u.M = (int)m; u.N = (int)T; u.K = (int)m;
    u.A = w.Lis; u.lda = sh.ldm; u.flags = G_ALOWER | G_TB;
    u.B = Y; u.ldb = m;
    u.C = w.U; u.ldc = sh.ldT;
    MCK(gemm1(Dt::F64, u, s));
    GemmProblem v;                       // V = Li^T U = S^{-1} Y^T
    v.M = (int)m; v.N = (int)T; v.K = (int)m;
    v.A = w.Lis; v.lda = sh.ldm; v.flags = G_TA;
    v.B = w.U; v.ldb = sh.ldT;
    v.C = w.V; v.ldc = sh.ldT;
    MCK(gemm1(Dt::F64, v, s));
    GemmProblem j;                       // J = V^T G^T   (T x N)
    j.M = (int)T; j.N = (int)N; j.K = (int)m;
    j.A = w.V; j.lda = sh.ldT; j.flags = G_TA | G_TB;
    j.B = w.G; j.ldb = sh.ldm;
    j.C = J; j.ldc = N;
    MCK(gemm1(Dt::F64, j, s));
    DevStatus hstat{};
    MCK(hipMemcpyAsync(&hstat, w.status, sizeof hstat, hipMemcpyDeviceToHost, s));
    MCK(hipStreamSynchronize(s));
    if (hstat.key != kStatusClear) {
        err = "mne_solve: X C X^T + R is not positive definite (pivot row " + std::to_string(status_row(hstat.key)) +
              ")";
        return KF_ENOTPD;
    }
    return KF_OK;
}

#undef MCK

bool args_ok(int64_t N, int64_t m, int64_t T, const void* X, const void* C, const void* R, const void* Y,
             const void* J) {
    return N > 0 && m > 0 && T > 0 && N <= (1 << 20) && m <= (1 << 16) && T <= (1 << 24) && X && C && R && Y && J;
}

}  // namespace

extern "C" {

kf_status mne_solve(int64_t N, int64_t m, int64_t T, const double* X, const double* C, const double* R,
                    const double* Y, double* J, void* stream) {
    set_last_error("");
    if (!args_ok(N, m, T, X, C, R, Y, J)) {
        set_last_error("mne_solve: sizes must be positive (N <= 2^20, m <= 2^16, T <= 2^24) and pointers non-null");
        return KF_EINVAL;
    }
    const MneShape sh = mne_shape(N, m, T);
    void* base = nullptr;
    if (hipMalloc(&base, sh.total) != hipSuccess) {
        (void)hipGetLastError();
        set_last_error("mne_solve: device allocation of " + std::to_string(sh.total) + " bytes failed");
        return KF_ENOMEM;
    }
    std::string err;
    const kf_status st = mne_run(N, m, T, X, C, R, Y, J, static_cast<hipStream_t>(stream), sh, carve(base, sh), err);
    if (st == KF_EHIP) (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    (void)hipFree(base);
    if (st != KF_OK) set_last_error(err);
    return st;
}

kf_status mne_solve_noalloc(int64_t N, int64_t m, int64_t T, const double* X, const double* C, const double* R,
                            const double* Y, double* J, void* stream) {
    set_last_error("");
    if (!args_ok(N, m, T, X, C, R, Y, J)) {
        set_last_error("mne_solve_noalloc: sizes must be positive (N <= 2^20, m <= 2^16, T <= 2^24) and "
                       "pointers non-null");
        return KF_EINVAL;
    }
    const MneShape sh = mne_shape(N, m, T);
    if (sh.total > kScratchBytes) {
        set_last_error("mne_solve_noalloc: this shape needs " + std::to_string(sh.total) +
                       " bytes of workspace; the fixed device array holds " + std::to_string(kScratchBytes));
        return KF_EINVAL;
    }
    void* base = nullptr;
    const hipError_t e = scratch_address(&base);
    if (e != hipSuccess) {
        set_last_error(std::string("mne_solve_noalloc: device address of the scratch array: ") + hipGetErrorString(e));
        return KF_EHIP;
    }
    std::string err;
    const kf_status st = mne_run(N, m, T, X, C, R, Y, J, static_cast<hipStream_t>(stream), sh, carve(base, sh), err);
    if (st == KF_EHIP) (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (st != KF_OK) set_last_error(err);
    return st;
}

}  // extern "C"
