/*
 * kfmeg.h -- C ABI of the MI355X (gfx950) Kalman filter / fixed-interval
 * smoother for the dynamic MEG inverse problem (Long, Purdon, Temereanca,
 * Desai, Hamalainen, Brown, Ann. Appl. Stat. 5(2B), 2011).
 *
 * Model (Section 2, eqn1 and eqn3 with F = I, the random walk):
 *     x_t = x_{t-1} + w_t,   w_t ~ N(0, Q)          (Sigma_w in the paper)
 *     y_t = X x_t + v_t,     v_t ~ N(0, R)          (H and Sigma_epsilon)
 * with x_0 ~ N(x0, P0). N is the state dimension (sources, or 3 x sites for
 * free orientation), m the number of sensors, T the number of time steps.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers to float64 data, row-major and
 *    contiguous (leading dimension = number of columns), unless stated.
 *  - The caller owns every buffer it passes; kf_create copies its inputs into
 *    plan-owned storage, so they may be freed after it returns. Y and output
 *    buffers must stay valid for the duration of the call.
 *  - Work is enqueued on the plan's stream (a hipStream_t passed as void*,
 *    NULL = the null stream) and every call synchronises that stream before it
 *    returns, so the returned status is final. A plan also owns streams of its
 *    own (the smoother's gain batches and the filter's N-sized work run on side
 *    streams; on a device with at least 128 compute units, the filter's m x m
 *    chain and its covariance downdates run on two streams restricted to
 *    disjoint sets of compute units); every call orders them after the plan's
 *    stream at its start and joins them back into it before it returns.
 *  - Argument errors are reported before any launch. Nothing throws or
 *    aborts across this boundary; kf_last_error() gives a message.
 *  - A plan is used by one host thread at a time; distinct plans may run
 *    concurrently on distinct streams.
 */
#ifndef KFMEG_H
#define KFMEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kf_plan kf_plan;

typedef enum {
    KF_OK = 0,
    KF_EINVAL = 1,   /* bad argument (shape, null pointer, non-finite data) */
    KF_ENOTPD = 2,   /* S or P_{t+1|t} not positive definite (step and matrix in the message) */
    KF_ENOMEM = 3,   /* device allocation failed or the HBM budget is too small */
    KF_EHIP = 4,     /* a HIP runtime call failed */
    KF_ESTATE = 5,   /* call out of order (kf_smooth before a completed kf_filter) */
    KF_ECANCELED = 6 /* serving: the job was cancelled before it started */
} kf_status;

typedef enum {
    KF_FP64 = 0,     /* every product and factorisation in float64 */
    KF_MIXED = 1     /* N x N products on FP32 MFMA (FP32 accumulate); Cholesky of S and of
                        P_{t+1|t}, the smoother gain and all epilogues in float64 */
} kf_precision;

typedef struct {
    int precision;            /* kf_precision */
    int store_fp32;           /* store the filtered covariances P_{t|t} in float32 */
    size_t hbm_budget_bytes;  /* cap on the covariance store; 0 = whatever is free */
    int checkpoint_stride;    /* keep every k-th P_{t|t} and recompute the rest in the
                                 backward pass; 0 = automatic (only if the store does not fit) */
    int keep_gain_factors;    /* keep the factors of each step's gain (C_t = L_t^-1 X P_{t|t-1},
                                 L_t^-1, L_t^-1 e_t) for kf_smooth_means: T_max (m N + m^2 + m)
                                 doubles more; 0 = off */
} kf_options;

/* Defaults: KF_FP64, float64 store, no budget cap, automatic checkpointing, no gain factors kept. */
void kf_default_options(kf_options* opt);

/*
 * kf_create: allocate a plan for state dimension N, m sensors and up to T_max
 * steps, and copy the model into it.
 *   X  (m x N) lead field, Q (N x N) and P0 (N x N) symmetric positive
 *   (semi)definite, R (m x m) symmetric positive definite, x0 (N).
 * The inputs define eqn1, eqn3 and the initial condition that follows eqn10
 * (x0 and P0 are inputs rather than the paper's MNE-based choice).
 * Returns KF_EINVAL for non-positive sizes or null pointers, KF_ENOMEM if the
 * workspaces do not fit. *out is NULL on failure.
 */
kf_status kf_create(kf_plan** out, int64_t N, int64_t m, int64_t T_max,
                    const double* X, const double* Q, const double* R,
                    const double* x0, const double* P0,
                    const kf_options* opt, void* stream);

/*
 * kf_filter: the Kalman filter, eqn6-eqn10 and the covariance update that
 * follows eqn10, for t = 1..T (1 <= T <= T_max), starting from x0, P0.
 *   Y          (T x m) data, row t-1 = y_t
 *   x_filt     (T x N) out: x_{t|t}
 *   Pdiag_filt (T x N) out, or NULL: diagonals of P_{t|t}
 * The filtered covariances stay in the plan for kf_smooth. Returns KF_ENOTPD
 * (with the step in kf_last_error) if S_t = X P_{t|t-1} X^T + R is not
 * positive definite, KF_EINVAL if Y holds a non-finite value.
 */
kf_status kf_filter(kf_plan* plan, int64_t T, const double* Y,
                    double* x_filt, double* Pdiag_filt);

/*
 * kf_smooth: the fixed-interval smoother eqn11-eqn13 (standard
 * Rauch-Tung-Striebel form; the printed eqn12/eqn13 carry misprints) for
 * t = T-1..1 from the last kf_filter call, initialised with x_{T|T}, P_{T|T}.
 *   x_smooth     (T x N) out: x_{t|T}
 *   Pdiag_smooth (T x N) out, or NULL: diagonals of P_{t|T}
 *   P_smooth     (T x N x N) out, or NULL: every P_{t|T} (small sizes only)
 * Returns KF_ESTATE without a completed kf_filter, KF_ENOTPD if
 * P_{t+1|t} = P_{t|t} + Q is not positive definite.
 */
kf_status kf_smooth(kf_plan* plan, double* x_smooth, double* Pdiag_smooth,
                    double* P_smooth);

/*
 * kf_filter_batch / kf_smooth_batch: the same filter and smoother for B >= 1
 * data sets that share the model (X, Q, R, x0, P0). The covariance recursion
 * (eqn7-eqn9 and the update after eqn10, and eqn11, eqn13 in the smoother)
 * does not involve the data, so it runs once and the B means advance together
 * as B-row matrix products.
 *   Y          (B x T x m) data, Y[b][t-1] = y_t of data set b
 *   x_filt     (B x T x N) out: x_{t|t} of each data set
 *   x_smooth   (B x T x N) out: x_{t|T} of each data set
 *   Pdiag_*, P_smooth as for kf_filter / kf_smooth (shared by all data sets)
 * kf_smooth_batch returns KF_ESTATE unless B equals the B of the last filter
 * call on the plan; kf_filter and kf_smooth are the B = 1 case. Not available
 * on plans owned by a serving context (KF_EINVAL). The plan allocates
 * 2 B (m + N) doubles of workspace on the first call with a larger B.
 */
kf_status kf_filter_batch(kf_plan* plan, int64_t B, int64_t T, const double* Y,
                          double* x_filt, double* Pdiag_filt);
kf_status kf_smooth_batch(kf_plan* plan, int64_t B, double* x_smooth,
                          double* Pdiag_smooth, double* P_smooth);

/*
 * kf_smooth_means / kf_smooth_means_batch: the smoothed means x_{t|T} alone,
 * without the smoother gain A_t of eqn11 and so without factorising any
 * N x N matrix. They equal the means of eqn12 (read as in kf_smooth) in exact
 * arithmetic, through the backward information recursion (modified
 * Bryson-Frazier form): with lambda_{T+1} = 0, for t = T..1,
 *   x_{t|T}  = x_{t|t} + P_{t|t} lambda_{t+1}
 *   lambda_t = lambda_{t+1} + X^T L_t^-T (L_t^-1 e_t - C_t lambda_{t+1})
 * where S_t = L_t L_t^T (eqn8), e_t the innovation of eqn10 and
 * C_t = L_t^-1 X P_{t|t-1}. Per step this is one N x N matrix-vector product
 * and O(m N) work instead of O(N^3).
 *   x_smooth (T x N), or (B x T x N) for the batch form with the B of the
 *            last filter call.
 * Needs a plan created with keep_gain_factors (KF_ESTATE otherwise, or without
 * a completed filter call). Diagonals of P_{t|T} are not produced.
 */
kf_status kf_smooth_means(kf_plan* plan, double* x_smooth);
kf_status kf_smooth_means_batch(kf_plan* plan, int64_t B, double* x_smooth);

/*
 * kf_smooth_assoc: the same smoothed means and covariances as kf_smooth
 * (eqn11-eqn13, RTS reading), computed as a suffix scan over time with an
 * associative operator instead of the step-by-step back-recursion. Step t < T
 * contributes the element (A_t, x_{t|t} - A_t F x_{t|t}, P_{t|t} - A_t F P_{t|t})
 * with the gain A_t of eqn11, step T the element (0, x_{T|T}, P_{T|T}); the
 * operator is (E, g, L) o (E', g', L') = (E E', E g' + g, E L' E^T + L), and the
 * product of the elements from t to T is (0, x_{t|T}, P_{t|T}). The scan runs in
 * blocks of about sqrt(T) steps, so its depth is about 3 sqrt(T) groups of
 * independent products instead of T dependent steps, at about twice the
 * products of kf_smooth. On one GPU kf_smooth, which already overlaps its
 * independent gain work with the back-recursion, is the faster of the two;
 * the scan's blocks are independent units of work for several devices.
 *   x_smooth, Pdiag_smooth, P_smooth as for kf_smooth.
 * Needs a float64 plan (KF_EINVAL for mixed precision or a serving plan) whose
 * last kf_filter call ran one data set and stored every P_{t|t} in float64 (no
 * float32 store, no checkpointing; KF_ESTATE otherwise). Allocates T + 23
 * float64 N x N matrices (rows padded to 16 elements) for the call,
 * kf_smooth_assoc_bytes(N, T) bytes (KF_ENOMEM if that fails), and
 * overwrites the stored P_{t|t}: afterwards the plan needs a new kf_filter
 * call before any smoother call or kf_get_filtered_cov. KF_ENOTPD as for
 * kf_smooth.
 */
kf_status kf_smooth_assoc(kf_plan* plan, double* x_smooth, double* Pdiag_smooth,
                          double* P_smooth);

/*
 * Device bytes kf_smooth_assoc allocates for one call on a plan of N sources after a
 * kf_filter call over T steps (on top of the plan's own kf_plan_bytes), so that a
 * caller can budget them; 0 for N <= 0 or T <= 0. Host arithmetic only.
 */
size_t kf_smooth_assoc_bytes(int64_t N, int64_t T);

/*
 * kf_set_transition: use x_t = F x_{t-1} + w_t (eqn3) instead of the random
 * walk, with F (N x N) sparse in CSR form: row_ptr (N+1 int32, from 0 to nnz),
 * col_idx (nnz int32, in [0, N)), val (nnz float64), all device pointers, copied
 * into the plan (the caller may free them afterwards). The six-neighbour model
 * of eqn2 is such an F with seven entries per row. The filter then predicts
 * x_{t|t-1} = F x_{t-1|t-1}, P_{t|t-1} = F P_{t-1|t-1} F^T + Q (eqn6, eqn7),
 * and the smoother uses A_t = P_{t|t} F^T P_{t+1|t}^-1 (eqn11) and
 * x_{t+1|t} = F x_{t|t} in eqn12; kf_smooth_means applies F^T to lambda.
 * nnz = 0 with null pointers restores F = I. Adds 2 N^2 float64 of workspace;
 * invalidates the last filter call. Not available on serving plans. Returns
 * KF_EINVAL for a malformed matrix.
 */
kf_status kf_set_transition(kf_plan* plan, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* val);

/* Copy the stored filtered covariance P_{t|t} (1 <= t <= T) into P_out (N x N, device). */
kf_status kf_get_filtered_cov(kf_plan* plan, int64_t t, double* P_out);

/*
 * mne_solve: the minimum-norm estimate of eqn5 for every column of the data,
 *   J_t = C X^T (X C X^T + R)^{-1} y_t,   t = 1..T,
 * with C (N x N) the symmetric positive definite source prior (lambda R in
 * eqn5; any SPD matrix is accepted), R (m x m) the sensor noise covariance.
 *   Y (T x m) in, J (T x N) out.
 * Stateless: allocates its own workspace, synchronises `stream` before it
 * returns. KF_ENOTPD if X C X^T + R is not positive definite.
 */
kf_status mne_solve(int64_t N, int64_t m, int64_t T, const double* X, const double* C,
                    const double* R, const double* Y, double* J, void* stream);

/*
 * mne_solve_noalloc: mne_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, launches and results (bit for bit) as mne_solve,
 * but its workspace comes from one fixed 64 MiB device array of the library
 * (one per GPU, held until the process ends) instead of an allocation: it calls
 * no hipMalloc, hipFree or other allocating routine. The workspace of a call is
 * 8 (N ldm + 2 m ldm + 2 m ldT + k m^2) bytes plus a 16-byte status record, each
 * part rounded up to 256 bytes, with ldm = m and ldT = T rounded up to
 * multiples of 16 and k = min(32, max(1, N / 128)); a shape that needs more than
 * 64 MiB returns KF_EINVAL before any launch (N = 5124, m = 306 fits up to
 * T of about 5800). The array keeps the last call's contents; everything a call
 * reads from it is written first by that call. Calls on one GPU share the array:
 * calls that overlap in time on the same GPU (on different streams or threads)
 * race and must be serialised by the caller. Synchronises `stream` before it
 * returns; KF_ENOTPD if X C X^T + R is not positive definite, KF_EHIP if the
 * array's device address cannot be obtained.
 */
kf_status mne_solve_noalloc(int64_t N, int64_t m, int64_t T, const double* X, const double* C,
                            const double* R, const double* Y, double* J, void* stream);

/*
 * kf_init_from_mne: the parameter set-up of Section 2.4. Computes the MNE
 * estimates J_t (eqn5, prior covariance C) for every row of Y (T x m, T >= 3),
 * returns x0_out = J_1 (the estimate of the first sample) and
 *   Q_out = sample covariance of the differences J_t - J_{t-1}, t = 2..T
 *           (divisor T - 2) + reg * I,
 * an estimate of Sigma_w of rank at most T - 2 before the regulariser.
 * x0_out (N) and Q_out (N x N, exactly symmetric) are device buffers the
 * caller owns. Synchronises `stream` before it returns.
 */
kf_status kf_init_from_mne(int64_t N, int64_t m, int64_t T, const double* X, const double* C,
                           const double* R, const double* Y, double reg, double* x0_out,
                           double* Q_out, void* stream);

/* Free a plan and everything it owns. NULL is accepted. */
void kf_destroy(kf_plan* plan);

/* Message for the last failed call on this plan (or of mne_solve if plan is NULL). */
const char* kf_last_error(const kf_plan* plan);

/*
 * Profiling of the smoother's N x N x N products (the triangular products
 * that form A_t, eqn11, and the two products of eqn13), which carry most of
 * the arithmetic. With profiling on (on = 1), kf_smooth brackets each such
 * launch with a pair of HIP events on the stream it runs on, the closing one
 * recorded right after the product kernel (before any split reduction), so an
 * event pair spans one dispatch; kf_get_profile returns the summed event time
 * in ms, the summed algorithmic flops (N^3 for each triangular or half-output
 * product, 2 N^3 for the full one) and the number of launches since profiling
 * was last switched on. on = 2 also serialises the smoother onto the plan's
 * stream (the gain batches no longer overlap the back-recursion), so that each
 * product runs alone; its float64 products then run as a separately named
 * kernel instantiation. on = 0 switches both off. kf_set_profiling resets the
 * totals; KF_EINVAL for other values of on.
 */
kf_status kf_set_profiling(kf_plan* plan, int on);
kf_status kf_get_profile(const kf_plan* plan, double* kernel_ms, double* kernel_flops, int64_t* launches);

/*
 * Device bytes a plan of this shape would allocate with one batch of smoother
 * gains in flight: workspaces plus the full covariance store for T steps under
 * `opt` (serving plans are sized this way; a plan made by kf_create also forms
 * a second gain batch on another stream when the HBM budget leaves room for
 * its 3 gb or more extra N x N workspaces, gb <= 8 the gain-batch width).
 */
size_t kf_plan_bytes(int64_t N, int64_t m, int64_t T, const kf_options* opt);

/*
 * Serving: continuous batching of filter + smoother jobs (kf_filter then
 * kf_smooth) of different N, m and T on one GPU.
 *
 * kfs_create reserves one device arena of hbm_budget_bytes (0 = free HBM less
 * 4 GiB) and starts max_active worker slots, each with its own stream. Jobs are
 * taken in arrival order; a job starts as soon as a slot is free and its plan
 * (workspaces, covariance store, filtered means; kf_plan_bytes) fits in the
 * arena next to the running jobs. If the full store of P_{t|t} does not fit, the
 * job starts with the smallest checkpoint stride that fits instead of waiting.
 * Running jobs' kernels overlap on the device; a job's results do not depend on
 * the other jobs. `opt` sets the precision and store type of every job.
 *
 * kfs_submit enqueues a job and returns at once. All array arguments are device
 * pointers as in kf_create / kf_smooth and must stay valid until kfs_wait for
 * that job returns. x_smooth (T x N) and Pdiag_smooth (T x N, or NULL) receive
 * x_{t|T} and diag P_{t|T}. `stream` (a hipStream_t, NULL = the null stream) is the
 * stream the caller wrote the inputs on: the job's work starts only after everything
 * enqueued on it before the call has finished, so inputs produced by asynchronous GPU
 * work are safe to pass. The outputs are complete when kfs_wait returns; KF_EHIP if
 * the ordering event cannot be recorded.
 * kfs_wait blocks until the job is done and returns its status (KF_ENOTPD,
 * KF_ENOMEM if it can never fit the budget, ...); latency_ms = completion minus
 * submission.
 * kfs_cancel removes a job that has not started yet: its kfs_wait returns
 * KF_ECANCELED and its buffers are free at once. A job that is running or done
 * is not interrupted (KF_ESTATE); KF_EINVAL for an unknown id.
 * kfs_get_stats: latency percentiles over completed jobs, throughput over the
 * span from the first submission to the last completion, peak arena use (never
 * above the budget) and the most jobs that ran at once.
 * kfs_destroy waits for queued and running jobs, then frees everything.
 */
typedef struct kfs_server kfs_server;
typedef struct {
    double p50_ms, p99_ms, mean_ms, max_ms;
    double jobs_per_s, steps_per_s;
    int64_t submitted, completed, failed, checkpointed;
    size_t peak_bytes, budget_bytes;
    int max_concurrent;
    int64_t canceled;
} kfs_stats;

kf_status kfs_create(kfs_server** out, size_t hbm_budget_bytes, int max_active, const kf_options* opt);
kf_status kfs_submit(kfs_server* srv, int64_t N, int64_t m, int64_t T, const double* X, const double* Q,
                     const double* R, const double* x0, const double* P0, const double* Y,
                     double* x_smooth, double* Pdiag_smooth, void* stream, int64_t* job_id);
kf_status kfs_wait(kfs_server* srv, int64_t job_id, double* latency_ms);
kf_status kfs_cancel(kfs_server* srv, int64_t job_id);
kf_status kfs_job_info(kfs_server* srv, int64_t job_id, int* done, int* checkpoint_stride,
                       double* queued_ms, double* run_ms);
kf_status kfs_get_stats(kfs_server* srv, kfs_stats* out);
const char* kfs_last_error(kfs_server* srv);
void kfs_destroy(kfs_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* KFMEG_H */
