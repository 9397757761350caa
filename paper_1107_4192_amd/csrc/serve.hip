// Serving loop: continuous batching of filter + smoother jobs on one GPU.
//
// Jobs queue in arrival order. A job is admitted as soon as a slot and HBM for its
// plan free up: the plan's buffers (workspaces, covariance store, filtered means)
// come from one device arena sized to the HBM budget, and admission reserves the
// plan's byte count. When the full store of P_{t|t} does not fit next to the jobs
// already running, the job is admitted with the smallest checkpoint stride that
// fits (filtered covariances recomputed between checkpoints in the backward pass)
// rather than waiting. Each slot is a worker thread with its own HIP stream, so
// the kernels of all admitted jobs overlap on the device; every job's arithmetic
// is independent of the others (own buffers, deterministic kernels), so a job
// gives the same result alone and in the mix.
#include "kf_internal.h"
#include "arena.h"
#include "../../include/kfmeg.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace kfmeg {
kf_status create_plan(kf_plan** out, int64_t N, int64_t m, int64_t T_max, const double* X, const double* Q,
                      const double* R, const double* x0, const double* P0, const kf_options* opt, void* stream,
                      DeviceArena* arena);
size_t plan_bytes_ex(int64_t N, int64_t m, int64_t T, const kf_options* opt, int gb);
}

using namespace kfmeg;
using Clock = std::chrono::steady_clock;

namespace {

struct Job {
    int64_t id = 0, N = 0, m = 0, T = 0;
    const double *X = nullptr, *Q = nullptr, *R = nullptr, *x0 = nullptr, *P0 = nullptr, *Y = nullptr;
    double *xs = nullptr, *dPs = nullptr;
    Clock::time_point arrival, start, end;
    bool done = false;
    kf_status status = KF_OK;
    std::string err;
    int stride = 1;
    size_t reserved = 0;
    hipEvent_t ready = nullptr;   // recorded on the submitter's stream: inputs are written
    ~Job() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

constexpr size_t kSlack = (size_t)64 << 10;   // arena alignment of ~60 buffers per plan

// Bytes a job takes in the arena: its plan (checkpoint stride, gain-batch width) plus
// its filtered means.
size_t job_bytes(const Job& j, const kf_options& o, int stride, int gb) {
    kf_options q = o;
    q.checkpoint_stride = stride;
    return plan_bytes_ex(j.N, j.m, j.T, &q, gb) + (size_t)j.T * j.N * sizeof(double) + kSlack;
}

// Smallest footprint over all checkpoint strides (the job fits an empty device iff this does).
size_t min_job_bytes(const Job& j, const kf_options& o) {
    size_t best = job_bytes(j, o, 1, 1);
    for (int s = 2; s <= j.T; ++s) best = std::min(best, job_bytes(j, o, s, 1));
    return best;
}

// The same order of preference as plan creation: full store before checkpoints, and
// within a stride the widest gain batch that fits.
bool fit(const Job& j, const kf_options& o, size_t room, int* stride, size_t* bytes) {
    for (int s = 1; s <= j.T; ++s) {
        for (int gb = kMaxBatch; gb >= 1; gb /= 2) {
            const size_t b = job_bytes(j, o, s, gb);
            if (b <= room) {
                *stride = s;
                *bytes = b;
                return true;
            }
        }
    }
    return false;
}

}  // namespace

struct kfs_server {
    DeviceArena arena;
    size_t budget = 0;
    int max_active = 1;
    kf_options opt{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job*> queue;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::vector<std::thread> workers;
    bool stop = false;
    int64_t next_id = 1;
    size_t reserved = 0;
    int active = 0, max_conc = 0;
    int64_t completed = 0, failed = 0, checkpointed = 0, canceled = 0, retry_after = -1;
    std::vector<double> latencies;
    int64_t steps_done = 0;
    Clock::time_point first_arrival, last_end;
    bool any = false;
    std::string err;

    // Decide whether the head job can start now (with which checkpoint stride and footprint).
    bool admissible(int* stride, size_t* bytes) {
        if (queue.empty()) return false;
        if (retry_after >= 0 && completed + failed <= retry_after) return false;
        if (active >= max_active) return false;
        return fit(*queue.front(), opt, budget - reserved, stride, bytes);
    }

    void finish(Job* j, kf_status st, const std::string& msg) {
        std::lock_guard<std::mutex> lk(mu);
        reserved -= j->reserved;
        --active;
        j->status = st;
        j->err = msg;
        j->end = Clock::now();
        j->done = true;
        if (st == KF_OK) {
            ++completed;
            latencies.push_back(std::chrono::duration<double, std::milli>(j->end - j->arrival).count());
            steps_done += j->T;
            last_end = j->end;
        } else {
            ++failed;
        }
        cv.notify_all();
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
        for (;;) {
            Job* j = nullptr;
            int stride = 1;
            size_t bytes = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    if (stop && queue.empty()) return true;
                    if (admissible(&stride, &bytes)) return true;
                    // nothing running and the head can never fit: fail it
                    if (!queue.empty() && active == 0 && min_job_bytes(*queue.front(), opt) > budget) return true;
                    return false;
                });
                if (queue.empty()) {
                    if (stop) break;
                    continue;
                }
                j = queue.front();
                if (!admissible(&stride, &bytes)) {  // the never-fits case
                    queue.pop_front();
                    j->done = true;
                    j->status = KF_ENOMEM;
                    j->err = "job does not fit the serving HBM budget even with checkpointing";
                    j->end = Clock::now();
                    ++failed;
                    cv.notify_all();
                    continue;
                }
                queue.pop_front();
                j->stride = stride;
                j->reserved = bytes;
                reserved += j->reserved;
                ++active;
                max_conc = std::max(max_conc, active);
                if (stride > 1) ++checkpointed;
                j->start = Clock::now();
            }
            kf_options o = opt;
            o.checkpoint_stride = stride;
            o.hbm_budget_bytes = j->reserved;
            // The job's inputs may still be being produced on the submitter's stream.
            if (j->ready && st) (void)hipStreamWaitEvent(st, j->ready, 0);
            double* xf = static_cast<double*>(arena.alloc((size_t)j->T * j->N * sizeof(double)));
            kf_plan* plan = nullptr;
            kf_status s = xf ? create_plan(&plan, j->N, j->m, j->T, j->X, j->Q, j->R, j->x0, j->P0, &o, st, &arena)
                             : KF_ENOMEM;
            if (s == KF_ENOMEM) {
                // the arena is too fragmented for now: retry after the next completion
                if (xf) arena.release(xf);
                std::lock_guard<std::mutex> lk(mu);
                reserved -= j->reserved;
                --active;
                if (stride > 1) --checkpointed;
                if (active > 0) {
                    queue.push_front(j);
                    retry_after = completed + failed;
                    cv.notify_all();
                    continue;
                }
                j->done = true;
                j->status = KF_ENOMEM;
                j->err = "device arena exhausted";
                j->end = Clock::now();
                ++failed;
                cv.notify_all();
                continue;
            }
            std::string msg;
            if (s == KF_OK) s = kf_filter(plan, j->T, j->Y, xf, nullptr);
            if (s == KF_OK) s = kf_smooth(plan, j->xs, j->dPs, nullptr);
            if (s != KF_OK) msg = plan ? kf_last_error(plan) : kf_last_error(nullptr);
            kf_destroy(plan);
            arena.release(xf);
            finish(j, s, msg);
        }
        if (st) (void)hipStreamDestroy(st);
    }
};

extern "C" {

kf_status kfs_create(kfs_server** out, size_t hbm_budget_bytes, int max_active, const kf_options* opt) {
    if (!out || max_active < 1 || max_active > 64) return KF_EINVAL;
    *out = nullptr;
    auto* s = new kfs_server();
    kf_default_options(&s->opt);
    if (opt) s->opt = *opt;
    s->opt.checkpoint_stride = 0;
    s->opt.hbm_budget_bytes = 0;
    s->opt.keep_gain_factors = 0;        // jobs run the full smoother
    (void)hipGetDevice(&s->device);
    size_t budget = hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return KF_EHIP;
        }
        budget = fr > ((size_t)4 << 30) ? fr - ((size_t)4 << 30) : fr / 2;
    }
    if (s->arena.init(budget) != hipSuccess) {
        delete s;
        return KF_ENOMEM;
    }
    s->budget = s->arena.capacity();
    s->max_active = max_active;
    for (int i = 0; i < max_active; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return KF_OK;
}

kf_status kfs_submit(kfs_server* s, int64_t N, int64_t m, int64_t T, const double* X, const double* Q,
                     const double* R, const double* x0, const double* P0, const double* Y, double* x_smooth,
                     double* Pdiag_smooth, void* stream, int64_t* job_id) {
    if (!s || N <= 0 || m <= 0 || T <= 0 || !X || !Q || !R || !x0 || !P0 || !Y || !x_smooth) return KF_EINVAL;
    auto j = std::make_unique<Job>();
    // Order the job after the work already enqueued on the submitter's stream.
    if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(j->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
        if (j->ready) (void)hipEventDestroy(j->ready);
        (void)hipGetLastError();
        return KF_EHIP;
    }
    j->N = N; j->m = m; j->T = T;
    j->X = X; j->Q = Q; j->R = R; j->x0 = x0; j->P0 = P0; j->Y = Y;
    j->xs = x_smooth; j->dPs = Pdiag_smooth;
    j->arrival = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->next_id++;
    if (!s->any) {
        s->first_arrival = j->arrival;
        s->any = true;
    }
    if (job_id) *job_id = j->id;
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
    s->cv.notify_all();
    return KF_OK;
}

kf_status kfs_wait(kfs_server* s, int64_t job_id, double* latency_ms) {
    if (!s) return KF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return KF_EINVAL;
    Job* j = it->second.get();
    s->cv.wait(lk, [&] { return j->done; });
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(j->end - j->arrival).count();
    if (j->status != KF_OK) s->err = j->err;
    return j->status;
}

kf_status kfs_cancel(kfs_server* s, int64_t job_id) {
    if (!s) return KF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return KF_EINVAL;
    Job* j = it->second.get();
    auto q = std::find(s->queue.begin(), s->queue.end(), j);
    if (q == s->queue.end()) return KF_ESTATE;     // running or finished
    s->queue.erase(q);
    j->done = true;
    j->status = KF_ECANCELED;
    j->err = "job cancelled before it started";
    j->end = Clock::now();
    ++s->canceled;
    s->cv.notify_all();
    return KF_OK;
}

kf_status kfs_job_info(kfs_server* s, int64_t job_id, int* done, int* checkpoint_stride, double* queued_ms,
                       double* run_ms) {
    if (!s) return KF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return KF_EINVAL;
    const Job& j = *it->second;
    if (done) *done = j.done ? 1 : 0;
    if (checkpoint_stride) *checkpoint_stride = j.stride;
    using ms = std::chrono::duration<double, std::milli>;
    if (queued_ms) *queued_ms = j.done ? ms(j.start - j.arrival).count() : 0.0;
    if (run_ms) *run_ms = j.done ? ms(j.end - j.start).count() : 0.0;
    return KF_OK;
}

kf_status kfs_get_stats(kfs_server* s, kfs_stats* out) {
    if (!s || !out) return KF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (double)(l.size() - 1);
        const size_t lo = (size_t)pos, hi = std::min(lo + 1, l.size() - 1);
        return l[lo] + (pos - (double)lo) * (l[hi] - l[lo]);
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0.0;
    for (double v : l) sum += v;
    out->mean_ms = l.empty() ? 0.0 : sum / (double)l.size();
    out->max_ms = l.empty() ? 0.0 : l.back();
    const double span = s->any && s->completed ? std::chrono::duration<double>(s->last_end - s->first_arrival).count()
                                               : 0.0;
    out->jobs_per_s = span > 0 ? (double)s->completed / span : 0.0;
    out->steps_per_s = span > 0 ? (double)s->steps_done / span : 0.0;
    out->submitted = (int64_t)s->jobs.size();
    out->completed = s->completed;
    out->failed = s->failed;
    out->checkpointed = s->checkpointed;
    out->peak_bytes = s->arena.peak();
    out->budget_bytes = s->budget;
    out->max_concurrent = s->max_conc;
    out->canceled = s->canceled;
    return KF_OK;
}

const char* kfs_last_error(kfs_server* s) { return s ? s->err.c_str() : ""; }

void kfs_destroy(kfs_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    for (auto& t : s->workers) t.join();
    delete s;
}

}  // extern "C"
