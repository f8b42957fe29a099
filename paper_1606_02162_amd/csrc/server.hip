// Layout server: continuous batching of layout jobs on one GPU.
//
// Jobs (host graph, k, parameters, initial positions) are queued by
// gila_submit.  Five threads own the device work, each on streams of its own:
//   admitter  admits queued jobs in arrival order as slots and the HBM budget
//             allow (footprint bound from the graph).  Jobs small enough for
//             the LDS-resident batch kernel go to the small-job worker, larger
//             ones to the builder.
//   small     two workers: each lays out the small jobs waiting when it wakes
//             together in one batched launch, on a stream of its own.
//   builder   uploads a large job's graph and builds its k-hop lists on its
//             build stream, then hands the job to the ticker.
//   ticker    advances every resident large job by `tick_iterations`
//             iterations per tick on the compute streams -- a replay of the
//             job's captured tick graph, whose caps are read from the device
//             copy of its schedule -- copies each job's control block to a
//             pinned host slot, waits for the tick, and retires jobs that
//             finished (all iterations, or the halting rule).  Builds and
//             batched launches overlap with the ticks.
// A job's arithmetic depends only on its own graph and parameters (the
// iteration plan is per graph; ticks split a run without changing its bits),
// so each result is the same alone and in any mix of concurrent jobs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "gila_internal.h"
#include "host_logic.h"

namespace gila {

enum JobState { kPending = 0, kResident = 1, kDone = 2, kFailed = 3, kCanceled = 4 };

struct Job {
    uint64_t id = 0;
    int32_t k = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    gila_params params{};
    std::vector<double> temps;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> init;
    std::vector<double> result;
    int state = kPending;
    int status = GILA_OK;
    std::atomic<bool> cancel{false};
    bool small = false;
    int64_t footprint = 0;
    // device state of a resident job
    int64_t* d_rp = nullptr;
    int32_t* d_ci = nullptr;
    void* d_pos = nullptr;
    gila_khop* kh = nullptr;
    int32_t h = 0;
    int32_t h_target = 0;
    int lane = 0;  // which compute stream the job's ticks run on
    int32_t slot = -1;  // its pinned host control-block slot (and event) while resident
    bool in_tick = false;  // a tick is queued and its event not yet seen
    char msg[256] = {0};  // why it failed (the failing thread's last error)
    gila_stats stats{};
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Bytes a job may hold on the device (host_logic.h: walk-count bound of P).
static int64_t footprint_bytes(const Job& j) {
    return host::footprint_bytes(j.n, j.nnz, j.k, j.rp.data(), j.ci.data());
}

}  // namespace gila

struct gila_server {
    int device = 0;
    gila::host::AdmitState adm;        // budget, slots, bytes reserved, jobs in flight
    int32_t tick_iters = 50;
    int32_t small_max_n = 1024;      // 0 = the most that fits the batch kernel's LDS
    std::atomic<uint64_t> fail_alloc_ticket{0};  // test hook: this job's allocation fails
    std::mutex mu;
    std::condition_variable cv;        // wakes the admitter
    std::condition_variable cv_small;  // wakes the small-job worker
    std::condition_variable cv_build;  // wakes the builder
    std::condition_variable cv_tick;   // wakes the ticker
    std::condition_variable cv_done;   // wakes waiters
    std::deque<uint64_t> pending;
    std::map<uint64_t, gila::Job*> jobs;
    std::map<uint64_t, std::pair<double, double>> times;  // queued ms, total ms
    std::vector<gila::Job*> small_queue;  // admitted small jobs
    std::deque<gila::Job*> build_queue;   // admitted large jobs, not yet built
    std::vector<gila::Job*> ready;        // built large jobs, not yet ticked
    std::vector<gila::Job*> resident;     // large jobs owned by the ticker
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th_admit, th_build, th_tick;
    static constexpr int kSmallWorkers = 2;
    std::thread th_small[kSmallWorkers];
    static constexpr int kComputeStreams = 3;
    hipStream_t compute[kComputeStreams] = {nullptr, nullptr, nullptr};
    hipStream_t build = nullptr;
    hipStream_t small[kSmallWorkers] = {nullptr, nullptr};
    gila::Ctl* host_ctl = nullptr;      // pinned, [max_slots]: resident jobs' control blocks
    std::vector<hipEvent_t> slot_ev;    // [max_slots]: end of each resident job's tick
    std::vector<int32_t> free_slots;
    hipStream_t download = nullptr;     // final positions of large jobs
    int64_t jobs_done = 0, ticks = 0;
    int32_t peak_resident = 0;
};

namespace gila {

// Releases a job's device memory into the library's cache once the work on
// `st` (the last stream that used it) is done: no device-wide synchronisation.
static void release_device(Job* j, hipStream_t st) {
    const Release rel{true, st};
    if (j->kh) free_khop(j->kh, rel);
    rel(j->d_rp);
    rel(j->d_ci);
    rel(j->d_pos);
    j->kh = nullptr;
    j->d_rp = nullptr;
    j->d_ci = nullptr;
    j->d_pos = nullptr;
}

// Scheduler-side completion (mutex held by the caller).
static void finish_job(gila_server* s, Job* j, int state, int status) {
    j->state = state;
    j->status = status;
    if (state == kFailed) std::snprintf(j->msg, sizeof(j->msg), "%s", gila_last_error());
    j->t_done = now_s();
    host::admit_release(s->adm, j->footprint);
    if (state == kDone) s->jobs_done += 1;
    s->times[j->id] = {(j->t_admit - j->t_submit) * 1e3, (j->t_done - j->t_submit) * 1e3};
    s->cv_done.notify_all();
    s->cv.notify_one();  // slots and budget were released
}

static int upload_job(gila_server* s, Job* j, hipStream_t st) {
    if (s->fail_alloc_ticket == j->id) return fail(GILA_ENOMEM, "injected allocation failure");
    const size_t pb = j->params.precision == GILA_FP64 ? 16 : 8;
    GILA_TRY(dalloc_t(&j->d_rp, (size_t)j->n + 1));
    GILA_TRY(dalloc_t(&j->d_ci, (size_t)std::max<int64_t>(j->nnz, 1)));
    GILA_TRY(dalloc(&j->d_pos, (size_t)std::max(j->n, 1) * pb));
    GILA_HIP(hipMemcpyAsync(j->d_rp, j->rp.data(), sizeof(int64_t) * (j->n + 1),
                            hipMemcpyHostToDevice, st));
    if (j->nnz > 0)
        GILA_HIP(hipMemcpyAsync(j->d_ci, j->ci.data(), sizeof(int32_t) * j->nnz,
                                hipMemcpyHostToDevice, st));
    if (pb == 16) {
        GILA_HIP(hipMemcpyAsync(j->d_pos, j->init.data(), sizeof(double) * 2 * j->n,
                                hipMemcpyHostToDevice, st));
    } else {
        std::vector<float> f((size_t)2 * j->n);
        for (size_t i = 0; i < f.size(); ++i) f[i] = (float)j->init[i];
        GILA_HIP(hipMemcpyAsync(j->d_pos, f.data(), sizeof(float) * f.size(),
                                hipMemcpyHostToDevice, st));
        GILA_HIP(hipStreamSynchronize(st));  // f leaves scope
    }
    return GILA_OK;
}

static int download_positions(Job* j, hipStream_t st) {
    j->result.assign((size_t)2 * j->n, 0.0);
    if (j->n == 0) return GILA_OK;
    if (j->params.precision == GILA_FP64) {
        GILA_HIP(hipMemcpyAsync(j->result.data(), j->d_pos, sizeof(double) * 2 * j->n,
                                hipMemcpyDeviceToHost, st));
        GILA_HIP(hipStreamSynchronize(st));
    } else {
        std::vector<float> f((size_t)2 * j->n);
        GILA_HIP(hipMemcpyAsync(f.data(), j->d_pos, sizeof(float) * f.size(),
                                hipMemcpyDeviceToHost, st));
        GILA_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < f.size(); ++i) j->result[i] = f[i];
    }
    return GILA_OK;
}

// Lays out a group of small jobs of one precision in one batched launch.
// The group's graphs and positions travel in one device allocation and one
// copy each way.
static void run_small_group(gila_server* s, std::vector<Job*>& group, hipStream_t sst) {
    std::vector<Job*> ok;
    for (Job* j : group) {
        if (s->fail_alloc_ticket == j->id) {
            std::lock_guard<std::mutex> lk(s->mu);
            finish_job(s, j, kFailed, fail(GILA_ENOMEM, "injected allocation failure"));
            continue;
        }
        ok.push_back(j);
    }
    if (ok.empty()) return;
    const bool fp64 = ok[0]->params.precision == GILA_FP64;
    const size_t pb = fp64 ? 16 : 8;
    // offsets of each job's arrays in the staging buffers
    std::vector<size_t> orp(ok.size()), oci(ok.size()), opos(ok.size());
    size_t nrp = 0, nci = 0, npos = 0;
    for (size_t i = 0; i < ok.size(); ++i) {
        orp[i] = nrp;
        oci[i] = nci;
        opos[i] = npos;
        nrp += (size_t)ok[i]->n + 1;
        nci += (size_t)ok[i]->nnz;
        npos += (size_t)ok[i]->n;
    }
    std::vector<int64_t> h_rp(nrp);
    std::vector<int32_t> h_ci(std::max<size_t>(nci, 1));
    std::vector<unsigned char> h_pos(std::max<size_t>(npos, 1) * pb);
    for (size_t i = 0; i < ok.size(); ++i) {
        const Job* j = ok[i];
        std::copy(j->rp.begin(), j->rp.begin() + j->n + 1, h_rp.begin() + orp[i]);
        std::copy(j->ci.begin(), j->ci.end(), h_ci.begin() + oci[i]);
        if (fp64) {
            std::memcpy(h_pos.data() + opos[i] * pb, j->init.data(), sizeof(double) * 2 * j->n);
        } else {
            float* f = reinterpret_cast<float*>(h_pos.data() + opos[i] * pb);
            for (size_t e = 0; e < (size_t)2 * j->n; ++e) f[e] = (float)j->init[e];
        }
    }
    const size_t brp = (nrp * 8 + 255) & ~(size_t)255, bci = (nci * 4 + 255) & ~(size_t)255;
    const size_t bytes = brp + bci + std::max<size_t>(npos, 1) * pb;
    void* arena = nullptr;
    int rc = dalloc(&arena, bytes);
    char* base = static_cast<char*>(arena);
    if (rc == GILA_OK && hipMemcpyAsync(base, h_rp.data(), nrp * 8, hipMemcpyHostToDevice,
                                        sst) != hipSuccess)
        rc = fail(GILA_EDEVICE, "upload");
    if (rc == GILA_OK && nci > 0 &&
        hipMemcpyAsync(base + brp, h_ci.data(), nci * 4, hipMemcpyHostToDevice, sst) !=
            hipSuccess)
        rc = fail(GILA_EDEVICE, "upload");
    if (rc == GILA_OK && npos > 0 &&
        hipMemcpyAsync(base + brp + bci, h_pos.data(), npos * pb, hipMemcpyHostToDevice,
                       sst) != hipSuccess)
        rc = fail(GILA_EDEVICE, "upload");
    std::vector<gila_csr> csr(ok.size());
    std::vector<int32_t> ks(ok.size());
    std::vector<gila_params> ps(ok.size());
    std::vector<void*> pos(ok.size());
    for (size_t i = 0; i < ok.size(); ++i) {
        const Job* j = ok[i];
        csr[i] = gila_csr{j->n, j->nnz, reinterpret_cast<const int64_t*>(base) + orp[i],
                          reinterpret_cast<const int32_t*>(base + brp) + oci[i]};
        ks[i] = j->k;
        ps[i] = j->params;
        pos[i] = base + brp + bci + opos[i] * pb;
    }
    std::vector<gila_stats> st(ok.size());
    std::vector<int> rcs(ok.size(), rc);
    auto run_range = [&](size_t lo, size_t hi) {
        TraceRange trace_range("gila_server: small-job batch");
        gila_batch* b = nullptr;
        const int32_t cnt = (int32_t)(hi - lo);
        int r = batch_build(&csr[lo], cnt, &ks[lo], sst, &b);
        if (r == GILA_OK) r = batch_run(b, &ps[lo], &pos[lo], sst, &st[lo], false);
        if (b) free_batch(b, Release{true, sst});
        for (size_t i = lo; i < hi; ++i) rcs[i] = r;
        return r;
    };
    // one launch for the group; if it is refused (say one graph is malformed)
    // each job runs on its own, so only the offending job fails
    if (rc == GILA_OK && run_range(0, ok.size()) != GILA_OK && ok.size() > 1)
        for (size_t i = 0; i < ok.size(); ++i) run_range(i, i + 1);
    if (rc == GILA_OK && npos > 0 &&
        (hipMemcpyAsync(h_pos.data(), base + brp + bci, npos * pb, hipMemcpyDeviceToHost,
                        sst) != hipSuccess ||
         hipStreamSynchronize(sst) != hipSuccess))
        for (auto& r : rcs) r = GILA_EDEVICE;
    dfree_on(arena, sst);
    for (size_t i = 0; i < ok.size(); ++i) {
        Job* j = ok[i];
        const int r = rcs[i];
        if (r == GILA_OK) {
            j->result.assign((size_t)2 * j->n, 0.0);
            if (fp64) {
                std::memcpy(j->result.data(), h_pos.data() + opos[i] * pb, sizeof(double) * 2 * j->n);
            } else {
                const float* f = reinterpret_cast<const float*>(h_pos.data() + opos[i] * pb);
                for (size_t e = 0; e < (size_t)2 * j->n; ++e) j->result[e] = f[e];
            }
        }
        std::lock_guard<std::mutex> lk(s->mu);
        j->stats = st[i];
        finish_job(s, j, j->cancel ? kCanceled : (r == GILA_OK ? kDone : kFailed),
                   j->cancel ? GILA_ECANCELED : r);
    }
}

static int admit_large(gila_server* s, Job* j) {
    TraceRange trace_range("gila_server: large-job build");
    GILA_TRY(upload_job(s, j, s->build));
    gila_csr c{j->n, j->nnz, j->d_rp, j->d_ci};
    GILA_TRY(build_khop(&c, j->k, s->build, &j->kh));
    GILA_TRY(prepare_precision(j->kh, j->params.precision, s->build));
    GILA_HIP(hipStreamSynchronize(s->build));
    j->h = 0;
    return GILA_OK;
}

// Admitter thread: admits queued jobs in arrival order while slots and budget
// allow; small jobs go to the small-job worker, large ones are built here and
// handed to the ticker.
static void admitter(gila_server* s) {
    (void)quiet(hipSetDevice(s->device));
    for (;;) {
        std::vector<Job*> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                if (s->stop) return true;
                if (s->pending.empty()) return false;
                const Job* j = s->jobs[s->pending.front()];
                return host::admit_can_progress(s->adm, host::QueuedJob{j->footprint, j->cancel});
            });
            if (s->stop) break;
            for (uint64_t id : s->pending)
                if (s->jobs[id]->footprint < 0) fresh.push_back(s->jobs[id]);
        }
        // footprint bounds of newly queued jobs, outside the lock (a queued
        // job is never deleted, so the pointers stay valid)
        for (Job* j : fresh) {
            const int64_t f = footprint_bytes(*j);
            std::lock_guard<std::mutex> lk(s->mu);
            j->footprint = f;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        bool small_added = false, large_added = false;
        while (!s->pending.empty()) {
            Job* j = s->jobs[s->pending.front()];
            // (a job that arrived after the bounds were taken waits: footprint < 0)
            const host::AdmitOutcome o =
                host::admit_front(s->adm, host::QueuedJob{j->footprint, j->cancel});
            if (o == host::kAdmitWait) break;
            s->pending.pop_front();
            if (o == host::kAdmitDrop || o == host::kAdmitReject) {
                j->state = o == host::kAdmitDrop ? kCanceled : kFailed;
                j->status = o == host::kAdmitDrop ? GILA_ECANCELED : GILA_ENOMEM;
                if (o == host::kAdmitReject)
                    std::snprintf(j->msg, sizeof(j->msg), "footprint bound %lld bytes exceeds "
                                  "the budget of %lld", (long long)j->footprint,
                                  (long long)s->adm.budget);
                j->t_done = now_s();
                s->cv_done.notify_all();
                continue;
            }
            j->state = kResident;
            j->t_admit = now_s();
            if (j->small) {
                s->small_queue.push_back(j);
                small_added = true;
            } else {
                s->build_queue.push_back(j);
                large_added = true;
            }
        }
        if (small_added) s->cv_small.notify_one();
        if (large_added) s->cv_build.notify_one();
    }
}

// Builder: graph upload and k-hop lists of admitted large jobs, one at a time
// in admission order, then the job joins the ticker's resident set.
static void builder(gila_server* s) {
    (void)quiet(hipSetDevice(s->device));
    for (;;) {
        Job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_build.wait(lk, [&] { return s->stop || !s->build_queue.empty(); });
            if (s->stop) break;
            j = s->build_queue.front();
            s->build_queue.pop_front();
        }
        const int rc = j->cancel ? GILA_ECANCELED : admit_large(s, j);
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc != GILA_OK) {
            release_device(j, s->build);
            finish_job(s, j, j->cancel ? kCanceled : kFailed, rc);
        } else {
            j->lane = (int)(j->id % gila_server::kComputeStreams);
            s->ready.push_back(j);
            s->cv_tick.notify_one();
        }
    }
}

// Small-job workers (kSmallWorkers, each with a stream of its own): a worker
// lays out everything admitted so far in batched launches (one per
// precision); jobs admitted while it runs go to the other worker, so they do
// not wait for that group to finish.
static void small_worker(gila_server* s, int w) {
    (void)quiet(hipSetDevice(s->device));
    for (;;) {
        std::vector<Job*> take;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_small.wait(lk, [&] { return s->stop || !s->small_queue.empty(); });
            if (s->stop) break;
            take.swap(s->small_queue);
        }
        std::map<int, std::vector<Job*>> groups;
        for (Job* j : take) groups[j->params.precision].push_back(j);
        for (auto& kv : groups) run_small_group(s, kv.second, s->small[w]);
    }
}

// Ticker: keeps every resident large job advancing.  A job's tick -- a replay
// of its tick graph, then its control block into its pinned slot -- is
// followed by an event on its compute stream; as soon as that event has
// completed the job is retired or given its next tick, whatever the other
// jobs are doing (a job waits only for the work queued before it on the
// stream it shares).  Final positions are copied on a stream of their own, so
// they do not queue behind other jobs' ticks.
static void ticker(gila_server* s) {
    (void)quiet(hipSetDevice(s->device));
    std::vector<Job*> mine;  // resident jobs, owned by this thread
    for (;;) {
        int32_t tick_iters = 1;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (mine.empty())
                s->cv_tick.wait(lk, [&] { return s->stop || !s->ready.empty(); });
            else
                s->cv_tick.wait_for(lk, std::chrono::microseconds(20),
                                    [&] { return s->stop || !s->ready.empty(); });
            if (s->stop) break;
            for (Job* j : s->ready) {  // at most max_slots jobs are in flight
                j->slot = s->free_slots.back();
                s->free_slots.pop_back();
                j->in_tick = false;
                mine.push_back(j);
            }
            s->ready.clear();
            s->resident = mine;
            s->peak_resident = std::max<int32_t>(s->peak_resident, (int32_t)mine.size());
            tick_iters = s->tick_iters;
        }
        std::vector<Job*> keep;
        int64_t ticks = 0;
        for (Job* j : mine) {
            int rc = GILA_OK;
            bool finished = false;
            if (j->in_tick) {
                const hipError_t q = hipEventQuery(s->slot_ev[j->slot]);
                // pending work, or a query refused while another thread
                // captures a stream: not an error, asked again next round
                if (q == hipErrorNotReady || q == hipErrorStreamCaptureUnsupported ||
                    q == hipErrorStreamCaptureImplicit) {
                    (void)hipGetLastError();
                    keep.push_back(j);
                    continue;
                }
                j->in_tick = false;
                if (q != hipSuccess) {
                    rc = fail(GILA_EDEVICE, "tick failed: %s", hipGetErrorString(q));
                    finished = true;
                } else {
                    const Ctl c = s->host_ctl[j->slot];  // copied at the end of the tick
                    j->stats.iterations_run += j->h_target > j->h ? c.iters_run : 0;
                    j->stats.stopped = c.stopped == 1 ? 1 : 0;
                    if (j->h_target > j->h) {
                        j->stats.moved = c.moved;
                        j->stats.max_disp = c.max_disp;
                        j->stats.energy = c.energy;
                        j->stats.coincident = c.coincident;
                        j->stats.nonfinite = c.nonfinite;
                    }
                    j->h = j->h_target;
                    finished = c.stopped || j->h >= j->params.iterations;
                    if (finished) rc = nonfinite_status(c);
                    if (finished && rc == GILA_OK) rc = download_positions(j, s->download);
                }
            }
            if (!finished && j->cancel) finished = true;  // between ticks only
            if (!finished) {
                // the next tick, asynchronously
                TraceRange trace_range("gila_server: tick enqueue");
                j->h_target = std::min(j->h + tick_iters, j->params.iterations);
                hipStream_t st = s->compute[j->lane];
                rc = enqueue_tick(j->kh, &j->params, j->h, j->h_target - j->h, tick_iters,
                                  j->d_pos, st);
                if (rc == GILA_OK && hipMemcpyAsync(&s->host_ctl[j->slot], j->kh->ctl, sizeof(Ctl),
                                                    hipMemcpyDeviceToHost, st) != hipSuccess)
                    rc = fail(GILA_EDEVICE, "control block copy failed");
                if (rc == GILA_OK && hipEventRecord(s->slot_ev[j->slot], st) != hipSuccess)
                    rc = fail(GILA_EDEVICE, "tick event record failed");
                if (rc == GILA_OK) {
                    j->in_tick = true;
                    ++ticks;
                    keep.push_back(j);
                    continue;
                }
                // a job whose tick could not be queued waits for what it queued
                (void)quiet(hipStreamSynchronize(st));
            }
            release_device(j, s->compute[j->lane]);
            std::lock_guard<std::mutex> lk(s->mu);
            s->free_slots.push_back(j->slot);
            j->slot = -1;
            finish_job(s, j, j->cancel ? kCanceled : (rc == GILA_OK ? kDone : kFailed),
                       j->cancel ? GILA_ECANCELED : rc);
        }
        mine.swap(keep);
        std::lock_guard<std::mutex> lk(s->mu);
        s->resident = mine;
        s->ticks += ticks;
    }
}

// Cheap host checks at submission (host_logic.h).
static int validate_host_csr(const gila_csr* g) {
    char msg[256];
    const int rc = host::validate_host_csr(g, msg, sizeof(msg));
    return rc == GILA_OK ? GILA_OK : fail(rc, "%s", msg);
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_server_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_slots,
                       gila_server** out) {
    clear_error();
    if (!out) return fail(GILA_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1) return fail(GILA_EINVAL, "max_slots must be >= 1");
    if (hbm_budget_bytes < 0) return fail(GILA_EINVAL, "negative budget");
    int ndev = 0;
    GILA_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(GILA_EINVAL, "no device %d", device);
    DeviceGuard dg(device);
    gila_server* s = new gila_server();
    s->device = device;
    s->adm.max_slots = max_slots;
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return fail(GILA_EDEVICE, "hipMemGetInfo failed");
        }
        hbm_budget_bytes = (int64_t)(0.9 * (double)fr);
    }
    s->adm.budget = hbm_budget_bytes;
    if (hipHostMalloc((void**)&s->host_ctl, sizeof(Ctl) * (size_t)max_slots,
                      hipHostMallocDefault) != hipSuccess) {
        delete s;
        return fail(GILA_ENOMEM, "pinned control blocks");
    }
    for (int32_t i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->slot_ev.assign((size_t)max_slots, nullptr);
    bool ok = hipStreamCreateWithFlags(&s->build, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->small[0], hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->small[1], hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->download, hipStreamNonBlocking) == hipSuccess;
    for (auto& e : s->slot_ev)
        ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    for (int c = 0; c < gila_server::kComputeStreams && ok; ++c)
        ok = hipStreamCreateWithFlags(&s->compute[c], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        for (int c = 0; c < gila_server::kComputeStreams; ++c)
            if (s->compute[c]) (void)quiet(hipStreamDestroy(s->compute[c]));
        if (s->build) (void)quiet(hipStreamDestroy(s->build));
        for (auto& q : s->small)
            if (q) (void)quiet(hipStreamDestroy(q));
        if (s->download) (void)quiet(hipStreamDestroy(s->download));
        for (auto& e : s->slot_ev)
            if (e) (void)quiet(hipEventDestroy(e));
        (void)quiet(hipHostFree(s->host_ctl));
        delete s;
        return fail(GILA_EDEVICE, "cannot create streams or events");
    }
    s->th_admit = std::thread(admitter, s);
    for (int w = 0; w < gila_server::kSmallWorkers; ++w) s->th_small[w] = std::thread(small_worker, s, w);
    s->th_build = std::thread(builder, s);
    s->th_tick = std::thread(ticker, s);
    *out = s;
    return GILA_OK;
}

int gila_server_config(gila_server* s, const char* key, int64_t value) {
    clear_error();
    if (!s || !key) return fail(GILA_EINVAL, "server or key is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!std::strcmp(key, "tick_iterations")) {
        if (value < 1) return fail(GILA_EINVAL, "tick_iterations must be >= 1");
        s->tick_iters = (int32_t)value;
    } else if (!std::strcmp(key, "small_max_vertices")) {
        if (value < 0) return fail(GILA_EINVAL, "small_max_vertices must be >= 0");
        s->small_max_n = (int32_t)value;
    } else if (!std::strcmp(key, "fail_alloc_ticket")) {
        s->fail_alloc_ticket = (uint64_t)value;
    } else {
        return fail(GILA_EINVAL, "unknown key '%s'", key);
    }
    return GILA_OK;
}

int gila_submit(gila_server* s, const gila_csr* g_host, int32_t k, const gila_params* params,
                const double* init_pos_host, uint64_t* ticket) {
    clear_error();
    if (!s || !ticket) return fail(GILA_EINVAL, "server or ticket is NULL");
    if (k < 1) return fail(GILA_EINVAL, "k must be >= 1");
    GILA_TRY(validate_host_csr(g_host));
    GILA_TRY(check_params(params, true));
    if (params->force_model != GILA_MODEL_FR)
        return fail(GILA_EUNSUPPORTED, "the server runs the FR model only");
    if (g_host->n > 0 && !init_pos_host) return fail(GILA_EINVAL, "init_pos_host is NULL");
    Job* j = new Job();
    j->k = k;
    j->n = g_host->n;
    j->nnz = g_host->nnz;
    j->rp.assign(g_host->row_ptr, g_host->row_ptr + (g_host->n > 0 ? g_host->n + 1 : 0));
    if (j->rp.empty()) j->rp.push_back(0);
    j->ci.assign(g_host->col_idx, g_host->col_idx + g_host->nnz);
    j->init.assign(init_pos_host, init_pos_host + 2 * (size_t)g_host->n);
    j->temps.assign(params->temperature, params->temperature + params->iterations);
    j->params = *params;
    j->params.temperature = j->temps.data();
    j->footprint = -1;  // computed by the admitter when the job is first considered
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // the batch kernel holds both position buffers (n + 1 slots) in LDS
        const size_t cap = device_info(s->device).max_lds_per_block - 2048;
        const size_t per = 2 * (params->precision == GILA_FP64 ? 16 : 8);
        const int32_t fits = (int32_t)std::min<size_t>(65535, cap / per - 1);
        const int32_t lim = s->small_max_n == 0 ? fits : std::min(s->small_max_n, fits);
        j->small = j->n <= lim;
        j->id = s->next_id++;
        j->t_submit = now_s();
        s->jobs[j->id] = j;
        s->pending.push_back(j->id);
        *ticket = j->id;
    }
    s->cv.notify_one();
    return GILA_OK;
}

static int take_result(gila_server* s, Job* j, double* out_pos, gila_stats* out) {
    // mutex held
    const int state = j->state, status = j->status;
    char msg[sizeof(j->msg)];
    std::memcpy(msg, j->msg, sizeof(msg));
    if (state == kDone) {
        if (out_pos && j->n > 0) std::memcpy(out_pos, j->result.data(), sizeof(double) * 2 * j->n);
        if (out) *out = j->stats;
    }
    s->jobs.erase(j->id);
    delete j;
    // a gila_wait on the same ticket in another thread re-checks and returns
    s->cv_done.notify_all();
    if (state == kDone) return GILA_OK;
    if (state == kCanceled) return fail(GILA_ECANCELED, "job was cancelled");
    return fail(status, "job failed: %s (%s)", gila_strerror(status), msg);
}

int gila_poll(gila_server* s, uint64_t ticket, double* out_pos_host, gila_stats* out) {
    clear_error();
    if (!s) return fail(GILA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(GILA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Job* j = it->second;
    if (j->state == kPending || j->state == kResident) return GILA_EAGAIN;
    return take_result(s, j, out_pos_host, out);
}

int gila_wait(gila_server* s, uint64_t ticket, double* out_pos_host, gila_stats* out) {
    clear_error();
    if (!s) return fail(GILA_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->jobs.find(ticket) == s->jobs.end())
        return fail(GILA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    // the job is looked up afresh on every wake-up: another thread may have
    // taken its result (gila_poll or gila_wait on the same ticket) meanwhile
    s->cv_done.wait(lk, [&] {
        const auto it = s->jobs.find(ticket);
        return it == s->jobs.end() || (it->second->state != kPending && it->second->state != kResident);
    });
    const auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return fail(GILA_EINVAL, "the result of ticket %llu was taken by another call",
                    (unsigned long long)ticket);
    return take_result(s, it->second, out_pos_host, out);
}

int gila_cancel(gila_server* s, uint64_t ticket) {
    clear_error();
    if (!s) return fail(GILA_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(GILA_EINVAL, "unknown ticket");
        it->second->cancel = true;
    }
    s->cv.notify_one();
    s->cv_tick.notify_one();
    return GILA_OK;
}

int gila_job_latency(gila_server* s, uint64_t ticket, double* queued_ms, double* total_ms) {
    clear_error();
    if (!s) return fail(GILA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->times.find(ticket);
    if (it == s->times.end()) return fail(GILA_EAGAIN, "job %llu has not finished",
                                          (unsigned long long)ticket);
    if (queued_ms) *queued_ms = it->second.first;
    if (total_ms) *total_ms = it->second.second;
    return GILA_OK;
}

int gila_server_info(gila_server* s, int64_t* jobs_done, int64_t* ticks, int32_t* peak_resident,
                     int64_t* bytes_in_use) {
    if (!s) return fail(GILA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (jobs_done) *jobs_done = s->jobs_done;
    if (ticks) *ticks = s->ticks;
    if (peak_resident) *peak_resident = s->peak_resident;
    if (bytes_in_use) *bytes_in_use = s->adm.reserved;
    return GILA_OK;
}

void gila_server_destroy(gila_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->cv_small.notify_all();
    s->cv_build.notify_all();
    s->cv_tick.notify_all();
    if (s->th_admit.joinable()) s->th_admit.join();
    for (auto& t : s->th_small)
        if (t.joinable()) t.join();
    if (s->th_build.joinable()) s->th_build.join();
    if (s->th_tick.joinable()) s->th_tick.join();
    DeviceGuard dg(s->device);
    for (int c = 0; c < gila_server::kComputeStreams; ++c) (void)quiet(hipStreamSynchronize(s->compute[c]));
    (void)quiet(hipStreamSynchronize(s->build));
    for (auto& q : s->small) (void)quiet(hipStreamSynchronize(q));
    (void)quiet(hipStreamSynchronize(s->download));
    for (Job* j : s->resident) release_device(j, s->build);
    for (Job* j : s->ready) release_device(j, s->build);
    for (auto& kv : s->jobs) delete kv.second;
    for (int c = 0; c < gila_server::kComputeStreams; ++c) (void)quiet(hipStreamDestroy(s->compute[c]));
    (void)quiet(hipStreamDestroy(s->build));
    for (auto& q : s->small) (void)quiet(hipStreamDestroy(q));
    (void)quiet(hipStreamDestroy(s->download));
    for (auto& e : s->slot_ev) (void)quiet(hipEventDestroy(e));
    (void)quiet(hipHostFree(s->host_ctl));
    delete s;
}

}  // extern "C"
