// Served RQA: a request loop that admits independent jobs by device-memory
// footprint and runs them with continuous batching.
//
// * The server owns one device pool of `budget` bytes, carved up by a
//   first-fit allocator; a job is admitted (FIFO) when its footprint fits, so
//   no hipMalloc happens on the request path.
// * A worker thread groups the jobs admitted since its last launch into one
//   batched launch of the engine; jobs that arrive while earlier launches run
//   are launched on another stream and overlap with them on the device.
// * Latency: a large job (above kBigCells cells) gets a launch of its own (a
//   batch completes as a whole, so small jobs batched with a large one would
//   wait for it).  The streams are split in two classes: large launches use
//   the first half, small ones the second, each picking the stream of its
//   class with the least work in flight, so a small launch never queues
//   behind a large one on a stream.  A large launch runs one persistent
//   workgroup per compute unit, which leaves workgroup slots free for the
//   small launches (a persistent grid would hold every slot until the large
//   job ends) and shortens the large job's own critical path (its strips are
//   sequential chains of tiles that run faster with fewer waves per SIMD).
// * Each launch copies its histograms into pinned host buffers (recycled
//   through a cache) and then fires a host callback that marks its jobs done
//   and returns their device memory to the pool; the worker then admits more.
// * No HIP call is made while the server mutex is held: host callbacks take the
//   mutex, and a HIP call that waits on a stream could otherwise wait for a
//   callback that waits for the mutex.
// Results are integer histograms, so a job's result does not depend on what
// else runs beside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rqa_internal.h"
#include "rqa_policy.h"

using namespace rqa;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

enum JobState { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct ServedJob {
    uint64_t ticket = 0;
    rqa_params p{};
    const float *series = nullptr;
    int64_t n_points = 0;
    int64_t n_vec = 0;
    size_t footprint = 0;
    size_t hist_bytes = 0;
    size_t off = 0;
    hipEvent_t ready = nullptr;    // recorded on the caller's stream at submit
    uint64_t *host = nullptr;      // pinned: 3*(n+1) histograms + info record
    size_t host_bytes = 0;
    int state = kQueued;
    int rc = RQA_OK;
};

constexpr size_t kMaxBatch = 256;

double job_cells(const ServedJob *j) { return static_cast<double>(j->n_vec) * j->n_vec; }
constexpr size_t kInfoWords = kInfoBytes / sizeof(uint64_t);

}  // namespace

struct rqa_server {
    std::mutex mu;
    std::condition_variable cv;        // worker wake-ups
    std::condition_variable done_cv;   // job completions
    int device = 0;
    char *pool_base = nullptr;
    size_t budget = 0;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<char *> launch_scratch;   // per stream, device
    std::vector<void *> staging;          // per stream, pinned host
    std::vector<hipEvent_t> staging_free; // per stream: staging consumed
    std::vector<double> load;             // per stream: cells of the launches in flight
    int ncu = 0;                          // compute units of the device
    std::deque<ServedJob *> pending;
    std::unordered_map<uint64_t, ServedJob *> jobs;
    std::multimap<size_t, void *> pinned_free;   // recycled pinned result buffers
    uint64_t next_ticket = 1;
    int inflight = 0;
    uint64_t completions = 0;   // launches finished so far
    bool stop = false;
    std::thread worker;
};

namespace {

struct Launch {
    rqa_server *srv;
    std::vector<ServedJob *> jobs;
    size_t slot;
    double cells;
};

size_t job_hist_bytes(int64_t n_vec) {
    return align256(sizeof(uint64_t) * 3 * static_cast<size_t>(n_vec + 1));
}

size_t job_scratch_bytes(const rqa_params &p, int64_t n_points, int64_t n_vec) {
    Job one;
    one.n_points = n_points;
    one.n_vec = n_vec;
    one.kp = make_kparams(p);
    one.waves = engine_default_waves(n_vec);
    return align256(engine_job_scratch_bytes(one));
}

// Pinned buffer of at least `bytes` from the cache (lock held), or nullptr.
void *take_pinned(rqa_server *srv, size_t bytes, size_t *got) {
    auto it = srv->pinned_free.lower_bound(bytes);
    if (it == srv->pinned_free.end()) return nullptr;
    void *p = it->second;
    *got = it->first;
    srv->pinned_free.erase(it);
    return p;
}

void on_launch_done(void *arg) {
    Launch *ln = static_cast<Launch *>(arg);
    rqa_server *srv = ln->srv;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (ServedJob *j : ln->jobs) {
            int flag = 0;
            std::memcpy(&flag, j->host + 3 * (j->n_vec + 1), sizeof(int));
            j->rc = (flag & 1) ? RQA_ENONFINITE : flag ? RQA_EDEVICE : RQA_OK;
            j->state = flag ? kFailed : kDone;
            srv->pool.release(j->off, j->footprint);
        }
        srv->load[ln->slot] -= ln->cells;
        --srv->inflight;
        ++srv->completions;
    }
    srv->cv.notify_all();
    srv->done_cv.notify_all();
    delete ln;
}

// Launch the next admissible queued jobs (FIFO, stopping at the first that
// does not fit) as one batched launch: either one large job alone or a run of
// small ones.  Entered and left with `lk` held; the HIP calls run with it
// released.  Returns the number of jobs launched.
size_t admit_and_launch(rqa_server *srv, std::unique_lock<std::mutex> &lk) {
    std::deque<AdmitJob> queue;
    for (const ServedJob *j : srv->pending) {
        queue.push_back(AdmitJob{job_cells(j), j->footprint});
        if (queue.size() >= kMaxBatch) break;
    }
    const Admission adm = plan_launch(queue, srv->pool, kMaxBatch);
    if (adm.offsets.empty()) return 0;
    std::vector<ServedJob *> batch;
    for (size_t off : adm.offsets) {
        ServedJob *j = srv->pending.front();
        srv->pending.pop_front();
        j->off = off;
        j->state = kRunning;
        batch.push_back(j);
    }
    const double cells = adm.cells;
    const bool big = adm.big;
    const size_t slot = pick_stream(srv->load, big);
    srv->load[slot] += cells;
    ++srv->inflight;
    lk.unlock();

    hipStream_t st = srv->streams[slot];
    std::vector<Job> ej;
    ej.reserve(batch.size());
    int rc = RQA_OK;
    for (ServedJob *j : batch) {
        if (hipStreamWaitEvent(st, j->ready, 0) != hipSuccess) rc = RQA_EDEVICE;
        char *base = srv->pool_base + j->off;
        Job e;
        e.series = j->series;
        e.n_points = j->n_points;
        e.n_vec = j->n_vec;
        e.hist = reinterpret_cast<uint64_t *>(base);
        e.flag = reinterpret_cast<int *>(base + j->hist_bytes);
        e.scratch = base + j->hist_bytes + kInfoBytes;
        e.kp = make_kparams(j->p);
        e.waves = engine_default_waves(j->n_vec);
        ej.push_back(e);
    }
    if (rc == RQA_OK)
        rc = engine_launch(ej, srv->launch_scratch[slot], srv->staging[slot],
                           srv->staging_free[slot], big ? srv->ncu : 0, st, nullptr, nullptr);
    for (size_t k = 0; k < batch.size() && rc == RQA_OK; ++k) {
        ServedJob *j = batch[k];
        const size_t hb = sizeof(uint64_t) * 3 * static_cast<size_t>(j->n_vec + 1);
        if (hipMemcpyAsync(j->host, ej[k].hist, hb, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(j->host + 3 * (j->n_vec + 1), ej[k].flag, kInfoBytes,
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = RQA_EDEVICE;
    }
    Launch *ln = new Launch{srv, batch, slot, cells};
    if (rc == RQA_OK && hipLaunchHostFunc(st, on_launch_done, ln) == hipSuccess) {
        lk.lock();
        return batch.size();
    }
    // The launch failed: wait for the stream, then fail the jobs.
    hipStreamSynchronize(st);
    delete ln;
    lk.lock();
    for (ServedJob *j : batch) {
        j->state = kFailed;
        j->rc = rc == RQA_OK ? RQA_EDEVICE : rc;
        srv->pool.release(j->off, j->footprint);
    }
    srv->load[slot] -= cells;
    --srv->inflight;
    ++srv->completions;
    srv->done_cv.notify_all();
    return batch.size();
}

void worker_main(rqa_server *srv) {
    hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        srv->cv.wait(lk, [srv] { return srv->stop || !srv->pending.empty(); });
        if (srv->stop && srv->pending.empty()) break;
        const size_t before = srv->pending.size();
        const uint64_t seen = srv->completions;
        if (admit_and_launch(srv, lk) > 0) continue;
        if (srv->inflight == 0) {
            // Nothing runs, so the whole pool is free, and still the head job does
            // not fit (cannot happen for jobs accepted by rqa_submit).
            ServedJob *j = srv->pending.front();
            srv->pending.pop_front();
            j->state = kFailed;
            j->rc = RQA_EBUDGET;
            srv->done_cv.notify_all();
            continue;
        }
        // Wait until a launch completes (returning memory to the pool), new jobs
        // arrive, or a stop is requested.
        srv->cv.wait(lk, [srv, before, seen] {
            return srv->stop || srv->completions != seen || srv->pending.size() != before;
        });
    }
}

// Copy a finished job's results out and retire it (lock held; no HIP calls).
// Hands back the job's event, to be destroyed once the lock is released.
int collect(rqa_server *srv, ServedJob *j, rqa_measures *out, uint64_t *diag, uint64_t *vert,
            uint64_t *white, hipEvent_t *ev_out) {
    const int64_t n = j->n_vec;
    const int rc = j->rc;
    if (rc == RQA_OK) {
        const uint64_t *hd = j->host, *hv = hd + (n + 1), *hw = hv + (n + 1);
        if (diag) std::memcpy(diag, hd, sizeof(uint64_t) * (n + 1));
        if (vert) std::memcpy(vert, hv, sizeof(uint64_t) * (n + 1));
        if (white) std::memcpy(white, hw, sizeof(uint64_t) * (n + 1));
        if (out) {
            JobStats stats;
            std::memcpy(&stats, reinterpret_cast<const char *>(hw + (n + 1)) + 8, sizeof stats);
            measures_from_stats(stats, n, n, j->p, out);
        }
    }
    srv->jobs.erase(j->ticket);
    srv->pinned_free.emplace(j->host_bytes, j->host);
    *ev_out = j->ready;
    delete j;
    return rc;
}

}  // namespace

extern "C" {

int rqa_job_footprint(const rqa_params *p, int64_t n_points, size_t *bytes) {
    if (!p || !bytes) return RQA_EINVAL;
    int rc = validate_params(*p);
    if (rc != RQA_OK) return rc;
    const int64_t nv = n_points - static_cast<int64_t>(p->m - 1) * p->tau;
    if (nv < 1) return RQA_ETOOSHORT;
    *bytes = job_hist_bytes(nv) + kInfoBytes + job_scratch_bytes(*p, n_points, nv);
    return RQA_OK;
}

int rqa_server_create(rqa_server **out, size_t budget_bytes, int32_t streams) {
    if (!out || budget_bytes < 4096 || streams < 1 || streams > 16) return RQA_EINVAL;
    std::unique_ptr<rqa_server> srv(new (std::nothrow) rqa_server);
    if (!srv) return RQA_ENOMEM;
    if (hipGetDevice(&srv->device) != hipSuccess ||
        hipDeviceGetAttribute(&srv->ncu, hipDeviceAttributeMultiprocessorCount, srv->device) !=
            hipSuccess)
        return RQA_EDEVICE;
    void *base = nullptr;
    if (hipMalloc(&base, budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return RQA_ENOMEM;
    }
    srv->pool_base = static_cast<char *>(base);
    srv->budget = budget_bytes;
    srv->pool.reset(budget_bytes);
    const size_t ls = align256(engine_launch_scratch_bytes(kMaxBatch));
    bool ok = true;
    for (int32_t k = 0; k < streams && ok; ++k) {
        hipStream_t st = nullptr;
        void *d = nullptr, *h = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) srv->streams.push_back(st);
        ok = ok && hipMalloc(&d, ls) == hipSuccess;
        if (ok) srv->launch_scratch.push_back(static_cast<char *>(d));
        ok = ok && hipHostMalloc(&h, ls, hipHostMallocDefault) == hipSuccess;
        if (ok) srv->staging.push_back(h);
        hipEvent_t ev = nullptr;
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) srv->staging_free.push_back(ev);
        srv->load.push_back(0.0);
    }
    if (!ok) {
        (void)hipGetLastError();
        for (hipStream_t s : srv->streams) hipStreamDestroy(s);
        for (char *d : srv->launch_scratch) hipFree(d);
        for (void *h : srv->staging) hipHostFree(h);
        for (hipEvent_t e : srv->staging_free) hipEventDestroy(e);
        hipFree(base);
        return RQA_ENOMEM;
    }
    rqa_server *raw = srv.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return RQA_OK;
}

int rqa_submit(rqa_server *srv, const rqa_params *p, const float *d_series, int64_t n_points,
               void *hip_stream, uint64_t *ticket) {
    if (!srv || !p || !d_series || !ticket || n_points < 0) return RQA_EINVAL;
    size_t fp = 0;
    int rc = rqa_job_footprint(p, n_points, &fp);
    if (rc != RQA_OK) return rc;
    if (fp > srv->budget) return RQA_EBUDGET;
    ServedJob *j = new (std::nothrow) ServedJob;
    if (!j) return RQA_ENOMEM;
    j->p = *p;
    j->series = d_series;
    j->n_points = n_points;
    j->n_vec = n_points - static_cast<int64_t>(p->m - 1) * p->tau;
    j->footprint = fp;
    j->hist_bytes = job_hist_bytes(j->n_vec);
    const size_t need = sizeof(uint64_t) * (3 * static_cast<size_t>(j->n_vec + 1) + kInfoWords);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        j->host = static_cast<uint64_t *>(take_pinned(srv, need, &j->host_bytes));
    }
    if (!j->host) {
        size_t cap = 4096;
        while (cap < need) cap <<= 1;
        if (hipHostMalloc(reinterpret_cast<void **>(&j->host), cap, hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            delete j;
            return RQA_ENOMEM;
        }
        j->host_bytes = cap;
    }
    std::memset(j->host + 3 * (j->n_vec + 1), 0, kInfoBytes);
    if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(j->ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->pinned_free.emplace(j->host_bytes, j->host);
        delete j;
        return RQA_EDEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        j->ticket = srv->next_ticket++;
        srv->jobs[j->ticket] = j;
        srv->pending.push_back(j);
        *ticket = j->ticket;
    }
    srv->cv.notify_all();
    return RQA_OK;
}

int rqa_poll(rqa_server *srv, uint64_t ticket, rqa_measures *out, uint64_t *diag, uint64_t *vert,
             uint64_t *white, int64_t hist_len) {
    if (!srv) return RQA_EINVAL;
    hipEvent_t ev = nullptr;
    int rc;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end()) return RQA_ENOTFOUND;
        ServedJob *j = it->second;
        if ((diag || vert || white) && hist_len < j->n_vec + 1) return RQA_ESIZE;
        if (j->state == kQueued || j->state == kRunning) return RQA_EAGAIN;
        rc = collect(srv, j, out, diag, vert, white, &ev);
    }
    if (ev) hipEventDestroy(ev);
    return rc;
}

int rqa_wait(rqa_server *srv, uint64_t ticket, rqa_measures *out, uint64_t *diag, uint64_t *vert,
             uint64_t *white, int64_t hist_len) {
    if (!srv) return RQA_EINVAL;
    hipEvent_t ev = nullptr;
    int rc;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end()) return RQA_ENOTFOUND;
        ServedJob *j = it->second;
        if ((diag || vert || white) && hist_len < j->n_vec + 1) return RQA_ESIZE;
        srv->done_cv.wait(lk, [j] { return j->state == kDone || j->state == kFailed; });
        rc = collect(srv, j, out, diag, vert, white, &ev);
    }
    if (ev) hipEventDestroy(ev);
    return rc;
}

void rqa_server_destroy(rqa_server *srv) {
    if (!srv) return;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->done_cv.wait(lk, [srv] { return srv->pending.empty() && srv->inflight == 0; });
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (hipStream_t s : srv->streams) {
        hipStreamSynchronize(s);
        hipStreamDestroy(s);
    }
    for (char *d : srv->launch_scratch) hipFree(d);
    for (void *h : srv->staging) hipHostFree(h);
    for (hipEvent_t e : srv->staging_free) hipEventDestroy(e);
    for (auto &kv : srv->jobs) {
        hipHostFree(kv.second->host);
        hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    for (auto &kv : srv->pinned_free) hipHostFree(kv.second);
    hipFree(srv->pool_base);
    delete srv;
}

}  // extern "C"
