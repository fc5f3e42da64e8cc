// C ABI of librqa: parameter validation, device workspace, enqueue of the hot
// path on the caller's stream, and result retrieval (Sect. 7: Settings ->
// RQAComputation.create -> run -> RQAResult; missing devices and invalid input
// are reported as errors, never aborts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rqa_internal.h"

namespace rqa {

int validate_params(const rqa_params &p) {
    if (p.m < 1 || p.tau < 1) return RQA_EINVAL;
    if (!(p.eps >= 0.0f) || std::isinf(p.eps)) return RQA_EINVAL;
    if (p.norm < RQA_NORM_L1 || p.norm > RQA_NORM_LINF) return RQA_EINVAL;
    if (p.lmin < 1 || p.vmin < 1 || p.wmin < 1 || p.theiler < 0) return RQA_EINVAL;
    // (m-1)*tau must fit comfortably in 32 bits for device index arithmetic.
    if (static_cast<int64_t>(p.m - 1) * p.tau > (int64_t(1) << 30)) return RQA_EINVAL;
    return RQA_OK;
}

Workspace::~Workspace() {
    if (base) {
        int cur = -1;
        hipGetDevice(&cur);
        if (device >= 0 && cur != device) hipSetDevice(device);
        hipFree(base);
        if (device >= 0 && cur != device && cur >= 0) hipSetDevice(cur);
    }
}

int Workspace::reserve(size_t need) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RQA_EDEVICE;
    need = (need + 255) & ~size_t(255);
    if (base && device == dev && bytes >= need) return RQA_OK;
    if (base) {
        if (device != dev) {
            hipSetDevice(device);
            hipDeviceSynchronize();
            hipFree(base);
            hipSetDevice(dev);
        } else {
            hipDeviceSynchronize();
            hipFree(base);
        }
        base = nullptr;
        bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        return RQA_ENOMEM;
    }
    base = p;
    bytes = need;
    device = dev;
    return RQA_OK;
}

}  // namespace rqa

using namespace rqa;

// ---------------------------------------------------------------------------
// Workgroup-shape autotuner.  For a launch signature (norm, m, size class,
// number of jobs) it times each candidate shape on real runs (the tile phase,
// measured with hipEvents when the run's result is fetched) and then keeps the
// fastest.  Results never depend on the shape, so trial runs are ordinary runs.
// The table is process-wide; with RQA_AUTOTUNE_CACHE=<file> decisions persist
// across processes as "key waves" lines.
// ---------------------------------------------------------------------------
namespace {

constexpr int kCandidates[] = {2, 4, 8};
constexpr int kNumCandidates = 3;
// A trial this much slower than the best so far ends the trials in its
// direction (fewer or more waves than the default shape): at N = 1M the
// 4-wave shape is 12% slower than 8 waves and 2 waves 65% slower.
constexpr double kGiveUp = 1.10;

struct TuneEntry {
    int cand[kNumCandidates] = {};   // trial order: the default shape first, then fewer
    int ncand = 0;                   // waves, then more
    int dflt = 0;
    int next = 0;          // next candidate to try
    int best = 0;          // best waves so far
    double best_ms = 1e300;
    bool done = false;
};

void tune_init(TuneEntry &e, int dflt) {
    e.dflt = dflt;
    e.ncand = 0;
    e.cand[e.ncand++] = dflt;
    for (int k = kNumCandidates - 1; k >= 0; --k)
        if (kCandidates[k] < dflt) e.cand[e.ncand++] = kCandidates[k];
    for (int k = 0; k < kNumCandidates; ++k)
        if (kCandidates[k] > dflt) e.cand[e.ncand++] = kCandidates[k];
}

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("RQA_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    int waves;
    while (f >> key >> waves) {
        if (waves < 1 || waves > 8) continue;
        TuneEntry &e = g_tune[key];
        e.best = waves;
        e.done = true;
    }
}

void tune_store_locked(const std::string &key, int waves) {
    const char *path = std::getenv("RQA_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << waves << "\n";
}

int ilog2(int64_t v) {
    int l = 0;
    while (v > 1) { v >>= 1; ++l; }
    return l;
}

std::string tune_key(const rqa_params &p, int64_t nmax, int32_t count) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "norm%d_m%d_n2^%d_jobs2^%d_w%d", p.norm, p.m <= 6 ? p.m : 0,
                  ilog2(nmax), ilog2(count), p.theiler > 64 ? 65 : p.theiler);
    return buf;
}

uint64_t fnv(uint64_t h, const void *data, size_t bytes) {
    const unsigned char *c = static_cast<const unsigned char *>(data);
    for (size_t k = 0; k < bytes; ++k) h = (h ^ c[k]) * 1099511628211ull;
    return h;
}

}  // namespace

struct rqa_handle {
    rqa_params p{};
    Workspace ws;
    void *staging = nullptr;        // pinned host buffer for launch descriptors
    size_t staging_bytes = 0;
    hipEvent_t staging_free = nullptr;   // recorded when a launch has read `staging`
    bool profiling = false;
    bool prof_valid = false;
    PhaseEvents prof{};
    int waves = 0;                  // 0 = autotuned
    int groups = 0;                 // 0 = fill the device
    int64_t ws_limit = 0;           // line-summary bytes of a one-series run (0 = default)
    JobPlan plan{};                 // how the last run's first job was cut
    bool has_run = false;
    bool batched = false;
    hipStream_t stream = nullptr;
    std::vector<int64_t> nvec;      // per job: rows (delay vectors)
    std::vector<int64_t> ncols;     // per job: columns
    std::vector<int64_t> hlen;      // per job: histogram entries
    std::vector<size_t> job_off;    // per job: byte offset of its histograms in ws.base
    size_t info_block_off = 0;      // info records (flag + statistics) of all jobs
    size_t hist_block_off = 0;      // histograms of all jobs, contiguous
    size_t hist_block_bytes = 0;
    char *info_cache = nullptr;     // pinned host copies
    size_t info_cache_bytes = 0;
    uint64_t *host_cache = nullptr;
    size_t host_cache_bytes = 0;
    bool info_valid = false;
    bool cache_valid = false;
    bool last_from_graph = false;   // the last run was a graph replay
    // autotuning trial in flight
    bool trial = false;
    int trial_waves = 0;
    std::string trial_key;
    // graph replay of repeated identical launches
    uint64_t last_sig = 0;
    uint64_t graph_sig = 0;
    hipGraphExec_t graph = nullptr;
    void *graph_staging = nullptr;
    hipStream_t capture_stream = nullptr;
    // recurrence plot output: tail scratch, and the event after the last plot
    float *plot_tail = nullptr;
    size_t plot_tail_bytes = 0;
    hipEvent_t plot_done = nullptr;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void drop_graph(rqa_handle *h) {
    if (h->graph) hipGraphExecDestroy(h->graph);
    if (h->graph_staging) hipHostFree(h->graph_staging);
    h->graph = nullptr;
    h->graph_staging = nullptr;
    h->graph_sig = 0;
}

int ensure_events(rqa_handle *h) {
    if (!h->prof.ev[0]) {
        for (hipEvent_t &e : h->prof.ev)
            if (hipEventCreate(&e) != hipSuccess) return RQA_EDEVICE;
    }
    return RQA_OK;
}

// Capture the launch of `jobs` into a graph (own staging buffer, own capture
// stream) and instantiate it.
int capture_graph(rqa_handle *h, const std::vector<Job> &jobs, char *base, uint64_t sig) {
    drop_graph(h);
    if (!h->capture_stream &&
        hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return RQA_EDEVICE;
    if (hipHostMalloc(&h->graph_staging, align256(engine_launch_scratch_bytes(jobs.size())),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        h->graph_staging = nullptr;
        return RQA_ENOMEM;
    }
    if (hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return RQA_EDEVICE;
    int rc = engine_launch(jobs, base, h->graph_staging, nullptr, h->groups, h->capture_stream,
                           nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->capture_stream, &g);
    if (rc != RQA_OK || ec != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        (void)hipGetLastError();
        drop_graph(h);
        return rc != RQA_OK ? rc : RQA_EDEVICE;
    }
    const hipError_t ei = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        h->graph = nullptr;
        drop_graph(h);
        return RQA_EDEVICE;
    }
    h->graph_sig = sig;
    return RQA_OK;
}

// Lay out the workspace for `jobs` and enqueue them: [launch scratch][info
// records of every job][histograms of every job][job scratch], so that a fetch
// copies the small records in one go and the histograms, when asked for, in one
// more.  `sig` identifies the launch apart from the workspace; an identical
// repeat replays a captured graph.
int launch(rqa_handle *h, std::vector<Job> &jobs, int waves, bool trial, const std::string &key,
           uint64_t sig, void *stream, bool batched) {
    const int32_t count = static_cast<int32_t>(jobs.size());
    std::vector<int64_t> nvec(count), ncols(count), hlen(count);
    std::vector<size_t> off(count);
    size_t total = align256(engine_launch_scratch_bytes(count));
    const size_t info_block_off = total;
    total += align256(kInfoBytes * static_cast<size_t>(count));
    const size_t hist_block_off = total;
    for (int32_t w = 0; w < count; ++w) jobs[w].waves = waves;
    // A job run alone (a series, a cross pair or a given matrix) is cut into
    // row bands when its line summaries would exceed the workspace limit.
    if (count == 1) {
        size_t limit = static_cast<size_t>(h->ws_limit);
        if (limit == 0) {
            int dev = 0;
            size_t total_mem = 0;
            if (hipGetDevice(&dev) != hipSuccess || hipDeviceTotalMem(&total_mem, dev) != hipSuccess)
                return RQA_EDEVICE;
            limit = total_mem / 4;
        }
        jobs[0].band_strips = engine_band_strips(jobs[0], limit);
        sig = fnv(sig, &jobs[0].band_strips, sizeof jobs[0].band_strips);
    }
    Job first = jobs[0];
    if (count > 1 && first.segs == 0) first.segs = 1;   // as the engine launches it
    const JobPlan plan = engine_job_plan(first);
    for (int32_t w = 0; w < count; ++w) {
        nvec[w] = jobs[w].n_vec;
        ncols[w] = jobs[w].mode == kModeAuto ? jobs[w].n_vec : jobs[w].n_cols;
        hlen[w] = jobs[w].hist_len();
        off[w] = total;
        total += align256(sizeof(uint64_t) * 3 * static_cast<size_t>(hlen[w]));
    }
    const size_t hist_block_bytes = total - hist_block_off;
    std::vector<size_t> soff(count);
    for (int32_t w = 0; w < count; ++w) {
        soff[w] = total;
        total += align256(engine_job_scratch_bytes(jobs[w]));
    }
    void *old_base = h->ws.base;
    int rc = h->ws.reserve(total);
    if (rc != RQA_OK) return rc;
    if (h->ws.base != old_base) drop_graph(h);
    const size_t stage = align256(engine_launch_scratch_bytes(count));
    if (!h->staging_free &&
        hipEventCreateWithFlags(&h->staging_free, hipEventDisableTiming) != hipSuccess)
        return RQA_EDEVICE;
    if (h->staging_bytes < stage) {
        if (h->has_run) hipEventSynchronize(h->staging_free);
        if (h->staging) hipHostFree(h->staging);
        h->staging = nullptr;
        h->staging_bytes = 0;
        if (hipHostMalloc(&h->staging, stage, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return RQA_ENOMEM;
        }
        h->staging_bytes = stage;
    }
    char *base = static_cast<char *>(h->ws.base);
    for (int32_t w = 0; w < count; ++w) {
        Job &jb = jobs[w];
        jb.hist = reinterpret_cast<uint64_t *>(base + off[w]);
        jb.flag = reinterpret_cast<int *>(base + info_block_off + kInfoBytes * w);
        jb.scratch = base + soff[w];
    }
    hipStream_t st = static_cast<hipStream_t>(stream);

    sig = fnv(sig, &h->p, sizeof h->p);
    sig = fnv(sig, &waves, sizeof waves);
    sig = fnv(sig, &h->groups, sizeof h->groups);
    sig = fnv(sig, &base, sizeof base);
    const bool plain = !h->profiling && !trial;

    h->last_from_graph = false;
    if (plain && h->graph && h->graph_sig == sig) {
        if (hipGraphLaunch(h->graph, st) != hipSuccess) return RQA_EDEVICE;
        h->prof_valid = false;
        h->last_from_graph = true;
    } else if (plain && h->last_sig == sig && capture_graph(h, jobs, base, sig) == RQA_OK) {
        if (hipGraphLaunch(h->graph, st) != hipSuccess) return RQA_EDEVICE;
        h->prof_valid = false;
        h->last_from_graph = true;
    } else {
        const bool timed = h->profiling || trial;
        if (timed && (rc = ensure_events(h)) != RQA_OK) return rc;
        rc = engine_launch(jobs, base, h->staging, h->staging_free, h->groups, st,
                           timed ? &h->prof : nullptr);
        h->prof_valid = timed && rc == RQA_OK;
        if (rc != RQA_OK) return rc;
    }
    h->last_sig = sig;
    h->plan = plan;
    h->trial = trial;
    h->trial_waves = waves;
    h->trial_key = key;
    h->nvec = std::move(nvec);
    h->ncols = std::move(ncols);
    h->hlen = std::move(hlen);
    h->job_off = std::move(off);
    h->info_block_off = info_block_off;
    h->hist_block_off = hist_block_off;
    h->hist_block_bytes = hist_block_bytes;
    h->info_valid = false;
    h->cache_valid = false;
    h->stream = st;
    h->has_run = true;
    h->batched = batched;
    return RQA_OK;
}

int enqueue(rqa_handle *h, const float *d_series, int64_t n_points, const int64_t *offsets,
            const int64_t *lengths, int32_t count, void *stream, bool batched) {
    if (!h || !d_series) return RQA_EINVAL;
    std::vector<Job> jobs(count);
    const KParams kp = make_kparams(h->p);
    int64_t nmax = 0;
    for (int32_t w = 0; w < count; ++w) {
        const int64_t o = offsets ? offsets[w] : 0;
        const int64_t len = lengths ? lengths[w] : n_points;
        if (o < 0 || len < 0 || o > n_points || len > n_points - o) return RQA_EINVAL;
        const int64_t nv = len - static_cast<int64_t>(h->p.m - 1) * h->p.tau;
        if (nv < 1) return RQA_ETOOSHORT;
        if (nv > (int64_t(1) << 31) - 2) return RQA_EINVAL;
        Job &jb = jobs[w];
        jb.series = d_series + o;
        jb.n_points = len;
        jb.n_vec = nv;
        jb.n_cols = nv;
        jb.kp = kp;
        nmax = std::max(nmax, nv);
    }

    // Workgroup shape: fixed by rqa_set_tiling, else tuned per signature.
    bool trial = false;
    int waves = h->waves;
    std::string key;
    if (waves == 0) {
        key = tune_key(h->p, nmax, count);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        TuneEntry &e = g_tune[key];
        if (!e.done && e.ncand == 0) tune_init(e, engine_default_waves(nmax));
        if (e.done) {
            waves = e.best;
        } else {
            waves = e.cand[e.next];
            trial = true;
        }
    }
    uint64_t sig = 1469598103934665603ull;
    const int32_t mode = kModeAuto;
    sig = fnv(sig, &mode, sizeof mode);
    sig = fnv(sig, &d_series, sizeof d_series);
    sig = fnv(sig, &n_points, sizeof n_points);
    sig = fnv(sig, &count, sizeof count);
    if (offsets) sig = fnv(sig, offsets, sizeof(int64_t) * count);
    if (lengths) sig = fnv(sig, lengths, sizeof(int64_t) * count);
    return launch(h, jobs, waves, trial, key, sig, stream, batched);
}

// One job over a full (not symmetric) matrix: the cross recurrence matrix of
// (a, b), or a given bit matrix.
int enqueue_full(rqa_handle *h, Job jb, void *stream) {
    if (jb.n_vec > (int64_t(1) << 31) - 2 || jb.n_cols > (int64_t(1) << 31) - 2)
        return RQA_EINVAL;
    jb.kp = make_kparams(h->p);
    const int waves = h->waves > 0 ? h->waves : engine_default_waves(jb.n_vec);
    std::vector<Job> jobs(1, jb);
    uint64_t sig = 1469598103934665603ull;
    sig = fnv(sig, &jb.mode, sizeof jb.mode);
    sig = fnv(sig, &jb.series, sizeof jb.series);
    sig = fnv(sig, &jb.n_points, sizeof jb.n_points);
    sig = fnv(sig, &jb.series_b, sizeof jb.series_b);
    sig = fnv(sig, &jb.n_points_b, sizeof jb.n_points_b);
    sig = fnv(sig, &jb.bits, sizeof jb.bits);
    sig = fnv(sig, &jb.n_vec, sizeof jb.n_vec);
    sig = fnv(sig, &jb.n_cols, sizeof jb.n_cols);
    sig = fnv(sig, &jb.words, sizeof jb.words);
    return launch(h, jobs, waves, false, std::string(), sig, stream, false);
}

// Record the tile-phase time of a finished autotuning trial.
void finish_trial(rqa_handle *h) {
    if (!h->trial) return;
    h->trial = false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->prof.ev[1], h->prof.ev[2]) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneEntry &e = g_tune[h->trial_key];
    const int w = h->trial_waves;
    if (e.done || e.ncand == 0 || e.cand[e.next] != w) return;
    if (ms < e.best_ms) {
        e.best_ms = ms;
        e.best = w;
    } else if (ms > kGiveUp * e.best_ms && w != e.dflt) {
        // drop the untried shapes beyond this one, on its side of the default
        int keep = e.next + 1;
        for (int k = e.next + 1; k < e.ncand; ++k) {
            const bool beyond = w < e.dflt ? e.cand[k] < w : e.cand[k] > w;
            if (!beyond) e.cand[keep++] = e.cand[k];
        }
        e.ncand = keep;
    }
    if (++e.next >= e.ncand) {
        e.done = true;
        tune_store_locked(h->trial_key, e.best);
    }
}

int fetch(rqa_handle *h, int32_t index, rqa_measures *out, uint64_t *diag, uint64_t *vert,
          uint64_t *white, int64_t hist_len) {
    if (!h) return RQA_EINVAL;
    if (!h->has_run) return RQA_ESTATE;
    if (index < 0 || index >= static_cast<int32_t>(h->nvec.size())) return RQA_EINVAL;
    const int64_t n = h->nvec[index];
    const int64_t hl = h->hlen[index];
    if ((diag || vert || white) && hist_len < hl) return RQA_ESIZE;
    // Grow a pinned host buffer.
    auto grow = [](void **buf, size_t *have, size_t need) -> int {
        if (*have >= need) return RQA_OK;
        if (*buf) hipHostFree(*buf);
        *buf = nullptr;
        *have = 0;
        if (hipHostMalloc(buf, need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return RQA_ENOMEM;
        }
        *have = need;
        return RQA_OK;
    };
    const size_t info_bytes = kInfoBytes * h->nvec.size();
    if (!h->info_valid) {
        // One copy of every job's flag and statistics.
        int rc = grow(reinterpret_cast<void **>(&h->info_cache), &h->info_cache_bytes, info_bytes);
        if (rc != RQA_OK) return rc;
        if (hipMemcpyAsync(h->info_cache, static_cast<const char *>(h->ws.base) + h->info_block_off,
                           info_bytes, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return RQA_EDEVICE;
        finish_trial(h);
        h->info_valid = true;
    }
    const char *info = h->info_cache + kInfoBytes * static_cast<size_t>(index);
    int flag = 0;
    std::memcpy(&flag, info, sizeof(int));
    if (flag & 1) return RQA_ENONFINITE;
    if (flag) return RQA_EDEVICE;   // internal consistency check failed on the device
    if (diag || vert || white) {
        // Entries above a histogram's longest line are zero (the device
        // statistics hold the longest lines), so only the prefixes cross PCIe
        // and the tails are cleared on the host.  A launch of one job copies
        // its three prefixes; a batch copies the block of all its jobs once.
        JobStats st;
        std::memcpy(&st, info + 8, sizeof st);
        int64_t used[3];
        for (int k = 0; k < 3; ++k)
            used[k] = std::min<int64_t>(hl, static_cast<int64_t>(st.longest[k]) + 1);
        const bool single = h->nvec.size() == 1;
        if (!h->cache_valid) {
            int rc = grow(reinterpret_cast<void **>(&h->host_cache), &h->host_cache_bytes,
                          h->hist_block_bytes);
            if (rc != RQA_OK) return rc;
            const char *dev = static_cast<const char *>(h->ws.base) + h->hist_block_off;
            bool ok = true;
            if (single) {
                for (int k = 0; k < 3 && ok; ++k)
                    ok = hipMemcpyAsync(reinterpret_cast<char *>(h->host_cache) +
                                            sizeof(uint64_t) * k * hl,
                                        dev + sizeof(uint64_t) * k * hl, sizeof(uint64_t) * used[k],
                                        hipMemcpyDeviceToHost, h->stream) == hipSuccess;
            } else {
                ok = hipMemcpyAsync(h->host_cache, dev, h->hist_block_bytes, hipMemcpyDeviceToHost,
                                    h->stream) == hipSuccess;
            }
            if (!ok || hipStreamSynchronize(h->stream) != hipSuccess) return RQA_EDEVICE;
            h->cache_valid = true;
        }
        const uint64_t *hd = reinterpret_cast<const uint64_t *>(
            reinterpret_cast<const char *>(h->host_cache) + (h->job_off[index] - h->hist_block_off));
        uint64_t *dst[3] = {diag, vert, white};
        for (int k = 0; k < 3; ++k) {
            if (!dst[k]) continue;
            std::memcpy(dst[k], hd + k * hl, sizeof(uint64_t) * used[k]);
            std::memset(dst[k] + used[k], 0, sizeof(uint64_t) * (hl - used[k]));
        }
    }
    if (out) {
        JobStats st;
        std::memcpy(&st, info + 8, sizeof st);
        measures_from_stats(st, n, h->ncols[index], h->p, out);
    }
    return RQA_OK;
}

}  // namespace

extern "C" {

int rqa_create(rqa_handle **out, int32_t m, int32_t tau, float eps, int32_t norm, int32_t lmin,
               int32_t vmin, int32_t wmin, int32_t theiler) {
    if (!out) return RQA_EINVAL;
    rqa_params p{m, tau, eps, norm, lmin, vmin, wmin, theiler};
    const int rc = validate_params(p);
    if (rc != RQA_OK) return rc;
    rqa_handle *h = new (std::nothrow) rqa_handle;
    if (!h) return RQA_ENOMEM;
    h->p = p;
    *out = h;
    return RQA_OK;
}

int rqa_hist_len(const rqa_handle *h, int64_t n_points, int64_t *len) {
    if (!h || !len) return RQA_EINVAL;
    const int64_t nv = n_points - static_cast<int64_t>(h->p.m - 1) * h->p.tau;
    if (nv < 1) return RQA_ETOOSHORT;
    *len = nv + 1;
    return RQA_OK;
}

int rqa_run(rqa_handle *h, const float *d_series, int64_t n_points, void *hip_stream) {
    if (!h) return RQA_EINVAL;
    if (n_points < 0) return RQA_EINVAL;
    return enqueue(h, d_series, n_points, nullptr, nullptr, 1, hip_stream, false);
}

int rqa_cross_hist_len(const rqa_handle *h, int64_t na_points, int64_t nb_points, int64_t *len) {
    if (!h || !len) return RQA_EINVAL;
    const int64_t d = static_cast<int64_t>(h->p.m - 1) * h->p.tau;
    const int64_t na = na_points - d, nb = nb_points - d;
    if (na < 1 || nb < 1) return RQA_ETOOSHORT;
    *len = std::max(na, nb) + 1;
    return RQA_OK;
}

int rqa_run_cross(rqa_handle *h, const float *d_a, int64_t na_points, const float *d_b,
                  int64_t nb_points, void *hip_stream) {
    if (!h || !d_a || !d_b || na_points < 0 || nb_points < 0) return RQA_EINVAL;
    const int64_t d = static_cast<int64_t>(h->p.m - 1) * h->p.tau;
    Job jb;
    jb.mode = kModeCross;
    jb.series = d_a;
    jb.n_points = na_points;
    jb.n_vec = na_points - d;
    jb.series_b = d_b;
    jb.n_points_b = nb_points;
    jb.n_cols = nb_points - d;
    if (jb.n_vec < 1 || jb.n_cols < 1) return RQA_ETOOSHORT;
    return enqueue_full(h, jb, hip_stream);
}

int rqa_run_matrix(rqa_handle *h, const uint64_t *d_bits, int64_t n_rows, int64_t n_cols,
                   int64_t words_per_row, void *hip_stream) {
    if (!h || !d_bits || n_rows < 1 || n_cols < 1 || words_per_row < (n_cols + 63) / 64)
        return RQA_EINVAL;
    Job jb;
    jb.mode = kModeMatrix;
    jb.n_vec = n_rows;
    jb.n_cols = n_cols;
    jb.bits = d_bits;
    jb.words = words_per_row;
    return enqueue_full(h, jb, hip_stream);
}

namespace {

// Enqueue a recurrence plot; the tail scratch is reused, so a plot waits (on the
// device) for the previous one of this handle.
int plot(rqa_handle *h, const float *a, int64_t na_points, const float *b, int64_t nb_points,
         uint64_t *d_bits, int64_t words, void *hip_stream) {
    const KParams kp = make_kparams(h->p);
    const int64_t d = static_cast<int64_t>(h->p.m - 1) * h->p.tau;
    const int64_t na = na_points - d, nb = b ? nb_points - d : na;
    if (na < 1 || nb < 1) return RQA_ETOOSHORT;
    if (na > (int64_t(1) << 31) - 2 || nb > (int64_t(1) << 31) - 2) return RQA_EINVAL;
    if (words < (nb + 63) / 64) return RQA_ESIZE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t need = sizeof(float) * static_cast<size_t>(engine_plot_scratch_floats(kp, nb));
    if (!h->plot_done && hipEventCreateWithFlags(&h->plot_done, hipEventDisableTiming) != hipSuccess)
        return RQA_EDEVICE;
    if (h->plot_tail_bytes < need) {
        if (h->plot_tail) {
            hipEventSynchronize(h->plot_done);
            hipFree(h->plot_tail);
        }
        h->plot_tail = nullptr;
        h->plot_tail_bytes = 0;
        if (hipMalloc(&h->plot_tail, need) != hipSuccess) {
            (void)hipGetLastError();
            return RQA_ENOMEM;
        }
        h->plot_tail_bytes = need;
    } else if (hipStreamWaitEvent(st, h->plot_done, 0) != hipSuccess) {
        return RQA_EDEVICE;
    }
    const int rc = engine_plot(kp, a, na_points, b, nb_points, d_bits, words, h->plot_tail, st);
    if (rc != RQA_OK) return rc;
    return hipEventRecord(h->plot_done, st) == hipSuccess ? RQA_OK : RQA_EDEVICE;
}

}  // namespace

int rqa_plot(rqa_handle *h, const float *d_series, int64_t n_points, uint64_t *d_bits,
             int64_t words_per_row, void *hip_stream) {
    if (!h || !d_series || !d_bits || n_points < 0 || words_per_row < 1) return RQA_EINVAL;
    return plot(h, d_series, n_points, nullptr, 0, d_bits, words_per_row, hip_stream);
}

int rqa_plot_cross(rqa_handle *h, const float *d_a, int64_t na_points, const float *d_b,
                   int64_t nb_points, uint64_t *d_bits, int64_t words_per_row, void *hip_stream) {
    if (!h || !d_a || !d_b || !d_bits || na_points < 0 || nb_points < 0 || words_per_row < 1)
        return RQA_EINVAL;
    return plot(h, d_a, na_points, d_b, nb_points, d_bits, words_per_row, hip_stream);
}

int rqa_result(rqa_handle *h, rqa_measures *out, uint64_t *diag, uint64_t *vert, uint64_t *white,
               int64_t hist_len) {
    if (h && h->has_run && h->batched) return RQA_ESTATE;
    return fetch(h, 0, out, diag, vert, white, hist_len);
}

int rqa_run_batch(rqa_handle *h, const float *d_series, int64_t n_points, const int64_t *offsets,
                  const int64_t *lengths, int32_t count, void *hip_stream) {
    if (!h || !offsets || !lengths || count < 1 || n_points < 0) return RQA_EINVAL;
    return enqueue(h, d_series, n_points, offsets, lengths, count, hip_stream, true);
}

int rqa_result_batch(rqa_handle *h, int32_t index, rqa_measures *out, uint64_t *diag,
                     uint64_t *vert, uint64_t *white, int64_t hist_len) {
    return fetch(h, index, out, diag, vert, white, hist_len);
}

int rqa_result_batch_all(rqa_handle *h, rqa_measures *out, int32_t *status, int32_t count) {
    if (!h || !out || count < 1) return RQA_EINVAL;
    if (!h->has_run) return RQA_ESTATE;
    if (count != static_cast<int32_t>(h->nvec.size())) return RQA_ESIZE;
    int first = RQA_OK;
    for (int32_t k = 0; k < count; ++k) {
        const int rc = fetch(h, k, &out[k], nullptr, nullptr, nullptr, 0);
        if (rc != RQA_OK) {
            // No result for this window: NaN measures, nothing recurrent.
            const double nan = std::numeric_limits<double>::quiet_NaN();
            out[k] = rqa_measures{nan, nan, nan, nan, nan, nan, nan, nan, nan, nan, nan, nan, nan,
                                  0u, h->nvec[k]};
            if (first == RQA_OK) first = rc;
        }
        if (status) status[k] = rc;
    }
    return first;
}

int rqa_measures_from_hist(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                           int64_t n, const rqa_params *p, rqa_measures *out) {
    if (!diag || !vert || !white || !p || !out || n < 1) return RQA_EINVAL;
    const int rc = validate_params(*p);
    if (rc != RQA_OK) return rc;
    measures_from_hist(diag, vert, white, n, *p, out);
    return RQA_OK;
}

int rqa_set_tiling(rqa_handle *h, int32_t waves_per_group, int32_t groups) {
    if (!h || waves_per_group < 0 || waves_per_group > 8 || groups < 0) return RQA_EINVAL;
    h->waves = waves_per_group;
    h->groups = groups;
    return RQA_OK;
}

int rqa_set_profiling(rqa_handle *h, int32_t enable) {
    if (!h) return RQA_EINVAL;
    h->profiling = enable != 0;
    h->prof_valid = false;
    return RQA_OK;
}

int rqa_get_timings(rqa_handle *h, double *prepare_ms, double *tiles_ms, double *stitch_ms) {
    if (!h) return RQA_EINVAL;
    if (!h->prof_valid) return RQA_ESTATE;
    if (hipEventSynchronize(h->prof.ev[3]) != hipSuccess) return RQA_EDEVICE;
    float a = 0.f, b = 0.f, c = 0.f;
    if (hipEventElapsedTime(&a, h->prof.ev[0], h->prof.ev[1]) != hipSuccess ||
        hipEventElapsedTime(&b, h->prof.ev[1], h->prof.ev[2]) != hipSuccess ||
        hipEventElapsedTime(&c, h->prof.ev[2], h->prof.ev[3]) != hipSuccess)
        return RQA_EDEVICE;
    if (prepare_ms) *prepare_ms = a;
    if (tiles_ms) *tiles_ms = b;
    if (stitch_ms) *stitch_ms = c;
    return RQA_OK;
}

int rqa_last_launch(const rqa_handle *h, int32_t *waves, int32_t *graph_replay) {
    if (!h) return RQA_EINVAL;
    if (!h->has_run) return RQA_ESTATE;
    if (waves) *waves = h->trial_waves;
    if (graph_replay) *graph_replay = h->last_from_graph ? 1 : 0;
    return RQA_OK;
}

int rqa_workspace_plan(const rqa_params *p, int64_t n_points, int32_t waves, int64_t limit_bytes,
                       int32_t *bands, int32_t *band_strips, int32_t *segs,
                       int64_t *workspace_bytes) {
    if (!p || waves < 0 || waves > 8 || limit_bytes < 0) return RQA_EINVAL;
    int rc = validate_params(*p);
    if (rc != RQA_OK) return rc;
    const int64_t nv = n_points - static_cast<int64_t>(p->m - 1) * p->tau;
    if (nv < 1) return RQA_ETOOSHORT;
    if (nv > (int64_t(1) << 31) - 2) return RQA_EINVAL;
    Job jb;
    jb.n_points = n_points;
    jb.n_vec = nv;
    jb.n_cols = nv;
    jb.kp = make_kparams(*p);
    jb.waves = waves > 0 ? waves : engine_default_waves(nv);
    jb.band_strips = engine_band_strips(jb, static_cast<size_t>(limit_bytes));
    const JobPlan plan = engine_job_plan(jb);
    if (bands) *bands = plan.bands;
    if (band_strips) *band_strips = plan.band_strips;
    if (segs) *segs = plan.segs;
    if (workspace_bytes) *workspace_bytes = static_cast<int64_t>(plan.scratch_bytes);
    return RQA_OK;
}

int rqa_set_workspace_limit(rqa_handle *h, int64_t bytes) {
    if (!h || bytes < 0) return RQA_EINVAL;
    h->ws_limit = bytes;
    return RQA_OK;
}

int rqa_last_plan(const rqa_handle *h, int32_t *bands, int32_t *band_strips, int32_t *segs,
                  int32_t *strip_rows, int64_t *workspace_bytes) {
    if (!h) return RQA_EINVAL;
    if (!h->has_run) return RQA_ESTATE;
    if (bands) *bands = h->plan.bands;
    if (band_strips) *band_strips = h->plan.band_strips;
    if (segs) *segs = h->plan.segs;
    if (strip_rows) *strip_rows = h->plan.strip_rows;
    if (workspace_bytes) *workspace_bytes = static_cast<int64_t>(h->plan.scratch_bytes);
    return RQA_OK;
}

void rqa_destroy(rqa_handle *h) {
    if (!h) return;
    if (h->has_run) hipStreamSynchronize(h->stream);
    if (h->staging) hipHostFree(h->staging);
    if (h->staging_free) hipEventDestroy(h->staging_free);
    for (hipEvent_t e : h->prof.ev)
        if (e) hipEventDestroy(e);
    drop_graph(h);
    if (h->capture_stream) hipStreamDestroy(h->capture_stream);
    if (h->host_cache) hipHostFree(h->host_cache);
    if (h->info_cache) hipHostFree(h->info_cache);
    if (h->plot_done) {
        hipEventSynchronize(h->plot_done);
        hipEventDestroy(h->plot_done);
    }
    if (h->plot_tail) hipFree(h->plot_tail);
    delete h;
}

const char *rqa_strerror(int code) {
    switch (code) {
        case RQA_OK: return "ok";
        case RQA_EINVAL: return "invalid argument";
        case RQA_ETOOSHORT: return "series too short for the embedding (fewer than one delay vector)";
        case RQA_ENOMEM: return "out of memory";
        case RQA_EDEVICE: return "HIP device error";
        case RQA_ENONFINITE: return "series contains NaN or infinity";
        case RQA_ESIZE: return "output buffer too small";
        case RQA_ESTATE: return "invalid call order";
        case RQA_EBUDGET: return "job exceeds the memory budget (server pool or static scratch)";
        case RQA_EAGAIN: return "job not finished";
        case RQA_ENOTFOUND: return "unknown ticket";
        default: return "unknown error";
    }
}

}  // extern "C"
