// C ABI of librqa: parameter validation, device workspace, enqueue of the hot
// path on the caller's stream, and result retrieval (Sect. 7: Settings ->
// RQAComputation.create -> run -> RQAResult; missing devices and invalid input
// are reported as errors, never aborts).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
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

struct rqa_handle {
    rqa_params p{};
    Workspace ws;
    void *staging = nullptr;        // pinned host buffer for launch descriptors
    size_t staging_bytes = 0;
    hipEvent_t staging_free = nullptr;   // recorded when a launch has read `staging`
    bool profiling = false;
    bool prof_valid = false;
    PhaseEvents prof{};
    int waves = 0;                  // 0 = default tiling
    int groups = 0;                 // 0 = one workgroup per compute unit
    bool has_run = false;
    bool batched = false;
    hipStream_t stream = nullptr;
    std::vector<int64_t> nvec;      // per job
    std::vector<size_t> job_off;    // per job: byte offset of its region in ws.base
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr size_t kFlagBytes = 256;

int enqueue(rqa_handle *h, const float *d_series, int64_t n_points, const int64_t *offsets,
            const int64_t *lengths, int32_t count, void *stream, bool batched) {
    if (!h || !d_series) return RQA_EINVAL;
    std::vector<Job> jobs(count);
    const KParams kp = make_kparams(h->p);
    std::vector<int64_t> nvec(count);
    std::vector<size_t> off(count);
    size_t total = align256(engine_launch_scratch_bytes(count));
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
        jb.kp = kp;
        nvec[w] = nv;
        off[w] = total;
        total += align256(sizeof(uint64_t) * 3 * static_cast<size_t>(nv + 1)) + kFlagBytes +
                 align256(engine_job_scratch_bytes(jb, h->waves));
    }
    int rc = h->ws.reserve(total);
    if (rc != RQA_OK) return rc;
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
        char *p = base + off[w];
        const size_t hb = align256(sizeof(uint64_t) * 3 * static_cast<size_t>(jb.n_vec + 1));
        jb.hist = reinterpret_cast<uint64_t *>(p);
        jb.flag = reinterpret_cast<int *>(p + hb);
        jb.scratch = p + hb + kFlagBytes;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (h->profiling && !h->prof.ev[0]) {
        for (hipEvent_t &e : h->prof.ev)
            if (hipEventCreate(&e) != hipSuccess) return RQA_EDEVICE;
    }
    rc = engine_launch(jobs, base, h->staging, h->staging_free, h->waves, h->groups, st,
                       h->profiling ? &h->prof : nullptr);
    h->prof_valid = h->profiling && rc == RQA_OK;
    if (rc != RQA_OK) return rc;
    h->nvec = std::move(nvec);
    h->job_off = std::move(off);
    h->stream = st;
    h->has_run = true;
    h->batched = batched;
    return RQA_OK;
}

int fetch(rqa_handle *h, int32_t index, rqa_measures *out, uint64_t *diag, uint64_t *vert,
          uint64_t *white, int64_t hist_len) {
    if (!h) return RQA_EINVAL;
    if (!h->has_run) return RQA_ESTATE;
    if (index < 0 || index >= static_cast<int32_t>(h->nvec.size())) return RQA_EINVAL;
    const int64_t n = h->nvec[index];
    if ((diag || vert || white) && hist_len < n + 1) return RQA_ESIZE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return RQA_EDEVICE;
    const char *p = static_cast<const char *>(h->ws.base) + h->job_off[index];
    const size_t hb = align256(sizeof(uint64_t) * 3 * static_cast<size_t>(n + 1));
    int flag = 0;
    if (hipMemcpy(&flag, p + hb, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return RQA_EDEVICE;
    if (flag & 1) return RQA_ENONFINITE;
    if (flag) return RQA_EDEVICE;   // internal consistency check failed on the device
    std::vector<uint64_t> host(static_cast<size_t>(3 * (n + 1)));
    if (hipMemcpy(host.data(), p, host.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return RQA_EDEVICE;
    const uint64_t *hd = host.data(), *hv = hd + (n + 1), *hw = hv + (n + 1);
    if (diag) std::memcpy(diag, hd, sizeof(uint64_t) * (n + 1));
    if (vert) std::memcpy(vert, hv, sizeof(uint64_t) * (n + 1));
    if (white) std::memcpy(white, hw, sizeof(uint64_t) * (n + 1));
    if (out) measures_from_hist(hd, hv, hw, n, h->p, out);
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

int rqa_measures_from_hist(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                           int64_t n, const rqa_params *p, rqa_measures *out) {
    if (!diag || !vert || !white || !p || !out || n < 1) return RQA_EINVAL;
    const int rc = validate_params(*p);
    if (rc != RQA_OK) return rc;
    measures_from_hist(diag, vert, white, n, *p, out);
    return RQA_OK;
}

int rqa_set_tiling(rqa_handle *h, int32_t waves_per_group, int32_t groups) {
    if (!h || waves_per_group < 0 || waves_per_group > 16 || groups < 0) return RQA_EINVAL;
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

void rqa_destroy(rqa_handle *h) {
    if (!h) return;
    if (h->has_run) hipStreamSynchronize(h->stream);
    if (h->staging) hipHostFree(h->staging);
    if (h->staging_free) hipEventDestroy(h->staging_free);
    for (hipEvent_t e : h->prof.ev)
        if (e) hipEventDestroy(e);
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
        case RQA_EBUDGET: return "job exceeds the server memory budget";
        case RQA_EAGAIN: return "job not finished";
        case RQA_ENOTFOUND: return "unknown ticket";
        default: return "unknown error";
    }
}

}  // extern "C"
