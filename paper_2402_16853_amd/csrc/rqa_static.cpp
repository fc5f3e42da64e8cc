// rqa_run_static: the whole RQA of one device series with no allocation of any
// kind.  Every byte of device scratch the kernels need (launch descriptors,
// work counters, the statistics record, the tail copy, the row-lead records
// and the strip-edge summaries) lies in one file-scope device array of
// RQA_STATIC_SCRATCH_BYTES, which each GPU the library runs on holds until the
// process ends; the caller passes the series and the output histograms and
// flag.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rqa_internal.h"

// The scratch array.  In host code its name is only a stand-in: the device
// address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[RQA_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device with
// that device current.
int scratch_on_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return RQA_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return RQA_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RQA_OK;
}

}  // namespace

extern "C" int rqa_run_static(const rqa_params *p, const float *d_series, int64_t n_points,
                              uint64_t *d_hist, int64_t hist_len, int32_t *d_flag,
                              void *hip_stream) {
    using namespace rqa;
    if (!p || !d_series || !d_hist || !d_flag || n_points < 0) return RQA_EINVAL;
    int rc = validate_params(*p);
    if (rc != RQA_OK) return rc;
    const int64_t nv = n_points - static_cast<int64_t>(p->m - 1) * p->tau;
    if (nv < 1) return RQA_ETOOSHORT;
    if (nv > (int64_t(1) << 31) - 2) return RQA_EINVAL;
    if (hist_len < nv + 1) return RQA_ESIZE;
    Job jb;
    jb.mode = kModeAuto;
    jb.series = d_series;
    jb.n_points = n_points;
    jb.n_vec = nv;
    jb.n_cols = nv;
    jb.kp = make_kparams(*p);
    jb.waves = engine_default_waves(nv);
    jb.segs = 1;   // whole strips: the least scratch
    jb.hist = d_hist;
    jb.hist_stride = hist_len;
    jb.flag = reinterpret_cast<int *>(d_flag);
    if (engine_static_bytes(jb) > RQA_STATIC_SCRATCH_BYTES) return RQA_EBUDGET;
    void *base = nullptr;
    rc = scratch_on_current_device(&base);
    if (rc != RQA_OK) return rc;
    return engine_launch_static(jb, base, static_cast<hipStream_t>(hip_stream));
}
