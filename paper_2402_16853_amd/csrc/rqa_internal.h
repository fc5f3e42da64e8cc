// Internal declarations shared by the host runtime and the kernel launchers of
// librqa.  Not part of the public ABI (see include/rqa.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "rqa.h"

namespace rqa {

// Parameters in the form the kernels consume.
struct KParams {
    int32_t m;
    int32_t tau;
    float eps;      // L1 / Linf threshold
    float eps_sq;   // fl32(eps*eps), L2 threshold on the squared sum
    float d0_bound; // |d_0| above this makes a pair non-recurrent whatever the
                    // other coordinates (L1, Linf: eps; L2: the largest t with
                    // fl32(t*t) <= eps_sq)
    int32_t norm;
    int32_t theiler;
    int32_t lmin, vmin, wmin;   // minimum diagonal / vertical / white line lengths
};

// Per-job summary of the three histograms, reduced on the device: exact integer
// moments and longest lines, and the FP64 entropies of the lines at or above the
// minimum lengths (index 0 diagonal, 1 vertical, 2 white vertical).
struct JobStats {
    uint64_t cnt_all[3];    // number of lines
    uint64_t mass_all[3];   // sum of their lengths
    uint64_t cnt_min[3];    // number of lines of length >= minimum
    uint64_t mass_min[3];   // sum of their lengths
    uint64_t longest[3];    // longest line (0 if none)
    double ent[3];          // -sum p ln p over lengths >= minimum, p = count / cnt_min
};

// Bytes of the per-job info record: int flag at offset 0, JobStats at 8.
constexpr size_t kInfoBytes = 256;
static_assert(8 + sizeof(JobStats) <= kInfoBytes, "info record too small");

KParams make_kparams(const rqa_params &p);

// What a job's matrix is.
enum JobMode : int32_t {
    kModeAuto = 0,     // recurrence matrix of one series (symmetric; upper triangle evaluated)
    kModeCross = 1,    // cross recurrence matrix: rows from series a, columns from series b
    kModeMatrix = 2,   // a given bit matrix (row-major 64-bit words)
};

// One independent RQA problem inside a launch: a window of a device series, a
// pair of series (cross recurrence) or a given bit matrix.
struct Job {
    int32_t mode = kModeAuto;
    const float *series = nullptr;  // first point of the window (device); rows' series
    int64_t n_points = 0;           // points in the window
    int64_t n_vec = 0;              // delay vectors (rows)
    const float *series_b = nullptr;   // cross: columns' series (device)
    int64_t n_points_b = 0;
    int64_t n_cols = 0;             // columns (auto: n_vec)
    const uint64_t *bits = nullptr; // given matrix (device): n_vec rows of `words` u64
    int64_t words = 0;
    uint64_t *hist = nullptr;       // device: 3*hist_len() u64 -- diag | vert | white
    int *flag = nullptr;            // device info record (kInfoBytes): flag at 0, JobStats at 8
    void *scratch = nullptr;        // device: engine_job_scratch_bytes(*this) bytes
    void *stats = nullptr;          // device JobStats record (nullptr: at flag + 8)
    int64_t hist_stride = 0;        // entries from one histogram to the next (0: hist_len())
    KParams kp{};                   // parameters of this job
    int waves = 0;                  // waves per workgroup (strip height 64*waves), > 0
    int segs = 0;                   // auto mode: column segments per strip (0: the engine
                                    // decides, 1 for a job launched with others); scratch
                                    // is sized for the largest choice
    int band_strips = 0;            // auto mode, a job launched alone: strips per row
                                    // band (0: one band).  The strip-edge summaries then
                                    // hold one band's strips and per-line carries pass
                                    // the open runs from band to band
    // Histogram entries (index = line length, 0 unused): longest line + 1.
    int64_t hist_len() const {
        return (mode == kModeAuto ? n_vec : (n_cols > n_vec ? n_cols : n_vec)) + 1;
    }
};

// Device workspace owned by a handle (or a served job); grown on demand.
struct Workspace {
    int device = -1;
    void *base = nullptr;
    size_t bytes = 0;
    ~Workspace();
    int reserve(size_t need);   // RQA_OK / RQA_ENOMEM / RQA_EDEVICE
};

// Device scratch one job needs beyond its histograms and flag (segment
// summaries and line-end records), and the per-launch scratch (work
// descriptors and the work counter) of a launch over `njobs` jobs.
size_t engine_job_scratch_bytes(const Job &job);
size_t engine_launch_scratch_bytes(size_t njobs);

// Row bands for a job (auto mode) launched alone whose scratch would exceed
// `limit` bytes: the largest number of strips per band whose scratch fits, at
// least 1; 0 when the job fits in one band or `limit` is 0.  The job's waves
// (strip height) must be set.
int engine_band_strips(const Job &job, size_t limit);

// How a launch of `job` alone is cut: row bands, strips per band, column
// segments per strip, strip height, and the job's scratch bytes.
struct JobPlan {
    int bands, band_strips, segs, strip_rows;
    size_t scratch_bytes;
};
JobPlan engine_job_plan(const Job &job);

// Default waves per workgroup for a job of n delay vectors.
int engine_default_waves(int64_t n);

// Optional phase events recorded on the launch stream: [0] before preparation,
// [1] before the tile kernel(s), [2] after them, [3] after the stitch kernel.
struct PhaseEvents {
    hipEvent_t ev[4];
};

// Enqueue the full hot path for all jobs on `stream` as one batched pass:
// validation, zeroing, the fused tile kernel, the stitch/join kernel.
// `launch_scratch` holds engine_launch_scratch_bytes(jobs.size()) device bytes;
// `staging` is pinned host memory of the same size; `staging_free` (may be
// null) is an event the engine waits on before rewriting `staging` and records
// once the launch has consumed it.  Each job's `waves` fixes its strip height;
// jobs are grouped per (norm, m, waves) into one tile-kernel launch each.
// groups = 0 sizes each tile launch to fill the device.
// Optional auxiliary streams: when a launch holds jobs of several (norm, m,
// waves) groups, their tile kernels fork onto these streams and join back, so
// small groups share the device instead of running one after another.
struct AuxStreams {
    static constexpr int kMax = 4;
    int count = 0;
    hipStream_t s[kMax] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMax] = {};
    int create(int n);    // RQA_OK or RQA_EDEVICE
    void destroy();
};

int engine_launch(const std::vector<Job> &jobs, void *launch_scratch, void *staging,
                  hipEvent_t staging_free, int groups, hipStream_t stream,
                  const PhaseEvents *phases = nullptr, AuxStreams *aux = nullptr);

// The launch of one job (auto mode) without host staging: descriptors are
// written by a kernel from its arguments and every scratch byte lies in
// `scratch` (engine_static_bytes(jb) device bytes): the job's histograms
// (jb.hist, stride jb.hist_stride) and flag (jb.flag) are the caller's.  No
// allocation, no host-to-device copy.
size_t engine_static_bytes(const Job &jb);
int engine_launch_static(Job jb, void *scratch, hipStream_t stream);

// Recurrence plot: the masked matrix of series a (b == nullptr) or the cross
// matrix of a and b, bit-packed into `bits` (rows of `words` u64), on `stream`.
// `scratch` holds engine_plot_scratch_floats(kp, nb) device floats (the last
// column tile's coordinates and the column boxes of the exact tile pruning),
// nb being the number of column vectors.
int64_t engine_plot_scratch_floats(const KParams &kp, int64_t nb);
int engine_plot(const KParams &kp, const float *a, int64_t na_points, const float *b,
                int64_t nb_points, uint64_t *bits, int64_t words, float *scratch,
                hipStream_t stream);

// Host FP64 measures from histograms of length n+1.
void measures_from_hist(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                        int64_t n, const rqa_params &p, rqa_measures *out);

// Host FP64 measures from the device-reduced statistics of an n_rows x n_cols
// matrix (n_cols = n_rows for the recurrence matrix of one series).
void measures_from_stats(const JobStats &st, int64_t n_rows, int64_t n_cols, const rqa_params &p,
                         rqa_measures *out);

int validate_params(const rqa_params &p);

}  // namespace rqa
