/*
 * rqa.h -- C ABI of librqa: recurrence quantification analysis (RQA) of FP32
 * time series on an MI355X (gfx950) GPU.
 *
 * Method (Rawald, Sips, Marwan, "PyRQA - Conducting Recurrence Quantification
 * Analysis on Very Long Time Series Efficiently"):
 *   Sect. 2   time-delay embedding, similarity of vector pairs under a norm,
 *             fixed-radius neighbourhood -> binary recurrence matrix; diagonal,
 *             vertical and white vertical lines; their frequency distributions
 *             and the measures derived from them;
 *   Sect. 4.2 the three operators (create the recurrence matrix, detect diagonal
 *             lines, detect vertical lines) -- fused here into one pass over
 *             tiles of the upper triangle; the N x N matrix is never stored;
 *   Sect. 4.1 divide & recombine with carry-over of lines that cross tile
 *             borders;
 *   Sect. 7.2 the parameter set (embedding_dimension, time_delay,
 *             similarity_measure, FixedRadius(radius), minimum diagonal,
 *             vertical and white vertical line lengths);
 *   Sect. 8.1 Tab. 3 the measure names (RR, DET, L, Lmax, DIV, L_entr, LAM, TT,
 *             Vmax, V_entr).
 *
 * Conventions (identical in every entry point):
 *  - n_points is the length of the scalar series; the number of delay vectors is
 *    n = n_points - (m-1)*tau.
 *  - Cell (i,j) is recurrent when the norm of x_i - x_j, accumulated in FP32 in
 *    ascending coordinate order without fused multiply-add, is <= eps (for L2
 *    the squared sum is compared with fl32(eps*eps)); cells with |i-j| < theiler
 *    are forced to 0.  The matrix is symmetric.
 *  - Histograms cover the whole n x n masked matrix (both triangles, runs that
 *    touch the border included) and are indexed by line length: entry l counts
 *    the lines of length l, entry 0 is always 0; length n+1 arrays.
 *  - Device pointers are hipMalloc'd (or PyTorch CUDA tensor) memory on the
 *    current HIP device; host pointers are ordinary host memory.
 *  - Every function returns RQA_OK (0) or a negative RQA_E* code; nothing
 *    aborts.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef RQA_H
#define RQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define RQA_OK 0
#define RQA_EINVAL (-1)      /* an argument is out of range or a pointer is NULL   */
#define RQA_ETOOSHORT (-2)   /* n_points gives fewer than one delay vector          */
#define RQA_ENOMEM (-3)      /* device or host allocation failed                     */
#define RQA_EDEVICE (-4)     /* a HIP call, a launch or a device-side check failed  */
#define RQA_ENONFINITE (-5)  /* the series holds NaN or +-Inf (detected on device)   */
#define RQA_ESIZE (-6)       /* a caller buffer is shorter than required             */
#define RQA_ESTATE (-7)      /* call order violated (e.g. result before run)         */
#define RQA_EBUDGET (-8)     /* a job needs more device memory than the server owns
                                or than rqa_run_static's scratch holds             */
#define RQA_EAGAIN (-9)      /* a served job is not finished yet                     */
#define RQA_ENOTFOUND (-10)  /* unknown ticket                                       */

/* Similarity measures (Sect. 7.2: L1, L2 and L-infinity norms). */
#define RQA_NORM_L1 1
#define RQA_NORM_L2 2
#define RQA_NORM_LINF 3

/* RQA parameters, the fields of PyRQA's Settings (Sect. 7.2) plus a Theiler
 * window.  m >= 1, tau >= 1, eps finite and >= 0, norm in {1,2,3},
 * lmin/vmin/wmin >= 1, theiler >= 0. */
typedef struct rqa_params {
    int32_t m;        /* embedding dimension                                 */
    int32_t tau;      /* time delay                                          */
    float eps;        /* fixed radius                                        */
    int32_t norm;     /* RQA_NORM_*                                          */
    int32_t lmin;     /* minimum diagonal line length                        */
    int32_t vmin;     /* minimum vertical line length                        */
    int32_t wmin;     /* minimum white vertical line length                  */
    int32_t theiler;  /* cells with |i-j| < theiler are not recurrences      */
} rqa_params;

/* Measures in FP64, computed on the host from the integer histograms D (diag),
 * V (vert), W (white).  N_rec = sum l*D(l); A = n^2 minus the Theiler band.
 *   rr = N_rec/A; det = sum_{l>=lmin} l D / N_rec; l = sum_{l>=lmin} l D / sum_{l>=lmin} D;
 *   lmax = max{l: D(l)>0}; div = 1/lmax; l_entr = -sum p ln p over l >= lmin;
 *   lam = sum_{v>=vmin} v V / sum v V; tt = sum_{v>=vmin} v V / sum_{v>=vmin} V;
 *   vmax, v_entr likewise; w = sum_{w>=wmin} w W / sum_{w>=wmin} W; wmax, w_entr.
 * A ratio with a zero denominator is NaN. */
typedef struct rqa_measures {
    double rr, det, l, lmax, div, l_entr, lam, tt, vmax, v_entr, w, wmax, w_entr;
    uint64_t n_rec;   /* number of recurrence points (both triangles)        */
    int64_t n_vec;    /* number of delay vectors n                           */
} rqa_measures;

typedef struct rqa_handle rqa_handle;

/* Create a computation for one parameter set (Sect. 7.3 RQAComputation.create).
 * On success *out owns its device workspace (allocated lazily on the first run
 * on the device that is current then).  RQA_EINVAL leaves *out untouched. */
int rqa_create(rqa_handle **out, int32_t m, int32_t tau, float eps, int32_t norm,
               int32_t lmin, int32_t vmin, int32_t wmin, int32_t theiler);

/* Histogram length n+1 for a series of n_points under h's embedding.
 * RQA_ETOOSHORT if n < 1. */
int rqa_hist_len(const rqa_handle *h, int64_t n_points, int64_t *len);

/* Enqueue the whole RQA of one device series on hip_stream (a hipStream_t;
 * NULL = the null stream) and return without waiting (Sect. 7.4 run()).
 * d_series: n_points contiguous FP32 values in device memory, owned by the
 * caller, who keeps it alive and unmodified until rqa_result returns.
 * Host-detectable errors return immediately; a non-finite series is flagged on
 * the device and reported by rqa_result. */
int rqa_run(rqa_handle *h, const float *d_series, int64_t n_points, void *hip_stream);

/* Wait for the last rqa_run (or rqa_run_cross / rqa_run_matrix), copy its
 * histograms into caller-owned HOST arrays of hist_len >= n+1 entries
 * (max(rows, columns)+1 for the full-matrix runs; any of diag/vert/white may
 * be NULL) and fill *out
 * (may be NULL).  RQA_ESTATE without a prior run, RQA_ESIZE if hist_len is too
 * small, RQA_ENONFINITE if the series held NaN/Inf. */
int rqa_result(rqa_handle *h, rqa_measures *out, uint64_t *diag, uint64_t *vert,
               uint64_t *white, int64_t hist_len);

/* Cross recurrence quantification (cRQA, Sect. 3.3: the delay vectors of two
 * series on the two axes; Sect. 4.2: a non-symmetric matrix has 2N-1 diagonals).
 * Rows are the vectors of series a, columns those of series b, both embedded
 * with h's m and tau and compared with h's norm and radius; the Theiler window
 * masks cells with |i-j| < theiler by index (0 for none).  Every diagonal
 * k = j - i in [-(n_a-1), n_b-1] and every column (over all n_a rows) is walked
 * once; runs are counted once.  d_a / d_b: na_points / nb_points contiguous FP32
 * values in device memory, owned by the caller and kept alive until
 * rqa_result returns.  Asynchronous on hip_stream like rqa_run; fetch with
 * rqa_result, whose histograms then have max(n_a, n_b)+1 entries (see
 * rqa_cross_hist_len) and whose RR is over the n_a*n_b cells outside the band;
 * rqa_measures.n_vec reports n_a.  RQA_ETOOSHORT if either series has fewer
 * points than (m-1)*tau+1. */
int rqa_run_cross(rqa_handle *h, const float *d_a, int64_t na_points, const float *d_b,
                  int64_t nb_points, void *hip_stream);

/* Histogram length max(n_a, n_b)+1 of rqa_run_cross for these series lengths. */
int rqa_cross_hist_len(const rqa_handle *h, int64_t na_points, int64_t nb_points,
                       int64_t *len);

/* Quantification of a precomputed recurrence matrix (Sect. 9 lists it among
 * the planned features): the same three histograms and measures for a given
 * n_rows x n_cols binary matrix in device memory, row-major, words_per_row
 * (>= ceil(n_cols/64)) 64-bit words per row, bit b of word c of row i = cell
 * (i, 64c+b); bits past column n_cols-1 are ignored.  The matrix is not assumed
 * symmetric: every diagonal and column is walked once.  Only h's minimum line
 * lengths and Theiler window (cells |i-j| < theiler count as 0) are used.  The
 * caller owns d_bits and keeps it alive until rqa_result returns; histograms
 * have max(n_rows, n_cols)+1 entries.  Asynchronous like rqa_run. */
int rqa_run_matrix(rqa_handle *h, const uint64_t *d_bits, int64_t n_rows, int64_t n_cols,
                   int64_t words_per_row, void *hip_stream);

/* Recurrence plot output (Sect. 4: the approach also produces recurrence
 * plots; Sect. 7 workflow: RecurrencePlotComputation / RecurrencePlotResult).
 * Writes the n x n recurrence matrix of the series under h's embedding, norm,
 * radius and Theiler window (cells |i-j| < theiler are 0) into caller-owned
 * DEVICE memory d_bits: row-major, words_per_row (>= ceil(n/64)) 64-bit words
 * per row, bit b of word c of row i = cell (i, 64c+b); bits past column n-1 are
 * 0 and words past ceil(n/64) are left unchanged.  n*words_per_row*8 bytes
 * (125 MB at n = 100,000): meant for small series and windows.  The output can
 * be fed back to rqa_run_matrix.  Asynchronous on hip_stream; the caller keeps
 * d_series and d_bits alive until the stream has passed the call.  The handle
 * keeps a device scratch buffer for the plot (the last column tile's
 * coordinates and one 32-byte record per 64 columns); a plot with more
 * columns than any before on this handle grows it (hipMalloc, after the
 * previous plot has passed), RQA_ENOMEM if that fails.
 * RQA_ESIZE if words_per_row is too small, RQA_ETOOSHORT as rqa_run. */
int rqa_plot(rqa_handle *h, const float *d_series, int64_t n_points, uint64_t *d_bits,
             int64_t words_per_row, void *hip_stream);

/* Cross recurrence plot: the n_a x n_b matrix of rqa_run_cross, packed as by
 * rqa_plot (words_per_row >= ceil(n_b/64)). */
int rqa_plot_cross(rqa_handle *h, const float *d_a, int64_t na_points, const float *d_b,
                   int64_t nb_points, uint64_t *d_bits, int64_t words_per_row,
                   void *hip_stream);

/* Batched windowed RQA (many windows of uneven length over one device series,
 * one persistent launch; the RQA X "epochs" idea of Sect. 3 run in parallel).
 * offsets/lengths: count host int64 values, copied during the call; window w
 * is d_series[offsets[w] .. offsets[w]+lengths[w]).  Every window uses h's
 * parameters.  Asynchronous on hip_stream like rqa_run. */
int rqa_run_batch(rqa_handle *h, const float *d_series, int64_t n_points,
                  const int64_t *offsets, const int64_t *lengths, int32_t count,
                  void *hip_stream);

/* Results of window `index` of the last rqa_run_batch (waits for it). */
int rqa_result_batch(rqa_handle *h, int32_t index, rqa_measures *out, uint64_t *diag,
                     uint64_t *vert, uint64_t *white, int64_t hist_len);

/* The measures of every window of the last run in one call (waits for it;
 * the per-window quantities of Sect. 2, for the windows of Sect. 3's epochs):
 * out[w] for w < count, with count equal to the number of windows (else
 * RQA_ESIZE).  out and status (optional, may be NULL) are caller-owned host
 * arrays of count entries.  status[w] is what rqa_result_batch returns for
 * window w; a window without a result (e.g. RQA_ENONFINITE) gets NaN measures,
 * n_rec 0 and its n_vec.  Returns RQA_OK, or the code of the first window that
 * has no result.
 * Same values as rqa_result_batch, without a call per window. */
int rqa_result_batch_all(rqa_handle *h, rqa_measures *out, int32_t *status, int32_t count);

/* Measures from host histograms of length n+1 (FP64, same definitions as
 * rqa_result). */
int rqa_measures_from_hist(const uint64_t *diag, const uint64_t *vert,
                           const uint64_t *white, int64_t n, const rqa_params *p,
                           rqa_measures *out);

/* Tile-shape override: waves per workgroup (1..8, rows per strip = 64*waves;
 * 0 = chosen by the built-in autotuner, which times the candidate shapes 2, 4
 * and 8 waves on the first runs of each launch signature, the default shape
 * first; a shape more than 10% slower than the best so far ends the trials
 * beyond it; RQA_AUTOTUNE_CACHE=<file> persists its choices) and workgroups
 * per launch (0 = fill the device).  Results never depend on these. */
int rqa_set_tiling(rqa_handle *h, int32_t waves_per_group, int32_t groups);

/* Phase timing (hipEvents recorded on the run's stream).  With profiling on,
 * each rqa_run / rqa_run_batch records events around its three phases; after
 * the run, rqa_get_timings waits for it and returns the milliseconds spent in
 * preparation (validation, zeroing), in the fused tile kernel (operators I-III,
 * Sect. 4.2) and in the stitch/join kernel (recombination, Sect. 4.1).  Any
 * output pointer may be NULL.  RQA_ESTATE if the last run was not profiled. */
int rqa_set_profiling(rqa_handle *h, int32_t enable);
int rqa_get_timings(rqa_handle *h, double *prepare_ms, double *tiles_ms, double *stitch_ms);

/* How the last run was launched: waves per workgroup (chosen by the autotuner
 * unless fixed with rqa_set_tiling) and whether it was replayed from a captured
 * hipGraph (identical repeated launches are captured once and replayed).
 * RQA_ESTATE before the first run. */
int rqa_last_launch(const rqa_handle *h, int32_t *waves, int32_t *graph_replay);

/* Memory bound of the recombination (Sect. 4.1, Divide & Recombine: the matrix
 * is processed in parts that fit the memory, and lines crossing their borders
 * pass on through carry-over state).  A run keeps, per strip of rows and line,
 * the runs at the strip's edges until they are joined: O(n_rows n_cols / strip
 * height) bytes.  When that would exceed `bytes`, the run walks the strips in
 * row bands: each band's tile kernel writes its edge runs, the band's stitch
 * joins them into one open run per column and per diagonal (carries of
 * O(n_rows + n_cols)), and the next band reuses the space.  Results are
 * identical (with several bands, the tile phase of rqa_get_timings also holds
 * the stitch of every band but the last).  bytes = 0 restores the default: a
 * quarter of the device's memory.  Applies to a job run alone: rqa_run (one
 * series, or a batch of one window), rqa_run_cross and rqa_run_matrix; batches
 * of several windows are not banded.  RQA_EINVAL for bytes < 0; a bound below
 * what one band needs runs with one strip per band (and may then fail with
 * RQA_ENOMEM). */
int rqa_set_workspace_limit(rqa_handle *h, int64_t bytes);

/* How the last run was cut: row bands and strips per band (1 and all strips
 * when unbanded), column segments per strip, rows per strip, and the device
 * workspace of its first job's line summaries in bytes.  Any output pointer
 * may be NULL.  RQA_ESTATE before the first run. */
int rqa_last_plan(const rqa_handle *h, int32_t *bands, int32_t *band_strips, int32_t *segs,
                  int32_t *strip_rows, int64_t *workspace_bytes);

/* The same cut computed on the host, without a device or a run: for a series
 * of n_points run alone with `waves` waves per workgroup (1..8; 0 = the
 * library's default shape) and line summaries bounded by limit_bytes (0 = no
 * bound, one band).  Any output pointer may be NULL.  RQA_EINVAL for invalid
 * parameters or arguments, RQA_ETOOSHORT if the series has no delay vector. */
int rqa_workspace_plan(const rqa_params *p, int64_t n_points, int32_t waves, int64_t limit_bytes,
                       int32_t *bands, int32_t *band_strips, int32_t *segs,
                       int64_t *workspace_bytes);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * RQA as rqa_run + rqa_result of one device series under the parameters *p,
 * enqueued on hip_stream with no allocation at all (no hipMalloc, hipFree,
 * pinned host buffer or host-to-device copy): the kernels' scratch lies in a
 * static device array of RQA_STATIC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  That limit admits series of up
 * to about 92,000 delay vectors; a larger one returns RQA_EBUDGET.
 *   d_series: n_points FP32 values in device memory (caller-owned, alive and
 *             unmodified until the stream has passed the call);
 *   d_hist:   caller-owned DEVICE array of 3*hist_len uint64, hist_len >= n+1
 *             (else RQA_ESIZE): diag at [0, hist_len), vert at [hist_len,
 *             2 hist_len), white at [2 hist_len, 3 hist_len); entries 0..n of
 *             each are written, the rest are left unchanged;
 *   d_flag:   caller-owned DEVICE int32, written 0 when the run is valid; bit 0
 *             set means the series holds NaN or +-Inf (rqa_result's
 *             RQA_ENONFINITE), any other bit an internal device error.
 * Measures follow from the histograms copied to the host with
 * rqa_measures_from_hist.  Host-detectable errors (RQA_EINVAL, RQA_ETOOSHORT,
 * RQA_ESIZE, RQA_EBUDGET) return before anything is enqueued.  All calls on one
 * GPU share its scratch array, which keeps the last call's contents: calls
 * whose work overlaps on one GPU (other streams, other threads) race, so
 * serialise them, e.g. on one stream. */
#define RQA_STATIC_SCRATCH_BYTES (64u << 20)
int rqa_run_static(const rqa_params *p, const float *d_series, int64_t n_points,
                   uint64_t *d_hist, int64_t hist_len, int32_t *d_flag, void *hip_stream);

/* Release the handle and its device workspace (waits for outstanding work). */
void rqa_destroy(rqa_handle *h);

/* Static description of a return code. */
const char *rqa_strerror(int code);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent jobs under a device-memory
 * budget.  Jobs are admitted while their footprint fits, run on a pool of
 * streams so that jobs submitted while others run overlap on the device, and
 * are retired as they complete.  Thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct rqa_server rqa_server;

/* budget_bytes: device memory the server may hold for job workspaces;
 * streams: concurrent launch slots (1..16).  With two or more streams, the
 * first half runs large jobs (above 2e9 matrix cells, each launched alone)
 * and the second half batches of small ones, so small jobs never queue behind
 * a large one; with one stream everything shares it. */
int rqa_server_create(rqa_server **out, size_t budget_bytes, int32_t streams);

/* Device bytes of the server pool a job of n_points occupies while it runs
 * (histograms, flag and engine scratch; the series stays the caller's). */
int rqa_job_footprint(const rqa_params *p, int64_t n_points, size_t *bytes);

/* Submit a job.  d_series: n_points FP32 values in device memory, produced on
 * hip_stream (the job starts only after the work enqueued there so far); the
 * caller keeps it alive and unmodified until the job is retired by rqa_poll or
 * rqa_wait.  RQA_EBUDGET if the job alone exceeds the budget; otherwise it is
 * queued until its footprint fits.  *ticket identifies the job. */
int rqa_submit(rqa_server *srv, const rqa_params *p, const float *d_series,
               int64_t n_points, void *hip_stream, uint64_t *ticket);

/* Poll (RQA_EAGAIN while running) or wait for a job; on success the job is
 * retired and its result copied (histogram pointers may be NULL). */
int rqa_poll(rqa_server *srv, uint64_t ticket, rqa_measures *out, uint64_t *diag,
             uint64_t *vert, uint64_t *white, int64_t hist_len);
int rqa_wait(rqa_server *srv, uint64_t ticket, rqa_measures *out, uint64_t *diag,
             uint64_t *vert, uint64_t *white, int64_t hist_len);

/* Drain all jobs and release the server. */
void rqa_server_destroy(rqa_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* RQA_H */
