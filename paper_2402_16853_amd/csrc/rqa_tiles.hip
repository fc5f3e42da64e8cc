// Fused RQA engine for gfx950: recurrence predicate, diagonal / vertical /
// white-vertical run extraction and histogram recombination in one pass over
// the upper triangle of the recurrence matrix, which is never stored.
//
// Mapping of the paper's method (Sect. 4):
//  * operator I (similarity of one vector pair) -- evaluated once per unique pair
//    i < j with j - i >= max(theiler, 1): the matrix is symmetric, so the lower
//    triangle is recovered by mirroring (Sect. 4.2 notes that a symmetric matrix
//    needs only N-1 diagonals);
//  * operators II and III (lines along one diagonal / one column) -- run-length
//    state machines over 64-bit bit-words of 64x64 tiles;
//  * divide & recombine with carry-over (Sect. 4.1) -- open runs are carried
//    across tile edges in registers (left to right) and through LDS between the
//    waves of a workgroup (top to bottom); runs that touch the top or bottom edge
//    of a workgroup's strip are summarised and joined by the stitch kernel.
//
// Geometry.  n delay vectors, w' = max(theiler, 1).  U = {(i,j): j - i >= w'}.
// A workgroup of W waves owns a strip of H = 64*W consecutive rows; wave w owns
// rows R = R0 + 64w .. R+63, one row per lane, and walks the 64-column tiles
// c = c0 .. c_last of its strip left to right.  The waves run as a pipeline:
// wave w consumes the carries that wave w-1 produced for the same tile, through
// an LDS ring per wave pair with produced / consumed counters (no workgroup
// barrier per tile; a wave may run up to kRing tiles ahead of the one below).
//
// Full-matrix lines from U:
//  * a diagonal k >= w' of U and its mirror -k: each run counted twice;
//  * column j of the full matrix = [column j of U: rows 0..j-w'] ++ [middle] ++
//    [row j of U: columns j+w'..n-1], the middle being the Theiler band (white,
//    theiler >= 1) or the single recurrent cell (j,j) (theiler = 0).  Runs inside
//    either segment are counted where they are found; the trailing run of the
//    column segment, the middle and the leading run of the row segment are
//    merged by the join step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "rqa_internal.h"

namespace rqa {

KParams make_kparams(const rqa_params &p) {
    KParams k;
    k.m = p.m;
    k.tau = p.tau;
    k.eps = p.eps;
    volatile float e = p.eps;   // one FP32 rounding of eps*eps, no contraction
    k.eps_sq = e * e;
    // First-coordinate bound.  The accumulated distance a never falls below the
    // first coordinate's term (a sum or max of non-negative terms, and rounding
    // is monotone), and that term is monotone in |d_0|, so |d_0| > d0_bound
    // decides "not recurrent" exactly.
    if (p.norm != RQA_NORM_L2) {
        k.d0_bound = p.eps;
    } else if (!std::isfinite(k.eps_sq)) {
        k.d0_bound = std::numeric_limits<float>::infinity();
    } else {
        // Largest t >= 0 with fl32(t*t) <= eps_sq: binary search over the bit
        // patterns of non-negative floats, which are ordered like the values
        // (fl32(0*0) = 0 <= eps_sq; fl32(inf*inf) = inf > eps_sq).
        uint32_t lo = 0u, hi = 0x7F800000u;
        while (hi - lo > 1u) {
            const uint32_t mid = lo + (hi - lo) / 2u;
            float t;
            std::memcpy(&t, &mid, sizeof t);
            volatile float tv = t;
            volatile float sq = tv * tv;
            if (sq <= k.eps_sq) lo = mid; else hi = mid;
        }
        std::memcpy(&k.d0_bound, &lo, sizeof lo);
    }
    k.norm = p.norm;
    k.theiler = p.theiler;
    k.lmin = p.lmin;
    k.vmin = p.vmin;
    k.wmin = p.wmin;
    return k;
}

namespace {

constexpr int kMaxWaves = 8;
constexpr int kCapD = 1024;    // LDS bins for diagonal lengths < kCapD
constexpr int kCapV = 1024;    // LDS bins for vertical lengths < kCapV
constexpr int kCapW = 6016;    // LDS bins for white-vertical lengths < kCapW
constexpr int kMaxM = 6;       // embedding dimensions held in registers
constexpr int kRing = 4;       // carry slots per pair of consecutive waves (tiles in flight)
constexpr uint32_t kSpinLimit = 1u << 20;   // polls (~28 ms) before a neighbour wait gives up
constexpr int kStitchThreads = 512;
constexpr int kStitchBatch = 8;   // strips whose summaries a stitch thread loads at once
constexpr int kStitchCapV = 2048; // stitch LDS bins for vertical lengths < kStitchCapV (the
                                  // stitch joins the runs that cross strip edges: long ones)
constexpr int kStatThreads = 256;
constexpr int kStatMaxBlocks = 64;
// Column boxes (exact pruning of the predicate, see tile_bits): per 64-column
// tile one record of kBoxStride floats holding (lo_k, hi_k) for the first
// kBoxK coordinates.  The box array of a job starts with a header of
// kBoxHeader floats whose first word tells whether the job uses the boxes (set
// by k_box_probe).
constexpr int kBoxK = 3;
constexpr int kBoxStride = 8;
constexpr int kBoxHeader = 64;
constexpr int kProbeThreads = 256;   // sampled (row block, tile) pairs per job

// Device-side description of one job (one series or window).
struct JobDesc {
    const float *s;            // series of the rows (n_points values)
    const float *sb;           // series of the columns (auto: s)
    const uint64_t *bits;      // given matrix: n rows of `words` u64 (bit b of word c = column 64c+b)
    int64_t words;
    int64_t n_points_b;        // points of sb
    const float *tail;         // coordinates of the last column tile, zero padded
    unsigned long long *hd;    // histograms, n+1 entries each
    unsigned long long *hv;
    unsigned long long *hw;
    int *flag;                 // non-finite flag
    uint32_t *lead;            // leading run of each row of U: len | color<<31
    uint32_t *hfirst;          // auto, segments > 1: per (row, segment) first / last run of
    uint32_t *hlast;           // the row's piece in the segment, len | color<<31
    uint16_t *vfirst;          // per (strip, column): first run len | color<<15
    uint16_t *vlast;           // per (strip, column): last run len | color<<15
    uint16_t *dfirst;          // per (strip, diagonal): black run at the top edge
    uint16_t *dlast;           // per (strip, diagonal): black run at the bottom edge
    int64_t n_points;
    int32_t n;                 // delay vectors (rows)
    int32_t nb;                // columns (auto: n)
    int32_t hmax;              // longest possible line; histograms hold hmax+1 entries
    int32_t mode;              // JobMode
    int32_t m, tau, norm, theiler, wp;
    float thr;                 // eps (L1, Linf) or fl32(eps*eps) (L2)
    float thr0;                // first-coordinate bound (KParams::d0_bound)
    int32_t H;                 // strip height
    int32_t nstrips;
    int32_t segs;              // column segments per strip (1: strips are not cut)
    int32_t seg_tiles;         // column tiles per segment; segment g covers the column
                               // tiles [seg_base + g*seg_tiles, seg_base + (g+1)*seg_tiles)
    int32_t seg_base;          // first column tile of segment 0 (auto: wp/64; full: 0)
    int32_t dw;                // diagonal summary slots per (strip, segment) block (segs > 1
                               // or full matrix)
    int32_t c_last;            // last column tile (nb-1)/64
    int32_t tail_len;          // floats in tail
    int32_t strip_base;        // first work item of this job within its group
    int32_t stitch_block0;     // first stitch block of this job
    int32_t mins[3];           // lmin, vmin, wmin
    int32_t stat_blocks;       // blocks of the statistics kernels for this job
    JobStats *stats;           // device statistics record
    double *ent_part;          // [3][kStatMaxBlocks] entropy partial sums
    float *box;                // column boxes (header + records), nullptr if none
    int32_t spin_limit;        // polls before a neighbour wait gives up (kSpinLimit)
    int32_t wait_bias;         // added to every wait target: 0, or (fault injection
                               // for tests) a bias no counter reaches
    // Row bands (auto mode): the launch walks strips [s_lo, s_hi) of band_strips
    // per band; summary slots are relative to strip s_lo (strip_offset(s_lo) =
    // soff_lo).  With several bands the open run of each column of U and of
    // each diagonal passes to the next band through cstate / dstate.
    int32_t s_lo, s_hi;
    int32_t band_strips, nbands;
    int64_t soff_lo;
    uint32_t *cstate;          // per column: open run len | color<<31 (nbands > 1)
    uint32_t *dstate;          // per diagonal: open black run length (nbands > 1)
};

struct GroupDesc {
    int32_t job0, job1;        // jobs [job0, job1) of the descriptor table
    int32_t items;             // total strips of the group
    int32_t pad;
};

__host__ __device__ inline int64_t strip_offset(int32_t s, int32_t n, int32_t wp, int32_t H) {
    // sum_{s' < s} (n - wp - s' H): entries of the strips before s
    return (int64_t)s * (n - wp) - (int64_t)H * ((int64_t)s * (s - 1) / 2);
}

// ---------------------------------------------------------------------------
// Bit-word helpers (64-bit words split in two VGPRs; bit p = position p along a
// line).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mk64(uint32_t lo, uint32_t hi) {
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t range_mask(uint32_t lo, uint32_t hi) {
    // bits [lo, hi), 0 <= lo <= hi <= 64
    const uint64_t a = lo >= 64 ? 0ull : (~0ull << lo);
    const uint64_t b = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return a & b;
}

// Lane exchange within 32-lane halves: lane l reads lane l^D (ds_swizzle in
// xor mode; no VALU work).
template <int D>
__device__ __forceinline__ uint32_t swizzle_xor(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (D << 10));
}

// One butterfly stage of the 64x64 bit transpose, D in {16,8,4,2,1}: lanes l and
// l^D exchange bit blocks.  M marks the bit positions whose D-bit is 0.  The
// lower lane keeps its M positions and takes the partner's M positions moved up
// by D; the upper lane keeps its ~M positions and takes the partner's ~M
// positions moved down by D.  The move is a rotation (v_alignbit); the bits it
// wraps around fall outside the selected positions, so one v_bfi finishes the
// stage.
template <int D, uint32_t M>
__device__ __forceinline__ void transpose_stage(uint32_t &lo, uint32_t &hi, int lane) {
    const bool up = (lane & D) != 0;
    const uint32_t keep = up ? ~M : M;
    const uint32_t amt = up ? (uint32_t)D : (uint32_t)(32 - D);
    const uint32_t rl = swizzle_xor<D>(lo);
    const uint32_t rh = swizzle_xor<D>(hi);
    const uint32_t sl = __builtin_amdgcn_alignbit(rl, rl, amt);
    const uint32_t sh = __builtin_amdgcn_alignbit(rh, rh, amt);
    lo = (keep & lo) | (~keep & sl);
    hi = (keep & hi) | (~keep & sh);
}

// In-register transpose of a 64x64 bit matrix held one row per lane: on return
// lane l holds column l (bit r = old lane r's bit l).  The 32-lane stage is one
// v_permlane32_swap (upper lanes of `lo` <-> lower lanes of `hi`); the other five
// stages are butterflies within 32-lane halves.
__device__ __forceinline__ void transpose64(uint32_t &lo, uint32_t &hi, int lane) {
    const auto sw = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
    lo = sw[0];
    hi = sw[1];
    transpose_stage<16, 0x0000FFFFu>(lo, hi, lane);
    transpose_stage<8, 0x00FF00FFu>(lo, hi, lane);
    transpose_stage<4, 0x0F0F0F0Fu>(lo, hi, lane);
    transpose_stage<2, 0x33333333u>(lo, hi, lane);
    transpose_stage<1, 0x55555555u>(lo, hi, lane);
}

// 64-bit rotate right by r (0..63), branch-free.
__device__ __forceinline__ void rotr64(uint32_t &lo, uint32_t &hi, uint32_t r) {
    const bool sw = (r & 32) != 0;
    const uint32_t a = sw ? hi : lo;
    const uint32_t b = sw ? lo : hi;
    const uint32_t s = r & 31;
    lo = __builtin_amdgcn_alignbit(b, a, s);
    hi = __builtin_amdgcn_alignbit(a, b, s);
}

// ---------------------------------------------------------------------------
// Run state machine.  A line is cut into segments; `Run` is the open run at the
// current position: colour (1 = recurrent), length so far, and whether it is the
// first run of the current segment (then it is recorded instead of counted).
// ---------------------------------------------------------------------------
struct Run {
    uint32_t color;
    uint32_t len;
    uint32_t first;
};

__device__ __forceinline__ uint32_t pack_run(const Run &r) {
    return (r.len & 0xFFFFu) | (r.color << 16) | (r.first << 17);
}
__device__ __forceinline__ Run unpack_run(uint32_t v) {
    return Run{(v >> 16) & 1u, v & 0xFFFFu, (v >> 17) & 1u};
}

// Global-memory access through address-space-1 pointers.  The kernels reach
// HBM through pointers held in the job descriptor, which the compiler cannot
// prove global; it would emit flat instructions, and every flat access also
// counts against the LDS/scalar wait counter, so a later wait for a scalar load
// would also wait for outstanding histogram atomics and summary stores.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *glb(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
__device__ __forceinline__ void g_add(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add(glb(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_or(int *p, int v) {
    __hip_atomic_fetch_or(glb(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Bins {
    uint32_t *d, *v, *w;
};

// Count `wt` lines of length len: LDS bin below the cap, else the global
// histogram.  A length beyond the histogram (n) cannot occur for a correct run
// and is reported through bit 1 of the job flag instead of being written.
__device__ __forceinline__ void emit(uint32_t *bins, int cap, unsigned long long *glob, uint32_t len,
                                     uint32_t wt, uint32_t n, int *flag) {
    if (len < (uint32_t)cap && len <= n)
        atomicAdd(bins + len, wt);
    else if (len <= n)
        g_add(glob + len, (unsigned long long)wt);
    else
        g_or(flag, 2);
}

enum LineKind { kHoriz = 0, kVert = 1, kDiag = 2 };

struct LineCtx {
    const JobDesc *jd;
    Bins bins;
    int64_t sum_idx;    // summary index of this line in this strip (vert / diag)
    bool sum_ok;        // summary slot exists (diagonal inside the strip's range)
    uint32_t row;       // row index (horizontal)
};

// A run of colour `c` and length `len` has ended.  DW: how many lines a
// diagonal run stands for (2 in the upper triangle of a symmetric matrix, whose
// mirror diagonal repeats it; 1 in a full matrix).
template <int KIND, int DW = 2>
__device__ __forceinline__ void finish_run(const LineCtx &lc, uint32_t c, uint32_t len, uint32_t first) {
    const JobDesc &j = *lc.jd;
    if (KIND == kDiag) {
        if (first) {
            if (lc.sum_ok) *glb(j.dfirst + lc.sum_idx) = (uint16_t)(c ? len : 0u);
        } else if (c) {
            emit(lc.bins.d, kCapD, j.hd, len, (uint32_t)DW, (uint32_t)j.hmax, j.flag);
        }
    } else if (KIND == kVert) {
        if (first)
            *glb(j.vfirst + lc.sum_idx) = (uint16_t)(len | (c << 15));
        else if (c)
            emit(lc.bins.v, kCapV, j.hv, len, 1u, (uint32_t)j.hmax, j.flag);
        else
            emit(lc.bins.w, kCapW, j.hw, len, 1u, (uint32_t)j.hmax, j.flag);
    } else {
        if (first) {
            if (lc.sum_ok) *glb(j.hfirst + lc.sum_idx) = len | (c << 31);   // a row piece
            else *glb(j.lead + lc.row) = len | (c << 31);
        } else if (c)
            emit(lc.bins.v, kCapV, j.hv, len, 1u, (uint32_t)j.hmax, j.flag);
        else
            emit(lc.bins.w, kCapW, j.hw, len, 1u, (uint32_t)j.hmax, j.flag);
    }
}

// A run that starts and ends inside one window: 1 <= len <= 63, never the
// first run of a segment, below every LDS bin cap and every histogram length.
template <int KIND, int DW>
__device__ __forceinline__ void emit_inner(const LineCtx &lc, uint32_t c, uint32_t len) {
    if (KIND == kDiag) {
        if (c) atomicAdd(lc.bins.d + len, (uint32_t)DW);
    } else {
        atomicAdd((c ? lc.bins.v : lc.bins.w) + len, 1u);
    }
}

// Index of the lowest set bit of a non-zero 64-bit word.
__device__ __forceinline__ uint32_t low_bit(uint64_t t) { return (uint32_t)__builtin_ctzll(t); }

// Advance `st` over the bits [lo, hi) of x (win = mask of those bits),
// finishing every run that ends there.  The colour changes are the set bits
// of x ^ (x shifted by one, with the open run's colour entering at lo).  The
// first change ends the open run (which may be a segment's first run or carry a
// long length); every later run lies inside the window.
template <int KIND, int DW = 2>
__device__ __forceinline__ void run_segment(uint64_t x, uint64_t win, uint32_t lo, uint32_t hi,
                                            Run &st, const LineCtx &lc) {
    if (lo >= hi) return;
    const uint64_t prev = ((x << 1) & ~(1ull << lo)) | ((uint64_t)st.color << lo);
    uint64_t t = (x ^ prev) & win;
    if (t == 0) {
        st.len += hi - lo;
        return;
    }
    uint32_t p = low_bit(t);
    finish_run<KIND, DW>(lc, st.color, st.len + (p - lo), st.first);
    uint32_t c = st.color ^ 1u;
    uint32_t sp = p;
    t &= t - 1ull;
    while (t) {
        p = low_bit(t);
        emit_inner<KIND, DW>(lc, c, p - sp);
        c ^= 1u;
        sp = p;
        t &= t - 1ull;
    }
    st = Run{c, hi - sp, 0u};
}

// Series pointer in the constant address space: loads through it with a
// wave-uniform address become scalar (s_load) loads, so the column coordinates
// arrive in SGPRs and feed the VALU as scalar operands.
typedef const __attribute__((address_space(4))) float *ConstF;

__device__ __forceinline__ ConstF to_const(const float *p) { return (ConstF)(p); }

// ---------------------------------------------------------------------------
// Recurrence predicate for one column against the 64 rows of a wave.
// Returns a word whose bit 31 is set when the pair is NOT recurrent: the sign of
// fl(thr - a) is set exactly when a > thr (IEEE subtraction of two finite floats
// is zero only for equal operands).  a is accumulated in FP32, coordinates in
// ascending order, no FMA.
// ---------------------------------------------------------------------------
template <int NORM, int M>
__device__ __forceinline__ uint32_t nonrec_sign(ConstF col, int tau, const float *xr, float thr) {
    float a;
    if (NORM == RQA_NORM_L1) {
        a = fabsf(col[0] - xr[0]);
#pragma unroll
        for (int k = 1; k < M; ++k) a = a + fabsf(col[k * tau] - xr[k]);
    } else if (NORM == RQA_NORM_L2) {
        const float d = col[0] - xr[0];
        a = d * d;
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const float e = col[k * tau] - xr[k];
            a = a + e * e;
        }
    } else {
        a = fabsf(col[0] - xr[0]);
#pragma unroll
        for (int k = 1; k < M; ++k) a = fmaxf(a, fabsf(col[k * tau] - xr[k]));
    }
    return __float_as_uint(thr - a);
}

// The same, with the first coordinate's difference d0 = col[0] - xr[0] given.
template <int NORM, int M>
__device__ __forceinline__ uint32_t nonrec_sign_d0(float d0, ConstF col, int tau, const float *xr,
                                                   float thr) {
    float a;
    if (NORM == RQA_NORM_L1) {
        a = fabsf(d0);
#pragma unroll
        for (int k = 1; k < M; ++k) a = a + fabsf(col[k * tau] - xr[k]);
    } else if (NORM == RQA_NORM_L2) {
        a = d0 * d0;
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const float e = col[k * tau] - xr[k];
            a = a + e * e;
        }
    } else {
        a = fabsf(d0);
#pragma unroll
        for (int k = 1; k < M; ++k) a = fmaxf(a, fabsf(col[k * tau] - xr[k]));
    }
    return __float_as_uint(thr - a);
}

// The same, for column b of a chunk whose coordinate k starts at ck[k].
template <int NORM, int M>
__device__ __forceinline__ uint32_t nonrec_sign_rows(const ConstF *ck, int b, const float *xr,
                                                     float thr) {
    float a;
    if (NORM == RQA_NORM_L1) {
        a = fabsf(ck[0][b] - xr[0]);
#pragma unroll
        for (int k = 1; k < M; ++k) a = a + fabsf(ck[k][b] - xr[k]);
    } else if (NORM == RQA_NORM_L2) {
        const float d = ck[0][b] - xr[0];
        a = d * d;
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const float e = ck[k][b] - xr[k];
            a = a + e * e;
        }
    } else {
        a = fabsf(ck[0][b] - xr[0]);
#pragma unroll
        for (int k = 1; k < M; ++k) a = fmaxf(a, fabsf(ck[k][b] - xr[k]));
    }
    return __float_as_uint(thr - a);
}

// Generic embedding dimension: row coordinates read from memory.
template <int NORM>
__device__ __forceinline__ uint32_t nonrec_sign_dyn(ConstF col, const float *__restrict__ rowp,
                                                    int m, int tau, float thr) {
    const auto row = glb(rowp);
    float a;
    if (NORM == RQA_NORM_L1) {
        a = fabsf(col[0] - row[0]);
        for (int k = 1; k < m; ++k) a = a + fabsf(col[(int64_t)k * tau] - row[(int64_t)k * tau]);
    } else if (NORM == RQA_NORM_L2) {
        const float d = col[0] - row[0];
        a = d * d;
        for (int k = 1; k < m; ++k) {
            const float e = col[(int64_t)k * tau] - row[(int64_t)k * tau];
            a = a + e * e;
        }
    } else {
        a = fabsf(col[0] - row[0]);
        for (int k = 1; k < m; ++k) a = fmaxf(a, fabsf(col[(int64_t)k * tau] - row[(int64_t)k * tau]));
    }
    return __float_as_uint(thr - a);
}

// Box test.  `rec` holds, for the first kBoxK coordinates k of a tile's
// columns, lo_k = the smallest float l with fl(cmin_k - l) <= b and hi_k = the
// largest float h with fl(h - cmax_k) <= b, where cmin_k / cmax_k are the
// smallest / largest k-th coordinate of those columns and b is the
// per-coordinate bound of KParams::d0_bound.  Subtraction is monotone in each
// operand, so a row coordinate x_k < lo_k (or > hi_k) makes |d_k| > b against
// every column of the tile, and the accumulated distance, never below its
// largest term, then exceeds the threshold: the pair is not recurrent.  True
// when every row of the wave is decided so by some coordinate.
template <int M>
__device__ __forceinline__ bool box_decides(ConstF rec, const float *xr) {
    constexpr int K = M < kBoxK ? M : kBoxK;
    bool out = false;
#pragma unroll
    for (int k = 0; k < K; ++k) out = out | (xr[k] < rec[2 * k]) | (xr[k] > rec[2 * k + 1]);
    return __builtin_amdgcn_ballot_w64(!out) == 0ull;
}

// Recurrence bits of one 64x64 tile for this lane's row: bit b <-> column
// jbase + b.  `cols` points at the coordinate of column jbase (uniform).  The 64
// columns are taken in eight chunks of 8 (highest first), each fully unrolled,
// so that at most 8*m column coordinates are live in SGPRs (chunks of 16 left
// too few SGPRs for the rest of the kernel, which then spilled into VGPR lanes;
// measured 10% slower).
// Exact pruning, two variants:
//  * `box` (this tile's box record, or nullptr): when the box decides every
//    row of the wave, the tile has no recurrent cell and no column is
//    evaluated.  Otherwise every pair is evaluated: a box test per 8-column
//    chunk decides far more chunks on smooth series (Lorenz: 64% of the chunks
//    of undecided tiles, against 24% for the first-coordinate test), but its
//    record took SGPRs the kernel did not have (spills) and measured slower
//    than evaluating the chunk;
//  * m >= 5 (the first-coordinate test): each chunk first takes the first
//    coordinate's differences; when no lane of the wave has |d_0| <= thr0 in
//    the chunk, all 8 x 64 pairs are non-recurrent and the other coordinates
//    are not evaluated.
template <int NORM, int M>
__device__ __forceinline__ void tile_bits(ConstF cols, int tau, const float *xr,
                                          const float *__restrict__ rowp, int m, float thr_s,
                                          float thr0_s, ConstF box, uint32_t &lo, uint32_t &hi) {
    // The thresholds are uniform, but as scalar operands they would make the
    // subtraction and the compare read an SGPR too; VALU instructions with only
    // VGPR operands issue faster on gfx950 (measured: the six-instruction
    // L-infinity column sustains ~1.5 instead of ~1.2 wave-instructions per
    // clock per CU).  The empty asm pins the copies in VGPRs.
    float thr = thr_s, thr0 = thr0_s;
    asm volatile("" : "+v"(thr), "+v"(thr0));
    if (M > 0 && box != nullptr && box_decides<M>(box, xr)) {
        lo = 0u;
        hi = 0u;
        return;
    }
#pragma unroll 1
    for (int half = 1; half >= 0; --half) {
        uint32_t acc = 0;
#pragma unroll 1
        for (int sub = 3; sub >= 0; --sub) {
            const int b0 = half * 32 + sub * 8;
            ConstF cb = cols + b0;
            if (M > 0) {
                // Embedding dimensions of 5 and 6 always take the first-
                // coordinate path: their 40-48 column coordinates do not fit
                // the SGPRs left, and without the loads pinned ahead of the
                // test the compiler rebuilt their addresses with long chains
                // of 64-bit scalar adds (measured 29% slower on the L1, m = 5
                // windows).
                if (M >= 5) {
                    // All of the chunk's coordinates are loaded up front (the
                    // empty asm keeps the compiler from sinking the loads of
                    // the other coordinates into the branch, which would add a
                    // second wait); the first coordinate's differences decide
                    // whether the rest is evaluated.
                    float d0[8];
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        d0[b] = cb[b] - xr[0];
#pragma unroll
                        for (int k = 1; k < (M > 0 ? M : 1); ++k) {
                            const float ck = cb[b + k * tau];
                            asm volatile("" ::"s"(ck));
                        }
                    }
                    const float near =
                        fminf(fminf(fminf(fabsf(d0[0]), fabsf(d0[1])), fminf(fabsf(d0[2]), fabsf(d0[3]))),
                              fminf(fminf(fabsf(d0[4]), fabsf(d0[5])), fminf(fabsf(d0[6]), fabsf(d0[7]))));
                    if (__builtin_amdgcn_ballot_w64(near <= thr0) == 0ull) {
                        acc = (acc << 8) | 0xFFu;
                    } else {
#pragma unroll
                        for (int b = 7; b >= 0; --b)
                            acc = __builtin_amdgcn_alignbit(
                                acc, nonrec_sign_d0<NORM, M>(d0[b], cb + b, tau, xr, thr), 31);
                    }
                } else {
                    // One uniform pointer per coordinate: each coordinate's 8
                    // columns are then one s_load_dwordx8 at a fixed offset
                    // (indexing cb[b + k*tau] instead made the compiler build
                    // 8*m addresses with 64-bit scalar adds).
                    ConstF ck[M > 0 ? M : 1];
#pragma unroll
                    for (int k = 0; k < (M > 0 ? M : 1); ++k) ck[k] = cb + k * tau;
#pragma unroll
                    for (int b = 7; b >= 0; --b)
                        acc = __builtin_amdgcn_alignbit(
                            acc, nonrec_sign_rows<NORM, M>(ck, b, xr, thr), 31);
                }
            } else {
                for (int b = 7; b >= 0; --b)
                    acc = __builtin_amdgcn_alignbit(
                        acc, nonrec_sign_dyn<NORM>(cb + b, rowp, m, tau, thr), 31);
            }
        }
        if (half) hi = ~acc; else lo = ~acc;
    }
}

// ---------------------------------------------------------------------------
// Column boxes.  Ordered keys of the non-NaN floats (unsigned order = float
// order, -0 just below +0), used to bisect over float values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fval(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Largest float h with fl(h - cmax) <= b (h = +inf when b = +inf).
__device__ float box_hi(float cmax, float b) {
    if (b == INFINITY) return INFINITY;
    uint32_t t = fkey(-INFINITY), f = fkey(INFINITY);   // P(t) true, P(f) false
    while (f - t > 1u) {
        const uint32_t mid = t + (f - t) / 2u;
        if (fval(mid) - cmax <= b) t = mid; else f = mid;
    }
    return fval(t);
}

// Smallest float l with fl(cmin - l) <= b (l = -inf when b = +inf).
__device__ float box_lo(float cmin, float b) {
    if (b == INFINITY) return -INFINITY;
    uint32_t f = fkey(-INFINITY), t = fkey(INFINITY);   // Q(f) false, Q(t) true
    while (t - f > 1u) {
        const uint32_t mid = f + (t - f) / 2u;
        if (cmin - fval(mid) <= b) t = mid; else f = mid;
    }
    return fval(t);
}

// ---------------------------------------------------------------------------
// Kernel 1: per-job preparation -- zero the histograms, flag non-finite input,
// build the zero-padded tail of the last column tile, reset work counters.
// grid.y = job index.
// ---------------------------------------------------------------------------
__global__ void k_prepare(const JobDesc *__restrict__ jobs) {
    const JobDesc &j = jobs[blockIdx.y];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t hl = (int64_t)j.hmax + 1;
    for (int64_t t = tid; t < hl; t += stride) {
        j.hd[t] = 0ull;
        j.hv[t] = 0ull;
        j.hw[t] = 0ull;
    }
    if (tid < (int64_t)(sizeof(JobStats) / 8))
        reinterpret_cast<unsigned long long *>(j.stats)[tid] = 0ull;
    if (j.mode == kModeMatrix) return;   // a given matrix has no series
    bool bad = false;
    for (int64_t t = tid; t < j.n_points; t += stride) bad |= !__builtin_isfinite(j.s[t]);
    if (j.mode == kModeCross)
        for (int64_t t = tid; t < j.n_points_b; t += stride) bad |= !__builtin_isfinite(j.sb[t]);
    if (bad) atomicOr(j.flag, 1);   // bit 0: non-finite input
    // Column coordinates of the last tile, from the columns' series.
    const int64_t base = (int64_t)j.c_last * 64;
    float *tail = const_cast<float *>(j.tail);
    for (int64_t t = tid; t < j.tail_len; t += stride)
        tail[t] = base + t < j.n_points_b ? j.sb[base + t] : 0.0f;
}

// Column boxes of every column tile of a job (grid.y = job; one thread per
// (tile, coordinate)).  Only columns < nb count.
__global__ void k_box_bounds(const JobDesc *__restrict__ jobs) {
    const JobDesc &j = jobs[blockIdx.y];
    if (j.box == nullptr) return;
    const int K = j.m < kBoxK ? j.m : kBoxK;
    const int64_t total = (int64_t)(j.c_last + 1) * K;
    const float b = j.thr0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % K);
        const int64_t c = t / K;
        const int64_t j0 = c * 64;
        const int64_t j1 = j0 + 64 < j.nb ? j0 + 64 : j.nb;
        float cmin = INFINITY, cmax = -INFINITY;
        const float *col = j.sb + (int64_t)k * j.tau;
        for (int64_t q = j0; q < j1; ++q) {
            const float v = col[q];
            cmin = fminf(cmin, v);
            cmax = fmaxf(cmax, v);
        }
        float *rec = j.box + kBoxHeader + c * kBoxStride;
        rec[2 * k] = box_lo(cmin, b);
        rec[2 * k + 1] = box_hi(cmax, b);
    }
}

// Whether a job uses its boxes: one block per job samples kProbeThreads
// (64-row block, column tile) pairs of the evaluated region and counts the
// tiles whose box decides all 64 rows.  A decided tile saves its whole
// predicate, an undecided one costs the test (one scalar load and a compare
// per coordinate), so the boxes are used when at least 1 in 64 sampled tiles
// is decided.  Only speed depends on this.
__global__ void __launch_bounds__(kProbeThreads) k_box_probe(const JobDesc *__restrict__ jobs) {
    const JobDesc &j = jobs[blockIdx.x];
    if (j.box == nullptr) return;
    __shared__ int decided, sampled;
    if (threadIdx.x == 0) { decided = 0; sampled = 0; }
    __syncthreads();
    const int K = j.m < kBoxK ? j.m : kBoxK;
    // splitmix64 of (job, thread): the sample position
    uint64_t z = ((uint64_t)blockIdx.x << 32) + threadIdx.x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int blocks = (j.n + 63) / 64;
    const int r0 = (int)((z & 0xFFFFFFFFull) % (uint64_t)blocks) * 64;
    const int cmin_tile = j.mode == kModeAuto ? (r0 + j.wp) / 64 : 0;
    if (cmin_tile <= j.c_last) {
        const int c = cmin_tile + (int)((z >> 32) % (uint64_t)(j.c_last - cmin_tile + 1));
        const float *rec = j.box + kBoxHeader + (int64_t)c * kBoxStride;
        bool all = true;
        for (int i = r0; i < r0 + 64 && all; ++i) {
            const int ii = i < j.n ? i : j.n - 1;
            bool out = false;
            for (int k = 0; k < K; ++k) {
                const float x = j.s[ii + (int64_t)k * j.tau];
                out = out || x < rec[2 * k] || x > rec[2 * k + 1];
            }
            all = out;
        }
        if (all) atomicAdd(&decided, 1);
        atomicAdd(&sampled, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        reinterpret_cast<int *>(j.box)[0] = (sampled > 0 && 64 * decided >= sampled) ? 1 : 0;
}

// Reset the non-finite flags and the work counters (runs before k_prepare).
__global__ void k_reset(const JobDesc *__restrict__ jobs, int njobs, int *counters, int ncounters) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < njobs) *jobs[t].flag = 0;
    if (t < ncounters) counters[t] = 0;
}

// Write the descriptors of a one-job launch from kernel arguments (the launch
// path that may not copy from host memory: nothing to stage, nothing to free).
__global__ void k_setup(const JobDesc d, const GroupDesc g, JobDesc *ddesc, GroupDesc *dgroups) {
    if (threadIdx.x == 0) {
        *ddesc = d;
        *dgroups = g;
    }
}

// Move a one-job launch to row band b: its strips [b K, min((b+1) K, S)), the
// origin of their summary slots, the band's work items, and a fresh work
// counter (K strips per band, S strips in all).
__global__ void k_band(JobDesc *jobs, GroupDesc *groups, int *counters, int b) {
    if (threadIdx.x != 0) return;
    JobDesc &j = jobs[0];
    const int lo = b * j.band_strips;
    const int hi = lo + j.band_strips < j.nstrips ? lo + j.band_strips : j.nstrips;
    j.s_lo = lo;
    j.s_hi = hi;
    j.soff_lo = strip_offset(lo, j.n, j.wp, j.H);
    groups[0].items = (hi - lo) * j.segs;
    counters[0] = 0;
}

// ---------------------------------------------------------------------------
// Kernel 2: the fused tile pass.  Persistent workgroups pull (job, strip) work
// items of one (norm, m) group from a counter.
// ---------------------------------------------------------------------------
// LDS of a tile workgroup (dynamic shared memory): privatised histogram bins;
// for each pair of consecutive waves a ring of kRing carry slots (vertical and
// diagonal states of one tile, one u32 per lane); the produced / consumed tile
// counters of those rings; the current work item.  Sized for the launch's wave
// count (48 KB for 8 waves).  The kernel is compiled for six waves per SIMD (at
// most 80 VGPRs, no spills), i.e. three 8-wave workgroups per CU.
struct StripLds {
    uint32_t *bd, *bv, *bw;
    uint32_t *vslot;    // [kRing][waves][64]
    uint32_t *dslot;    // [kRing][waves][64]
    int *prod;          // [kMaxWaves]: tiles whose carries wave w has written
    int *cons;          // [kMaxWaves]: tiles whose carries wave w+1 has read
    int *item;
    int nw;
    __device__ uint32_t &vs(int buf, int w, int lane) { return vslot[(buf * nw + w) * 64 + lane]; }
    __device__ uint32_t &ds(int buf, int w, int lane) { return dslot[(buf * nw + w) * 64 + lane]; }
};

__host__ __device__ constexpr size_t strip_lds_bytes(int waves) {
    return sizeof(uint32_t) * ((size_t)kCapD + kCapV + kCapW + 2 * (size_t)kRing * waves * 64 +
                               2 * kMaxWaves) + 16;
}

// Wait (wave-uniform) until the counter reaches `target`.  Each wait is bounded:
// past `limit` polls it gives up and returns false, so a wave never hangs.
__device__ __forceinline__ bool wait_counter(int *ctr, int target, const JobDesc &j) {
    int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (v >= target) return true;
    // The bound is read only when the first poll fails (most waits need none;
    // reading it, and the target's bias, from the descriptor on every wait
    // cost 2.5 ms of 74 on the 1M-point workload).
    const uint32_t limit = (uint32_t)j.spin_limit;
    for (uint32_t spin = 0; spin < limit; ++spin) {
        __builtin_amdgcn_s_sleep(1);
        v = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (v >= target) return true;
    }
    return false;
}

__device__ __forceinline__ void publish_counter(int *ctr, int value) {
    __hip_atomic_store(ctr, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ void flush_bins(const StripLds &L, const JobDesc &j) {
    const int hl = j.hmax + 1;
    for (int t = threadIdx.x; t < kCapW; t += blockDim.x) {
        if (t < kCapD) {
            const uint32_t v = L.bd[t];
            if (v) { if (t < hl) g_add(j.hd + t, (unsigned long long)v); L.bd[t] = 0; }
        }
        if (t < kCapV) {
            const uint32_t v = L.bv[t];
            if (v) { if (t < hl) g_add(j.hv + t, (unsigned long long)v); L.bv[t] = 0; }
        }
        const uint32_t v = L.bw[t];
        if (v) { if (t < hl) g_add(j.hw + t, (unsigned long long)v); L.bw[t] = 0; }
    }
}

// One strip of one job.  MODE kModeAuto: the upper triangle U of the symmetric
// recurrence matrix of one series (horizontal runs are the row segments of the
// full columns, joined through the band by the stitch).  MODE kModeCross /
// kModeMatrix: a full n x nb matrix that is not symmetric (every diagonal and
// every column walked once; no horizontal runs).
template <int NORM, int M, int MODE>
__device__ void process_strip(const JobDesc &j, int item, StripLds &L) {
    static_assert(kMaxWaves <= 8, "LDS budget assumes at most 8 waves per workgroup");
    constexpr bool FULL = MODE != kModeAuto;
    constexpr int kDW = FULL ? 1 : 2;   // lines per diagonal run found
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int nw = blockDim.x >> 6;
    const int n = j.n, wp = j.wp, H = j.H, tau = j.tau;   // n: rows
    const int nb = FULL ? j.nb : n;                        // columns
    const int64_t band = j.theiler;                        // full matrix: cells |i-j| < band are 0
    // Work item: a (strip, column segment) block; with one segment per strip
    // (auto mode, many strips) the whole strip.
    const int G = j.segs;
    const bool BLK = FULL || G > 1;              // per-block diagonal summaries
    const int lstrip = item / G;                 // strip within the row band (auto)
    const int strip = j.s_lo + lstrip;
    const int seg = item - lstrip * G;
    const int R0 = strip * H;
    const int R = R0 + 64 * wave;
    const int i = R + lane;                      // this lane's row
    const int c0 = FULL ? 0 : (R0 + wp) >> 6;
    const int T = j.c_last - c0 + 1;             // tiles of the strip
    // Tiles [ta, tb) of this block (relative to c0): the segment's absolute
    // column tiles cut to the strip's.  A block that does not start at the
    // strip's first tile begins with the row and diagonal runs that enter
    // through its left edge, of unknown history.
    const int sa = j.seg_base + seg * j.seg_tiles - c0;
    const int ta = sa > 0 ? sa : 0;
    const int tb = sa + j.seg_tiles < T ? sa + j.seg_tiles : T;
    if (ta >= tb) return;                        // the triangle leaves this block empty
    const bool seg_start = ta > 0;
    // Some row of this wave has cells to walk, and the first tile that has.
    const bool wave_has_u = FULL ? R <= n - 1 : R + wp <= n - 1;
    const int cfirst = FULL ? 0 : (R + wp) >> 6;
    const int64_t soff = FULL ? 0 : strip_offset(strip, n, wp, H) - j.soff_lo;
    // Summary slots: columns -- per (strip, column), in triangular strip order
    // from the row band's first strip in auto mode; diagonals -- auto with one
    // segment: per (strip, diagonal of U) in the same order; otherwise per
    // work item (a (strip, segment) block) j.dw slots for the diagonals
    // k = x0-(R0+H-1) .. x1-1-R0 that have a cell in the block's columns [x0, x1).
    const int x0 = (c0 + ta) * 64;
    const int x1 = (c0 + tb) * 64 < nb ? (c0 + tb) * 64 : nb;
    const int64_t vbase = FULL ? (int64_t)lstrip * nb : soff - R0 - wp;
    const int64_t dbase = BLK ? (int64_t)item * j.dw + (R0 + H - 1) - x0 : soff - wp;
    const int kmin = BLK ? (FULL || x0 - (R0 + H - 1) > wp ? x0 - (R0 + H - 1) : wp) : wp;
    const int kmax = BLK ? x1 - 1 - R0 : n - 1 - R0;
    auto dok = [&](int k) -> bool { return k >= kmin && k <= kmax; };

    // Column boxes of this job, when the probe chose to use them.
    // (The header is read as a scalar load, so `box` is known to be uniform
    // and the records are read with scalar loads too.)
    ConstF box = nullptr;
    if constexpr (MODE != kModeMatrix && M > 0) {
        const ConstF bx = to_const(j.box);
        if (bx != nullptr && __float_as_int(bx[0]) != 0) box = bx + kBoxHeader;
    }

    // Row coordinates of this lane (clamped for rows past the end).
    const int irow = i < n ? i : n - 1;
    const float *rowp = MODE == kModeMatrix ? nullptr : j.s + irow;
    float xr[M > 0 ? M : 1] = {};
    if constexpr (MODE != kModeMatrix) {
#pragma unroll
        for (int k = 0; k < (M > 0 ? M : 1); ++k) xr[k] = M > 0 ? glb(rowp)[(int64_t)k * tau] : 0.0f;
        // Wait for these loads here, once per strip: gfx950 counts outstanding
        // global stores and atomics in the same counter as loads, so a wait
        // for them at their first use inside the tile loop would also wait
        // for every summary store and histogram atomic still in flight.
#pragma unroll
        for (int k = 0; k < (M > 0 ? M : 1); ++k) asm volatile("" : "+v"(xr[k]));
    }

    Bins bins{L.bd, L.bv, L.bw};
    // Horizontal runs: with segments, each row's piece in this block records
    // its first and last runs (hfirst / hlast); otherwise the row's first run
    // is its lead.
    const LineCtx hctx{&j, bins, (int64_t)(i - j.s_lo * H) * G + seg, G > 1, (uint32_t)i};
    Run hs{0, 0, 0};          // horizontal run of this lane's row (auto)
    bool hstarted = false;
    Run left{0, 0, 0};        // diagonal carry from the previous tile (upper part end)

    // The waves form a pipeline over the tiles: wave w reads the carries that
    // wave w-1 wrote for the same tile and writes its own for wave w+1, through a
    // ring of kRing slots per wave pair.  A wave waits only for its neighbours:
    // for the tile's carries from above and for a free slot below.
    const int tfirst = cfirst - c0 > ta ? cfirst - c0 : ta;   // first tile with cells for this wave
    if (wave > 0) publish_counter(&L.cons[wave - 1], wave_has_u ? tfirst : 0x7FFFFFFF);
    bool sync_ok = true;
    const int wbias = j.wait_bias;   // 0 (a test injecting give-ups sets it), read once per strip
    // Given matrix: the next tile's row word is loaded while the current tile
    // is processed (one load in flight per lane hides the memory latency that
    // otherwise sets the pace of a strip; loading 2, 4 or 8 tiles ahead
    // measured no faster).
    const auto mrow = MODE == kModeMatrix && i < n ? glb(j.bits) + (int64_t)i * j.words : nullptr;
    uint64_t mnext = 0;
    if constexpr (MODE == kModeMatrix) {
        if (mrow && wave_has_u && tfirst < tb) mnext = mrow[c0 + tfirst];
    }
    for (int t = wave_has_u ? tfirst : tb; t < tb; ++t) {
        const int c = c0 + t;
        const int slot = t & (kRing - 1);
        {
            const int jbase = c * 64;
            uint32_t xlo, xhi;
            if constexpr (MODE == kModeMatrix) {
                const uint64_t word = mnext;
                if (mrow && t + 1 < tb) mnext = mrow[c + 1];
                xlo = (uint32_t)word;
                xhi = (uint32_t)(word >> 32);
            } else {
                const ConstF cols = to_const((c == j.c_last) ? j.tail : j.sb + jbase);
                tile_bits<NORM, M>(cols, tau, xr, rowp, j.m, j.thr, j.thr0,
                                          box == nullptr ? nullptr : box + (int64_t)c * kBoxStride,
                                          xlo, xhi);
            }

            // Interior tile: no cell needs masking, and every column and
            // diagonal continues below this wave.
            bool interior;
            if constexpr (FULL) {
                interior = R + 64 <= n - 1 && jbase + 63 <= nb - 1 &&
                           (band == 0 || (int64_t)jbase - (R + 63) >= band ||
                            (int64_t)R - (jbase + 63) >= band);
            } else {
                interior = jbase >= R + 64 + wp && jbase + 63 <= n - 1;
            }
            int lo_v = 0, hi_v = 64;
            uint64_t vmask = ~0ull;
            uint64_t X = mk64(xlo, xhi);
            if (!interior) {
                if constexpr (FULL) {
                    // Valid cells of this row: columns [0, nb) outside the band.
                    vmask = 0ull;
                    if (i < n) {
                        const int hv = nb - jbase < 64 ? nb - jbase : 64;
                        vmask = hv > 0 ? range_mask(0, hv) : 0ull;
                        if (band > 0) {
                            int64_t blo = (int64_t)i - band + 1 - jbase, bhi = (int64_t)i + band - jbase;
                            blo = blo < 0 ? 0 : blo;
                            bhi = bhi > 64 ? 64 : bhi;
                            if (blo < bhi) vmask &= ~range_mask((uint32_t)blo, (uint32_t)bhi);
                        }
                    }
                } else {
                    // Valid cells of this row: columns [i + wp, n-1], rows < n.
                    lo_v = i + wp - jbase;
                    lo_v = lo_v < 0 ? 0 : lo_v;
                    if (i >= n || lo_v > 64) lo_v = 64;
                    hi_v = n - jbase;
                    hi_v = hi_v > 64 ? 64 : hi_v;
                    vmask = lo_v < hi_v ? range_mask(lo_v, hi_v) : 0ull;
                }
                X &= vmask;
                xlo = (uint32_t)X;
                xhi = (uint32_t)(X >> 32);
            }

            const bool any = __ballot(X != 0ull) != 0ull;

            // First tile of a full-matrix block that does not start at the left
            // border: the diagonals entering through its left edge start a
            // segment here.  Lane q's lower part (q > 0) begins at cell
            // (R + 64 - q, jbase), bit 0 of lane 64 - q's row word; lane 0's
            // lower part is empty and its diagonal enters the block in the wave
            // below, which starts it (`fresh_up`).
            const bool fresh = seg_start && t == ta;
            if (fresh) {
                const uint64_t col0 = __ballot((X & 1ull) != 0ull);
                left = lane == 0 ? Run{0u, 0u, 0u}
                                 : Run{(uint32_t)(col0 >> (64 - lane)) & 1u, 0u, 1u};
                // A row of U that began left of this block enters it here.
                if constexpr (!FULL) {
                    if (i < n && i + wp < jbase) {
                        hs = Run{(uint32_t)(X & 1ull), 0u, 1u};
                        hstarted = true;
                    }
                }
            }
            // The upper part of this lane's diagonal starts a segment in this
            // tile: on the strip's top edge (wave 0), or for lane 0 on the
            // block's left edge.
            const bool fresh_up = wave == 0 || (fresh && lane == 0);

            // This tile's carries from the wave above, and a free slot below.
            // After one wait has given up the wave stops waiting (the job is
            // flagged as failed), so a strip finishes in bounded time.
            if (wave > 0 && sync_ok)
                sync_ok = wait_counter(&L.prod[wave - 1], t + 1 + wbias, j);
            if (wave < nw - 1 && sync_ok)
                sync_ok = wait_counter(&L.cons[wave], t - kRing + 1 + wbias, j);

            if (interior && !any) {
                // No recurrence in an interior tile: every open run sees 64
                // white cells.  Only carried states change; a black run that
                // was open ends at the tile's first cell.
                if constexpr (!FULL) {
                    if (hs.color) {
                        finish_run<kHoriz>(hctx, 1u, hs.len, hs.first);
                        hs = Run{0u, 64u, 0u};
                    } else {
                        hs.len += 64u;
                    }
                }
                {
                    Run st = wave == 0 ? Run{0u, 0u, 1u} : unpack_run(L.vs(slot, wave - 1, lane));
                    const int64_t sidx = vbase + (jbase + lane);
                    if (st.color) {
                        const LineCtx lc{&j, bins, sidx, true, 0u};
                        finish_run<kVert>(lc, 1u, st.len, st.first);
                        st = Run{0u, 64u, 0u};
                    } else {
                        st.len += 64u;
                    }
                    if (wave == nw - 1) {
                        const uint16_t pk = (uint16_t)(st.len | (st.color << 15));
                        if (st.first) *glb(j.vfirst + sidx) = pk;   // one run: its last is its first
                        else *glb(j.vlast + sidx) = pk;
                    } else {
                        L.vs(slot, wave, lane) = pack_run(st);
                    }
                }
                {
                    // Interior: both diagonal parts of every lane are valid and
                    // continue on the next row.
                    const int kup = jbase + lane - R;
                    const int klo = kup - 64;
                    Run up;
                    if (fresh_up) {
                        if (!FULL || dok(kup)) *glb(j.dfirst + dbase + kup) = 0;   // white first cell
                        up = Run{0u, 0u, 0u};
                    } else {
                        up = unpack_run(L.ds(slot, wave - 1, lane));
                    }
                    if (up.color) {
                        const LineCtx lc{&j, bins, dbase + kup, true, 0u};
                        finish_run<kDiag, kDW>(lc, 1u, up.len, up.first);
                        up = Run{0u, 0u, 0u};
                    }
                    // Lane 0's lower part is empty (its diagonal left this wave
                    // at the previous tile's corner): its run goes on unchanged.
                    Run lw = left;
                    if (lw.color && lane != 0) {
                        const LineCtx lc{&j, bins, dbase + klo, !FULL || dok(klo), 0u};
                        finish_run<kDiag, kDW>(lc, 1u, lw.len, lw.first);
                        lw = Run{0u, 0u, 0u};
                    }
                    if (wave < nw - 1) {
                        L.ds(slot, wave, lane) = pack_run(lw);
                    } else if (!FULL || dok(klo)) {
                        const uint16_t b = (uint16_t)(lw.color ? lw.len : 0u);
                        // A black run over the whole piece: the stitch reads only its first
                        // (a white one reads as 0 and needs its last too).
                        if (lw.first && lw.color) {
                            *glb(j.dfirst + dbase + klo) = b;
                        } else {
                            *glb(j.dlast + dbase + klo) = b;
                            if (lw.first) *glb(j.dfirst + dbase + klo) = b;
                        }
                    }
                    left = up;
                }
                if (wave > 0) publish_counter(&L.cons[wave - 1], t + 1);
                if (wave < nw - 1) publish_counter(&L.prod[wave], t + 1);
                continue;
            }

            if (interior && __ballot(X != ~0ull) == 0ull) {
                // Every cell of an interior tile recurrent (dense series): the
                // mirror image of the empty case.  Open white runs end at the
                // tile's first cell, black runs grow by the cells they cross.
                if constexpr (!FULL) {
                    if (!hs.color) {
                        finish_run<kHoriz>(hctx, 0u, hs.len, hs.first);
                        hs = Run{1u, 64u, 0u};
                    } else {
                        hs.len += 64u;
                    }
                }
                {
                    Run st = wave == 0 ? Run{1u, 0u, 1u} : unpack_run(L.vs(slot, wave - 1, lane));
                    const int64_t sidx = vbase + (jbase + lane);
                    if (!st.color) {
                        const LineCtx lc{&j, bins, sidx, true, 0u};
                        finish_run<kVert>(lc, 0u, st.len, st.first);
                        st = Run{1u, 64u, 0u};
                    } else {
                        st.len += 64u;
                    }
                    if (wave == nw - 1) {
                        const uint16_t pk = (uint16_t)(st.len | (st.color << 15));
                        if (st.first) *glb(j.vfirst + sidx) = pk;   // one run: its last is its first
                        else *glb(j.vlast + sidx) = pk;
                    } else {
                        L.vs(slot, wave, lane) = pack_run(st);
                    }
                }
                {
                    // Lane q's diagonal has 64 - q cells in the upper part and
                    // q in the lower part (none for lane 0, whose lower run
                    // passes through unchanged).
                    const int kup = jbase + lane - R;
                    const int klo = kup - 64;
                    const uint32_t nup = 64u - (uint32_t)lane;
                    Run up;
                    if (fresh_up) {
                        up = Run{1u, nup, 1u};   // black first run from the block's edge
                    } else {
                        up = unpack_run(L.ds(slot, wave - 1, lane));
                        if (up.color) {
                            up.len += nup;
                        } else {
                            if (up.first) {
                                const LineCtx lc{&j, bins, dbase + kup, !FULL || dok(kup), 0u};
                                finish_run<kDiag, kDW>(lc, 0u, up.len, 1u);
                            }
                            up = Run{1u, nup, 0u};
                        }
                    }
                    Run lw = left;
                    if (lane != 0) {
                        if (lw.color) {
                            lw.len += (uint32_t)lane;
                        } else {
                            if (lw.first) {
                                const LineCtx lc{&j, bins, dbase + klo, !FULL || dok(klo), 0u};
                                finish_run<kDiag, kDW>(lc, 0u, lw.len, 1u);
                            }
                            lw = Run{1u, (uint32_t)lane, 0u};
                        }
                    }
                    if (wave < nw - 1) {
                        L.ds(slot, wave, lane) = pack_run(lw);
                    } else if (!FULL || dok(klo)) {
                        const uint16_t b = (uint16_t)(lw.color ? lw.len : 0u);
                        // A black run over the whole piece: the stitch reads only its first
                        // (a white one reads as 0 and needs its last too).
                        if (lw.first && lw.color) {
                            *glb(j.dfirst + dbase + klo) = b;
                        } else {
                            *glb(j.dlast + dbase + klo) = b;
                            if (lw.first) *glb(j.dfirst + dbase + klo) = b;
                        }
                    }
                    left = up;
                }
                if (wave > 0) publish_counter(&L.cons[wave - 1], t + 1);
                if (wave < nw - 1) publish_counter(&L.prod[wave], t + 1);
                continue;
            }

            // ---- horizontal runs (row i of U) ----
            if constexpr (!FULL) {
                if (lo_v < hi_v) {
                    if (!hstarted) {
                        hstarted = true;
                        hs = Run{(uint32_t)((X >> lo_v) & 1ull), 0u, 1u};
                    }
                    run_segment<kHoriz>(X, vmask, (uint32_t)lo_v, (uint32_t)hi_v, hs, hctx);
                }
            }

            // ---- vertical runs (columns) ----
            {
                uint32_t ylo = xlo, yhi = xhi;
                if (any) transpose64(ylo, yhi, lane);
                else { ylo = 0; yhi = 0; }
                const uint64_t Y = mk64(ylo, yhi);
                const int jc = jbase + lane;
                // last valid local row of column jc: the band (auto) or the
                // bottom border (full) ends its segment
                const int e = interior ? 64 : (FULL ? n - 1 - R : jc - wp - R);
                if (interior || (jc <= nb - 1 && e >= 0)) {
                    const uint32_t vhi = e >= 63 ? 64u : (uint32_t)(e + 1);
                    Run st;
                    if (wave == 0) st = Run{(uint32_t)(Y & 1ull), 0u, 1u};
                    else st = unpack_run(L.vs(slot, wave - 1, lane));
                    const int64_t sidx = vbase + jc;
                    LineCtx lc{&j, bins, sidx, true, 0u};
                    const uint64_t vwin = vhi >= 64 ? ~0ull : ((1ull << vhi) - 1ull);
                    run_segment<kVert>(Y, vwin, 0u, vhi, st, lc);
                    if (e <= 63 || wave == nw - 1) {
                        const uint16_t pk = (uint16_t)(st.len | (st.color << 15));
                        if (st.first) *glb(j.vfirst + sidx) = pk;   // one run: its last is its first
                        else *glb(j.vlast + sidx) = pk;
                    } else {
                        L.vs(slot, wave, lane) = pack_run(st);
                    }
                }
            }

            // ---- diagonal runs ----
            {
                uint32_t zlo = xlo, zhi = xhi;
                if (any) {
                    rotr64(zlo, zhi, (uint32_t)lane);
                    transpose64(zlo, zhi, lane);
                } else {
                    zlo = 0;
                    zhi = 0;
                }
                const uint64_t D = mk64(zlo, zhi);
                const int q = lane;
                const int kup = jbase + q - R;          // diagonal of the upper part
                const int klo = kup - 64;               // diagonal of the lower part
                const uint64_t upwin = q == 0 ? ~0ull : ((1ull << (64 - q)) - 1ull);
                Run up;
                if (fresh_up) {
                    // Segment start on the strip's top row (or the block's left
                    // edge).  A white first cell means "no black run at the
                    // edge": record it at once (white diagonal runs are never
                    // counted, so their length does not matter).
                    up = Run{(uint32_t)(D & 1ull), 0u, 1u};
                    if (!up.color) {
                        if (dok(kup)) *glb(j.dfirst + dbase + kup) = 0;
                        up.first = 0;
                    }
                } else if (jbase + q > nb - 1) {
                    up = Run{0u, 0u, 0u};   // starts past the border
                } else {
                    up = unpack_run(L.ds(slot, wave - 1, lane));
                }
                {
                    LineCtx lc{&j, bins, dbase + kup, dok(kup), 0u};
                    run_segment<kDiag, kDW>(D, upwin, 0u, (uint32_t)(64 - q), up, lc);
                }
                Run lw = left;
                {
                    const bool ok = dok(klo);
                    LineCtx lc{&j, bins, dbase + klo, ok, 0u};
                    run_segment<kDiag, kDW>(D, ~upwin, (uint32_t)(64 - q), 64u, lw, lc);
                    // The lower part ends on row R+63.  Diagonals with no cell on
                    // the next row end here at the right (or, full matrix,
                    // bottom) border; the others go to the wave below or, from
                    // the last wave, into the summary.
                    const bool ends = FULL ? (R + 64 > n - 1 || R + 64 + klo > nb - 1)
                                           : (R + 64 + klo > n - 1);
                    if (ends) {
                        if (lw.color || lw.first) finish_run<kDiag, kDW>(lc, lw.color, lw.len, lw.first);
                    } else if (wave < nw - 1) {
                        L.ds(slot, wave, lane) = pack_run(lw);
                    } else if (ok) {
                        const uint16_t b = (uint16_t)(lw.color ? lw.len : 0u);
                        // A black run over the whole piece: the stitch reads only its first
                        // (a white one reads as 0 and needs its last too).
                        if (lw.first && lw.color) {
                            *glb(j.dfirst + dbase + klo) = b;
                        } else {
                            *glb(j.dlast + dbase + klo) = b;
                            if (lw.first) *glb(j.dfirst + dbase + klo) = b;
                        }
                    }
                }
                left = up;
            }
        }
        if (wave > 0) publish_counter(&L.cons[wave - 1], t + 1);
        if (wave < nw - 1) publish_counter(&L.prod[wave], t + 1);
    }
    if (!sync_ok) g_or(j.flag, 8);   // a neighbour wait gave up: result invalid

    if (wave_has_u) {
        // Rows end at column n-1: their last run is complete; a block that is
        // not the strip's last records each row's open run as its last.
        if constexpr (!FULL) {
            if (hstarted) {
                if (tb == T) {
                    finish_run<kHoriz>(hctx, hs.color, hs.len, hs.first);
                } else {
                    const uint32_t h = hs.len | (hs.color << 31);
                    if (hs.first) *glb(j.hfirst + hctx.sum_idx) = h;
                    else *glb(j.hlast + hctx.sum_idx) = h;
                }
            }
        }
        // Upper parts that left the last tile on its right edge end at the
        // border, and so do those whose next cell (one row down, in the next
        // block) lies below the matrix; the others go on in the next block:
        // recorded as the block's last runs.
        const int kup = (c0 + tb - 1) * 64 + lane - R;
        if (tb == T || R + 64 - lane > n - 1) {
            LineCtx lc{&j, bins, dbase + kup, dok(kup), 0u};
            if (left.color || left.first) finish_run<kDiag, kDW>(lc, left.color, left.len, left.first);
        } else if (dok(kup)) {
            const uint16_t b = (uint16_t)(left.color ? left.len : 0u);
            // A black run over the whole piece: the stitch reads only its first
            // (a white one reads as 0 and needs its last too).
            if (left.first && left.color) {
                *glb(j.dfirst + dbase + kup) = b;
            } else {
                *glb(j.dlast + dbase + kup) = b;
                if (left.first) *glb(j.dfirst + dbase + kup) = b;
            }
        }
    }
}

template <int NORM, int M, int MODE>
__global__ void __launch_bounds__(64 * kMaxWaves) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_tiles(const JobDesc *__restrict__ jobs, const GroupDesc *__restrict__ groups, int g,
        int *counters) {
    extern __shared__ uint32_t lds_words[];
    const int nw = blockDim.x >> 6;
    StripLds L;
    L.bd = lds_words;
    L.bv = L.bd + kCapD;
    L.bw = L.bv + kCapV;
    L.vslot = L.bw + kCapW;
    L.dslot = L.vslot + kRing * nw * 64;
    L.prod = reinterpret_cast<int *>(L.dslot + kRing * nw * 64);
    L.cons = L.prod + kMaxWaves;
    L.item = L.cons + kMaxWaves;
    L.nw = nw;
    const GroupDesc gd = groups[g];
    for (int t = threadIdx.x; t < kCapW; t += blockDim.x) {
        if (t < kCapD) L.bd[t] = 0;
        if (t < kCapV) L.bv[t] = 0;
        L.bw[t] = 0;
    }
    __syncthreads();
    while (true) {
        if (threadIdx.x == 0) *L.item = atomicAdd(counters + g, 1);
        if (threadIdx.x < 2 * kMaxWaves) L.prod[threadIdx.x] = 0;   // prod and cons
        __syncthreads();
        const int item = *L.item;
        __syncthreads();
        if (item >= gd.items) break;
        // locate the job: largest job index in [job0, job1) with strip_base <= item
        int lo = gd.job0, hi = gd.job1 - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].strip_base <= item) lo = mid; else hi = mid - 1;
        }
        // By reference: fields are re-read with scalar loads where needed
        // instead of occupying SGPRs for the whole strip.
        const JobDesc &j = jobs[lo];
        process_strip<NORM, M, MODE>(j, item - j.strip_base, L);
        __syncthreads();
        flush_bins(L, j);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Kernel 3: stitch and join.  One thread per line: columns j in [0, n) fold their
// per-strip segment summaries and join the trailing run of column j of U with
// the middle and the leading run of row j of U; diagonals k in [w', n) fold
// their summaries.  Runs crossing strip edges are counted here.
// ---------------------------------------------------------------------------
struct StitchLds {
    uint32_t bd[kCapD];
    uint32_t bv[kStitchCapV];
    uint32_t bw[kCapW];
};

// Global histogram add in which the active lanes of the wave that add to the
// same bin are combined into one atomic (64-bit atomics on one address
// serialise in L2; in the stitch, neighbouring lines of a smooth series end long
// runs of equal length together).
__device__ __forceinline__ void g_add_combined(unsigned long long *p, uint32_t w) {
    const uint64_t a = (uint64_t)(uintptr_t)p;
    // At most 64 rounds: each retires at least the first active lane (its own
    // address matches); the bound keeps a wave from spinning whatever happens.
    for (int round = 0; round < 64; ++round) {
        // readfirstlane returns int: go through uint32_t so that the low half
        // is not sign-extended into the high one.
        const uint32_t lo0 = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
        const uint32_t hi0 = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
        const uint64_t a0 = ((uint64_t)hi0 << 32) | (uint64_t)lo0;
        // The ballot is taken by every active lane, before the branch.
        const uint64_t same = __builtin_amdgcn_ballot_w64(a == a0);
        if (a == a0) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
            if (below == 0u)
                g_add(p, (unsigned long long)w * (unsigned long long)__builtin_popcountll(same));
            break;
        }
    }
}

// Stitch emission: LDS bin below the cap, else the combined global add.
__device__ __forceinline__ void emit_stitch(uint32_t *bins, int cap, unsigned long long *glob,
                                            uint32_t len, uint32_t wt, uint32_t n, int *flag) {
    if (len < (uint32_t)cap && len <= n)
        atomicAdd(bins + len, wt);
    else if (len <= n)
        g_add_combined(glob + len, wt);
    else
        g_or(flag, 2);
}

__device__ __forceinline__ void emit_line(StitchLds &L, const JobDesc &j, uint32_t color,
                                          uint32_t len) {
    if (len == 0) return;
    if (color) emit_stitch(L.bv, kStitchCapV, j.hv, len, 1u, (uint32_t)j.hmax, j.flag);
    else emit_stitch(L.bw, kCapW, j.hw, len, 1u, (uint32_t)j.hmax, j.flag);
}

// Segment of column x (a column of segment g lies in the column tiles
// [seg_base + g*seg_tiles, seg_base + (g+1)*seg_tiles)).
__device__ __forceinline__ int seg_of(const JobDesc &j, int x) {
    return ((x >> 6) - j.seg_base) / j.seg_tiles;
}

// Row r of U, cut into pieces by the column segments (auto mode, segs > 1):
// fold the pieces' first and last runs in order, count the runs that span
// piece edges and return the row's first (leading) run, which the join with
// column r needs.  Runs inside a piece were counted by the tile kernel, and so
// was the last piece's final run at column n-1 unless it is that piece's
// first.
__device__ void row_pieces(StitchLds &L, const JobDesc &j, int r, uint32_t &lc, uint32_t &ll) {
    const int n = j.n;
    const int a = r + j.wp;                     // first column of the row
    const int W = j.seg_tiles * 64;
    bool lead_open = true, have = false;
    uint32_t oc = 0, ol = 0;
    lc = 0;
    ll = 0;
    auto close = [&](uint32_t c, uint32_t l) {
        if (lead_open) { lc = c; ll = l; lead_open = false; }
        else emit_line(L, j, c, l);
    };
    const int gl = seg_of(j, n - 1);
    for (int g = seg_of(j, a); g <= gl; ++g) {
        const int g0 = (j.seg_base + g * j.seg_tiles) * 64;
        const int lo = a > g0 ? a : g0;
        const int hi = n - 1 < g0 + W - 1 ? n - 1 : g0 + W - 1;
        const uint32_t len = (uint32_t)(hi - lo + 1);
        const bool last = g == gl;
        const int64_t idx = (int64_t)(r - j.s_lo * j.H) * j.segs + g;   // rows of the band
        const uint32_t f = *glb(j.hfirst + idx);
        const uint32_t fc = f >> 31, fl = f & 0x7FFFFFFFu;
        if (have && fc == oc) {
            ol += fl;
        } else {
            if (have) close(oc, ol);
            oc = fc;
            ol = fl;
            have = true;
        }
        if (fl == len && !last) continue;       // the piece is one run: it stays open
        close(oc, ol);                          // the open run ends in this piece
        have = false;
        if (!last) {
            const uint32_t h = *glb(j.hlast + idx);
            oc = h >> 31;
            ol = h & 0x7FFFFFFFu;
            have = true;
        }
    }
}

// Stitch of a full (not symmetric) matrix: lines [0, nb) are the columns, lines
// [nb, nb + n + nb - 1) the diagonals k = -(n-1) .. nb-1.  A diagonal that
// starts inside a strip (at the left border) has no top-edge summary there.
__device__ __forceinline__ void stitch_full(StitchLds &L, const JobDesc &j, int64_t line) {
    const int n = j.n, nb = j.nb, H = j.H, S = j.nstrips;
    // Strips [s_lo, s_hi) of one row band (all strips with one band): a line
    // goes on from the open run an earlier band left in cstate / dstate, and
    // leaves its own there unless its last piece is in this band.
    const int s_lo = j.s_lo, s_hi = j.s_hi;
    const bool first_band = s_lo == 0, last_band = s_hi >= S;
    if (line < nb) {
        const int col = (int)line;
        uint32_t oc = 0, ol = 0;
        if (!first_band) {
            const uint32_t c = *glb(j.cstate + col);
            oc = c >> 31;
            ol = c & 0x7FFFFFFFu;
        }
        for (int s0 = s_lo; s0 < s_hi; s0 += kStitchBatch) {
            uint32_t fv[kStitchBatch], lv[kStitchBatch];
#pragma unroll
            for (int u = 0; u < kStitchBatch; ++u) {
                const int64_t idx = (int64_t)(s0 + u - s_lo) * nb + col;
                if (s0 + u < s_hi) {
                    fv[u] = *glb(j.vfirst + idx);
                    lv[u] = *glb(j.vlast + idx);
                }
            }
#pragma unroll
            for (int u = 0; u < kStitchBatch; ++u) {
                const int s = s0 + u;
                if (s >= s_hi) break;
                const uint32_t Ls = s < S - 1 ? (uint32_t)H : (uint32_t)(n - s * H);
                const uint32_t f = fv[u], l = lv[u];
                const uint32_t fc = f >> 15, fl = f & 0x7FFFu;
                if (fl == Ls) {   // the segment is one run
                    if (ol && oc == fc) ol += Ls;
                    else { emit_line(L, j, oc, ol); oc = fc; ol = Ls; }
                } else {
                    if (ol && oc == fc) emit_line(L, j, fc, ol + fl);
                    else { emit_line(L, j, oc, ol); emit_line(L, j, fc, fl); }
                    oc = l >> 15;
                    ol = l & 0x7FFFu;
                }
            }
        }
        if (last_band) emit_line(L, j, oc, ol);
        else *glb(j.cstate + col) = ol | (oc << 31);
    } else if (line < (int64_t)nb + n + nb - 1) {
        // Diagonal k: its pieces in the (strip, segment) blocks it crosses, in
        // order; a block's first and last black runs are folded across edges.
        const int dk = (int)(line - nb);                            // carry slot
        const int k = dk - (n - 1);
        const int r0 = k < 0 ? -k : 0;                              // first row
        const int r1 = n - 1 < nb - 1 - k ? n - 1 : nb - 1 - k;     // last row
        const int sa = r0 / H > s_lo ? r0 / H : s_lo;               // its strips in this band
        const int sb = r1 / H < s_hi - 1 ? r1 / H : s_hi - 1;
        if (sa > sb) return;
        const int W = j.seg_tiles * 64;                             // segment width
        uint32_t open = r0 / H < s_lo ? (uint32_t)*glb(j.dstate + dk) : 0u;
        for (int s = sa; s <= sb; ++s) {
            const int ra = r0 > s * H ? r0 : s * H;
            const int rb = r1 < s * H + H - 1 ? r1 : s * H + H - 1;
            const int ca = ra + k, cb = rb + k;                     // its columns in strip s
            for (int g = ca / W; g <= cb / W; ++g) {
                const int lo = ca > g * W ? ca : g * W;
                const int hi = cb < g * W + W - 1 ? cb : g * W + W - 1;
                const uint32_t len = (uint32_t)(hi - lo + 1);
                const bool last = rb == r1 && hi == cb;
                const int64_t idx = (int64_t)((s - s_lo) * j.segs + g) * j.dw + (s * H + H - 1 - g * W) + k;
                // A piece that begins where the diagonal begins, below the
                // strip's top row, starts at the matrix's left border: nothing
                // enters it, and its runs were counted where they ended.
                if (!(lo == ca && ra > s * H)) {
                    const uint32_t fb = *glb(j.dfirst + idx);
                    if (!last && fb == len) { open += len; continue; }
                    if (open + fb) emit_stitch(L.bd, kCapD, j.hd, open + fb, 1u, (uint32_t)j.hmax, j.flag);
                }
                open = last ? 0u : (uint32_t)*glb(j.dlast + idx);
            }
        }
        if (r1 / H > sb) *glb(j.dstate + dk) = open;
    }
}

// Stitch of the recurrence matrix of one series over the strips [s_lo, s_hi)
// of one row band (all strips when the job has one band).  Lines of the band:
// the columns [s_lo H, n), then the diagonals k = 0 .. n-1-s_lo H; the other
// lines have no piece in these strips.  A line whose pieces go on in a later
// band keeps its open run in cstate / dstate; column col joins the band and
// row col of U in the band that holds that row (its lead, or its pieces).
__device__ __forceinline__ void stitch_auto(StitchLds &L, const JobDesc &j, int64_t line) {
    const int n = j.n, wp = j.wp, H = j.H;
    const int s_lo = j.s_lo, s_hi = j.s_hi;
    const bool last_band = s_hi >= j.nstrips;
    const bool carried = j.nbands > 1 && s_lo > 0;   // open runs come from earlier bands
    const int64_t lines = (int64_t)n - (int64_t)s_lo * H;
    if (line < lines) {
        // ---- column col of the full matrix ----
        const int col = (int)((int64_t)s_lo * H + line);
        const int s_last = col >= wp ? (col - wp) / H : -1;   // strips holding column col of U
        const bool has_row = col + wp <= n - 1;               // row col of U has cells
        const int js = has_row ? col / H : (s_last > 0 ? s_last : 0);
        const bool join = js >= s_lo && (js < s_hi || last_band);
        const int sb = s_last < s_hi - 1 ? s_last : s_hi - 1;   // last strip folded here
        uint32_t oc = 0, ol = 0;   // open run after folding column `col` of U
        if (carried && s_last >= 0 && (join || sb >= s_lo)) {
            const uint32_t c = *glb(j.cstate + col);
            oc = c >> 31;
            ol = c & 0x7FFFFFFFu;
        }
        // The summaries of kStitchBatch strips are loaded before any is
        // folded, so a thread has that many loads in flight.
        for (int s0 = s_lo; s0 <= sb; s0 += kStitchBatch) {
            uint32_t fv[kStitchBatch], lv[kStitchBatch];
#pragma unroll
            for (int u = 0; u < kStitchBatch; ++u) {
                const int s = s0 + u;
                if (s <= sb) {
                    const int64_t idx = strip_offset(s, n, wp, H) - j.soff_lo + (col - s * H - wp);
                    fv[u] = *glb(j.vfirst + idx);
                    lv[u] = *glb(j.vlast + idx);
                }
            }
#pragma unroll
            for (int u = 0; u < kStitchBatch; ++u) {
                const int s = s0 + u;
                if (s > sb) break;
                const uint32_t Ls = s < s_last ? (uint32_t)H : (uint32_t)(col - wp - s * H + 1);
                const uint32_t f = fv[u], l = lv[u];
                const uint32_t fc = f >> 15, fl = f & 0x7FFFu;
                if (fl == Ls) {   // the segment is one run
                    if (ol && oc == fc) ol += Ls;
                    else { emit_line(L, j, oc, ol); oc = fc; ol = Ls; }
                } else {
                    if (ol && oc == fc) emit_line(L, j, fc, ol + fl);
                    else { emit_line(L, j, oc, ol); emit_line(L, j, fc, fl); }
                    oc = l >> 15;
                    ol = l & 0x7FFFu;
                }
            }
        }
        if (!join) {
            if (sb >= s_lo) *glb(j.cstate + col) = ol | (oc << 31);
            return;
        }
        // join: [trailing run of the column of U] [middle] [leading run of row col of U]
        uint32_t mc, ml;
        if (j.theiler == 0) { mc = 1; ml = 1; }
        else {
            const int w = j.theiler;
            const int up = col < w - 1 ? col : w - 1;
            const int dn = (n - 1 - col) < w - 1 ? (n - 1 - col) : w - 1;
            mc = 0;
            ml = (uint32_t)(up + 1 + dn);
        }
        if (ol && oc == mc) ol += ml;
        else { emit_line(L, j, oc, ol); oc = mc; ol = ml; }
        if (has_row) {
            uint32_t hc, hl;
            if (j.segs > 1) {
                row_pieces(L, j, col, hc, hl);
            } else {
                const uint32_t ld = *glb(j.lead + col);
                hc = ld >> 31;
                hl = ld & 0x7FFFFFFFu;
            }
            if (oc == hc) ol += hl;
            else { emit_line(L, j, oc, ol); oc = hc; ol = hl; }
        }
        emit_line(L, j, oc, ol);
    } else if (line < 2 * lines) {
        // ---- diagonal k of U (and its mirror) ----
        const int k = (int)(line - lines);
        if (k >= wp && j.segs > 1) {
            // its pieces in the (strip, segment) blocks it crosses, in order
            const int r1 = n - 1 - k;
            const int s_end = r1 / H;                           // >= s_lo
            const int sb = s_end < s_hi - 1 ? s_end : s_hi - 1;
            uint32_t open = carried ? (uint32_t)*glb(j.dstate + k) : 0u;
            for (int s = s_lo; s <= sb; ++s) {
                const int ra = s * H;
                const int rb = r1 < s * H + H - 1 ? r1 : s * H + H - 1;
                const int ca = ra + k, cb = rb + k;
                const int xs = ((s * H + wp) >> 6) * 64;   // the strip's first column tile
                for (int g = seg_of(j, ca); g <= seg_of(j, cb); ++g) {
                    const int g0 = (j.seg_base + g * j.seg_tiles) * 64;
                    const int lo = ca > g0 ? ca : g0;
                    const int hi = cb < g0 + j.seg_tiles * 64 - 1 ? cb : g0 + j.seg_tiles * 64 - 1;
                    const uint32_t len = (uint32_t)(hi - lo + 1);
                    const bool last = rb == r1 && hi == cb;
                    const int bx0 = g0 > xs ? g0 : xs;      // the block's first column
                    const int64_t idx = (int64_t)((s - s_lo) * j.segs + g) * j.dw +
                                        (s * H + H - 1 - bx0) + k;
                    const uint32_t fb = *glb(j.dfirst + idx);
                    if (!last && fb == len) { open += len; continue; }
                    if (open + fb) emit_stitch(L.bd, kCapD, j.hd, open + fb, 2u, (uint32_t)n, j.flag);
                    open = last ? 0u : (uint32_t)*glb(j.dlast + idx);
                }
            }
            if (s_end > sb) *glb(j.dstate + k) = open;
        } else if (k >= wp) {
            const int s_last = (n - 1 - k) / H;                 // >= s_lo
            const int sb = s_last < s_hi - 1 ? s_last : s_hi - 1;
            uint32_t open = carried ? (uint32_t)*glb(j.dstate + k) : 0u;
            for (int s0 = s_lo; s0 <= sb; s0 += kStitchBatch) {
                uint32_t fv[kStitchBatch], lv[kStitchBatch];
#pragma unroll
                for (int u = 0; u < kStitchBatch; ++u) {
                    const int s = s0 + u;
                    if (s <= sb) {
                        const int64_t idx = strip_offset(s, n, wp, H) - j.soff_lo + (k - wp);
                        fv[u] = *glb(j.dfirst + idx);
                        lv[u] = *glb(j.dlast + idx);
                    }
                }
#pragma unroll
                for (int u = 0; u < kStitchBatch; ++u) {
                    const int s = s0 + u;
                    if (s > sb) break;
                    const uint32_t fb = fv[u];
                    if (s < s_last && fb == (uint32_t)H) { open += H; continue; }
                    if (open + fb) emit_stitch(L.bd, kCapD, j.hd, open + fb, 2u, (uint32_t)n, j.flag);
                    open = s < s_last ? lv[u] : 0u;
                }
            }
            if (s_last > sb) *glb(j.dstate + k) = open;
        } else if (k == 0 && j.theiler == 0 && s_lo == 0) {
            // main diagonal: every cell (i,i) is recurrent (distance 0 <= eps)
            emit(L.bd, kCapD, j.hd, (uint32_t)n, 1u, (uint32_t)n, j.flag);
        }
    }
}

__global__ void __launch_bounds__(kStitchThreads) k_stitch(const JobDesc *__restrict__ jobs,
                                                           int njobs) {
    __shared__ StitchLds L;
    static_assert(kStitchCapV <= kCapW, "bins are cleared and flushed in one pass over kCapW");
    for (int t = threadIdx.x; t < kCapW; t += blockDim.x) {
        if (t < kCapD) L.bd[t] = 0;
        if (t < kStitchCapV) L.bv[t] = 0;
        L.bw[t] = 0;
    }
    __syncthreads();
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].stitch_block0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const JobDesc &j = jobs[lo];
    const int n = j.n;
    const int64_t line = (int64_t)(blockIdx.x - j.stitch_block0) * blockDim.x + threadIdx.x;
    if (j.mode != kModeAuto) stitch_full(L, j, line);
    else stitch_auto(L, j, line);
    __syncthreads();
    const int hl = n + 1;
    for (int t = threadIdx.x; t < kCapW; t += blockDim.x) {
        if (t < kCapD && L.bd[t] && t < hl) g_add(j.hd + t, (unsigned long long)L.bd[t]);
        if (t < kStitchCapV && L.bv[t] && t < hl) g_add(j.hv + t, (unsigned long long)L.bv[t]);
        if (L.bw[t] && t < hl) g_add(j.hw + t, (unsigned long long)L.bw[t]);
    }
}

// ---------------------------------------------------------------------------
// Kernels 4-6: statistics of the finished histograms (the inputs of the RQA
// measures), so that a result fetch needs only a few hundred bytes.  Integer
// moments are exact (u64); the entropy partial sums use a fixed reduction
// order, so a job's statistics depend only on its own histograms.
// grid = (kStatMaxBlocks, jobs); block b of a job covers one contiguous chunk of
// lengths.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chunk_of(const JobDesc &j, int b, int64_t &lo, int64_t &hi) {
    const int64_t len = (int64_t)j.hmax + 1;
    const int64_t per = (len + j.stat_blocks - 1) / j.stat_blocks;
    lo = (int64_t)b * per;
    hi = lo + per < len ? lo + per : len;
}

__global__ void __launch_bounds__(kStatThreads) k_stats_moments(const JobDesc *__restrict__ jobs) {
    const JobDesc &j = jobs[blockIdx.y];
    if ((int)blockIdx.x >= j.stat_blocks) return;
    __shared__ unsigned long long red[5][kStatThreads];
    int64_t lo, hi;
    chunk_of(j, blockIdx.x, lo, hi);
    const unsigned long long *hs[3] = {j.hd, j.hv, j.hw};
    for (int h = 0; h < 3; ++h) {
        unsigned long long ca = 0, ma = 0, cm = 0, mm = 0, lg = 0;
        for (int64_t l = lo + threadIdx.x; l < hi; l += kStatThreads) {
            const unsigned long long c = hs[h][l];
            if (l == 0 || c == 0) continue;
            ca += c;
            ma += c * (unsigned long long)l;
            if (l >= j.mins[h]) {
                cm += c;
                mm += c * (unsigned long long)l;
            }
            lg = (unsigned long long)l;
        }
        red[0][threadIdx.x] = ca;
        red[1][threadIdx.x] = ma;
        red[2][threadIdx.x] = cm;
        red[3][threadIdx.x] = mm;
        red[4][threadIdx.x] = lg;
        __syncthreads();
        for (int s = kStatThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
                red[4][threadIdx.x] = red[4][threadIdx.x] > red[4][threadIdx.x + s]
                                          ? red[4][threadIdx.x] : red[4][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            JobStats *st = j.stats;
            if (red[0][0]) atomicAdd(&st->cnt_all[h], red[0][0]);
            if (red[1][0]) atomicAdd(&st->mass_all[h], red[1][0]);
            if (red[2][0]) atomicAdd(&st->cnt_min[h], red[2][0]);
            if (red[3][0]) atomicAdd(&st->mass_min[h], red[3][0]);
            if (red[4][0]) atomicMax(&st->longest[h], red[4][0]);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kStatThreads) k_stats_entropy(const JobDesc *__restrict__ jobs) {
    const JobDesc &j = jobs[blockIdx.y];
    if ((int)blockIdx.x >= j.stat_blocks) return;
    __shared__ double red[kStatThreads];
    int64_t lo, hi;
    chunk_of(j, blockIdx.x, lo, hi);
    const unsigned long long *hs[3] = {j.hd, j.hv, j.hw};
    for (int h = 0; h < 3; ++h) {
        const unsigned long long total = j.stats->cnt_min[h];
        double acc = 0.0;
        if (total) {
            const double C = (double)total;
            const int64_t from = lo > j.mins[h] ? lo : (int64_t)j.mins[h];
            for (int64_t l = from + threadIdx.x; l < hi; l += kStatThreads) {
                const unsigned long long c = hs[h][l];
                if (l == 0 || c == 0) continue;
                const double p = (double)c / C;
                acc -= p * log(p);
            }
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kStatThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) j.ent_part[h * kStatMaxBlocks + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void k_stats_final(const JobDesc *__restrict__ jobs, int njobs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * njobs) return;
    const JobDesc &j = jobs[t / 3];
    const int h = t % 3;
    double e = 0.0;
    for (int b = 0; b < j.stat_blocks; ++b) e = e + j.ent_part[h * kStatMaxBlocks + b];
    j.stats->ent[h] = e;
}

// ---------------------------------------------------------------------------
// Recurrence plot output: the masked matrix bit-packed row-major (bit b of word c
// of row i = cell (i, 64c+b)).  A wave owns one 64-row tile row and a chunk of
// column tiles.  For the matrix of one series only tiles on or above the
// diagonal are evaluated; each one above it is also written transposed into the
// mirror tile (the matrix is exactly symmetric).
// ---------------------------------------------------------------------------
struct PlotDesc {
    const float *a;            // rows' series
    const float *b;            // columns' series (one series: a)
    const float *tail;         // coordinates of the last column tile, zero padded
    uint64_t *bits;
    int64_t words;             // 64-bit words per output row
    int64_t nb_points;         // points of b
    int32_t n, nb, m, tau, theiler;
    float thr, thr0;
    int32_t row_tiles, col_tiles, chunks, cross;
    int32_t xchunks;           // column chunks per XCD: ceil(chunks / 8)
    float *box;                // per column tile kBoxStride floats: (lo_k, hi_k), k < kBoxK
    int32_t tail_len;
};

constexpr int kPlotChunk = 16;   // column tiles per wave

// Column boxes of the plot's column tiles (the records k_box_bounds writes for
// a job, for the plot's columns; always used: the test costs one scalar load
// and a few compares per tile).
__global__ void k_plot_boxes(const PlotDesc d) {
    const int K = d.m < kBoxK ? d.m : kBoxK;
    const int64_t total = (int64_t)d.col_tiles * K;
    const float bnd = d.thr0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % K);
        const int64_t c = t / K;
        const int64_t j0 = c * 64;
        const int64_t j1 = j0 + 64 < d.nb ? j0 + 64 : d.nb;
        float cmin = INFINITY, cmax = -INFINITY;
        const float *col = d.b + (int64_t)k * d.tau;
        for (int64_t q = j0; q < j1; ++q) {
            const float v = col[q];
            cmin = fminf(cmin, v);
            cmax = fmaxf(cmax, v);
        }
        float *rec = d.box + c * kBoxStride;
        rec[2 * k] = box_lo(cmin, bnd);
        rec[2 * k + 1] = box_hi(cmax, bnd);
    }
}

__global__ void k_plot_tail(const PlotDesc d) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t base = (int64_t)(d.col_tiles - 1) * 64;
    if (t < d.tail_len)
        const_cast<float *>(d.tail)[t] = base + t < d.nb_points ? d.b[base + t] : 0.0f;
}

template <int NORM, int M>
__global__ void __launch_bounds__(256) k_plot(const PlotDesc d) {
    const int lane = threadIdx.x & 63;
    // Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8), each XCD
    // with its own L2.  XCD x takes the column chunks q = x, x + 8, ... (a
    // balanced share of the triangle), and its consecutive waves take
    // consecutive row tiles of one chunk: the mirror tiles they write are then
    // neighbouring words of the same rows, which meet in that XCD's L2.
    const int x = (int)blockIdx.x & 7;
    const int L = __builtin_amdgcn_readfirstlane((int)(blockIdx.x >> 3) * 4 + (int)(threadIdx.x >> 6));
    const int qq = L / d.row_tiles, r = L - qq * d.row_tiles;
    const int q = qq * 8 + x;
    if (qq >= d.xchunks || q >= d.chunks) return;
    const int n = d.n, nb = d.nb, R = r * 64, i = R + lane;
    const int irow = i < n ? i : n - 1;
    const float *rowp = d.a + irow;
    float xr[M > 0 ? M : 1];
#pragma unroll
    for (int k = 0; k < (M > 0 ? M : 1); ++k) xr[k] = M > 0 ? glb(rowp)[(int64_t)k * d.tau] : 0.0f;
    const int cq = q * kPlotChunk;
    int cbeg = cq;
    const int cend = cbeg + kPlotChunk < d.col_tiles ? cbeg + kPlotChunk : d.col_tiles;
    if (!d.cross && cbeg < r) cbeg = r;
    const int64_t band = d.theiler;
    // A whole chunk: this lane's row words are written together at its end.
    const bool whole = cbeg == cq && cend - cq == kPlotChunk;
    uint64_t rowbuf[kPlotChunk];
#pragma unroll
    for (int u = 0; u < kPlotChunk; ++u) {
        const int c = cq + u;
        if (c < cbeg || c >= cend) continue;
        const int jbase = c * 64;
        const ConstF cols = to_const(c == d.col_tiles - 1 ? d.tail : d.b + jbase);
        uint32_t xlo, xhi;
        // The predicate path of the tile kernel: a tile that its column box
        // rules out for every row is empty without evaluating a pair.
        tile_bits<NORM, M>(cols, d.tau, xr, rowp, d.m, d.thr, d.thr0,
                                  M > 0 ? to_const(d.box) + (int64_t)c * kBoxStride : nullptr, xlo,
                                  xhi);
        uint64_t vm = 0ull;
        if (i < n) {
            const int hv = nb - jbase < 64 ? nb - jbase : 64;
            vm = range_mask(0, (uint32_t)hv);
            if (band > 0) {
                int64_t blo = (int64_t)i - band + 1 - jbase, bhi = (int64_t)i + band - jbase;
                blo = blo < 0 ? 0 : blo;
                bhi = bhi > 64 ? 64 : bhi;
                if (blo < bhi) vm &= ~range_mask((uint32_t)blo, (uint32_t)bhi);
            }
        }
        const uint64_t X = mk64(xlo, xhi) & vm;
        if (whole) rowbuf[u] = X;
        else if (i < n) d.bits[(int64_t)i * d.words + c] = X;
        if (!d.cross && c > r) {
            uint32_t lo = (uint32_t)X, hi = (uint32_t)(X >> 32);
            transpose64(lo, hi, lane);
            const int jr = jbase + lane;   // row of the mirror tile
            if (jr < n) d.bits[(int64_t)jr * d.words + r] = mk64(lo, hi);
        }
    }
    if (whole && i < n) {
        uint64_t *dst = d.bits + (int64_t)i * d.words + cq;
#pragma unroll
        for (int u = 0; u < kPlotChunk; ++u) dst[u] = rowbuf[u];
    }
}

using PlotKernel = void (*)(const PlotDesc);

template <int NORM>
PlotKernel pick_plot(int m) {
    switch (m) {
        case 1: return k_plot<NORM, 1>;
        case 2: return k_plot<NORM, 2>;
        case 3: return k_plot<NORM, 3>;
        case 4: return k_plot<NORM, 4>;
        case 5: return k_plot<NORM, 5>;
        case 6: return k_plot<NORM, 6>;
        default: return k_plot<NORM, 0>;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
using TileKernel = void (*)(const JobDesc *, const GroupDesc *, int, int *);

template <int NORM, int MODE>
TileKernel pick_kernel(int m) {
    switch (m) {
        case 1: return k_tiles<NORM, 1, MODE>;
        case 2: return k_tiles<NORM, 2, MODE>;
        case 3: return k_tiles<NORM, 3, MODE>;
        case 4: return k_tiles<NORM, 4, MODE>;
        case 5: return k_tiles<NORM, 5, MODE>;
        case 6: return k_tiles<NORM, 6, MODE>;
        default: return k_tiles<NORM, 0, MODE>;
    }
}

template <int MODE>
TileKernel tile_kernel_mode(int norm, int m) {
    if (norm == RQA_NORM_L1) return pick_kernel<RQA_NORM_L1, MODE>(m);
    if (norm == RQA_NORM_L2) return pick_kernel<RQA_NORM_L2, MODE>(m);
    return pick_kernel<RQA_NORM_LINF, MODE>(m);
}

TileKernel tile_kernel(int mode, int norm, int m) {
    if (mode == kModeMatrix) return k_tiles<RQA_NORM_LINF, 1, kModeMatrix>;   // no predicate
    if (mode == kModeCross) return tile_kernel_mode<kModeCross>(norm, m);
    return tile_kernel_mode<kModeAuto>(norm, m);
}

int group_key(const Job &jb) {
    const int nm = jb.mode == kModeMatrix ? 0 : jb.kp.norm * 16 + (jb.kp.m <= kMaxM ? jb.kp.m : 0);
    return ((jb.mode * 64) + nm) * 32 + jb.waves;
}

struct Layout {
    int H, nstrips;
    int band, nbands;      // strips per row band (auto mode) and the number of bands
    int segs, seg_tiles;   // column segments per strip and their width (tiles)
    int seg_base;          // first column tile of segment 0
    int64_t hentries;      // row pieces (auto, segs > 1): rows of one band * segs
    int items;             // work items of the largest band: band * segs
    int dw;                // full matrix: diagonal summary slots per block
    int64_t ventries;      // vertical summary entries per array (first, last), one band
    int64_t dentries;      // diagonal summary entries per array, one band
    int64_t tail_len;
    int64_t box_floats;    // column boxes (header + records), 0 if none
    size_t off_tail, off_lead, off_vf, off_vl, off_df, off_dl, off_ent, off_hf, off_hl, off_box,
        off_cs, off_ds, bytes;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Work items (strips x column segments) a single series run alone is cut
// into: a few times the workgroups one launch keeps resident (256 CUs x 3).
constexpr int kTargetItems = 2048;
// Work items of a series cut into column segments (per row band when banded)
// and of a full-matrix job: shorter chains of tiles, so that the launch's
// last, partly idle round of items is short (cross recurrence of 2 x 262,144
// points 10.3 -> 9.3 ms, given 65,516^2 matrix 0.72 -> 0.50 ms against 2,048
// items; 16,384 items made the given matrix slower again).
constexpr int kSegItems = 8192;    // (one series alone, one band or several)
constexpr int kFullItems = 8192;

// Offset of the first evaluated diagonal of U, max(theiler, 1), clamped to n:
// every window of n or more masks the whole matrix alike, and the clamp keeps
// the kernels' 32-bit row + offset arithmetic from overflowing.
int effective_wp(int32_t theiler, int64_t n) {
    const int64_t w = theiler > 1 ? theiler : 1;
    return (int)(w < n ? w : (n > 1 ? n : 1));
}

int default_waves_impl(int64_t n) {
    // Eight waves per workgroup (two workgroups per compute unit) measured
    // fastest for long series; short series use four so that more strips exist.
    if (n >= 4096 * 8) return 8;
    return 4;
}

// Column segments of an auto-mode job when it runs alone (`nstrips`: the
// strips of one launch, i.e. of one row band): enough for about kSegItems
// work items, each at least 64 tiles wide; 1 for jobs whose first strip is
// shorter than 128 tiles (their chains are short) or that have more than
// kTargetItems / 2 strips already (the 1,048,576-point workload has 2,048,
// the paper's 1,000,001-point sine 1,954: cutting it in two measured 5%
// slower, the extra summaries costing more than the shorter chains gain).
// kSegItems rather than kTargetItems items: shorter chains measured faster
// on dense jobs (a 199,873-vector served job at RR 5%: 13.9 ms with 2,048
// items, 12.1 with 4,096, 11.5 with 8,192; a 300,000-point Lorenz series
// 9.2 / 8.3 / 7.8 ms).
int auto_segs_max(int64_t n, int wp, int H, int nstrips) {
    const int T0 = (int)((n - 1) / 64 - wp / 64 + 1);
    if (nstrips < 1 || T0 < 128 || 2 * nstrips > kTargetItems) return 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>((kSegItems + nstrips - 1) / nstrips, T0 / 64));
}

Layout layout_of(const Job &jb) {
    Layout L{};
    const int64_t n = jb.n_vec;
    const int wp = effective_wp(jb.kp.theiler, n);
    L.H = 64 * (jb.waves > 0 ? jb.waves : default_waves_impl(n));
    if (jb.mode == kModeAuto) {
        L.nstrips = n - wp > 0 ? (int)((n - wp + L.H - 1) / L.H) : 0;
        // Row bands: the summaries hold the strips of one band (the first,
        // whose strips are the longest); the open runs of every line pass
        // from band to band in per-line carries.
        L.band = jb.band_strips > 0 && jb.band_strips < L.nstrips ? jb.band_strips : L.nstrips;
        L.nbands = L.band > 0 ? (L.nstrips + L.band - 1) / L.band : 1;
        // sum over the band's strips of (n - wp - s H) entries
        L.ventries = strip_offset(L.band, (int32_t)n, wp, L.H);
        // Segments: as set on the job, else the most it could be given.
        const int T0 = (int)((n - 1) / 64 - wp / 64 + 1);
        int segs = jb.segs > 0 ? jb.segs : auto_segs_max(n, wp, L.H, L.band);
        L.seg_base = wp / 64;
        L.seg_tiles = (T0 + segs - 1) / segs;
        L.segs = segs > 1 ? (T0 + L.seg_tiles - 1) / L.seg_tiles : 1;
        if (L.segs > 1) {
            L.dw = L.seg_tiles * 64 + L.H - 1;
            L.dentries = (int64_t)L.band * L.segs * L.dw;
            L.hentries = std::min<int64_t>(n, (int64_t)L.band * L.H) * L.segs;
        } else {
            L.dw = 0;
            L.dentries = L.ventries;
            L.hentries = 0;
        }
    } else {
        // A strip of a full matrix walks every column tile; its chain of
        // tiles is cut into column segments walked by different workgroups,
        // enough of them for about kFullItems work items, each at least
        // max(8, H/64) tiles wide (so a diagonal crosses at most one segment
        // edge inside a strip).
        const int64_t nb = jb.n_cols;
        L.nstrips = (int)((n + L.H - 1) / L.H);
        // Row bands as in auto mode: summaries for one band's strips.
        L.band = jb.band_strips > 0 && jb.band_strips < L.nstrips ? jb.band_strips : L.nstrips;
        L.nbands = (L.nstrips + L.band - 1) / L.band;
        const int T = (int)((nb - 1) / 64 + 1);
        const int min_tiles = std::max(8, L.H / 64);
        int segs = (int)std::min<int64_t>((kFullItems + L.band - 1) / L.band,
                                          std::max(1, T / min_tiles));
        segs = std::max(segs, 1);
        L.seg_base = 0;
        L.seg_tiles = (T + segs - 1) / segs;
        L.segs = (T + L.seg_tiles - 1) / L.seg_tiles;
        L.dw = L.seg_tiles * 64 + L.H - 1;
        L.ventries = (int64_t)L.band * nb;
        L.dentries = (int64_t)L.band * L.segs * L.dw;
        L.hentries = 0;
    }
    L.items = L.band * L.segs;
    if (L.ventries < 1) L.ventries = 1;
    if (L.dentries < 1) L.dentries = 1;
    L.tail_len = jb.mode == kModeMatrix ? 0 : 64 + (int64_t)(jb.kp.m - 1) * jb.kp.tau;
    const int64_t lead = jb.mode == kModeAuto ? n : 1;
    size_t off = 0;
    L.off_tail = off; off += a256(sizeof(float) * (size_t)L.tail_len);
    L.off_lead = off; off += a256(sizeof(uint32_t) * (size_t)lead);
    L.off_vf = off; off += a256(sizeof(uint16_t) * (size_t)L.ventries);
    L.off_vl = off; off += a256(sizeof(uint16_t) * (size_t)L.ventries);
    L.off_df = off; off += a256(sizeof(uint16_t) * (size_t)L.dentries);
    L.off_dl = off; off += a256(sizeof(uint16_t) * (size_t)L.dentries);
    L.off_ent = off; off += a256(sizeof(double) * 3 * kStatMaxBlocks);
    L.off_hf = off; off += a256(sizeof(uint32_t) * (size_t)L.hentries);
    L.off_hl = off; off += a256(sizeof(uint32_t) * (size_t)L.hentries);
    // Boxes for the modes with a predicate and the embedding dimensions whose
    // row coordinates live in registers.
    const int64_t ncols = jb.mode == kModeAuto ? n : jb.n_cols;
    L.box_floats = (jb.mode != kModeMatrix && jb.kp.m <= kMaxM)
                       ? kBoxHeader + ((ncols - 1) / 64 + 1) * (int64_t)kBoxStride : 0;
    L.off_box = off; off += a256(sizeof(float) * (size_t)L.box_floats);
    // Per-line carries between bands: the open run of each column (of U in
    // auto mode) and of each diagonal (n - 1 + nb of them in a full matrix).
    const bool banded = L.nbands > 1;
    const size_t ccarries = banded ? (size_t)(jb.mode == kModeAuto ? n : jb.n_cols) : 0;
    const size_t dcarries = banded ? (size_t)(jb.mode == kModeAuto ? n : n + jb.n_cols - 1) : 0;
    L.off_cs = off; off += a256(sizeof(uint32_t) * ccarries);
    L.off_ds = off; off += a256(sizeof(uint32_t) * dcarries);
    L.bytes = off;
    return L;
}


// Device descriptor of one job whose work items start at `strip_base` of its
// group and whose stitch blocks start at `stitch_block0`.
JobDesc make_desc(const Job &jb, const Layout &lay, int strip_base, int stitch_block0) {
    const KParams &kp = jb.kp;
    char *scr = static_cast<char *>(jb.scratch);
    JobDesc d{};
    const bool full = jb.mode != kModeAuto;
    const int64_t hlen = jb.hist_len();
    const int64_t stride = jb.hist_stride > 0 ? jb.hist_stride : hlen;
    const int64_t ncols = full ? jb.n_cols : jb.n_vec;
    d.s = jb.series;
    d.sb = jb.mode == kModeCross ? jb.series_b : jb.series;
    d.n_points_b = jb.mode == kModeCross ? jb.n_points_b : jb.n_points;
    d.bits = jb.bits;
    d.words = jb.words;
    d.tail = reinterpret_cast<const float *>(scr + lay.off_tail);
    d.hd = reinterpret_cast<unsigned long long *>(jb.hist);
    d.hv = d.hd + stride;
    d.hw = d.hv + stride;
    d.flag = jb.flag;
    d.lead = reinterpret_cast<uint32_t *>(scr + lay.off_lead);
    d.vfirst = reinterpret_cast<uint16_t *>(scr + lay.off_vf);
    d.vlast = reinterpret_cast<uint16_t *>(scr + lay.off_vl);
    d.dfirst = reinterpret_cast<uint16_t *>(scr + lay.off_df);
    d.dlast = reinterpret_cast<uint16_t *>(scr + lay.off_dl);
    d.n_points = jb.n_points;
    d.n = (int32_t)jb.n_vec;
    d.nb = (int32_t)ncols;
    d.hmax = (int32_t)(hlen - 1);
    d.mode = jb.mode;
    d.m = kp.m;
    d.tau = kp.tau;
    d.norm = kp.norm;
    d.theiler = kp.theiler;
    d.wp = effective_wp(kp.theiler, jb.n_vec);
    d.thr = kp.norm == RQA_NORM_L2 ? kp.eps_sq : kp.eps;
    d.thr0 = kp.d0_bound;
    d.H = lay.H;
    d.nstrips = lay.nstrips;
    d.segs = lay.segs;
    d.seg_tiles = lay.seg_tiles;
    d.seg_base = lay.seg_base;
    d.dw = lay.dw;
    d.hfirst = lay.hentries > 0 ? reinterpret_cast<uint32_t *>(scr + lay.off_hf) : nullptr;
    d.hlast = lay.hentries > 0 ? reinterpret_cast<uint32_t *>(scr + lay.off_hl) : nullptr;
    d.s_lo = 0;
    d.s_hi = lay.band;
    d.band_strips = lay.band;
    d.nbands = lay.nbands;
    d.soff_lo = 0;
    d.cstate = lay.nbands > 1 ? reinterpret_cast<uint32_t *>(scr + lay.off_cs) : nullptr;
    d.dstate = lay.nbands > 1 ? reinterpret_cast<uint32_t *>(scr + lay.off_ds) : nullptr;
    d.c_last = (int32_t)((ncols - 1) / 64);
    d.tail_len = (int32_t)lay.tail_len;
    d.strip_base = strip_base;
    d.stitch_block0 = stitch_block0;
    d.mins[0] = kp.lmin;
    d.mins[1] = kp.vmin;
    d.mins[2] = kp.wmin;
    // 2,048 lengths (8 per thread) per statistics block: the blocks' loops
    // are chains of dependent loads, so short chains finish sooner.
    d.stat_blocks = (int32_t)std::min<int64_t>(kStatMaxBlocks, std::max<int64_t>(1, (hlen + 2047) / 2048));
    d.stats = jb.stats ? reinterpret_cast<JobStats *>(jb.stats)
                       : reinterpret_cast<JobStats *>(reinterpret_cast<char *>(jb.flag) + 8);
    d.ent_part = reinterpret_cast<double *>(scr + lay.off_ent);
    d.box = lay.box_floats > 0 ? reinterpret_cast<float *>(scr + lay.off_box) : nullptr;
    // Fault injection for tests of the give-up path: with
    // RQA_DEBUG_WAIT_GIVEUP=1 in the environment every neighbour wait of the
    // tile kernel aims at a count no wave reaches and gives up after 64
    // polls; the kernels still finish and the job reports RQA_EDEVICE.
    const char *giveup = std::getenv("RQA_DEBUG_WAIT_GIVEUP");
    const bool inject = giveup && giveup[0] == '1';
    d.spin_limit = inject ? 64 : (int32_t)kSpinLimit;
    d.wait_bias = inject ? (1 << 30) : 0;
    return d;
}

// Blocks of k_box_bounds for one job: one thread per box entry, at most 128
// blocks (the kernel strides over the rest).
int box_blocks_of(const Layout &lay) {
    const int64_t entries = lay.box_floats > 0 ? (lay.box_floats - kBoxHeader) / kBoxStride * kBoxK : 0;
    return (int)std::min<int64_t>(128, std::max<int64_t>(1, (entries + 255) / 256));
}

int stitch_blocks_of(const Job &jb) {
    const bool full = jb.mode != kModeAuto;
    const int64_t lines = full ? jb.n_cols + jb.n_vec + jb.n_cols - 1 : 2 * jb.n_vec;
    return (int)((lines + kStitchThreads - 1) / kStitchThreads);
}

}  // namespace

size_t engine_job_scratch_bytes(const Job &job) { return layout_of(job).bytes; }

int engine_band_strips(const Job &job, size_t limit) {
    if (limit == 0) return 0;
    Job jb = job;
    jb.band_strips = 0;
    const Layout all = layout_of(jb);
    if (all.bytes <= limit || all.nstrips <= 1) return 0;
    // The largest band whose scratch fits (the scratch grows with the band,
    // up to the jumps where the column segments per strip change).
    int lo = 1, hi = all.nstrips - 1;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        jb.band_strips = mid;
        if (layout_of(jb).bytes <= limit) lo = mid; else hi = mid - 1;
    }
    jb.band_strips = lo;
    while (lo > 1 && layout_of(jb).bytes > limit) jb.band_strips = --lo;
    return lo;
}

JobPlan engine_job_plan(const Job &job) {
    const Layout lay = layout_of(job);
    JobPlan p{};
    p.bands = lay.nbands;
    p.band_strips = lay.band;
    p.segs = lay.segs;
    p.strip_rows = lay.H;
    p.scratch_bytes = lay.bytes;
    return p;
}

int engine_default_waves(int64_t n) { return default_waves_impl(n); }

size_t engine_launch_scratch_bytes(size_t njobs) {
    return a256(sizeof(JobDesc) * njobs) + a256(sizeof(GroupDesc) * 64) + 256;
}

int AuxStreams::create(int n) {
    n = n < kMax ? n : kMax;
    for (int k = 0; k < n; ++k) {
        if (hipStreamCreateWithFlags(&s[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&join[k], hipEventDisableTiming) != hipSuccess) {
            count = k;
            destroy();
            return RQA_EDEVICE;
        }
        count = k + 1;
    }
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
        destroy();
        return RQA_EDEVICE;
    }
    return RQA_OK;
}

void AuxStreams::destroy() {
    for (int k = 0; k < count; ++k) {
        if (s[k]) hipStreamDestroy(s[k]);
        if (join[k]) hipEventDestroy(join[k]);
        s[k] = nullptr;
        join[k] = nullptr;
    }
    if (fork) hipEventDestroy(fork);
    fork = nullptr;
    count = 0;
}

int engine_launch(const std::vector<Job> &jobs_in, void *launch_scratch, void *staging,
                  hipEvent_t staging_free, int groups_req, hipStream_t st,
                  const PhaseEvents *phases, AuxStreams *aux) {
    const int njobs = (int)jobs_in.size();
    if (njobs == 0) return RQA_OK;
    for (const Job &jb : jobs_in)
        if (jb.waves < 1 || jb.waves > kMaxWaves) return RQA_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RQA_EDEVICE;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return RQA_EDEVICE;

    // Order: by (norm, m, waves) group, then by decreasing size (largest strips first).
    std::vector<int> order(njobs);
    for (int k = 0; k < njobs; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ga = group_key(jobs_in[a]), gb = group_key(jobs_in[b]);
        if (ga != gb) return ga < gb;
        return jobs_in[a].n_vec > jobs_in[b].n_vec;
    });

    // The previous launch that used `staging` must have consumed it.
    if (staging_free && hipEventSynchronize(staging_free) != hipSuccess) return RQA_EDEVICE;

    char *dbase = static_cast<char *>(launch_scratch);
    JobDesc *hdesc = static_cast<JobDesc *>(staging);
    GroupDesc *hgroups = reinterpret_cast<GroupDesc *>(static_cast<char *>(staging) +
                                                       a256(sizeof(JobDesc) * njobs));
    JobDesc *ddesc = reinterpret_cast<JobDesc *>(dbase);
    GroupDesc *dgroups = reinterpret_cast<GroupDesc *>(dbase + a256(sizeof(JobDesc) * njobs));
    int *dcounters = reinterpret_cast<int *>(dbase + a256(sizeof(JobDesc) * njobs) +
                                             a256(sizeof(GroupDesc) * 64));

    std::vector<int> gkeys;
    int stitch_blocks = 0;
    int stat_grid = 1;
    int box_grid = 1;
    int ngroups = 0;
    int strip_acc = 0;
    for (int r = 0; r < njobs; ++r) {
        // A job launched with others keeps whole strips: the launch has work
        // items enough, and its scratch is sized for any choice.
        Job jb = jobs_in[order[r]];
        if (jb.segs == 0 && njobs > 1) jb.segs = 1;
        const Layout lay = layout_of(jb);
        const int key = group_key(jb);
        if (ngroups == 0 || gkeys.back() != key) {
            if (ngroups == 64) return RQA_EINVAL;
            if (ngroups > 0) hgroups[ngroups - 1].items = strip_acc;
            gkeys.push_back(key);
            hgroups[ngroups] = GroupDesc{r, r + 1, 0, 0};
            ++ngroups;
            strip_acc = 0;
        }
        hgroups[ngroups - 1].job1 = r + 1;
        JobDesc d = make_desc(jb, lay, strip_acc, stitch_blocks);
        stat_grid = std::max(stat_grid, (int)d.stat_blocks);
        box_grid = std::max(box_grid, box_blocks_of(lay));
        strip_acc += lay.items;
        stitch_blocks += stitch_blocks_of(jb);
        hdesc[r] = d;
    }
    hgroups[ngroups - 1].items = strip_acc;

    const size_t desc_bytes = a256(sizeof(JobDesc) * njobs) + a256(sizeof(GroupDesc) * 64);
    if (hipMemcpyAsync(dbase, staging, desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return RQA_EDEVICE;
    if (staging_free && hipEventRecord(staging_free, st) != hipSuccess) return RQA_EDEVICE;

    if (phases) hipEventRecord(phases->ev[0], st);
    hipLaunchKernelGGL(k_reset, dim3((std::max(njobs, 64) + 255) / 256), dim3(256), 0, st, ddesc,
                       njobs, dcounters, 64);
    hipLaunchKernelGGL(k_prepare, dim3(64, njobs), dim3(256), 0, st, ddesc);
    hipLaunchKernelGGL(k_box_bounds, dim3(box_grid, njobs), dim3(256), 0, st, ddesc);
    hipLaunchKernelGGL(k_box_probe, dim3(njobs), dim3(kProbeThreads), 0, st, ddesc);

    if (phases) hipEventRecord(phases->ev[1], st);
    if (njobs == 1 && hdesc[0].nbands > 1) {
        // One job in row bands: per band the tile kernel over the band's
        // strips, then the stitch of the lines those strips cross.
        const JobDesc &d = hdesc[0];
        const Job &jb = jobs_in[0];
        TileKernel kern = tile_kernel(jb.mode, jb.kp.norm, jb.kp.m);
        int occ = 0;
        const size_t lds = strip_lds_bytes(jb.waves);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * jb.waves, lds) != hipSuccess ||
            occ < 1)
            occ = 1;
        const int full_grid = groups_req > 0 ? groups_req : ncu * occ;
        for (int b = 0; b < d.nbands; ++b) {
            const int lo = b * d.band_strips;
            const int hi = std::min(lo + d.band_strips, d.nstrips);
            const int items = (hi - lo) * d.segs;
            const int64_t lines = d.mode == kModeAuto ? 2 * ((int64_t)d.n - (int64_t)lo * d.H)
                                                      : (int64_t)d.nb + d.n + d.nb - 1;
            hipLaunchKernelGGL(k_band, dim3(1), dim3(64), 0, st, ddesc, dgroups, dcounters, b);
            if (items > 0)
                hipLaunchKernelGGL(kern, dim3(std::min(full_grid, items)), dim3(64 * jb.waves), lds, st,
                                   ddesc, dgroups, 0, dcounters);
            if (phases && b == d.nbands - 1) hipEventRecord(phases->ev[2], st);
            if (lines > 0)
                hipLaunchKernelGGL(k_stitch, dim3((unsigned)((lines + kStitchThreads - 1) / kStitchThreads)),
                                   dim3(kStitchThreads), 0, st, ddesc, 1);
        }
        hipLaunchKernelGGL(k_stats_moments, dim3(stat_grid, 1), dim3(kStatThreads), 0, st, ddesc);
        hipLaunchKernelGGL(k_stats_entropy, dim3(stat_grid, 1), dim3(kStatThreads), 0, st, ddesc);
        hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, st, ddesc, 1);
        if (phases) hipEventRecord(phases->ev[3], st);
        return hipGetLastError() == hipSuccess ? RQA_OK : RQA_EDEVICE;
    }
    int active = 0;
    for (int g = 0; g < ngroups; ++g) active += hgroups[g].items > 0;
    const bool fork = aux && aux->count > 0 && active > 1;
    if (fork) hipEventRecord(aux->fork, st);
    bool used[AuxStreams::kMax] = {};
    int launched = 0;
    for (int g = 0; g < ngroups; ++g) {
        const GroupDesc &gd = hgroups[g];
        if (gd.items == 0) continue;
        const KParams &kp = jobs_in[order[gd.job0]].kp;
        const int w = jobs_in[order[gd.job0]].waves;
        TileKernel kern = tile_kernel(jobs_in[order[gd.job0]].mode, kp.norm, kp.m);
        int occ = 0;
        const size_t lds = strip_lds_bytes(w);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * w, lds) != hipSuccess ||
            occ < 1)
            occ = 1;
        int grid = groups_req > 0 ? groups_req : ncu * occ;
        grid = std::min(grid, gd.items);
        // The first group runs on the launch stream; further groups fork.
        hipStream_t gs = st;
        if (fork && launched > 0) {
            const int k = (launched - 1) % aux->count;
            gs = aux->s[k];
            if (!used[k]) hipStreamWaitEvent(gs, aux->fork, 0);
            used[k] = true;
        }
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * w), lds, gs, ddesc, dgroups, g, dcounters);
        ++launched;
    }
    if (fork) {
        for (int k = 0; k < aux->count; ++k) {
            if (!used[k]) continue;
            hipEventRecord(aux->join[k], aux->s[k]);
            hipStreamWaitEvent(st, aux->join[k], 0);
        }
    }
    if (phases) hipEventRecord(phases->ev[2], st);
    if (stitch_blocks > 0)
        hipLaunchKernelGGL(k_stitch, dim3(stitch_blocks), dim3(kStitchThreads), 0, st, ddesc, njobs);
    hipLaunchKernelGGL(k_stats_moments, dim3(stat_grid, njobs), dim3(kStatThreads), 0, st, ddesc);
    hipLaunchKernelGGL(k_stats_entropy, dim3(stat_grid, njobs), dim3(kStatThreads), 0, st, ddesc);
    hipLaunchKernelGGL(k_stats_final, dim3((3 * njobs + 255) / 256), dim3(256), 0, st, ddesc, njobs);
    if (phases) hipEventRecord(phases->ev[3], st);
    return hipGetLastError() == hipSuccess ? RQA_OK : RQA_EDEVICE;
}

size_t engine_static_bytes(const Job &jb) {
    return engine_launch_scratch_bytes(1) + a256(kInfoBytes) + layout_of(jb).bytes;
}

int engine_launch_static(Job jb, void *scratch, hipStream_t st) {
    if (jb.waves < 1 || jb.waves > kMaxWaves || jb.mode != kModeAuto) return RQA_EINVAL;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return RQA_EDEVICE;
    // [descriptors | groups | counters][statistics record][job scratch]
    char *base = static_cast<char *>(scratch);
    JobDesc *ddesc = reinterpret_cast<JobDesc *>(base);
    GroupDesc *dgroups = reinterpret_cast<GroupDesc *>(base + a256(sizeof(JobDesc)));
    int *dcounters = reinterpret_cast<int *>(base + a256(sizeof(JobDesc)) +
                                             a256(sizeof(GroupDesc) * 64));
    jb.stats = base + engine_launch_scratch_bytes(1);
    jb.scratch = base + engine_launch_scratch_bytes(1) + a256(kInfoBytes);
    const Layout lay = layout_of(jb);
    const JobDesc d = make_desc(jb, lay, 0, 0);
    const GroupDesc g{0, 1, lay.items, 0};
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, d, g, ddesc, dgroups);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, st, ddesc, 1, dcounters, 64);
    hipLaunchKernelGGL(k_prepare, dim3(64, 1), dim3(256), 0, st, ddesc);
    hipLaunchKernelGGL(k_box_bounds, dim3(box_blocks_of(lay), 1), dim3(256), 0, st, ddesc);
    hipLaunchKernelGGL(k_box_probe, dim3(1), dim3(kProbeThreads), 0, st, ddesc);
    if (lay.items > 0) {
        TileKernel kern = tile_kernel(kModeAuto, jb.kp.norm, jb.kp.m);
        int occ = 0;
        const size_t lds = strip_lds_bytes(jb.waves);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * jb.waves, lds) != hipSuccess ||
            occ < 1)
            occ = 1;
        const int grid = std::min(ncu * occ, lay.items);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * jb.waves), lds, st, ddesc, dgroups, 0,
                           dcounters);
    }
    hipLaunchKernelGGL(k_stitch, dim3(stitch_blocks_of(jb)), dim3(kStitchThreads), 0, st, ddesc, 1);
    hipLaunchKernelGGL(k_stats_moments, dim3(d.stat_blocks, 1), dim3(kStatThreads), 0, st, ddesc);
    hipLaunchKernelGGL(k_stats_entropy, dim3(d.stat_blocks, 1), dim3(kStatThreads), 0, st, ddesc);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, st, ddesc, 1);
    return hipGetLastError() == hipSuccess ? RQA_OK : RQA_EDEVICE;
}

// The last column tile's coordinates, then (32-byte aligned) the column boxes.
static int64_t plot_tail_floats(const KParams &kp) {
    return (64 + (int64_t)(kp.m - 1) * kp.tau + 7) / 8 * 8;
}
int64_t engine_plot_scratch_floats(const KParams &kp, int64_t nb) {
    return plot_tail_floats(kp) + (nb + 63) / 64 * kBoxStride;
}

int engine_plot(const KParams &kp, const float *a, int64_t na_points, const float *b,
                int64_t nb_points, uint64_t *bits, int64_t words, float *scratch, hipStream_t st) {
    const int64_t d = (int64_t)(kp.m - 1) * kp.tau;
    const bool cross = b != nullptr;
    const int64_t n = na_points - d, nb = cross ? nb_points - d : n;
    PlotDesc pd{};
    pd.a = a;
    pd.b = cross ? b : a;
    pd.tail = scratch;
    pd.box = scratch + plot_tail_floats(kp);
    pd.bits = bits;
    pd.words = words;
    pd.nb_points = cross ? nb_points : na_points;
    pd.n = (int32_t)n;
    pd.nb = (int32_t)nb;
    pd.m = kp.m;
    pd.tau = kp.tau;
    pd.theiler = kp.theiler;
    pd.thr = kp.norm == RQA_NORM_L2 ? kp.eps_sq : kp.eps;
    pd.thr0 = kp.d0_bound;
    pd.row_tiles = (int32_t)((n + 63) / 64);
    pd.col_tiles = (int32_t)((nb + 63) / 64);
    pd.chunks = (pd.col_tiles + kPlotChunk - 1) / kPlotChunk;
    pd.xchunks = (pd.chunks + 7) / 8;
    pd.cross = cross ? 1 : 0;
    pd.tail_len = (int32_t)(64 + (int64_t)(kp.m - 1) * kp.tau);
    hipLaunchKernelGGL(k_plot_tail, dim3((pd.tail_len + 255) / 256), dim3(256), 0, st, pd);
    if (kp.m > 0) {
        const int64_t box_threads = (int64_t)pd.col_tiles * std::min(kp.m, kBoxK);
        const int box_grid = (int)std::min<int64_t>((box_threads + 255) / 256, 4096);
        hipLaunchKernelGGL(k_plot_boxes, dim3(box_grid), dim3(256), 0, st, pd);
    }
    PlotKernel kern = kp.norm == RQA_NORM_L1 ? pick_plot<RQA_NORM_L1>(kp.m)
                      : kp.norm == RQA_NORM_L2 ? pick_plot<RQA_NORM_L2>(kp.m)
                                               : pick_plot<RQA_NORM_LINF>(kp.m);
    const int64_t xwaves = (int64_t)pd.row_tiles * pd.xchunks;   // waves per XCD
    hipLaunchKernelGGL(kern, dim3((unsigned)(8 * ((xwaves + 3) / 4))), dim3(256), 0, st, pd);
    return hipGetLastError() == hipSuccess ? RQA_OK : RQA_EDEVICE;
}

}  // namespace rqa
