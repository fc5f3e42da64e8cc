// Host-side policy of the RQA server, free of HIP so that it can be tested on
// a CPU: the first-fit device-pool allocator, the admission of queued jobs
// into one launch, and the choice of a stream for that launch.
#pragma once

#include <cstddef>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace rqa {

// First-fit allocator over [0, size) with a coalescing free list.
class Pool {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    // Free ranges (offset -> bytes), for checks.
    const std::map<size_t, size_t> &free_ranges() const { return free_; }

private:
    std::map<size_t, size_t> free_;
};

// A queued job as the admission policy sees it.
struct AdmitJob {
    double cells;       // matrix cells (n_vec^2)
    size_t footprint;   // pool bytes while it runs
};

// Jobs above this many cells (~45k delay vectors) are launched alone: a batch
// completes as a whole, so small jobs batched with a large one would wait for
// it.
constexpr double kBigCells = 2.0e9;

// The next launch: FIFO from the head of `queue`, stopping at the first job
// that does not fit the pool, at a large job (which starts a launch of its
// own), or at `max_batch` jobs.  Allocates each admitted job in `pool` and
// returns its offset; `big` tells whether the launch is one large job.
struct Admission {
    std::vector<size_t> offsets;   // of the first offsets.size() queued jobs
    double cells = 0.0;
    bool big = false;
};

inline Admission plan_launch(const std::deque<AdmitJob> &queue, Pool &pool, size_t max_batch) {
    Admission a;
    for (const AdmitJob &j : queue) {
        if (a.offsets.size() >= max_batch) break;
        const bool big = j.cells > kBigCells;
        if (big && !a.offsets.empty()) break;
        size_t off = 0;
        if (!pool.alloc(j.footprint, &off)) break;
        a.offsets.push_back(off);
        a.cells += j.cells;
        if (big) {
            a.big = true;
            break;
        }
    }
    return a;
}

// Stream of a launch: with two or more streams, large launches use the first
// half and small ones the second, each taking the stream of its class with the
// least work (cells) in flight; with one stream everything shares it.
inline size_t pick_stream(const std::vector<double> &load, bool big) {
    const size_t ns = load.size();
    const size_t half = ns > 1 ? ns / 2 : 1;
    const size_t lo = (big || ns == 1) ? 0 : half, hi = big ? half : ns;
    size_t slot = lo;
    for (size_t c = lo + 1; c < hi; ++c)
        if (load[c] < load[slot]) slot = c;
    return slot;
}

}  // namespace rqa
