// CPU checks of librqa's host code, built with g++ and AddressSanitizer /
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py:
//   host_checks measures <in> <out>  FP64 measures (rqa_measures.cpp) of the
//                                    histograms in <in>, raw rqa_measures to <out>
//   host_checks policy <seed>        the server's pool allocator, admission and
//                                    stream choice (rqa_policy.h) against a
//                                    shadow model, over random operations
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <random>
#include <vector>

#include "rqa_internal.h"
#include "rqa_policy.h"

namespace {

int fail(const char *what) {
    std::fprintf(stderr, "host_checks: %s\n", what);
    return 1;
}

// <in>: int64 cases, then per case int64 n, rqa_params, 3*(n+1) uint64.
int run_measures(const char *in, const char *out) {
    FILE *f = std::fopen(in, "rb");
    FILE *g = std::fopen(out, "wb");
    if (!f || !g) return fail("cannot open files");
    int64_t cases = 0;
    if (std::fread(&cases, sizeof cases, 1, f) != 1) return fail("short input");
    for (int64_t c = 0; c < cases; ++c) {
        int64_t n = 0;
        rqa_params p{};
        if (std::fread(&n, sizeof n, 1, f) != 1 || std::fread(&p, sizeof p, 1, f) != 1 || n < 1)
            return fail("bad case header");
        // exact-size buffers, so that any read past n+1 entries is caught
        std::vector<uint64_t> d(n + 1), v(n + 1), w(n + 1);
        for (std::vector<uint64_t> *h : {&d, &v, &w})
            if (std::fread(h->data(), sizeof(uint64_t), n + 1, f) != (size_t)(n + 1))
                return fail("short histogram");
        rqa_measures m{};
        rqa::measures_from_hist(d.data(), v.data(), w.data(), n, p, &m);
        std::fwrite(&m, sizeof m, 1, g);
    }
    std::fclose(f);
    std::fclose(g);
    return 0;
}

// Shadow model of the pool: a byte map of [0, size), 1 = allocated.
int run_policy(unsigned seed) {
    std::mt19937_64 rng(seed);
    const size_t size = 1u << 16;
    rqa::Pool pool;
    pool.reset(size);
    std::vector<unsigned char> used(size, 0);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t bytes = 1 + rng() % 4096;
            size_t off = 0;
            // first fit: the lowest offset with `bytes` free bytes in a row
            size_t want = size;
            for (size_t o = 0, run = 0; o < size; ++o) {
                run = used[o] ? 0 : run + 1;
                if (run == bytes) { want = o + 1 - bytes; break; }
            }
            // the pool's free ranges are maximal (coalesced), so first fit over
            // them is first fit over the bytes
            const bool ok = pool.alloc(bytes, &off);
            if (ok != (want < size)) return fail("alloc disagrees with the shadow map");
            if (!ok) continue;
            if (off != want) return fail("alloc is not first fit");
            for (size_t o = off; o < off + bytes; ++o) used[o] = 1;
            live.push_back({off, bytes});
        } else {
            const size_t k = rng() % live.size();
            pool.release(live[k].off, live[k].bytes);
            for (size_t o = live[k].off; o < live[k].off + live[k].bytes; ++o) used[o] = 0;
            live[k] = live.back();
            live.pop_back();
        }
        // free ranges are exactly the maximal runs of free bytes
        size_t o = 0;
        for (const auto &fr : pool.free_ranges()) {
            for (; o < fr.first; ++o)
                if (!used[o]) return fail("free byte missing from the free list");
            if (fr.first > 0 && !used[fr.first - 1]) return fail("free ranges not coalesced");
            for (size_t q = fr.first; q < fr.first + fr.second; ++q)
                if (used[q]) return fail("allocated byte in the free list");
            o = fr.first + fr.second;
            if (o < size && !used[o]) return fail("free range not maximal");
        }
        for (; o < size; ++o)
            if (!used[o]) return fail("free tail missing from the free list");
    }
    // Admission: FIFO, stops at the first job that does not fit, a large job
    // alone, at most max_batch jobs.
    for (int trial = 0; trial < 2000; ++trial) {
        rqa::Pool p2;
        const size_t cap = 1 + rng() % 100000;
        p2.reset(cap);
        std::deque<rqa::AdmitJob> q;
        const int nq = (int)(rng() % 12);
        for (int k = 0; k < nq; ++k) {
            const bool big = rng() % 4 == 0;
            q.push_back({big ? rqa::kBigCells * 1.5 : (double)(rng() % 1000000),
                         (size_t)(1 + rng() % 20000)});
        }
        const size_t max_batch = 1 + rng() % 6;
        const rqa::Admission a = rqa::plan_launch(q, p2, max_batch);
        size_t expect = 0, sum = 0;
        bool big = false;
        for (const auto &j : q) {
            if (expect >= max_batch) break;
            const bool jb = j.cells > rqa::kBigCells;
            if (jb && expect > 0) break;
            if (sum + j.footprint > cap) break;   // fresh pool: allocations are contiguous
            sum += j.footprint;
            ++expect;
            if (jb) { big = true; break; }
        }
        if (a.offsets.size() != expect || a.big != big) return fail("admission differs from FIFO");
        size_t off = 0;
        for (size_t k = 0; k < a.offsets.size(); ++k) {
            if (a.offsets[k] != off) return fail("admitted jobs not packed first-fit");
            off += q[k].footprint;
        }
    }
    // Stream choice: classes by halves, least load within the class.
    for (int trial = 0; trial < 2000; ++trial) {
        const size_t ns = 1 + rng() % 16;
        std::vector<double> load(ns);
        for (double &x : load) x = (double)(rng() % 100);
        for (int big = 0; big < 2; ++big) {
            const size_t s = rqa::pick_stream(load, big != 0);
            const size_t half = ns > 1 ? ns / 2 : 1;
            const size_t lo = (big || ns == 1) ? 0 : half, hi = big ? half : ns;
            if (s < lo || s >= hi) return fail("stream outside its class");
            for (size_t c = lo; c < hi; ++c)
                if (load[c] < load[s]) return fail("stream not the least loaded of its class");
        }
    }
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc >= 4 && std::strcmp(argv[1], "measures") == 0) return run_measures(argv[2], argv[3]);
    if (argc >= 3 && std::strcmp(argv[1], "policy") == 0)
        return run_policy((unsigned)std::strtoul(argv[2], nullptr, 10));
    return fail("usage: host_checks measures <in> <out> | policy <seed>");
}
