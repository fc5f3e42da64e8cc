"""Benchmark of the RQA hot path on one MI355X.

Headline: full RQA (validation, fused predicate + line detection, stitch/join,
histogram read-back and FP64 measures) of the Lorenz-63 x-coordinate,
N = 1,048,576 points, m=3, tau=10, L-infinity, eps = 0.05 std, lmin=vmin=wmin=2,
Theiler window 1.  value = n_vec^2 recurrence-matrix cells per second (Gcells/s)
with the series already resident in device memory.

Also reported (outside the timed K steps):
  roofline      live hipEvent time of the fused tile kernel: algorithmic FP32
                operations (6 per unique pair for L-infinity, m=3) per second
                vs the FP32 vector peak derived from unit counts and clock
                (78.6 T ops/s; also vs the published 157.3 TFLOP/s); traffic =
                HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
                summary, null once the kernel changed; executed VALU work from
                the committed counter summary
  cpu_baseline  the CPU oracle on a bounded sample of the same series
  batched       400 uneven sliding windows of uniform noise in one launch, vs the
                same windows run one by one
  served        a Poisson stream (200 req/s, 60 s of arrivals) of mixed jobs
                through the continuous-batching server: p50/p99 latency and
                Gcells/s; and its capacity on a closed batch of the jobs vs the
                same jobs run one by one (no allocation or tuning timed)
  cross / plot / matrix
                cross recurrence of two Lorenz trajectories (262,144 points each),
                the packed recurrence plot of 65,536 points, and the RQA of that
                plot as a given matrix
  paper_e2      the paper's own runtime workload (1,000,001-point sine), timed as
                a full RQA and set beside the paper's totals (Tab. 4)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

METRIC = "recurrence cells/s (Gcells/s) full RQA @N=1M, 1 GPU; batched p50/p99 latency"

# FP32 vector peak in operations/s, derived from the unit counts and clock:
# 256 CUs x 128 FP32 lanes per clock per CU x 2.4 GHz = 78.6 T ops/s.  AMD's
# published 157.3 TFLOP/s counts each of those lane-operations as a fused
# multiply-add (2 flops); the predicate's operations (subtract, max, add,
# compare) are one operation per lane each, so 78.6 T is their ceiling.  The
# bench line also gives the fraction against the published figure.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
PUBLISHED_FP32_TFLOPS = 157.3
TILES_SRC = os.path.join(REPO, "paper_2402_16853_amd", "csrc", "rqa_tiles.hip")
CALIB_SRC = os.path.join(REPO, "paper_2402_16853_amd", "csrc", "calib.hip")
PMC_SUMMARY = os.path.join(REPO, "profiles", "k_tiles_lorenz_N1048576_pmc.md")
VALU_PROBE_SUMMARY = os.path.join(REPO, "profiles", "valu_issue_probe.md")


def summary_fields(path, src):
    """The "- key: value" lines of a committed profile summary, or {} when the
    source it was measured with (sha256 recorded in the summary) has changed."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return {}
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return fields if fields.get("source sha256") == sha else {}


def predicate_ceiling():
    """Sustained issue rate of the predicate's own instruction stream
    (libcalib.so, committed probe summary), or None if stale."""
    f = summary_fields(VALU_PROBE_SUMMARY, CALIB_SRC)
    try:
        return {"tops": float(f["predicate ceiling T ops/s"]),
                "valu_per_clk_per_cu": float(f["VALU wave-instructions per clock per CU"]),
                "source": "profiles/valu_issue_probe.md (bench.py --probe-valu)"}
    except (KeyError, ValueError):
        return None


def profile_fields():
    """Figures of the committed k_tiles counter summary, or {} when the kernel
    source has changed since the counters were taken."""
    return summary_fields(PMC_SUMMARY, TILES_SRC)


def measured_traffic():
    """HBM bytes per k_tiles launch from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when the kernel source has changed since it was taken."""
    try:
        return int(profile_fields()["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def measured_valu(kernel_ms):
    """VALU work the tile kernel executed (committed counter summary): wave-
    instructions per launch and the lane-operation rate of this run's kernel
    time against the 78.6 T peak.  The predicate is pruned exactly (whole
    tiles are skipped when a column box rules out every row), so the executed
    rate differs from the algorithmic one."""
    f = profile_fields()
    try:
        insts = float(f["VALU wave-instructions per launch"])
        util = float(f["VALU lane utilisation"])
    except (KeyError, ValueError):
        return None
    tops = insts * 64 * util / (kernel_ms * 1e-3) / 1e12
    return {"valu_insts_per_launch": insts, "lane_utilisation": util,
            "executed_lane_ops_tops": round(tops, 3),
            "executed_frac": round(tops / VALU_PEAK_TOPS, 4)}


def measured_lds(kernel_ms):
    """LDS throughput of k_tiles: the committed per-launch LDS bytes over this
    run's kernel time, against the probed LDS read peak (None if stale)."""
    f = profile_fields()
    try:
        nbytes = int(f["LDS bytes per launch"])
        peak = float(f["LDS peak TB/s"])
    except (KeyError, ValueError):
        return None
    tbps = nbytes / (kernel_ms * 1e-3) / 1e12
    return {"achieved": round(tbps, 3), "peak": peak, "unit": "TB/s", "frac": round(tbps / peak, 4),
            "bytes_per_launch": nbytes}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ops_per_pair(m: int, norm: int) -> int:
    """Algorithmic FP32 operations of one predicate evaluation: m subtractions,
    m-1 accumulations (add or max), m squarings for L2, one comparison."""
    return 3 * m if norm == 2 else 2 * m


def unique_pairs(n: int, theiler: int) -> int:
    """Pairs i < j with j - i >= max(theiler, 1)."""
    w = max(theiler, 1)
    k = n - w
    return k * (k + 1) // 2 if k > 0 else 0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def settle(comp, run, fetch, limit=8):
    """Setup before the warm-up: let the built-in autotuner time its candidate
    workgroup shapes (each candidate is one complete run) until its choice is
    stable, so that no tuning trial falls into the timed steps."""
    seen = []
    for _ in range(limit):
        run()
        fetch()
        seen.append(comp.last_launch()["waves"])
        if len(seen) >= 2 and seen[-1] == seen[-2]:
            break


def bench_headline(args, torch, RQA, workload):
    s, p = workload("lorenz", seed=args.seed)
    n = len(s) - (p.m - 1) * p.tau
    dev = torch.device("cuda:0")
    ds = torch.from_numpy(s).to(dev)
    comp = RQA.from_params(p)
    comp.set_profiling(True)
    if args.sweep:
        for w in (2, 4, 8):
            comp.set_tiling(w, 0)
            comp.run(ds)
            comp.result(histograms=False)
            t = []
            for _ in range(2):
                comp.run(ds)
                comp.result(histograms=False)
                t.append(comp.timings())
            log(f"[sweep] waves={w} tiles {np.mean([x['tiles_ms'] for x in t]):.2f} ms "
                f"stitch {np.mean([x['stitch_ms'] for x in t]):.2f} ms")
    comp.set_tiling(args.waves, 0)
    settle(comp, lambda: comp.run(ds), lambda: comp.result(histograms=False))
    log(f"[bench] lorenz N={len(s)} n_vec={n} eps={p.eps:.6g} waves={comp.last_launch()['waves']}; "
        f"warmup {args.warmup}")
    # Host buffers for the histograms, reused across steps as a caller that
    # loops would (fresh 8 MB arrays per step cost ~1.6 ms of page faults).
    out_bufs = tuple(np.zeros(n + 1, dtype=np.uint64) for _ in range(3))
    for _ in range(args.warmup):
        comp.run(ds)
        comp.result(histograms=True, out=out_bufs)
    tiles, stitch, prep = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        comp.run(ds)
        res = comp.result(histograms=True, out=out_bufs)
        tm = comp.timings()
        tiles.append(tm["tiles_ms"])
        stitch.append(tm["stitch_ms"])
        prep.append(tm["prepare_ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cells = float(n) * float(n)
    gcells = cells / (ms * 1e-3) / 1e9
    tile_ms = float(np.mean(tiles))
    ops = unique_pairs(n, p.theiler) * ops_per_pair(p.m, p.norm)
    achieved = ops / (tile_ms * 1e-3) / 1e12
    log(f"[bench] {ms:.2f} ms/step  tiles {tile_ms:.2f} ms  stitch {np.mean(stitch):.2f} ms  "
        f"prepare {np.mean(prep):.2f} ms  RR={res.measures['rr']:.6f} DET={res.measures['det']:.6f}")
    ceiling = predicate_ceiling()
    if ceiling:
        ceiling["frac"] = round(achieved / ceiling["tops"], 4)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": measured_traffic(),
            "frac_vs_published_fp32": round(achieved / PUBLISHED_FP32_TFLOPS, 4),
            "published_fp32_tflops": PUBLISHED_FP32_TFLOPS,
            "lds": measured_lds(tile_ms),
            "executed": measured_valu(tile_ms),
            "predicate_ceiling": ceiling,
            "kernel": "k_tiles<Linf,m=3>", "kernel_ms": round(tile_ms, 3),
            "ops_per_launch": ops,
            "stitch_ms": round(float(np.mean(stitch)), 3),
            "prepare_ms": round(float(np.mean(prep)), 3)}
    out = {"ms": ms, "gcells": gcells, "n": n, "p": p, "roof": roof, "series": s,
           "measures": res.measures}
    comp.close()
    del ds
    return out


def bench_cpu_baseline(args, hl):
    import oracle
    threads = os.cpu_count() or 1
    s = hl["series"][: args.cpu_points]
    p = hl["p"]
    n = len(s) - (p.m - 1) * p.tau
    log(f"[bench] cpu oracle sample: first {len(s)} points ({threads} threads)")
    t0 = time.perf_counter()
    oracle.histograms(s, p.m, p.tau, p.eps, p.norm, p.theiler, threads=threads)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, on a tenth of the sample
    s1 = hl["series"][: max(args.cpu_points // 10, 1000)]
    n1 = len(s1) - (p.m - 1) * p.tau
    t1 = time.perf_counter()
    oracle.histograms(s1, p.m, p.tau, p.eps, p.norm, p.theiler, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": round(float(n) * n / dt / 1e9, 4), "unit": "Gcells/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"first {len(s)} points of the same Lorenz series (n_vec={n}), "
                      f"full matrix, {threads} threads, {cpu_model()}",
            "single_thread": {"value": round(float(n1) * n1 / dt1 / 1e9, 4), "unit": "Gcells/s",
                              "seconds": round(dt1, 2),
                              "sample": f"first {len(s1)} points, 1 thread"}}


def bench_batched(args, torch, RQA, workload, windows_plan):
    s, p = workload("uniform", seed=args.seed)
    off, ln = windows_plan(len(s), 400, 1000, 20000, seed=args.seed)
    dev = torch.device("cuda:0")
    ds = torch.from_numpy(s).to(dev)
    comp = RQA.from_params(p)
    nv = ln - (p.m - 1) * p.tau
    cells = float(np.sum(nv.astype(np.float64) ** 2))
    log(f"[bench] batched: {len(off)} windows, {cells:.3e} cells")

    def fetch_all():
        # every window's measures in one library call
        meas, status = comp.results_batch()
        if status.any():
            raise RuntimeError(f"batched windows failed: {np.unique(status).tolist()}")
        return meas

    settle(comp, lambda: comp.run_batch(ds, off, ln), fetch_all)
    for _ in range(2):
        comp.run_batch(ds, off, ln)
        fetch_all()
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        comp.run_batch(ds, off, ln)
        fetch_all()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    # one profiled run (hipEvents around each phase) for the tile kernel's rate
    comp.set_profiling(True)
    comp.run_batch(ds, off, ln)
    comp.result_batch(0, histograms=False)
    tm = comp.timings()
    comp.set_profiling(False)
    ops = sum(unique_pairs(int(v), p.theiler) for v in nv) * ops_per_pair(p.m, p.norm)
    tile_tops = ops / (tm["tiles_ms"] * 1e-3) / 1e12
    # the same windows, one launch each
    single = RQA.from_params(p)
    views = [ds[int(o):int(o) + int(L)] for o, L in zip(off, ln)]
    # every window once before timing, so that the autotuner has settled for
    # every size class (each class sees its candidate shapes) and the
    # handle's workspace has reached its largest size
    for v in views:
        single.run(v)
        single.result(histograms=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in views:
        single.run(v)
        single.result(histograms=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    comp.close()
    single.close()
    return {"windows": int(len(off)), "cells": cells, "ms": round(tb * 1e3, 3),
            "gcells_per_s": round(cells / tb / 1e9, 3),
            "sequential_ms": round(ts * 1e3, 3),
            "sequential_gcells_per_s": round(cells / ts / 1e9, 3),
            "speedup_vs_sequential": round(ts / tb, 3),
            "tiles_ms": round(tm["tiles_ms"], 3), "stitch_ms": round(tm["stitch_ms"], 3),
            "tile_tops": round(tile_tops, 3), "valu_frac": round(tile_tops / VALU_PEAK_TOPS, 4)}


def bench_full_matrices(args, torch, RQA, workload):
    """Cross recurrence of two Lorenz trajectories, the recurrence plot of one,
    and the RQA of that plot as a given matrix (headline embedding and radius)."""
    n_pts = 262_144
    a, p = workload("lorenz", seed=args.seed + 1, n=n_pts)
    b, _ = workload("lorenz", seed=args.seed + 2, n=n_pts)
    d = (p.m - 1) * p.tau
    dev = torch.device("cuda:0")
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    comp = RQA.from_params(p)
    comp.set_profiling(True)
    out = {}
    # cross recurrence: every cell of the n_a x n_b matrix is evaluated
    na, nb = n_pts - d, n_pts - d
    settle(comp, lambda: comp.run_cross(da, db), lambda: comp.result(histograms=False))
    comp.run_cross(da, db)
    comp.result(histograms=False)
    tm, tl = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        comp.run_cross(da, db)
        r = comp.result(histograms=False)
        tm.append(time.perf_counter() - t0)
        tl.append(comp.timings()["tiles_ms"])
    cells = float(na) * nb
    ms = float(np.median(tm)) * 1e3
    tile_ms = float(np.median(tl))
    ops = cells * ops_per_pair(p.m, p.norm)
    out["cross"] = {"workload": f"lorenz63_x seeds {args.seed + 1},{args.seed + 2} N={n_pts} each, "
                                f"m={p.m} tau={p.tau} Linf eps={p.eps:.6g}",
                    "cells": cells, "ms": round(ms, 3), "gcells_per_s": round(cells / ms / 1e6, 3),
                    "tiles_ms": round(tile_ms, 3), "waves": comp.last_launch()["waves"],
                    "valu_frac": round(ops / (tile_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
                    "rr": r.measures["rr"], "det": r.measures["det"]}
    log(f"[bench] cross: {ms:.2f} ms, tiles {tile_ms:.2f} ms")
    # recurrence plot of the first 65,536 points, then its RQA as a given matrix
    n_plot = 65_536
    n = n_plot - d
    words = (n + 63) // 64
    dsp = da[:n_plot].contiguous()
    bits = comp.plot(dsp)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tp = []
    for _ in range(3):
        ev0.record()
        bits = comp.plot(dsp)
        ev1.record()
        torch.cuda.synchronize()
        tp.append(ev0.elapsed_time(ev1))
    pms = float(np.median(tp))
    wbytes = float(n) * words * 8
    out["plot"] = {"workload": f"recurrence plot of lorenz63_x N={n_plot}, packed {n}x{words} words",
                   "ms": round(pms, 3), "gcells_per_s": round(float(n) * n / pms / 1e6, 3),
                   "write_gb_per_s": round(wbytes / pms / 1e6, 3), "bytes_written": wbytes}
    log(f"[bench] plot: {pms:.3f} ms")
    settle(comp, lambda: comp.run_matrix(bits, n), lambda: comp.result(histograms=False))
    comp.run_matrix(bits, n)
    comp.result(histograms=False)
    tl = []
    for _ in range(3):
        comp.run_matrix(bits, n)
        comp.result(histograms=False)
        tl.append(comp.timings()["tiles_ms"])
    mms = float(np.median(tl))
    out["matrix"] = {"workload": f"given {n}x{n} bit matrix (the plot above)",
                     "tiles_ms": round(mms, 3), "waves": comp.last_launch()["waves"],
                     "gcells_per_s": round(float(n) * n / mms / 1e6, 3),
                     "read_gb_per_s": round(wbytes / mms / 1e6, 3),
                     "hbm_frac": round(wbytes / mms / 1e6 / 8000.0, 4)}
    log(f"[bench] matrix: tiles {mms:.3f} ms")
    comp.close()
    return out


def bench_paper_e2(args, torch, RQA, workload):
    """The paper's runtime workload (Sect. 8.2): sin(linspace(0, 1000 pi, 1000001)),
    m=2, tau=2, radius 1.0 (Euclidean), minimum lengths 2, with and without the
    line of identity; full RQA (histograms and measures to the host), compared
    with the paper's totals on its stated hardware (Tab. 4)."""
    s, p = workload("sine")
    dev = torch.device("cuda:0")
    ds = torch.from_numpy(s).to(dev)
    out = {"workload": "sin(linspace(0, 1000 pi, 1000001)), m=2, tau=2, L2, eps=1.0, min lengths 2",
           "paper_4gpu_s": 68.94, "paper_1gpu_s": 204.81,
           "paper_hardware": "GTX 690 processors (4 GPUs / 1 GPU), OpenCL, Tab. 4",
           "paper_crp_s": 28480.09}
    for w in (1, 0):
        q = type(p)(m=p.m, tau=p.tau, eps=p.eps, norm=p.norm, lmin=2, vmin=2, wmin=2, theiler=w)
        comp = RQA.from_params(q)
        settle(comp, lambda: comp.run(ds), lambda: comp.result(histograms=False))
        bufs = tuple(np.zeros(comp.hist_len(ds.numel()), dtype=np.uint64) for _ in range(3))
        comp.run(ds)
        comp.result(histograms=True, out=bufs)
        t = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            comp.run(ds)
            r = comp.result(histograms=True, out=bufs)
            t.append(time.perf_counter() - t0)
        comp.close()
        sec = float(np.median(t))
        out[f"theiler{w}"] = {"s": round(sec, 4), "rr": r.measures["rr"], "det": r.measures["det"],
                              "speedup_vs_paper_1gpu": round(204.81 / sec, 1),
                              "speedup_vs_paper_4gpu": round(68.94 / sec, 1)}
        log(f"[bench] paper E2 sine, Theiler {w}: {sec * 1e3:.1f} ms")
    return out


def bench_bands(args, torch, RQA, workload, hl):
    """Recombination in bounded memory: the headline series with its line
    summaries held to 1 GiB (row bands with per-line carries) next to the
    one-band run, and a 4,194,304-point Lorenz-63 series with the default limit
    (a quarter of the device's memory) and with 1 GiB.  Full RQA per run
    (histograms and measures to the host), median of 3 after one warm run."""
    dev = torch.device("cuda:0")

    def timed(comp, ds, limit):
        comp.set_workspace_limit(limit)
        comp.run(ds)
        comp.result(histograms=True)
        t = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            comp.run(ds)
            comp.result(histograms=True)
            t.append(time.perf_counter() - t0)
        return float(np.median(t)) * 1e3, comp.last_plan()

    out = {}
    s, p = hl["series"], hl["p"]
    n = hl["n"]
    ds = torch.from_numpy(s).to(dev)
    comp = RQA.from_params(p)
    comp.set_tiling(8, 0)
    one_ms, one_plan = timed(comp, ds, 1 << 50)
    ms, plan = timed(comp, ds, 1 << 30)
    comp.close()
    del ds
    out["N1048576"] = {"limit_bytes": 1 << 30, "ms": round(ms, 2),
                       "gcells_per_s": round(float(n) * n / (ms * 1e-3) / 1e9, 1), **plan,
                       "one_band": {"ms": round(one_ms, 2), **one_plan}}
    log(f"[bench] bands N=1M: 1 GiB {ms:.1f} ms ({plan['bands']} bands, "
        f"{plan['workspace_bytes'] / 1e9:.2f} GB) vs one band {one_ms:.1f} ms "
        f"({one_plan['workspace_bytes'] / 1e9:.2f} GB)")
    s4, p4 = workload("lorenz", seed=args.seed, n=4_194_304)
    n4 = len(s4) - (p4.m - 1) * p4.tau
    ds = torch.from_numpy(s4).to(dev)
    comp = RQA.from_params(p4)
    comp.set_tiling(8, 0)
    big = {"n_points": len(s4), "n_vec": n4, "eps": p4.eps}
    for tag, limit in (("default_limit", 0), ("limit_1GiB", 1 << 30)):
        ms, plan = timed(comp, ds, limit)
        big[tag] = {"ms": round(ms, 1), "gcells_per_s": round(float(n4) * n4 / (ms * 1e-3) / 1e9, 1),
                    **plan}
        log(f"[bench] bands N=4M {tag}: {ms:.0f} ms ({plan['bands']} bands, "
            f"{plan['workspace_bytes'] / 1e9:.2f} GB)")
    comp.close()
    del ds
    out["N4194304"] = big
    return out


def default_waves(n_vec: int) -> int:
    """Waves per workgroup the server uses for a job of n_vec delay vectors
    (the library's default shape: 8 from 32,768 vectors, else 4)."""
    return 8 if n_vec >= 4096 * 8 else 4


def bench_served(args, torch, RQA, Server, reqs):
    """Latency of a Poisson stream through the continuous-batching server, and
    its capacity against the same jobs run one at a time.

    * Poisson: every request submitted at its arrival time (200 req/s, at least
      60 s of arrivals by default), latency = submit to result on the host.
    * capacity: the first `capacity_requests` jobs submitted at once (closed
      loop), total time to the last result.
    * sequential: the same jobs one after another through rqa_run +
      rqa_result, each on a handle created, shaped like the server's (fixed
      workgroup shape, no autotuning trials) and run once before the timed run
      (so no allocation is timed, as the server's pool allocates nothing per
      job); the sum of the timed runs."""
    dev = torch.device("cuda:0")
    dser = [torch.from_numpy(r.series).to(dev) for r in reqs]
    torch.cuda.synchronize()
    nvec = [len(r.series) - (r.params.m - 1) * r.params.tau for r in reqs]
    cells = float(sum(float(v) * v for v in nvec))
    budget = 16 << 30
    srv = Server(budget, streams=4)
    log(f"[bench] served: {len(reqs)} requests over {reqs[-1].arrival:.2f} s, {cells:.3e} cells")
    for r, d in list(zip(reqs, dser))[:4]:
        srv.wait(srv.submit(r.params, d), histograms=False)
    lat = []
    pending = {}
    t_start = time.perf_counter()
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t_start
        while i < len(reqs) and reqs[i].arrival <= now:
            t_sub = time.perf_counter()
            pending[srv.submit(reqs[i].params, dser[i])] = t_sub
            i += 1
        done = []
        for t, t_sub in pending.items():
            if srv.poll(t, histograms=False) is not None:
                lat.append(time.perf_counter() - t_sub)
                done.append(t)
        for t in done:
            del pending[t]
        if not done:
            time.sleep(0.0002)
    span = time.perf_counter() - t_start
    # capacity: a closed batch of the first jobs
    nc = min(args.capacity_requests, len(reqs))
    cap_cells = float(sum(float(v) * v for v in nvec[:nc]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [srv.submit(r.params, d) for r, d in zip(reqs[:nc], dser[:nc])]
    for t in tickets:
        srv.wait(t, histograms=False)
    t_cap = time.perf_counter() - t0
    srv.close()
    # the same jobs one at a time, untimed allocation and shape
    t_seq = 0.0
    for r, d, n in zip(reqs[:nc], dser[:nc], nvec[:nc]):
        c = RQA.from_params(r.params)
        c.set_tiling(default_waves(n), 0)
        c.run(d)
        c.result(histograms=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.run(d)
        c.result(histograms=False)
        t_seq += time.perf_counter() - t0
        c.close()
    # the stream's largest job alone: through the server (nothing else queued)
    # and through rqa_run on a handle of its own, warm, median of 5
    big = max(range(len(reqs)), key=lambda k: float(nvec[k]) * nvec[k])
    srv = Server(budget, streams=4)
    srv.wait(srv.submit(reqs[big].params, dser[big]), histograms=False)
    t_srv = []
    for _ in range(5):
        t0 = time.perf_counter()
        srv.wait(srv.submit(reqs[big].params, dser[big]), histograms=False)
        t_srv.append(time.perf_counter() - t0)
    srv.close()
    c = RQA.from_params(reqs[big].params)
    c.set_tiling(default_waves(nvec[big]), 0)
    c.run(dser[big])
    c.result(histograms=False)
    t_run = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.run(dser[big])
        c.result(histograms=False)
        t_run.append(time.perf_counter() - t0)
    plan = c.last_plan()
    c.close()
    largest = {"n_points": len(reqs[big].series), "n_vec": int(nvec[big]),
               "m": reqs[big].params.m, "norm": reqs[big].params.norm,
               "served_alone_ms": round(float(np.median(t_srv)) * 1e3, 3),
               "run_alone_ms": round(float(np.median(t_run)) * 1e3, 3),
               "column_segments": plan["segs"]}
    log(f"[bench] served: largest job ({largest['n_points']} points) alone "
        f"{largest['served_alone_ms']:.2f} ms through the server, "
        f"{largest['run_alone_ms']:.2f} ms through rqa_run")
    lat_ms = np.array(lat) * 1e3
    return {"requests": len(reqs), "rate_hz": 200.0, "arrival_span_s": round(reqs[-1].arrival, 3),
            "cells": cells, "latency_samples": int(len(lat_ms)),
            "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
            "p99_rank_from_top": int(round(0.01 * len(lat_ms))),
            "span_s": round(span, 3), "gcells_per_s": round(cells / span / 1e9, 3),
            "capacity": {"requests": nc, "cells": cap_cells, "s": round(t_cap, 3),
                         "gcells_per_s": round(cap_cells / t_cap / 1e9, 3),
                         "sequential_s": round(t_seq, 3),
                         "sequential_gcells_per_s": round(cap_cells / t_seq / 1e9, 3),
                         "speedup_vs_sequential": round(t_seq / t_cap, 3)},
            "largest_job": largest}


def probe_valu():
    """Sustained issue rate of the predicate loop alone (16 columns per trip:
    96 predicate VALU instructions + 1 bookkeeping), as wave-instructions per
    clock per CU at 2.4 GHz and as FP32 algorithmic ops/s (6 per column-lane),
    over grids from one workgroup per CU up to 32 per CU (the median of three
    launches each); the last line gives the largest rate, the ceiling."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(REPO, "paper_2402_16853_amd", "libcalib.so"))
    lib.calib_predicate.restype = ctypes.c_int
    lib.calib_predicate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double)]
    iters = 4000
    best = None
    for blocks, threads in ((256, 512), (512, 512), (768, 512), (1024, 512), (1536, 512),
                            (2048, 512), (3072, 512), (4096, 512), (8192, 512),
                            (1024, 256), (2048, 256), (4096, 256), (8192, 256)):
        runs = []
        for _ in range(3):
            ms = ctypes.c_double()
            rc = lib.calib_predicate(blocks, threads, iters, ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"calib_predicate failed ({rc})")
            runs.append(ms.value)
        t = float(np.median(runs))
        waves = blocks * threads // 64
        rate = waves * iters * 97.0 / (t * 1e-3) / 256 / 2.4e9
        ops = waves * iters * 16 * 6 * 64 / (t * 1e-3) / 1e12
        rec = {"probe": "valu", "blocks": blocks, "threads": threads, "ms": round(t, 3),
               "valu_per_clk_per_cu_at_2.4GHz": round(rate, 3), "predicate_tops": round(ops, 3)}
        print(json.dumps(rec), flush=True)
        if best is None or ops > best["predicate_tops"]:
            best = rec
    print(json.dumps({"probe": "valu", "ceiling": best}), flush=True)


def probe_lds():
    """LDS read bandwidth (conflict-free 16-byte reads), TB/s and bytes per clock
    per CU at 2.4 GHz."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(REPO, "paper_2402_16853_amd", "libcalib.so"))
    lib.calib_lds.restype = ctypes.c_int
    lib.calib_lds.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_double)]
    iters = 20000
    for blocks, threads in ((256, 1024), (512, 1024), (512, 512), (1024, 256)):
        ms = ctypes.c_double()
        rc = lib.calib_lds(blocks, threads, iters, ctypes.byref(ms))
        nbytes = float(blocks) * threads * iters * 16
        tbps = nbytes / (ms.value * 1e-3) / 1e12
        print(json.dumps({"probe": "lds", "blocks": blocks, "threads": threads, "rc": rc,
                          "ms": round(ms.value, 3), "tb_per_s": round(tbps, 3),
                          "bytes_per_clk_per_cu_at_2.4GHz": round(tbps * 1e12 / 256 / 2.4e9, 1)}),
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-points", type=int, default=300_000)
    ap.add_argument("--requests", type=int, default=12_000,
                    help="served requests (200 req/s: 12,000 = 60 s of arrivals)")
    ap.add_argument("--capacity-requests", type=int, default=2_000,
                    help="served jobs of the closed-loop capacity run and its sequential baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--only", default="", help="comma list of extra phases to run after the "
                    "headline: batched, served, full, e2, bands, cpu (default: all)")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (0 = default)")
    ap.add_argument("--sweep", action="store_true", help="time the tile kernel per waves setting")
    ap.add_argument("--probe-valu", action="store_true",
                    help="only measure the issue rate of the predicate's VALU instruction "
                         "stream (libcalib.so) and exit")
    ap.add_argument("--probe-lds", action="store_true",
                    help="only measure the LDS read bandwidth (libcalib.so) and exit")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the RQA engine here is single-GPU); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    only = set(x for x in args.only.split(",") if x)

    def want(phase, flag):
        return not args.quick and not flag and (not only or phase in only)

    reqs = None
    if not (args.probe_valu or args.probe_lds or args.probe_copy) and want("served", args.no_served):
        # Made before anything touches the GPU: the series come from forked
        # worker processes.
        from workloads import served_requests
        t0 = time.perf_counter()
        reqs = served_requests(args.requests, rate_hz=200.0, seed=args.seed,
                               workers=min(16, os.cpu_count() or 1))
        log(f"[bench] served stream: {len(reqs)} requests made in {time.perf_counter() - t0:.1f} s")

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.probe_valu:
        probe_valu()
        return
    if args.probe_lds:
        probe_lds()
        return
    if args.probe_copy:
        n = args.probe_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[probe] copied {args.probe_copy} MiB three times")
        return
    from paper_2402_16853_amd import RQA, Server
    from workloads import workload, windows_plan

    hl = bench_headline(args, torch, RQA, workload)
    extra = {}
    if want("batched", args.no_batched):
        extra["batched"] = bench_batched(args, torch, RQA, workload, windows_plan)
    if want("served", args.no_served):
        extra["served"] = bench_served(args, torch, RQA, Server, reqs)
    if want("full", False):
        extra.update(bench_full_matrices(args, torch, RQA, workload))
    if want("e2", False):
        extra["paper_e2"] = bench_paper_e2(args, torch, RQA, workload)
    if want("bands", False):
        extra["bands"] = bench_bands(args, torch, RQA, workload, hl)
    cpu = None
    if want("cpu", args.no_cpu):
        cpu = bench_cpu_baseline(args, hl)

    p = hl["p"]
    line = {
        "metric": METRIC, "value": round(hl["gcells"], 3), "unit": "Gcells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(hl["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lorenz63_x_N1048576_m3_tau10_linf_eps0.05std_w1",
                   "n_points": len(hl["series"]), "n_vec": hl["n"], "m": p.m, "tau": p.tau,
                   "norm": "Linf", "eps": p.eps, "lmin": p.lmin, "vmin": p.vmin, "wmin": p.wmin,
                   "theiler": p.theiler, "seed": args.seed},
        "roofline": hl["roof"],
        "cpu_baseline": cpu,
        "measures": {k: (None if not np.isfinite(v) else round(float(v), 9))
                     for k, v in hl["measures"].items()},
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
