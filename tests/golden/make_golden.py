"""Write oracle histograms for full-size workloads that are too slow to
recompute in every test run.  Calls only the CPU oracle (oracle/) and the
seeded generators (workloads/); nothing here touches the HIP path.

    python tests/golden/make_golden.py lorenz 0        # ~10-20 min on 8 cores
    python tests/golden/make_golden.py sine 0          # the paper's 1,000,001-point sine
    python tests/golden/make_golden.py lorenz_cross    # cross recurrence, 2 x 262,144 points
    python tests/golden/make_golden.py lorenz 0 --measures-only
                                    # recompute the measures from the stored histograms
    python tests/golden/make_golden.py sine_w0         # the sine with the line of identity
    python tests/golden/make_golden.py windows400      # all 400 windows of the batched workload
    python tests/golden/make_golden.py served_large    # the largest jobs of the served stream

The last three store, per histogram, a digest (SHA-256 of the dense uint64
array, little-endian, index = line length) and its moments instead of the
sparse histogram itself: equal digests mean equal arrays element by element,
and the files stay small (the white-line histograms of these workloads have
thousands of occupied lengths each).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, REPO)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import workload  # noqa: E402

sys.path.insert(0, os.path.dirname(HERE))
from golden_digest import digest  # noqa: E402


def sparse(h):
    nz = np.nonzero(h)[0]
    return {int(k): int(h[k]) for k in nz}


def main(name, seed):
    s, p = workload(name, seed=seed)
    t0 = time.time()
    (d, v, w), meas = oracle.rqa(s, p)
    dt = time.time() - t0
    out = {
        "workload": name, "seed": seed, "n_points": len(s), "n_vec": len(d) - 1,
        "params": p.asdict(), "oracle_seconds": round(dt, 1),
        "series_sha_prefix": __import__("hashlib").sha256(s.tobytes()).hexdigest()[:16],
        "diag": sparse(d), "vert": sparse(v), "white": sparse(w),
        "measures": {k: (None if not np.isfinite(x) else x) for k, x in meas.items()},
    }
    path = os.path.join(HERE, f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, f"{dt:.1f}s")


def main_cross(n_points=262_144, seed_a=1, seed_b=2):
    """Cross recurrence of two Lorenz-63 trajectories (x-coordinate, seeds 1 and
    2, 262,144 points each; the embedding and radius of the first series'
    workload): the full-matrix workload of the benchmark."""
    a, p = workload("lorenz", seed=seed_a, n=n_points)
    b, _ = workload("lorenz", seed=seed_b, n=n_points)
    t0 = time.time()
    (d, v, w), meas = oracle.cross_rqa(a, b, p)
    dt = time.time() - t0
    sha = __import__("hashlib").sha256
    out = {
        "workload": "lorenz_cross", "seeds": [seed_a, seed_b], "n_points": n_points,
        "n_vec": len(a) - (p.m - 1) * p.tau, "hist_len": len(d), "params": p.asdict(),
        "oracle_seconds": round(dt, 1),
        "series_sha_prefix": [sha(a.tobytes()).hexdigest()[:16], sha(b.tobytes()).hexdigest()[:16]],
        "diag": sparse(d), "vert": sparse(v), "white": sparse(w),
        "measures": {k: (None if not np.isfinite(x) else x) for k, x in meas.items()},
    }
    path = os.path.join(HERE, "lorenz_cross_seed1_2.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, f"{dt:.1f}s")


def _record(hists, meas):
    d, v, w = hists
    return {"diag": digest(d), "vert": digest(v), "white": digest(w),
            "measures": {k: (None if not np.isfinite(x) else x) for k, x in meas.items()}}


def main_sine_w0():
    """The paper's runtime workload (1,000,001-point sine, m=2, tau=2, L2, radius
    1.0) with the line of identity kept (Theiler window 0)."""
    s, p = workload("sine")
    p = type(p)(**{**p.asdict(), "theiler": 0})
    t0 = time.time()
    hists, meas = oracle.rqa(s, p)
    dt = time.time() - t0
    out = {"workload": "sine", "n_points": len(s), "n_vec": len(hists[0]) - 1,
           "params": p.asdict(), "oracle_seconds": round(dt, 1),
           "series_sha_prefix": __import__("hashlib").sha256(s.tobytes()).hexdigest()[:16],
           **_record(hists, meas)}
    path = os.path.join(HERE, "sine_w0_digest.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, f"{dt:.1f}s")


def main_windows400(seed=0):
    """Every window of the batched workload: uniform noise, N = 500,000, 400
    windows of 1,000..20,000 points (m=5, tau=2, L1, eps=0.3)."""
    from workloads import windows_plan
    s, p = workload("uniform", seed=seed)
    off, ln = windows_plan(len(s), 400, 1000, 20000, seed=seed)
    t0 = time.time()
    wins = []
    for o, L in zip(off, ln):
        hists, meas = oracle.rqa(s[o:o + L], p)
        wins.append({"offset": int(o), "length": int(L), **_record(hists, meas)})
    dt = time.time() - t0
    out = {"workload": "uniform windows400", "seed": seed, "n_points": len(s),
           "params": p.asdict(), "oracle_seconds": round(dt, 1),
           "series_sha_prefix": __import__("hashlib").sha256(s.tobytes()).hexdigest()[:16],
           "windows": wins}
    path = os.path.join(HERE, f"windows400_seed{seed}_digest.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, f"{dt:.1f}s")


def main_served_large(count=400, seed=0, largest=16):
    """The `largest` longest jobs among the first `count` requests of the served
    stream (Poisson 200 req/s, lengths log-uniform 1e3..2e5, mixed m, tau, norm,
    eps at RR ~ 5%), keyed by request index: the jobs that set the served
    latency tail."""
    from workloads import served_requests
    reqs = served_requests(count, rate_hz=200.0, seed=seed, workers=8)
    pick = sorted(sorted(range(count), key=lambda k: -len(reqs[k].series))[:largest])
    t0 = time.time()
    jobs = []
    for k in pick:
        r = reqs[k]
        hists, meas = oracle.rqa(r.series, r.params)
        jobs.append({"request": k, "n_points": len(r.series), "params": r.params.asdict(),
                     "series_sha_prefix": __import__("hashlib").sha256(r.series.tobytes()).hexdigest()[:16],
                     **_record(hists, meas)})
        print(f"request {k} n={len(r.series)} {time.time() - t0:.0f}s", flush=True)
    dt = time.time() - t0
    out = {"workload": "served stream", "count": count, "seed": seed, "rate_hz": 200.0,
           "oracle_seconds": round(dt, 1), "jobs": jobs}
    path = os.path.join(HERE, f"served_large_seed{seed}_digest.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, f"{dt:.1f}s")


def refresh_measures(name, seed):
    """Recompute the stored measures from the stored histograms (after a change
    to the oracle's measure arithmetic; the histograms stay as written)."""
    path = os.path.join(HERE, f"{name}_seed{seed}.json")
    g = json.load(open(path))
    n = g["n_vec"]
    dense = []
    for key in ("diag", "vert", "white"):
        h = np.zeros(n + 1, dtype=np.uint64)
        for k, v in g[key].items():
            h[int(k)] = v
        dense.append(h)
    p = g["params"]
    meas = oracle.measures(*dense, p["theiler"], p["lmin"], p["vmin"], p["wmin"])
    g["measures"] = {k: (None if not np.isfinite(x) else x) for k, x in meas.items()}
    with open(path, "w") as f:
        json.dump(g, f)
    print(path, "measures refreshed")


if __name__ == "__main__":
    if sys.argv[1] == "lorenz_cross":
        main_cross()
    elif sys.argv[1] == "sine_w0":
        main_sine_w0()
    elif sys.argv[1] == "windows400":
        main_windows400()
    elif sys.argv[1] == "served_large":
        main_served_large()
    elif "--measures-only" in sys.argv:
        args = [a for a in sys.argv[1:] if a != "--measures-only"]
        refresh_measures(args[0], int(args[1]) if len(args) > 1 else 0)
    else:
        main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
