"""Write oracle histograms for full-size workloads that are too slow to
recompute in every test run.  Calls only the CPU oracle (oracle/) and the
seeded generators (workloads/); nothing here touches the HIP path.

    python tests/golden/make_golden.py lorenz 0        # ~10-20 min on 8 cores
    python tests/golden/make_golden.py sine 0          # the paper's 1,000,001-point sine
    python tests/golden/make_golden.py lorenz_cross    # cross recurrence, 2 x 262,144 points
    python tests/golden/make_golden.py lorenz 0 --measures-only
                                    # recompute the measures from the stored histograms
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
    elif "--measures-only" in sys.argv:
        args = [a for a in sys.argv[1:] if a != "--measures-only"]
        refresh_measures(args[0], int(args[1]) if len(args) > 1 else 0)
    else:
        main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
