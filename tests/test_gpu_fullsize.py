"""Full-size parity (GPU): the Lorenz-63 headline workload (N = 1,048,576,
m=3, tau=10, L-infinity, eps = 0.05 std, Theiler 1) in the launch configuration
the benchmark times, against oracle histograms stored in tests/golden/ (written
by tests/golden/make_golden.py, which calls only the CPU oracle; about 16 min on
8 cores, too slow to recompute per run)."""
import hashlib
import json
import os

import numpy as np
import pytest

from workloads import workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lorenz_seed0.json")


def dense(sparse, n):
    h = np.zeros(n + 1, dtype=np.uint64)
    for k, v in sparse.items():
        h[int(k)] = v
    return h


def test_lorenz_full_size_bit_exact(cuda):
    import torch
    from paper_2402_16853_amd import RQA
    g = json.load(open(GOLDEN))
    s, p = workload("lorenz", seed=g["seed"])
    assert hashlib.sha256(s.tobytes()).hexdigest()[:16] == g["series_sha_prefix"], \
        "generator output changed; regenerate the golden"
    assert p.asdict() == g["params"]
    n = g["n_vec"]
    print(f"[case] lorenz full size n_vec={n}", flush=True)
    comp = RQA.from_params(p)
    res = comp(torch.from_numpy(s).to(cuda))
    comp.close()
    for name in ("diag", "vert", "white"):
        ref = dense(g[name], n)
        got = getattr(res, name)
        assert np.array_equal(got, ref), f"{name} differs at {np.nonzero(got != ref)[0][:8]}"
    for k, ref in g["measures"].items():
        got = res.measures[k]
        if ref is None:
            assert np.isnan(got), k
        else:
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (k, got, ref)
