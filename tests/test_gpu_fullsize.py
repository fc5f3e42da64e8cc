"""Full-size parity (GPU) in the launch configurations the benchmark times
(every workgroup shape the autotuner may pick: 8, 4 and 2 waves; the bench
settles on 8 at these sizes), against oracle histograms stored in tests/golden/ (written by
tests/golden/make_golden.py, which calls only the CPU oracle; 15-30 min each on
8 cores, too slow to recompute per run):

* the Lorenz-63 headline workload (N = 1,048,576, m=3, tau=10, L-infinity,
  eps = 0.05 std, Theiler 1);
* the paper's runtime workload, a sine of 1,000,001 points (m=2, tau=2, L2,
  eps=1.0, Theiler 1), whose recurrence rate is about one half: most runs are
  hundreds of cells long and cross strip edges;
* the cross recurrence of two Lorenz-63 trajectories of 262,144 points each
  (the benchmark's full-matrix workload);
* the sine again with the line of identity kept (Theiler 0), stored as digests
  of the dense histograms."""
import hashlib
import json
import os

import numpy as np
import pytest

from workloads import workload

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# Workgroup shapes (waves per workgroup) the autotuner chooses among.
TUNER_SHAPES = (8, 4, 2)


def check_measures(res, ref_measures):
    for k, ref in ref_measures.items():
        got = res.measures[k]
        if ref is None:
            assert np.isnan(got), k
        else:
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (k, got, ref)


def dense(sparse, n):
    h = np.zeros(n + 1, dtype=np.uint64)
    for k, v in sparse.items():
        h[int(k)] = v
    return h


@pytest.mark.parametrize("name", ["lorenz", "sine"])
def test_full_size_bit_exact(name, cuda):
    import torch
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(GOLDEN_DIR, f"{name}_seed0.json")))
    s, p = workload(name, seed=g["seed"])
    assert hashlib.sha256(s.tobytes()).hexdigest()[:16] == g["series_sha_prefix"], \
        "generator output changed; regenerate the golden"
    assert p.asdict() == g["params"]
    n = g["n_vec"]
    comp = RQA.from_params(p)
    ds = torch.from_numpy(s).to(cuda)
    refs = {h: dense(g[h], n) for h in ("diag", "vert", "white")}
    for waves in TUNER_SHAPES:
        print(f"[case] {name} full size n_vec={n} waves={waves}", flush=True)
        comp.set_tiling(waves, 0)
        res = comp(ds)
        assert comp.last_launch()["waves"] == waves
        for h in ("diag", "vert", "white"):
            got = getattr(res, h)
            assert np.array_equal(got, refs[h]), \
                f"{name} waves {waves} {h} differs at {np.nonzero(got != refs[h])[0][:8]}"
        check_measures(res, g["measures"])
    comp.close()


def test_cross_full_size_bit_exact(cuda):
    """Cross recurrence of two Lorenz-63 trajectories of 262,144 points each
    (6.9e10 cells, every one evaluated), as the benchmark runs it."""
    import torch
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(GOLDEN_DIR, "lorenz_cross_seed1_2.json")))
    a, p = workload("lorenz", seed=g["seeds"][0], n=g["n_points"])
    b, _ = workload("lorenz", seed=g["seeds"][1], n=g["n_points"])
    for x, want in zip((a, b), g["series_sha_prefix"]):
        assert hashlib.sha256(x.tobytes()).hexdigest()[:16] == want, \
            "generator output changed; regenerate the golden"
    assert p.asdict() == g["params"]
    comp = RQA.from_params(p)
    da, db = torch.from_numpy(a).to(cuda), torch.from_numpy(b).to(cuda)
    hl = g["hist_len"]
    for waves in TUNER_SHAPES:
        print(f"[case] lorenz cross full size n_points={g['n_points']} waves={waves}", flush=True)
        comp.set_tiling(waves, 0)
        res = comp.cross(da, db)
        for h in ("diag", "vert", "white"):
            ref = dense(g[h], hl - 1)
            got = getattr(res, h)
            assert got.shape == ref.shape, (h, got.shape, ref.shape)
            assert np.array_equal(got, ref), \
                f"cross waves {waves} {h} differs at {np.nonzero(got != ref)[0][:8]}"
        check_measures(res, g["measures"])
    comp.close()


def test_sine_with_line_of_identity(cuda):
    """The paper's runtime workload with the line of identity kept (Theiler 0),
    as the benchmark also times it: histograms equal the oracle's (digests of
    the dense arrays), measures within 1e-12."""
    import torch
    from golden_digest import check_record
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(GOLDEN_DIR, "sine_w0_digest.json")))
    s, p = workload("sine")
    assert hashlib.sha256(s.tobytes()).hexdigest()[:16] == g["series_sha_prefix"]
    p = type(p)(**{**p.asdict(), "theiler": 0})
    assert p.asdict() == g["params"]
    comp = RQA.from_params(p)
    ds = torch.from_numpy(s).to(cuda)
    for waves in TUNER_SHAPES:
        print(f"[case] sine theiler 0 full size waves={waves}", flush=True)
        comp.set_tiling(waves, 0)
        check_record(comp(ds), g, f"sine w=0 waves {waves}")
    comp.close()
