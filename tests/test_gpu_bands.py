"""Row bands: recombination in bounded memory (GPU).

A run whose strip-edge summaries would exceed the workspace limit walks its
strips in row bands. Each band's stitch folds the band's summaries into one
open run per column and per diagonal, and the next band goes on from those
carries (paper Sect. 4.1, Divide & Recombine with carry-over state). The
histograms must be those of the oracle, and of the same run in one band, bit
for bit:

* small series, bands of one strip and of a few strips, every norm, Theiler
  windows 0, 1, 3, 70 and windows wider than a strip (the join of column j
  with row j of U then happens bands after column j's last piece), with and
  without column segments;
* the full-size Lorenz-63 and sine workloads with a 1 GB limit, against the
  stored oracle histograms;
* a 4,194,304-point Lorenz-63 series (the oracle would take hours): two
  different band structures agree bit for bit, and the histograms satisfy the
  identities any correct line count does.
"""
import json
import os

import numpy as np
import pytest

from workloads import Params, workload

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-12
UNLIMITED = 1 << 50


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def assert_same(res, ref_hist, ref_meas, tag):
    for name, a, b in zip(("diag", "vert", "white"), (res.diag, res.vert, res.white), ref_hist):
        assert a.shape == b.shape, f"{tag} {name} length {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:8]
            raise AssertionError(f"{tag} {name} differs at lengths {bad.tolist()}: "
                                 f"gpu {a[bad].tolist()} ref {b[bad].tolist()}")
    for k, ref in ref_meas.items():
        got = res.measures[k]
        if np.isnan(ref):
            assert np.isnan(got), f"{tag} {k}: {got} vs NaN"
        else:
            assert abs(got - ref) <= TOL * max(1.0, abs(ref)), f"{tag} {k}: {got} vs {ref}"


def run(comp, ds, limit):
    comp.set_workspace_limit(limit)
    res = comp(ds)
    return res, comp.last_plan()


SMALL = [
    # (series kind, n points, m, tau, norm, eps, theiler, waves)
    ("lorenz", 3000, 3, 10, 3, None, 1, 1),
    ("lorenz", 3000, 3, 10, 3, None, 0, 2),
    ("ar1", 2500, 2, 1, 1, 0.3, 3, 1),
    ("ar1", 2500, 2, 1, 2, 0.3, 70, 1),
    ("ar1", 2000, 1, 1, 3, 0.2, 200, 1),     # window > strip height: deferred joins
    ("sine", 4000, 2, 2, 2, 1.0, 1, 1),     # long runs across every band edge
    ("sine", 4000, 2, 2, 2, 1.0, 0, 4),
    ("logistic", 1500, 5, 1, 1, 0.4, 2, 2),
    ("ar1", 1800, 7, 1, 2, 1.2, 1, 1),      # m beyond the register-held dimensions
    ("ar1", 1800, 8, 2, 3, 0.6, 5, 2),
]


def small_series(kind, n):
    rng = np.random.default_rng(n + len(kind))
    if kind == "lorenz":
        s, p = workload("lorenz", seed=3, n=n)
        return s, p.eps
    if kind == "ar1":
        x = np.zeros(n)
        e = rng.normal(size=n)
        for t in range(1, n):
            x[t] = 0.9 * x[t - 1] + e[t]
        return (x / x.std()).astype(np.float32), None
    if kind == "sine":
        return np.sin(np.linspace(0, 20 * np.pi, n)).astype(np.float32), None
    s, _ = workload("logistic", seed=2, n=n)
    return s, None


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_bands_match_oracle(case, cuda, oracle_lib):
    import torch
    from paper_2402_16853_amd import RQA
    kind, n, m, tau, norm, eps, w, waves = SMALL[case]
    s, eps0 = small_series(kind, n)
    p = Params(m=m, tau=tau, eps=float(eps if eps is not None else eps0), norm=norm, theiler=w)
    ref = oracle_lib.rqa(s, p)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    comp.set_tiling(waves, 0)
    _announce("one band", kind=kind, n=n, m=m, norm=norm, w=w, waves=waves)
    whole, plan1 = run(comp, ds, UNLIMITED)
    assert plan1["bands"] == 1
    assert_same(whole, *ref, tag=f"{kind} one band")
    full_bytes = plan1["workspace_bytes"]
    for limit in (1, full_bytes // 4, full_bytes // 2):
        _announce("bands", kind=kind, n=n, w=w, waves=waves, limit=limit)
        res, plan = run(comp, ds, limit)
        assert plan["bands"] > 1, plan
        # within the limit, unless even one strip per band exceeds it
        assert plan["workspace_bytes"] <= limit or plan["band_strips"] == 1, plan
        assert_same(res, *ref, tag=f"{kind} limit {limit} plan {plan}")
    comp.close()


@pytest.mark.parametrize("waves", [1, 2])
def test_bands_with_column_segments(waves, cuda, oracle_lib):
    """A series long enough for column segments (first strip of 128 tiles or
    more): row pieces and diagonal blocks are folded per band."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("lorenz", seed=5, n=20_000)
    ref = oracle_lib.rqa(s, p)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    comp.set_tiling(waves, 0)
    whole, plan1 = run(comp, ds, UNLIMITED)
    assert plan1["bands"] == 1
    for limit in (plan1["workspace_bytes"] // 6, plan1["workspace_bytes"] // 3):
        _announce("bands+segments", waves=waves, limit=limit)
        res, plan = run(comp, ds, limit)
        assert plan["bands"] > 1 and plan["segs"] > 1, plan
        assert plan["workspace_bytes"] <= limit, plan
        assert_same(res, *ref, tag=f"segments waves {waves} plan {plan}")
    comp.close()


def dense(sparse, n):
    h = np.zeros(n + 1, dtype=np.uint64)
    for k, v in sparse.items():
        h[int(k)] = v
    return h


@pytest.mark.parametrize("name", ["lorenz", "sine"])
def test_full_size_in_one_gigabyte(name, cuda):
    """The full-size workloads with at most 1 GB of line summaries (about
    8.6 GB in one band at N = 1M), against the oracle's stored histograms."""
    import torch
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(GOLDEN_DIR, f"{name}_seed0.json")))
    s, p = workload(name, seed=g["seed"])
    n = g["n_vec"]
    comp = RQA.from_params(p)
    comp.set_tiling(8, 0)
    _announce("full size 1 GB", name=name, n_vec=n)
    res, plan = run(comp, torch.from_numpy(s).to(cuda), 1 << 30)
    print(f"[plan] {plan}", flush=True)
    assert plan["bands"] > 1 and plan["workspace_bytes"] <= 1 << 30, plan
    for h in ("diag", "vert", "white"):
        got, want = getattr(res, h), dense(g[h], n)
        assert np.array_equal(got, want), f"{name} {h} differs at {np.nonzero(got != want)[0][:8]}"
    for k, ref in g["measures"].items():
        got = res.measures[k]
        if ref is None:
            assert np.isnan(got), k
        else:
            assert abs(got - ref) <= TOL * max(1.0, abs(ref)), (k, got, ref)
    comp.close()


def test_four_million_points(cuda):
    """N = 4,194,304 (Lorenz-63, the headline's parameters): 138 GB of line
    summaries in one band.  With the default limit (a quarter of the device's
    memory) and with 1 GB the bands differ, and so do every band edge; the
    histograms must agree, and any correct count satisfies
    sum l P_diag(l) = sum v P_vert(v) = recurrent cells (outside the band) and
    sum v P_vert(v) + sum w P_white(w) = n^2."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("lorenz", seed=0, n=4_194_304)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    comp.set_tiling(8, 0)
    _announce("4M default limit", n_points=len(s))
    a, plan_a = run(comp, ds, 0)
    print(f"[plan] {plan_a}", flush=True)
    _announce("4M 1 GB limit", n_points=len(s))
    b, plan_b = run(comp, ds, 1 << 30)
    print(f"[plan] {plan_b}", flush=True)
    comp.close()
    assert plan_a["bands"] > 1 and plan_b["bands"] > plan_a["bands"], (plan_a, plan_b)
    assert plan_b["workspace_bytes"] <= 1 << 30
    for h in ("diag", "vert", "white"):
        assert np.array_equal(getattr(a, h), getattr(b, h)), h
    n = int(a.n_vec)
    assert len(a.diag) == n + 1
    # exact integer sums (float64 would round above 2^53)
    ld = sum(int(k) * int(c) for k, c in zip(np.nonzero(a.diag)[0], a.diag[np.nonzero(a.diag)]))
    lv = sum(int(k) * int(c) for k, c in zip(np.nonzero(a.vert)[0], a.vert[np.nonzero(a.vert)]))
    lw = sum(int(k) * int(c) for k, c in zip(np.nonzero(a.white)[0], a.white[np.nonzero(a.white)]))
    assert ld == lv == int(a.n_rec), (ld, lv, a.n_rec)
    assert lv + lw == n * n, (lv, lw, n)
    # the recurrence rate stays that of the 1M-point series (same attractor, same eps rule)
    assert 0.0005 < a.measures["rr"] < 0.005, a.measures["rr"]


def test_tiny_series_and_wide_windows(cuda, oracle_lib):
    """Short series (a strip or two), windows at and beyond n: one strip per
    band, against the oracle."""
    import torch
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(44)
    for n in (3, 64, 65, 130, 300):
        s = rng.random(n).astype(np.float32)
        for w in (0, 1, 2, 63, 64, n - 1, n, n + 5):
            p = Params(m=1, tau=1, eps=0.3, norm=3, theiler=w)
            ref = oracle_lib.rqa(s, p)
            comp = RQA.from_params(p)
            comp.set_tiling(1, 0)
            _announce("tiny", n=n, w=w)
            res, plan = run(comp, torch.from_numpy(s).to(cuda), 1)
            comp.close()
            assert_same(res, *ref, tag=f"tiny n={n} w={w} plan {plan}")


def test_batch_of_one_window_in_bands(cuda, oracle_lib):
    """rqa_run_batch with a single window is a run alone: it may be banded."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("lorenz", seed=9, n=9_000)
    ds = torch.from_numpy(s).to(cuda)
    ref = oracle_lib.rqa(s[500:7_500], p)
    comp = RQA.from_params(p)
    comp.set_tiling(2, 0)
    comp.set_workspace_limit(1)
    _announce("batch of one", n=7_000)
    comp.run_batch(ds, [500], [7_000])
    res = comp.result_batch(0)
    plan = comp.last_plan()
    comp.close()
    assert plan["bands"] > 1, plan
    assert_same(res, *ref, tag=f"batch of one {plan}")


def test_banded_graph_replays(cuda, oracle_lib):
    """Identical repeated banded launches are captured once into a hipGraph
    and replayed; the band kernel rewrites the descriptors inside the graph.
    Every replay, with the program's own work in between, equals the oracle."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("lorenz", seed=4, n=6_000)
    ref = oracle_lib.rqa(s, p)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    comp.set_tiling(1, 0)
    comp.set_workspace_limit(1)
    replays = 0
    for k in range(5):
        _announce("banded replay", k=k)
        res = comp(ds)
        replays += comp.last_launch()["graph_replay"]
        assert comp.last_plan()["bands"] > 1
        assert_same(res, *ref, tag=f"run {k}")
        torch.cuda.synchronize()
        (ds * 2.0).sum().item()            # unrelated eager work between replays
    comp.close()
    assert replays >= 3, replays


def test_non_finite_input_in_bands(cuda):
    """A non-finite value anywhere in the series fails the banded run with
    RQA_ENONFINITE, as it fails the run in one band; the next finite run on
    the same handle is exact again."""
    import torch
    from paper_2402_16853_amd import RQA, RQAError
    s, p = workload("lorenz", seed=6, n=5_000)
    bad = s.copy()
    bad[3_333] = np.nan
    comp = RQA.from_params(p)
    comp.set_tiling(1, 0)
    comp.set_workspace_limit(1)
    good_ref = comp(torch.from_numpy(s).to(cuda))
    _announce("non-finite in bands")
    with pytest.raises(RQAError) as err:
        comp(torch.from_numpy(bad).to(cuda))
    assert "NONFINITE" in str(err.value)
    again = comp(torch.from_numpy(s).to(cuda))
    assert comp.last_plan()["bands"] > 1
    for h in ("diag", "vert", "white"):
        assert np.array_equal(getattr(again, h), getattr(good_ref, h)), h
    comp.close()


def _pack(R):
    nr, nc = R.shape
    words = (nc + 63) // 64
    padded = np.zeros((nr, words * 64), dtype=np.uint64)
    padded[:, :nc] = R
    weights = np.uint64(1) << np.arange(64, dtype=np.uint64)
    return (padded.reshape(nr, words, 64) * weights).sum(axis=2, dtype=np.uint64)


@pytest.mark.parametrize("case", range(6))
def test_cross_and_given_matrix_in_bands(case, cuda, oracle_lib):
    """Full (not symmetric) matrices in row bands: cross recurrence of unequal
    series (wide and tall, Theiler bands 0 and 3, long lines across band
    edges) and given bit matrices, one strip per band and a few strips per
    band, against the oracle."""
    import torch
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(900 + case)
    if case < 4:
        na, nb = [(3000, 2100), (1500, 4100), (2600, 2600), (900, 3300)][case]
        t = np.arange(max(na, nb) + 40)
        base = np.sin(2 * np.pi * t / 311.0) + 0.03 * rng.normal(size=len(t))
        a = base[:na].astype(np.float32)
        b = base[17:17 + nb].astype(np.float32)
        p = Params(m=2, tau=2, eps=0.12, norm=(2, 3, 1, 3)[case], theiler=(0, 3, 0, 3)[case])
        ref = oracle_lib.cross_rqa(a, b, p)
        run = lambda comp: comp.cross(torch.from_numpy(a).to(cuda), torch.from_numpy(b).to(cuda))
    else:
        nr, nc = (1900, 1300) if case == 4 else (700, 2500)
        R = (rng.random((nr, nc)) < (0.2 if case == 4 else 0.6)).astype(np.uint64)
        ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
        R[((ii // 150) + (jj // 170)) % 3 == 0] = 1        # long lines in every direction
        bits = _pack(R)
        p = Params(m=1, tau=1, eps=0.0, norm=3, theiler=(0, 2)[case - 4])
        ref_h = oracle_lib.matrix_histograms(bits, nr, nc, p.theiler)
        ref = (ref_h, oracle_lib.rect_measures(*ref_h, nr, nc, p.theiler, p.lmin, p.vmin, p.wmin))
        dbits = torch.from_numpy(bits.view(np.int64)).to(cuda)
        run = lambda comp: comp.matrix(dbits, nc)
    comp = RQA.from_params(p)
    comp.set_tiling(1 + case % 2, 0)
    _announce("full one band", case=case)
    whole, plan1 = run(comp), comp.last_plan()
    assert plan1["bands"] == 1, plan1
    assert_same(whole, *ref, tag=f"full case {case} one band")
    for limit in (1, plan1["workspace_bytes"] // 3):
        comp.set_workspace_limit(limit)
        _announce("full bands", case=case, limit=limit)
        res = run(comp)
        plan = comp.last_plan()
        assert plan["bands"] > 1, plan
        assert_same(res, *ref, tag=f"full case {case} limit {limit} plan {plan}")
    comp.close()


def test_cross_full_size_in_bands(cuda):
    """The 2 x 262,144-point Lorenz cross recurrence (1.1 GB of summaries in
    one band) with 256 MiB, against the oracle's stored histograms."""
    import torch
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(GOLDEN_DIR, "lorenz_cross_seed1_2.json")))
    a, p = workload("lorenz", seed=g["seeds"][0], n=g["n_points"])
    b, _ = workload("lorenz", seed=g["seeds"][1], n=g["n_points"])
    comp = RQA.from_params(p)
    comp.set_tiling(8, 0)
    comp.set_workspace_limit(256 << 20)
    _announce("cross full size 256 MiB")
    res = comp.cross(torch.from_numpy(a).to(cuda), torch.from_numpy(b).to(cuda))
    plan = comp.last_plan()
    print(f"[plan] {plan}", flush=True)
    comp.close()
    assert plan["bands"] > 1 and plan["workspace_bytes"] <= 256 << 20, plan
    hl = g["hist_len"]
    for h in ("diag", "vert", "white"):
        got, want = getattr(res, h), dense(g[h], hl - 1)
        assert np.array_equal(got, want), f"cross {h} differs at {np.nonzero(got != want)[0][:8]}"
