"""Batched windowed RQA (GPU): every window of one batched launch equals the
oracle on that window and the same window run alone; windows of uneven length,
tiny windows and ragged tails are mixed in one launch."""
import numpy as np
import pytest

from workloads import Params, windows_plan, workload

pytestmark = pytest.mark.gpu


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def same_hist(res, ref, tag):
    for name, a, b in (("diag", res.diag, ref[0]), ("vert", res.vert, ref[1]),
                       ("white", res.white, ref[2])):
        assert np.array_equal(a, b), f"{tag}: {name} differs at {np.nonzero(a != b)[0][:6]}"


def test_batch_matches_oracle_and_single(cuda, oracle_lib):
    import torch
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(11)
    s = rng.random(40_000).astype(np.float32)
    p = Params(m=5, tau=2, eps=0.3, norm=1, theiler=1)
    lengths = np.array([9, 10, 11, 64 + 8, 65 + 8, 700, 1000, 1500, 2047, 2500, 3100, 64 * 20 + 8]
                       + list(rng.integers(1000, 3000, size=12)), dtype=np.int64)
    offsets = np.array([rng.integers(0, len(s) - L + 1) for L in lengths], dtype=np.int64)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    _announce("batch", windows=len(lengths))
    comp.run_batch(ds, offsets, lengths)
    batch = [comp.result_batch(w) for w in range(len(lengths))]
    single = RQA.from_params(p)
    for w, (o, L) in enumerate(zip(offsets, lengths)):
        win = s[o:o + L]
        ref = oracle_lib.histograms(win, p.m, p.tau, p.eps, p.norm, p.theiler)
        same_hist(batch[w], ref, f"window {w} len {L} vs oracle")
        _announce("single", window=w, length=int(L))
        alone = single(ds[int(o):int(o) + int(L)])
        same_hist(batch[w], (alone.diag, alone.vert, alone.white), f"window {w} batch vs alone")
        for k, v in alone.measures.items():
            b = batch[w].measures[k]
            assert (np.isnan(v) and np.isnan(b)) or v == b, (w, k)
    comp.close()
    single.close()


def test_windowed_config_full(cuda):
    """Uniform noise N=500,000, 400 windows of 1,000..20,000 points, m=5, tau=2, L1,
    eps=0.3: all 400 windows in one launch, in every workgroup shape the
    autotuner may pick.  Every window's three histograms equal the oracle's
    (digests of the dense arrays stored by tests/golden/make_golden.py, which
    calls only the oracle), and its measures agree within 1e-12."""
    import json
    import os

    import torch
    from golden_digest import check_record
    from paper_2402_16853_amd import RQA
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "windows400_seed0_digest.json")))
    s, p = workload("uniform", seed=0)
    assert p.asdict() == g["params"]
    off, ln = windows_plan(len(s), 400, 1000, 20000, seed=0)
    assert [(int(o), int(L)) for o, L in zip(off, ln)] == \
        [(w["offset"], w["length"]) for w in g["windows"]], "window plan changed"
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    for waves in (0, 8, 4, 2):
        _announce("windows400", waves=waves)
        comp.set_tiling(waves, 0)
        comp.run_batch(ds, off, ln)
        for w, rec in enumerate(g["windows"]):
            check_record(comp.result_batch(w), rec, f"waves {waves} window {w} len {ln[w]}")
    comp.close()


def test_repeat_and_shape_independence(cuda):
    """Two launches with different workgroup shapes give identical results."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("uniform", seed=1, n=60_000)
    off, ln = windows_plan(len(s), 30, 500, 6000, seed=1)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    outs = []
    for waves, groups in ((0, 0), (2, 5), (8, 1), (0, 0)):
        _announce("repeat", waves=waves, groups=groups)
        comp.set_tiling(waves, groups)
        comp.run_batch(ds, off, ln)
        outs.append([comp.result_batch(w) for w in range(len(off))])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            same_hist(a, (b.diag, b.vert, b.white), "shape/repeat")
    comp.close()


def test_graph_replays_match_eager(cuda):
    """Identical repeated launches are replayed from a captured hipGraph (after the
    autotuner has settled); every replay, with unrelated eager work and
    synchronisations in between, equals the first eager result."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("uniform", seed=4, n=80_000)
    off, ln = windows_plan(len(s), 40, 500, 8000, seed=4)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    other = RQA(2, 1, 0.2, "euclidean")
    ref = None
    replays = 0
    for rep in range(10):
        _announce("graph", rep=rep)
        comp.run_batch(ds, off, ln)
        res = [comp.result_batch(w) for w in range(len(off))]
        replays += comp.last_launch()["graph_replay"]
        if ref is None:
            ref = res
        else:
            for a, b in zip(ref, res):
                same_hist(b, (a.diag, a.vert, a.white), f"replay {rep}")
        other(ds[:5000])            # eager work on another handle between replays
        torch.cuda.synchronize()
    assert replays >= 4, "the repeated launch was never replayed from a graph"
    comp.close()
    other.close()


def test_bulk_measures_match_per_window(cuda):
    """rqa_result_batch_all gives every window's measures in one call, equal to
    rqa_result_batch window by window; a window holding a NaN gets status
    RQA_ENONFINITE and NaN measures while the others are unaffected."""
    import ctypes

    import torch
    from paper_2402_16853_amd import RQA
    from paper_2402_16853_amd._lib import RQAError, RqaMeasures, lib
    rng = np.random.default_rng(21)
    s = rng.random(60_000).astype(np.float32)
    p = Params(m=3, tau=4, eps=0.2, norm=2, theiler=1)
    lengths = np.array([20, 64 + 8, 999, 2048 + 8, 5000, 12_345, 3000, 777], dtype=np.int64)
    offsets = np.array([0, 100, 1000, 5000, 10_000, 20_000, 40_000, 50_000], dtype=np.int64)
    s[40_000 + 1234] = np.nan        # inside window 6 only
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    _announce("bulk", windows=len(lengths))
    comp.run_batch(ds, offsets, lengths)
    bulk, status = comp.results_batch()
    assert status.tolist() == [0, 0, 0, 0, 0, 0, -5, 0]
    names = [f[0] for f in RqaMeasures._fields_]
    for w in range(len(lengths)):
        if status[w]:
            with pytest.raises(RQAError):
                comp.result_batch(w, histograms=False)
            assert all(np.isnan(bulk[k][w]) for k in names if k not in ("n_rec", "n_vec"))
            assert bulk["n_rec"][w] == 0 and bulk["n_vec"][w] == lengths[w] - (p.m - 1) * p.tau
            continue
        one = comp.result_batch(w, histograms=False)
        for k in names:
            a, b = float(bulk[k][w]), float(one.measures[k])
            assert (np.isnan(a) and np.isnan(b)) or a == b, (w, k, a, b)
    many = (RqaMeasures * 3)()
    assert lib().rqa_result_batch_all(comp._h, ctypes.cast(many, ctypes.c_void_p), None, 3) == -6
    comp.close()
