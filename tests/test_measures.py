"""RQA measures from histograms: hand-computed values (oracle and the library's
host code), and agreement of the two implementations on oracle histograms.

The library side runs only host code (rqa_measures_from_hist), so this test
needs no GPU."""
import math

import numpy as np
import pytest

import oracle
from workloads import Params, workload


def hand_histograms():
    n = 10
    D = np.zeros(n + 1, dtype=np.uint64)
    V = np.zeros(n + 1, dtype=np.uint64)
    W = np.zeros(n + 1, dtype=np.uint64)
    D[1], D[2], D[5] = 4, 2, 2
    V[1], V[3] = 6, 2
    W[2], W[4] = 3, 1
    return D, V, W


HAND = {
    "rr": 18 / 90, "det": 14 / 18, "l": 3.5, "lmax": 5.0, "div": 0.2, "l_entr": math.log(2),
    "lam": 0.5, "tt": 3.0, "vmax": 3.0, "v_entr": 0.0, "w": 2.5, "wmax": 4.0,
    "w_entr": -(0.75 * math.log(0.75) + 0.25 * math.log(0.25)), "n_rec": 18.0, "n_vec": 10.0,
}


def close(a, b, tol=1e-12):
    if math.isnan(b):
        return math.isnan(a)
    return abs(a - b) <= tol * max(1.0, abs(b))


def test_oracle_hand_values():
    D, V, W = hand_histograms()
    ms = oracle.measures(D, V, W, theiler=1, lmin=2, vmin=2, wmin=2)
    for k, ref in HAND.items():
        assert close(ms[k], ref), (k, ms[k], ref)


def test_library_hand_values():
    from paper_2402_16853_amd import measures_from_hist
    D, V, W = hand_histograms()
    ms = measures_from_hist(D, V, W, Params(m=1, tau=1, eps=0.1, norm=2, lmin=2, vmin=2, wmin=2,
                                            theiler=1))
    for k, ref in HAND.items():
        assert close(ms[k], ref), (k, ms[k], ref)


def test_empty_histograms_give_nan():
    from paper_2402_16853_amd import measures_from_hist
    z = np.zeros(6, dtype=np.uint64)
    w = z.copy()
    w[5] = 5
    p = Params(m=1, tau=1, eps=0.1, norm=2, theiler=1)
    for ms in (oracle.measures(z, z, w, 1, 2, 2, 2), measures_from_hist(z, z, w, p)):
        assert ms["rr"] == 0.0
        for k in ("det", "l", "div", "l_entr", "lam", "tt", "v_entr"):
            assert math.isnan(ms[k]), k
        assert ms["lmax"] == 0.0 and ms["vmax"] == 0.0 and ms["wmax"] == 5.0


@pytest.mark.parametrize("name,seed", [("logistic", 0), ("logistic", 1), ("ar1_season", 2)])
@pytest.mark.parametrize("theiler", [0, 1, 4])
def test_library_matches_oracle_measures(name, seed, theiler):
    from paper_2402_16853_amd import measures_from_hist
    s, p = workload(name, seed=seed, n=1500)
    p = Params(m=p.m, tau=p.tau, eps=p.eps, norm=p.norm, lmin=3, vmin=2, wmin=4, theiler=theiler)
    (d, v, w), ref = oracle.rqa(s, p)
    got = measures_from_hist(d, v, w, p)
    for k, r in ref.items():
        assert close(got[k], r), (k, got[k], r)


def _exact_entropy(h, floor):
    """The entropy with its terms summed exactly (math.fsum, Shewchuk's exact
    summation): an independent value for the long-histogram case."""
    ls = [l for l in range(max(floor, 1), len(h)) if h[l]]
    total = float(sum(int(h[l]) for l in ls))
    terms = [-(float(h[l]) / total) * math.log(float(h[l]) / total) for l in ls]
    return math.fsum(terms)


@pytest.mark.parametrize("classes", [2_000, 250_000])
def test_entropy_of_long_histograms(classes):
    """A histogram with ~10^5 occupied lengths (as a long, almost periodic
    series produces): both implementations give the entropy within a few ulps
    of the exactly summed value.  A plain running sum is ~1e-11 off here, which
    this bound rejects."""
    from paper_2402_16853_amd import measures_from_hist
    rng = np.random.default_rng(classes)
    n = classes + 10
    h = np.zeros(n + 1, dtype=np.uint64)
    h[2:classes + 2] = (rng.pareto(1.5, size=classes) * 50 + 1).astype(np.uint64)
    ref = _exact_entropy(h, 2)
    z = np.zeros(n + 1, dtype=np.uint64)
    p = Params(m=1, tau=1, eps=0.1, norm=2, lmin=2, vmin=2, wmin=2, theiler=1)
    for got in (oracle.measures(h, z, z, 1, 2, 2, 2)["l_entr"],
                measures_from_hist(h, z, z, p)["l_entr"]):
        assert abs(got - ref) <= 8 * np.spacing(ref), (got, ref)
    naive = 0.0
    tot = float(h[2:].sum())
    for c in h[2:]:
        if c:
            naive -= (float(c) / tot) * math.log(float(c) / tot)
    if classes > 100_000:
        assert abs(naive - ref) > 8 * np.spacing(ref)   # the case the bound is for
