"""Host logic of the row-band planner (no GPU): how a one-series run is cut
when its line summaries are bounded (rqa_workspace_plan, the same code the run
itself uses).  The summaries of one band are O(strips per band x n); the
per-line carries between bands are O(n)."""
import itertools
import math

import pytest

from workloads import Params


def plan(p, n_points, waves, limit):
    from paper_2402_16853_amd import workspace_plan
    return workspace_plan(p, n_points, waves, limit)


P = Params(m=3, tau=10, eps=0.4, norm=3, theiler=1)


def strips(n_points, p, waves):
    n = n_points - (p.m - 1) * p.tau
    wp = min(max(p.theiler, 1), n)
    return max(0, math.ceil((n - wp) / (64 * waves)))


@pytest.mark.parametrize("n_points,waves", list(itertools.product(
    [200, 3_000, 40_000, 300_000, 1_048_576, 4_194_304], [1, 2, 4, 8])))
def test_plan_properties(n_points, waves):
    S = strips(n_points, P, waves)
    whole = plan(P, n_points, waves, 0)
    assert whole["bands"] == 1 and whole["band_strips"] == S
    prev_bands = 1
    for frac in (1.0, 0.5, 0.2, 0.05, 0.01, 0.0):
        limit = max(1, int(whole["workspace_bytes"] * frac))
        q = plan(P, n_points, waves, limit)
        k = q["band_strips"]
        assert 1 <= k <= max(S, 1)
        assert q["bands"] == (math.ceil(S / k) if S > 0 else 1)
        # within the bound, unless even one strip per band exceeds it
        assert q["workspace_bytes"] <= limit or k == 1, (limit, q)
        # a looser bound never needs more bands
        assert q["bands"] >= prev_bands or frac == 1.0
        prev_bands = q["bands"]
        if frac == 1.0:
            assert q == {**whole}, q


def test_one_gigabyte_at_one_and_four_million_points():
    """The cuts the benchmark and the GPU tests run: 8.6 GB of summaries at
    N = 1,048,576 and 137 GB at N = 4,194,304 in one band; under 1 GiB both
    are banded, and the summaries shrink about in proportion to the band."""
    one = plan(P, 1_048_576, 8, 0)
    assert 8.0e9 < one["workspace_bytes"] < 9.0e9
    q = plan(P, 1_048_576, 8, 1 << 30)
    assert q["bands"] > 1 and q["workspace_bytes"] <= 1 << 30
    big = plan(P, 4_194_304, 8, 0)
    assert 1.3e11 < big["workspace_bytes"] < 1.45e11
    q4 = plan(P, 4_194_304, 8, 1 << 30)
    assert q4["bands"] > 100 and q4["workspace_bytes"] <= 1 << 30
    # the O(n) part: a band of one strip still fits in a few bytes per vector
    tiny = plan(P, 4_194_304, 8, 1)
    assert tiny["band_strips"] == 1 and tiny["workspace_bytes"] < 64 * 4_194_304


def test_theiler_and_short_series():
    for w in (0, 1, 63, 64, 65, 500, 10**6):
        p = Params(m=2, tau=3, eps=0.5, norm=2, theiler=w)
        for n in (5, 64, 65, 700, 5_000):
            S = strips(n, p, 1)
            q = plan(p, n, 1, 1)             # the smallest bands: one strip each
            assert q["bands"] == max(1, S), (w, n, q)
            if S:
                assert q["band_strips"] == 1, (w, n, q)


def test_invalid_arguments():
    from paper_2402_16853_amd import RQAError
    with pytest.raises(RQAError):
        plan(P, 1000, 9, 0)                # waves 1..8
    with pytest.raises(RQAError):
        plan(P, 1000, 4, -1)               # negative bound
    with pytest.raises(RQAError):
        plan(P, 15, 4, 0)                  # no delay vector
    with pytest.raises(RQAError):
        plan(Params(m=0, tau=1, eps=0.5, norm=3), 1000, 4, 0)
