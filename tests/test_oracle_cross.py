"""Pins of the cross recurrence and given-matrix oracle functions against facts
that do not come from them:

* brute force: the independent pure-Python materialised matrix (rectangular,
  every diagonal and column scanned explicitly) on tiny series of unequal length;
* the symmetric special case: cross(s, s) with any Theiler window is the auto
  recurrence matrix, whose histograms the auto oracle computes by a different
  walk (upper-triangle diagonals counted twice);
* transposition: swapping the two series transposes the matrix, which maps
  diagonal k to -k and leaves the diagonal histogram unchanged;
* closed form: two constant series give an all-ones n_a x n_b matrix;
* the given-matrix histograms reproduce both the brute force and the cross
  oracle from the packed matrix; bits past the last column are ignored.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import Params


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("seed", range(40))
def test_cross_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(1, 4))
    tau = int(rng.integers(1, 3))
    na = int(rng.integers(1, 30)) + (m - 1) * tau
    nb = int(rng.integers(1, 30)) + (m - 1) * tau
    a = rng.random(na).astype(np.float32)
    b = rng.random(nb).astype(np.float32)
    norm = int(rng.integers(1, 4))
    w = int(rng.choice([0, 0, 1, 2, 5]))
    eps = float(rng.uniform(0.1, 0.6))
    ref = brute.cross_histograms(a, b, m, tau, eps, norm, w)
    got = oracle.cross_histograms(a, b, m, tau, eps, norm, w)
    assert same(got, ref), (seed, m, tau, na, nb, norm, w)


@pytest.mark.parametrize("seed,w", [(0, 0), (1, 1), (2, 3), (3, 0), (4, 7)])
def test_cross_of_a_series_with_itself_is_auto(seed, w):
    rng = np.random.default_rng(seed)
    s = (np.cumsum(rng.normal(size=400)) * 0.1).astype(np.float32)
    for norm in (1, 2, 3):
        auto = oracle.histograms(s, 3, 2, 0.3, norm, w)
        cross = oracle.cross_histograms(s, s, 3, 2, 0.3, norm, w)
        assert same(cross, auto), (seed, w, norm)
        p = Params(m=3, tau=2, eps=0.3, norm=norm, theiler=w)
        n = len(s) - 4
        ma = oracle.measures(*auto, w, p.lmin, p.vmin, p.wmin)
        mc = oracle.rect_measures(*cross, n, n, w, p.lmin, p.vmin, p.wmin)
        for k in ma:
            assert (np.isnan(ma[k]) and np.isnan(mc[k])) or ma[k] == mc[k], k


@pytest.mark.parametrize("seed", range(6))
def test_cross_transpose_keeps_diagonals(seed):
    rng = np.random.default_rng(50 + seed)
    a = rng.random(300).astype(np.float32)
    b = rng.random(170).astype(np.float32)
    d1, v1, w1 = oracle.cross_histograms(a, b, 2, 3, 0.25, 3, seed % 3)
    d2, v2, w2 = oracle.cross_histograms(b, a, 2, 3, 0.25, 3, seed % 3)
    assert np.array_equal(d1, d2)
    # total cells of each orientation: columns of length n_a vs n_b
    L = np.arange(len(v1), dtype=np.float64)
    assert (L * v1).sum() + (L * w1).sum() == 297 * 167
    assert (L * v2).sum() + (L * w2).sum() == 297 * 167
    assert (L * v1).sum() == (L * v2).sum() == (L * d1).sum()


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 5), (5, 1), (7, 4), (40, 65)])
def test_cross_constant_closed_form(na, nb):
    a = np.full(na, 0.5, dtype=np.float32)
    b = np.full(nb, 0.5, dtype=np.float32)
    d, v, w = oracle.cross_histograms(a, b, 1, 1, 0.0, 2, 0)
    L = max(na, nb) + 1
    D = np.zeros(L, dtype=np.uint64)
    for k in range(-(na - 1), nb):
        D[min(na, nb - k) - max(0, -k)] += 1
    V = np.zeros(L, dtype=np.uint64)
    V[na] = nb
    assert np.array_equal(d, D) and np.array_equal(v, V) and not w.any()
    ms = oracle.rect_measures(d, v, w, na, nb, 0, 2, 2, 2)
    assert ms["rr"] == 1.0 and ms["n_vec"] == na


@pytest.mark.parametrize("seed", range(10))
def test_given_matrix_histograms(seed):
    rng = np.random.default_rng(200 + seed)
    nr, nc = int(rng.integers(1, 90)), int(rng.integers(1, 140))
    R = (rng.random((nr, nc)) < rng.uniform(0.05, 0.7)).astype(int).tolist()
    bits = brute.pack_rows(R)
    # junk past the last column must not matter
    if nc % 64:
        bits[:, -1] |= np.uint64(~((1 << (nc % 64)) - 1) & ((1 << 64) - 1))
    w = int(rng.choice([0, 0, 1, 3]))
    Rm = [[R[i][j] if abs(i - j) >= w else 0 for j in range(nc)] for i in range(nr)]
    ref = brute.histograms_from_matrix(Rm)
    assert same(oracle.matrix_histograms(bits, nr, nc, w), ref)


def test_given_matrix_matches_cross_oracle():
    rng = np.random.default_rng(9)
    a = rng.random(180).astype(np.float32)
    b = rng.random(250).astype(np.float32)
    R = brute.cross_matrix(a, b, 2, 1, 0.2, 1, 0)
    got = oracle.matrix_histograms(brute.pack_rows(R), len(R), len(R[0]), 0)
    assert same(got, oracle.cross_histograms(a, b, 2, 1, 0.2, 1, 0))


@pytest.mark.parametrize("seed", range(8))
def test_plot_matches_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    m, tau = int(rng.integers(1, 4)), int(rng.integers(1, 3))
    n = int(rng.integers(1, 80)) + (m - 1) * tau
    s = rng.random(n).astype(np.float32)
    p = Params(m=m, tau=tau, eps=float(rng.uniform(0.1, 0.5)), norm=int(rng.integers(1, 4)),
               theiler=int(rng.choice([0, 1, 3])))
    got = oracle.plot(s, p)
    assert np.array_equal(got, brute.pack_rows(brute.matrix(s, m, tau, p.eps, p.norm, p.theiler)))
    b = rng.random(int(rng.integers(1, 90)) + (m - 1) * tau).astype(np.float32)
    got = oracle.plot(s, p, b)
    ref = brute.pack_rows(brute.cross_matrix(s, b, m, tau, p.eps, p.norm, p.theiler))
    assert np.array_equal(got, ref)


def test_plot_histograms_match_line_oracles():
    """Lines counted on the packed plot equal the auto and cross line oracles."""
    rng = np.random.default_rng(77)
    s = (np.cumsum(rng.normal(size=900)) * 0.1).astype(np.float32)
    b = (np.cumsum(rng.normal(size=700)) * 0.1).astype(np.float32)
    p = Params(m=3, tau=2, eps=0.2, norm=2, theiler=2)
    n, nb = 896, 696
    assert same(oracle.matrix_histograms(oracle.plot(s, p), n, n, 0),
                oracle.histograms(s, 3, 2, 0.2, 2, 2))
    assert same(oracle.matrix_histograms(oracle.plot(s, p, b), n, nb, 0),
                oracle.cross_histograms(s, b, 3, 2, 0.2, 2, 2))


@pytest.mark.parametrize("na,nb,w", [(7, 4, 1), (4, 7, 2), (30, 11, 5), (11, 30, 5), (9, 40, 9),
                                     (40, 9, 10), (13, 6, 7), (6, 13, 20), (25, 25, 3),
                                     (1, 17, 1), (17, 1, 2), (50, 23, 23)])
def test_rect_rr_denominator_brute_force(na, nb, w):
    """The RR denominator of a rectangular matrix with a Theiler band (the cells
    with |i-j| >= w, Sect. 3 reading of the band for cross recurrence), counted
    cell by cell: RR equals N_rec over that count, for unequal shapes, bands
    wider than the shorter side and bands that cover everything."""
    rng = np.random.default_rng(na * 1000 + nb * 10 + w)
    a = rng.random(na).astype(np.float32)
    b = rng.random(nb).astype(np.float32)
    R = brute.cross_matrix(a, b, 1, 1, 0.4, 3, w)
    n_rec = sum(sum(row) for row in R)
    outside = sum(1 for i in range(na) for j in range(nb) if abs(i - j) >= w)
    hists = oracle.cross_histograms(a, b, 1, 1, 0.4, 3, w)
    ms = oracle.rect_measures(*hists, na, nb, w, 2, 2, 2)
    assert ms["n_rec"] == n_rec
    if outside == 0:
        assert np.isnan(ms["rr"])
    else:
        assert ms["rr"] == n_rec / outside, (ms["rr"], n_rec, outside)
    # all-ones rectangle: every cell outside the band is recurrent, RR = 1
    c = oracle.cross_histograms(np.zeros(na, np.float32), np.zeros(nb, np.float32), 1, 1, 0.0, 3, w)
    mc = oracle.rect_measures(*c, na, nb, w, 2, 2, 2)
    assert mc["n_rec"] == outside
    assert (np.isnan(mc["rr"]) if outside == 0 else mc["rr"] == 1.0)
