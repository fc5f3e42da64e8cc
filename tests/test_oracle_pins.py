"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* brute force: an independent pure-Python implementation that materialises the
  whole matrix and scans every diagonal and column of both triangles (no
  diagonal doubling, no band shortcuts);
* exhaustive: every 0/1 series up to length 9 with eps = 0.5, where every FP32
  operation is exact and R_ij is "x_i equals x_j";
* closed forms: a constant series (fully recurrent outside the Theiler band) and
  a periodic sequence t mod p (recurrent exactly when p divides i - j);
* invariants: first moments of the histograms equal the number of recurrence
  points counted directly, total column length is n^2, diagonal bins are even,
  s -> -s and power-of-two rescaling leave the histograms unchanged;
* the m = 1 special case, where L1 and L-infinity reduce to |s_i - s_j| <= eps;
* isolated copied segments: a known set of diagonal lines and the column runs
  they cut, written out cell by cell.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import corner_lines


def hist(s, m, tau, eps, norm, w):
    return oracle.histograms(np.asarray(s, dtype=np.float32), m, tau, eps, norm, w)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_random(seed):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(1, 5))
    tau = int(rng.integers(1, 4))
    n = int(rng.integers(1, 26))
    N = n + (m - 1) * tau
    s = rng.random(N).astype(np.float32)
    norm = int(rng.integers(1, 4))
    w = int(rng.integers(0, 5))
    eps = float(rng.uniform(0.05, 0.7))
    assert same(hist(s, m, tau, eps, norm, w), brute.histograms(s, m, tau, eps, norm, w))


def test_exhaustive_binary_series():
    combos = [(1, 1, 0), (1, 1, 1), (2, 1, 1), (2, 2, 0), (3, 1, 2), (2, 3, 1)]
    checked = 0
    for N in range(1, 10):
        for bits in itertools.product((0.0, 1.0), repeat=N):
            s = np.array(bits, dtype=np.float32)
            for (m, tau, w) in combos:
                if N - (m - 1) * tau < 1:
                    continue
                norm = 1 + (checked % 3)
                a = hist(s, m, tau, 0.5, norm, w)
                b = brute.histograms(s, m, tau, 0.5, norm, w)
                assert same(a, b), (bits, m, tau, w, norm)
                checked += 1
    assert checked > 2500


@pytest.mark.parametrize("n,w", [(1, 0), (1, 1), (2, 1), (7, 0), (7, 1), (9, 3), (40, 1), (40, 5)])
def test_constant_series_closed_form(n, w):
    s = np.full(n, 0.75, dtype=np.float32)
    d, v, wh = hist(s, 1, 1, 0.0, 2, w)
    D = np.zeros(n + 1, dtype=np.uint64)
    V = np.zeros(n + 1, dtype=np.uint64)
    W = np.zeros(n + 1, dtype=np.uint64)
    if w == 0:
        D[1:n] = 2
        D[n] += 1
        V[n] = n
    else:
        if n - w >= 1:
            D[1:n - w + 1] = 2
            V[1:n - w + 1] = 2
        for j in range(n):
            band = min(j, w - 1) + 1 + min(n - 1 - j, w - 1)
            W[band] += 1
    assert np.array_equal(d, D) and np.array_equal(v, V) and np.array_equal(wh, W)
    if w == 1 and n >= 3:
        ms = oracle.measures(d, v, wh, w, 2, 2, 2)
        assert ms["rr"] == 1.0
        assert math.isclose(ms["det"], 1 - 2 / (n * (n - 1)), rel_tol=1e-15)
        assert math.isclose(ms["lam"], 1 - 2 / (n * (n - 1)), rel_tol=1e-15)
        assert math.isclose(ms["l"], (n * (n - 1) - 2) / (2 * (n - 2)), rel_tol=1e-15)
        assert ms["lmax"] == n - 1 and ms["vmax"] == n - 1
        assert math.isclose(ms["l_entr"], math.log(n - 2), rel_tol=1e-13)


@pytest.mark.parametrize("p,m,tau,norm", [(2, 1, 1, 3), (3, 2, 1, 2), (5, 3, 2, 1), (7, 2, 4, 3),
                                          (11, 4, 3, 2)])
def test_periodic_closed_form(p, m, tau, norm):
    N = 300 + (m - 1) * tau
    s = (np.arange(N) % p).astype(np.float32)
    n = N - (m - 1) * tau
    d, v, wh = hist(s, m, tau, 0.5, norm, 1)
    D = np.zeros(n + 1, dtype=np.uint64)
    for q in range(1, (n - 1) // p + 1):
        D[n - q * p] += 2
    assert np.array_equal(d, D)
    n_rec = sum(2 * (n - q * p) for q in range(1, (n - 1) // p + 1))
    V = np.zeros(n + 1, dtype=np.uint64)
    V[1] = n_rec
    assert np.array_equal(v, V)
    # white runs: per column the gaps between consecutive recurrences
    W = np.zeros(n + 1, dtype=np.uint64)
    for j in range(n):
        rows = [i for i in range(n) if i != j and (i - j) % p == 0]
        edges = [-1] + rows + [n]
        for a, b in zip(edges[:-1], edges[1:]):
            if b - a - 1 > 0:
                W[b - a - 1] += 1
    assert np.array_equal(wh, W)


@pytest.mark.parametrize("seed", range(12))
def test_invariants(seed):
    rng = np.random.default_rng(77 + seed)
    m = int(rng.integers(1, 5))
    tau = int(rng.integers(1, 4))
    N = int(rng.integers(50, 400))
    s = np.cumsum(rng.normal(size=N)).astype(np.float32) * 0.1
    norm = int(rng.integers(1, 4))
    w = int(rng.integers(0, 4))
    eps = float(np.float32(rng.uniform(0.05, 0.5)))
    n = N - (m - 1) * tau
    d, v, wh = hist(s, m, tau, eps, norm, w)
    L = np.arange(n + 1, dtype=np.float64)
    # direct count of recurrence points with numpy FP32 in coordinate order
    X = np.stack([s[k * tau:k * tau + n] for k in range(m)], axis=1).astype(np.float32)
    diff = X[:, None, :] - X[None, :, :]
    if norm == 1:
        acc = np.abs(diff[..., 0])
        for k in range(1, m):
            acc = (acc + np.abs(diff[..., k])).astype(np.float32)
        R = acc <= np.float32(eps)
    elif norm == 2:
        acc = diff[..., 0] * diff[..., 0]
        for k in range(1, m):
            acc = (acc + diff[..., k] * diff[..., k]).astype(np.float32)
        R = acc <= np.float32(np.float32(eps) * np.float32(eps))
    else:
        R = np.abs(diff).max(axis=2) <= np.float32(eps)
    ii, jj = np.indices((n, n))
    R &= np.abs(ii - jj) >= w
    n_rec = int(R.sum())
    assert int((L * d).sum()) == n_rec
    assert int((L * v).sum()) == n_rec
    assert int((L * v).sum() + (L * wh).sum()) == n * n
    dd = d.copy()
    if w == 0:
        dd[n] -= 1
    assert np.all(dd % 2 == 0)
    # symmetry of the predicate under negation and power-of-two scaling
    assert same((d, v, wh), hist(-s, m, tau, eps, norm, w))
    assert same((d, v, wh), hist(s * np.float32(8.0), m, tau, eps * 8.0, norm, w))


@pytest.mark.parametrize("norm", [1, 3])
def test_single_coordinate_textbook(norm):
    """m = 1: both L1 and L-infinity reduce to |s_i - s_j| <= eps."""
    rng = np.random.default_rng(5)
    s = rng.random(120).astype(np.float32)
    eps = np.float32(0.1)
    R = np.abs(s[:, None] - s[None, :]) <= eps
    n = len(s)
    ii, jj = np.indices((n, n))
    R &= ii != jj
    ref = brute.histograms_from_matrix(R.astype(int).tolist())
    assert same(hist(s, 1, 1, float(eps), norm, 1), ref)


def test_rejects_bad_arguments():
    s = np.zeros(10, dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.histograms(s, 4, 4, 0.1, 1, 1)     # too short
    with pytest.raises(ValueError):
        oracle.histograms(s, 1, 1, -1.0, 1, 1)    # negative radius
    with pytest.raises(ValueError):
        oracle.histograms(s, 1, 1, 0.1, 4, 1)     # unknown norm


@pytest.mark.parametrize("boundaries,half,norm", [(2, 20, 1), (8, 20, 3), (5, 7, 2)])
def test_copied_segments_closed_form(boundaries, half, norm):
    """Each copied segment of length 2*half is one diagonal line (counted in both
    triangles); every black cell sits alone in its column, cutting it into two
    white runs; all other columns are white from end to end."""
    s = corner_lines(boundaries, half)
    n = len(s)
    d, v, wh = hist(s, 1, 1, 0.25, norm, 1)
    D = np.zeros(n + 1, dtype=np.uint64)
    V = np.zeros(n + 1, dtype=np.uint64)
    W = np.zeros(n + 1, dtype=np.uint64)
    D[2 * half] = 2 * boundaries
    black_rows = {}
    for q in range(1, boundaries + 1):
        r0, k = 64 * q, 1024 + 128 * q
        for r in range(r0 - half, r0 + half):
            black_rows[r + k] = r          # upper triangle: column r+k, row r
            black_rows[r] = r + k          # lower triangle: column r, row r+k
    V[1] = len(black_rows)
    for col in range(n):
        if col in black_rows:
            i = black_rows[col]
            W[i] += 1
            W[n - 1 - i] += 1
        else:
            W[n] += 1
    assert np.array_equal(d, D) and np.array_equal(v, V) and np.array_equal(wh, W)
