"""Seeded series generators and parameter sets (inputs only, no RQA arithmetic).

Every generator works in FP64 and returns a contiguous ``numpy.float32`` array:
the FP32 array is the input both the oracle and the HIP path receive, so the
generator's own rounding never enters a parity comparison.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

NORM_L1 = 1
NORM_L2 = 2
NORM_LINF = 3
NORM_NAMES = {NORM_L1: "L1", NORM_L2: "L2", NORM_LINF: "Linf"}


@dataclass(frozen=True)
class Params:
    """RQA parameters: embedding dimension ``m``, time delay ``tau``, fixed
    radius ``eps`` (an FP32 value), norm (1=L1, 2=L2, 3=L-infinity), minimum
    diagonal / vertical / white-vertical line lengths and the Theiler window."""
    m: int
    tau: int
    eps: float
    norm: int
    lmin: int = 2
    vmin: int = 2
    wmin: int = 2
    theiler: int = 1

    def __post_init__(self):
        object.__setattr__(self, "eps", float(np.float32(self.eps)))

    def asdict(self):
        return asdict(self)


def n_vectors(n_points: int, m: int, tau: int) -> int:
    """Number of delay vectors a series of ``n_points`` yields."""
    return n_points - (m - 1) * tau


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def logistic_series(n: int, r: float, x0: float) -> np.ndarray:
    """x_{t+1} = r x_t (1 - x_t), x_0 given, no transient discarded."""
    out = np.empty(n, dtype=np.float64)
    x = float(x0)
    for t in range(n):
        out[t] = x
        x = r * x * (1.0 - x)
    return _f32(out)


def ar1_series(n: int, phi: float, rng: np.random.Generator) -> np.ndarray:
    """Stationary AR(1) with unit variance: y_t = phi y_{t-1} + e_t,
    e_t ~ N(0, 1 - phi^2), y_0 ~ N(0, 1).  Returned in FP64."""
    e = rng.normal(0.0, math.sqrt(max(1.0 - phi * phi, 0.0)), size=n)
    y = np.empty(n, dtype=np.float64)
    prev = rng.normal()
    for t in range(n):
        prev = phi * prev + e[t]
        y[t] = prev
    return y


def ar1_seasonal_series(n: int, seed: int, phi: float = 0.95, period: float = 365.0,
                        sigma: float = 0.3) -> np.ndarray:
    """AR(1) (phi, unit stationary variance) + sin(2 pi t / period) + N(0, sigma^2),
    z-normalised in FP64 (population std)."""
    rng = np.random.default_rng(seed)
    y = ar1_series(n, phi, rng)
    t = np.arange(n, dtype=np.float64)
    y = y + np.sin(2.0 * math.pi * t / period) + rng.normal(0.0, sigma, size=n)
    y = (y - y.mean()) / y.std()
    return _f32(y)


def lorenz_x_series(n: int, seed: int, dt: float = 0.01, transient: int = 10_000,
                    sigma: float = 10.0, rho: float = 28.0, beta: float = 8.0 / 3.0) -> np.ndarray:
    """x-coordinate of Lorenz-63 integrated with classical RK4 in FP64.

    Initial state U(-10, 10)^3 + (0, 0, 25) from the seed; ``transient`` steps are
    discarded, then ``n`` consecutive states are recorded."""
    rng = np.random.default_rng(seed)
    x, y, z = (rng.uniform(-10.0, 10.0, size=3) + np.array([0.0, 0.0, 25.0])).tolist()
    h = dt
    h2 = 0.5 * dt
    h6 = dt / 6.0
    out = np.empty(n, dtype=np.float64)
    total = transient + n
    for step in range(total):
        if step >= transient:
            out[step - transient] = x
        k1x = sigma * (y - x); k1y = x * (rho - z) - y; k1z = x * y - beta * z
        ax = x + h2 * k1x; ay = y + h2 * k1y; az = z + h2 * k1z
        k2x = sigma * (ay - ax); k2y = ax * (rho - az) - ay; k2z = ax * ay - beta * az
        ax = x + h2 * k2x; ay = y + h2 * k2y; az = z + h2 * k2z
        k3x = sigma * (ay - ax); k3y = ax * (rho - az) - ay; k3z = ax * ay - beta * az
        ax = x + h * k3x; ay = y + h * k3y; az = z + h * k3z
        k4x = sigma * (ay - ax); k4y = ax * (rho - az) - ay; k4z = ax * ay - beta * az
        x += h6 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
        y += h6 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y)
        z += h6 * (k1z + 2.0 * k2z + 2.0 * k3z + k4z)
    return _f32(out)


def uniform_series(n: int, seed: int) -> np.ndarray:
    """i.i.d. U[0, 1) noise."""
    return _f32(np.random.default_rng(seed).random(n))


def sine_series(n: int = 1_000_001, cycles_pi: float = 1000.0) -> np.ndarray:
    """sin(linspace(0, cycles_pi * pi, n)), the runtime series of Sect. 8.2."""
    return _f32(np.sin(np.linspace(0.0, cycles_pi * math.pi, n)))


def corner_lines(boundaries: int = 8, half: int = 20) -> np.ndarray:
    """Strictly increasing series with copied segments: for q = 1..boundaries the
    values s[64q-half : 64q+half] reappear shifted by k_q = 1024 + 128 q.  With
    m = 1 and eps < 1 the only recurrences are these copies, so the matrix holds
    exactly one diagonal line of length 2*half per q (and its mirror image),
    passing from row 64q-1 to row 64q, i.e. through the corner shared by four
    64x64 tiles, with empty tiles on either side.  A structural test input for
    runs that cross tile, wave and strip boundaries."""
    n = 1024 + 192 * (boundaries + 1) + 64
    s = np.arange(n, dtype=np.float64)
    for q in range(1, boundaries + 1):
        r0, k = 64 * q, 1024 + 128 * q
        s[r0 - half + k:r0 + half + k] = s[r0 - half:r0 + half]
    return _f32(s)


def population_std_fp64(series: np.ndarray) -> float:
    """Population standard deviation (ddof=0) accumulated in FP64."""
    return float(np.asarray(series, dtype=np.float64).std())


def workload(name: str, seed: int = 0, n: int | None = None):
    """Return ``(series, Params)`` for a named single-series workload.

    ``n`` overrides the series length (used for scaled-down test cases of the
    same generator and parameters)."""
    if name == "logistic":
        rng = np.random.default_rng(seed)
        x0 = rng.uniform(0.05, 0.95)
        s = logistic_series(n or 2_000, 3.9, x0)
        return s, Params(m=2, tau=1, eps=0.1, norm=NORM_L2, lmin=2, vmin=2, wmin=2, theiler=1)
    if name == "ar1_season":
        s = ar1_seasonal_series(n or 100_000, seed)
        return s, Params(m=3, tau=6, eps=0.5, norm=NORM_L2, lmin=2, vmin=2, wmin=2, theiler=1)
    if name == "lorenz":
        s = lorenz_x_series(n or 1_048_576, seed)
        eps = np.float32(0.05 * population_std_fp64(s))
        return s, Params(m=3, tau=10, eps=float(eps), norm=NORM_LINF, lmin=2, vmin=2, wmin=2,
                         theiler=1)
    if name == "sine":
        s = sine_series(n or 1_000_001)
        return s, Params(m=2, tau=2, eps=1.0, norm=NORM_L2, lmin=2, vmin=2, wmin=2, theiler=1)
    if name == "uniform":
        s = uniform_series(n or 500_000, seed)
        return s, Params(m=5, tau=2, eps=0.3, norm=NORM_L1, lmin=2, vmin=2, wmin=2, theiler=1)
    raise KeyError(name)


def windows_plan(n_points: int = 500_000, count: int = 400, min_len: int = 1_000,
                 max_len: int = 20_000, seed: int = 0):
    """Sliding windows of uneven length: lengths ~ U{min_len..max_len}, offsets
    ~ U{0..N-len}.  Returns ``(offsets, lengths)`` as int64 arrays."""
    rng = np.random.default_rng(seed + 7919)
    lengths = rng.integers(min_len, max_len + 1, size=count).astype(np.int64)
    lengths = np.minimum(lengths, n_points)
    offsets = np.array([rng.integers(0, n_points - L + 1) for L in lengths], dtype=np.int64)
    return offsets, lengths


def _pair_distances_fp64(series: np.ndarray, m: int, tau: int, norm: int, pairs: int,
                         rng: np.random.Generator) -> np.ndarray:
    """Distances (FP64) between ``pairs`` random delay-vector pairs, used only to
    pick a client-side threshold."""
    s = np.asarray(series, dtype=np.float64)
    nv = n_vectors(len(s), m, tau)
    i = rng.integers(0, nv, size=pairs)
    j = rng.integers(0, nv, size=pairs)
    same = i == j
    j[same] = (j[same] + 1) % nv
    d = np.stack([s[i + k * tau] - s[j + k * tau] for k in range(m)], axis=1)
    if norm == NORM_L1:
        return np.abs(d).sum(axis=1)
    if norm == NORM_L2:
        return np.sqrt((d * d).sum(axis=1))
    return np.abs(d).max(axis=1)


@dataclass
class Request:
    """One served RQA job: arrival time (s), the series and its parameters."""
    rid: int
    arrival: float
    series: np.ndarray
    params: Params
    kind: str


def served_request(rid: int, arrival: float = 0.0, seed: int = 0, min_len: int = 1_000,
                   max_len: int = 200_000, target_rr: float = 0.05) -> Request:
    """Request ``rid`` of the served stream: an independent series drawn from
    its own generator (seeded by (seed, rid)), so that any request can be made
    alone and a stream can be made in parallel.  Half logistic maps with
    r ~ U(3.6, 4.0), half AR(1) with phi ~ U(0.5, 0.99); length log-uniform in
    [min_len, max_len]; m ~ U{2,3,4}, tau ~ U{1..8}, norm ~ U{L1, L2, Linf};
    eps = fl32 of the ``target_rr`` quantile of distances over 2^16 random
    pairs."""
    rng = np.random.default_rng([seed + 104729, rid])
    m = int(rng.integers(2, 5))
    tau = int(rng.integers(1, 9))
    norm = int(rng.integers(1, 4))
    length = int(round(math.exp(rng.uniform(math.log(min_len), math.log(max_len)))))
    length = max(length, (m - 1) * tau + 2)
    if rid % 2 == 0:
        r = rng.uniform(3.6, 4.0)
        s = logistic_series(length, r, rng.uniform(0.05, 0.95))
        kind = "logistic"
    else:
        phi = rng.uniform(0.5, 0.99)
        y = ar1_series(length, phi, rng)
        sd = y.std()
        y = (y - y.mean()) / (sd if sd > 0 else 1.0)
        s = _f32(y)
        kind = "ar1"
    d = _pair_distances_fp64(s, m, tau, norm, 1 << 16, rng)
    eps = float(np.float32(np.quantile(d, target_rr)))
    return Request(rid, arrival, s, Params(m=m, tau=tau, eps=eps, norm=norm), kind)


def _served_one(args):
    return served_request(*args)


def served_requests(count: int, rate_hz: float = 200.0, seed: int = 0,
                    min_len: int = 1_000, max_len: int = 200_000, target_rr: float = 0.05,
                    workers: int = 1):
    """Poisson stream of ``count`` independent seeded requests (see
    ``served_request``) at ``rate_hz``: the inter-arrival times come from a
    generator of their own.  ``workers`` > 1 makes the series in that many
    forked processes (the result is the same)."""
    gaps = np.random.default_rng([seed + 104729, 1 << 40]).exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps)
    jobs = [(rid, float(arrivals[rid]), seed, min_len, max_len, target_rr) for rid in range(count)]
    if workers > 1 and count > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_served_one, jobs, chunksize=max(1, count // (8 * workers)))
    return [_served_one(j) for j in jobs]
