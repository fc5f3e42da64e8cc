"""HIP path vs the CPU oracle, element by element (GPU).

Histograms must match bit-exactly; measures (FP64 from identical integers) within
1e-12 relative.  Cases span several 64x64 tiles and strips with ragged tails,
every norm, several m/tau, Theiler windows 0..large, and several workgroup
shapes.  Each case prints its parameters before touching the GPU.
"""
import numpy as np
import pytest

from workloads import Params, corner_lines, workload

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def assert_same(res, ref_hist, ref_meas, tag=""):
    d0, v0, w0 = ref_hist
    for name, a, b in (("diag", res.diag, d0), ("vert", res.vert, v0), ("white", res.white, w0)):
        assert a.shape == b.shape, f"{tag} {name} length {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:8]
            raise AssertionError(f"{tag} {name} differs at lengths {bad.tolist()}: "
                                 f"gpu {a[bad].tolist()} oracle {b[bad].tolist()}")
    for k, ref in ref_meas.items():
        got = res.measures[k]
        if np.isnan(ref):
            assert np.isnan(got), f"{tag} {k}: {got} vs NaN"
        else:
            assert abs(got - ref) <= TOL * max(1.0, abs(ref)), f"{tag} {k}: {got} vs {ref}"


def run_gpu(series, p, cuda, waves=0, groups=0):
    import torch
    from paper_2402_16853_amd import RQA
    comp = RQA.from_params(p)
    if waves or groups:
        comp.set_tiling(waves, groups)
    res = comp(torch.from_numpy(np.ascontiguousarray(series, dtype=np.float32)).to(cuda))
    comp.close()
    return res


def random_case(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 8))
    tau = int(rng.integers(1, 5))
    n_vec = int(rng.choice([1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 511, 777, 1024, 1100, 2100,
                            3000]))
    N = n_vec + (m - 1) * tau
    kind = rng.integers(0, 3)
    if kind == 0:
        s = rng.random(N)
    elif kind == 1:
        s = np.cumsum(rng.normal(size=N)) * 0.1
    else:
        s = np.sin(np.arange(N) * 0.3) + 0.05 * rng.normal(size=N)
    s = s.astype(np.float32)
    norm = int(rng.integers(1, 4))
    theiler = int(rng.choice([0, 1, 2, 5, 63, 64, 65, 300]))
    eps = float(rng.uniform(0.05, 0.5))
    return s, Params(m=m, tau=tau, eps=eps, norm=norm, lmin=int(rng.integers(1, 4)),
                     vmin=int(rng.integers(1, 4)), wmin=int(rng.integers(1, 4)), theiler=theiler)


@pytest.mark.parametrize("seed", list(range(40)))
def test_random_small(seed, cuda, oracle_lib):
    s, p = random_case(seed)
    ref = oracle_lib.rqa(s, p)
    for waves in (1, 4):
        _announce("random", seed=seed, n=len(s), m=p.m, tau=p.tau, norm=p.norm, w=p.theiler,
                  waves=waves)
        res = run_gpu(s, p, cuda, waves=waves)
        assert_same(res, *ref, tag=f"seed {seed} waves {waves}")


@pytest.mark.parametrize("waves", [1, 2, 3, 5, 8])
def test_tile_shapes(waves, cuda, oracle_lib):
    """The result does not depend on the workgroup shape or count."""
    s, p = workload("logistic", seed=3, n=3_333)
    ref = oracle_lib.rqa(s, p)
    for groups in (0, 1, 7):
        _announce("shapes", waves=waves, groups=groups, n=len(s))
        assert_same(run_gpu(s, p, cuda, waves=waves, groups=groups), *ref,
                    tag=f"waves {waves} groups {groups}")


def test_logistic_config(cuda, oracle_lib):
    """Logistic map r=3.9, N=2,000, m=2, tau=1, L2, eps=0.1."""
    for seed in range(3):
        s, p = workload("logistic", seed=seed)
        _announce("logistic", seed=seed)
        assert_same(run_gpu(s, p, cuda), *oracle_lib.rqa(s, p), tag=f"logistic {seed}")


def test_constant_and_periodic(cuda, oracle_lib):
    for theiler in (0, 1, 3):
        s = np.full(1500, 0.25, dtype=np.float32)
        p = Params(m=2, tau=3, eps=0.0, norm=3, theiler=theiler)
        _announce("constant", theiler=theiler)
        assert_same(run_gpu(s, p, cuda), *oracle_lib.rqa(s, p), tag=f"constant w={theiler}")
    s = (np.arange(2000) % 7).astype(np.float32)
    p = Params(m=3, tau=2, eps=0.5, norm=2, theiler=1)
    _announce("periodic")
    assert_same(run_gpu(s, p, cuda, waves=2), *oracle_lib.rqa(s, p), tag="periodic")


def test_ar1_config(cuda, oracle_lib):
    """AR(1)+seasonal, N=100,000, m=3, tau=6, L2, eps=0.5 (full size)."""
    s, p = workload("ar1_season", seed=0)
    ref = oracle_lib.rqa(s, p)
    _announce("ar1_season", n=len(s))
    assert_same(run_gpu(s, p, cuda), *ref, tag="ar1_season")


@pytest.mark.parametrize("waves", [1, 2, 3, 4, 8])
def test_lines_through_empty_tile_corners(waves, cuda, oracle_lib):
    """Isolated diagonal lines crossing from row 64q-1 to row 64q at a tile corner,
    next to tiles with no recurrence at all: runs carried across wave and strip
    boundaries through empty tiles."""
    s = corner_lines(8, 20)
    for norm, m in ((1, 1), (3, 1), (2, 2)):
        p = Params(m=m, tau=1, eps=0.25, norm=norm, theiler=1)
        _announce("corner_lines", waves=waves, norm=norm, m=m, n=len(s))
        assert_same(run_gpu(s, p, cuda, waves=waves), *oracle_lib.rqa(s, p),
                    tag=f"corner lines waves {waves} norm {norm} m {m}")


@pytest.mark.parametrize("eps", [0.0, 1e-30, 1e-23, 2.5e-23, 3e-23, 0.3, 1e19, 3e19])
def test_l2_threshold_extremes(eps, cuda, oracle_lib):
    """Euclidean thresholds whose square underflows, sits at the rounding
    boundary or overflows: the first-coordinate bound that lets the kernel skip
    the other coordinates must agree with the full predicate everywhere."""
    import time
    rng = np.random.default_rng(5)
    base = (np.arange(1500) % 7).astype(np.float64)
    s = base + np.where(rng.random(1500) < 0.3, rng.normal(size=1500) * 1e-23, 0.0)
    s = np.concatenate([s, rng.normal(size=600) * 1e18]).astype(np.float32)
    p = Params(m=3, tau=2, eps=eps, norm=2, theiler=1)
    _announce("l2_extremes", eps=eps, n=len(s))
    t0 = time.perf_counter()
    res = run_gpu(s, p, cuda, waves=4)
    assert time.perf_counter() - t0 < 30.0
    assert_same(res, *oracle_lib.rqa(s, p), tag=f"L2 eps={eps}")


@pytest.mark.parametrize("case", ["constant_5000", "sine_24000"])
def test_long_runs_across_strips(case, cuda, oracle_lib):
    """Runs longer than the stitch's LDS bins, ended together by neighbouring
    lines (a constant series: every vertical run spans the column; a slow sine:
    runs of ~500-1,100 rows crossing strip edges in step): the global-atomic
    path that combines equal lengths within a wave."""
    if case == "constant_5000":
        s = np.full(5000, 0.5, dtype=np.float32)
        p = Params(m=2, tau=1, eps=0.0, norm=3, theiler=1)
    else:
        s = np.sin(np.linspace(0.0, 24.0 * np.pi, 24_001)).astype(np.float32)
        p = Params(m=2, tau=2, eps=1.0, norm=2, theiler=1)
    ref = oracle_lib.rqa(s, p)
    for waves in (2, 8):
        _announce("long_runs", case=case, waves=waves, n=len(s))
        assert_same(run_gpu(s, p, cuda, waves=waves), *ref, tag=f"{case} waves {waves}")


@pytest.mark.parametrize("theiler", ["n-1", "n", "n+1", "2^31-1"])
def test_theiler_at_and_beyond_n(theiler, cuda, oracle_lib):
    """Theiler windows that mask all but a corner of the matrix, all of it, or
    reach the top of the 32-bit range: the window is clamped to n before any
    row + window sum is formed on the device, with the same results."""
    rng = np.random.default_rng(8)
    s = (np.cumsum(rng.normal(size=700)) * 0.05).astype(np.float32)
    n = len(s) - 2
    w = {"n-1": n - 1, "n": n, "n+1": n + 1, "2^31-1": 2**31 - 1}[theiler]
    p = Params(m=2, tau=2, eps=5.0, norm=3, theiler=w)
    ref = oracle_lib.rqa(s, p)
    for waves in (1, 8):
        _announce("theiler_large", theiler=w, n=n, waves=waves)
        assert_same(run_gpu(s, p, cuda, waves=waves), *ref, tag=f"theiler {w} waves {waves}")


@pytest.mark.parametrize("waves", [1, 2, 8])
def test_auto_column_segments(waves, cuda, oracle_lib):
    """A job launched alone whose strips are long is cut into column segments
    (blocks walked by different workgroups): rows of U, diagonals and their
    mirrors cross the segment edges.  Lorenz and AR(1) series of 20,000-40,000
    points, Theiler windows 0, 1 and 70, every norm."""
    cases = [("lorenz", 30_000, 0), ("lorenz", 20_000, 70), ("ar1_season", 40_000, 1)]
    for name, n, w in cases:
        s, p = workload(name, seed=5, n=n)
        for norm in (1, 2, 3):
            q = Params(m=p.m, tau=p.tau, eps=p.eps, norm=norm, theiler=w)
            _announce("auto_segments", name=name, n=n, w=w, norm=norm, waves=waves)
            assert_same(run_gpu(s, q, cuda, waves=waves), *oracle_lib.rqa(s, q),
                        tag=f"{name} n={n} w={w} norm={norm} waves={waves}")


def test_result_into_caller_buffers(cuda, oracle_lib):
    """result(out=...) fills the caller's host arrays: the same histograms as new
    arrays and as the oracle, entries past hist_len untouched, twice in a row
    into the same buffers (the second run shorter, so its tails must be cleared),
    and arrays of the wrong kind refused before the library is called."""
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("logistic", seed=3, n=2_600)
    comp = RQA.from_params(p)
    bufs = tuple(np.full(4_000, 7, dtype=np.uint64) for _ in range(3))
    written = 0
    for n in (2_600, 900):
        x = np.ascontiguousarray(s[:n])
        _announce("result_out", n=n)
        comp.run(torch.from_numpy(x).to(cuda))
        fresh = comp.result()
        got = comp.result(out=bufs)
        hl = len(fresh.diag)
        written = max(written, hl)
        ref = oracle_lib.rqa(x, p)
        assert_same(got, *ref, tag=f"out n={n}")
        for a, b, buf in zip((got.diag, got.vert, got.white), (fresh.diag, fresh.vert, fresh.white), bufs):
            assert np.array_equal(a, b)
            assert np.shares_memory(a, buf)
            assert (buf[written:] == 7).all()
    for bad in ((bufs[0], bufs[1]),
                (bufs[0], bufs[1], np.zeros(4_000, dtype=np.int64)),
                (bufs[0], bufs[1], np.zeros(10, dtype=np.uint64)),
                (bufs[0], bufs[1], np.zeros(8_000, dtype=np.uint64)[::2])):
        with pytest.raises(ValueError):
            comp.result(out=bad)
    comp.close()
