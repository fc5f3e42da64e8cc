"""Full (non-symmetric) matrices on the HIP path vs the CPU oracle (GPU):
cross recurrence of two series and RQA of a given bit matrix.

Histograms bit-exact, measures within 1e-12 relative.  Cases cover unequal
lengths (wide and tall), single-row / single-column matrices, lengths around
tile multiples, every norm, Theiler windows, several workgroup shapes, and the
special case cross(s, s) = auto(s).  Each case prints its parameters first.
"""
import numpy as np
import pytest

from workloads import Params, workload

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def assert_same(res, ref_hist, ref_meas, tag=""):
    for name, a, b in zip(("diag", "vert", "white"), (res.diag, res.vert, res.white), ref_hist):
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


def dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(cuda)


def gpu_cross(a, b, p, cuda, waves=0):
    from paper_2402_16853_amd import RQA
    comp = RQA.from_params(p)
    if waves:
        comp.set_tiling(waves, 0)
    res = comp.cross(dev(a, cuda), dev(b, cuda))
    comp.close()
    return res


def random_pair(seed):
    rng = np.random.default_rng(7000 + seed)
    m = int(rng.integers(1, 6))
    tau = int(rng.integers(1, 4))
    sizes = [1, 2, 63, 64, 65, 127, 129, 300, 777, 1100, 2100]
    na = int(rng.choice(sizes)) + (m - 1) * tau
    nb = int(rng.choice(sizes)) + (m - 1) * tau
    kind = rng.integers(0, 3)
    if kind == 0:
        a, b = rng.random(na), rng.random(nb)
    elif kind == 1:
        a = np.cumsum(rng.normal(size=na)) * 0.1
        b = np.cumsum(rng.normal(size=nb)) * 0.1
    else:
        a = np.sin(np.arange(na) * 0.3) + 0.05 * rng.normal(size=na)
        b = np.sin(np.arange(nb) * 0.3 + 1.0) + 0.05 * rng.normal(size=nb)
    p = Params(m=m, tau=tau, eps=float(rng.uniform(0.05, 0.5)), norm=int(rng.integers(1, 4)),
               lmin=int(rng.integers(1, 4)), vmin=int(rng.integers(1, 4)),
               wmin=int(rng.integers(1, 4)), theiler=int(rng.choice([0, 0, 1, 3, 70])))
    return a.astype(np.float32), b.astype(np.float32), p


@pytest.mark.parametrize("seed", range(30))
def test_cross_random(seed, cuda, oracle_lib):
    a, b, p = random_pair(seed)
    ref = oracle_lib.cross_rqa(a, b, p)
    for waves in (1, 4):
        _announce("cross", seed=seed, na=len(a), nb=len(b), m=p.m, tau=p.tau, norm=p.norm,
                  w=p.theiler, waves=waves)
        assert_same(gpu_cross(a, b, p, cuda, waves), *ref, tag=f"seed {seed} waves {waves}")


@pytest.mark.parametrize("waves", [1, 2, 3, 8])
def test_cross_with_itself_is_auto(waves, cuda, oracle_lib):
    from paper_2402_16853_amd import RQA
    s, p = workload("logistic", seed=1, n=2_500)
    _announce("cross_self", waves=waves, n=len(s))
    comp = RQA.from_params(p)
    comp.set_tiling(waves, 0)
    auto = comp(dev(s, cuda))
    cross = comp.cross(dev(s, cuda), dev(s, cuda))
    comp.close()
    for name in ("diag", "vert", "white"):
        assert np.array_equal(getattr(auto, name), getattr(cross, name)), name
    assert_same(cross, *oracle_lib.rqa(s, p), tag="cross(s,s)")


def test_cross_lorenz_pair(cuda, oracle_lib):
    """Two Lorenz-63 trajectories (x-coordinate, different seeds) of unequal
    length with the benchmark's embedding and radius."""
    a, p = workload("lorenz", seed=1, n=20_000)
    b, _ = workload("lorenz", seed=2, n=13_000)
    _announce("cross_lorenz", na=len(a), nb=len(b))
    assert_same(gpu_cross(a, b, p, cuda), *oracle_lib.cross_rqa(a, b, p), tag="lorenz pair")


def pack(R):
    nr, nc = R.shape
    words = (nc + 63) // 64
    padded = np.zeros((nr, words * 64), dtype=np.uint64)
    padded[:, :nc] = R
    weights = np.uint64(1) << np.arange(64, dtype=np.uint64)
    return (padded.reshape(nr, words, 64) * weights).sum(axis=2, dtype=np.uint64)


@pytest.mark.parametrize("seed", range(12))
def test_given_matrix_random(seed, cuda, oracle_lib):
    import torch
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(8000 + seed)
    nr = int(rng.choice([1, 5, 64, 65, 200, 513, 1500]))
    nc = int(rng.choice([1, 7, 64, 100, 640, 1025]))
    dens = float(rng.choice([0.01, 0.1, 0.5, 0.9]))
    R = (rng.random((nr, nc)) < dens).astype(np.uint64)
    bits = pack(R)
    if nc % 64:                       # junk past the last column is ignored
        bits[:, -1] |= np.uint64(((1 << 64) - 1) ^ ((1 << (nc % 64)) - 1))
    w = int(rng.choice([0, 0, 1, 4]))
    p = Params(m=1, tau=1, eps=0.0, norm=3, lmin=int(rng.integers(1, 4)),
               vmin=int(rng.integers(1, 4)), wmin=int(rng.integers(1, 4)), theiler=w)
    ref_h = oracle_lib.matrix_histograms(bits, nr, nc, w)
    ref_m = oracle_lib.rect_measures(*ref_h, nr, nc, w, p.lmin, p.vmin, p.wmin)
    for waves in (1, 8):
        _announce("matrix", seed=seed, rows=nr, cols=nc, dens=dens, w=w, waves=waves)
        comp = RQA.from_params(p)
        comp.set_tiling(waves, 0)
        res = comp.matrix(torch.from_numpy(bits.view(np.int64)).to(cuda), nc)
        comp.close()
        assert_same(res, ref_h, ref_m, tag=f"matrix seed {seed} waves {waves}")


def test_given_matrix_of_a_cross_predicate(cuda, oracle_lib):
    """The packed cross recurrence matrix, given as bits, reproduces the cross run."""
    import torch
    from paper_2402_16853_amd import RQA
    from oracle import brute
    rng = np.random.default_rng(5)
    a = rng.random(150).astype(np.float32)
    b = rng.random(230).astype(np.float32)
    p = Params(m=2, tau=1, eps=0.2, norm=1, theiler=0)
    bits = brute.pack_rows(brute.cross_matrix(a, b, 2, 1, 0.2, 1, 0))
    _announce("matrix_of_cross", rows=bits.shape[0])
    comp = RQA.from_params(p)
    res_m = comp.matrix(torch.from_numpy(bits.view(np.int64)).to(cuda), 229)
    res_c = comp.cross(dev(a, cuda), dev(b, cuda))
    comp.close()
    for name in ("diag", "vert", "white"):
        assert np.array_equal(getattr(res_m, name), getattr(res_c, name)), name
    assert_same(res_c, *oracle_lib.cross_rqa(a, b, p), tag="cross")


@pytest.mark.parametrize("w", [0, 3])
def test_dense_full_matrices(w, cuda, oracle_lib):
    """Fully recurrent interior tiles in the full-matrix modes: two constant
    series (every cell recurrent), two slow sines (large recurrent blocks), and
    a given matrix of large all-ones / all-zeros blocks."""
    import torch
    from paper_2402_16853_amd import RQA
    cases = [
        (np.full(1500, 0.5), np.full(2300, 0.5), Params(m=2, tau=1, eps=0.0, norm=3, theiler=w)),
        (np.sin(np.linspace(0, 6 * np.pi, 2600)), np.sin(np.linspace(0.5, 9 * np.pi, 3100)),
         Params(m=2, tau=2, eps=1.0, norm=2, theiler=w)),
    ]
    for k, (a, b, p) in enumerate(cases):
        for waves in (2, 8):
            _announce("dense_cross", case=k, w=w, waves=waves, na=len(a), nb=len(b))
            assert_same(gpu_cross(a, b, p, cuda, waves=waves),
                        *oracle_lib.cross_rqa(a.astype(np.float32), b.astype(np.float32), p),
                        tag=f"dense cross {k} w={w} waves {waves}")
    nr, nc = 1500, 1100
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    R = (((ii // 200) + (jj // 300)) % 2 == 0).astype(np.uint64)
    bits = pack(R)
    p = Params(m=1, tau=1, eps=0.0, norm=3, theiler=w)
    ref_h = oracle_lib.matrix_histograms(bits, nr, nc, w)
    ref_m = oracle_lib.rect_measures(*ref_h, nr, nc, w, p.lmin, p.vmin, p.wmin)
    for waves in (2, 8):
        _announce("dense_matrix", w=w, waves=waves)
        comp = RQA.from_params(p)
        comp.set_tiling(waves, 0)
        res = comp.matrix(torch.from_numpy(bits.view(np.int64)).to(cuda), nc)
        comp.close()
        assert_same(res, ref_h, ref_m, tag=f"dense matrix w={w} waves {waves}")


@pytest.mark.parametrize("waves", [1, 4, 8])
def test_diagonals_across_column_segments(waves, cuda, oracle_lib):
    """Long diagonal lines that cross the column-segment edges of the full-matrix
    blocks (and the strip edges) at every offset: two copies of one slow,
    slightly noisy sine, the second shifted and longer, so that the cross matrix
    holds diagonal runs hundreds of cells long on many diagonals, together
    with runs that end exactly at segment edges."""
    rng = np.random.default_rng(81)
    t = np.arange(9000)
    base = np.sin(2 * np.pi * t / 377.0) + 0.02 * rng.normal(size=len(t))
    a = base[:6100].astype(np.float32)
    b = base[37:9000].astype(np.float32)
    for norm, eps in ((3, 0.08), (2, 0.1)):
        p = Params(m=2, tau=3, eps=eps, norm=norm, theiler=0)
        _announce("cross-segments", waves=waves, norm=norm, na=len(a), nb=len(b))
        ref = oracle_lib.cross_rqa(a, b, p)
        assert_same(gpu_cross(a, b, p, cuda, waves=waves), *ref, tag=f"segments w{waves} n{norm}")
        ref = oracle_lib.cross_rqa(b, a, p)
        assert_same(gpu_cross(b, a, p, cuda, waves=waves), *ref, tag=f"segments T w{waves} n{norm}")
