"""Recurrence plot output on the HIP path vs the CPU oracle (GPU): the packed
matrix must equal the oracle's bit for bit; a plot fed back through the
given-matrix RQA reproduces the series' own RQA; extra words per row are left
untouched; undersized rows are rejected."""
import ctypes

import numpy as np
import pytest

from workloads import Params, workload

pytestmark = pytest.mark.gpu


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(cuda)


@pytest.mark.parametrize("seed", range(16))
def test_plot_random(seed, cuda, oracle_lib):
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(9100 + seed)
    m, tau = int(rng.integers(1, 7)), int(rng.integers(1, 4))
    n = int(rng.choice([1, 2, 63, 64, 65, 200, 700, 1100])) + (m - 1) * tau
    nb = int(rng.choice([1, 64, 129, 500, 1030])) + (m - 1) * tau
    a = (np.cumsum(rng.normal(size=n)) * 0.1).astype(np.float32)
    b = (np.cumsum(rng.normal(size=nb)) * 0.1).astype(np.float32)
    p = Params(m=m, tau=tau, eps=float(rng.uniform(0.05, 0.5)), norm=int(rng.integers(1, 4)),
               theiler=int(rng.choice([0, 1, 5, 70])))
    comp = RQA.from_params(p)
    _announce("plot", seed=seed, n=n, m=m, tau=tau, norm=p.norm, w=p.theiler)
    got = comp.plot(dev(a, cuda)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle_lib.plot(a, p)), "auto plot"
    _announce("plot_cross", seed=seed, na=n, nb=nb)
    got = comp.plot(dev(a, cuda), dev(b, cuda)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle_lib.plot(a, p, b)), "cross plot"
    comp.close()


def test_plot_round_trip_through_matrix_rqa(cuda, oracle_lib):
    from paper_2402_16853_amd import RQA
    s, p = workload("logistic", seed=2, n=3_000)
    _announce("plot_round_trip", n=len(s))
    comp = RQA.from_params(p)
    direct = comp(dev(s, cuda))
    bits = comp.plot(dev(s, cuda))
    n = len(s) - (p.m - 1) * p.tau
    # the plot already holds the band as zeros; the matrix run adds nothing
    via = comp.matrix(bits, n)
    comp.close()
    for name in ("diag", "vert", "white"):
        assert np.array_equal(getattr(direct, name), getattr(via, name)), name
    ref = oracle_lib.rqa(s, p)
    assert np.array_equal(direct.diag, ref[0][0])


def test_plot_words_and_errors(cuda):
    import torch
    from paper_2402_16853_amd import RQA
    from paper_2402_16853_amd._lib import lib
    rng = np.random.default_rng(3)
    s = rng.random(300).astype(np.float32)
    p = Params(m=2, tau=1, eps=0.3, norm=2, theiler=1)
    comp = RQA.from_params(p)
    n = 299
    _announce("plot_words", n=n)
    out = torch.full((n, 9), -1, dtype=torch.int64, device=cuda)
    rc = lib().rqa_plot(comp._h, ctypes.c_void_p(dev(s, cuda).data_ptr()), 300,
                        ctypes.c_void_p(out.data_ptr()), 9, None)
    torch.cuda.synchronize()
    assert rc == 0
    o = out.cpu().numpy()
    assert (o[:, 5:] == -1).all()           # words past ceil(n/64) untouched
    ref = comp.plot(dev(s, cuda)).cpu().numpy()
    assert np.array_equal(o[:, :5], ref)
    small = torch.zeros((n, 4), dtype=torch.int64, device=cuda)
    assert lib().rqa_plot(comp._h, ctypes.c_void_p(dev(s, cuda).data_ptr()), 300,
                          ctypes.c_void_p(small.data_ptr()), 4, None) == -6
    comp.close()


def test_plot_and_matrix_at_benchmark_size(cuda, oracle_lib):
    """The benchmark's plot and given-matrix workload: the packed plot of the
    first 65,536 points of a 262,144-point Lorenz-63 series (its embedding and
    radius), then the RQA of that plot as a given matrix, against the oracle's
    RQA of the same points (histograms bit-exact, measures within 1e-12)."""
    from paper_2402_16853_amd import RQA
    a, p = workload("lorenz", seed=1, n=262_144)
    s = np.ascontiguousarray(a[:65_536])
    n = len(s) - (p.m - 1) * p.tau
    _announce("plot_matrix_65536", n=n)
    comp = RQA.from_params(p)
    bits = comp.plot(dev(s, cuda))
    via = comp.matrix(bits, n)
    comp.close()
    (d, v, w), meas = oracle_lib.rqa(s, p)
    for name, ref in (("diag", d), ("vert", v), ("white", w)):
        got = getattr(via, name)
        assert np.array_equal(got, ref), f"{name} differs at {np.nonzero(got != ref)[0][:8]}"
    for k, ref in meas.items():
        got = via.measures[k]
        assert (np.isnan(ref) and np.isnan(got)) or abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), k


@pytest.mark.parametrize("na,nb", [(8_193, None), (9_253, None), (3_000, 20_000), (20_000, 3_000)])
def test_plot_chunk_layouts(na, nb, cuda, oracle_lib):
    """Plots whose 16-tile column chunks do not divide evenly over the 8 XCD
    groups of the wave-to-tile map (9, 10 and 20 chunks; more or fewer row
    tiles than column tiles), against the oracle bit for bit."""
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(na + (nb or 0))
    p = Params(m=3, tau=2, eps=0.3, norm=3, theiler=1)
    a = (np.cumsum(rng.normal(size=na)) * 0.1).astype(np.float32)
    comp = RQA.from_params(p)
    if nb is None:
        _announce("plot_layout", n=na)
        got = comp.plot(dev(a, cuda)).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle_lib.plot(a, p)), "auto plot"
    else:
        b = (np.cumsum(rng.normal(size=nb)) * 0.1).astype(np.float32)
        _announce("plot_layout_cross", na=na, nb=nb)
        got = comp.plot(dev(a, cuda), dev(b, cuda)).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle_lib.plot(a, p, b)), "cross plot"
    comp.close()


def test_plot_scratch_grows_and_is_reused(cuda, oracle_lib):
    """One handle, plots of 300, 5,000 and again 300 points (the handle's plot
    scratch, which holds the column boxes, grows for the second and is reused
    for the third): every plot equals the oracle's."""
    from paper_2402_16853_amd import RQA
    rng = np.random.default_rng(77)
    p = Params(m=2, tau=3, eps=0.25, norm=2, theiler=1)
    comp = RQA.from_params(p)
    for k, n in enumerate((300, 5_000, 300)):
        a = (np.cumsum(rng.normal(size=n)) * 0.1).astype(np.float32)
        _announce("plot_scratch", call=k, n=n)
        got = comp.plot(dev(a, cuda)).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle_lib.plot(a, p)), f"plot {k} (n={n})"
    comp.close()
