"""The workgroup-shape autotuner (GPU): trials are ordinary runs whose
results equal the oracle's; the default shape is tried first; the tuner
settles within the three candidate shapes and then keeps its choice."""
import numpy as np
import pytest

from workloads import workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_points,default_waves", [(120_000, 8), (9_000, 4)])
def test_trials_start_at_default_and_settle(n_points, default_waves, cuda, oracle_lib):
    import torch
    from paper_2402_16853_amd import RQA
    # a seed of its own, so no earlier test has tuned this signature already
    s, p = workload("lorenz", seed=77, n=n_points)
    p = type(p)(m=p.m, tau=p.tau, eps=p.eps, norm=p.norm, lmin=3, vmin=3, wmin=3, theiler=5)
    ref = oracle_lib.rqa(s, p)[0] if n_points < 50_000 else None
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    shapes, first = [], None
    for k in range(6):
        print(f"[case] tuner n={n_points} run {k}", flush=True)
        res = comp(ds)
        shapes.append(comp.last_launch()["waves"])
        hist = (res.diag, res.vert, res.white)
        if first is None:
            first = hist
        for a, b in zip(hist, first):
            assert np.array_equal(a, b)
        if ref is not None:
            for a, b in zip(hist, ref):
                assert np.array_equal(a, b)
    comp.close()
    assert shapes[0] == default_waves, shapes
    assert set(shapes) <= {2, 4, 8}, shapes
    # at most three trials, then one shape for good
    assert len(set(shapes[3:])) == 1, shapes
