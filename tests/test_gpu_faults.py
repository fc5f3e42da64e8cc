"""Failure handling of the tile kernel's bounded waits (GPU), forced from the
host: with RQA_DEBUG_WAIT_GIVEUP=1 every neighbour wait aims at a count no
wave reaches and gives up after 64 polls.  Every kernel still runs to its end,
the job reports RQA_EDEVICE (single run, batched windows), and the next run on
the same handle, without the injection, is exact again."""
import numpy as np
import pytest

from workloads import windows_plan, workload

pytestmark = pytest.mark.gpu


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_wait_give_up_reports_edevice(cuda, oracle_lib, monkeypatch):
    import torch
    from paper_2402_16853_amd import RQA
    from paper_2402_16853_amd._lib import RQAError
    s, p = workload("logistic", seed=1, n=3_000)
    ds = torch.from_numpy(s).to(cuda)
    ref = oracle_lib.histograms(s, p.m, p.tau, p.eps, p.norm, p.theiler)
    comp = RQA.from_params(p)
    comp.set_tiling(4, 0)
    _announce("giveup", n=len(s), waves=4)
    monkeypatch.setenv("RQA_DEBUG_WAIT_GIVEUP", "1")
    with pytest.raises(RQAError) as err:
        comp(ds)
    assert err.value.code == -4
    monkeypatch.delenv("RQA_DEBUG_WAIT_GIVEUP")
    _announce("after-giveup", n=len(s))
    res = comp(ds)
    assert all(np.array_equal(a, b) for a, b in zip((res.diag, res.vert, res.white), ref))
    comp.close()


def test_wait_give_up_in_a_batch(cuda, oracle_lib, monkeypatch):
    import torch
    from paper_2402_16853_amd import RQA
    s, p = workload("uniform", seed=2, n=40_000)
    off, ln = windows_plan(len(s), 12, 700, 5000, seed=2)
    ds = torch.from_numpy(s).to(cuda)
    comp = RQA.from_params(p)
    comp.set_tiling(4, 0)
    _announce("giveup-batch", windows=len(off))
    monkeypatch.setenv("RQA_DEBUG_WAIT_GIVEUP", "1")
    comp.run_batch(ds, off, ln)
    _, status = comp.results_batch()
    assert (status == -4).all(), status
    monkeypatch.delenv("RQA_DEBUG_WAIT_GIVEUP")
    comp.run_batch(ds, off, ln)
    for w in range(len(off)):
        r = comp.result_batch(w)
        ref = oracle_lib.histograms(s[off[w]:off[w] + ln[w]], p.m, p.tau, p.eps, p.norm, p.theiler)
        assert all(np.array_equal(a, b) for a, b in zip((r.diag, r.vert, r.white), ref)), w
    comp.close()
