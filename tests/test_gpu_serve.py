"""Served RQA (GPU): jobs of mixed size and parameters submitted while others
run give exactly the result they give alone; admission respects the memory
budget; a job larger than the budget is rejected."""
import time

import numpy as np
import pytest

from workloads import Params, served_requests

pytestmark = pytest.mark.gpu


def _announce(tag, **kw):
    print(f"[case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def same(a, b, tag):
    for name in ("diag", "vert", "white"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.array_equal(x, y), f"{tag}: {name} differs at {np.nonzero(x != y)[0][:6]}"
    for k, v in a.measures.items():
        w = b.measures[k]
        assert (np.isnan(v) and np.isnan(w)) or v == w, (tag, k)


def test_mixed_stream_equals_alone(cuda, oracle_lib):
    import torch
    from paper_2402_16853_amd import RQA, Server
    reqs = served_requests(48, rate_hz=2000.0, seed=3, min_len=300, max_len=30_000)
    dser = [torch.from_numpy(r.series).to(cuda) for r in reqs]
    torch.cuda.synchronize()
    srv = Server(4 << 30, streams=4)
    _announce("serve-mixed", jobs=len(reqs))
    t0 = time.perf_counter()
    tickets = []
    for r, d in zip(reqs, dser):
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(0.0002)
        tickets.append(srv.submit(r.params, d))
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, d, got) in enumerate(zip(reqs, dser, served)):
        _announce("alone", job=k, n=len(r.series))
        alone = RQA.from_params(r.params)(d)
        same(got, alone, f"job {k}")
        if len(r.series) <= 4000:
            ref = oracle_lib.histograms(r.series, r.params.m, r.params.tau, r.params.eps,
                                        r.params.norm, r.params.theiler)
            assert all(np.array_equal(x, y) for x, y in zip((got.diag, got.vert, got.white), ref))


@pytest.mark.parametrize("streams", [1, 2, 3, 4])
def test_large_jobs_mixed_with_small(streams, cuda):
    """Large jobs (launched alone, one workgroup per compute unit, on their own
    stream class) interleaved with small ones give the results they give alone."""
    import torch
    from paper_2402_16853_amd import RQA, Server
    rng = np.random.default_rng(40 + streams)
    jobs = []
    for k in range(14):
        big = k % 4 == 1
        n = int(rng.integers(48_000, 70_000)) if big else int(rng.integers(500, 9_000))
        x = np.cumsum(rng.normal(size=n)).astype(np.float32) * 0.05
        p = Params(m=int(rng.integers(2, 5)), tau=int(rng.integers(1, 4)),
                   eps=float(rng.uniform(0.05, 0.3)), norm=int(rng.integers(1, 4)), theiler=1)
        jobs.append((p, torch.from_numpy(x).to(cuda)))
    torch.cuda.synchronize()
    srv = Server(8 << 30, streams=streams)
    _announce("serve-large-mixed", streams=streams, jobs=len(jobs),
              large=sum(1 for p, d in jobs if d.numel() >= 48_000))
    tickets = [srv.submit(p, d) for p, d in jobs]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for k, ((p, d), got) in enumerate(zip(jobs, served)):
        same(got, RQA.from_params(p)(d), f"streams {streams} job {k} n={d.numel()}")


def test_budget_admission(cuda):
    import torch
    from paper_2402_16853_amd import Server, RQAError
    p = Params(m=2, tau=1, eps=0.2, norm=3, theiler=1)
    rng = np.random.default_rng(9)
    series = [torch.from_numpy(rng.random(6000).astype(np.float32)).to(cuda) for _ in range(12)]
    fp = Server.footprint(p, 6000)
    srv = Server(int(fp * 2.5), streams=3)      # room for two jobs at a time
    _announce("serve-budget", footprint=fp)
    tickets = [srv.submit(p, s) for s in series]
    res = [srv.wait(t) for t in tickets]
    assert all(r.n_vec == 5999 for r in res)
    first = res[0]
    for r in res[1:]:
        assert r.n_vec == first.n_vec
    big = torch.zeros(60_000, dtype=torch.float32, device=cuda)
    with pytest.raises(RQAError):
        srv.submit(p, big)                       # footprint exceeds the whole budget
    srv.close()


def test_poll_before_done_and_nonfinite(cuda):
    import torch
    from paper_2402_16853_amd import Server, RQAError
    p = Params(m=3, tau=2, eps=0.3, norm=2, theiler=1)
    srv = Server(1 << 30, streams=2)
    x = torch.rand(20_000, device=cuda)
    bad = x.clone()
    bad[123] = float("nan")
    _announce("serve-poll")
    t1 = srv.submit(p, x)
    t2 = srv.submit(p, bad)
    r1 = None
    while r1 is None:
        r1 = srv.poll(t1)
        time.sleep(0.0005)
    assert r1.n_vec == 20_000 - 4
    with pytest.raises(RQAError):
        srv.wait(t2)
    srv.close()


def test_served_stream_largest_jobs_match_oracle(cuda, oracle_lib):
    """The 16 longest jobs among the first 400 requests of the served benchmark
    stream (up to 2e5 points each, mixed m, tau, norm; eps at RR ~ 5%), served
    in a mix with short jobs: each equals the oracle (digests of its dense
    histograms stored by tests/golden/make_golden.py, which calls only the
    oracle), and the short ones equal the oracle computed here."""
    import json
    import os

    import torch
    from golden_digest import check_record
    from paper_2402_16853_amd import Server
    from workloads import served_request
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "served_large_seed0_digest.json")))
    big = [served_request(rec["request"], 0.0, g["seed"]) for rec in g["jobs"]]
    small = served_requests(48, rate_hz=2000.0, seed=17, min_len=300, max_len=3000)
    mix = []
    for k in range(max(len(big), len(small))):
        if k < len(small):
            mix.append(("small", k, small[k]))
        if k < len(big):
            mix.append(("big", k, big[k]))
    dser = [torch.from_numpy(r.series).to(cuda) for _, _, r in mix]
    torch.cuda.synchronize()
    srv = Server(16 << 30, streams=4)
    _announce("serve-stream-largest", large=len(big), small=len(small))
    tickets = [srv.submit(r.params, d) for (_, _, r), d in zip(mix, dser)]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for (kind, k, r), got in zip(mix, served):
        if kind == "big":
            rec = g["jobs"][k]
            assert r.params.asdict() == rec["params"]
            check_record(got, rec, f"request {rec['request']} n={len(r.series)}")
        else:
            ref = oracle_lib.histograms(r.series, r.params.m, r.params.tau, r.params.eps,
                                        r.params.norm, r.params.theiler)
            assert all(np.array_equal(x, y) for x, y in zip((got.diag, got.vert, got.white), ref)), k
