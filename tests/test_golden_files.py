"""The stored oracle values under tests/golden/ still describe the current
generators and oracle (CPU, no GPU): the series hash, the parameters and a
sample of records are recomputed with the oracle and compared."""
import json
import os

import numpy as np
import pytest

import oracle
from golden_digest import digest
from workloads import served_requests, windows_plan, workload

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return json.load(open(path))


def _same(hists, meas, rec):
    for h, name in zip(hists, ("diag", "vert", "white")):
        assert digest(h) == rec[name], name
    for k, ref in rec["measures"].items():
        got = meas[k]
        assert (ref is None and np.isnan(got)) or got == ref, k


def test_windows400_sample():
    g = _load("windows400_seed0_digest.json")
    s, p = workload("uniform", seed=g["seed"])
    assert p.asdict() == g["params"]
    off, ln = windows_plan(len(s), 400, 1000, 20000, seed=g["seed"])
    assert len(g["windows"]) == 400
    for w in (0, 199, int(np.argmin(ln))):
        rec = g["windows"][w]
        assert (rec["offset"], rec["length"]) == (int(off[w]), int(ln[w]))
        _same(*oracle.rqa(s[off[w]:off[w] + ln[w]], p), rec)


def test_served_large_sample():
    """The stored jobs are the 16 longest of the first 400 requests, with the
    parameters and series the generator makes; the shortest is recomputed."""
    g = _load("served_large_seed0_digest.json")
    reqs = served_requests(g["count"], rate_hz=g["rate_hz"], seed=g["seed"], workers=4)
    longest = sorted(sorted(range(g["count"]), key=lambda k: -len(reqs[k].series))[:16])
    assert [rec["request"] for rec in g["jobs"]] == longest
    import hashlib
    for rec in g["jobs"]:
        r = reqs[rec["request"]]
        assert r.params.asdict() == rec["params"]
        assert hashlib.sha256(r.series.tobytes()).hexdigest()[:16] == rec["series_sha_prefix"]
    rec = min(g["jobs"], key=lambda x: x["n_points"])
    r = reqs[rec["request"]]
    _same(*oracle.rqa(r.series, r.params), rec)


def test_sine_w0_header():
    g = _load("sine_w0_digest.json")
    s, p = workload("sine")
    import hashlib
    assert hashlib.sha256(s.tobytes()).hexdigest()[:16] == g["series_sha_prefix"]
    assert g["params"]["theiler"] == 0 and g["n_vec"] == len(s) - 2
    # the line of identity is one diagonal line of length n; the other
    # diagonal lines come in mirrored pairs, so the number of lines is odd
    assert g["diag"]["lines"] % 2 == 1 and g["diag"]["longest"] == g["n_vec"]
