"""Digests of dense histograms, as stored by tests/golden/make_golden.py for the
workloads whose histograms are too large to keep element by element: SHA-256
of the uint64 array (little-endian, index = line length) plus its moments.
Equal digests mean equal arrays."""
import hashlib

import numpy as np


def digest(h):
    h = np.ascontiguousarray(h, dtype="<u8")
    nz = np.nonzero(h)[0]
    return {"sha256": hashlib.sha256(h.tobytes()).hexdigest(),
            "len": int(len(h)), "occupied": int(len(nz)),
            "lines": int(sum(int(x) for x in h[nz])),
            "cells": int(sum(int(h[k]) * int(k) for k in nz)),
            "longest": int(nz[-1]) if len(nz) else 0}


def check_record(res, rec, tag, tol=1e-12):
    """res: an RQAResult (histograms and measures); rec: a stored record with
    'diag' / 'vert' / 'white' digests and 'measures'."""
    for name in ("diag", "vert", "white"):
        got = digest(getattr(res, name))
        want = rec[name]
        assert got == want, f"{tag}: {name} histogram differs from the oracle's " \
                            f"(got {got}, oracle {want})"
    for k, ref in rec["measures"].items():
        got = res.measures[k]
        if ref is None:
            assert np.isnan(got), f"{tag} {k}: {got} vs NaN"
        else:
            assert abs(got - ref) <= tol * max(1.0, abs(ref)), f"{tag} {k}: {got} vs {ref}"
