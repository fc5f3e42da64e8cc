"""Independent brute-force RQA for tiny inputs (pure Python + numpy.float32 scalars).

TEST INFRASTRUCTURE ONLY.  It materialises the whole n x n matrix (so n must be
small) and counts runs along every row-wise diagonal, every column and every
column of zeros by scanning explicit Python lists.  It shares nothing with the
C oracle beyond following the same definition (Sect. 2): it does not use the
diagonal-doubling shortcut and it scans both triangles explicitly, so a mistake
in the oracle's symmetry handling, band mask or border handling shows up as a
mismatch.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def _dist_leq(xi, xj, norm, eps, eps_sq):
    """FP32 predicate, coordinates in ascending order, one rounding per op."""
    if norm == 1:
        acc = None
        for a, b in zip(xi, xj):
            t = abs(F32(a) - F32(b))
            acc = t if acc is None else F32(acc + t)
        return bool(acc <= eps)
    if norm == 2:
        acc = None
        for a, b in zip(xi, xj):
            d = F32(F32(a) - F32(b))
            sq = F32(d * d)
            acc = sq if acc is None else F32(acc + sq)
        return bool(acc <= eps_sq)
    best = F32(0.0)
    for a, b in zip(xi, xj):
        t = abs(F32(F32(a) - F32(b)))
        if t > best:
            best = t
    return bool(best <= eps)


def matrix(series, m, tau, eps, norm, theiler):
    """The masked recurrence matrix as a list of lists of 0/1 ints."""
    s = [F32(v) for v in np.asarray(series, dtype=np.float32).tolist()]
    n = len(s) - (m - 1) * tau
    vecs = [[s[i + k * tau] for k in range(m)] for i in range(n)]
    e = F32(eps)
    e2 = F32(e * e)
    R = [[0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if abs(i - j) < theiler:
                continue
            R[i][j] = 1 if _dist_leq(vecs[i], vecs[j], norm, e, e2) else 0
    return R


def _runs(seq, value):
    out = []
    run = 0
    for x in seq:
        if x == value:
            run += 1
        elif run:
            out.append(run)
            run = 0
    if run:
        out.append(run)
    return out


def cross_matrix(a, b, m, tau, eps, norm, theiler=0):
    """The masked cross recurrence matrix (rows: vectors of a, columns: vectors of
    b) as a list of lists of 0/1 ints."""
    sa = [F32(v) for v in np.asarray(a, dtype=np.float32).tolist()]
    sb = [F32(v) for v in np.asarray(b, dtype=np.float32).tolist()]
    na = len(sa) - (m - 1) * tau
    nb = len(sb) - (m - 1) * tau
    va = [[sa[i + k * tau] for k in range(m)] for i in range(na)]
    vb = [[sb[j + k * tau] for k in range(m)] for j in range(nb)]
    e = F32(eps)
    e2 = F32(e * e)
    R = [[0] * nb for _ in range(na)]
    for i in range(na):
        for j in range(nb):
            if abs(i - j) < theiler:
                continue
            R[i][j] = 1 if _dist_leq(va[i], vb[j], norm, e, e2) else 0
    return R


def histograms_from_matrix(R):
    """Histograms of a rectangular 0/1 matrix (list of rows): every diagonal,
    every column; arrays of length max(rows, cols)+1."""
    nr, nc = len(R), len(R[0])
    L = max(nr, nc) + 1
    diag = np.zeros(L, dtype=np.uint64)
    vert = np.zeros(L, dtype=np.uint64)
    white = np.zeros(L, dtype=np.uint64)
    for k in range(-(nr - 1), nc):
        line = [R[i][i + k] for i in range(nr) if 0 <= i + k < nc]
        for run in _runs(line, 1):
            diag[run] += 1
    for j in range(nc):
        col = [R[i][j] for i in range(nr)]
        for run in _runs(col, 1):
            vert[run] += 1
        for run in _runs(col, 0):
            white[run] += 1
    return diag, vert, white


def histograms(series, m, tau, eps, norm, theiler):
    return histograms_from_matrix(matrix(series, m, tau, eps, norm, theiler))


def cross_histograms(a, b, m, tau, eps, norm, theiler=0):
    return histograms_from_matrix(cross_matrix(a, b, m, tau, eps, norm, theiler))


def pack_rows(R):
    """Bit-pack a 0/1 matrix row-major into uint64 words (bit b of word c of row
    i = column 64c+b)."""
    nr, nc = len(R), len(R[0])
    words = (nc + 63) // 64
    out = np.zeros((nr, words), dtype=np.uint64)
    for i in range(nr):
        for j in range(nc):
            if R[i][j]:
                out[i, j >> 6] |= np.uint64(1) << np.uint64(j & 63)
    return out
