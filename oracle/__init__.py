"""CPU oracle for the RQA hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product library never loads
it.  It shares no code with the HIP implementation.

* ``histograms`` -- the plain definition (Sect. 2, Sect. 4.2 operators I-III)
  in C, compiled with ``gcc -O2 -ffp-contract=off`` (``rqa_oracle.c``).
* ``measures``   -- RR, DET, L, Lmax, DIV, L_entr, LAM, TT, Vmax, V_entr, W,
  Wmax, W_entr (names of Tab. 3) in FP64 from the histograms.
* ``cross_histograms`` / ``cross_measures`` -- cross recurrence of two series
  (rows: series a, columns: series b; 2N-1 diagonals, each run once).
* ``matrix_histograms`` -- the same histograms of a given bit matrix.
* ``plot`` -- the masked recurrence (or cross recurrence) matrix, bit-packed.
* ``brute``      -- an independent pure-Python brute force that materialises the
  whole matrix for tiny inputs; it pins the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rqa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MEASURE_NAMES = ("rr", "det", "l", "lmax", "div", "l_entr", "lam", "tt", "vmax",
                 "v_entr", "w", "wmax", "w_entr", "n_rec", "n_vec")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.rqa_oracle_histograms.restype = ctypes.c_int
        lib.rqa_oracle_histograms.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_float,
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int]
        lib.rqa_oracle_measures.restype = ctypes.c_int
        lib.rqa_oracle_measures.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.rqa_oracle_cross_histograms.restype = ctypes.c_int
        lib.rqa_oracle_cross_histograms.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
            ctypes.c_int, ctypes.c_float, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.rqa_oracle_matrix_histograms.restype = ctypes.c_int
        lib.rqa_oracle_matrix_histograms.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.rqa_oracle_rect_measures.restype = ctypes.c_int
        lib.rqa_oracle_rect_measures.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.rqa_oracle_plot.restype = ctypes.c_int
        lib.rqa_oracle_plot.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
            ctypes.c_int, ctypes.c_float, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_int64]
        lib.rqa_oracle_n_vectors.restype = ctypes.c_int64
        lib.rqa_oracle_n_vectors.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        _lib = lib
    return _lib


def n_vectors(n_points: int, m: int, tau: int) -> int:
    return int(_load().rqa_oracle_n_vectors(n_points, m, tau))


def histograms(series, m: int, tau: int, eps: float, norm: int, theiler: int, threads: int = 0):
    """Diagonal, vertical and white-vertical line-length histograms of the whole
    masked recurrence matrix, as three uint64 arrays of length n+1."""
    s = np.ascontiguousarray(series, dtype=np.float32)
    n = n_vectors(len(s), m, tau)
    if n < 1:
        raise ValueError("series too short for the embedding")
    d = np.zeros(n + 1, dtype=np.uint64)
    v = np.zeros(n + 1, dtype=np.uint64)
    w = np.zeros(n + 1, dtype=np.uint64)
    rc = _load().rqa_oracle_histograms(s.ctypes.data, len(s), m, tau, float(np.float32(eps)),
                                       norm, theiler, d.ctypes.data, v.ctypes.data,
                                       w.ctypes.data, threads)
    if rc != 0:
        raise ValueError("invalid oracle arguments")
    return d, v, w


def measures(diag, vert, white, theiler: int, lmin: int, vmin: int, wmin: int) -> dict:
    """RQA measures in FP64 from the three histograms (index = line length)."""
    d = np.ascontiguousarray(diag, dtype=np.uint64)
    v = np.ascontiguousarray(vert, dtype=np.uint64)
    w = np.ascontiguousarray(white, dtype=np.uint64)
    n = len(d) - 1
    out = np.zeros(len(MEASURE_NAMES), dtype=np.float64)
    rc = _load().rqa_oracle_measures(d.ctypes.data, v.ctypes.data, w.ctypes.data, n, theiler,
                                     lmin, vmin, wmin, out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid histogram arguments")
    return dict(zip(MEASURE_NAMES, out.tolist()))


def rqa(series, params, threads: int = 0):
    """Histograms and measures for one series and a parameter object with fields
    m, tau, eps, norm, lmin, vmin, wmin, theiler."""
    d, v, w = histograms(series, params.m, params.tau, params.eps, params.norm, params.theiler,
                         threads)
    return (d, v, w), measures(d, v, w, params.theiler, params.lmin, params.vmin, params.wmin)


def cross_histograms(a, b, m: int, tau: int, eps: float, norm: int, theiler: int = 0,
                     threads: int = 0):
    """Histograms of the cross recurrence matrix of series a (rows) and b
    (columns): three uint64 arrays of length max(n_a, n_b)+1."""
    sa = np.ascontiguousarray(a, dtype=np.float32)
    sb = np.ascontiguousarray(b, dtype=np.float32)
    na, nb = n_vectors(len(sa), m, tau), n_vectors(len(sb), m, tau)
    if na < 1 or nb < 1:
        raise ValueError("series too short for the embedding")
    L = max(na, nb) + 1
    d, v, w = (np.zeros(L, dtype=np.uint64) for _ in range(3))
    rc = _load().rqa_oracle_cross_histograms(sa.ctypes.data, len(sa), sb.ctypes.data, len(sb),
                                             m, tau, float(np.float32(eps)), norm, theiler,
                                             d.ctypes.data, v.ctypes.data, w.ctypes.data,
                                             threads)
    if rc != 0:
        raise ValueError("invalid oracle arguments")
    return d, v, w


def matrix_histograms(bits, n_rows: int, n_cols: int, theiler: int = 0, threads: int = 0):
    """Histograms of a given bit matrix: ``bits`` is a uint64 array of shape
    (n_rows, words) with bit b of word c of row i = column 64c+b."""
    B = np.ascontiguousarray(bits, dtype=np.uint64)
    if B.ndim != 2 or B.shape[0] != n_rows:
        raise ValueError("bits must have shape (n_rows, words)")
    L = max(n_rows, n_cols) + 1
    d, v, w = (np.zeros(L, dtype=np.uint64) for _ in range(3))
    rc = _load().rqa_oracle_matrix_histograms(B.ctypes.data, n_rows, n_cols, B.shape[1], theiler,
                                              d.ctypes.data, v.ctypes.data, w.ctypes.data,
                                              threads)
    if rc != 0:
        raise ValueError("invalid oracle arguments")
    return d, v, w


def rect_measures(diag, vert, white, n_rows: int, n_cols: int, theiler: int, lmin: int,
                  vmin: int, wmin: int) -> dict:
    """Measures of an n_rows x n_cols matrix (cross recurrence or a given
    matrix); ``n_vec`` reports n_rows."""
    d = np.ascontiguousarray(diag, dtype=np.uint64)
    v = np.ascontiguousarray(vert, dtype=np.uint64)
    w = np.ascontiguousarray(white, dtype=np.uint64)
    out = np.zeros(len(MEASURE_NAMES), dtype=np.float64)
    rc = _load().rqa_oracle_rect_measures(d.ctypes.data, v.ctypes.data, w.ctypes.data, n_rows,
                                          n_cols, theiler, lmin, vmin, wmin, out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid histogram arguments")
    return dict(zip(MEASURE_NAMES, out.tolist()))


def cross_rqa(a, b, params, threads: int = 0):
    """Cross recurrence histograms and measures for a parameter object."""
    d, v, w = cross_histograms(a, b, params.m, params.tau, params.eps, params.norm,
                               params.theiler, threads)
    na = n_vectors(len(a), params.m, params.tau)
    nb = n_vectors(len(b), params.m, params.tau)
    return (d, v, w), rect_measures(d, v, w, na, nb, params.theiler, params.lmin, params.vmin,
                                    params.wmin)


def plot(a, params, b=None, words: int | None = None):
    """The masked recurrence matrix of series a (or the cross matrix of a and b)
    packed row-major: uint64 array (rows, words), bit b of word c of row i =
    cell (i, 64c+b)."""
    sa = np.ascontiguousarray(a, dtype=np.float32)
    sb = None if b is None else np.ascontiguousarray(b, dtype=np.float32)
    na = n_vectors(len(sa), params.m, params.tau)
    nb = na if sb is None else n_vectors(len(sb), params.m, params.tau)
    if na < 1 or nb < 1:
        raise ValueError("series too short for the embedding")
    words = (nb + 63) // 64 if words is None else words
    out = np.zeros((na, words), dtype=np.uint64)
    rc = _load().rqa_oracle_plot(sa.ctypes.data, len(sa),
                                 None if sb is None else sb.ctypes.data,
                                 0 if sb is None else len(sb), params.m, params.tau,
                                 float(np.float32(params.eps)), params.norm, params.theiler,
                                 out.ctypes.data, words)
    if rc != 0:
        raise ValueError("invalid oracle arguments")
    return out
