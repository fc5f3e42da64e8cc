"""Python binding of librqa (argument marshalling only; every step of the hot
path runs in the HIP kernels of librqa.so).

Mirrors the workflow of Sect. 7: parameters (Settings), a computation created
from them, ``run`` on a series, and a result object with one member per
measure.  PyTorch provides the device memory (CUDA/HIP float32 tensors) and the
stream; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from ._lib import (RQA_OK, RQA_EINVAL, RQA_ESIZE, RQA_ESTATE, ENONFINITE, RqaMeasures,
                   RqaParams, check, lib, EAGAIN, RQAError)

NORMS = {"l1": 1, "taxicab": 1, "manhattan": 1, "l2": 2, "euclidean": 2,
         "linf": 3, "maximum": 3, "chebyshev": 3, 1: 1, 2: 2, 3: 3}

MEASURE_FIELDS = ("rr", "det", "l", "lmax", "div", "l_entr", "lam", "tt", "vmax", "v_entr",
                  "w", "wmax", "w_entr")


def norm_code(norm) -> int:
    key = norm.lower() if isinstance(norm, str) else norm
    if key not in NORMS:
        raise ValueError(f"unknown norm {norm!r}")
    return NORMS[key]


@dataclass
class RQAResult:
    """Measures (FP64) and the three line-length histograms (index = length)."""
    measures: dict
    diag: np.ndarray | None = None
    vert: np.ndarray | None = None
    white: np.ndarray | None = None
    n_vec: int = 0
    n_rec: int = 0
    extra: dict = field(default_factory=dict)

    # PyRQA-style attribute names (Tab. 3 of the paper)
    @property
    def recurrence_rate(self): return self.measures["rr"]
    @property
    def determinism(self): return self.measures["det"]
    @property
    def average_diagonal_line(self): return self.measures["l"]
    @property
    def longest_diagonal_line(self): return self.measures["lmax"]
    @property
    def divergence(self): return self.measures["div"]
    @property
    def entropy_diagonal_lines(self): return self.measures["l_entr"]
    @property
    def laminarity(self): return self.measures["lam"]
    @property
    def trapping_time(self): return self.measures["tt"]
    @property
    def longest_vertical_line(self): return self.measures["vmax"]
    @property
    def entropy_vertical_lines(self): return self.measures["v_entr"]
    @property
    def average_white_vertical_line(self): return self.measures["w"]
    @property
    def longest_white_vertical_line(self): return self.measures["wmax"]
    @property
    def entropy_white_vertical_lines(self): return self.measures["w_entr"]


def _measures_dict(ms: RqaMeasures) -> dict:
    d = {k: getattr(ms, k) for k in MEASURE_FIELDS}
    d["n_rec"] = float(ms.n_rec)
    d["n_vec"] = float(ms.n_vec)
    return d


def _device_series(series):
    import torch
    if not isinstance(series, torch.Tensor):
        raise TypeError("series must be a torch tensor on the GPU")
    if not series.is_cuda:
        raise ValueError("series must live in device memory (a CUDA/HIP tensor)")
    if series.dtype != torch.float32:
        raise ValueError("series must be float32")
    if series.dim() != 1 or not series.is_contiguous():
        raise ValueError("series must be a contiguous 1-D tensor")
    return series


def _device_bits(bits):
    import torch
    if not isinstance(bits, torch.Tensor):
        raise TypeError("bits must be a torch tensor on the GPU")
    if not bits.is_cuda:
        raise ValueError("bits must live in device memory (a CUDA/HIP tensor)")
    if bits.dtype not in (torch.int64, getattr(torch, "uint64", torch.int64)):
        raise ValueError("bits must be a 64-bit integer tensor")
    if bits.dim() != 2 or not bits.is_contiguous():
        raise ValueError("bits must be a contiguous 2-D tensor (rows, words)")
    return bits


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_params(m, tau, eps, norm, lmin=2, vmin=2, wmin=2, theiler=1) -> RqaParams:
    return RqaParams(int(m), int(tau), float(np.float32(eps)), norm_code(norm), int(lmin),
                     int(vmin), int(wmin), int(theiler))


class RQA:
    """One RQA computation (parameter set) bound to librqa's C ABI.

    ``embedding_dimension``/``time_delay``/``radius``/``similarity_measure`` and
    the minimum line lengths follow the Settings fields of Sect. 7.2; ``theiler``
    is the Theiler window."""

    def __init__(self, embedding_dimension, time_delay, radius, similarity_measure="euclidean",
                 min_diagonal_line_length=2, min_vertical_line_length=2,
                 min_white_vertical_line_length=2, theiler=1):
        self.params = make_params(embedding_dimension, time_delay, radius, similarity_measure,
                                  min_diagonal_line_length, min_vertical_line_length,
                                  min_white_vertical_line_length, theiler)
        h = ctypes.c_void_p()
        p = self.params
        check(lib().rqa_create(ctypes.byref(h), p.m, p.tau, p.eps, p.norm, p.lmin, p.vmin, p.wmin,
                               p.theiler), "rqa_create")
        self._h = h
        self._keep = None
        self._count = 0
        self._hlen = []     # histogram entries per job of the last run

    @classmethod
    def from_params(cls, p):
        """From any object with fields m, tau, eps, norm, lmin, vmin, wmin, theiler."""
        return cls(p.m, p.tau, p.eps, p.norm, p.lmin, p.vmin, p.wmin, p.theiler)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rqa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hist_len(self, n_points: int) -> int:
        out = ctypes.c_int64()
        check(lib().rqa_hist_len(self._h, int(n_points), ctypes.byref(out)), "rqa_hist_len")
        return out.value

    def set_profiling(self, enable: bool = True):
        check(lib().rqa_set_profiling(self._h, 1 if enable else 0), "rqa_set_profiling")

    def timings(self) -> dict:
        """Milliseconds of the last profiled run: prepare, tiles, stitch."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().rqa_get_timings(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "rqa_get_timings")
        return {"prepare_ms": a.value, "tiles_ms": b.value, "stitch_ms": c.value}

    def last_launch(self) -> dict:
        """Waves per workgroup of the last run and whether it was a graph replay."""
        w, g = ctypes.c_int32(), ctypes.c_int32()
        check(lib().rqa_last_launch(self._h, ctypes.byref(w), ctypes.byref(g)), "rqa_last_launch")
        return {"waves": w.value, "graph_replay": bool(g.value)}

    def set_tiling(self, waves_per_group: int = 0, groups: int = 0):
        check(lib().rqa_set_tiling(self._h, int(waves_per_group), int(groups)), "rqa_set_tiling")

    def set_workspace_limit(self, nbytes: int = 0):
        """Bound the line summaries of a one-series run to `nbytes` of device
        memory (0: a quarter of the device's memory); a run that would need more
        walks its strips in row bands with the same results."""
        check(lib().rqa_set_workspace_limit(self._h, int(nbytes)), "rqa_set_workspace_limit")

    def last_plan(self) -> dict:
        """How the last run was cut: row bands, strips per band, column
        segments per strip, rows per strip, workspace bytes of its first job."""
        b, k, g, r = (ctypes.c_int32() for _ in range(4))
        w = ctypes.c_int64()
        check(lib().rqa_last_plan(self._h, ctypes.byref(b), ctypes.byref(k), ctypes.byref(g),
                                  ctypes.byref(r), ctypes.byref(w)), "rqa_last_plan")
        return {"bands": b.value, "band_strips": k.value, "segs": g.value, "strip_rows": r.value,
                "workspace_bytes": w.value}

    def run(self, series, stream=None):
        """Enqueue the RQA of a device series (asynchronous)."""
        s = _device_series(series)
        check(lib().rqa_run(self._h, ctypes.c_void_p(s.data_ptr()), s.numel(), _stream_ptr(stream)),
              "rqa_run")
        self._keep = s
        self._count = 1
        self._hlen = [self.hist_len(s.numel())]
        return self

    def result(self, histograms: bool = True, out=None) -> RQAResult:
        """Measures and (with ``histograms``) the three line-length histograms
        of the last run.  ``out``: optional (diag, vert, white) host arrays of
        uint64, C-contiguous, writeable and at least ``hist_len`` long, that
        receive the histograms instead of new arrays (callers that loop reuse
        their buffers; the result then holds views of their first hist_len
        entries)."""
        return self._fetch(None, histograms, out)

    def __call__(self, series, stream=None) -> RQAResult:
        self.run(series, stream)
        return self.result()

    def run_batch(self, series, offsets, lengths, stream=None):
        """Enqueue windows series[offsets[w]:offsets[w]+lengths[w]] in one launch."""
        s = _device_series(series)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        ln = np.ascontiguousarray(lengths, dtype=np.int64)
        if off.shape != ln.shape or off.ndim != 1:
            raise ValueError("offsets and lengths must be 1-D arrays of equal length")
        check(lib().rqa_run_batch(self._h, ctypes.c_void_p(s.data_ptr()), s.numel(),
                                  off.ctypes.data_as(ctypes.c_void_p),
                                  ln.ctypes.data_as(ctypes.c_void_p), len(off),
                                  _stream_ptr(stream)), "rqa_run_batch")
        self._keep = s
        self._count = len(off)
        self._hlen = [int(L) - (self.params.m - 1) * self.params.tau + 1 for L in ln]
        return self

    def run_cross(self, a, b, stream=None):
        """Enqueue the cross recurrence RQA of device series a (rows) and b
        (columns) (asynchronous)."""
        sa, sb = _device_series(a), _device_series(b)
        check(lib().rqa_run_cross(self._h, ctypes.c_void_p(sa.data_ptr()), sa.numel(),
                                  ctypes.c_void_p(sb.data_ptr()), sb.numel(),
                                  _stream_ptr(stream)), "rqa_run_cross")
        out = ctypes.c_int64()
        check(lib().rqa_cross_hist_len(self._h, sa.numel(), sb.numel(), ctypes.byref(out)),
              "rqa_cross_hist_len")
        self._keep = (sa, sb)
        self._count = 1
        self._hlen = [out.value]
        return self

    def cross(self, a, b, stream=None) -> RQAResult:
        self.run_cross(a, b, stream)
        return self.result()

    def run_matrix(self, bits, n_cols: int, stream=None):
        """Enqueue the RQA of a given binary matrix: ``bits`` is a device int64
        tensor of shape (n_rows, words), bit b of word c of row i = cell
        (i, 64c+b) (asynchronous)."""
        B = _device_bits(bits)
        n_rows, words = B.shape
        check(lib().rqa_run_matrix(self._h, ctypes.c_void_p(B.data_ptr()), int(n_rows),
                                   int(n_cols), int(words), _stream_ptr(stream)), "rqa_run_matrix")
        self._keep = B
        self._count = 1
        self._hlen = [max(int(n_rows), int(n_cols)) + 1]
        return self

    def plot(self, series, other=None, words: int | None = None, stream=None):
        """Recurrence plot of a device series (or the cross recurrence plot of
        series and ``other``): a device int64 tensor (rows, words), bit b of word
        c of row i = cell (i, 64c+b).  Enqueued on the stream; the tensor is
        ready once the stream reaches this point."""
        import torch
        s = _device_series(series)
        d = (self.params.m - 1) * self.params.tau
        n = s.numel() - d
        nb = n if other is None else other.numel() - d
        if n < 1 or nb < 1:
            raise RQAError(-2, "plot: series too short for the embedding")
        words = (nb + 63) // 64 if words is None else int(words)
        out = torch.empty((n, words), dtype=torch.int64, device=s.device)
        if other is None:
            rc = lib().rqa_plot(self._h, ctypes.c_void_p(s.data_ptr()), s.numel(),
                                ctypes.c_void_p(out.data_ptr()), words, _stream_ptr(stream))
        else:
            o = _device_series(other)
            rc = lib().rqa_plot_cross(self._h, ctypes.c_void_p(s.data_ptr()), s.numel(),
                                      ctypes.c_void_p(o.data_ptr()), o.numel(),
                                      ctypes.c_void_p(out.data_ptr()), words, _stream_ptr(stream))
        check(rc, "rqa_plot")
        return out

    def matrix(self, bits, n_cols: int, stream=None) -> RQAResult:
        self.run_matrix(bits, n_cols, stream)
        return self.result()

    def result_batch(self, index: int, histograms: bool = True, out=None) -> RQAResult:
        """One window of the last batch; ``out`` as for :meth:`result`."""
        return self._fetch(int(index), histograms, out)

    def results_batch(self):
        """Measures of every window of the last run in one library call: a numpy
        structured array (fields as rqa_measures) and the per-window status codes
        (0 = OK; a window without a result has NaN measures)."""
        count = len(self._hlen) if self._hlen else 0
        if count < 1:
            raise RuntimeError("rqa_result_batch_all: no run")
        out = (RqaMeasures * count)()
        status = np.zeros(count, dtype=np.int32)
        rc = lib().rqa_result_batch_all(self._h, ctypes.cast(out, ctypes.c_void_p),
                                        status.ctypes.data_as(ctypes.c_void_p), count)
        # A window's own failure is in its status; only errors of the call
        # itself raise (no run, count mismatch, bad arguments).
        if rc in (RQA_EINVAL, RQA_ESTATE, RQA_ESIZE):
            check(rc, "rqa_result_batch_all")
        return np.ctypeslib.as_array(out).copy(), status

    def _fetch(self, index, histograms, out=None):
        hl = self._hlen[0 if index is None else index] if self._hlen else 0
        ms = RqaMeasures()
        if histograms and hl > 1:
            if out is None:
                # filled completely by the library
                d, v, w = (np.empty(hl, dtype=np.uint64) for _ in range(3))
            else:
                if len(out) != 3:
                    raise ValueError("out must hold three arrays (diag, vert, white)")
                for a in out:
                    if (not isinstance(a, np.ndarray) or a.dtype != np.uint64 or a.ndim != 1
                            or not a.flags.c_contiguous or not a.flags.writeable or a.size < hl):
                        raise ValueError(f"each out array must be a writeable, C-contiguous 1-D "
                                         f"uint64 array of at least {hl} entries")
                d, v, w = (a[:hl] for a in out)
            ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in (d, v, w)]
        else:
            d = v = w = None
            ptrs = [None, None, None]
        if index is None:
            rc = lib().rqa_result(self._h, ctypes.byref(ms), *ptrs, hl)
            check(rc, "rqa_result")
        else:
            rc = lib().rqa_result_batch(self._h, index, ctypes.byref(ms), *ptrs, hl)
            check(rc, "rqa_result_batch")
        return RQAResult(_measures_dict(ms), d, v, w, int(ms.n_vec), int(ms.n_rec))


def measures_from_hist(diag, vert, white, params) -> dict:
    """FP64 measures from host histograms through the library's own code."""
    d = np.ascontiguousarray(diag, dtype=np.uint64)
    v = np.ascontiguousarray(vert, dtype=np.uint64)
    w = np.ascontiguousarray(white, dtype=np.uint64)
    p = params if isinstance(params, RqaParams) else make_params(
        params.m, params.tau, params.eps, params.norm, params.lmin, params.vmin, params.wmin,
        params.theiler)
    ms = RqaMeasures()
    check(lib().rqa_measures_from_hist(d.ctypes.data_as(ctypes.c_void_p),
                                       v.ctypes.data_as(ctypes.c_void_p),
                                       w.ctypes.data_as(ctypes.c_void_p), len(d) - 1,
                                       ctypes.byref(p), ctypes.byref(ms)), "rqa_measures_from_hist")
    return _measures_dict(ms)


def workspace_plan(params, n_points: int, waves: int = 0, limit_bytes: int = 0) -> dict:
    """How a run of one series of n_points would be cut (host only): row bands,
    strips per band, column segments per strip and the line-summary workspace,
    for `waves` waves per workgroup (0: default) and a bound of limit_bytes
    (0: none)."""
    p = params if isinstance(params, RqaParams) else make_params(
        params.m, params.tau, params.eps, params.norm, params.lmin, params.vmin, params.wmin,
        params.theiler)
    b, k, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    w = ctypes.c_int64()
    check(lib().rqa_workspace_plan(ctypes.byref(p), int(n_points), int(waves), int(limit_bytes),
                                   ctypes.byref(b), ctypes.byref(k), ctypes.byref(g),
                                   ctypes.byref(w)), "rqa_workspace_plan")
    return {"bands": b.value, "band_strips": k.value, "segs": g.value, "workspace_bytes": w.value}


class Server:
    """Continuous-batching RQA server over librqa's serving API."""

    def __init__(self, budget_bytes: int, streams: int = 4):
        h = ctypes.c_void_p()
        check(lib().rqa_server_create(ctypes.byref(h), int(budget_bytes), int(streams)),
              "rqa_server_create")
        self._h = h
        self._jobs = {}

    @staticmethod
    def footprint(params, n_points: int) -> int:
        p = params if isinstance(params, RqaParams) else make_params(
            params.m, params.tau, params.eps, params.norm, params.lmin, params.vmin, params.wmin,
            params.theiler)
        out = ctypes.c_size_t()
        check(lib().rqa_job_footprint(ctypes.byref(p), int(n_points), ctypes.byref(out)),
              "rqa_job_footprint")
        return out.value

    def submit(self, params, series, stream=None) -> int:
        s = _device_series(series)
        p = params if isinstance(params, RqaParams) else make_params(
            params.m, params.tau, params.eps, params.norm, params.lmin, params.vmin, params.wmin,
            params.theiler)
        t = ctypes.c_uint64()
        check(lib().rqa_submit(self._h, ctypes.byref(p), ctypes.c_void_p(s.data_ptr()), s.numel(),
                               _stream_ptr(stream), ctypes.byref(t)), "rqa_submit")
        self._jobs[t.value] = (s, s.numel() - (p.m - 1) * p.tau)
        return t.value

    def _collect(self, fn, ticket, histograms):
        if ticket not in self._jobs:
            raise KeyError(ticket)
        n = self._jobs[ticket][1]
        ms = RqaMeasures()
        if histograms:
            arrs = [np.zeros(n + 1, dtype=np.uint64) for _ in range(3)]
            ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        else:
            arrs = [None] * 3
            ptrs = [None] * 3
        rc = fn(self._h, ctypes.c_uint64(ticket), ctypes.byref(ms), *ptrs, n + 1)
        if rc == EAGAIN:
            return None
        del self._jobs[ticket]
        check(rc, "rqa_poll/wait")
        return RQAResult(_measures_dict(ms), *arrs, int(ms.n_vec), int(ms.n_rec))

    def poll(self, ticket: int, histograms: bool = True):
        """Result if the job is done, else None."""
        return self._collect(lib().rqa_poll, ticket, histograms)

    def wait(self, ticket: int, histograms: bool = True) -> RQAResult:
        return self._collect(lib().rqa_wait, ticket, histograms)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rqa_server_destroy(self._h)
            self._h = None
        self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["RQA", "RQAResult", "RQAError", "Server", "measures_from_hist", "make_params",
           "norm_code"]
