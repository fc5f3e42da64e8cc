"""ctypes declarations of librqa.so (argument marshalling only).

The library is built in-tree by ``paper_2402_16853_amd.build`` (or
``__graft_entry__.build()``); importing this module never compiles anything and
fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librqa.so")

RQA_OK = 0
ERRORS = {
    -1: "RQA_EINVAL", -2: "RQA_ETOOSHORT", -3: "RQA_ENOMEM", -4: "RQA_EDEVICE",
    -5: "RQA_ENONFINITE", -6: "RQA_ESIZE", -7: "RQA_ESTATE", -8: "RQA_EBUDGET",
    -9: "RQA_EAGAIN", -10: "RQA_ENOTFOUND",
}
EAGAIN = -9
ENONFINITE = -5
RQA_EINVAL = -1
RQA_ESIZE = -6
RQA_ESTATE = -7


class RqaParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("tau", ctypes.c_int32), ("eps", ctypes.c_float),
                ("norm", ctypes.c_int32), ("lmin", ctypes.c_int32), ("vmin", ctypes.c_int32),
                ("wmin", ctypes.c_int32), ("theiler", ctypes.c_int32)]


class RqaMeasures(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in
                ("rr", "det", "l", "lmax", "div", "l_entr", "lam", "tt", "vmax", "v_entr",
                 "w", "wmax", "w_entr")] + [("n_rec", ctypes.c_uint64), ("n_vec", ctypes.c_int64)]


# Every symbol declared in include/rqa.h with its ctypes signature.
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = {
    "rqa_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _I32, ctypes.c_float, _I32, _I32, _I32,
                                  _I32, _I32]),
    "rqa_hist_len": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_I64)]),
    "rqa_run": (ctypes.c_int, [_P, _P, _I64, _P]),
    "rqa_result": (ctypes.c_int, [_P, ctypes.POINTER(RqaMeasures), _P, _P, _P, _I64]),
    "rqa_run_batch": (ctypes.c_int, [_P, _P, _I64, _P, _P, _I32, _P]),
    "rqa_run_cross": (ctypes.c_int, [_P, _P, _I64, _P, _I64, _P]),
    "rqa_cross_hist_len": (ctypes.c_int, [_P, _I64, _I64, ctypes.POINTER(_I64)]),
    "rqa_run_matrix": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _P]),
    "rqa_plot": (ctypes.c_int, [_P, _P, _I64, _P, _I64, _P]),
    "rqa_plot_cross": (ctypes.c_int, [_P, _P, _I64, _P, _I64, _P, _I64, _P]),
    "rqa_result_batch": (ctypes.c_int, [_P, _I32, ctypes.POINTER(RqaMeasures), _P, _P, _P, _I64]),
    "rqa_result_batch_all": (ctypes.c_int, [_P, _P, _P, _I32]),
    "rqa_measures_from_hist": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.POINTER(RqaParams),
                                              ctypes.POINTER(RqaMeasures)]),
    "rqa_set_tiling": (ctypes.c_int, [_P, _I32, _I32]),
    "rqa_set_profiling": (ctypes.c_int, [_P, _I32]),
    "rqa_get_timings": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "rqa_last_launch": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "rqa_destroy": (None, [_P]),
    "rqa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "rqa_server_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, _I32]),
    "rqa_job_footprint": (ctypes.c_int, [ctypes.POINTER(RqaParams), _I64,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "rqa_submit": (ctypes.c_int, [_P, ctypes.POINTER(RqaParams), _P, _I64, _P,
                                  ctypes.POINTER(ctypes.c_uint64)]),
    "rqa_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(RqaMeasures), _P, _P, _P,
                                _I64]),
    "rqa_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(RqaMeasures), _P, _P, _P,
                                _I64]),
    "rqa_server_destroy": (None, [_P]),
    "rqa_run_static": (ctypes.c_int, [ctypes.POINTER(RqaParams), _P, _I64, _P, _I64, _P, _P]),
    "rqa_set_workspace_limit": (ctypes.c_int, [_P, _I64]),
    "rqa_workspace_plan": (ctypes.c_int, [ctypes.POINTER(RqaParams), _I64, _I32, _I64,
                                          ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                          ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "rqa_last_plan": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_I64)]),
}

_lib = None


class RQAError(RuntimeError):
    """Raised for a negative return code of librqa."""

    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = lib().rqa_strerror(code).decode()
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})" if where else msg)


def lib():
    """Load librqa.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"librqa.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2402_16853_amd.build` (HIP, gfx950)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(code: int, where: str = "") -> int:
    if code < 0:
        raise RQAError(code, where)
    return code
