"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/rqa.h, and host-side validation returns the documented
error codes without touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2402_16853_amd._lib import LIB_PATH, SIGNATURES, RqaMeasures, RqaParams, lib

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(REPO, "include")
    for f in os.listdir(inc):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(rqa_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = names - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"
    assert names <= set(SIGNATURES), f"binding lacks: {sorted(names - set(SIGNATURES))}"


def test_no_torch_in_the_abi():
    text = open(os.path.join(REPO, "include", "rqa.h")).read()
    assert "torch" not in text.lower().replace("pytorch cuda tensor", "")
    assert "extern \"C\"" in text


def create(m=2, tau=1, eps=0.1, norm=2, lmin=2, vmin=2, wmin=2, theiler=1):
    h = ctypes.c_void_p()
    rc = lib().rqa_create(ctypes.byref(h), m, tau, eps, norm, lmin, vmin, wmin, theiler)
    return rc, h


@pytest.mark.parametrize("args", [
    dict(m=0), dict(tau=0), dict(eps=-0.5), dict(eps=float("nan")), dict(eps=float("inf")),
    dict(norm=0), dict(norm=4), dict(lmin=0), dict(vmin=0), dict(wmin=0), dict(theiler=-1),
])
def test_create_rejects_invalid(args):
    rc, h = create(**args)
    assert rc == -1 and not h.value


def test_handle_lifecycle_and_host_errors():
    L = lib()
    rc, h = create(m=3, tau=2)
    assert rc == 0 and h.value
    n = ctypes.c_int64()
    assert L.rqa_hist_len(h, 100, ctypes.byref(n)) == 0 and n.value == 100 - 4 + 1
    assert L.rqa_hist_len(h, 4, ctypes.byref(n)) == -2          # too short
    ms = RqaMeasures()
    assert L.rqa_result(h, ctypes.byref(ms), None, None, None, 0) == -7   # no run yet
    assert L.rqa_run(h, None, 100, None) == -1                   # null series
    assert L.rqa_run_batch(h, None, 100, None, None, 0, None) == -1
    many = (RqaMeasures * 4)()
    assert L.rqa_result_batch_all(h, ctypes.cast(many, ctypes.c_void_p), None, 4) == -7  # no run
    assert L.rqa_result_batch_all(h, None, None, 4) == -1
    assert L.rqa_result_batch_all(None, ctypes.cast(many, ctypes.c_void_p), None, 4) == -1
    assert L.rqa_set_tiling(h, 9, 0) == -1
    assert L.rqa_set_tiling(h, 4, 0) == 0
    assert L.rqa_set_workspace_limit(h, -1) == -1
    assert L.rqa_set_workspace_limit(None, 1 << 30) == -1
    assert L.rqa_set_workspace_limit(h, 1 << 30) == 0
    assert L.rqa_set_workspace_limit(h, 0) == 0
    b = ctypes.c_int32()
    assert L.rqa_last_plan(h, ctypes.byref(b), None, None, None, None) == -7   # no run yet
    assert L.rqa_last_plan(None, ctypes.byref(b), None, None, None, None) == -1
    L.rqa_destroy(h)
    L.rqa_destroy(None)


def test_strerror_covers_codes():
    L = lib()
    seen = set()
    for code in range(0, -11, -1):
        msg = L.rqa_strerror(code).decode()
        assert msg and msg != "unknown error"
        seen.add(msg)
    assert len(seen) == 11
    assert L.rqa_strerror(-99).decode() == "unknown error"


def test_footprint_and_measure_validation():
    L = lib()
    p = RqaParams(3, 10, 0.5, 3, 2, 2, 2, 1)
    out = ctypes.c_size_t()
    assert L.rqa_job_footprint(ctypes.byref(p), 1_048_576, ctypes.byref(out)) == 0
    n = 1_048_576 - 20
    assert out.value >= 3 * 8 * (n + 1)
    assert L.rqa_job_footprint(ctypes.byref(p), 10, ctypes.byref(out)) == -2
    bad = RqaParams(3, 10, -1.0, 3, 2, 2, 2, 1)
    assert L.rqa_job_footprint(ctypes.byref(bad), 1000, ctypes.byref(out)) == -1
    z = np.zeros(5, dtype=np.uint64)
    ms = RqaMeasures()
    assert L.rqa_measures_from_hist(None, None, None, 4, ctypes.byref(p), ctypes.byref(ms)) == -1
    zp = z.ctypes.data_as(ctypes.c_void_p)
    assert L.rqa_measures_from_hist(zp, zp, zp, 0, ctypes.byref(p), ctypes.byref(ms)) == -1
    assert L.rqa_measures_from_hist(zp, zp, zp, 4, ctypes.byref(bad), ctypes.byref(ms)) == -1


def test_server_argument_checks():
    L = lib()
    srv = ctypes.c_void_p()
    assert L.rqa_server_create(ctypes.byref(srv), 100, 4) == -1     # budget too small
    assert L.rqa_server_create(ctypes.byref(srv), 1 << 20, 0) == -1  # no streams
    assert L.rqa_server_create(None, 1 << 20, 4) == -1
    t = ctypes.c_uint64()
    p = RqaParams(2, 1, 0.1, 2, 2, 2, 2, 1)
    assert L.rqa_submit(None, ctypes.byref(p), None, 10, None, ctypes.byref(t)) == -1
    assert L.rqa_poll(None, 1, None, None, None, None, 0) == -1
    assert L.rqa_wait(None, 1, None, None, None, None, 0) == -1
    L.rqa_server_destroy(None)


def test_python_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_2402_16853_amd import RQA
    comp = RQA(2, 1, 0.1, "euclidean")
    with pytest.raises(ValueError):
        comp.run(torch.zeros(100, dtype=torch.float32))          # CPU tensor: no fallback
    with pytest.raises(TypeError):
        comp.run(np.zeros(100, dtype=np.float32))
    comp.close()


def test_run_static_host_errors():
    """rqa_run_static rejects bad arguments and series beyond its static scratch
    on the host, before any HIP call (fake device pointers are never touched)."""
    L = lib()
    fake = ctypes.c_void_p(0x1000)
    p = RqaParams(3, 2, 0.1, 2, 2, 2, 2, 1)
    assert L.rqa_run_static(None, fake, 1000, fake, 1000, fake, None) == -1
    assert L.rqa_run_static(ctypes.byref(p), None, 1000, fake, 1000, fake, None) == -1
    assert L.rqa_run_static(ctypes.byref(p), fake, 1000, None, 1000, fake, None) == -1
    assert L.rqa_run_static(ctypes.byref(p), fake, 1000, fake, 1000, None, None) == -1
    assert L.rqa_run_static(ctypes.byref(RqaParams(0, 2, 0.1, 2, 2, 2, 2, 1)), fake, 1000, fake,
                            1000, fake, None) == -1
    assert L.rqa_run_static(ctypes.byref(p), fake, 4, fake, 10, fake, None) == -2
    assert L.rqa_run_static(ctypes.byref(p), fake, 1000, fake, 996, fake, None) == -6
    assert L.rqa_run_static(ctypes.byref(p), fake, 300_000, fake, 300_000, fake, None) == -8
    assert b"static scratch" in L.rqa_strerror(-8)
