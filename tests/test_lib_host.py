"""Host-side checks of libbpdc.so (no GPU needed): the library loads, exports
every entry point of include/bpdc.h, validates its inputs before touching a
device, and generates / compiles the code-specialised lane kernel."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2510_08695_amd as P
    if not os.path.exists(P.lib_path()):
        pytest.fail("libbpdc.so is not built (run __graft_entry__.build())")
    return P


def header_functions():
    text = open(os.path.join(ROOT, "include", "bpdc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:bpdc_status|const char\*)\s+(bpdc_\w+)\s*\(", text, re.M)))


def test_exports_every_header_symbol(P):
    L = P.lib()
    names = header_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) <= set(P._lib.EXPORTS) | {"bpdc_status_string", "bpdc_last_error", "bpdc_version"}


def test_version_and_status_strings(P):
    L = P.lib()
    assert b"gfx950" in L.bpdc_version()
    for s in range(6):
        assert L.bpdc_status_string(s)


def _csr_struct(P, rows, cols, rp, ci):
    rp = np.asarray(rp, np.int32)
    ci = np.asarray(ci if len(ci) else [0], np.int32)
    s = P._lib._Csr(rows, cols, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                    ci.ctypes.data_as(C.POINTER(C.c_int32)))
    return s, (rp, ci)


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "out_of_range", "prior_zero", "prior_one",
                                 "cols_mismatch", "bad_rowptr"])
def test_code_create_rejects_invalid_input(P, bad):
    L = P.lib()
    rp, ci, cols = [0, 2, 4], [0, 1, 1, 2], 3
    pri = np.full(3, 0.1)
    drp, dci, dcols = [0, 2], [0, 2], 3
    if bad == "unsorted":
        ci = [1, 0, 1, 2]
    elif bad == "duplicate":
        ci = [0, 0, 1, 2]
    elif bad == "out_of_range":
        ci = [0, 1, 1, 3]
    elif bad == "prior_zero":
        pri[1] = 0.0
    elif bad == "prior_one":
        pri[2] = 1.0
    elif bad == "cols_mismatch":
        dcols = 4
    elif bad == "bad_rowptr":
        rp = [0, 3, 2]
    H, k1 = _csr_struct(P, 2, cols, rp, ci)
    D, k2 = _csr_struct(P, 1, dcols, drp, dci)
    out = C.c_void_p()
    st = L.bpdc_code_create(C.byref(H), C.byref(D), pri.ctypes.data_as(C.c_void_p), C.byref(out))
    assert st == 1, (st, L.bpdc_last_error())
    assert not out.value
    assert L.bpdc_last_error()


def test_null_arguments_are_rejected(P):
    L = P.lib()
    assert L.bpdc_code_create(None, None, None, None) == 1
    assert L.bpdc_plan_create(None, 0, None, 0, None) == 1
    assert L.bpdc_decode(None, 0, None, 0, 0, None, None, None, None, None, None, 0, None) == 1
    assert L.bpdc_code_destroy(None) == 0 and L.bpdc_plan_destroy(None) == 0


def test_lane_kernel_generation_and_compilation(P, tmp_path, monkeypatch):
    monkeypatch.setenv("BPDC_CACHE_DIR", str(tmp_path))
    c = synth.toric_code(4)
    P.lane_precompile(c.H, c.D, posterior=True)
    files = list(tmp_path.iterdir())
    # every tile the plan autotuner may time: the toric code's translations give lane
    # groups of 4, 2 and 1 lanes per shot, each with claims of 8, 16 and 32 shots
    assert len(files) == 9 and all(f.stat().st_size > 1000 for f in files)
    # compiling again finds them all in the cache
    P.lane_precompile(c.H, c.D, posterior=True)
    assert len(list(tmp_path.iterdir())) == 9
    monkeypatch.setenv("BPDC_LANE_CHUNK", "16")
    monkeypatch.setenv("BPDC_LANE_MAX_LANES", "2")
    P.lane_precompile(c.H, c.D, posterior=True)
    assert len(list(tmp_path.iterdir())) == 9    # (2 lanes, 16) and (1 lane, 16) were cached already
    # a code too large for one lane per shot is refused, not compiled
    big = synth.hgp_code(synth.random_regular_classical(16, 4001), with_logicals=False)
    with pytest.raises(P.BpdcError, match="unsupported"):
        P.lane_precompile(big.H, big.D)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; --gpus 2 exits with a message (before any GPU call)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
