"""The C-ABI library loads on the CPU and exports every entry point that
include/pcba.h declares (no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcba.h")
LIB = os.path.join(ROOT, "paper_2003_01758_amd", "libpcba.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pcba_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pcba_create_problem", "pcba_solve", "pcba_result", "pcba_destroy_problem",
                     "pcba_solve_batch", "pcba_engine_submit", "pcba_engine_run",
                     "pcba_engine_poll", "pcba_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_and_argument_validation_without_device():
    from paper_2003_01758_amd import pcba
    o = pcba.default_options()
    assert o.eps == 1e-3 and o.delta == 1e-4 and o.max_iters == 28 and o.max_boxes == 1 << 20
    # the C side fills every field: a layout mismatch would misplace these
    assert o.rederive_every == 16 and o.stale_filter == 0 and o.retire_satisfied == 1
    assert o.time_limit_s == 0.0 and o.tile_coefs == 0 and o.wg_per_cu == 0 and ctypes.sizeof(o) == 96
    assert o.direction_rule == 0 and o.subdiv_lambda == 0.5 and o.split_engine == pcba.SPLIT_VALU
    assert o.persistent_steps == 0
    # argument errors are detected before any device call
    L = pcba.lib()
    assert L.pcba_set_cut_split(-1, 4096) == pcba.E_ARG and L.pcba_set_cut_split(1024, 32) == pcba.E_ARG
    h = ctypes.c_void_p()
    rc = L.pcba_create_problem(0, None, None, None, None, 0, None, None, 0, None, None, None,
                               ctypes.byref(h))
    assert rc == pcba.E_ARG and b"l outside" in L.pcba_last_error()
    import numpy as np
    lo = np.array([0.0, 1.0])
    hi = np.array([1.0, 1.0])   # lo >= hi on axis 1
    deg = np.array([1, 1], dtype=np.int32)
    coef = np.ones(4)
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               0, None, None, 0, None, None, None, ctypes.byref(h))
    assert rc == pcba.E_ARG
    hi = np.array([1.0, 2.0])
    coef[2] = np.nan
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               0, None, None, 0, None, None, None, ctypes.byref(h))
    assert rc == pcba.E_ARG
    bad = pcba.default_options(eps=0.0)
    coef[2] = 1.0
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               0, None, None, 0, None, None, ctypes.byref(bad), ctypes.byref(h))
    assert rc == pcba.E_ARG
    bad = pcba.default_options(retire_satisfied=2)
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               0, None, None, 0, None, None, ctypes.byref(bad), ctypes.byref(h))
    assert rc == pcba.E_ARG and b"retire_satisfied" in L.pcba_last_error()
    # a round (fused_round = 1) splits every axis: l <= 2, and no retiring
    assert pcba.default_options().fused_round == 0
    bad = pcba.default_options(fused_round=1)   # retire_satisfied stays 1
    g1 = np.ones(4)
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               1, deg.ctypes.data, g1.ctypes.data, 0, None, None, ctypes.byref(bad),
                               ctypes.byref(h))
    assert rc == pcba.E_ARG and b"fused_round" in L.pcba_last_error()
    bad = pcba.default_options(fused_round=1, retire_satisfied=0)
    lo3, hi3, deg3 = np.zeros(3), np.ones(3), np.array([1, 1, 1], dtype=np.int32)
    rc = L.pcba_create_problem(3, lo3.ctypes.data, hi3.ctypes.data, deg3.ctypes.data, np.ones(8).ctypes.data,
                               0, None, None, 0, None, None, ctypes.byref(bad), ctypes.byref(h))
    assert rc == pcba.E_ARG and b"l <= 2" in L.pcba_last_error()
    # launch-shape knobs: tile size in range, workgroup count not negative
    for kw in (dict(tile_coefs=100), dict(tile_coefs=4096), dict(wg_per_cu=-1),
               dict(tile_coefs=2048, fused_round=1, retire_satisfied=0),
               # subdivision variants: rule 0 or 1, lambda inside (0,1), not with
               # rounds, and FP32 away from the midpoint without re-derivation; split
               # engine 0 (vector ALUs) or 1 (matrix cores)
               dict(direction_rule=2), dict(subdiv_lambda=0.0), dict(subdiv_lambda=1.0), dict(split_engine=2), dict(persistent_steps=2),
               dict(fused_round=1, retire_satisfied=0, direction_rule=1),
               dict(fused_round=1, retire_satisfied=0, subdiv_lambda=0.25),
               dict(precision=1, subdiv_lambda=0.25)):
        bad = pcba.default_options(**kw)
        rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                                   0, None, None, 0, None, None, ctypes.byref(bad), ctypes.byref(h))
        assert rc == pcba.E_ARG, kw
    bad = pcba.default_options(fused_round=2, retire_satisfied=0)
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg.ctypes.data, coef.ctypes.data,
                               0, None, None, 0, None, None, ctypes.byref(bad), ctypes.byref(h))
    assert rc == pcba.E_ARG
    deg16 = np.array([16, 1], dtype=np.int32)
    rc = L.pcba_create_problem(2, lo.ctypes.data, hi.ctypes.data, deg16.ctypes.data,
                               np.ones(34).ctypes.data, 0, None, None, 0, None, None, None,
                               ctypes.byref(h))
    assert rc == pcba.E_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_result_batch_argument_checks_without_device():
    from paper_2003_01758_amd import pcba
    L = pcba.lib()
    out = (pcba.Result * 2)()
    assert L.pcba_result_batch(None, 2, ctypes.addressof(out)) == pcba.E_ARG
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.pcba_result_batch(arr, 2, ctypes.addressof(out)) == pcba.E_ARG
    assert L.pcba_result_batch(arr, -1, ctypes.addressof(out)) == pcba.E_ARG
    assert L.pcba_result_batch(arr, 0, None) == 0
    # the record layout the binding's structured array uses is the C one
    assert pcba.RESULT_DTYPE.itemsize == ctypes.sizeof(pcba.Result)
