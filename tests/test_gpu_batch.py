"""The 256-instance mixed batch through the C ABI, at full size.

All 256 instances (2 or 3 variables, constraint degree 4 to 10, 50 to 1000
constraints, up to about 1.2 million words per item) run as one batch, in FP64
plain mode and in FP32 mode.  The instances the oracle solves in seconds have
stored oracle results (tests/golden/c3_oracle.json, written by a script that
calls only the oracle): FP64 plain must reproduce them exactly and FP32 must
land within eps.  Every instance, stored or not, is checked for what holds at
any size: the bracket, the stopping width, the returned box's feasibility at
its centre, FP64 certification of the FP32 answer, and agreement of the two
precisions within eps."""
import json
import os
import time

import numpy as np
import pytest

from paper_2003_01758_amd.instances import make_instance, poly_eval

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BATCH = 256


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


@pytest.fixture(scope="module")
def insts():
    return [make_instance(3, k) for k in range(BATCH)]


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "c3_oracle.json")) as f:
        return {int(k): v for k, v in json.load(f)["results"].items()}


def _solve(gpu, insts, precision):
    t0 = time.perf_counter()
    probs = [gpu.Problem(i, precision=precision) for i in insts]
    print(f"[c3] {precision}: {len(probs)} problems created in {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    batch = gpu.Batch(probs)
    res = gpu.solve_batch(batch)
    # the one-call result array (pcba_result_batch) holds the same records
    arr = gpu.results(batch)
    for r, a in zip(res, arr):
        for k in ("outcome", "has_x", "p_up", "p_lo", "steps", "rounds", "list_len", "peak_len",
                  "certified", "p_cert", "seconds", "capacity"):
            assert r[k] == a[k] or (np.isnan(r[k]) and np.isnan(a[k])), k
        l = len(r["x_lo"])
        assert np.array_equal(r["x_lo"], a["x_lo"][:l]) and np.array_equal(r["x_index"], a["x_index"][:l])
    for p in probs:
        p.close()
    print(f"[c3] {precision}: solved in {time.perf_counter() - t0:.1f} s", flush=True)
    return res


@pytest.fixture(scope="module")
def res64(gpu, insts):
    return _solve(gpu, insts, "fp64")


@pytest.fixture(scope="module")
def res32(gpu, insts):
    return _solve(gpu, insts, "fp32")


def _check_any_size(inst, r, gpu):
    assert r["outcome"] in (gpu.OPTIMAL, gpu.INFEASIBLE), r["outcome"]
    if r["outcome"] != gpu.OPTIMAL:
        return
    assert r["p_lo"] <= r["p_up"]
    assert r["p_up"] - r["p_lo"] <= inst.eps
    assert np.max(r["x_hi"] - r["x_lo"]) <= inst.delta
    c = 0.5 * (r["x_lo"] + r["x_hi"])
    assert max(poly_eval(g, c) for g in inst.ineq) <= 1e-6
    assert r["p_lo"] - 1e-9 <= poly_eval(inst.cost, c) <= r["p_up"] + 1e-9


def test_fp64_batch_matches_oracle(gpu, insts, golden, res64):
    assert len(golden) >= 100
    for k, want in golden.items():
        r = res64[k]
        assert r["outcome"] == want["outcome"], k
        assert r["p_up"] == want["p_up"] and r["p_lo"] == want["p_lo"], k
        assert r["steps"] == want["steps"] and r["peak_len"] == want["peak_len"], k
        if r["outcome"] == gpu.OPTIMAL:
            assert list(r["x_index"]) == want["x_index"], k
    for k, (inst, r) in enumerate(zip(insts, res64)):
        _check_any_size(inst, r, gpu)


def test_fp32_batch_within_eps_and_certified(gpu, insts, golden, res32, res64):
    for k, want in golden.items():
        r = res32[k]
        assert r["outcome"] == want["outcome"], k
        if r["outcome"] == gpu.OPTIMAL:
            assert abs(r["p_up"] - want["p_up"]) <= insts[k].eps, k
    for k, (inst, r, r64) in enumerate(zip(insts, res32, res64)):
        _check_any_size(inst, r, gpu)
        assert r["outcome"] == r64["outcome"], k
        if r["outcome"] == gpu.OPTIMAL:
            assert r["certified"], k
            assert r["p_cert"] <= r["p_up"] + 1e-9, k
            assert abs(r["p_up"] - r64["p_up"]) <= inst.eps, k
