"""The benchmark script's host-side contract (no GPU): more than one GPU is
refused with a message, the counter-calibration entry exists, and the
algorithmic byte count follows the definition (every carried patch of every
parent read once, every carried patch of every kept child written once)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_copy_calibration_entry_exists():
    assert callable(bench.copy_calibration)


class _Opts:
    rederive_every = 0


class _Fake:
    options = _Opts()

    def trace(self):
        return {"k_in": np.array([1, 2]), "k_kept": np.array([2, 3])}

    def trace_patches(self):
        return {"a_in": np.array([5, 7]), "a_kept": np.array([7, 4])}


class _Inst:
    cost = np.zeros((3, 3))
    ineq_deg = np.array([[2, 2], [2, 2]])
    eq_deg = np.zeros((0, 2), dtype=int)
    n_eq = 0


def test_algorithmic_bytes_follow_the_definition():
    # cost 9 coefficients, inequality patches 9 coefficients, FP64
    got = bench.algorithmic_bytes(_Fake(), _Inst(), "fp64")
    items = (1 + 2) + (2 + 3)
    ineq = (5 + 7) + (7 + 4)
    assert got == 8 * (9 * items + 9 * ineq)
    # FP32: half the coefficient bytes plus one 4-byte error bound per patch
    got32 = bench.algorithmic_bytes(_Fake(), _Inst(), "fp32")
    assert got32 == 4 * (9 * items + 9 * ineq) + 4 * (items + ineq)


def test_count_certified_over_the_result_array():
    # the timed loop counts certified plans on the structured array of
    # pcba_result_batch; it must agree with certified() record by record
    from paper_2003_01758_amd import pcba
    res = np.zeros(6, dtype=pcba.RESULT_DTYPE)
    res["outcome"] = [pcba.OPTIMAL, pcba.OPTIMAL, pcba.INFEASIBLE, pcba.MAX_ITER, pcba.MEMORY_LIMIT,
                      pcba.OPTIMAL]
    res["certified"] = [1, 0, 0, 0, 1, 1]
    # INFEASIBLE counts only where bounds are rigorously widened (FP32)
    for precision, want in (("fp64", 2), ("fp32", 3)):
        assert bench.count_certified(res, pcba, precision) == \
            sum(1 for r in res if bench.certified(r, pcba, precision)) == want
