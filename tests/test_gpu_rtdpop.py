"""RTD planning problems (obstacle points through the FRS-like polynomial,
waypoint cost; Sec. II-C, Sec. VI) on the GPU against the FP64 oracle,
including plans that are infeasible: the outcome the oracle reaches, FP64
step traces identical, FP32 within eps and certified."""
import numpy as np
import pytest

from oracle import ref
from paper_2003_01758_amd import instances as I
from paper_2003_01758_amd.instances import Instance, make_instance, poly_eval

pytestmark = pytest.mark.gpu

# instances the oracle solves in well under a second; 3, 18, 19 and 21 are infeasible
FAST = [0, 2, 3, 4, 5, 9, 10, 11, 12, 15, 17, 18, 19, 20, 21, 23, 24, 25]


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


@pytest.fixture(scope="module")
def oracle_results():
    out = {}
    for k in FAST:
        o = ref.RefSolver(make_instance(6, k))
        o.solve()
        out[k] = o.result()
    return out


@pytest.mark.parametrize("k", [0, 3, 9])
def test_fp64_step_trace_matches_oracle(gpu, k):
    inst = make_instance(6, k)
    print(f"[rtdpop fp64 trace] {k}", flush=True)
    g = gpu.Problem(inst)
    o = ref.RefSolver(inst)
    for step in range(100):
        so = o.step()
        rg = g.step(1)
        ro = o.result()
        assert rg["outcome"] == so, step
        assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"], step
        gi, _ = g.list()
        oi, _ = o.list()
        assert np.array_equal(gi, oi), step
        if so != ref.RUNNING:
            break


def test_batch_matches_oracle_both_precisions(gpu, oracle_results):
    insts = [make_instance(6, k) for k in FAST]
    print(f"[rtdpop batch] {len(insts)} plans", flush=True)
    r64 = gpu.solve_batch([gpu.Problem(i) for i in insts])
    r32 = gpu.solve_batch([gpu.Problem(i, precision="fp32") for i in insts])
    n_inf = 0
    for k, inst, a, b in zip(FAST, insts, r64, r32):
        o = oracle_results[k]
        assert a["outcome"] == b["outcome"] == o["outcome"], k
        if o["outcome"] == ref.INFEASIBLE:
            n_inf += 1
            continue
        assert a["p_up"] == o["p_up"] and a["p_lo"] == o["p_lo"] and a["steps"] == o["steps"], k
        assert a["certified"] and b["certified"], k
        assert abs(b["p_up"] - o["p_up"]) <= inst.eps, k
        c = 0.5 * (b["x_lo"] + b["x_hi"])
        assert max(poly_eval(g, c) for g in inst.ineq) <= 1e-6, k
    assert n_inf == 4


@pytest.mark.parametrize("k", [0, 9])
def test_round_mode_matches_oracle(gpu, k):
    inst = make_instance(6, k)
    o = ref.RefSolver(inst, fused=True)
    o.solve()
    ro = o.result()
    rg = gpu.Problem(inst, retire_satisfied=0, fused_round=1).solve()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"] and rg["steps"] == ro["steps"]
    r32 = gpu.Problem(inst, precision="fp32", retire_satisfied=0, fused_round=1).solve()
    assert r32["outcome"] == ref.OPTIMAL and r32["certified"]
    assert abs(r32["p_up"] - ro["p_up"]) <= inst.eps


def test_problem_from_the_library_constructor(gpu, oracle_results):
    # the constraints made by pcba_rtd_constraints from the same obstacle
    # points give the same plan (coefficients agree to rounding)
    k = 9
    rng = np.random.Generator(np.random.PCG64(I.SEED_STRIDE * 6 + k))
    pts, _, cost = I.rtd_pop(rng)
    g = gpu.rtd_constraints(I.frs_polynomial(), pts, I.EPS_Q)
    inst = Instance("rtdpop-lib", 2, np.array([0.0, -1.0]), np.array([1.0, 1.0]), cost, list(g), [],
                    max_boxes=1 << 20)
    r = gpu.Problem(inst).solve()
    o = oracle_results[k]
    assert r["outcome"] == o["outcome"] == ref.OPTIMAL
    assert abs(r["p_up"] - o["p_up"]) <= inst.eps and r["certified"]
