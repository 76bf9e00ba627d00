"""The multi-waypoint plan workload (Sec. VI: the cost is a product over
waypoints of the squared distance of the endpoint map, multi-modal): the
generator's structure, the oracle against brute force on a grid, and the GPU
path against the oracle."""
import numpy as np
import pytest

from oracle import ref
from paper_2003_01758_amd.instances import make_instance, poly_eval, poly_eval_many


def test_waypoint_cost_structure():
    for k in range(3):
        inst = make_instance(5, k)
        # two squared distances of a (3,3) map: multi-degree (12,12)
        assert inst.cost.shape == (13, 13)
        assert len(inst.ineq) == 100
        # a product of sums of squares is nonnegative everywhere
        g = np.linspace(-1.0, 1.0, 101)
        X, Y = np.meshgrid(g, g, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel()], 1)
        assert poly_eval_many(inst.cost, pts).min() >= -1e-9
        # the planted point is feasible with margin
        assert max(poly_eval(q, inst.q0) for q in inst.ineq) < 0.0


def test_waypoint_oracle_against_grid():
    inst = make_instance(5, 2)
    s = ref.RefSolver(inst)
    assert s.solve() == ref.OPTIMAL
    r = s.result()
    n = 401
    g = np.linspace(-1.0, 1.0, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    feas = np.ones(len(pts), dtype=bool)
    for q in inst.ineq:
        feas &= poly_eval_many(q, pts) <= 0.0
    vals = poly_eval_many(inst.cost, pts)
    f_grid = vals[feas].min()
    # p_lo <= f* <= f_grid (rigorous); p_up within eps plus the grid's resolution
    assert r["p_lo"] <= f_grid + 1e-12
    grad = np.abs(np.gradient(vals.reshape(n, n), g[1] - g[0])).max()
    assert r["p_up"] <= f_grid + inst.eps + grad * (g[1] - g[0])
    assert r["p_up"] - r["p_lo"] <= inst.eps
    c = 0.5 * (r["x_lo"] + r["x_hi"])
    assert all(poly_eval(q, c) <= 0.0 for q in inst.ineq)


@pytest.mark.gpu
@pytest.mark.parametrize("k", [0, 1, 2])
def test_waypoint_gpu_matches_oracle(k):
    from paper_2003_01758_amd import pcba
    inst = make_instance(5, k)
    print(f"[waypoints] {k}", flush=True)
    o = ref.RefSolver(inst)
    o.solve()
    ro = o.result()
    rg = pcba.Problem(inst).solve()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"]
    assert rg["steps"] == ro["steps"] and rg["peak_len"] == ro["peak_len"]
    assert np.array_equal(rg["x_index"], ro["x_index"])
    assert rg["certified"]
    r32 = pcba.Problem(inst, precision="fp32").solve()
    assert r32["outcome"] == ref.OPTIMAL and r32["certified"]
    assert abs(r32["p_up"] - ro["p_up"]) <= inst.eps
    c = 0.5 * (r32["x_lo"] + r32["x_hi"])
    assert max(poly_eval(q, c) for q in inst.ineq) <= 1e-6
