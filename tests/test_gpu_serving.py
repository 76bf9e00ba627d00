"""Continuous batching: plans that arrive while others are on the GPU are
admitted as the footprint budget frees up.  Every served plan is checked
against the FP64 oracle solving the same plan alone: in FP64 plain mode the
estimate, the least lower bound, the step count and the returned box are
identical; in FP32 mode the estimate is within eps and certified (Alg. PCBA,
return step; Def. of feasibility).  Each result also equals the library's own
solve of the plan alone."""
import numpy as np
import pytest

from oracle import ref
from paper_2003_01758_amd.instances import make_instance, truncate

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_served_results_match_oracle(precision):
    from paper_2003_01758_amd import pcba, serve
    reqs = [truncate(make_instance(4, k), 60 + 20 * (k % 5)) for k in range(16)]
    arrivals = np.sort(np.random.default_rng(3).uniform(0.0, 0.05, size=len(reqs)))
    probe = pcba.Problem(reqs[0], precision=precision)
    budget = 3 * probe.footprint(128)      # a few plans resident at a time
    probe.close()
    srv = serve.Server(budget, reserve_boxes=128, steps_per_round=3, precision=precision,
                       deadline_s=30.0)
    recs = srv.serve(reqs, arrivals)
    stats = serve.summarize(recs, 0.05)
    assert stats["plans"] == len(reqs) and stats["certified"] == len(reqs)
    for k, (inst, r) in enumerate(zip(reqs, recs)):
        o = ref.RefSolver(inst)
        o.solve()
        ro = o.result()
        assert r["outcome"] == ro["outcome"] == pcba.OPTIMAL, k
        assert r["certified"], k
        if precision == "fp64":
            assert r["p_up"] == ro["p_up"] and r["p_lo"] == ro["p_lo"], k
            assert r["steps"] == ro["steps"], k
            assert list(r["x_index"]) == [int(v) for v in ro["x_index"]], k
        else:
            assert abs(r["p_up"] - ro["p_up"]) <= inst.eps, k
        alone = pcba.Problem(inst, precision=precision).solve()
        assert r["p_up"] == alone["p_up"] and r["steps"] == alone["steps"], k
