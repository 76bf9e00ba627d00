"""Continuous batching: plans that arrive while others are on the GPU are
admitted as the footprint budget frees up, and every plan's result is the same
as when it is solved alone."""
import numpy as np
import pytest

from paper_2003_01758_amd.instances import make_instance, truncate

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_served_results_equal_alone(precision):
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
    for inst, r in zip(reqs, recs):
        alone = pcba.Problem(inst, precision=precision).solve()
        assert r["outcome"] == alone["outcome"] == pcba.OPTIMAL
        assert r["p_up"] == alone["p_up"] and r["steps"] == alone["steps"]
