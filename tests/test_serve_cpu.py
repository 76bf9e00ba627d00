"""Host-side pieces of the serving loop (no device call)."""
import numpy as np


def test_poisson_arrivals_rate():
    from paper_2003_01758_amd import serve
    t = serve.poisson_arrivals(200.0, 60.0, seed=1)
    assert 11500 < len(t) < 12500 and np.all(np.diff(t) > 0) and t[-1] < 60.0
