"""Pins of the oracle's round mode (every pass splits along all l axes).

The paper splits one direction per pass; the round mode is a reading of the
library's own (children are convex combinations of their parent's
coefficients, so extrema nest).  Its primitive is pinned to exact rational
Bernstein coefficients over each sub-box, and its solve to the one-direction
oracle at every round end, and to the printed benchmark optima."""
import numpy as np
import pytest

import paper_problems as pp
from oracle import exact, ref
from paper_2003_01758_amd.instances import make_instance, truncate


def rel_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(1.0, float(np.abs(b).max())))


@pytest.mark.parametrize("shape", [(5, 5), (7, 4), (11, 11), (3, 4, 5)])
def test_round_split_matches_exact_subboxes(shape):
    # child c of the round covers, along axis k, the left half if bit
    # (l-1-k) of c is clear and the right half otherwise
    rng = np.random.default_rng(5)
    mono = rng.integers(-5, 6, size=shape)
    l = len(shape)
    lo, hi = [-1.0] * l, [1.0] * l
    parent = ref.to_bernstein(mono.astype(float), lo, hi)
    kids = ref.split_round(parent)
    assert kids.shape == (1 << l,) + tuple(shape)
    growth = 2.0 ** (sum(s - 1 for s in shape) / 2)
    for c in range(1 << l):
        blo = [0.0 if (c >> (l - 1 - k)) & 1 else -1.0 for k in range(l)]
        bhi = [1.0 if (c >> (l - 1 - k)) & 1 else 0.0 for k in range(l)]
        want = exact.to_float(exact.bernstein_exact(mono, blo, bhi))
        assert rel_err(kids[c], want) <= 1e-14 * growth, c


def test_round_split_is_two_axis_splits_in_order():
    rng = np.random.default_rng(9)
    P = rng.normal(size=(6, 8))
    kids = ref.split_round(P)
    L, R = ref.split(P, 0)
    want = [*ref.split(L, 1), *ref.split(R, 1)]
    for c in range(4):
        assert np.array_equal(kids[c], want[c])


def _round_ends(inst):
    """The one-direction oracle's state after every l-th pass, until it stops."""
    o = ref.RefSolver(inst)
    ends = []
    while True:
        out = o.step()
        r = o.result()
        if r["steps"] % inst.l == 0 and r["steps"] > 0:
            ids, pat = o.list()
            ends.append((out, r, ids, pat))
        if out != ref.RUNNING:
            return ends, out, r


CASES = {
    "small0": lambda: make_instance(0, 0),
    "small3": lambda: make_instance(0, 3),
    "small5": lambda: make_instance(0, 5),
    "rtd40": lambda: truncate(make_instance(1, 1), 40),
    "waypoints30": lambda: truncate(make_instance(5, 0), 30),
}


@pytest.mark.parametrize("name", list(CASES))
def test_round_mode_equals_one_direction_passes_at_round_ends(name):
    inst = CASES[name]()
    ends, last_out, last = _round_ends(inst)
    f = ref.RefSolver(inst, fused=True)
    for q, (out, r, ids, pat) in enumerate(ends):
        fo = f.step()
        fr = f.result()
        assert fr["steps"] == q + 1 and fr["rounds"] == r["rounds"]
        assert np.array_equal(fr["depth"], r["depth"])
        assert fr["p_up"] == r["p_up"] and fr["p_lo"] == r["p_lo"], q
        assert fr["has_x"] == r["has_x"]
        if r["has_x"]:
            assert np.array_equal(fr["x_index"], r["x_index"]) and np.array_equal(fr["x_depth"], r["x_depth"])
        fids, fpat = f.list()
        assert np.array_equal(fids, ids), q
        assert np.array_equal(fpat, pat), q
        assert fo == out, q
    if last["steps"] % inst.l == 0:
        assert f.result()["outcome"] == last_out
        return
    # the one-direction passes stopped mid-round (the width test already holds
    # after the first direction of a round, and the bracket closed there): the
    # round mode stops at the end of that round with the same outcome and a
    # bracket inside theirs (more splits only narrow it)
    fo = f.step()
    fr = f.result()
    assert fo == last_out
    assert fr["p_up"] <= last["p_up"] and fr["p_lo"] >= last["p_lo"]
    assert fr["p_up"] - fr["p_lo"] <= inst.eps


def test_round_mode_memory_test_counts_all_children():
    # 2^l * length(L) > M ends the solve before the round that would exceed M
    inst = make_instance(0, 5).with_options(max_boxes=64)
    f = ref.RefSolver(inst, fused=True)
    while f.step() == ref.RUNNING:
        pass
    r = f.result()
    assert r["outcome"] == ref.MEMORY_LIMIT
    assert 4 * r["list_len"] > 64 and 4 * r["peak_len"] > 64
    o = ref.RefSolver(inst)
    o.solve()
    # the one-direction passes test 2 * length(L) <= M at every pass, so they go
    # at least as far
    assert o.result()["steps"] >= inst.l * r["steps"]


def test_round_mode_cannot_change_after_the_first_pass():
    f = ref.RefSolver(make_instance(0, 1))
    f.step()
    assert f.L.pcba_ref_set_fused(f.h, 1) != 0


@pytest.mark.parametrize("name", ["P1", "P2", "P3"])
def test_round_mode_reaches_printed_optimum(name):
    p = next(q for q in pp.load()["benchmarks"] if q["name"] == name)
    inst = pp.benchmark_instance(p)
    B = ref.to_bernstein(inst.cost, inst.lo, inst.hi)
    eps = 1e-7 * (B.max() - B.min())
    s = ref.RefSolver(inst, fused=True, eps=eps, delta=1e9, eps_eq=1e-6, max_boxes=1 << 18, max_iters=28)
    out = s.solve()
    r = s.result()
    assert inst.l == 2 and out == ref.OPTIMAL
    tol = 1e-9 * max(1.0, abs(p["optimum"]))
    assert r["p_lo"] <= p["optimum"] + tol
    assert r["p_up"] - p["optimum"] <= eps + tol
