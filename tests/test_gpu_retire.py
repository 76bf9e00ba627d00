"""Retiring satisfied inequalities (library option retire_satisfied) against
the paper's method without it.

An inequality whose patch on a box has max B <= 0 holds on the whole box
(Thm. of enclosure); subdivision forms convex combinations of a patch's
coefficients, and in FP64 the rounded midpoint of two numbers lies between
them, so every descendant's patch also has max B <= 0 and can neither make a
box infeasible nor stop it from being feasible.  Dropping such patches must
therefore leave every FP64 step bit for bit unchanged: the same box ids, the
same bounds, the same outcome, and the same coefficients for every patch still
carried, while a dropped patch is one whose full-list coefficients are all
<= 0."""
import numpy as np
import pytest

from oracle import ref
from paper_2003_01758_amd.instances import make_instance, truncate

pytestmark = pytest.mark.gpu

CASES = {
    "small0": lambda: make_instance(0, 0),
    "rtd60": lambda: truncate(make_instance(1, 4), 60),
    "batch_l3": lambda: truncate(make_instance(3, 1), 30),
    "d4_eq": lambda: truncate(make_instance(2, 0), 12).with_options(max_boxes=1 << 11),
}


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


def _ineq_slices(inst, o):
    s0 = int(np.prod(inst.cost.shape))
    s1 = int(np.prod(o.kind_degree(1) + 1))
    return [slice(s0 + i * s1, s0 + (i + 1) * s1) for i in range(inst.n_ineq)]


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_steps_unchanged_by_retiring(gpu, name):
    inst = CASES[name]()
    print(f"[retire trace] {name}", flush=True)
    full = gpu.Problem(inst, retire_satisfied=0)
    ret = gpu.Problem(inst, retire_satisfied=1)
    o = ref.RefSolver(inst)
    sl = _ineq_slices(inst, o)
    dropped = 0
    for step in range(200):
        a = full.step(1)
        b = ret.step(1)
        for key in ("outcome", "steps", "list_len", "has_x", "p_up", "p_lo"):
            assert a[key] == b[key], (step, key)
        assert np.array_equal(a["x_index"], b["x_index"])
        ia, pa = full.list()
        ib, pb = ret.list()
        assert np.array_equal(ia, ib), step
        nan = np.isnan(pb)
        # only whole inequality patches are ever dropped
        keep_cols = np.ones(pb.shape[1], dtype=bool)
        for s in sl:
            keep_cols[s] = False
        assert not nan[:, keep_cols].any()
        for s in sl:
            gone = nan[:, s]
            assert np.all(gone.all(axis=1) | ~gone.any(axis=1))
            rows = gone.all(axis=1)
            if rows.any():
                dropped += int(rows.sum())
                # the dropped patch is satisfied on the box: every coefficient <= 0
                assert pa[rows, s].max() <= 0.0, step
        assert np.array_equal(pa[~nan], pb[~nan]), step
        if a["outcome"] != gpu.RUNNING:
            break
    if inst.n_ineq:
        assert dropped > 0


@pytest.mark.parametrize("name", ["small0", "rtd60", "batch_l3"])
def test_carried_patch_counts(gpu, name):
    inst = CASES[name]()
    print(f"[retire counts] {name}", flush=True)
    g = gpu.Problem(inst)
    o = ref.RefSolver(inst)
    sl = _ineq_slices(inst, o)
    carried = [inst.n_ineq]   # before step s: patches carried by the list
    for step in range(200):
        r = g.step(1)
        _, pat = g.list()
        carried.append(int(sum((~np.isnan(pat[:, s])).all(axis=1).sum() for s in sl)))
        if r["outcome"] != gpu.RUNNING:
            break
    tr = g.trace()
    pt = g.trace_patches()
    n = len(tr["k_in"])
    assert n == len(carried) - 1
    for s in range(n):
        assert pt["a_in"][s] == carried[s], s
        if s + 1 < n:
            assert pt["a_kept"][s] == pt["a_in"][s + 1], s
        assert pt["a_in"][s] <= tr["k_in"][s] * inst.n_ineq
    # the same counts without retiring are the list lengths times alpha
    f = gpu.Problem(inst, retire_satisfied=0)
    f.solve()
    tf, pf = f.trace(), f.trace_patches()
    assert np.array_equal(pf["a_in"], tf["k_in"].astype(np.int64) * inst.n_ineq)
    assert np.array_equal(pf["a_kept"], tf["k_kept"].astype(np.int64) * inst.n_ineq)
    assert pt["a_in"].sum() < pf["a_in"].sum()


@pytest.mark.parametrize("k", [0, 1])
def test_fp32_retiring_stays_within_eps_and_certified(gpu, k):
    inst = make_instance(1, k)
    print(f"[retire fp32] rtd {k}", flush=True)
    a = gpu.Problem(inst, precision="fp32", retire_satisfied=1).solve()
    b = gpu.Problem(inst, precision="fp32", retire_satisfied=0).solve()
    o = ref.RefSolver(inst)
    o.solve()
    ro = o.result()
    for r in (a, b):
        assert r["outcome"] == ro["outcome"] == gpu.OPTIMAL
        assert abs(r["p_up"] - ro["p_up"]) <= inst.eps
        assert r["certified"]
