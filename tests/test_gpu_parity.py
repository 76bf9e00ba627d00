"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

FP64 plain mode follows the same arithmetic as the oracle (same root
conversion order, the same de Casteljau recurrence, exact min/max and
comparisons), so lists, bounds and outcomes are compared step by step and
patches within 1e-12 of the largest coefficient of the patch.  FP32 mode widens
every bound by its carried rounding bound, so only final results are compared
(optimum within eps, same outcome, certified), plus soundness of the bound
against oracle patches derived box by box."""
import math
import os

import numpy as np
import pytest

import paper_problems as pp
from oracle import ref
from paper_2003_01758_amd.instances import Instance, make_instance, poly_eval, truncate

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


def _circle():
    cost = np.zeros((2, 2))
    cost[1, 0] = cost[0, 1] = 1.0
    h = np.zeros((3, 3))
    h[2, 0] = h[0, 2] = 1.0
    h[0, 0] = -1.0
    return Instance("circle", 2, np.array([-2.0, -2.0]), np.array([2.0, 2.0]), cost, [], [h],
                    eps=1e-4, delta=1e9, eps_eq=1e-3, max_boxes=1 << 18, max_iters=28)


def _bench(name, **kw):
    p = next(q for q in pp.load()["benchmarks"] if q["name"] == name)
    inst = pp.benchmark_instance(p)
    B = ref.to_bernstein(inst.cost, inst.lo, inst.hi)
    opts = dict(eps=1e-7 * (B.max() - B.min()), delta=1e9, eps_eq=1e-6, max_boxes=1 << 18)
    opts.update(kw)
    return inst.with_options(**opts)


CASES = {
    "small0": lambda: make_instance(0, 0),
    "small1": lambda: make_instance(0, 1),
    "small7": lambda: make_instance(0, 7),
    "rtd40": lambda: truncate(make_instance(1, 3), 40),
    "batch_l3": lambda: truncate(make_instance(3, 1), 30),
    "P4": lambda: _bench("P4"),
    "P7_memory": lambda: _bench("P7", max_boxes=1 << 11),
    "circle_eq": _circle,
    "d4_eq": lambda: truncate(make_instance(2, 0), 12).with_options(max_boxes=1 << 11),
}


def _patch_close(a, b):
    # a: the library's item (inequality patches it no longer carries are NaN,
    # and must be satisfied: every oracle coefficient <= 0); b: the oracle's
    scale = max(1.0, float(np.abs(b).max()))
    gone = np.isnan(a)
    if gone.any() and not float(b[gone].max()) <= 0.0:
        return False
    return float(np.abs(a[~gone] - b[~gone]).max(initial=0.0)) <= REL * scale


@pytest.mark.parametrize("name", list(CASES))
def test_root_patches_match_oracle(gpu, name):
    inst = CASES[name]()
    g = gpu.Problem(inst)
    o = ref.RefSolver(inst)
    want = o.derive(np.zeros(inst.l, dtype=np.int32), np.zeros(inst.l, dtype=np.uint32))
    got = g.root()
    assert got.shape == want.shape
    assert _patch_close(got, want)


@pytest.fixture
def cut_split(gpu, request):
    # split: every cut over workgroups of 64 children once a step has more
    # than 64 children (the library's default splits from 32,768 on)
    if request.param == "split":
        gpu.set_cut_split(64, 64)
    yield request.param
    gpu.set_cut_split()


@pytest.mark.parametrize("cut_split", ["one", "split"], indirect=True)
@pytest.mark.parametrize("retire", [1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_step_trace_matches_oracle(gpu, name, retire, cut_split):
    inst = CASES[name]()
    print(f"[fp64 trace] {name} retire={retire} cut={cut_split}", flush=True)
    g = gpu.Problem(inst, retire_satisfied=retire)
    o = ref.RefSolver(inst)
    for step in range(200):
        so = o.step()
        rg = g.step(1)
        ro = o.result()
        assert rg["outcome"] == so, f"step {step}"
        for key in ("steps", "rounds", "list_len", "next_dir", "has_x"):
            assert rg[key] == ro[key], (step, key)
        assert np.array_equal(rg["depth"], ro["depth"])
        assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"], step
        if ro["has_x"]:
            assert np.array_equal(rg["x_index"], ro["x_index"])
            assert np.array_equal(rg["x_depth"], ro["x_depth"])
        gi, gp = g.list()
        oi, op = o.list()
        assert np.array_equal(gi, oi), f"box ids differ at step {step}"
        for row in range(len(oi)):
            assert _patch_close(gp[row], op[row]), (step, row)
        if so != ref.RUNNING:
            break
    assert g.result()["peak_len"] == o.result()["peak_len"]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_fp64_full_rtd_solve_matches_oracle(gpu, k):
    inst = make_instance(1, k)
    print(f"[fp64 rtd] {k}", flush=True)
    rg = gpu.Problem(inst).solve()
    o = ref.RefSolver(inst)
    o.solve()
    ro = o.result()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"]
    assert rg["steps"] == ro["steps"] and rg["peak_len"] == ro["peak_len"]
    assert np.array_equal(rg["x_index"], ro["x_index"])
    assert rg["certified"]
    assert rg["p_cert"] >= rg["p_up"] - 1e-9 and rg["p_cert"] - rg["p_up"] <= 1e-9
    c = 0.5 * (rg["x_lo"] + rg["x_hi"])
    assert max(poly_eval(q, c) for q in inst.ineq) <= 1e-6


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("name", ["small0", "small1", "rtd40", "batch_l3", "P4", "circle_eq"])
def test_fp32_solve_matches_oracle_within_eps(gpu, name, engine):
    inst = CASES[name]()
    print(f"[fp32 solve] {name} {engine}", flush=True)
    rg = gpu.Problem(inst, precision="fp32", split_engine=engine).solve()
    o = ref.RefSolver(inst)
    o.solve()
    ro = o.result()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    eps = inst.eps
    assert abs(rg["p_up"] - ro["p_up"]) <= eps
    assert rg["p_lo"] <= ro["p_up"] + 1e-12 and ro["p_lo"] <= rg["p_up"] + 1e-12
    assert rg["certified"]
    assert rg["p_cert"] <= rg["p_up"] + 1e-9
    c = 0.5 * (rg["x_lo"] + rg["x_hi"])
    for q in inst.ineq:
        assert poly_eval(q, c) <= 1e-6
    for q in inst.eq:
        assert abs(poly_eval(q, c)) <= inst.eps_eq + 1e-6


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("name,rederive", [("rtd40", 8), ("rtd40", 0), ("small1", 3), ("batch_l3", 5)])
def test_fp32_error_bound_is_sound(gpu, name, rederive, engine):
    # every FP32 coefficient stays within its patch's carried bound of the FP64
    # patch the oracle derives for the same box id
    inst = CASES[name]()
    print(f"[fp32 bound] {name} rederive={rederive} {engine}", flush=True)
    g = gpu.Problem(inst, precision="fp32", rederive_every=rederive, split_engine=engine)
    o = ref.RefSolver(inst)
    sizes = [int(np.prod(inst.cost.shape))]
    kdeg = [o.kind_degree(1), o.kind_degree(2)]
    sizes += [int(np.prod(kdeg[0] + 1))] * inst.n_ineq + [int(np.prod(kdeg[1] + 1))] * inst.n_eq
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(1)
    worst = seen = 0.0
    for step in range(60):
        r = g.step(1)
        ids, pat = g.list()
        err = g.errors()
        for row in rng.choice(len(ids), size=min(6, len(ids)), replace=False) if len(ids) else []:
            want = o.derive(r["depth"], ids[row])
            for p in range(len(sizes)):
                got = pat[row, offs[p]:offs[p + 1]]
                w = want[offs[p]:offs[p + 1]]
                if np.isnan(got).all():
                    # retired on an ancestor whose widened bound was <= 0
                    assert w.max() <= 1e-12 * max(1.0, np.abs(w).max()), (step, row, p)
                    continue
                d = np.abs(got - w).max()
                assert d <= err[row, p], (step, row, p, d, err[row, p])
                seen = max(seen, float(err[row, p]))
                if err[row, p] > 0:
                    worst = max(worst, d / err[row, p])
        if rederive == 0 and seen > 0:
            # every bound checked came from a subdivision: err_max covers it
            assert r["err_max"] >= seen, step
        if r["outcome"] != gpu.RUNNING:
            break
    print(f"largest error / bound seen: {worst:.3g}")


def test_batch_results_equal_alone(gpu):
    names = ["small0", "small1", "rtd40", "P4", "circle_eq", "small7"]
    insts = [CASES[n]() for n in names]
    alone = [gpu.Problem(i).solve() for i in insts]
    probs = [gpu.Problem(i) for i in insts]
    mixed = gpu.solve_batch(probs)
    for n, a, b in zip(names, alone, mixed):
        for key in ("outcome", "p_up", "p_lo", "steps", "peak_len", "certified", "p_cert"):
            assert a[key] == b[key], (n, key)
        assert np.array_equal(a["x_index"], b["x_index"])


def test_fp32_batch_results_equal_alone(gpu):
    # the batch mixes both split engines: each problem's tiles take its own
    names = ["small0", "rtd40", "batch_l3", "small0", "rtd40", "batch_l3"]
    engines = ["valu"] * 3 + ["mfma"] * 3
    insts = [CASES[n]() for n in names]
    alone = [gpu.Problem(i, precision="fp32", split_engine=e).solve() for i, e in zip(insts, engines)]
    mixed = gpu.solve_batch([gpu.Problem(i, precision="fp32", split_engine=e) for i, e in zip(insts, engines)])
    for n, a, b in zip(names, alone, mixed):
        for key in ("outcome", "p_up", "p_lo", "steps", "certified"):
            assert a[key] == b[key], (n, key)


def test_outcome_codes_match_oracle(gpu):
    cases = [
        (truncate(make_instance(1, 2), 50), dict(max_boxes=8)),
        (make_instance(0, 1), dict(max_iters=3)),
    ]
    g = np.zeros((3, 1))
    g[0, 0], g[2, 0] = 1.0, 1.0
    cost = np.zeros((2, 2))
    cost[1, 1] = 1.0
    a = np.zeros((2, 1)); a[0, 0], a[1, 0] = -0.3, 1.0
    b = np.zeros((2, 1)); b[0, 0], b[1, 0] = 0.31, -1.0
    box = dict(eps=1e-6, delta=1e-3, eps_eq=1e-6, max_boxes=1 << 12)
    cases.append((Instance("inf1", 2, np.zeros(2), np.ones(2), cost, [g], [], **box), {}))
    cases.append((Instance("inf2", 2, np.zeros(2), np.ones(2), cost, [a, b], [], **box), {}))
    for inst, kw in cases:
        rg = gpu.Problem(inst.with_options(**kw)).solve()
        o = ref.RefSolver(inst.with_options(**kw))
        o.solve()
        ro = o.result()
        assert rg["outcome"] == ro["outcome"], inst.name
        assert rg["steps"] == ro["steps"] and rg["list_len"] == ro["list_len"]
        assert (math.isinf(rg["p_up"]) and math.isinf(ro["p_up"])) or rg["p_up"] == ro["p_up"]


def test_list_growth_keeps_parity(gpu):
    # the device list starts small and grows; the 4-D case grows well past it
    inst = truncate(make_instance(2, 0), 20).with_options(max_boxes=1 << 13)
    rg = gpu.Problem(inst).solve()
    o = ref.RefSolver(inst)
    o.solve()
    ro = o.result()
    assert rg["outcome"] == ro["outcome"]
    assert rg["peak_len"] == ro["peak_len"] and ro["peak_len"] > 64
    assert rg["capacity"] > 64
    assert rg["p_lo"] == ro["p_lo"] and rg["steps"] == ro["steps"]


def test_engine_admission_by_footprint(gpu):
    insts = [make_instance(0, k) for k in range(6)]
    probs = [gpu.Problem(i) for i in insts]
    # each admitted problem is charged for max(its list capacity, the reserve)
    one = probs[0].footprint(max(128, probs[0].result()["capacity"]))
    budget = int(one * 2.5)
    eng = gpu.Engine(budget_bytes=budget, reserve_boxes=128)
    queue = list(probs)
    done = []
    most = 0
    for _ in range(1000):
        while queue and eng.submit(queue[0]):
            queue.pop(0)
        resident = len(probs) - len(queue) - len(done)
        most = max(most, resident)
        # only the oldest resident problem may grow past the budget, and then
        # nothing else is admitted beside it
        assert eng.used_bytes() <= budget or resident == 1
        eng.run(4)
        done += eng.poll()
        if len(done) == len(probs):
            break
    assert len(done) == len(probs)
    assert most == 2
    for p, i in zip(probs, insts):
        alone = gpu.Problem(i).solve()
        r = p.result()
        assert r["p_up"] == alone["p_up"] and r["outcome"] == alone["outcome"]


@pytest.mark.parametrize("stale", [0, 1])
def test_fp64_large_list_trace_matches_oracle(gpu, stale):
    # tens of thousands of work units per step: every workgroup walks many
    # units, so the pipelined kernel's unit-to-unit hand-over is exercised;
    # per-step list length and least lower bound against the oracle's trace
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(here, "golden", "d4_trace.json")))["steps"]
    inst = truncate(make_instance(2, 0), 100).with_options(max_boxes=1 << 16)
    print(f"[fp64 large trace] stale={stale}", flush=True)
    g = gpu.Problem(inst, stale_filter=stale)
    g.step(len(gold))
    tr = g.trace()
    assert len(tr["k_kept"]) == len(gold)
    for s, row in enumerate(gold):
        assert tr["k_kept"][s] == row["k"], (s, tr["k_kept"][s], row["k"])
        assert tr["p_lo"][s] == row["p_lo"], s


@pytest.mark.parametrize("prec,retire,rederive", [("fp64", 0, 16), ("fp64", 1, 16), ("fp32", 0, 0), ("fp32", 1, 16)])
def test_persistent_steps_equal_launches(gpu, prec, retire, rederive):
    # several whole steps per cooperative launch (grid barriers between the
    # subdivision and the cut) against one launch per kernel per step: the
    # same operations in the same order, so every result is identical
    insts = [CASES[n]() for n in ("small0", "small1", "rtd40", "P4", "batch_l3", "small7")]
    print(f"[persistent] {prec} retire={retire} rederive={rederive}", flush=True)
    out = []
    for persist in (0, 1):
        probs = [gpu.Problem(i, precision=prec, retire_satisfied=retire, rederive_every=rederive,
                             persistent_steps=persist) for i in insts]
        out.append(gpu.solve_batch(probs))
        for p in probs:
            p.close()
    for k, (a, b) in enumerate(zip(*out)):
        for key in ("outcome", "p_up", "p_lo", "steps", "peak_len", "certified", "p_cert"):
            assert a[key] == b[key], (k, key)
        assert np.array_equal(a["x_index"], b["x_index"]), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_cut_batch_equals_one_workgroup_cut(gpu, prec):
    # a batch of problems of different sizes: with the cut split over
    # workgroups of 64 children (problem b, part g from one grid) every result
    # equals the one-workgroup cut's
    insts = [CASES[n]() for n in ("small0", "rtd40", "P4", "batch_l3", "circle_eq", "small7")]
    print(f"[split cut batch] {prec}", flush=True)
    out = []
    for split in (0, 64):
        gpu.set_cut_split(split, 64)
        try:
            probs = [gpu.Problem(i, precision=prec) for i in insts]
            out.append(gpu.solve_batch(probs))
            for p in probs:
                p.close()
        finally:
            gpu.set_cut_split()
    for k, (a, b) in enumerate(zip(*out)):
        for key in ("outcome", "p_up", "p_lo", "steps", "peak_len", "certified", "p_cert"):
            assert a[key] == b[key], (k, key)
        assert np.array_equal(a["x_index"], b["x_index"]), k
