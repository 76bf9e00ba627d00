"""Round mode (fused_round = 1: every pass splits all l axes, 2^l children per
box, then one cut-off test) through the C ABI, against the oracle's round mode.

FP64 plain mode runs the same sequence of de Casteljau operations as the
oracle (axis 0, then axis 1 of both halves), so step traces are compared step
by step: outcome, bracket, box ids, patches within 1e-12 of the patch's
largest coefficient.  FP32 mode runs both splits as products with the
subdivision matrices of Sec. II-E on the matrix cores and widens every bound
by its carried rounding bound: final results within eps of the oracle, the
certificate, feasibility at the centre of x*, and the carried bound against
the oracle's FP64 patches derived box by box."""
import numpy as np
import pytest

import paper_problems as pp
from oracle import ref
from paper_2003_01758_amd.instances import make_instance, poly_eval, truncate

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


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
    "P2": lambda: _bench("P2"),
    "small5_memory": lambda: make_instance(0, 5).with_options(max_boxes=64),
    "waypoints30": lambda: truncate(make_instance(5, 0), 30),
}


def _patch_close(a, b):
    scale = max(1.0, float(np.abs(b).max()))
    return float(np.abs(a - b).max(initial=0.0)) <= REL * scale


@pytest.fixture
def cut_split(gpu, request):
    # split: every cut over workgroups of 64 children once a round has more
    # than 64 children (four per parent)
    if request.param == "split":
        gpu.set_cut_split(64, 64)
    yield request.param
    gpu.set_cut_split()


@pytest.mark.parametrize("cut_split", ["one", "split"], indirect=True)
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_round_trace_matches_oracle(gpu, name, cut_split):
    inst = CASES[name]()
    print(f"[round fp64 trace] {name} cut={cut_split}", flush=True)
    g = gpu.Problem(inst, retire_satisfied=0, fused_round=1)
    o = ref.RefSolver(inst, fused=True)
    for step in range(200):
        so = o.step()
        rg = g.step(1)
        ro = o.result()
        assert rg["outcome"] == so, f"step {step}"
        for key in ("steps", "rounds", "list_len", "has_x"):
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


@pytest.mark.parametrize("k", [0, 1])
def test_fp64_round_full_rtd_solve_matches_oracle(gpu, k):
    inst = make_instance(1, k)
    print(f"[round fp64 rtd] {k}", flush=True)
    rg = gpu.Problem(inst, retire_satisfied=0, fused_round=1).solve()
    o = ref.RefSolver(inst, fused=True)
    o.solve()
    ro = o.result()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    assert rg["p_up"] == ro["p_up"] and rg["p_lo"] == ro["p_lo"]
    assert rg["steps"] == ro["steps"] and rg["peak_len"] == ro["peak_len"]
    assert np.array_equal(rg["x_index"], ro["x_index"])
    assert rg["certified"]
    c = 0.5 * (rg["x_lo"] + rg["x_hi"])
    assert max(poly_eval(q, c) for q in inst.ineq) <= 1e-6


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("name", ["small0", "small1", "rtd40", "P2", "waypoints30"])
def test_fp32_round_solve_matches_oracle_within_eps(gpu, name, engine):
    inst = CASES[name]()
    print(f"[round fp32 solve] {name} {engine}", flush=True)
    rg = gpu.Problem(inst, precision="fp32", retire_satisfied=0, fused_round=1, split_engine=engine).solve()
    o = ref.RefSolver(inst, fused=True)
    o.solve()
    ro = o.result()
    assert rg["outcome"] == ro["outcome"] == ref.OPTIMAL
    assert abs(rg["p_up"] - ro["p_up"]) <= inst.eps
    assert rg["p_lo"] <= ro["p_up"] + 1e-12 and ro["p_lo"] <= rg["p_up"] + 1e-12
    assert rg["certified"]
    c = 0.5 * (rg["x_lo"] + rg["x_hi"])
    for q in inst.ineq:
        assert poly_eval(q, c) <= 1e-6


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("name,rederive", [("rtd40", 4), ("rtd40", 0), ("small1", 3)])
def test_fp32_round_error_bound_is_sound(gpu, name, rederive, engine):
    # every FP32 coefficient after a round (two splits, by de Casteljau or as
    # products on the matrix cores) stays within its patch's carried bound of
    # the oracle's FP64 patch of the same box
    inst = CASES[name]()
    print(f"[round fp32 bound] {name} rederive={rederive} {engine}", flush=True)
    g = gpu.Problem(inst, precision="fp32", retire_satisfied=0, fused_round=1, rederive_every=rederive,
                    split_engine=engine)
    o = ref.RefSolver(inst)
    sizes = [int(np.prod(inst.cost.shape))]
    kdeg = [o.kind_degree(1), o.kind_degree(2)]
    sizes += [int(np.prod(kdeg[0] + 1))] * inst.n_ineq + [int(np.prod(kdeg[1] + 1))] * inst.n_eq
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(2)
    checked = 0
    for step in range(40):
        r = g.step(1)
        ids, pat = g.list()
        err = g.errors()
        for row in rng.choice(len(ids), size=min(6, len(ids)), replace=False) if len(ids) else []:
            want = o.derive(r["depth"], ids[row])
            for p in range(len(sizes)):
                got = pat[row, offs[p]:offs[p + 1]]
                w = want[offs[p]:offs[p + 1]]
                d = np.abs(got - w).max()
                assert d <= err[row, p], (step, row, p, d, err[row, p])
                checked += 1
        if r["outcome"] != gpu.RUNNING:
            break
    assert checked > 0


def test_round_batch_mixes_modes_and_precisions(gpu):
    # one-direction and round problems of both precisions in the same launches:
    # each result equals the problem solved alone
    specs = [(make_instance(0, 0), "fp64", 1), (make_instance(0, 0), "fp64", 0),
             (truncate(make_instance(1, 2), 30), "fp32", 1), (truncate(make_instance(1, 2), 30), "fp32", 0),
             (make_instance(0, 4), "fp32", 1), (truncate(make_instance(3, 1), 20), "fp64", 0)]
    def mk(inst, prec, fused):
        return gpu.Problem(inst, precision=prec, retire_satisfied=0, fused_round=fused)
    alone = [mk(*s).solve() for s in specs]
    mixed = gpu.solve_batch([mk(*s) for s in specs])
    for k, (a, b) in enumerate(zip(alone, mixed)):
        for key in ("outcome", "p_up", "p_lo", "steps", "certified"):
            assert a[key] == b[key], (k, key)
