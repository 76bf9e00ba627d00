"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle/pcba_ref.c (a wrong weight,
index, sign or operand; a dropped condition), builds the copy on the CPU and
runs a quick battery of the pins used elsewhere: closed forms, exact-rational
interpolation, vertex values, a printed benchmark optimum, a planted optimum,
the circle equality, infeasibility, and the list invariants.  Every planted
mistake must fail at least one pin; the unmodified source must pass them all.
"""
import math
import os
import subprocess
import tempfile
from math import comb

import numpy as np
import pytest

import paper_problems as pp
from oracle import exact, ref
from paper_2003_01758_amd.instances import Instance, make_instance, poly_eval

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pcba_ref.c")

MUTATIONS = {
    "split_weight": ("c[i] = (c[i] + c[i + 1]) * 0.5;", "c[i] = (c[i] + c[i + 1]) * 0.4999;"),
    "split_right_index": ("c[i] = (c[i] + c[i + 1]) * 0.5;\n                left[base + m * stride] = c[0];\n"
                          "                right[base + (n - m) * stride] = c[n - m];",
                          "c[i] = (c[i] + c[i + 1]) * 0.5;\n                left[base + m * stride] = c[0];\n"
                          "                right[base + (n - m) * stride] = c[0];"),
    "conversion_binomial": ("U[k * m + i] = binom(k, i) / binom(n, i);",
                            "U[k * m + i] = binom(k, i) / binom(n, k);"),
    "premap_sign": ("for (int t = 0; t < j - i; ++t) lp *= lo[r];",
                    "for (int t = 0; t < j - i; ++t) lp *= -lo[r];"),
    "premap_width": ("for (int t = 0; t < i; ++t) wi *= w;",
                     "for (int t = 0; t < i; ++t) wi *= hi[r];"),
    "transposed_operand": ("acc += A[k * m + i] * in[base + i * stride];",
                           "acc += A[i * m + k] * in[base + i * stride];"),
    "infeasible_uses_max": ("if (mn > 0.0) b.infeasible = 1;", "if (mx > 0.0) b.infeasible = 1;"),
    "feasible_uses_min": ("if (!(mx <= 0.0)) b.feasible = 0;", "if (!(mn <= 0.0)) b.feasible = 0;"),
    "keep_uses_max": ("keep[c] = (char)(!bd[c].infeasible && bd[c].minP <= h->p_up);",
                      "keep[c] = (char)(!bd[c].infeasible && bd[c].maxP <= h->p_up);"),
    "direction_stuck": ("if (h->rule == 0) return first ? 0 : (r_prev + 1) % h->l;",
                        "if (h->rule == 0) return first ? 0 : r_prev;"),
    "right_child_id": ("cids[(2 * k + 1) * l + r] = 2u * h->ids[k * l + r] + 1u;",
                       "cids[(2 * k + 1) * l + r] = 2u * h->ids[k * l + r];"),
    "eq_band_upper": ("if (!(-h->eps_eq <= mn && mn <= 0.0 && 0.0 <= mx && mx <= h->eps_eq))",
                      "if (!(-h->eps_eq <= mn && mn <= 0.0 && 0.0 <= mx))"),
    "width_off_by_one": ("if (h->lam == 0.5) return ldexp(w, -d);",
                         "if (h->lam == 0.5) return ldexp(w, -d - 2);"),
    "split_lambda_swapped": ("c[i] = mu * c[i] + lambda * c[i + 1];", "c[i] = lambda * c[i] + mu * c[i + 1];"),
    "lambda_box_bits": ("if ((i >> t) & 1u) a = m; else b = m;", "if ((i >> t) & 1u) b = m; else a = m;"),
    "maxwidth_narrowest": ("if (wk > bw) { bw = wk; best = k; }", "if (wk < bw) { bw = wk; best = k; }"),
    "round_id_bit_order": ("cids[(nc * k + c) * l + q] = 2u * h->ids[k * l + q] + (unsigned)((c >> (l - 1 - q)) & 1);",
                           "cids[(nc * k + c) * l + q] = 2u * h->ids[k * l + q] + (unsigned)((c >> q) & 1);"),
    "round_depth_one_axis": ("for (int q = 0; q < l; ++q) h->depth[q] += 1;", "h->depth[0] += 1;"),
    "round_memory_test": ("if (nc * K > h->M)", "if (2 * K > h->M)"),
    "round_axis_order": ("if (pcba_ref_split(l, deg, k, a + c * S,", "if (pcba_ref_split(l, deg, l - 1 - k, a + c * S,"),
    "p_up_uses_min": ("if (bd[c].feasible && (arg < 0 || bd[c].maxP < m)) { m = bd[c].maxP; arg = c; }",
                      "if (bd[c].feasible && (arg < 0 || bd[c].minP < m)) { m = bd[c].minP; arg = c; }"),
}


def build_variant(name, tmp):
    src = open(SRC).read()
    if name is not None:
        old, new = MUTATIONS[name]
        assert src.count(old) == 1, f"mutation {name} does not apply"
        src = src.replace(old, new)
    d = os.path.join(tmp, name or "clean")
    os.makedirs(d, exist_ok=True)
    for f in ("pcba_ref.h",):
        with open(os.path.join(d, f), "w") as out:
            out.write(open(os.path.join(ROOT, "oracle", f)).read())
    c = os.path.join(d, "pcba_ref.c")
    with open(c, "w") as out:
        out.write(src)
    so = os.path.join(d, "libpcba_ref.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c,
                    "-lm"], check=True)
    return ref.load(so)


def battery(L):
    """Returns the names of the pins that fail for the oracle build L."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    # closed form of x^k
    def closed_form():
        n = 6
        for k in range(n + 1):
            mono = np.zeros(n + 1)
            mono[k] = 1.0
            beta = ref.to_bernstein(mono, [0.0], [1.0], L=L)
            if np.max(np.abs(beta - [comb(i, k) / comb(n, k) for i in range(n + 1)])) > 1e-14:
                return False
        return True
    check("closed_form", closed_form)

    # exact interpolation on a box straddling zero, and of the split halves
    def exact_interp():
        rng = np.random.default_rng(4)
        mono = rng.integers(-5, 6, size=(4, 3))
        lo, hi = [-1.0, -0.5], [0.5, 1.5]
        beta = ref.to_bernstein(mono.astype(float), lo, hi, L=L)
        want = exact.to_float(exact.bernstein_exact(mono, lo, hi))
        if np.max(np.abs(beta - want)) > 1e-12 * max(1, np.abs(want).max()):
            return False
        for r in range(2):
            left, right = ref.split(beta, r, L=L)
            mid = 0.5 * (lo[r] + hi[r])
            hl = list(hi); hl[r] = mid
            lr = list(lo); lr[r] = mid
            wl = exact.to_float(exact.bernstein_exact(mono, lo, hl))
            wr = exact.to_float(exact.bernstein_exact(mono, lr, hi))
            if np.max(np.abs(left - wl)) > 1e-12 * max(1, np.abs(wl).max()):
                return False
            if np.max(np.abs(right - wr)) > 1e-12 * max(1, np.abs(wr).max()):
                return False
        return True
    check("exact_interpolation", exact_interp)

    # vertex coefficients are the values at the corners
    def vertices():
        rng = np.random.default_rng(8)
        mono = rng.normal(size=(5, 4))
        lo, hi = np.array([-0.7, 0.2]), np.array([0.9, 1.1])
        beta = ref.to_bernstein(mono, lo, hi, L=L)
        for cx in (0, 1):
            for cy in (0, 1):
                x = [hi[0] if cx else lo[0], hi[1] if cy else lo[1]]
                if abs(beta[4 * cx, 3 * cy] - poly_eval(mono, x)) > 1e-12:
                    return False
        return True
    check("vertices", vertices)

    def solve(inst, **kw):
        s = ref.RefSolver(inst, L=L, **kw)
        return s, s.solve(), s.result()

    # printed optimum of a benchmark problem (P3) with the paper's eps rule
    def p3():
        p = next(q for q in pp.load()["benchmarks"] if q["name"] == "P3")
        inst = pp.benchmark_instance(p)
        B = ref.to_bernstein(inst.cost, inst.lo, inst.hi)
        eps = 1e-7 * (B.max() - B.min())
        _, out, r = solve(inst, eps=eps, delta=1e9, eps_eq=1e-6, max_boxes=1 << 16, max_iters=28)
        return out == ref.OPTIMAL and r["p_lo"] <= p["optimum"] + 1e-9 and \
            r["p_up"] - p["optimum"] <= eps + 1e-9
    check("benchmark_P3", p3)

    # planted optimum (Dixon-Price, 2 variables)
    def planted():
        p = next(q for q in pp.load()["objectives"] if q["name"] == "DP2")
        inst = pp.planted_constraint_instance(p, 20, seed=5)
        _, out, r = solve(inst, eps=1e-4, delta=1e9, eps_eq=1e-6, max_boxes=1 << 16, max_iters=28)
        return out == ref.OPTIMAL and r["p_lo"] <= 1e-9 and r["p_up"] <= 1e-4 + 1e-9
    check("planted_DP2", planted)

    # equality: min x1 + x2 on the unit circle
    def circle():
        cost = np.zeros((2, 2)); cost[1, 0] = cost[0, 1] = 1.0
        h = np.zeros((3, 3)); h[2, 0] = h[0, 2] = 1.0; h[0, 0] = -1.0
        inst = Instance("c", 2, np.array([-2.0, -2.0]), np.array([2.0, 2.0]), cost, [], [h],
                        eps=1e-4, delta=1e9, eps_eq=1e-3, max_boxes=1 << 16, max_iters=28)
        _, out, r = solve(inst)
        c = 0.5 * (r["x_lo"] + r["x_hi"])
        return out == ref.OPTIMAL and r["p_lo"] <= -math.sqrt(2) + 1e-12 and \
            -math.sqrt(2.002) - 1e-12 <= r["p_up"] <= -math.sqrt(2) + 1e-4 and \
            abs(c @ c - 1.0) <= 1e-3 + 1e-6
    check("circle", circle)

    # equality with a constant cost: the first box certified inside the band
    # ends the solve, and its centre lies within the band of the circle
    def flat_circle():
        cost = np.zeros((1, 1))
        h = np.zeros((3, 3)); h[2, 0] = h[0, 2] = 1.0; h[0, 0] = -1.0
        inst = Instance("f", 2, np.array([-2.0, -2.0]), np.array([2.0, 2.0]), cost, [], [h],
                        eps=1e-4, delta=1e9, eps_eq=1e-3, max_boxes=1 << 18, max_iters=28)
        _, out, r = solve(inst)
        c = 0.5 * (r["x_lo"] + r["x_hi"])
        return out == ref.OPTIMAL and abs(c @ c - 1.0) <= 1e-3 + 1e-6
    check("flat_circle", flat_circle)

    # infeasibility: x1 <= 0.3 and x1 >= 0.31
    def infeasible():
        cost = np.zeros((2, 2)); cost[1, 1] = 1.0
        a = np.zeros((2, 1)); a[0, 0], a[1, 0] = -0.3, 1.0
        b = np.zeros((2, 1)); b[0, 0], b[1, 0] = 0.31, -1.0
        inst = Instance("i", 2, np.zeros(2), np.ones(2), cost, [a, b], [], eps=1e-6, delta=1e-3,
                        eps_eq=1e-6, max_boxes=1 << 12)
        return solve(inst)[1] == ref.INFEASIBLE
    check("infeasible", infeasible)

    # a feasible small instance: the returned box's centre is feasible, the
    # stopping width holds, and the list ids are distinct and in range
    def small():
        inst = make_instance(0, 2)
        s = ref.RefSolver(inst, L=L)
        for _ in range(200):
            out = s.step()
            r = s.result()
            ids, _ = s.list()
            if len(ids) and len(np.unique(ids, axis=0)) != len(ids):
                return False
            if np.any(ids >= (np.uint64(1) << r["depth"].astype(np.uint64))):
                return False
            if out != ref.RUNNING:
                break
        c = 0.5 * (r["x_lo"] + r["x_hi"])
        return out == ref.OPTIMAL and all(poly_eval(g, c) <= 0 for g in inst.ineq) and \
            np.max(r["x_hi"] - r["x_lo"]) <= inst.delta and \
            np.max(r["x_hi"] - r["x_lo"]) > inst.delta / 4 and \
            r["p_lo"] - 1e-12 <= poly_eval(inst.cost, c) <= r["p_up"] + 1e-12
    check("small_invariants", small)

    # round mode: the round split against exact sub-boxes, the round-end state
    # against the one-direction passes, and its memory test
    def round_split():
        rng = np.random.default_rng(6)
        mono = rng.integers(-5, 6, size=(4, 6))
        P = ref.to_bernstein(mono.astype(float), [-1.0, -1.0], [1.0, 1.0], L=L)
        kids = ref.split_round(P, L=L)
        for c in range(4):
            blo = [0.0 if (c >> (1 - k)) & 1 else -1.0 for k in range(2)]
            bhi = [1.0 if (c >> (1 - k)) & 1 else 0.0 for k in range(2)]
            want = exact.to_float(exact.bernstein_exact(mono, blo, bhi))
            if np.max(np.abs(kids[c] - want)) > 1e-12 * max(1, np.abs(want).max()):
                return False
        return True
    check("round_split", round_split)

    def round_ends():
        inst = make_instance(0, 3)
        o = ref.RefSolver(inst, L=L)
        f = ref.RefSolver(inst, L=L, fused=True)
        for _ in range(10):
            o.step()
            o.step()
            f.step()
            ro, rf = o.result(), f.result()
            if ro["p_up"] != rf["p_up"] or ro["p_lo"] != rf["p_lo"] or \
                    not np.array_equal(ro["depth"], rf["depth"]) or \
                    not np.array_equal(o.list()[0], f.list()[0]):
                return False
        return True
    check("round_ends", round_ends)

    def round_memory():
        f = ref.RefSolver(make_instance(0, 5).with_options(max_boxes=64), L=L, fused=True)
        out = f.solve()
        r = f.result()
        return out == ref.MEMORY_LIMIT and 4 * r["list_len"] > 64 and 2 * r["list_len"] <= 64
    check("round_memory", round_memory)

    # subdivision at a parameter lambda: both parts against exact Bernstein
    # coefficients over [a, a + lambda (b-a)] and [a + lambda (b-a), b]
    def split_lambda():
        rng = np.random.default_rng(12)
        mono = rng.integers(-5, 6, size=(5, 4))
        lo, hi = [-1.0, 0.0], [1.0, 2.0]
        P = ref.to_bernstein(mono.astype(float), lo, hi, L=L)
        for r, lam in ((0, 0.25), (1, 0.375), (0, 0.75)):
            left, right = ref.split_at(P, r, lam, L=L)
            cut = lo[r] + lam * (hi[r] - lo[r])
            hl = list(hi); hl[r] = cut
            lr = list(lo); lr[r] = cut
            wl = exact.to_float(exact.bernstein_exact(mono, lo, hl))
            wr = exact.to_float(exact.bernstein_exact(mono, lr, hi))
            if np.max(np.abs(left - wl)) > 1e-12 * max(1, np.abs(wl).max()):
                return False
            if np.max(np.abs(right - wr)) > 1e-12 * max(1, np.abs(wr).max()):
                return False
        return True
    check("split_lambda", split_lambda)

    # a solve at lambda = 3/8: the returned box contains the planted minimiser's
    # value within the bracket, and its reported interval is the box of its id
    def lambda_solve():
        p = next(q for q in pp.load()["objectives"] if q["name"] == "DP2")
        inst = pp.planted_constraint_instance(p, 10, seed=3)
        s = ref.RefSolver(inst, L=L, lam=0.375, eps=1e-4, delta=1e-3, eps_eq=1e-6, max_boxes=1 << 16,
                          max_iters=28)
        out = s.solve()
        r = s.result()
        c = 0.5 * (r["x_lo"] + r["x_hi"])
        widest = max((inst.hi[k] - inst.lo[k]) * 0.625 ** r["depth"][k] for k in range(2))
        return out == ref.OPTIMAL and r["p_lo"] <= 1e-9 and r["p_up"] <= 1e-4 + 1e-9 and \
            all(poly_eval(g, c) <= 0 for g in inst.ineq) and widest <= 1e-3 and \
            r["p_lo"] - 1e-12 <= poly_eval(inst.cost, c) <= r["p_up"] + 1e-12
    check("lambda_solve", lambda_solve)

    # maximum-width rule on a box four times wider along x1: the direction
    # follows the widths of the boxes
    def maxwidth_order():
        cost = np.zeros((3, 3)); cost[2, 0] = 1.0; cost[0, 2] = 1.0
        inst = Instance("w", 2, np.array([-2.0, -0.5]), np.array([2.0, 0.5]), cost, [], [],
                        eps=1e-6, delta=1e-3, eps_eq=1e-6, max_boxes=1 << 16)
        s = ref.RefSolver(inst, L=L, rule=1)
        seq = [s.result()["next_dir"]]
        for _ in range(8):
            s.step()
            seq.append(s.result()["next_dir"])
        # widths (4,1) -> (2,1) -> (1,1), a tie to x1 -> (1/2,1) -> then alternating
        return seq[:6] == [0, 0, 0, 1, 0, 1]
    check("maxwidth_order", maxwidth_order)
    return failed


@pytest.fixture(scope="module")
def tmpdir_mut():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_clean_source_passes_the_battery(tmpdir_mut):
    assert battery(build_variant(None, tmpdir_mut)) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmpdir_mut):
    failed = battery(build_variant(name, tmpdir_mut))
    assert failed, f"mutation {name} passed every pin"
