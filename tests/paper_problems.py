"""Builds Instance objects from the paper's printed problems (tests/golden).

Expressions are expanded to monomial tensors with sympy; nothing here does
Bernstein arithmetic."""
from __future__ import annotations

import json
import os

import numpy as np
import sympy as sp

from paper_2003_01758_amd.instances import Instance, poly_eval

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_problems.json")
X = sp.symbols("x1:9")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def _namespace(nv, defs=None):
    ns = {f"x{i + 1}": X[i] for i in range(nv)}
    ns["pi"] = sp.pi
    for k, v in (defs or {}).items():
        ns[k] = sp.sympify(v, locals=ns)
    return ns


def to_tensor(expr, nv: int) -> np.ndarray:
    poly = sp.Poly(sp.expand(expr), *X[:nv])
    degs = [max([m[k] for m in poly.monoms()] + [0]) for k in range(nv)]
    t = np.zeros([d + 1 for d in degs])
    for mon, c in zip(poly.monoms(), poly.coeffs()):
        t[tuple(mon)] += float(c)
    return t


def x_opt(p) -> np.ndarray:
    if "x_opt" in p:
        return np.array(p["x_opt"], dtype=float)
    return np.array([float(sp.sympify(e)) for e in p["x_opt_expr"]])


def benchmark_instance(p, **kw) -> Instance:
    nv = p["vars"]
    ns = _namespace(nv, p.get("defs"))
    cost = to_tensor(sp.sympify(p["cost"], locals=ns), nv)
    ineq = [to_tensor(sp.sympify(g, locals=ns), nv) for g in p.get("ineq", [])]
    eq = [to_tensor(sp.sympify(h, locals=ns), nv) for h in p.get("eq", [])]
    lo = np.array(p["lo"], dtype=float)
    hi = np.array(p["hi"], dtype=float)
    return Instance(p["name"], nv, lo, hi, cost, ineq, eq, **kw)


def planted_constraint_instance(p, n_constraints: int, seed: int, margin=(0.1, 0.5),
                                **kw) -> Instance:
    """Objective p with random degree-2 constraints planted feasible at the
    printed optimiser: g_temp has every monomial of total degree <= 2 with a
    coefficient uniform in [-5,5], and g = g_temp - g_temp(x*) (Sec. V-C), minus
    a margin drawn from U(margin) so that x* is strictly feasible.  (With the
    margin at zero every constraint is active at x*, the feasible set near x* has
    an empty interior, and no box around x* can ever be certified feasible.)"""
    nv = p["vars"]
    ns = _namespace(nv)
    cost = to_tensor(sp.sympify(p["cost"], locals=ns), nv)
    xs = x_opt(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    ineq = []
    for _ in range(n_constraints):
        g = np.zeros((3,) * nv)
        for idx in np.ndindex(*g.shape):
            if sum(idx) <= 2:
                g[idx] = rng.uniform(-5.0, 5.0)
        g[(0,) * nv] -= poly_eval(g, xs) + (rng.uniform(*margin) if margin else 0.0)
        ineq.append(g)
    return Instance(p["name"], nv, np.array(p["lo"], float), np.array(p["hi"], float),
                    cost, ineq, [], q0=xs, **kw)
