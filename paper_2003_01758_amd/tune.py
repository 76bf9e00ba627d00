"""Autotuner of the launch shape of the subdivision kernel.

A class of problems (dimension, multi-degrees, a bucket of the inequality
count, precision, retiring, round mode) is tuned on a sample of its problems:
each candidate shape -- coefficients per tile (`tile_coefs`), workgroups per
compute unit (`wg_per_cu`) and, in FP32 mode, the steps between FP64
re-derivations (`rederive_every`) -- solves the sample as one batch a few
times, timed on the host around each batched solve, and the fastest median
wins.  The tile size and the workgroup count change how the work is cut, not
what is computed: FP64 results are the same bit for bit under every shape (a
fibre's de Casteljau steps do not depend on which tile holds it), and FP32
bounds stay rigorous.  Choices are kept in a JSON cache keyed by the class.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import pcba

# candidate shapes: tile sizes around the default (2,816 coefficients per FP64
# tile, twice that in FP32, half in a round of l = 2), one or two workgroups
# per compute unit
TILES = {"fp64": (1408, 2048, 2816, 3584), "fp32": (2816, 4096, 5632, 7168)}
WGS = (0, 1)
REDERIVE = (8, 16, 32, 0)   # directional steps between FP64 re-derivations (halved for rounds; 0 never)


def class_key(inst, precision: str, opts: dict) -> str:
    """The class a problem is tuned in."""
    degs = [list(inst.cost.shape)]
    if inst.n_ineq:
        degs.append([int(d) + 1 for d in np.max(inst.ineq_deg, axis=0)])
    if inst.n_eq:
        degs.append([int(d) + 1 for d in np.max(inst.eq_deg, axis=0)])
    bucket = 0 if inst.n_ineq == 0 else int(round(math.log2(inst.n_ineq)))
    return json.dumps({"l": int(inst.l), "sizes": degs, "ineq_log2": bucket, "eq": int(inst.n_eq),
                       "precision": precision, "retire": int(opts.get("retire_satisfied", 1)),
                       "round": int(opts.get("fused_round", 0)),
                       "mfma": int(opts.get("split_engine", 0)) if precision == "fp32" else 0},
                      sort_keys=True)


def candidates(precision: str, opts: dict, l: int):
    """Candidate launch shapes for a class (tile sizes a round can hold only)."""
    tiles = TILES[precision]
    if opts.get("fused_round", 0):
        cap = 2 * tiles[-1] // (1 << l)
        tiles = tuple(t for t in tiles if t <= cap) or (cap,)
    return [{"tile_coefs": t, "wg_per_cu": w} for t in tiles for w in WGS]


def _certified(res, precision):
    ok = (res["outcome"] == pcba.OPTIMAL) & (res["certified"] != 0)
    if precision == "fp32":
        ok = ok | (res["outcome"] == pcba.INFEASIBLE)
    return int(np.count_nonzero(ok))


def _time_batch(insts, precision, opts, reps, limit_s=0.0, need=0):
    """Median seconds of `reps` batched solves after one untimed solve, and the
    problems certified; with limit_s, every problem carries that time limit, so
    a shape that makes the solve far slower than the default ends early (its
    problems stop with TIMEOUT) instead of running on.  A candidate that
    certifies fewer than `need` problems (a re-derivation period whose FP32
    bounds outgrow eps before delta is reached) is not a candidate either."""
    if limit_s > 0:
        opts = dict(opts, time_limit_s=limit_s)
    probs = [pcba.Problem(i, precision=precision, **opts) for i in insts]
    batch = pcba.Batch(probs)
    pcba.reset_batch(batch)
    res = pcba.solve_batch(batch, as_array=True)     # first solve: list growth, caches
    cert = _certified(res, precision)
    times = [math.inf] if cert < need else []
    for _ in range(reps if cert >= need else 0):
        t0 = time.perf_counter()
        pcba.reset_batch(batch)
        res = pcba.solve_batch(batch, as_array=True)
        times.append(time.perf_counter() - t0)
        if np.any(res["outcome"] == pcba.TIMEOUT):
            times = [math.inf]     # stopped by the limit: not a candidate
            break
    for p in probs:
        p.close()
    return float(np.median(times)), cert


def tune(insts, precision: str, opts: dict, reps: int = 3, log=None) -> dict:
    """The fastest candidate shape for the batch `insts` (the options in opts
    fixed); returns the shape with its median batch time and the default's.
    Candidates must certify as many problems as the default does."""
    base, need = _time_batch(insts, precision, opts, reps)
    best = {"shape": {}, "seconds": base}

    def trial(cand):
        o = dict(opts)
        o.update(cand)
        t, _ = _time_batch(insts, precision, o, reps, limit_s=4.0 * base + 0.05, need=need)
        if log:
            log(f"[tune] {precision} {cand}: {t * 1e3:.2f} ms")
        if t < best["seconds"]:
            best["shape"], best["seconds"] = cand, t

    # the launch shape first, then (FP32) the re-derivation period under it
    for cand in candidates(precision, opts, int(insts[0].l)):
        trial(cand)
    if precision == "fp32" and "rederive_every" not in opts:
        shape = dict(best["shape"])
        per = 2 if opts.get("fused_round", 0) else 1    # a round is two directional steps
        for r in REDERIVE:
            trial(dict(shape, rederive_every=max(1, r // per) if r else 0))
    best["default_seconds"] = base
    return best


# tuned shapes kept with the package, written from measured runs
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


class Cache:
    """Tuned shapes by class, in a JSON file."""

    def __init__(self, path: str):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, rec: dict, write: bool = True):
        self.data[key] = rec
        if not write:
            return
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(self.path, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)


def tuned_options(insts, precision: str, opts: dict, cache: Cache | None = None, reps: int = 3, log=None,
                  retune: bool = False, write: bool = True) -> dict:
    """opts plus the tuned shape of the class of insts[0]: the cache's entry,
    or (none, or retune) one tuned on insts and put in the cache (written to
    its file if `write`)."""
    key = class_key(insts[0], precision, opts)
    rec = None if (retune or cache is None) else cache.get(key)
    if rec is None:
        rec = tune(insts, precision, opts, reps=reps, log=log)
        if cache:
            cache.put(key, rec, write=write)
    elif log:
        log(f"[tune] {precision}: shape from the cache: {rec['shape']}")
    out = dict(opts)
    out.update(rec["shape"])
    return out
