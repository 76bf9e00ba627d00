#!/usr/bin/env python3
"""Benchmark of the PCBA hot path on one MI355X.

Workload: batches of RTD-shaped plans (2 decision variables on [-1,1]^2, a
goal-distance cost of multi-degree (6,6), 500 obstacle constraints of
multi-degree (10,10); eps 1e-3, delta 1e-4, M 2^20, N 28), seeded synthetic
instances.  One step = every problem of the batch solved from its root item to
a certified outcome: root conversion on the device, then memory test,
subdivision + bounds, cut-off test + compaction, stopping tests, FP64
certification, then every plan's result record copied into one host array.
Inputs are resident in device memory when the timed region starts
(pcba_reset recomputes the root patches from the resident monomials).

Prints one JSON line: certified solves/s of the best of the FP32 path
(rigorously widened bounds, FP64 certification; the split by de Casteljau on
the vector ALUs or as products on the matrix cores) and the plain FP64 path, with
p50/p99 per-plan latency, both paths' figures, the roofline of the dominant
kernel (HIP events around its launches over a second, instrumented pass of the
same steps), and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import gc
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "certified solves/s + p99 latency at opt tol 1e-3, FP32-MFMA vs FP64 plain"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def certified(r, pcba, precision):
    """OPTIMAL with the FP64 certificate of x*, or INFEASIBLE decided on
    rigorously widened bounds (the FP32 path; FP64 plain bounds are unwidened,
    so its infeasibility verdicts are not counted)."""
    return (r["outcome"] == pcba.OPTIMAL and bool(r["certified"])) or \
        (r["outcome"] == pcba.INFEASIBLE and precision == "fp32")


def count_certified(res, pcba, precision):
    """certified() over a structured result array."""
    ok = (res["outcome"] == pcba.OPTIMAL) & (res["certified"] != 0)
    if precision == "fp32":
        ok = ok | (res["outcome"] == pcba.INFEASIBLE)
    return int(np.count_nonzero(ok))


def patch_words(inst):
    """Coefficients per patch of each kind (each kind at its common multi-degree)."""
    def size(degs):
        return int(np.prod(np.max(np.atleast_2d(degs), axis=0) + 1)) if len(degs) else 0
    return int(np.prod(np.array(inst.cost.shape))), size(inst.ineq_deg), size(inst.eq_deg)


def algorithmic_bytes(p, inst, precision):
    """Bytes the subdivide+bound kernel must move over the last solve: every
    parent's carried patches read once and every kept child's carried patches
    written once (plus, in FP32, one error term per such patch).  Steps that
    ran in the FP32 re-derivation kernel instead are left out."""
    s0, s1, s2 = patch_words(inst)
    el = 4 if precision == "fp32" else 8
    tr, pt = p.trace(), p.trace_patches()
    total = 0.0
    for q in range(len(tr["k_in"])):
        if precision == "fp32" and p.options.rederive_every > 0 and (q + 1) % p.options.rederive_every == 0:
            continue
        items = float(tr["k_in"][q] + tr["k_kept"][q])
        ineq = float(pt["a_in"][q] + pt["a_kept"][q])
        total += items * (s0 + inst.n_eq * s2) * el + ineq * s1 * el
        if precision == "fp32":
            total += (items * (1 + inst.n_eq) + ineq) * 4
    return total


def warm(pcba, insts, precision, warmup, **opts):
    """The batch's problems, created and solved `warmup` times (untimed)."""
    probs = [pcba.Problem(i, precision=precision, **opts) for i in insts]
    for w in range(warmup):
        pcba.reset_batch(probs)
        pcba.solve_batch(probs)
        log(f"[bench] {precision} warmup {w + 1}/{warmup} done")
    return probs


def run_mode(pcba, probs, insts, precision, steps):
    """Times `steps` batch solves (throughput and latency, no instrumentation),
    then repeats them with HIP events around every kernel launch for the
    per-kernel times and the roofline of the subdivide+bound kernel."""
    lat, cert, results = [], 0, []
    elapsed = 0.0
    # the timed solves measure the library: no Python garbage collection
    # inside, the handle array built once, and every plan's result copied
    # into one host array by a single call (pcba_result_batch)
    batch = pcba.Batch(probs)
    gc.collect()
    gc.disable()
    for s in range(steps):
        t0 = time.perf_counter()
        pcba.reset_batch(batch)
        res = pcba.solve_batch(batch, as_array=True)
        elapsed += time.perf_counter() - t0
        lat += res["seconds"].tolist()
        cert += count_certified(res, pcba, precision)
        results = res
        log(f"[bench] {precision} step {s + 1}/{steps}: {elapsed * 1e3 / (s + 1):.2f} ms/step")
    gc.enable()
    # the same steps with every launch bracketed by HIP events on the library's stream
    sub_kernel = "sub_fp32" if precision == "fp32" else "sub_fp64"
    bytes_sub = 0.0
    pcba.profile_reset()
    pcba.profile_enable(True)
    prof_elapsed = 0.0
    for s in range(steps):
        t0 = time.perf_counter()
        pcba.reset_batch(batch)
        pcba.solve_batch(batch, as_array=True)
        prof_elapsed += time.perf_counter() - t0
        for p, i in zip(probs, insts):
            bytes_sub += algorithmic_bytes(p, i, precision)
    pcba.profile_enable(False)
    prof = pcba.profile_read()
    log(f"[bench] {precision} instrumented pass: {prof_elapsed * 1e3 / steps:.2f} ms/step")
    for p in probs:
        p.close()
    ms_sub, n_sub = prof[sub_kernel]
    return dict(
        solves_per_s=cert / elapsed,
        ms_per_step=elapsed * 1e3 / steps,
        p50_ms=float(np.percentile(lat, 50) * 1e3),
        p99_ms=float(np.percentile(lat, 99) * 1e3),
        certified=cert, total=len(lat),
        results=results, profile=prof,
        sub_kernel=sub_kernel, bytes_sub=bytes_sub, ms_sub=ms_sub, launches_sub=n_sub,
        instrumented_ms_per_step=prof_elapsed * 1e3 / steps,
    )


def single_plan(pcba, inst, precision, reps, **opts):
    """One plan solved alone, `reps` times (after one warm-up): per-solve wall
    time from reset to certified result, and whether every solve certified."""
    p = pcba.Problem(inst, precision=precision, **opts)
    pcba.reset_batch([p])
    pcba.solve_batch([p])
    t, ok = [], True
    gc.collect()
    gc.disable()
    for _ in range(reps):
        t0 = time.perf_counter()
        pcba.reset_batch([p])
        r = pcba.solve_batch([p])[0]
        t.append(time.perf_counter() - t0)
        ok = ok and certified(r, pcba, precision)
    gc.enable()
    p.close()
    return {"p50_ms": round(float(np.percentile(t, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(t, 99)) * 1e3, 4), "certified": ok, "reps": reps}


def measured_traffic(mode_name, kernel):
    """HBM bytes per launch of a mode's subdivide kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE runs scaled by a copy of known
    size), or None when the kernel source has changed since the counters were
    taken or the mode was not counted."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sub_rtd256_r0_hbm_bytes.md")
    try:
        line = [ln for ln in open(path) if ln.strip().startswith("{")][-1]
        rec = json.loads(line)
    except (OSError, IndexError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2003_01758_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernels_hip_sha256"):
        return None
    k = rec.get("modes", {}).get(mode_name)
    if not k or k.get("kernel") != kernel:
        return None
    return float(k["bytes_per_dispatch"])


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


_ORACLE_INSTS = []   # set before the worker processes fork


def _oracle_solve(i):
    from oracle import ref
    s = ref.RefSolver(_ORACLE_INSTS[i])
    s.solve()
    r = s.result()
    certified = r["outcome"] == ref.OPTIMAL or r["outcome"] == ref.INFEASIBLE
    return r["p_up"], certified


def cpu_baseline(insts, budget_s, workers):
    """The FP64 oracle on the host: independent plans solved by a pool of
    worker processes (one per core of the share), submitted until the time
    budget is spent; the rate counts every plan finished by then."""
    import multiprocessing as mp
    from oracle import ref
    ref.lib()   # built before the workers start
    _ORACLE_INSTS[:] = insts
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    done, p_up = 0, {}
    with ctx.Pool(workers) as pool:
        pending = []
        k = 0
        while True:
            while len(pending) < 2 * workers and time.perf_counter() - t0 < budget_s:
                i = k % len(insts)
                pending.append((i, pool.apply_async(_oracle_solve, (i,))))
                k += 1
            if not pending:
                break
            i, a = pending.pop(0)
            pu, ok = a.get()
            done += 1 if ok else 0
            p_up.setdefault(i, pu)
            if time.perf_counter() - t0 >= budget_s and all(x[1].ready() for x in pending):
                for j, b in pending:
                    pu, ok = b.get()
                    done += 1 if ok else 0
                    p_up.setdefault(j, pu)
                break
    dt = time.perf_counter() - t0
    return done / dt, done, dt, p_up


def copy_calibration(mib: int, reps: int):
    """Device-to-device copies of a known size: the reference reading for the
    hardware byte counters (FETCH_SIZE, WRITE_SIZE) under rocprofv3."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    n = mib << 20
    a, b = C.c_void_p(), C.c_void_p()
    if hip.hipMalloc(C.byref(a), C.c_size_t(n)) or hip.hipMalloc(C.byref(b), C.c_size_t(n)):
        sys.exit("hipMalloc failed")
    hip.hipMemset(a, 1, C.c_size_t(n))
    hip.hipDeviceSynchronize()
    for _ in range(reps):
        hip.hipMemcpy(b, a, C.c_size_t(n), 3)   # device to device
    hip.hipDeviceSynchronize()
    hip.hipFree(a)
    hip.hipFree(b)
    print(json.dumps({"copy_bytes": n, "copies": reps}), flush=True)


def cut_scaling(max_steps: int = 80, max_children: int = 600000):
    """The cut kernel's time per step against the step's children, on the 4-D
    workload (100 inequalities, 2 equalities, M 2^21, retiring on), with the cut
    in one workgroup per problem and split across workgroups: one JSON line per
    step (HIP events around the cut's launches)."""
    from paper_2003_01758_amd import pcba
    from paper_2003_01758_amd.instances import make_instance
    rows = {}
    for mode, split in (("one", 0), ("split", 32768)):
        pcba.set_cut_split(split, 4096)
        g = pcba.Problem(make_instance(2, 0).with_options(max_boxes=1 << 21), retire_satisfied=1)
        pcba.profile_enable(True)
        for step in range(max_steps):
            pcba.profile_reset()
            r = g.step(1)
            ms, n = pcba.profile_read()["cut"]
            kin = int(g.trace()["k_in"][step])
            rows.setdefault(step, {})[mode] = (2 * kin, ms * 1e3, n)
            if r["outcome"] != pcba.RUNNING or 2 * kin > max_children:
                break
        pcba.profile_enable(False)
        g.close()
    pcba.set_cut_split()
    for step in sorted(rows):
        d = rows[step]
        if "one" in d and "split" in d and d["one"][0] == d["split"][0]:
            c = d["one"][0]
            print(json.dumps({"step": step, "children": c, "cut_us_one_workgroup": round(d["one"][1], 2),
                              "cut_us_split": round(d["split"][1], 2),
                              "ns_per_child_one": round(1e3 * d["one"][1] / max(c, 1), 3),
                              "ns_per_child_split": round(1e3 * d["split"][1] / max(c, 1), 3)}), flush=True)


MODE_FLAGS = {
    "r0": ("retire_satisfied", 0),   # every box carries every constraint (Alg. Subdivision)
    "r1": ("retire_satisfied", 1),   # constraints certified satisfied on a box are dropped
    "f1": ("fused_round", 1),        # each pass splits both axes: S_a P S_b^T, one cut per round
    "s1": ("stale_filter", 1),       # children already above the previous estimate are not written
    "mm": ("split_engine", 1),       # FP32 split on the matrix cores (default: de Casteljau on the VALUs)
}


def parse_modes(spec):
    """'fp64:r0,fp32:r0,...' -> [(name, precision, options)]."""
    out = []
    for tok in spec.split(","):
        tok = tok.strip()
        if not tok:
            continue
        parts = tok.split(":")
        prec = parts[0]
        if prec not in ("fp64", "fp32"):
            raise SystemExit(f"unknown precision in mode {tok!r}")
        opts = {}
        for f in parts[1:]:
            if f not in MODE_FLAGS:
                raise SystemExit(f"unknown flag {f!r} in mode {tok!r}")
            k, v = MODE_FLAGS[f]
            opts[k] = v
        out.append((tok, prec, opts))
    return out


def roofline_of(mode_name, r):
    achieved = r["bytes_sub"] / (r["ms_sub"] * 1e-3) / 1e9 if r["ms_sub"] > 0 else None
    return {
        "kernel": r["sub_kernel"],
        "bound": "hbm",
        "achieved": round(achieved, 2) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": measured_traffic(mode_name, r["sub_kernel"]),
        "bytes_per_launch": round(r["bytes_sub"] / max(1, r["launches_sub"]), 1),
        "avg_launch_us": round(r["ms_sub"] * 1e3 / max(1, r["launches_sub"]), 3),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="oracle worker processes (the host's share of cores)")
    ap.add_argument("--rederive", type=int, default=None, help="FP32 re-derivation period (steps)")
    ap.add_argument("--stale", type=int, default=None, help="1/0: stale-estimate write filter")
    ap.add_argument("--cut-scaling", action="store_true",
                    help="only measure the cut kernel against the list length (4-D workload) and exit")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run device copies of this many MiB (counter calibration) and exit")
    ap.add_argument("--tune", type=int, default=1,
                    help="each mode's launch shape (tile size, workgroups per CU, FP32 re-derivation "
                         "period): 1 the tuned shape kept with the package, tuned now where it has "
                         "none; 2 tuned now; 0 the library's defaults")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned shapes to read and to write tuning results to "
                         "(default: the package's, read only)")
    ap.add_argument("--single-reps", type=int, default=20,
                    help="solves of one plan alone per headline precision for the single-plan latency (0: skip)")
    ap.add_argument("--modes", default="fp64:r0,fp32:r0,fp32:r0:mm,fp64:r0:f1,fp32:r0:f1,fp64:r1,fp32:r1,fp32:r1:mm",
                    help="comma-separated modes precision[:flag...]; flags: " + ", ".join(MODE_FLAGS) +
                         ". The headline is the best mode that transforms every constraint (r0)")
    args = ap.parse_args()
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib, 2)
        return
    if args.cut_scaling:
        cut_scaling()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    from paper_2003_01758_amd import pcba
    from paper_2003_01758_amd.instances import make_instance

    modes = parse_modes(args.modes)
    insts = [make_instance(1, k) for k in range(args.batch)]
    log(f"[bench] {len(insts)} rtd-shaped plans, {insts[0].n_ineq} constraints, "
        f"{insts[0].words_per_item()} words per item; modes {[m[0] for m in modes]}")
    common = {}
    if args.stale is not None:
        common["stale_filter"] = args.stale
    results = {}
    for name, prec, opts in modes:
        o = dict(common)
        o.update(opts)
        if prec == "fp32" and args.rederive is not None:
            o["rederive_every"] = args.rederive
        if args.tune:
            from paper_2003_01758_amd import tune
            cache = tune.Cache(args.tune_cache or tune.DEFAULT_CACHE)
            o = tune.tuned_options(insts, prec, o, cache=cache, reps=3, log=log, retune=args.tune == 2,
                                   write=args.tune_cache is not None)
            log(f"[bench] {name}: tuned options {o}")
        probs = warm(pcba, insts, prec, args.warmup, **o)
        r = run_mode(pcba, probs, insts, prec, args.steps)
        r["precision"], r["options"] = prec, o
        results[name] = r
        log(f"[bench] {name}: {r['solves_per_s']:.1f} certified solves/s, "
            f"p50/p99 {r['p50_ms']:.2f}/{r['p99_ms']:.2f} ms")

    # the headline: the best mode on the path every constraint is transformed
    # in (no retiring); otherwise the best mode measured
    hot = [n for n, _, o in modes if o.get("retire_satisfied", 1) == 0] or list(results)
    head = max(hot, key=lambda n: results[n]["solves_per_s"])
    best = results[head]

    single = None
    if args.single_reps > 0:
        single = {}
        for name in hot:
            r = results[name]
            single[name] = single_plan(pcba, insts[0], r["precision"], args.single_reps, **r["options"])

    # parity of the GPU paths on the last batch (all provably within eps of f*)
    dp = 0.0
    names = list(results)
    for a in names:
        for b in names:
            for x, y in zip(results[a]["results"], results[b]["results"]):
                if x["outcome"] == y["outcome"] == pcba.OPTIMAL:
                    dp = max(dp, abs(x["p_up"] - y["p_up"]))

    def summary(name):
        r = results[name]
        d = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
             if k in ("solves_per_s", "ms_per_step", "p50_ms", "p99_ms", "certified", "total",
                      "instrumented_ms_per_step")}
        d["options"] = r["options"]
        d["precision"] = r["precision"]
        d["kernel_ms"] = {k: round(v[0], 3) for k, v in r["profile"].items()}
        d["kernel_launches"] = {k: v[1] for k, v in r["profile"].items()}
        d["roofline"] = roofline_of(name, r)
        return d

    out = {
        "metric": METRIC,
        "value": round(best["solves_per_s"], 3),
        "unit": "certified solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(best["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if best["precision"] == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "rtd-shaped plans: l=2 on [-1,1]^2, goal-distance cost (6,6), "
                        "500 obstacle constraints (10,10), eps 1e-3, delta 1e-4, M 2^20, N 28",
            "batch": args.batch,
            "mode": head,
            "options": best["options"],
            "path": ("fp32 patches with rigorous widening + fp64 root, re-derivation and certification"
                     if best["precision"] == "fp32" else "fp64 plain") +
                    ("; every constraint transformed at every step" if best["options"].get("retire_satisfied", 1) == 0
                     else "; constraints certified satisfied on a box are dropped"),
        },
        "p50_ms": round(best["p50_ms"], 4),
        "p99_ms": round(best["p99_ms"], 4),
        "certified": f"{best['certified']}/{best['total']}",
        "modes": {n: summary(n) for n in results},
        "max_abs_p_between_modes": dp,
        # the metric's comparison on the hot path (every constraint transformed):
        # FP32 split on the matrix cores and on the vector ALUs against FP64 plain
        "fp32_vs_fp64_r0": {n: {"solves_per_s": round(results[n]["solves_per_s"], 3),
                                "p99_ms": round(results[n]["p99_ms"], 4)} for n in hot},
        "single_plan": single,
        "roofline": roofline_of(head, best),
    }
    if not args.no_cpu:
        rate, n, dt, p_ref = cpu_baseline(insts, args.cpu_seconds, args.cpu_workers)
        out["cpu_baseline"] = {
            "value": round(rate, 4), "unit": "certified solves/s", "cores": args.cpu_workers, "kind": "oracle",
            "sample": f"{n} solves of the {len(insts)} plans (cycled) in {dt:.1f} s, FP64 oracle, "
                      f"{args.cpu_workers} worker processes on {cpu_model()} "
                      f"({os.cpu_count()} logical CPUs visible)",
        }
        drefs = []
        for name, r in results.items():
            # FP64 plain one-direction modes repeat the oracle's operations (round
            # mode ends at round boundaries: within eps, not equal)
            if r["precision"] == "fp64" and not r["options"].get("fused_round", 0):
                drefs += [abs(r["results"][i]["p_up"] - pu) for i, pu in p_ref.items()
                          if r["results"][i]["outcome"] == pcba.OPTIMAL]
        out["max_abs_p_fp64_vs_oracle"] = max(drefs) if drefs else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
