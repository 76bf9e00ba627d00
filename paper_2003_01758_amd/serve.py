"""Receding-horizon serving loop over the PCBA engine (continuous batching).

Plans arrive as a Poisson process.  Each arrival is turned into a problem
(host-to-device upload of its monomials and the FP64 root conversion), queued,
and admitted into the engine as soon as its device footprint fits the budget.
Every engine round advances all admitted, unfinished plans together by a few
PCBA steps; finished plans are certified and handed back, freeing their share
of the budget for the next admissions.  The replanning period of the paper's
receding-horizon planner (a new plan every 0.5 s, a solver budget of 0.4 s,
Sec. VI) motivates the per-plan deadline.

Usage: python -m paper_2003_01758_amd.serve --rate 200 --duration 60
       python -m paper_2003_01758_amd.serve --sweep 500,1000,2000,4000 --duration 10
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time

import numpy as np

from . import pcba
from .instances import make_instance


def poisson_arrivals(rate: float, duration: float, seed: int = 0):
    """Arrival times of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


class Server:
    """Continuous batching of plan requests on one GPU."""

    def __init__(self, budget_bytes: int, reserve_boxes: int = 256, steps_per_round: int = 2,
                 precision: str = "fp32", deadline_s: float = 0.5, max_waiting: int = 64, **options):
        self.engine = pcba.Engine(budget_bytes=budget_bytes, reserve_boxes=reserve_boxes)
        self.steps = steps_per_round
        # problems created (device memory held) but not yet admitted: arrivals
        # beyond these wait as requests, so an overload grows a host queue, not
        # device allocations
        self.max_waiting = max_waiting
        self.precision = precision
        self.deadline = deadline_s
        self.options = options

    def serve(self, requests, arrivals, log=None):
        """requests[i] is an Instance arriving at arrivals[i] seconds after the
        start.  Returns one record per request: arrival, completion, latency,
        outcome, certified, p_up, deadline_missed."""
        order = np.argsort(arrivals)
        pending = collections.deque((float(arrivals[i]), int(i)) for i in order)
        queue = collections.deque()
        inflight = {}
        records = [None] * len(requests)
        t0 = time.perf_counter()
        n_done = 0
        last_log = t0
        while n_done < len(requests):
            now = time.perf_counter() - t0
            # arrivals up to now become problems on the device
            while pending and pending[0][0] <= now and len(queue) < self.max_waiting:
                ta, i = pending.popleft()
                prob = pcba.Problem(requests[i], precision=self.precision,
                                    time_limit_s=self.deadline, **self.options)
                queue.append((ta, i, prob))
            # admission while the footprint budget allows
            while queue and self.engine.submit(queue[0][2]):
                ta, i, prob = queue.popleft()
                inflight[prob.h.value] = (ta, i, prob)
            if inflight:
                self.engine.run(self.steps)
                done = self.engine.poll(len(inflight))
                tdone = time.perf_counter() - t0
                for prob in done:
                    ta, i, _ = inflight.pop(prob.h.value)
                    r = prob.result()
                    lat = tdone - ta
                    # an infeasibility verdict is rigorous only on widened (FP32) bounds
                    certified = (r["outcome"] == pcba.OPTIMAL and r["certified"]) or \
                        (r["outcome"] == pcba.INFEASIBLE and self.precision == "fp32")
                    records[i] = dict(arrival=ta, done=tdone, latency=lat, outcome=r["outcome"],
                                      certified=bool(certified), p_up=r["p_up"], p_lo=r["p_lo"],
                                      steps=r["steps"], x_index=[int(v) for v in r["x_index"]],
                                      deadline_missed=bool(lat > self.deadline or not certified))
                    prob.close()
                    n_done += 1
            elif pending and not queue:
                # idle until the next arrival
                time.sleep(max(0.0, min(pending[0][0] - now, 0.001)))
            if log and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log(f"[serve] t={now:.1f}s done {n_done}/{len(requests)} in flight {len(inflight)} "
                    f"queued {len(queue)} used {self.engine.used_bytes() / 2**30:.2f} GiB")
        return records


def summarize(records, duration):
    lat = np.array([r["latency"] for r in records])
    cert = sum(r["certified"] for r in records)
    span = max(r["done"] for r in records)
    return dict(plans=len(records), certified=int(cert),
                certified_solves_per_s=cert / span,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                deadline_miss_rate=float(np.mean([r["deadline_missed"] for r in records])),
                wall_s=span, offered_s=duration)


def sweep(args, log):
    """Saturation: the highest Poisson arrival rate whose p99 latency (arrival
    to certified result) stays within the deadline with every plan certified."""
    pool = [make_instance(4, args.seed * 100000 + k) for k in range(args.pool)]
    best, rows = None, []
    for rate in [float(x) for x in args.sweep.split(",")]:
        arrivals = poisson_arrivals(rate, args.duration, args.seed)
        requests = [pool[k % len(pool)] for k in range(len(arrivals))]
        srv = Server(int(args.budget_gib * 2**30), precision=args.precision,
                     steps_per_round=args.steps_per_round)
        try:
            out = summarize(srv.serve(requests, arrivals), args.duration)
        except pcba.PcbaError as e:   # an overload the library refused: the rate is not served
            out = dict(plans=len(requests), certified=0, p50_ms=math.inf, p99_ms=math.inf,
                       deadline_miss_rate=1.0, error=str(e))
        out.update(rate=rate)
        rows.append(out)
        log(f"[sweep] rate {rate:.0f}/s: p50/p99 {out['p50_ms']:.2f}/{out['p99_ms']:.2f} ms, "
            f"miss rate {out['deadline_miss_rate']:.4f}, {out['certified']}/{out['plans']} certified")
        print(json.dumps(out), flush=True)
        if out["p99_ms"] > 1e3 * srv.deadline or out["certified"] < out["plans"]:
            break
        best = rate
    print(json.dumps({"sweep": rows, "precision": args.precision, "max_rate_within_deadline": best,
                      "deadline_s": 0.5, "duration_s": args.duration}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--steps-per-round", type=int, default=2)
    ap.add_argument("--pool", type=int, default=256,
                    help="distinct plans generated; arrivals cycle through them")
    ap.add_argument("--sweep", default=None,
                    help="comma-separated arrival rates, each served for --duration seconds in "
                         "turn, up to the first whose p99 latency misses the deadline; reports "
                         "the highest rate served within it")
    args = ap.parse_args()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.sweep:
        sweep(args, log)
        return
    arrivals = poisson_arrivals(args.rate, args.duration, args.seed)
    npool = min(args.pool, len(arrivals))
    log(f"[serve] {len(arrivals)} arrivals over {args.duration:.0f} s; generating {npool} distinct plans")
    pool = [make_instance(4, args.seed * 100000 + k) for k in range(npool)]
    requests = [pool[k % npool] for k in range(len(arrivals))]
    srv = Server(int(args.budget_gib * 2**30), precision=args.precision,
                 steps_per_round=args.steps_per_round)
    recs = srv.serve(requests, arrivals, log=log)
    out = summarize(recs, args.duration)
    out.update(rate=args.rate, precision=args.precision, distinct_plans=npool,
               workload="serve: l=2, cost (6,6), constraints (10,10), count log-uniform in "
                        "[100,2000], deadline 0.5 s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
