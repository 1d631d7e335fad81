"""Serving driver: replay a Poisson trace of GRAPE forward + gradient requests
through the continuous-batching engine of libqoc, or one request at a time,
and report latency percentiles and slice-step throughput.

Latency of a request = host time its F and gradient are available minus its
arrival time.  Throughput = slice-steps (sum of N over finished requests)
per second of makespan.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import qoc


def replay(problems, arrivals, precision="fp32", max_active=256, pool_bytes=96 << 30, host_bytes=8 << 30,
           keep_grad=False, engine=None, progress=None):
    """Submit problems[i] at arrivals[i] seconds after the start (all at once if
    every arrival is 0) and collect results.  Returns a dict with per-request
    latency, F (and gradients when keep_grad), makespan and throughput."""
    n = len(problems)
    own = engine is None
    eng = engine or qoc.Engine(precision, pool_bytes, host_bytes, max_active)
    order = np.argsort(arrivals, kind="stable")
    lat = np.zeros(n)
    F = np.zeros(n)
    grads = [None] * n if keep_grad else None
    id2i = {}
    done = 0
    nxt = 0
    t0 = time.perf_counter()
    try:
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                p = problems[i]
                id2i[eng.submit(p.H0, p.Hc, p.u, p.dt, p.V)] = i
                nxt += 1
            eng.step(wait=(nxt == n))
            got = eng.poll()
            t = time.perf_counter() - t0
            for rid, f in got:
                i = id2i.pop(rid)
                g = eng.fetch(rid)
                lat[i] = t - arrivals[i]
                F[i] = f
                if keep_grad:
                    grads[i] = g
                done += 1
                if progress and done % progress == 0:
                    print(f"[serve] {done}/{n} done at {t:.2f} s", flush=True)
            if not got and nxt < n:
                gap = arrivals[order[nxt]] - (time.perf_counter() - t0)
                if gap > 2e-4:
                    time.sleep(min(gap, 1e-3))
        makespan = time.perf_counter() - t0
    finally:
        if own:
            eng.close()
    slices = float(sum(p.N for p in problems))
    return {"latency": lat, "F": F, "grad": grads, "makespan": makespan, "slice_steps_per_s": slices / makespan,
            "requests_per_s": n / makespan}


def summary(res) -> dict:
    lat = res["latency"]
    return {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "mean_ms": round(1e3 * float(lat.mean()), 3),
            "max_ms": round(1e3 * float(lat.max()), 3),
            "makespan_s": round(res["makespan"], 3),
            "slice_steps_per_s": round(res["slice_steps_per_s"], 1),
            "requests_per_s": round(res["requests_per_s"], 1)}


def per_d(res, problems) -> dict:
    """Latency percentiles and slice-steps of the requests of each dimension."""
    lat = res["latency"]
    ds = np.array([p.d for p in problems])
    out = {}
    for d in sorted(set(ds.tolist())):
        sel = ds == d
        out[str(d)] = {"requests": int(sel.sum()), "p50_ms": round(1e3 * float(np.percentile(lat[sel], 50)), 3),
                       "p99_ms": round(1e3 * float(np.percentile(lat[sel], 99)), 3),
                       "slice_steps": int(sum(p.N for p, s in zip(problems, sel) if s))}
    return out


def build_requests(n, seed=5, N_range=(100, 2000)):
    """The serving workload: trace entries (d, N) and their problems."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from workloads import make_request, poisson_trace

    trace = poisson_trace(n, rate=0.0, seed=seed, N_range=N_range)  # shapes only; arrivals set later
    problems = [make_request(t["index"], t["d"], t["N"], trace_seed=seed) for t in trace]
    return trace, problems


def poisson_arrivals(n, rate, seed=5):
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1]))
    gaps = rng.exponential(1.0 / rate, size=n)
    return np.cumsum(gaps) - gaps[0]


def main(argv=None):
    ap = argparse.ArgumentParser(description="GRAPE serving benchmark")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--max-active", type=int, default=256)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    trace, problems = build_requests(args.requests, args.seed)
    n = len(problems)
    print(f"[serve] built {n} requests in {time.perf_counter() - t0:.1f} s", flush=True)
    zero = np.zeros(n)
    prog = max(1, n // 8)
    cap = replay(problems, zero, args.precision, args.max_active, progress=prog)
    capacity = cap["requests_per_s"]
    rate = args.load * capacity
    print(f"[serve] capacity {capacity:.1f} req/s; replaying at {rate:.1f} req/s", flush=True)
    arr = poisson_arrivals(n, rate, args.seed)
    mix = replay(problems, arr, args.precision, args.max_active, progress=prog)
    print(f"[serve] batched: {summary(mix)}", flush=True)
    alone = replay(problems, arr, args.precision, 1, progress=prog)
    out = {"requests": n, "precision": args.precision, "capacity_req_per_s": round(capacity, 1),
           "capacity_slice_steps_per_s": round(cap["slice_steps_per_s"], 1),
           "arrival_rate_req_per_s": round(rate, 1), "batched": summary(mix), "one_at_a_time": summary(alone),
           "max_abs_dF_batched_vs_alone": float(np.max(np.abs(mix["F"] - alone["F"]))),
           "per_d": {"batched": per_d(mix, problems), "one_at_a_time": per_d(alone, problems)}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
