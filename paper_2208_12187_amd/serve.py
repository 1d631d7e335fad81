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
           keep_grad=False, engine=None, progress=None, idle_sleep=1e-4):
    """Submit problems[i] at arrivals[i] seconds after the start (all at once if
    every arrival is 0) and collect results.  Returns a dict with per-request
    latency, F (and gradients when keep_grad), makespan and throughput.
    While nothing has finished and the next arrival is ahead, the loop sleeps
    at most idle_sleep seconds before polling again (0: spin), which bounds
    how late a finished request is noticed."""
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
                if idle_sleep > 0 and gap > 2 * idle_sleep:
                    time.sleep(min(gap, idle_sleep))
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


def run(n_requests=4096, precision="fp32", load=0.7, max_active=256, seed=5, log=None):
    """The serving benchmark: the trace offered all at once (capacity), then
    replayed with Poisson arrivals at `load` times that capacity, batched and
    again one request at a time on the same arrival times.  Returns the
    summary dict."""
    say = log or (lambda msg: None)
    t0 = time.perf_counter()
    trace, problems = build_requests(n_requests, seed)
    n = len(problems)
    say(f"[serve] built {n} requests in {time.perf_counter() - t0:.1f} s")
    prog = max(1, n // 8)
    cap = replay(problems, np.zeros(n), precision, max_active, progress=prog if log else None)
    capacity = cap["requests_per_s"]
    rate = load * capacity
    say(f"[serve] capacity {capacity:.1f} req/s; replaying at {rate:.1f} req/s")
    arr = poisson_arrivals(n, rate, seed)
    mix = replay(problems, arr, precision, max_active, progress=prog if log else None)
    say(f"[serve] batched: {summary(mix)}")
    alone = replay(problems, arr, precision, 1, progress=prog if log else None)
    say(f"[serve] one at a time: {summary(alone)}")
    return {"requests": n, "precision": precision, "trace_seed": seed,
            "capacity_req_per_s": round(capacity, 1),
            "capacity_slice_steps_per_s": round(cap["slice_steps_per_s"], 1),
            "arrival_rate_req_per_s": round(rate, 1), "load": load,
            "batched": summary(mix), "one_at_a_time": summary(alone),
            "max_abs_dF_batched_vs_alone": float(np.max(np.abs(mix["F"] - alone["F"]))),
            "per_d": {"batched": per_d(mix, problems), "one_at_a_time": per_d(alone, problems)}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="GRAPE serving benchmark")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--max-active", type=int, default=256)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    # progress on stderr, the summary as the one line on stdout
    out = run(args.requests, args.precision, args.load, args.max_active, args.seed,
              log=lambda msg: print(msg, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
