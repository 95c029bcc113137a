"""Serving loop over the batch engine: Poisson arrivals, admission by HBM
footprint, continuous batching, p50/p99 time-to-solution.

Three ways to run a request stream (each returns per-request results and
timings):
  * plain      -- one request at a time in arrival order, each on its own
                  single-grid context (weno_l2is_advance);
  * closed     -- every request admitted up front into one batch engine (as
                  many as the budget allows, refilled as runs finish), arrival
                  times ignored;
  * continuous -- requests admitted as they arrive and as memory frees up;
                  all admitted runs advance together, one batched step per
                  graph replay.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np
import torch

from . import capi


def _cell_stages(req):
    nx, ny, nz = req.shape
    return nx * ny * nz * 3 * req.target_steps


def run_plain(requests, steps_per_sync: int = 64, honour_arrivals: bool = True):
    """One request at a time on a single-grid context."""
    out = {}
    t0 = time.perf_counter()
    stream = torch.cuda.current_stream()
    for r in requests:
        if honour_arrivals:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        nx, ny, nz = r.shape
        ctx = capi.Context(nx, ny, nz, r.dx, stream=stream)
        U = torch.from_numpy(r.U0).cuda()
        ctx.set_time(0.0)
        while True:
            ctx.advance(U, steps_per_sync, r.t_end)
            t, _ = ctx.time()
            if not t < r.t_end or ctx.status() != 0:
                break
        res = U.cpu().numpy()
        done = time.perf_counter() - t0
        out[r.rid] = {"U": res, "t": t, "status": ctx.status(), "arrival": r.arrival,
                      "finish": done}
        ctx.close()
    return out, time.perf_counter() - t0


def run_batched(requests, budget_bytes: int, max_slots: int = 1024, continuous: bool = True,
                steps_per_poll: int = 4, keep_results: bool = True):
    """Batched execution; continuous=True honours arrival times (serving),
    False admits everything as soon as memory allows (closed batch)."""
    eng = capi.Batch(budget_bytes, max_slots)
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    slot_req = {}
    out = {}
    t0 = time.perf_counter()
    n_total = len(requests)
    while len(out) < n_total:
        now = time.perf_counter() - t0
        # admit arrived requests in arrival order while they fit
        while pending and (not continuous or pending[0].arrival <= now):
            r = pending[0]
            nx, ny, nz = r.shape
            slot = eng.admit(r.U0, nx, ny, nz, r.dx, r.t_end)
            if slot is None:
                break  # budget or slots exhausted: wait for a retirement
            slot_req[slot] = r
            pending.popleft()
        if slot_req:
            eng.advance(steps_per_poll)
            eng.stream.synchronize()
            for slot in eng.poll():
                r = slot_req.pop(slot)
                U, t, st = eng.fetch(slot)
                # a closed batch has every request in hand at time 0
                out[r.rid] = {"U": U if keep_results else None, "t": t, "status": st,
                              "arrival": r.arrival if continuous else 0.0,
                              "finish": time.perf_counter() - t0}
        elif pending:
            time.sleep(max(0.0, min(0.001, pending[0].arrival - now)))
    makespan = time.perf_counter() - t0
    eng.close()
    return out, makespan


def summarize(requests, out, makespan):
    lat = np.array([out[r.rid]["finish"] - out[r.rid]["arrival"] for r in requests])
    work = sum(_cell_stages(r) for r in requests)
    return {
        "requests": len(requests),
        "makespan_s": round(makespan, 4),
        "p50_s": round(float(np.percentile(lat, 50)), 5),
        "p99_s": round(float(np.percentile(lat, 99)), 5),
        "mean_s": round(float(lat.mean()), 5),
        "throughput_Mcell_stage_per_s": round(work / makespan / 1e6, 2),
        "failed": int(sum(1 for r in requests if out[r.rid]["status"] != 0)),
    }


def main(argv=None):
    """Run one request stream three ways and print one JSON line."""
    import argparse
    import json

    from . import workloads

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-req", type=int, default=1024)
    ap.add_argument("--rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--steps-min", type=int, default=50)
    ap.add_argument("--steps-max", type=int, default=2000)
    ap.add_argument("--steps-per-poll", type=int, default=4)
    ap.add_argument("--modes", default="continuous,closed,plain")
    a = ap.parse_args(argv)
    reqs = workloads.request_stream(n_req=a.n_req, rate=a.rate, seed=a.seed,
                                    steps=(a.steps_min, a.steps_max))
    budget = int(a.budget_gib * (1 << 30))
    out = {"metric": "served time-to-solution p50/p99 and Mcell-updates/s per RK stage",
           "unit": "s; Mcell-updates/s", "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"{a.n_req} Poisson Riemann runs at {a.rate}/s, 70% 1D "
                                  f"N in [128,8192], 30% 2D side in [64,512], "
                                  f"{a.steps_min}-{a.steps_max} steps",
                      "budget_bytes": budget}}
    results = {}
    for mode in a.modes.split(","):
        torch.cuda.synchronize()
        if mode == "plain":
            res, span = run_plain(reqs)
        else:
            res, span = run_batched(reqs, budget, continuous=(mode == "continuous"),
                                    steps_per_poll=a.steps_per_poll)
        out[mode] = summarize(reqs, res, span)
        results[mode] = res
        print(f"[serve] {mode}: {out[mode]}", flush=True)
    modes = list(results)
    same = True
    for m in modes[1:]:
        for r in reqs:
            x, y = results[modes[0]][r.rid]["U"], results[m][r.rid]["U"]
            same = same and np.array_equal(x, y.reshape(x.shape))
    out["bitwise_equal_across_modes"] = same
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
