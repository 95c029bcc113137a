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


def _cell_stages(req, steps):
    nx, ny, nz = req.shape
    return nx * ny * nz * 3 * steps


def run_plain(requests, steps_per_sync: int = 64, honour_arrivals: bool = True):
    """One request at a time on a single-grid context.  With
    honour_arrivals=False the requests run back to back and each one's
    latency is counted from its own start (a service time)."""
    out = {}
    t0 = time.perf_counter()
    stream = torch.cuda.current_stream()
    for r in requests:
        if honour_arrivals:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            arrival = r.arrival
        else:
            arrival = time.perf_counter() - t0
        nx, ny, nz = r.shape
        ctx = capi.Context(nx, ny, nz, r.dx, stream=stream)
        U = torch.from_numpy(r.U0).cuda()
        ctx.set_time(0.0)
        while True:
            ctx.advance(U, steps_per_sync, r.t_end)
            t, _, nsteps = ctx.clock()
            if not t < r.t_end or ctx.status() != 0:
                break
        res = U.cpu().numpy()
        done = time.perf_counter() - t0
        out[r.rid] = {"U": res, "t": t, "status": ctx.status(), "steps": nsteps,
                      "arrival": arrival, "finish": done}
        ctx.close()
    return out, time.perf_counter() - t0


def run_batched(requests, budget_bytes: int, max_slots: int = 1024, continuous: bool = True,
                steps_per_poll: int = 4, keep_results: bool = True, shape=None):
    """Batched execution; continuous=True honours arrival times (serving),
    False admits everything as soon as memory allows (closed batch).
    shape = (rows, blocks) of the batched kernels (e.g. from the autotuner)."""
    eng = capi.Batch(budget_bytes, max_slots)
    if shape:
        eng.tune(*shape)
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
                U, t, st, nsteps = eng.fetch(slot, with_steps=True)
                # a closed batch has every request in hand at time 0
                out[r.rid] = {"U": U if keep_results else None, "t": t, "status": st,
                              "steps": nsteps,
                              "arrival": r.arrival if continuous else 0.0,
                              "finish": time.perf_counter() - t0}
        elif pending:
            time.sleep(max(0.0, min(0.001, pending[0].arrival - now)))
    makespan = time.perf_counter() - t0
    eng.close()
    return out, makespan


def summarize(requests, out, makespan):
    """Latency percentiles and throughput over the requests that reached
    their end time; requests that stopped at a non-physical state are
    reported apart (count, their work, and where each stopped)."""
    ok = [r for r in requests if out[r.rid]["status"] == 0]
    bad = [r for r in requests if out[r.rid]["status"] != 0]
    lat = np.array([out[r.rid]["finish"] - out[r.rid]["arrival"] for r in ok])
    work = sum(_cell_stages(r, out[r.rid]["steps"]) for r in ok)
    pct = (lambda q: round(float(np.percentile(lat, q)), 5)) if lat.size else (lambda q: None)
    return {
        "requests": len(requests),
        "completed": len(ok),
        "makespan_s": round(makespan, 4),
        "p50_s": pct(50),
        "p99_s": pct(99),
        "mean_s": round(float(lat.mean()), 5) if lat.size else None,
        "steps": int(sum(out[r.rid]["steps"] for r in ok)),
        "throughput_Mcell_stage_per_s": round(work / makespan / 1e6, 2),
        "failed": len(bad),
        "failed_steps": int(sum(out[r.rid]["steps"] for r in bad)),
        "failed_Mcell_stages": round(sum(_cell_stages(r, out[r.rid]["steps"]) for r in bad) / 1e6, 3),
        "failed_runs": [{"rid": r.rid, "shape": list(r.shape), "steps": out[r.rid]["steps"],
                         "t": out[r.rid]["t"], "t_end": r.t_end} for r in bad],
    }


def main(argv=None):
    """Run one request stream three ways and print one JSON line."""
    import argparse

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-req", type=int, default=1024)
    ap.add_argument("--rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--steps-min", type=int, default=50)
    ap.add_argument("--steps-max", type=int, default=2000)
    ap.add_argument("--steps-per-poll", type=int, default=4)
    ap.add_argument("--modes", default="continuous,closed,plain")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="run the plain baseline on this many random requests only")
    a = ap.parse_args(argv)
    return serve_stream(a.n_req, a.rate, a.seed, a.budget_gib, (a.steps_min, a.steps_max),
                        a.steps_per_poll, a.modes.split(","), not a.no_autotune, a.plain_sample)


def serve_stream(n_req=1024, rate=200.0, seed=0, budget_gib=4.0, steps=(50, 2000),
                 steps_per_poll=4, modes=("continuous", "closed", "plain"), autotune=True,
                 plain_sample=0, log=print):
    """Run one seeded request stream in each mode; returns a dict with the
    per-mode summaries and whether all modes gave the same bits.
    plain_sample > 0 runs the plain per-grid baseline on that many requests
    drawn at random from the stream (back to back, arrival times ignored), a
    bounded throughput sample instead of the whole stream."""
    import json

    from . import autotune as tuner
    from . import workloads

    reqs = workloads.request_stream(n_req=n_req, rate=rate, seed=seed, steps=steps)
    budget = int(budget_gib * (1 << 30))
    shape = None
    if autotune:
        rows, blocks, times = tuner.tune_batch(reqs, budget, steps=4, max_runs=256)
        shape = (rows, blocks)
        log(f"[serve] autotuned batched kernels: rows={rows} blocks={blocks} "
            f"({times[shape]:.3f} ms/step on {min(256, n_req)} runs)")
    out = {"metric": "served time-to-solution p50/p99 and Mcell-updates/s per RK stage",
           "unit": "s; Mcell-updates/s", "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"{n_req} Poisson Riemann runs at {rate}/s, 70% 1D "
                                  f"N in [128,8192], 30% 2D side in [64,512], "
                                  f"{steps[0]}-{steps[1]} steps",
                      "budget_bytes": budget, "seed": seed,
                      "batched_shape": {"rows": shape[0], "blocks": shape[1]} if shape else None}}
    results = {}
    for mode in modes:
        torch.cuda.synchronize()
        if mode == "plain" and 0 < plain_sample < len(reqs):
            pick = np.random.default_rng(seed + 1).choice(len(reqs), plain_sample, replace=False)
            sub = [reqs[i] for i in sorted(pick)]
            res, span = run_plain(sub, honour_arrivals=False)
            name = "plain_sample"
            out[name] = summarize(sub, res, span)
            out[name]["note"] = (f"{plain_sample} requests drawn at random from the stream, "
                                 "run back to back; latency = each request's own service "
                                 "time (from its start, not from a stream arrival)")
        elif mode == "plain":
            res, span = run_plain(reqs)
            name = mode
            out[name] = summarize(reqs, res, span)
        else:
            res, span = run_batched(reqs, budget, continuous=(mode == "continuous"),
                                    steps_per_poll=steps_per_poll, shape=shape)
            name = mode
            out[name] = summarize(reqs, res, span)
        results[name] = res
        log(f"[serve] {name}: {out[name]}")
    names = list(results)
    same = True
    for m in names[1:]:
        for r in reqs:
            if r.rid not in results[m] or r.rid not in results[names[0]]:
                continue
            x, y = results[names[0]][r.rid]["U"], results[m][r.rid]["U"]
            same = same and np.array_equal(x, y.reshape(x.shape), equal_nan=True)
    out["bitwise_equal_across_modes"] = same
    log(json.dumps(out))
    return out


if __name__ == "__main__":
    main()
