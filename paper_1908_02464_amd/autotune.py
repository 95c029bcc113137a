"""Autotuner for the launch shapes: times candidate shapes on the device and
keeps the fastest.  None of the shapes changes a result bit (every face is
computed by the same arithmetic whatever thread computes it), so tuning is a
pure speed choice.

* Batched stage kernels (1D/2D, many grids): rows per work item of the 2D
  runs and the persistent grid size `blocks`, timed on a scratch engine
  holding a sample of the workload.
* Fused 3D stage kernel (one grid): z planes per workgroup `zchunk` and the
  occupancy target `waves_per_simd`, timed on a scratch copy of the state.
"""
from __future__ import annotations

import itertools

import torch

from . import capi

BATCH_ROWS = (4, 8, 16, 32)
BATCH_BLOCKS = (512, 1024, 2048, 4096, 8192)


def _time_batch(eng: capi.Batch, steps: int) -> float:
    eng.advance(1)  # (re)captures the graph for the current shape
    eng.stream.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(eng.stream)
    eng.advance(steps)
    b.record(eng.stream)
    b.synchronize()
    return a.elapsed_time(b) / steps


def tune_batch(requests, budget_bytes: int, steps: int = 8, max_runs: int = 256,
               rows=BATCH_ROWS, blocks=BATCH_BLOCKS, verbose: bool = False):
    """Best (rows, blocks) for a mix shaped like `requests` (the first
    `max_runs` that fit the budget, run with an end time they never reach).
    Returns (rows, blocks, {(rows, blocks): ms per step})."""
    eng = capi.Batch(budget_bytes, max(1, min(len(requests), max_runs)))
    n = 0
    for r in requests[:max_runs]:
        nx, ny, nz = r.shape
        if eng.admit(r.U0, nx, ny, nz, r.dx, 1e6) is None:
            break
        n += 1
    times = {}
    try:
        for r, bl in itertools.product(rows, blocks):
            eng.tune(r, bl)
            times[(r, bl)] = _time_batch(eng, steps)
            if verbose:
                print(f"[autotune] batch rows={r} blocks={bl}: {times[(r, bl)]:.4f} ms/step "
                      f"({n} runs)", flush=True)
    finally:
        eng.close()
    best = min(times, key=times.get)
    return best[0], best[1], times


def tune_fused(nx: int, ny: int, nz: int, dx: float, U: torch.Tensor, gamma: float = 1.4,
               params: capi.Params | None = None, steps: int = 4,
               zchunks=(0, 16, 32, 64, 128), wpes=(1, 2), verbose: bool = False):
    """Best (zchunk, waves_per_simd) of the fused stage kernel for this grid
    (zchunk: z planes in 3D, rows per item in 2D), timed on a scratch copy of
    U with a fixed dt.
    Returns (zchunk, wpe, {(zchunk, wpe): ms per step})."""
    ctx = capi.Context(nx, ny, nz, dx, gamma, params)
    W = U.clone()
    dt, _ = ctx.cfl_dt(W)
    times = {}
    try:
        for zc, w in itertools.product(zchunks, wpes):
            if zc > (nz if nz > 1 else ny):
                continue
            ctx.tune(capi.PATH_FUSED, zc, w)
            W.copy_(U)
            ctx.step(W, dt)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ctx.stream)
            for _ in range(steps):
                ctx.step(W, dt)
            b.record(ctx.stream)
            b.synchronize()
            times[(zc, w)] = a.elapsed_time(b) / steps
            if verbose:
                print(f"[autotune] fused zchunk={zc or 'auto'} wpe={w}: {times[(zc, w)]:.4f} ms/step",
                      flush=True)
    finally:
        ctx.close()
    best = min(times, key=times.get)
    return best[0], best[1], times
