#!/usr/bin/env python3
"""Benchmark: 3D Euler decaying turbulence, 256^3 periodic, FP64, SSP-RK3.

One "step" is one SSP-RK3 step (three right-hand-side stages plus the device
CFL reduction) of the whole hot path on the 256^3 grid, inputs resident in
HBM.  Prints one JSON line with the throughput in Mcell-updates/s per RK
stage, the roofline of the dominant kernel (HIP events on the library's
stream), the batched-serving leg (p50/p99 time-to-solution and throughput of
a Poisson stream of 1D/2D runs, beside plain per-grid launches) and the CPU
oracle timed on a bounded sample of the same 3D workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector, published
N = 256
SEED = 2024
GAMMA = 1.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "fused3d_rk_turbulence256.md")


def measured_profile():
    """The committed rocprofv3 counter summary of the stage kernel (HBM bytes
    and FP64 operations per launch), or (None, reason) if it is missing or
    the kernel sources changed since the counters were taken."""
    try:
        from paper_1908_02464_amd.rocprof_summary import source_hash
        txt = open(PROFILE).read()
        info = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        if info.get("source_hash") != source_hash():
            return None, "stale"
        return info, info.get("source_hash")
    except (OSError, ValueError, IndexError, KeyError):
        return None, "missing"


def host_identity():
    """CPU model, logical CPUs, CPUs this process may run on, OMP_NUM_THREADS."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(U0, dx, min_seconds=10.0):
    """The oracle as it stands on the same 256^3 periodic initial field: one
    thread for one right-hand side (one RK stage's flux evaluation), then
    every usable core (OpenMP over the lines of a sweep, the same bits) for
    whole SSP-RK3 steps until min_seconds have passed."""
    from oracle import pyoracle as orc
    host = host_identity()
    U = np.ascontiguousarray(U0)
    nz, ny, nx = U.shape[1:]
    ncell = nx * ny * nz
    p = orc.params(nx, ny, nz, dx, bc=[0] * 6)
    orc.threads(1)
    t0 = time.perf_counter()
    orc.rhs(U, dx, GAMMA, p)
    el1 = time.perf_counter() - t0
    rate1 = ncell / el1 / 1e6
    cores = host["usable_cpus"] or 1
    if host["omp_num_threads"]:
        cores = min(cores, int(host["omp_num_threads"]))
    used = orc.threads(cores)
    V = U.copy()
    steps, t0 = 0, time.perf_counter()
    while True:
        orc.step(V, dx, GAMMA, p)
        steps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    value = ncell * 3 * steps / el / 1e6
    orc.threads(1)
    return {"value": round(value, 4), "unit": "Mcell-updates/s per RK stage", "cores": used,
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the oracle on the full {nx}x{ny}x{nz} periodic "
                      f"initial field with {used} OpenMP threads ({el:.1f} s); single thread: one "
                      f"right-hand side of the same field ({el1:.1f} s)",
            "single_thread": {"value": round(rate1, 4), "unit": "Mcell-updates/s per RK stage",
                              "seconds": round(el1, 2)},
            "host": host}


def weno_fractions(torch, ctx, Ud, nvar=5):
    """Per direction: the fraction of faces with some field on the WENO
    branch, and the fraction of face-fields on it (flags of the state Ud)."""
    faces, fields = [], []
    for d in range(3):
        nf = N ** 2 * (N + 1)
        fl = torch.empty(nvar * nf, dtype=torch.uint8, device="cuda")
        sg = torch.empty(nvar * nf, dtype=torch.float64, device="cuda")
        ctx.face_debug(Ud, d, fl, sg)
        f = fl.view(nvar, nf)
        faces.append(float((f.min(dim=0).values == 0).double().mean().item()))
        fields.append(float((f == 0).double().mean().item()))
        del fl, sg
    torch.cuda.synchronize()
    return faces, fields


def variants_3d(torch, capi, U0, dx, steps=10, developed_at=400):
    """The same 256^3 field with every face on the WENO-L2IS branch (switch
    off) and with every face on the linear branch (switch forced), timed like
    the headline after two warm-up steps: the two ends between which the
    hybrid scheme's cost lies.  Then the hybrid on the developed field: the
    same initial field advanced on the device for developed_at steps, when
    shocklets have formed and a few percent of the face-fields take the WENO
    branch (the nonlinear half of the hot path, Eq.(20)-(28), runs in the
    correction kernel); timed over the next steps with its WENO fractions."""
    out = {}
    for name, hyb in (("weno_only", 2), ("linear_only", 3), ("developed", 0)):
        p = capi.params_default(N, N, N, dx, bc=[0] * 6, hybrid=hyb)
        ctx = capi.Context(N, N, N, dx, GAMMA, p)
        Ud = torch.from_numpy(U0).cuda()
        ctx.advance(Ud, developed_at if name == "developed" else 2, 1e300)
        extra = {}
        if name == "developed":
            faces, fields = weno_fractions(torch, ctx, Ud)
            extra = {"start_step": developed_at, "weno_face_fraction_xyz": [round(f, 5) for f in faces],
                     "weno_face_field_fraction_xyz": [round(f, 5) for f in fields]}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.advance(Ud, steps, 1e300)
        e1.record(ctx.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        ctx.timing(True)
        ctx.advance(Ud, 2, 1e300)
        kt = ctx.timing_read()
        ctx.timing(False)
        out[name] = {"steps": steps, "ms_per_step": round(ms / steps, 4),
                     "Mcell_updates_per_s_per_stage": round(N ** 3 * 3 * steps / (ms * 1e-3) / 1e6, 2),
                     "kernel_ms_per_step": {k: round(v[0] / 2, 4) for k, v in kt.items()},
                     "status": ctx.status(), **extra}
        log(f"[bench]   3D {name}: {out[name]['ms_per_step']} ms/step {extra}")
        ctx.close()
        del Ud
        torch.cuda.empty_cache()
    return out


def other_configs(torch, capi, workloads):
    """The 1D and 2D workloads run to their end: Sod 200 to t = 0.2,
    Shu-Osher 1600 to t = 1.8 (transmissive), the interacting blast waves on
    400 cells to t = 0.038 (reflective walls, Roe splitting), the
    broadband sound packet on 128 cells for one period (periodic, CFL 0.2),
    2D four-quadrant 1024^2 for 200 steps, the Mach 2000 jet on 640 x 160 to
    t = 0.001, the double Mach reflection on 512 x 128 and 1024 x 256 to
    t = 0.2.  Each through weno_l2is_advance on the fused 1D/2D kernel,
    timed with events on the library's stream after one untimed warm-up
    run."""
    out = {}
    cases = []
    U, dx = workloads.sod(200)
    cases.append(("sod200_t0.2", U, dx, (200, 1, 1), 0.2, None, {}))
    U, dx = workloads.shu_osher(1600)
    cases.append(("shu_osher1600_t1.8", U, dx, (1600, 1, 1), 1.8, None, {}))
    U, dx = workloads.blast_waves(400)
    cases.append(("blast_waves400_t0.038", U, dx, (400, 1, 1), 0.038, None,
                  {"split": 2, "bc": [2, 2, 1, 1, 1, 1]}))
    U, dx = workloads.sound_packet(128)
    cases.append(("sound_packet128_t1", U, dx, (128, 1, 1), 1.0, None,
                  {"cfl": 0.2, "bc": [0, 0, 1, 1, 1, 1]}))
    U, dx, _ = workloads.four_quadrant_2d(1024, 1024, 2024)
    cases.append(("quad2d_1024x1024_200steps", U, dx, (1024, 1024, 1), 1e300, 200, {}))
    # the Mach 2000 jet (Sec. 4.7, 640 x 160 to t = 0.001, global LF as the
    # paper's 2D runs): the WENO-IS weights of Eq.(14)-(15), and the present
    # scheme with lambda = 3600 sigma^s (with the printed c = 1 it goes
    # non-physical at step 52)
    Uj, dxj, infj = workloads.mach2000_jet(640, 160)
    jet = {"bc": [3, 1, 2, 1, 1, 1], "cfl": 0.25, "split": 1}
    cases.append(("jet640x160_t0.001_weno_is_b01", Uj, dxj, (640, 160, 1), 1e-3, None,
                  dict(jet, hybrid=2, weights=2)))
    cases.append(("jet640x160_t0.001_present_c3600", Uj, dxj, (640, 160, 1), 1e-3, None,
                  dict(jet, c_reg=3600.0)))
    # the double Mach reflection (Sec. 4.5) to t = 0.2 on the paper's two
    # grids (Table 1 times the 512 x 128 run)
    infs = {}
    for dnx, dny in ((512, 128), (1024, 256)):
        Ud, dxd, prm, infd = workloads.double_mach(dnx, dny)
        name = f"dmr{dnx}x{dny}_t0.2"
        infs[name] = infd
        cases.append((name, Ud, dxd, (dnx, dny, 1), 0.2, None, prm))
    for name, U0, dx, shape, t_end, nsteps, kw in cases:
        gamma = workloads.JET_GAMMA if name.startswith("jet") else GAMMA
        ctx = capi.Context(*shape, dx, gamma, capi.params_default(*shape, dx, **kw))
        if name.startswith("jet"):
            ctx.set_inflow(torch.from_numpy(infj).cuda())
        if name in infs:
            ctx.set_inflow(torch.from_numpy(infs[name]).cuda())
        ncell = shape[0] * shape[1] * shape[2]
        res = None
        for rep in range(2):  # warm-up run, then the timed one
            Ud = torch.from_numpy(U0).cuda()
            ctx.set_time(0.0)
            t0c = ctx.clock()[2]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            if nsteps:
                ctx.advance(Ud, nsteps, t_end)
            else:
                # calls of up to 256 steps; once the clock is near t_end the
                # next call asks for about the steps left at the latest dt
                # (a step past t_end still launches its kernels, which return
                # at once)
                chunk = 256
                while True:
                    ctx.advance(Ud, chunk, t_end)
                    t_now, dt_now = ctx.time()
                    if not t_now < t_end or ctx.status() != 0:
                        break
                    if dt_now > 0.0:
                        chunk = max(1, min(256, int(math.ceil((t_end - t_now) / dt_now * 1.05)) + 1))
            e1.record(ctx.stream)
            e1.synchronize()
            t, _, steps = ctx.clock()
            steps -= t0c
            ms = e0.elapsed_time(e1)
            res = {"steps": int(steps), "t": t if t_end < 1e299 else None, "ms_total": round(ms, 3),
                   "ms_per_step": round(ms / steps, 5),
                   "Mcell_updates_per_s_per_stage": round(ncell * 3 * steps / (ms * 1e-3) / 1e6, 2),
                   "status": ctx.status()}
        out[name] = res
        log(f"[bench]   {name}: {res}")
        ctx.close()
    return out


def weighting_ratios(torch, capi, workloads, steps=200):
    """Relative cost of the schemes the paper compares (Sec. 4.5-4.6, Tables
    1-2 time the whole runs on a CPU), here as GPU time per step of the 2D
    four-quadrant 1024^2 problem, with the paper's 2D splitting (global
    Lax-Friedrichs) and with the local one: the present hybrid scheme
    (regularized weights, Eq.(28), with the switch of Eq.(33)-(35)), the
    WENO-IS scheme of Wang et al. (pure WENO with the weights of
    Eq.(14)-(15)), the original WENO-IS weights (Eq.(8)), pure regularized
    WENO (switch off) and the optimal linear scheme alone (every face on the
    linear branch; it goes non-physical at the shocks of this problem, and a
    run that stops is not timed)."""
    U0, dx, _ = workloads.four_quadrant_2d(1024, 1024, 2024)
    shape = (1024, 1024, 1)
    schemes = {"present": {}, "weno_is_b01": {"hybrid": 2, "weights": 2},
               "weno_is": {"hybrid": 2, "weights": 1}, "weno_l2is_no_switch": {"hybrid": 2},
               "linear_only": {"hybrid": 3}}
    out = {}
    for split_name, split in (("lf", 1), ("llf", 0)):
        res = _weighting_times(torch, capi, U0, dx, shape, schemes, split, steps)
        base = res["present"]["ms_per_step"]
        res["present_over"] = {k: (round(base / v["ms_per_step"], 3) if v["status"] == 0 else None)
                               for k, v in res.items() if k != "present"}
        out[split_name] = res
        log(f"[bench]   weighting ratios ({split_name}): {res['present_over']}")
    out["config"] = f"2D four-quadrant 1024^2, {steps} steps, seed 2024; lf = global LF splitting (the paper's 2D choice), llf = local LF"
    out["paper_context"] = ("CPU wall time ratios, unnamed hardware: Present / WENO-Z = 0.728 (DMR "
                            "512x128) and 0.772 (viscous shock tube); Present / WENO-JS = 0.840, "
                            "0.795; Present / WENO-HY = 1.262, 1.142")
    return out


def _weighting_times(torch, capi, U0, dx, shape, schemes, split, steps):
    out = {}
    for name, kw in schemes.items():
        ctx = capi.Context(*shape, dx, GAMMA, capi.params_default(*shape, dx, split=split, **kw))
        ms = None
        for rep in range(2):  # warm-up run, then the timed one
            Ud = torch.from_numpy(U0).cuda()
            ctx.set_time(0.0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            ctx.advance(Ud, steps, 1e300)
            e1.record(ctx.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
        st = ctx.status()
        out[name] = {"ms_per_step": round(ms / steps, 5) if st == 0 else None, "status": st}
        ctx.close()
        del Ud
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--hybrid", type=int, default=0, help="0 per-field (paper), 2 WENO only, 3 linear only")
    ap.add_argument("--path", type=int, default=0,
                    help="kernel path: 0 auto (fused stage kernel), 1 per-direction sweeps")
    ap.add_argument("--zchunk", type=int, default=0, help="z planes per workgroup (0 = auto)")
    ap.add_argument("--wpe", type=int, default=0, help="fused kernel waves per SIMD (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1D / 2D single-grid workloads")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the 3D WENO-only / linear-only timings")
    ap.add_argument("--no-ratios", action="store_true",
                    help="skip the relative cost of the compared weightings (2D 1024^2)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the batched-serving leg (Poisson stream of 1D/2D Riemann runs)")
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--plain-sample", type=int, default=96,
                    help="requests in the plain per-grid baseline sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of a state array (known bytes) for counter scaling")
    ap.add_argument("--start-step", type=int, default=0,
                    help="advance the field this many steps before the warm-up (developed regime)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the hot path "
              "runs on one MI355X, and sharding across GPUs is described, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_02464_amd import capi, workloads

    log(f"[bench] generating 256^3 turbulence field (seed {SEED})")
    U0, dx = workloads.turbulence_3d(N, SEED)
    ncell = N ** 3
    nvar = 5
    params = capi.params_default(N, N, N, dx, bc=[0] * 6, hybrid=args.hybrid)
    stream = torch.cuda.current_stream()
    ctx = capi.Context(N, N, N, dx, GAMMA, params, stream)
    ctx.tune(args.path, args.zchunk, args.wpe)
    Ud = torch.from_numpy(U0).cuda()

    # steps through weno_l2is_advance: CFL dt on the device every step (the
    # clock target is never reached); from the second step of a call the
    # CFL maximum comes folded out of the previous step's last stage
    T_END = 1e300
    if args.start_step:
        log(f"[bench] advancing {args.start_step} steps to the developed field")
        ctx.advance(Ud, args.start_step, T_END)
        torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps")
    ctx.advance(Ud, args.warmup, T_END)
    torch.cuda.synchronize()

    # headline: K steps bracketed by events on the library's stream
    log(f"[bench] timing {args.steps} steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.advance(Ud, args.steps, T_END)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    value = ncell * 3 * args.steps / (ms * 1e-3) / 1e6

    # per-kernel durations from HIP events around every launch (second pass)
    log("[bench] per-kernel timing pass")
    ctx.timing(True)
    ctx.advance(Ud, args.steps, T_END)
    kt = ctx.timing_read()
    ctx.timing(False)
    assert ctx.status() == 0, "non-physical state during the benchmark"
    tot_ms = sum(v[0] for v in kt.values())
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_n = kt[dom]
    avg_ms = dom_ms / dom_n
    arr = nvar * ncell * 8  # bytes of one state array
    # algorithmic bytes per launch.  Fused stage kernel: the method's own
    # 8/3 state arrays per cell-stage (stage 1 reads U^n, writes U^(1);
    # stages 2, 3 read U^(k) and U^n, write U^(k+1)), averaged over the three
    # launches of a step.  Per-direction sweeps: the arrays each kernel's role
    # must move (x: read U, write partial; y: read U, read+write partial;
    # z + RK: read U^(k), partial, U^n in stages 2-3, write U^(k+1)).
    role_arrays = {"fused3d_rk": 8.0 / 3.0,
                   "sweep_x_write": 2.0, "sweep_y_accum": 3.0, "sweep_z_rk": 11.0 / 3.0,
                   "sweep_x_accum": 3.0, "sweep_y_write": 2.0, "sweep_z_accum": 3.0}
    dom_bytes = role_arrays.get(dom, 2.0) * arr
    achieved = dom_bytes / (avg_ms * 1e-3) / 1e9
    traffic, traffic_src, flops = (None, "n/a", None)
    if dom == "fused3d_rk":
        prof, traffic_src = measured_profile()
        if prof is not None:
            traffic = prof.get("traffic_bytes_per_launch")
            flops = prof.get("fp64_flops_per_launch")
    # Roofline of the stage kernel: its algorithmic HBM bytes over the
    # event-timed launch against the 8 TB/s peak (the unit the target is set
    # in), with the counted HBM traffic of the committed rocprofv3 summary
    # (same kernel-source hash, else null).  Beside it the FP64 side: the
    # FP64 operations counted for this kernel binary over the same time, against the
    # FP64 vector peak; the counters count every lane of a wave instruction,
    # so lanes left idle by partial waves make it an upper bound.
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (round(traffic) if traffic else None), "traffic_source": traffic_src,
                "algorithmic_bytes_per_launch": int(dom_bytes),
                "bytes_per_cell_stage": round(dom_bytes / ncell, 2),
                "avg_launch_ms": round(avg_ms, 4), "launches": dom_n}
    if flops:
        tflops = flops / (avg_ms * 1e-3) / 1e12
        roofline["fp64_valu"] = {"achieved_TFLOPs": round(tflops, 2), "peak_TFLOPs": FP64_VECTOR_TFLOPS,
                                 "frac_upper_bound": round(tflops / FP64_VECTOR_TFLOPS, 4),
                                 "flops_per_launch": round(flops),
                                 "flops_per_cell_stage": round(flops / ncell, 1)}
    # the method's own bytes per cell-stage: 8/3 state arrays (read U^(k), U^n,
    # write U^(k+1); stage 1 reads only U^n)
    path_bytes = 8.0 / 3.0 * nvar * 8
    path_gbs = value * 1e6 * path_bytes / 1e9

    # fraction of faces that took the nonlinear flux in some field (final state)
    weno_frac, weno_field_frac = weno_fractions(torch, ctx, Ud)

    if args.copy_calibration:
        cp = Ud.clone()  # reads and writes exactly one state array
        torch.cuda.synchronize()
        del cp

    ctx.close()
    del Ud
    torch.cuda.empty_cache()

    variants = None
    if not args.no_variants and args.hybrid == 0 and args.path == 0:
        log("[bench] 3D WENO-only / linear-only variants")
        variants = variants_3d(torch, capi, U0, dx)

    # the other single-grid workloads of the method (1D, 2D), one context each
    others = None
    if not args.no_configs:
        log("[bench] 1D / 2D configurations")
        others = other_configs(torch, capi, workloads)

    ratios = None
    if not args.no_ratios and not args.no_configs:
        log("[bench] relative cost of the compared weightings (2D 1024^2)")
        ratios = weighting_ratios(torch, capi, workloads)

    serving = None
    if not args.no_serve:
        # batched serving: 1024 independent 1D/2D Riemann runs arriving as a
        # Poisson stream (200/s), admitted by HBM footprint into one batched
        # launch sequence (continuous), the same stream as a closed batch,
        # and the plain per-grid launches on a random sample of it
        from paper_1908_02464_amd import serve
        log(f"[bench] serving leg: {args.serve_requests} requests")
        serving = serve.serve_stream(n_req=args.serve_requests, modes=("continuous", "closed", "plain"),
                                     plain_sample=args.plain_sample, log=log)
        for k in ("metric", "unit", "data", "dtype"):
            serving.pop(k, None)
        cont, plain = serving["continuous"], serving.get("plain_sample") or serving.get("plain")
        serving["speedup_continuous_vs_plain"] = round(
            cont["throughput_Mcell_stage_per_s"] / plain["throughput_Mcell_stage_per_s"], 2)
        for m in ("continuous", "closed", "plain", "plain_sample"):
            if m in serving and not serving[m].get("failed"):
                serving[m].pop("failed_runs", None)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(U0, dx, args.cpu_seconds)

    out = {
        "metric": "Mcell-updates/s per RK stage, % HBM roofline; batched p50/p99 latency",
        "value": round(value, 2),
        "unit": "Mcell-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D Euler compressible decaying turbulence, 256^3 periodic, FP64, "
                        "random-phase solenoidal field E(k)~k^4 exp(-2(k/4)^2), Mt=0.6, SSP-RK3, "
                        "CFL 0.5, device CFL dt, WENO-L2IS hybrid (LLF)",
            "cells": ncell, "rk_stages_per_step": 3, "seed": SEED,
            "hybrid": {0: "per-field", 1: "per-face", 2: "weno-only", 3: "linear-only"}[args.hybrid],
            "kernel_path": {0: "fused stage kernel", 1: "per-direction sweeps"}[args.path],
            "start_step": args.start_step,
            "weno_face_fraction_xyz": [round(f, 6) for f in weno_frac],
            "weno_face_field_fraction_xyz": [round(f, 6) for f in weno_field_frac],
        },
        "roofline": roofline,
        "variants_3d": variants,
        "path_roofline": {
            "bytes_per_cell_stage": round(path_bytes, 2),
            "achieved_GBs": round(path_gbs, 1),
            "frac_of_hbm_peak": round(path_gbs / HBM_PEAK_GBS, 4),
        },
        "kernel_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "configs_1d_2d": others,
        "weighting_ratios": ratios,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
