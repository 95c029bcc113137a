"""Host-side logic, on the CPU: the seeded input generators, the parameter
structure shared with the C ABI, the serving summary, the counter-summary
parser, the build flags and the benchmark's one-GPU guard.  No GPU call."""
import csv
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w
import riemann_exact as rx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1908_02464_amd", "libweno_l2is.so")
G = 1.4


def _prim(U):
    """(rho, velocity components, p) of a conserved state [nvar, ...]."""
    rho = U[0]
    dim = U.shape[0] - 2
    vel = [U[1 + k] / rho for k in range(dim)]
    p = (G - 1.0) * (U[-1] - 0.5 * rho * sum(v * v for v in vel))
    return rho, vel, p


# ----------------------------------------------------------- request stream
def test_request_stream_is_seeded_and_shaped_as_stated():
    a = w.request_stream(n_req=400, seed=3)
    b = w.request_stream(n_req=400, seed=3)
    assert [(r.arrival, r.shape, r.t_end) for r in a] == [(r.arrival, r.shape, r.t_end) for r in b]
    assert all(np.array_equal(x.U0, y.U0) for x, y in zip(a, b))
    c = w.request_stream(n_req=400, seed=4)
    assert [r.shape for r in a] != [r.shape for r in c]

    arrivals = np.array([r.arrival for r in a])
    gaps = np.diff(np.concatenate([[0.0], arrivals]))
    assert np.all(gaps > 0)
    # exponential inter-arrival times, mean 1/200 s: 400 samples put the
    # sample mean within 15 % (three standard errors) and the coefficient of
    # variation near 1
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.15
    assert 0.8 < gaps.std() / gaps.mean() < 1.2

    one_d = [r for r in a if r.shape[1] == 1]
    two_d = [r for r in a if r.shape[1] > 1]
    assert abs(len(one_d) / len(a) - 0.7) < 0.08
    assert all(128 <= r.shape[0] <= 8192 and r.shape[2] == 1 for r in one_d)
    assert all(64 <= r.shape[0] <= 512 and r.shape[0] == r.shape[1] for r in two_d)
    assert all(50 <= r.target_steps <= 2000 and r.t_end > 0 for r in a)
    for r in a[:40]:
        nx, ny, nz = r.shape
        assert r.U0.shape == ((3 if ny == 1 else 4), nz, ny, nx)
        rho, _, p = _prim(r.U0)
        assert np.all(rho > 0) and np.all(p > 0)


def test_request_end_times_follow_the_step_recipe():
    """t_end = target steps x CFL dx / largest initial signal speed, with the
    signal speed taken from the primitive states of the initial data."""
    for r in w.request_stream(n_req=60, seed=11):
        rho, vel, p = _prim(r.U0)
        c = np.sqrt(G * p / rho)
        if r.shape[1] == 1:
            smax = float(np.max(np.abs(vel[0]) + c))
        else:
            smax = float(np.max(np.abs(vel[0]) + np.abs(vel[1]) + 2.0 * c))
        assert r.t_end == pytest.approx(r.target_steps * 0.5 * r.dx / smax, rel=1e-12)


# ----------------------------------------------------------- random states
def test_random_two_state_never_generates_vacuum():
    rng = np.random.default_rng(0)
    for _ in range(300):
        left, right = w.random_two_state(rng)
        assert 0.1 <= left[0] <= 1.5 and 0.03 <= left[2] <= 1.5
        p_star, _ = rx.star_state(left, right)  # raises on vacuum
        assert p_star > 0


def test_four_quadrant_interfaces_have_no_vacuum_and_one_is_compressive():
    """Checked with the exact Riemann solver of the tests (not the
    generator's own condition): every interface's star pressure is positive,
    and at least one interface has converging normal velocities."""
    for seed in range(40):
        U, dx, q = w.four_quadrant_2d(40, 40, seed)
        assert U.shape == (4, 1, 40, 40) and dx == 1.0 / 40
        rho, vel, p = _prim(U)
        assert np.all(rho > 0) and np.all(p > 0)
        compressive = False
        # quadrant order 0 = (x>.5, y>.5), 1 = (x<.5, y>.5), 2 = (x<.5, y<.5), 3 = (x>.5, y<.5)
        for a, b, k in ((1, 0, 1), (2, 3, 1), (3, 0, 2), (2, 1, 2)):
            left, right = (q[a, 0], q[a, k], q[a, 3]), (q[b, 0], q[b, k], q[b, 3])
            p_star, _ = rx.star_state(left, right)
            assert p_star > 0
            compressive |= right[1] < left[1]
        assert compressive
        # the quadrant states sit where the generator says
        assert U[0, 0, -1, -1] == pytest.approx(q[0, 0]) and U[0, 0, 0, 0] == pytest.approx(q[2, 0])


def test_turbulence_field_is_solenoidal_with_the_stated_mach_number():
    n = 32
    U, dx = w.turbulence_3d(n, 5)
    assert U.shape == (5, n, n, n) and dx == pytest.approx(2 * np.pi / n)
    rho, vel, p = _prim(U)
    assert np.allclose(rho, 1.0)
    u2 = sum(v * v for v in vel)
    assert math.sqrt(float(np.mean(u2))) == pytest.approx(1.0, rel=1e-12)
    c = np.sqrt(G * p / rho)
    assert np.allclose(c, 1.0 / 0.6)
    # spectral divergence (arrays are [z, y, x])
    k = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    F = [np.fft.fftn(v) for v in vel]
    div = KX * F[0] + KY * F[1] + KZ * F[2]
    ref = max(np.abs(f).max() for f in F)
    # the Nyquist planes have no sign of k (the real part mixes k and -k
    # there); the spectrum leaves them ~1e-7 of the peak amplitude
    nyq = (np.abs(KX) == n // 2) | (np.abs(KY) == n // 2) | (np.abs(KZ) == n // 2)
    assert np.abs(div[~nyq]).max() <= 1e-12 * ref * n
    assert max(np.abs(f[nyq]).max() for f in F) <= 1e-6 * ref
    # shell energy spectrum peaks near k0 = 4 (E(k) ~ k^4 exp(-2 (k/4)^2))
    K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    e = sum(np.abs(np.fft.fftn(v)) ** 2 for v in vel)
    shells = np.array([e[(K >= s - 0.5) & (K < s + 0.5)].sum() for s in range(1, 12)])
    assert 3 <= 1 + int(np.argmax(shells)) <= 5


# ----------------------------------------------------------- C ABI structure
@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_params_defaults_match_the_header_and_the_oracle():
    from paper_1908_02464_amd import capi
    from oracle import pyoracle as orc
    p = capi.params_default(64, 48, 1, 0.01)
    assert (p.cfl, p.c_reg, p.eps_weno, p.thr_C, p.thr_alpha) == (0.5, 1.0, 1e-20, 1.0, 3)
    assert (p.split, p.hybrid) == (capi.SPLIT_LLF, 0)
    assert list(p.bc) == [1] * 6
    assert list(p.thr_L)[:2] == pytest.approx([0.64, 0.48])
    o = orc.params(64, 48, 1, 0.01)
    for a, b in (("cfl", "cfl"), ("c_reg", "c_reg"), ("eps_weno", "eps_w"), ("thr_C", "thr_C"),
                 ("thr_alpha", "thr_alpha"), ("split", "split"), ("hybrid", "hybrid")):
        assert getattr(p, a) == getattr(o, b), a
    assert list(p.bc) == list(o.bc) and list(p.thr_L)[:2] == list(o.thr_L)[:2]
    q = capi.params_default(8, 1, 1, 0.5, bc=[0, 0, 2, 2, 1, 1], hybrid=2)
    assert list(q.bc) == [0, 0, 2, 2, 1, 1] and q.hybrid == 2


def test_params_struct_layout_matches_the_c_header(tmp_path):
    """Offsets of weno_l2is_params as the C compiler lays it out from
    include/weno_l2is.h, against the ctypes mirror of the binding."""
    from paper_1908_02464_amd import capi
    src = tmp_path / "layout.c"
    fields = [f for f, _ in capi.Params._fields_]
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"weno_l2is.h\"\n"
                   "int main(void) {\n"
                   + "".join(f'  printf("%zu\\n", offsetof(weno_l2is_params, {f}));\n' for f in fields)
                   + '  printf("%zu\\n", sizeof(weno_l2is_params));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(capi.Params, f).offset for f in fields] + [__import__("ctypes").sizeof(capi.Params)]
    assert got == want


# ----------------------------------------------------------- serving summary
def test_serving_summary_latency_and_throughput():
    from paper_1908_02464_amd import serve

    class R:
        def __init__(self, rid, arrival, shape, t_end):
            self.rid, self.arrival, self.shape, self.t_end = rid, arrival, shape, t_end

    reqs = [R(i, 0.01 * i, (100 + i, 1, 1), 1.0) for i in range(100)]
    out = {r.rid: {"arrival": r.arrival, "finish": r.arrival + 0.5 + 0.01 * r.rid, "steps": 10,
                   "status": 0, "t": 1.0} for r in reqs}
    out[7]["status"] = 1
    out[7]["steps"] = 4
    s = serve.summarize(reqs, out, makespan=2.0)
    # the failed request stays out of the percentiles and the throughput
    ok = [i for i in range(100) if i != 7]
    lat = np.array([0.5 + 0.01 * i for i in ok])
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50), abs=1e-5)
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99), abs=1e-5)
    work = sum((100 + i) * 3 * 10 for i in ok)
    assert s["throughput_Mcell_stage_per_s"] == pytest.approx(work / 2.0 / 1e6, abs=0.01)
    assert s["steps"] == 990 and s["completed"] == 99
    assert s["failed"] == 1 and s["failed_runs"][0]["rid"] == 7 and s["failed_steps"] == 4
    assert s["failed_Mcell_stages"] == pytest.approx(107 * 3 * 4 / 1e6, abs=1e-3)
    # every latency is non-negative when arrival times are the starts
    assert s["p50_s"] > 0 and s["mean_s"] > 0


# ----------------------------------------------------------- counter summary
def test_rocprof_summary_parses_trace_and_scales_counters(tmp_path):
    from paper_1908_02464_amd import rocprof_summary as rs
    tr = tmp_path / "trace"
    tr.mkdir()
    with open(tr / "x_kernel_stats.csv", "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                     "StdDev"])
        wr.writerow(["void wl2::k<2>(args)", 4, 4000, 1000.0, 90.0, 900, 1100, 50])
        wr.writerow(["other", 1, 10, 10.0, 10.0, 10, 10, 0])
    st = rs.trace_stats(str(tr), "wl2::k<2>")
    assert list(st.values()) == [{"calls": 4, "avg_ns": 1000.0, "min_ns": 900.0, "max_ns": 1100.0,
                                  "pct": 90.0}]
    cn = tmp_path / "fetch"
    cn.mkdir()
    with open(cn / "x_counter_collection.csv", "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"])
        wr.writerow(["void wl2::k<2>(args)", "FETCH_SIZE", 100.0, 4096])
        wr.writerow(["void wl2::k<2>(args)", "FETCH_SIZE", 300.0, 4096])
        wr.writerow(["__amd_rocclr_copyBuffer", "FETCH_SIZE", rs.COPY_KIB / 2.0, 1 << 20])
    vals, cal = rs.counter(str(cn), "wl2::k<2>", "FETCH_SIZE")
    assert vals == [100.0, 300.0] and cal == [rs.COPY_KIB / 2.0]
    # the summary's source hash follows the kernel code, not its comments
    h = rs.source_hash()
    assert len(h) == 16 and h == rs.source_hash()
    a = 'int a; // note "x"\n/* two\n lines */ const char* s = "a // b"; char c = \'"\';\nf("" : "+v"(q));'
    b = 'int a;   // other\n// words\n const char* s = "a // b"; char c = \'"\'; f(""  :  "+v"(q));'
    assert rs.code_text(a) == rs.code_text(b)
    assert rs.code_text(a) == 'int a; const char* s = "a // b"; char c = \'"\'; f("" : "+v"(q));'
    assert rs.code_text(a.replace("int a", "int z")) != rs.code_text(a)


# ----------------------------------------------------------- build and bench
def test_build_flags_forbid_packed_fp32_and_cross_statement_contraction():
    from paper_1908_02464_amd import build
    f = build.compile_flags("wl2_fused3d.hip")
    s = " ".join(f)
    assert "--offload-arch=gfx950" in f
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in s
    assert "-ffp-contract=on" in f


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_committed_profile_summary_is_readable():
    """The committed stage-kernel summary carries the figures bench.py reads."""
    t = open(os.path.join(ROOT, "profiles", "fused3d_rk_turbulence256.md")).read()
    info = json.loads(t.split("```json", 1)[1].split("```", 1)[0])
    assert info["traffic_bytes_per_launch"] > 1.0e9
    assert info["fp64_flops_per_launch"] > 1.0e10
    assert len(info["source_hash"]) == 16
