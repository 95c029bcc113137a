"""Batched and served forms on the GPU, through the C ABI.

* A run's result does not depend on what else is in the batch: every run of
  a ragged mix of 1D and 2D grids equals, bit for bit, the same run admitted
  alone, and the same run on a single-grid context (weno_l2is_advance).
* The batched results match the CPU oracle advanced to the same end time
  (1e-10, the 100-step bar).
* Admission is bounded by the HBM budget and the slot table; retirement frees
  the memory for the next run.
* A run that reaches a non-physical state is retired with its status, alone;
  the other runs of the mix are unaffected.
* The serving loop (Poisson arrivals, continuous admission) returns for every
  request the result of running it alone.
"""
import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w
from gpu_util import params_pair, say, to_dev, to_host, z20

pytestmark = pytest.mark.gpu
G = 1.4
MiB = 1 << 20


@pytest.fixture(scope="module")
def capi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1908_02464_amd import capi as c
    c.lib()
    return c


def _mix():
    """(name, U0, dx, t_end) of a ragged mix: 1D and 2D, sizes that leave
    partial segments and partial wavefronts, 30-120 steps each."""
    out = []
    U, dx = w.sod(200)
    out.append(("sod200", U, dx, 0.1))
    left, right = w.random_two_state(np.random.default_rng(5))
    U, dx = w.riemann_1d(333, left, right)
    out.append(("two_state333", U, dx, 0.05))
    U, dx = w.shu_osher(517)
    out.append(("shu517", U, dx, 0.25))
    U, dx, _ = w.four_quadrant_2d(48, 40, 21)
    out.append(("quad48x40", U, dx, 0.08))
    U, dx, _ = w.four_quadrant_2d(37, 29, 22)
    out.append(("quad37x29", U, dx, 0.06))
    U, dx = w.riemann_1d(9, *w.LAX)
    out.append(("lax9", U, dx, 0.05))
    return out


def _shape(U):
    nx = U.shape[-1]
    ny = U.shape[-2] if U.ndim >= 3 else 1
    return nx, ny, 1


def _run_batch(capi, items, budget=256 * MiB, steps_per_poll=16, shape=None):
    eng = capi.Batch(budget, 64)
    if shape:
        eng.tune(*shape)
    slots = {}
    for name, U, dx, te in items:
        nx, ny, nz = _shape(U)
        s = eng.admit(U, nx, ny, nz, dx, te)
        assert s is not None, name
        slots[s] = name
    res = {}
    for _ in range(10000):
        if len(res) == len(items):
            break
        eng.advance(steps_per_poll)
        eng.stream.synchronize()
        for s in eng.poll():
            res[slots[s]] = eng.fetch(s)
    eng.close()
    assert len(res) == len(items)
    return res


def test_batch_mix_equals_alone_and_single_grid(capi):
    import torch
    items = _mix()
    say("[batch] mix of", len(items), "runs")
    mixed = _run_batch(capi, items)
    for it in items:
        name, U, dx, te = it
        alone = _run_batch(capi, [it])[name]
        Um, tm, sm = mixed[name]
        Ua, ta, sa = alone
        say(f"    {name}: t={tm} status={sm}")
        assert sm == 0 and sa == 0 and tm == te and ta == te
        assert np.array_equal(Um, Ua), name
        nx, ny, nz = _shape(U)
        ctx = capi.Context(nx, ny, nz, dx)
        Ud = to_dev(U)
        ctx.set_time(0.0)
        while ctx.time()[0] < te:
            ctx.advance(Ud, 64, te)
        torch.cuda.synchronize()
        Uc = to_host(Ud).reshape(Um.shape)
        ctx.close()
        d = float(np.abs(Uc - Um).max())
        say(f"    {name}: |batch - single-grid| = {d:.3e}")
        assert np.array_equal(Uc, Um), name


def test_batch_cancel_mid_run(capi):
    """Fetching a run before its t_end cancels it where it stands: its state
    and clock after k steps equal k steps of a single-grid context, and the
    run left in the batch finishes with the bits of running it alone."""
    import torch
    items = _mix()
    sod = next(it for it in items if it[0] == "sod200")
    quad = next(it for it in items if it[0] == "quad48x40")
    eng = capi.Batch(256 * MiB, 8)
    s_sod = eng.admit(sod[1], 200, 1, 1, sod[2], sod[3])
    s_quad = eng.admit(quad[1], 48, 40, 1, quad[2], quad[3])
    eng.advance(10)
    eng.stream.synchronize()
    Uc, tc, stc, kc = eng.fetch(s_sod, with_steps=True)
    assert stc == 0 and kc == 10 and 0.0 < tc < sod[3]
    ctx = capi.Context(200, 1, 1, sod[2])
    Ud = to_dev(sod[1])
    ctx.set_time(0.0)
    ctx.advance(Ud, 10, sod[3])
    t1, _, k1 = ctx.clock()
    torch.cuda.synchronize()
    assert k1 == 10 and t1 == tc
    assert np.array_equal(to_host(Ud).reshape(Uc.shape), Uc)
    ctx.close()
    res = None
    for _ in range(1000):
        eng.advance(16)
        eng.stream.synchronize()
        if s_quad in eng.poll():
            res = eng.fetch(s_quad)
            break
    eng.close()
    assert res is not None and res[1] == quad[3] and res[2] == 0
    alone = _run_batch(capi, [quad])["quad48x40"]
    assert np.array_equal(res[0], alone[0])


def test_batch_vs_oracle(orc, capi):
    items = _mix()
    res = _run_batch(capi, items)
    for name, U, dx, te in items:
        nx, ny, nz = _shape(U)
        po, _ = params_pair(orc, capi, (nx, ny, nz), dx)
        Uo = U.copy()
        t, n, st = orc.run(Uo, dx, G, po, te)
        Ug, tg, sg = res[name]
        err = z20(Ug.reshape(Uo.shape), Uo)
        say(f"    {name}: steps={n} t={t} z20={err:.3e}")
        assert st == 0 and sg == 0 and t == tg == te
        assert err <= 1e-10, name


def test_batch_budget_and_reuse(capi):
    say("[batch] budget")
    U1, dx1 = w.sod(1000)  # 3 arrays x 3 vars x 1000 x 8 B = 72000 B (+ alignment)
    U2, dx2 = w.sod(1000)
    eng = capi.Batch(100_000, 8)
    s1 = eng.admit(U1, 1000, 1, 1, dx1, 0.01)
    assert s1 is not None
    used, act = eng.usage()
    assert act == 1 and 72000 <= used <= 100_000
    assert eng.admit(U2, 1000, 1, 1, dx2, 0.01) is None  # over budget
    assert eng.usage() == (used, 1)
    while True:
        eng.advance(8)
        eng.stream.synchronize()
        done = eng.poll()
        if done:
            break
    assert done == [s1]
    U, t, st = eng.fetch(s1)
    assert st == 0 and t == 0.01
    assert eng.usage() == (0, 0)
    s2 = eng.admit(U2, 1000, 1, 1, dx2, 0.01)
    assert s2 is not None
    with pytest.raises(capi.WenoL2ISError):
        eng.fetch(7)  # never admitted
    eng.close()
    # slot table bound
    eng = capi.Batch(64 * MiB, 2)
    Us, dxs = w.sod(64)
    assert eng.admit(Us, 64, 1, 1, dxs, 0.1) is not None
    assert eng.admit(Us, 64, 1, 1, dxs, 0.1) is not None
    assert eng.admit(Us, 64, 1, 1, dxs, 0.1) is None
    eng.close()


def test_batch_rejects_unsupported(capi):
    eng = capi.Batch(64 * MiB, 4)
    U3, dx3 = w.turbulence_3d(8, 0)
    with pytest.raises(capi.WenoL2ISError):
        eng.admit(U3, 8, 8, 8, dx3, 0.1)  # 3D runs use the single-grid path
    Us, dxs = w.sod(64)
    p = capi.params_default(64, 1, 1, dxs, split=capi.SPLIT_LF)
    with pytest.raises(capi.WenoL2ISError):
        eng.admit(Us, 64, 1, 1, dxs, 0.1, params=p)
    with pytest.raises(capi.WenoL2ISError):
        eng.admit(Us, 64, 1, 1, dxs, -1.0)
    eng.close()


def test_batch_nonphysical_retired_alone(capi):
    say("[batch] non-physical run in a mix")
    items = _mix()[:3]
    bad, dxb = w.sod(128)
    bad = bad.copy()
    bad[2, 0, 0, 40] = -1.0  # negative energy: non-physical
    eng = capi.Batch(64 * MiB, 16)
    sb = eng.admit(bad, 128, 1, 1, dxb, 0.1)
    eng.advance(1)
    eng.stream.synchronize()
    done = eng.poll()
    assert done == [sb]
    _, _, st = eng.fetch(sb)
    assert st & 1
    eng.close()
    # with the bad run present for the whole time, the others are unchanged
    good = _run_batch(capi, items)
    eng = capi.Batch(64 * MiB, 16)
    slots = {eng.admit(bad, 128, 1, 1, dxb, 0.1): "bad"}
    for name, U, dx, te in items:
        nx, ny, nz = _shape(U)
        slots[eng.admit(U, nx, ny, nz, dx, te)] = name
    res = {}
    while len(res) < len(slots):
        eng.advance(16)
        eng.stream.synchronize()
        for s in eng.poll():
            res[slots[s]] = eng.fetch(s)
    eng.close()
    assert res["bad"][2] & 1
    for name, *_ in items:
        assert np.array_equal(res[name][0], good[name][0]), name


def test_serving_equals_alone(capi):
    from paper_1908_02464_amd import serve
    reqs = w.request_stream(n_req=24, rate=500.0, seed=3, n1d=(40, 600), n2d=(12, 48),
                            steps=(10, 80))
    say("[serve] 24 requests, continuous admission under a small budget")
    # a budget that holds only a few runs at once, so admission waits
    out_b, span_b = serve.run_batched(reqs, budget_bytes=2 * MiB, max_slots=64, continuous=True,
                                      steps_per_poll=4)
    out_p, span_p = serve.run_plain(reqs, honour_arrivals=False)
    s = serve.summarize(reqs, out_b, span_b)
    say("    batched", s)
    for r in reqs:
        a, b = out_b[r.rid], out_p[r.rid]
        assert a["status"] == 0 and b["status"] == 0, r.rid
        assert a["t"] == b["t"] == r.t_end, r.rid
        assert a["steps"] == b["steps"] > 0, r.rid
        assert np.array_equal(a["U"], b["U"].reshape(a["U"].shape)), r.rid


def test_batch_results_independent_of_launch_shape(capi):
    """Rows per work item and persistent grid size change no bit of any run."""
    items = _mix()
    ref = _run_batch(capi, items)
    for shape in [(4, 512), (16, 8192), (8, 64)]:
        say(f"[batch] rows={shape[0]} blocks={shape[1]}")
        got = _run_batch(capi, items, shape=shape)
        for name, *_ in items:
            assert np.array_equal(got[name][0], ref[name][0]), (name, shape)
    eng = capi.Batch(MiB, 4)
    for bad in [(-1, 0), (63, 0), (0, 63), (0, 65537)]:
        with pytest.raises(capi.WenoL2ISError):
            eng.tune(*bad)
    eng.close()


def test_batch_tune_mid_run(capi):
    """Changing the launch shape between advances of admitted runs."""
    items = _mix()
    ref = _run_batch(capi, items)
    eng = capi.Batch(256 * MiB, 64)
    slots = {}
    for name, U, dx, te in items:
        nx, ny, nz = _shape(U)
        slots[eng.admit(U, nx, ny, nz, dx, te)] = name
    res, k = {}, 0
    shapes = [(4, 1024), (16, 2048), (1, 4096)]
    while len(res) < len(items):
        eng.tune(*shapes[k % 3])
        k += 1
        eng.advance(7)
        eng.stream.synchronize()
        for s in eng.poll():
            res[slots[s]] = eng.fetch(s)
    eng.close()
    for name, *_ in items:
        assert np.array_equal(res[name][0], ref[name][0]), name


def test_autotuner_batch(capi):
    from paper_1908_02464_amd import autotune
    reqs = w.request_stream(n_req=16, rate=1000.0, seed=9, n1d=(64, 2000), n2d=(16, 128))
    rows, blocks, times = autotune.tune_batch(reqs, 64 * MiB, steps=2, rows=(4, 8),
                                              blocks=(512, 2048), verbose=True)
    assert (rows, blocks) in times and len(times) == 4
    assert all(t > 0 for t in times.values())


def test_fused_zchunk_bitwise_and_autotuner(capi):
    """z planes per workgroup and the occupancy target of the fused 3D kernel
    change no result bit; the tuner returns one of the timed shapes."""
    import torch
    from paper_1908_02464_amd import autotune
    U, dx = w.turbulence_3d(32, 4)
    U = U.copy()
    U[0, :, :, :16] *= 2.0
    U[4, :, :, :16] *= 2.0
    outs = []
    for zc, wpe in ((0, 2), (8, 2), (16, 1), (32, 2), (5, 1)):
        ctx = capi.Context(32, 32, 32, dx)
        ctx.tune(capi.PATH_FUSED, zc, wpe)
        Ud = to_dev(U)
        for _ in range(3):
            ctx.step(Ud)
        torch.cuda.synchronize()
        outs.append(to_host(Ud))
        ctx.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    zc, wpe, times = autotune.tune_fused(32, 32, 32, dx, to_dev(U), steps=2, zchunks=(0, 8, 32),
                                         verbose=True)
    assert (zc, wpe) in times and len(times) == 6


def test_batch_scheme_variants_and_boundaries(orc, capi):
    """One batch holding runs with different schemes and boundaries (Roe
    splitting, per-face switch, WENO only, linear only on smooth data, where
    it stays physical, the comparison weights of Eq.(8) and Eq.(14)-(15);
    periodic and reflective walls): each run equals, bit for bit, its single-grid run
    with the same parameters, and the oracle advanced to the same end time
    within 1e-10."""
    import torch
    U1, dx1 = w.sod(150)
    U2, dx2 = w.smooth_advection(96)
    left, right = w.random_two_state(np.random.default_rng(8))
    U3, dx3 = w.riemann_1d(120, left, right)
    U4, dx4, _ = w.four_quadrant_2d(50, 44, 23)
    U5, dx5, _ = w.four_quadrant_2d(33, 70, 24)
    runs = [("sod_roe", U1, dx1, 0.08, dict(split=capi.SPLIT_ROE)),
            ("adv_periodic_weno", U2, dx2, 0.2, dict(bc=[0, 0, 1, 1, 1, 1], hybrid=2)),
            ("two_state_reflective_face", U3, dx3, 0.05, dict(bc=[2, 2, 1, 1, 1, 1], hybrid=1)),
            ("adv_periodic_linear", U2, dx2, 0.2, dict(bc=[0, 0, 1, 1, 1, 1], hybrid=3)),
            ("quad_face_mixed_bc", U4, dx4, 0.03, dict(bc=[0, 0, 2, 2, 1, 1], hybrid=1)),
            ("quad_roe_reflective", U5, dx5, 0.04, dict(bc=[2, 1, 1, 2, 1, 1], split=capi.SPLIT_ROE)),
            ("sod_weno_is_b01", U1, dx1, 0.08, dict(hybrid=2, weights=2)),
            ("quad_hybrid_is", U4, dx4, 0.03, dict(weights=1))]
    eng = capi.Batch(128 * MiB, 16)
    slots = {}
    for name, U, dx, te, kw in runs:
        nx, ny, nz = _shape(U)
        slots[eng.admit(U, nx, ny, nz, dx, te, params=capi.params_default(nx, ny, nz, dx, **kw))] = name
    res = {}
    for _ in range(10000):
        if len(res) == len(runs):
            break
        eng.advance(8)
        eng.stream.synchronize()
        for s in eng.poll():
            res[slots[s]] = eng.fetch(s)
    eng.close()
    assert len(res) == len(runs)
    for name, U, dx, te, kw in runs:
        nx, ny, nz = _shape(U)
        Ub, tb, sb = res[name]
        assert sb == 0 and tb == te, name
        po, pg = params_pair(orc, capi, (nx, ny, nz), dx, **kw)
        ctx = capi.Context(nx, ny, nz, dx, G, pg)
        Ud = to_dev(U)
        ctx.set_time(0.0)
        while ctx.time()[0] < te:
            ctx.advance(Ud, 64, te)
        torch.cuda.synchronize()
        assert ctx.status() == 0
        Uc = to_host(Ud).reshape(Ub.shape)
        ctx.close()
        assert np.array_equal(Uc, Ub), name
        Uo = U.copy()
        t, n, st = orc.run(Uo, dx, G, po, te)
        err = z20(Ub.reshape(Uo.shape), Uo)
        say(f"    {name}: steps={n} z20={err:.3e}")
        assert st == 0 and t == te
        assert err <= 1e-10, name
