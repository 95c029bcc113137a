"""Whole-scheme pins for the oracle (CPU only).

* Two-state Riemann problems (Sec. 4.2: Sod, Lax, 123) against the exact
  solution: L1 error bounded and decreasing with N, shock position.
* Design order ~5 on smooth periodic advection (hybrid on and off), and
  third order of the time integrator under dt refinement at a fixed grid.
* Conservation to round-off on periodic grids, free-stream preservation,
  mirror symmetry, reflective walls equal the mirror-extended periodic
  problem, and 1D data embedded in 2D/3D (any axis) gives the 1D answer.
* The paper's interacting blast waves (Sec. 4.3) and broadband sound packet
  (Sec. 4.1): physical, conservative, and convergent under refinement.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w
import riemann_exact as rex

G = 1.4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_exact_solver_matches_published_star_states():
    """The exact solver itself reproduces the textbook star states."""
    with open(os.path.join(GOLDEN, "riemann_star_states.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        L, R = tuple(case["left"]), tuple(case["right"])
        p, u = rex.star_state(L, R, G)
        rl, rr = rex.star_densities(L, R, G)
        tol = case["tol"]
        assert abs(p - case["p_star"]) <= tol
        assert abs(u - case["u_star"]) <= tol
        assert abs(rl - case["rho_star_L"]) <= tol
        assert abs(rr - case["rho_star_R"]) <= tol


RIEMANN = [("sod", w.SOD, 0.2, 0.004), ("lax", w.LAX, 0.14, 0.011),
           ("123", w.PROBLEM_123, 0.15, 0.006)]


@pytest.mark.parametrize("name,states,t_end,bound", RIEMANN)
def test_riemann_problems_against_exact(orc, name, states, t_end, bound):
    errs = []
    for n in (100, 200, 400):
        U, dx = w.riemann_1d(n, *states)
        p = orc.params(n, 1, 1, dx)
        t, steps, st = orc.run(U, dx, G, p, t_end)
        assert st == 0 and t == t_end
        x = (np.arange(n) + 0.5) * dx
        rho, u, pr = rex.sample(states[0], states[1], (x - 0.5) / t_end, G)
        errs.append(np.mean(np.abs(U[0, 0, 0] - rho)))
        if n == 200:
            assert errs[-1] < bound, errs
    assert errs[1] < 0.8 * errs[0] and errs[2] < 0.8 * errs[1], errs


def test_sod_shock_position(orc):
    n = 400
    U, dx = w.sod(n)
    p = orc.params(n, 1, 1, dx)
    orc.run(U, dx, G, p, 0.2)
    x = (np.arange(n) + 0.5) * dx
    rho = U[0, 0, 0]
    # exact shock at x = 0.5 + S t
    ps, us = rex.star_state(*w.SOD, G)
    _, rsr = rex.star_densities(*w.SOD, G)
    S = us * rsr / (rsr - 0.125)  # mass conservation across the shock
    xs = 0.5 + S * 0.2
    # numerical shock: where rho crosses the mid value between rho*R and 0.125
    mid = 0.5 * (rsr + 0.125)
    i = np.where((rho[:-1] > mid) & (rho[1:] <= mid))[0][-1]
    assert abs(x[i] + 0.5 * dx - xs) < 2 * dx


def _advect(orc, n, t_end, hybrid, dt=None, weights=0):
    U, dx = w.smooth_advection(n)
    p = orc.params(n, 1, 1, dx, hybrid=hybrid, bc=[0, 0, 1, 1, 1, 1], weights=weights)
    if dt is None:
        # dt ~ dx^(5/3) keeps the RK3 error below the spatial error
        dt0 = 0.5 * (2.0 / 32) / (1.0 + np.sqrt(G))
        dt = dt0 * (32.0 / n) ** (5.0 / 3.0)
    steps = int(np.ceil(t_end / dt - 1e-9))
    dt = t_end / steps
    for _ in range(steps):
        _, st = orc.step(U, dx, G, p, dt)
        assert st == 0
    return U


# Pure WENO-L2IS converges at fifth order on the smooth profile (the paper
# states fifth order for the regularised weights, Sec. 3.1); measured
# 4.92 / 4.98 / 5.00 for N = 32..256, and still fifth order with lambda made
# 1e12 times larger.  A mistake that shifts weight to the low-order 2-point
# candidates or breaks a candidate reconstruction drops below 4.5.
@pytest.mark.parametrize("hybrid,min_rate", [(0, 4.6), (2, 4.5)])
def test_design_order_smooth_advection(orc, hybrid, min_rate):
    ns = [32, 64, 128, 256]
    errs = []
    for n in ns:
        U = _advect(orc, n, 2.0, hybrid)
        ex = w.smooth_advection_exact(n, 2.0)
        errs.append(np.mean(np.abs(U[0] - ex[0])))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert rates[-1] > min_rate and rates[-2] > min_rate, (errs, rates)


def test_comparison_weights_on_smooth_advection(orc):
    """Pure WENO with the original WENO-IS weights of Eq.(8) loses order on
    the smooth wave (its extrema are critical points: the 2-point stencils
    get too much weight, Sec. 2.4), converging at ~2.2 for N = 64..256; the
    beta_01 factor of Eq.(14)-(15) leaves that regime by N = 128 (errors
    1.0e-3, 1.6e-7, 4.7e-10 at N = 64, 128, 256)."""
    ns = [64, 128, 256]
    errs = {}
    for wts in (1, 2):
        errs[wts] = []
        for n in ns:
            U = _advect(orc, n, 2.0, 2, weights=wts)
            ex = w.smooth_advection_exact(n, 2.0)
            errs[wts].append(np.mean(np.abs(U[0] - ex[0])))
    rates = [np.log2(errs[1][i] / errs[1][i + 1]) for i in range(2)]
    assert max(rates) < 3.0, (errs, rates)
    assert errs[2][-1] < 1e-8 and errs[2][-1] < 1e-4 * errs[1][-1], errs


def test_hybrid_is_linear_everywhere_on_smooth_advection(orc):
    U, dx = w.smooth_advection(64)
    p = orc.params(64, 1, 1, dx, bc=[0, 0, 1, 1, 1, 1])
    fl, sg = orc.face_debug(U, dx, G, p, 0)
    assert np.all(fl == 1)
    assert sg.max() < (1.0 / 64) ** 3


def test_time_integrator_third_order(orc):
    n, T = 64, 0.25
    ref = _advect(orc, n, T, 3, dt=T / 640)
    errs = []
    for k in (10, 20, 40):
        U = _advect(orc, n, T, 3, dt=T / k)
        errs.append(np.abs(U - ref).max())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.8 < r < 3.3 for r in rates), (errs, rates)


@pytest.mark.parametrize("shape", [(64, 1, 1), (24, 20, 1), (12, 10, 8)])
def test_conservation_periodic(orc, shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(1)
    if nz > 1:
        U, dx = w.turbulence_3d(nx, 3, ny=ny, nz=nz)
        U = U * 1.0
        # add a density jump so WENO faces occur
        U[0, :, :, : nx // 2] *= 2.0
        U[-1, :, :, : nx // 2] *= 2.0
    elif ny > 1:
        U, dx, _ = w.four_quadrant_2d(nx, ny, 5)
    else:
        left, right = w.random_two_state(rng)
        U, dx = w.riemann_1d(nx, left, right)
    p = orc.params(nx, ny, nz, dx, bc=[0] * 6)
    s0 = U.reshape(U.shape[0], -1).sum(axis=1)
    a0 = np.abs(U).reshape(U.shape[0], -1).sum(axis=1)
    for _ in range(5):
        _, st = orc.step(U, dx, G, p)
        assert st == 0
    s1 = U.reshape(U.shape[0], -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * a0), (s1 - s0) / a0
    fl, _ = orc.face_debug(U, dx, G, p, 0)
    assert fl.min() == 0 and fl.max() == 1  # both branches exercised


@pytest.mark.parametrize("shape", [(16, 1, 1), (12, 9, 1), (8, 7, 6)])
@pytest.mark.parametrize("hybrid", [0, 2, 3])
def test_free_stream_preserved_exactly(orc, shape, hybrid):
    nx, ny, nz = shape
    dim = 1 + (ny > 1) + (nz > 1)
    rng = np.random.default_rng(dim)
    vel = list(rng.uniform(-1, 1, dim))
    U = w.conserved(np.full((nz, ny, nx), 0.7), [np.full((nz, ny, nx), v) for v in vel],
                    np.full((nz, ny, nx), 1.3))
    for bc in (0, 1, 2):
        if bc == 2:
            continue  # a wall reflects a moving stream
        p = orc.params(nx, ny, nz, 0.1, hybrid=hybrid, bc=[bc] * 6)
        assert np.all(orc.rhs(U, 0.1, G, p) == 0.0)


def test_mirror_symmetry(orc):
    """123 problem and a symmetric double blast stay mirror-symmetric.

    Rounding is not mirror-symmetric (the fields are summed in a fixed order)
    so the check is to a tolerance; a mistake in the mirrored f- stencil
    shows up at the 1e-3 level.  Pure WENO (no linear switch) on the
    near-vacuum 123 problem is left out: there the weights of Eq.(28) with
    eps = 1e-20 amplify round-off by ~100x per step for a few steps
    (lambda beta_k ~ eps), an intrinsic conditioning property."""
    cases = []
    n = 200
    U, dx = w.riemann_1d(n, *w.PROBLEM_123)
    cases.append((U, dx, 0.15, (0,)))
    x = (np.arange(n) + 0.5) / n
    pr = np.where(np.abs(x - 0.5) < 0.1, 100.0, 0.1)
    U = w.conserved(np.ones(n), [np.zeros(n)], pr).reshape(3, 1, 1, n)
    cases.append((U, 1.0 / n, 0.01, (0, 2)))
    for U, dx, T, hybs in cases:
        for hyb in hybs:
            V = U.copy()
            p = orc.params(n, 1, 1, dx, hybrid=hyb, bc=[2, 2, 1, 1, 1, 1])
            orc.run(V, dx, G, p, T)
            r = V[:, 0, 0]
            scale = np.abs(r).max(axis=1)
            tol = 1e-11
            assert np.all(np.abs(r[0] - r[0, ::-1]) <= tol * scale[0])
            assert np.all(np.abs(r[1] + r[1, ::-1]) <= tol * scale[1])
            assert np.all(np.abs(r[2] - r[2, ::-1]) <= tol * scale[2])


def test_blast_waves_refinement(orc):
    """Interacting blast waves (Sec. 4.3: reflective walls, Roe splitting,
    t = 0.038) stay physical with no limiter, conserve mass and energy to
    round-off (the walls pass no mass or energy flux), and the density
    converges under refinement: its mean distance to a 1600-cell run,
    block-averaged, falls by more than 1.5x per doubling from 100 to 400
    cells (about first order, as shocks dominate)."""
    def run(n):
        U, dx = w.blast_waves(n)
        m0 = U.sum(axis=(1, 2, 3))
        p = orc.params(n, 1, 1, dx, split=2, bc=[2, 2, 1, 1, 1, 1])
        t, _, st = orc.run(U, dx, G, p, 0.038)
        assert st == 0 and t == 0.038 and np.isfinite(U).all()
        rho = U[0, 0, 0]
        pr = (G - 1.0) * (U[2, 0, 0] - 0.5 * U[1, 0, 0] ** 2 / rho)
        assert rho.min() > 0.0 and pr.min() > 0.0
        m1 = U.sum(axis=(1, 2, 3))
        assert abs(m1[0] - m0[0]) <= 1e-12 * m0[0]
        assert abs(m1[2] - m0[2]) <= 1e-12 * m0[2]
        return rho
    fine = run(1600)
    errs = [np.abs(run(n) - fine.reshape(n, -1).mean(axis=1)).mean() for n in (100, 200, 400)]
    assert errs[0] > 1.5 * errs[1] > 2.25 * errs[2], errs


def _fourier_at(field, n):
    """The periodic cell-centred field on [0,1), interpolated to the n
    centres of a coarser grid through its Fourier series (exact for a
    band-limited field)."""
    m = field.size
    c = np.fft.rfft(field) / m
    k = np.arange(c.size)
    wgt = np.where((k == 0) | ((m % 2 == 0) & (k == m // 2)), 1.0, 2.0)
    x = (np.arange(n) + 0.5) / n
    return np.real((wgt * c)[None, :] * np.exp(2j * np.pi * k[None, :] * (x[:, None] - 0.5 / m))).sum(1)


def test_sound_packet_refinement(orc):
    """Broadband acoustic packet (Sec. 4.1: k0 = 12, eps = 1e-3, CFL 0.2,
    periodic, one period): the small smooth waves keep every face on the
    linear branch (detector far below its threshold), mass, momentum and
    energy are conserved to round-off, and the pressure converges: against
    a 1024-cell run, interpolated to the coarse centres through its Fourier
    series, the error falls by more than 8x from 128 to 256 cells (9.3x
    measured; the peak wavenumber has 10.7 points per wavelength at 128
    cells, short of the fifth-order regime)."""
    def run(n):
        U, dx = w.sound_packet(n)
        p = orc.params(n, 1, 1, dx, bc=[0, 0, 1, 1, 1, 1], cfl=0.2)
        fl, _ = orc.face_debug(U, dx, G, p, 0)
        assert fl.all()
        m0 = U.sum(axis=(1, 2, 3))
        t, _, st = orc.run(U, dx, G, p, 1.0)
        assert st == 0 and t == 1.0
        m1 = U.sum(axis=(1, 2, 3))
        assert np.all(np.abs(m1 - m0) <= 1e-12 * np.abs(m0).max())
        return (G - 1.0) * (U[2, 0, 0] - 0.5 * U[1, 0, 0] ** 2 / U[0, 0, 0])
    fine = run(1024)
    errs = []
    for n in (128, 256):
        ref = _fourier_at(fine, n)
        errs.append(np.sqrt(((run(n) - ref) ** 2).mean()) / np.sqrt(((ref - ref.mean()) ** 2).mean()))
    assert errs[0] > 8.0 * errs[1], errs
    assert errs[0] < 0.5, errs  # the packet survives one period at 128 cells


def test_reflective_wall_equals_mirror_extended_periodic(orc):
    n = 100
    rng = np.random.default_rng(4)
    left, right = w.random_two_state(rng)
    U, dx = w.riemann_1d(n, left, right)
    mirror = U[:, :, :, ::-1].copy()
    mirror[1] *= -1
    Ue = np.ascontiguousarray(np.concatenate([mirror, U], axis=3))
    pr = orc.params(n, 1, 1, dx, bc=[2, 2, 1, 1, 1, 1])
    pe = orc.params(2 * n, 1, 1, dx, bc=[0, 0, 1, 1, 1, 1], thr_L=[n * dx, 1, 1])
    for _ in range(30):
        dt1, _ = orc.step(U, dx, G, pr)
        orc.step(Ue, dx, G, pe, dt1)
    # the mirrored half is only mirror-symmetric up to rounding
    np.testing.assert_allclose(U, Ue[:, :, :, n:], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_1d_embedding_any_axis(orc, axis):
    n, m = 64, 5
    U1, dx = w.riemann_1d(n, *w.SOD)
    p1 = orc.params(n, 1, 1, dx, thr_L=[1.0, 1.0, 1.0])
    rho, mom, E = U1[0, 0, 0], U1[1, 0, 0], U1[2, 0, 0]
    shape = [m, m, m]
    shape[2 - axis] = n
    nz, ny, nx = shape
    zeros = np.zeros(shape)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    vel = [zeros.copy() for _ in range(3)]
    vel[axis] = np.broadcast_to((mom / rho).reshape(bshape), shape)
    U3 = w.conserved(np.broadcast_to(rho.reshape(bshape), shape), vel,
                     np.broadcast_to(((E - 0.5 * mom * mom / rho) * (G - 1)).reshape(bshape), shape))
    bc = [0] * 6
    bc[2 * axis] = bc[2 * axis + 1] = 1
    p3 = orc.params(nx, ny, nz, dx, bc=bc, thr_L=[1.0, 1.0, 1.0])
    for _ in range(10):
        dt, _ = orc.step(U1, dx, G, p1)
        orc.step(U3, dx, G, p3, dt)  # the multi-D CFL dt sums over directions
    sl = [0, 0, 0]
    sl[2 - axis] = slice(None)
    got = U3[(slice(None),) + tuple(sl)]
    np.testing.assert_allclose(got[0], U1[0, 0, 0], rtol=1e-13, atol=0)
    np.testing.assert_allclose(got[1 + axis], U1[1, 0, 0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(got[4], U1[2, 0, 0], rtol=1e-13, atol=0)
    others = [k for k in range(3) if k != axis]
    for k in others:
        assert np.all(got[1 + k] == 0.0)


def test_2d_transpose_symmetry(orc):
    """A four-quadrant state symmetric under x <-> y (u <-> v) keeps the
    symmetry: x and y sweeps agree."""
    n = 32
    rng = np.random.default_rng(12)
    q = w.random_quadrants(rng)
    q[3] = [q[1][0], q[1][2], q[1][1], q[1][3]]  # quadrant (x>.5,y<.5) mirrors (x<.5,y>.5)
    q[0][2] = q[0][1]
    q[2][2] = q[2][1]
    U, dx, _ = w.four_quadrant_2d(n, n, 0, quads=q)
    p = orc.params(n, n, 1, dx)
    for _ in range(10):
        orc.step(U, dx, G, p)
    np.testing.assert_allclose(U[0, 0], U[0, 0].T, rtol=1e-12)
    np.testing.assert_allclose(U[1, 0], U[2, 0].T, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(U[3, 0], U[3, 0].T, rtol=1e-12)


def test_rhs_at_matches_full_rhs(orc):
    U, dx = w.turbulence_3d(12, 8, ny=10, nz=9)
    U[0, :, :, :6] *= 1.5
    rng = np.random.default_rng(0)
    for split in (0, 1, 2):
        p = orc.params(12, 10, 9, dx, bc=[0, 0, 1, 1, 2, 2], split=split)
        full = orc.rhs(U, dx, G, p)
        cells = rng.choice(12 * 10 * 9, 40, replace=False)
        part = orc.rhs_at(U, dx, G, p, cells)
        np.testing.assert_array_equal(part, full.reshape(5, -1)[:, cells])


def test_nonphysical_state_reported(orc):
    U, dx = w.sod(50)
    U[2, 0, 0, 10] = -1.0  # negative energy -> negative pressure
    p = orc.params(50, 1, 1, dx)
    _, st = orc.cfl_dt(U, dx, G)
    assert st == 1
    t, steps, st = orc.run(U, dx, G, p, 0.1)
    assert st == 1 and steps == 0


def test_thread_count_changes_no_bit(orc):
    """The lines of a sweep may run on several threads (OpenMP build): each
    line writes only its own cells, so any thread count gives the same bits."""
    U, dx = w.turbulence_3d(16, 4, ny=14, nz=12)
    U = np.ascontiguousarray(U.copy())
    U[0, :, :, :8] *= 1.5
    p = orc.params(16, 14, 12, dx, bc=[0, 0, 1, 1, 2, 2])
    keep = orc.threads()
    try:
        outs = []
        for n in (1, 3, 8):
            orc.threads(n)
            V = U.copy()
            orc.step(V, dx, G, p)
            outs.append(V)
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
    finally:
        orc.threads(keep)
