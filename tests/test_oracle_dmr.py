"""Pins for the double Mach reflection boundaries of Sec. 4.5 (CPU only).

The bottom side is a wall from x = 0.1667 on with the post-shock state in
the ghosts left of it (the paper's lower boundary).  The top side holds the
exact position of the moving Mach 10 shock (the paper does not state it; the
problem's usual statement): post-shock ghosts left of x = 0.1667 + (y + 20 t)
/ 1.732, pre-shock right of it, evaluated at each RK stage's own time.

* The wall side reduces exactly to the reflective side (wall everywhere) and
  to prescribed-state ghosts (wall nowhere).
* The front side at time t equals the front moved by its speed times t at
  time 0, and a step evaluates the stages at t, t + dt, t + dt/2.
* An oblique Mach 10 shock with the exact-motion ghosts on both y sides
  moves at its speed (every row's shock within two cells of the exact line).
* The double Mach reflection itself at 128 x 32 to t = 0.2: physical, the
  incident shock at the top where the exact motion puts it, the peak density
  of the Mach stem region near the paper's largest contour (20.9).
"""
import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w

G = 1.4


def _dmr(nx=128, ny=32, **over):
    U, dx, prm, inf = w.double_mach(nx, ny)
    prm = dict(prm, **over)
    return U, dx, prm, inf


def test_wall_side_reduces_to_reflective_and_to_prescribed_state(orc):
    U, dx, prm, inf = _dmr()
    nx, ny = 128, 32
    g = prm["bgeom"]
    # wall everywhere (its start left of the grid) = a reflective side
    pw = orc.params(nx, ny, 1, dx, inflow=inf, **dict(prm, bgeom=[-1.0] + g[1:]))
    pr = orc.params(nx, ny, 1, dx, inflow=inf, **dict(prm, bc=[3, 1, 2, 5, 1, 1]))
    assert np.array_equal(orc.rhs(U, dx, G, pw), orc.rhs(U, dx, G, pr))
    # wall nowhere = post-shock ghosts under every cell = a front side whose
    # front lies right of the grid (the top side shares the front, so only
    # rows out of the top ghosts' reach are compared)
    pa = orc.params(nx, ny, 1, dx, inflow=inf, **dict(prm, bgeom=[1e9] + g[1:]))
    pf = orc.params(nx, ny, 1, dx, inflow=inf, **dict(prm, bc=[3, 1, 5, 5, 1, 1],
                                                       bgeom=[0.0, 1e9, 0.0, 0.0]))
    ra, rf = orc.rhs(U, dx, G, pa), orc.rhs(U, dx, G, pf)
    assert np.array_equal(ra[:, :, : ny - 4], rf[:, :, : ny - 4])
    assert not np.array_equal(ra, orc.rhs(U, dx, G, pw))


def test_state_sides_equal_a_grid_extended_by_their_ghost_rows(orc):
    """The rows next to the state sides see exactly the grid extended by
    three rows below and above, holding the ghost states of the definition:
    post-shock below the cells centred left of 0.1667 and the mirror image
    elsewhere; above, post- or pre-shock by the front's position at each
    ghost centre at time t."""
    nx, ny = 128, 32
    # LLF splitting: global LF speeds would also take the extended grid's
    # ghost rows, which are interior cells there
    U, dx, prm, inf = _dmr(nx, ny, split=0)
    p0 = orc.params(nx, ny, 1, dx, inflow=inf, **prm)
    t = 0.013
    orc.run(U, dx, G, p0, t)
    post, pre = np.array(prm["bstate"][0][:4]), np.array(prm["bstate"][1][:4])
    x0w, x0, slope, speed = prm["bgeom"]
    xc = (np.arange(nx) + 0.5) * dx
    E = np.zeros((4, 1, ny + 6, nx))
    E[:, :, 3:ny + 3] = U
    for k in range(3):  # ghost row -1-k below, ny+k above
        below = U[:, 0, k].copy()
        below[2] = -below[2]
        E[:, 0, 2 - k] = np.where(xc < x0w, post[:, None], below)
        yc = (ny + k + 0.5) * dx
        E[:, 0, ny + 3 + k] = np.where(xc < x0 + slope * yc + speed * t, post[:, None], pre[:, None])
    p = orc.params(nx, ny, 1, dx, inflow=inf, thr_L=[4.0, 1.0, 1.0], **prm)
    p.time = t
    infe = np.ascontiguousarray(np.repeat(post.reshape(4, 1), ny + 6, axis=1))
    pe = orc.params(nx, ny + 6, 1, dx, inflow=infe, thr_L=[4.0, 1.0, 1.0],
                    **dict(prm, bc=[3, 1, 1, 1, 1, 1]))
    r = orc.rhs(U, dx, G, p)
    re = orc.rhs(np.ascontiguousarray(E), dx, G, pe)
    assert np.array_equal(r, re[:, :, 3:ny + 3])


def test_front_side_follows_its_time_and_the_stage_times(orc):
    U, dx, prm, inf = _dmr()
    nx, ny = 128, 32
    t = 0.013
    p = orc.params(nx, ny, 1, dx, inflow=inf, **prm)
    p.time = t
    moved = list(prm["bgeom"])
    moved[1] = prm["bgeom"][1] + prm["bgeom"][3] * t
    q = orc.params(nx, ny, 1, dx, inflow=inf, **dict(prm, bgeom=moved))
    assert np.array_equal(orc.rhs(U, dx, G, p), orc.rhs(U, dx, G, q))
    # one SSP-RK3 step from t: the stages at t, t + dt, t + dt/2; t is
    # chosen so that the front passes a ghost centre of the first ghost row
    # between t + dt/2 and t + dt
    x0, slope, speed = prm["bgeom"][1:]
    dt, _ = orc.cfl_dt(U, dx, G, 0.5)
    yc = (ny + 0.5) * dx
    t = ((70 + 0.5) * dx - x0 - slope * yc) / speed - 0.75 * dt
    p.time = t
    V = U.copy()
    dt2, st = orc.step(V, dx, G, p)
    assert st == 0 and dt2 == dt
    ps = orc.params(nx, ny, 1, dx, inflow=inf, **prm)
    ps.time = t
    U1 = U + dt * orc.rhs(U, dx, G, ps)
    ps.time = t + dt
    U2 = 0.75 * U + 0.25 * (U1 + dt * orc.rhs(U1, dx, G, ps))
    ps.time = t + 0.5 * dt
    W = (1.0 / 3.0) * U + (2.0 / 3.0) * (U2 + dt * orc.rhs(U2, dx, G, ps))
    assert np.array_equal(V, W)
    # the third stage at t + dt would differ
    ps.time = t + dt
    W3 = (1.0 / 3.0) * U + (2.0 / 3.0) * (U2 + dt * orc.rhs(U2, dx, G, ps))
    assert not np.array_equal(W3, W)


def _crossings(rho, dx, mid):
    """x of the last fall of each row's density through mid."""
    out = []
    for r in rho:
        i = np.where((r[:-1] > mid) & (r[1:] <= mid))[0]
        out.append((i[-1] + 1.0) * dx if len(i) else np.nan)
    return np.array(out)


def test_oblique_mach10_shock_moves_at_its_speed(orc):
    """The exact-motion ghosts on both y sides: no wall, the shock stays a
    straight front moving at 20/1.732 along x (10 normal to itself)."""
    nx, ny = 128, 32
    U, dx, prm, inf = _dmr(nx, ny, bc=[3, 1, 5, 5, 1, 1])
    p = orc.params(nx, ny, 1, dx, inflow=inf, **prm)
    t_end = 0.05
    t, n, st = orc.run(U, dx, G, p, t_end)
    assert st == 0 and t == t_end
    y = (np.arange(ny) + 0.5) * dx
    xs = _crossings(U[0, 0], dx, 0.5 * (8.0 + 1.4))
    exact = w.DMR_X0 + (y + 20.0 * t_end) / w.DMR_SLOPE
    assert np.all(np.abs(xs - exact) < 2.0 * dx), (xs - exact) / dx


def test_double_mach_reflection_reduced(orc):
    """Sec. 4.5 at 128 x 32 to t = 0.2 (the paper's grids are 512 x 128 and
    1024 x 256): no non-physical state, the incident shock at the top within
    1.5 cells of the exact motion, the densest gas (Mach stem region) near
    the paper's largest contour, 20.9."""
    nx, ny = 128, 32
    U, dx, prm, inf = _dmr(nx, ny)
    p = orc.params(nx, ny, 1, dx, inflow=inf, **prm)
    t, n, st = orc.run(U, dx, G, p, 0.2)
    assert st == 0 and t == 0.2
    rho = U[0, 0]
    xs = _crossings(rho[-1:], dx, 0.5 * (8.0 + 1.4))[0]
    exact = w.DMR_X0 + (1.0 - 0.5 * dx + 20.0 * 0.2) / w.DMR_SLOPE
    assert abs(xs - exact) < 1.5 * dx, (xs, exact)
    assert 15.0 < rho.max() < 25.0 and rho.min() > 1.39
    # pre-shock gas ahead of the shock is untouched
    assert np.all(np.abs(rho[:, -8:] - 1.4) < 1e-6)
