"""Pins of the oracle's inflow boundary (Sec. 4.7: the jet's left side
prescribes the state of its ghosts), CPU only.

* A grid with an inflow side gives the same right-hand side, bit for bit, as
  the grid extended by three columns holding the inflow state with an
  outflow (copy) side: the two feed identical stencils to every face, and
  the extended grid uses only the pinned copy rule.
* A supersonic inflow into gas at rest converges to the exact Riemann
  solution of the two states (all its waves move into the grid, so the
  boundary sees the inflow state at all times).
* The Mach 2000 jet (Sec. 4.7): the time step bounds the inflow speed, the
  jet gas enters through the rows below y = 0.05 only, and the state stays
  physical while the jet forms.  (Later, at its bow shock, a pressure turns
  negative with every splitting and switch setting: step 43 with LLF on the
  paper's 640 x 160 grid.  The paper reports no failure there; this oracle
  does not reproduce that claim.)
* Misplaced inflow sides and a missing state are refused.
"""
import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w
import riemann_exact as rex

G = 1.4


def _prim_to_cons(rho, u, v, p, g):
    return np.array([rho, rho * u, rho * v, p / (g - 1.0) + 0.5 * rho * (u * u + v * v)])


def _jet_like(nx, ny, seed):
    """Ambient gas with small random variations and a per-row inflow state
    that differs between rows (a jet in the lower rows)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * rng.random((ny, nx))
    u = 0.3 * rng.standard_normal((ny, nx))
    v = 0.3 * rng.standard_normal((ny, nx))
    p = 1.0 + 0.2 * rng.random((ny, nx))
    U = _prim_to_cons(rho, u, v, p, G).reshape(4, 1, ny, nx)
    jet = np.arange(ny) < ny // 3
    inf = _prim_to_cons(np.where(jet, 3.0, 1.0) + 0.1 * rng.random(ny),
                        np.where(jet, 2.5, 0.1) + 0.1 * rng.random(ny),
                        0.2 * rng.standard_normal(ny), 1.0 + 0.1 * rng.random(ny), G)
    return np.ascontiguousarray(U), np.ascontiguousarray(inf)


@pytest.mark.parametrize("split,hybrid", [(0, 0), (2, 0), (0, 2), (0, 1)])
def test_inflow_equals_extended_grid(orc, split, hybrid):
    nx, ny, dx = 24, 16, 0.05
    U, inf = _jet_like(nx, ny, 7 + split + hybrid)
    bc = [3, 1, 2, 1, 1, 1]
    p_in = orc.params(nx, ny, 1, dx, bc=bc, split=split, hybrid=hybrid, inflow=inf,
                      thr_L=[nx * dx, ny * dx, dx])
    got = orc.rhs(U, dx, G, p_in)
    # three columns of the inflow state left of the grid, copied outwards
    E = np.concatenate([np.repeat(inf.reshape(4, 1, ny, 1), 3, axis=3), U], axis=3)
    E = np.ascontiguousarray(E)
    p_ext = orc.params(nx + 3, ny, 1, dx, bc=[1, 1, 2, 1, 1, 1], split=split, hybrid=hybrid,
                       thr_L=[nx * dx, ny * dx, dx])
    ref = orc.rhs(E, dx, G, p_ext)[..., 3:]
    assert np.array_equal(got, ref)
    # the inflow state matters: a copy side gives another answer
    p_copy = orc.params(nx, ny, 1, dx, bc=[1, 1, 2, 1, 1, 1], split=split, hybrid=hybrid,
                        thr_L=[nx * dx, ny * dx, dx])
    assert np.abs(orc.rhs(U, dx, G, p_copy) - got).max() > 1e-3
    # selected cells and the face detector agree as well
    cells = np.array([0, 1, 2, nx, 5 * nx + 3, (ny - 1) * nx], dtype=np.int64)
    at = orc.rhs_at(U, dx, G, p_in, cells)
    assert np.array_equal(at, got.reshape(4, -1)[:, cells])
    fl, sg = orc.face_debug(U, dx, G, p_in, 0)
    fe, se = orc.face_debug(E, dx, G, p_ext, 0)
    assert np.array_equal(fl, fe[..., 3:]) and np.array_equal(sg, se[..., 3:])


def _left_wave_speed(L, R, g):
    rho, u, p = L
    c = np.sqrt(g * p / rho)
    ps, _ = rex.star_state(L, R, g)
    if ps > p:  # shock
        return u - c * np.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
    return u - c  # rarefaction head


def test_inflow_supersonic_riemann_refinement(orc):
    L, R, t = (1.0, 3.0, 1.0), (0.125, 0.0, 0.1), 0.15
    assert _left_wave_speed(L, R, G) > 0.2  # every wave moves into the grid
    errs = []
    for n in (200, 400):
        x = (np.arange(n) + 0.5) / n
        U = np.ascontiguousarray(
            np.stack([np.full(n, R[0]), np.zeros(n), np.full(n, R[2] / (G - 1.0))]).reshape(3, 1, 1, n))
        inf = np.array([L[0], L[0] * L[1], L[2] / (G - 1.0) + 0.5 * L[0] * L[1] ** 2]).reshape(3, 1)
        p = orc.params(n, 1, 1, 1.0 / n, bc=[3, 1, 1, 1, 1, 1], inflow=inf)
        tt, _, st = orc.run(U, 1.0 / n, G, p, t)
        assert st == 0 and tt == t
        rho_ex = rex.sample(L, R, x / t, G)[0]
        errs.append(float(np.abs(U[0, 0, 0] - rho_ex).mean()))
    assert errs[0] < 0.03 and errs[1] < 0.75 * errs[0]


def test_mach2000_jet_forms(orc):
    """The jet at a quarter of the paper's resolution for 25 steps."""
    nx, ny = 160, 40
    U, dx, inf = w.mach2000_jet(nx, ny)
    g = w.JET_GAMMA
    p = orc.params(nx, ny, 1, dx, bc=[3, 1, 2, 1, 1, 1], cfl=0.25, inflow=inf)
    m0 = U[0].sum()
    c_jet = np.sqrt(g * 0.4127 / 5.0)
    for k in range(25):
        dt, st = orc.step(U, dx, g, p)
        assert st == 0
        if k == 0:  # bounded by the jet's speed, not the gas at rest (its
            # pressure carries the rounding of E - rho u^2 / 2 at E = 1.6e6)
            assert abs(dt / (0.25 * dx / (800.0 + 2.0 * c_jet)) - 1.0) < 1e-11
    rho = U[0, 0]
    assert np.isfinite(U).all() and rho.min() > 0
    assert U[0].sum() > m0  # mass came in
    assert rho[:8, :2].mean() > 2.0  # jet gas next to the inflow rows
    assert np.abs(rho[ny // 2:, :] - 0.5).max() < 1e-12  # nothing reached the upper half


def test_inflow_refused_where_undefined(orc):
    U = np.ones((4, 1, 8, 8))
    U[3] = 3.0
    inf = np.ones((4, 8))
    for bc, kw in [([1, 3, 1, 1, 1, 1], {"inflow": inf}),  # x+ side
                   ([1, 1, 3, 1, 1, 1], {"inflow": inf}),  # y- side
                   ([3, 1, 1, 1, 1, 1], {})]:               # no state
        p = orc.params(8, 8, 1, 0.1, bc=bc, **kw)
        assert orc.lib().orc_rhs(orc._dp(U), 8, 8, 1, 0.1, G, orc.C.byref(p),
                                 orc._dp(np.zeros_like(U))) == -1
    U3 = np.ones((5, 4, 4, 4))
    U3[4] = 3.0
    p = orc.params(4, 4, 4, 0.1, bc=[3, 1, 1, 1, 1, 1], inflow=np.ones((5, 16)))
    assert orc.lib().orc_rhs(orc._dp(U3), 4, 4, 4, 0.1, G, orc.C.byref(p),
                             orc._dp(np.zeros_like(U3))) == -1


def _jet_fail_step(orc, nx, ny, t_end=1e-3, **kw):
    """Steps the jet runs before its state goes non-physical (None: it
    reaches t_end)."""
    U, dx, inf = w.mach2000_jet(nx, ny)
    g = w.JET_GAMMA
    p = orc.params(nx, ny, 1, dx, bc=[3, 1, 2, 1, 1, 1], cfl=0.25, inflow=inf, **kw)
    t, n, st = orc.run(U, dx, g, p, t_end)
    return n if st else None


def test_mach2000_jet_robustness_by_weighting(orc):
    """Sec. 4.7 (reduced to 160 x 40, the paper's 2D splitting, global LF):
    the WENO-IS weights of Eq.(14)-(15) and of Eq.(8), as pure WENO
    schemes, carry the jet to t = 0.001 without a positivity limiter, as the
    paper reports for WENO-IS.  The present weights with the printed
    constants (lambda = c sigma^s, c = 1, sigma^s with the 1/60 of Eq.(28))
    do not: negative pressure in the jet's shear layer next to the inflow
    side within 30 (hybrid) or 60 (pure WENO) steps, with LF or LLF
    splitting; stronger regularization, lambda = 100 sigma^s, reaches
    t = 0.001.  (At 640 x 160: the same outcomes, the present scheme failing
    at step 52 with LF and 43 with LLF; altered oracles for readings Z1, Z6,
    Z13 and Z24 fail within 33-80 steps.)"""
    assert _jet_fail_step(orc, 160, 40, split=1, hybrid=2, weights=2) is None
    assert _jet_fail_step(orc, 160, 40, split=1, hybrid=2, weights=1) is None
    assert _jet_fail_step(orc, 160, 40, split=1, hybrid=2, c_reg=100.0) is None
    assert _jet_fail_step(orc, 160, 40, split=1, c_reg=100.0) is None
    n_lf = _jet_fail_step(orc, 160, 40, split=1)
    n_llf = _jet_fail_step(orc, 160, 40)
    n_pure = _jet_fail_step(orc, 160, 40, split=1, hybrid=2)
    assert n_lf is not None and n_lf < 40, n_lf
    assert n_llf is not None and n_llf < 60, n_llf
    assert n_pure is not None and n_pure < 80, n_pure
