"""Pins for the oracle's characteristic system and per-face flux (CPU only).

* The physical flux is compared with an independent numpy formula.
* L R = I; R diag(lambda) L equals the flux Jacobian at the Roe state, taken
  here by complex-step differentiation of the independent flux (exact to
  round-off); the Roe property A(U_R - U_L) = F_R - F_L holds.
* The detector of Eq.(30)-(31) vanishes exactly on polynomial data of degree
  <= 4 and equals the fifth difference on degree-5 data.
* The linear flux of Eq.(34) (as read: 1/60 included, splitting speed)
  equals the WENO path with lambda = 0, whose weights are the optimal d_k.
"""
import numpy as np
import pytest

GAMMA = 1.4


def flux_np(U, d, g=GAMMA):
    """Independent Euler flux along d for U (nvar,), real or complex."""
    nvar = U.shape[0]
    dim = nvar - 2
    rho = U[0]
    vel = [U[1 + k] / rho for k in range(dim)]
    E = U[-1]
    p = (g - 1) * (E - 0.5 * rho * sum(v * v for v in vel))
    F = [rho * vel[d]] + [rho * vel[d] * vel[k] + (p if k == d else 0) for k in range(dim)]
    F.append((E + p) * vel[d])
    return np.array(F)


def jacobian_cs(U, d, g=GAMMA):
    n = U.shape[0]
    J = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        Uc = U.astype(complex)
        Uc[k] += 1j * h
        J[:, k] = flux_np(Uc, d, g).imag / h
    return J


def rand_state(rng, nvar):
    dim = nvar - 2
    rho = rng.uniform(0.2, 2.0)
    vel = rng.uniform(-1.5, 1.5, dim)
    p = rng.uniform(0.1, 3.0)
    return np.array([rho] + list(rho * vel) + [p / (GAMMA - 1) + 0.5 * rho * vel @ vel])


CASES = [(nv, d) for nv in (3, 4, 5) for d in range(nv - 2)]


@pytest.mark.parametrize("nvar,d", CASES)
def test_physical_flux(orc, nvar, d):
    rng = np.random.default_rng(nvar * 10 + d)
    for _ in range(20):
        U = rand_state(rng, nvar)
        F, prim = orc.phys_flux(nvar, d, GAMMA, U)
        np.testing.assert_allclose(F, flux_np(U, d), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("nvar,d", CASES)
def test_eigensystem_and_roe_property(orc, nvar, d):
    rng = np.random.default_rng(100 + nvar * 10 + d)
    for _ in range(30):
        UL, UR = rand_state(rng, nvar), rand_state(rng, nvar)
        L, R, lam, roe = orc.roe_eigen(nvar, d, GAMMA, UL, UR)
        np.testing.assert_allclose(L @ R, np.eye(nvar), atol=1e-13)
        # Jacobian at the Roe state: any state with velocity u~ and enthalpy H~
        rho = 1.3
        ut = roe[1:1 + nvar - 2]
        Ht = roe[4]
        q = 0.5 * ut @ ut
        E = (rho * Ht + (GAMMA - 1) * rho * q) / GAMMA
        Ustar = np.array([rho] + list(rho * ut) + [E])
        A = jacobian_cs(Ustar, d)
        RLA = R @ np.diag(lam) @ L
        np.testing.assert_allclose(RLA, A, rtol=0, atol=1e-12 * (1 + np.abs(A).max()))
        # Roe property
        dF = flux_np(UR, d) - flux_np(UL, d)
        np.testing.assert_allclose(RLA @ (UR - UL), dF, rtol=0,
                                   atol=1e-12 * (1 + np.abs(dF).max()))
        # Roe density is the geometric mean
        assert abs(roe[0] - np.sqrt(UL[0] * UR[0])) <= 1e-15 * roe[0]
        # every characteristic variable carries density units: scaling the
        # mass unit (rho, p, E by s at fixed velocity and sound speed) scales
        # L.U by s; scaling the time unit (velocities and c by k) leaves it
        X = rand_state(rng, nvar)
        s = 2.5
        Ls = orc.roe_eigen(nvar, d, GAMMA, s * UL, s * UR)[0]
        np.testing.assert_allclose(Ls @ (s * X), s * (L @ X), rtol=1e-12,
                                   atol=1e-12 * np.abs(L @ X).max())
        k = np.array([1.0] + [3.0] * (nvar - 2) + [9.0])
        Lk = orc.roe_eigen(nvar, d, GAMMA, k * UL, k * UR)[0]
        np.testing.assert_allclose(Lk @ (k * X), L @ X, rtol=1e-11,
                                   atol=1e-11 * np.abs(L @ X).max())


def poly_stencil(rng, nvar, deg):
    """Six states whose components are integer polynomials of cell index."""
    m = np.arange(-2, 4, dtype=float)
    base = rand_state(rng, nvar)
    base = np.round(base * 8) / 8 + np.array([4.0] + [0.0] * (nvar - 2) + [40.0])
    U6 = np.zeros((6, nvar))
    for i in range(nvar):
        c = rng.integers(-2, 3, deg + 1).astype(float) / 64.0
        U6[:, i] = base[i] + np.polynomial.polynomial.polyval(m, c)
    return U6


@pytest.mark.parametrize("nvar,d", CASES)
def test_detector_annihilates_quartics(orc, nvar, d):
    rng = np.random.default_rng(7 + nvar + d)
    p = orc.params(8, 1, 1, 0.1)
    for deg in range(5):
        U6 = poly_stencil(rng, nvar, deg)
        _, fl, sg = orc.face_flux(nvar, d, GAMMA, p, 1e-7, U6)
        assert np.all(sg == 0.0), (deg, sg)
        assert np.all(fl == 1)


@pytest.mark.parametrize("nvar,d", CASES)
def test_detector_fifth_difference(orc, nvar, d):
    """Degree-5 data: dU5 = -120 a5, so dv^s = -2 L^s.a5 and
    sigma^s = (2 L^s.a5 / rho~)^2."""
    rng = np.random.default_rng(70 + nvar + d)
    p = orc.params(8, 1, 1, 0.1)
    m = np.arange(-2, 4, dtype=float)
    for _ in range(10):
        U6 = poly_stencil(rng, nvar, 2)
        a5 = rng.uniform(-1, 1, nvar) * 1e-3
        U6 = U6 + np.outer(m ** 5, a5)
        _, _, sg = orc.face_flux(nvar, d, GAMMA, p, 1e-7, U6)
        L, R, lam, roe = orc.roe_eigen(nvar, d, GAMMA, U6[2], U6[3])
        expect = (2.0 * (L @ a5) / roe[0]) ** 2
        np.testing.assert_allclose(sg, expect, rtol=1e-9)


@pytest.mark.parametrize("nvar,d", CASES)
@pytest.mark.parametrize("split", [0, 1, 2])
def test_linear_flux_equals_optimal_weight_weno(orc, nvar, d, split):
    rng = np.random.default_rng(300 + nvar * 10 + d + split)
    alpha_lf = np.full(nvar, 3.0)
    for _ in range(20):
        U6 = np.array([rand_state(rng, nvar) for _ in range(6)])
        plin = orc.params(8, 1, 1, 0.1, hybrid=orc.HYB_LINEAR_ONLY, split=split)
        pw = orc.params(8, 1, 1, 0.1, hybrid=orc.HYB_WENO_ONLY, c_reg=0.0, split=split)
        F1, fl1, _ = orc.face_flux(nvar, d, GAMMA, plin, 1e-7, U6, alpha_lf)
        F2, fl2, _ = orc.face_flux(nvar, d, GAMMA, pw, 1e-7, U6, alpha_lf)
        assert np.all(fl1 == 1) and np.all(fl2 == 0)
        np.testing.assert_allclose(F1, F2, rtol=0, atol=2e-13 * (1 + np.abs(F1).max()))


@pytest.mark.parametrize("nvar,d", CASES)
def test_constant_state_gives_physical_flux(orc, nvar, d):
    rng = np.random.default_rng(5 + nvar + d)
    for hyb in range(4):
        p = orc.params(8, 1, 1, 0.1, hybrid=hyb)
        U = rand_state(rng, nvar)
        U6 = np.tile(U, (6, 1))
        F, fl, sg = orc.face_flux(nvar, d, GAMMA, p, 1e-7, U6)
        np.testing.assert_allclose(F, flux_np(U, d), rtol=1e-14, atol=1e-14)
        assert np.all(sg == 0.0)


@pytest.mark.parametrize("nvar,d", CASES)
def test_switch_threshold_per_field_and_per_face(orc, nvar, d):
    rng = np.random.default_rng(900 + nvar + d)
    for _ in range(20):
        U6 = np.array([rand_state(rng, nvar) for _ in range(6)])
        p = orc.params(8, 1, 1, 0.1)
        _, _, sg = orc.face_flux(nvar, d, GAMMA, p, 1.0, U6)
        thr = float(np.median(sg))
        _, fl, _ = orc.face_flux(nvar, d, GAMMA, p, thr, U6)
        np.testing.assert_array_equal(fl, (sg < thr).astype(np.uint8))
        pf = orc.params(8, 1, 1, 0.1, hybrid=orc.HYB_PER_FACE)
        _, fl2, _ = orc.face_flux(nvar, d, GAMMA, pf, thr, U6)
        assert np.all(fl2 == (1 if sg.max() < thr else 0))
        # sigma == threshold takes the WENO branch
        _, fl3, _ = orc.face_flux(nvar, d, GAMMA, p, float(sg[0]), U6)
        assert fl3[0] == 0


def test_lf_and_roe_splitting_speeds(orc):
    """Roe splitting uses |lambda~|; LF uses the supplied global speed; LLF the
    stencil max.  With a stencil of identical states all three agree when the
    LF speed equals the cell eigenvalue magnitude."""
    rng = np.random.default_rng(3)
    nvar, d = 5, 1
    U = rand_state(rng, nvar)
    U6 = np.tile(U, (6, 1))
    F, prim = orc.phys_flux(nvar, d, GAMMA, U)
    un, c = prim[1 + d], prim[5]
    a = np.array([abs(un - c)] + [abs(un)] * 3 + [abs(un + c)])
    outs = []
    for split in (0, 1, 2):
        p = orc.params(8, 8, 8, 0.1, split=split, hybrid=orc.HYB_WENO_ONLY)
        outs.append(orc.face_flux(nvar, d, GAMMA, p, 1e-7, U6, a)[0])
    np.testing.assert_allclose(outs[0], outs[1], rtol=1e-14)
    np.testing.assert_allclose(outs[0], outs[2], rtol=1e-14)
