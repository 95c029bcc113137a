"""Pins for the oracle's scalar WENO-L2IS reconstruction (CPU only).

The closed forms of Eq.(6), (11) and (27) are checked against their
definitions computed here from scratch: the reconstruction polynomial of each
stencil is the polynomial whose cell averages over the stencil's cells equal
the given values (the implicit h of Eq.(3)); candidate fluxes are its value at
x_{j+1/2} (Eq.(7)), smoothness indicators the derivative integrals of
Eq.(9)/(10), and the L2 error terms the integral of Eq.(26), all integrated
by Gauss-Legendre quadrature.  The weights are pinned by their limits.
"""
import numpy as np
import pytest

STENCILS = {0: [0, 1], 1: [-1, 0], 2: [0, 1, 2], 3: [-2, -1, 0]}
S01 = [-1, 0, 1]
S5 = [-2, -1, 0, 1, 2]
D = np.array([0.4, 0.2, 0.3, 0.1])
GX, GW = np.polynomial.legendre.leggauss(12)
GX, GW = 0.5 * GX, 0.5 * GW  # cell [-1/2, 1/2]


def recon_poly(offsets, vals):
    """Polynomial (numpy Polynomial) with the given cell averages, dx = 1."""
    r = len(offsets)
    A = np.zeros((r, r))
    for i, o in enumerate(offsets):
        for p in range(r):
            A[i, p] = ((o + 0.5) ** (p + 1) - (o - 0.5) ** (p + 1)) / (p + 1)
    c = np.linalg.solve(A, np.asarray(vals, dtype=np.float64))
    return np.polynomial.Polynomial(c)


def sub(a, offs):
    return [a[o + 2] for o in offs]


def ref_quantities(a):
    P = {k: recon_poly(o, sub(a, o)) for k, o in STENCILS.items()}
    q = np.array([P[k](0.5) for k in range(4)])
    beta = np.zeros(4)
    for k in range(4):
        r = len(STENCILS[k])
        for l in range(1, r):
            beta[k] += np.sum(GW * P[k].deriv(l)(GX) ** 2)
    P5 = recon_poly(S5, sub(a, S5))
    tau5 = sum(np.sum(GW * P5.deriv(l)(GX) ** 2) for l in (3, 4))
    P01 = recon_poly(S01, sub(a, S01))
    ref = {0: P01, 1: P01, 2: P[2], 3: P[3]}
    E = np.array([np.sum(GW * (P[k](GX) - ref[k](GX)) ** 2) for k in range(4)])
    return q, beta, tau5, E


def draws(n=200, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        scale = 10.0 ** rng.uniform(-3, 3)
        out.append(scale * rng.standard_normal(5) + rng.uniform(-1, 1))
    return out


def test_candidate_fluxes_beta_tau_E_match_integral_definitions(orc):
    for a in draws():
        q, beta, tau5, E = ref_quantities(a)
        _, dbg = orc.weno_l2is(a, 1.0)
        s = max(np.abs(a).max(), 1e-300)
        np.testing.assert_allclose(dbg["q"], q, rtol=0, atol=1e-13 * s)
        np.testing.assert_allclose(dbg["beta"], beta, rtol=0, atol=1e-12 * s * s)
        assert abs(dbg["tau5"] - tau5) <= 1e-12 * s * s
        np.testing.assert_allclose(dbg["E"], E, rtol=0, atol=1e-12 * s * s)


def test_E_closed_form_is_perfect_square(orc):
    for a in draws(50, 3):
        _, dbg = orc.weno_l2is(a, 1.0)
        assert dbg["E"][0] == dbg["E"][1] and dbg["E"][2] == 0 and dbg["E"][3] == 0
        assert dbg["E"][0] >= 0


@pytest.mark.parametrize("deg,stencils", [(1, [0, 1, 2, 3]), (2, [2, 3])])
def test_polynomial_reproduction(orc, deg, stencils):
    """Candidate fluxes reproduce h(x_{j+1/2}) for polynomials h of degree
    < stencil width, given cell averages of h."""
    rng = np.random.default_rng(deg)
    for _ in range(20):
        h = np.polynomial.Polynomial(rng.integers(-5, 6, deg + 1).astype(float))
        H = h.integ()
        a = [H(o + 0.5) - H(o - 0.5) for o in range(-2, 3)]
        _, dbg = orc.weno_l2is(a, 1.0)
        for k in stencils:
            assert abs(dbg["q"][k] - h(0.5)) <= 1e-12 * (1 + abs(h(0.5)))


def test_optimal_combination_is_fifth_order_upwind(orc):
    """sum d_k q_k = (2, -13, 47, 27, -3)/60 . f and reproduces quartics."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        a = rng.standard_normal(5)
        _, dbg = orc.weno_l2is(a, 1.0)
        lhs = float(D @ dbg["q"])
        rhs = float(np.array([2, -13, 47, 27, -3]) @ a) / 60.0
        assert abs(lhs - rhs) <= 1e-14 * (1 + np.abs(a).max())
    for _ in range(10):
        h = np.polynomial.Polynomial(rng.integers(-4, 5, 5).astype(float))
        H = h.integ()
        a = [H(o + 0.5) - H(o - 0.5) for o in range(-2, 3)]
        _, dbg = orc.weno_l2is(a, 1.0)
        assert abs(float(D @ dbg["q"]) - h(0.5)) <= 1e-12 * (1 + abs(h(0.5)))


def test_weights_sum_to_one_and_nonnegative(orc):
    for lam in (0.0, 1e-12, 1e-3, 1.0, 1e6):
        for a in draws(100, 5):
            _, dbg = orc.weno_l2is(a, lam)
            w = dbg["omega"]
            assert np.all(w >= 0)
            assert abs(w.sum() - 1.0) <= 4e-16


def test_lambda_zero_gives_optimal_weights(orc):
    """lambda = 0: alpha_k = d_k exactly, the optimal linear scheme."""
    for a in draws(50, 9):
        f, dbg = orc.weno_l2is(a, 0.0)
        np.testing.assert_allclose(dbg["omega"], D / D.sum(), rtol=1e-15)
        lin = float(np.array([2, -13, 47, 27, -3]) @ a) / 60.0
        assert abs(f - lin) <= 1e-13 * (1 + np.abs(a).max())


def test_large_lambda_recovers_original_weno_is_weights(orc):
    """lambda -> inf: alpha_k -> d_k (1 + tau5 / beta_k), Eq.(8) with eps -> 0,
    evaluated from the quadrature-based indicators."""
    rng = np.random.default_rng(21)
    for _ in range(100):
        a = rng.standard_normal(5)
        q, beta, tau5, E = ref_quantities(a)
        if beta.min() < 1e-6:
            continue
        _, dbg = orc.weno_l2is(a, 1e30, eps_w=1e-20)
        alpha = D * (1.0 + tau5 / beta)
        np.testing.assert_allclose(dbg["omega"], alpha / alpha.sum(), rtol=1e-9)


def test_discontinuity_in_one_stencil_gets_negligible_weight(orc):
    """A jump inside S3 only (between f_{j-2} and f_{j-1}) with large lambda:
    omega_3 vanishes and the result stays on the smooth branch."""
    a = np.array([50.0, 1.0, 1.1, 1.2, 1.3])
    f, dbg = orc.weno_l2is(a, 1e3)
    assert dbg["omega"][3] < 1e-6
    assert abs(f - 1.15) < 1e-3


@pytest.mark.parametrize("lam", [1.0, 1e-6])
def test_fifth_order_on_smooth_data(orc, lam):
    """Away from critical points the reconstruction error is O(dx^5)."""
    errs = []
    hs = [0.1 / 2 ** k for k in range(4)]
    for h in hs:
        x0 = 0.37
        # cell averages of sin on cells centred at x0 + o h, h(x) = sin
        a = [(np.cos(x0 + (o - 0.5) * h) - np.cos(x0 + (o + 0.5) * h)) / h for o in range(-2, 3)]
        f, _ = orc.weno_l2is(a, lam)
        errs.append(abs(f - np.sin(x0 + 0.5 * h)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 4.6, rates


# ------------------------------------------ comparison weights (Sec. 2.2, 2.4)
W_IS, W_IS_B01 = 1, 2


def beta01_quadrature(a):
    """Eq.(9) on the 3-point stencil S01 = {j-1, j, j+1}: the first and
    second derivative integrals of its quadratic reconstruction."""
    P = recon_poly(S01, sub(a, S01))
    return sum(np.sum(GW * P.deriv(l)(GX) ** 2) for l in (1, 2))


@pytest.mark.parametrize("weights", [W_IS, W_IS_B01])
def test_comparison_weights_from_the_integral_definitions(orc, weights):
    """Eq.(8) (and with Eq.(14) the beta_01 factor on the two 2-point
    stencils) evaluated from the quadrature-based beta_k, tau_5 and beta_01:
    the weights and the flux of the oracle agree."""
    eps = 1e-20
    for a in draws(120, 31):
        q, beta, tau5, _ = ref_quantities(a)
        r = tau5 / (beta + eps)
        if weights == W_IS_B01:
            r01 = tau5 / (beta01_quadrature(a) + eps)
            r[:2] *= r01
        alpha = D * (1.0 + r)
        om = alpha / alpha.sum()
        f, dbg = orc.weno(a, weights, 0.0, eps)
        np.testing.assert_allclose(dbg["omega"], om, rtol=1e-9, atol=1e-13)
        assert abs(f - om @ q) <= 1e-10 * (1 + np.abs(a).max())
        assert np.all(dbg["omega"] >= 0) and abs(dbg["omega"].sum() - 1) <= 8.9e-16


def test_original_weights_are_the_large_lambda_limit(orc):
    """Two code paths of the oracle: Eq.(28) with lambda -> infinity equals
    Eq.(8) (E_k and eps drop out where beta_k is not tiny)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        a = rng.standard_normal(5)
        _, d1 = orc.weno(a, W_IS, 0.0, 1e-20)
        if d1["beta"].min() < 1e-6:
            continue
        _, d2 = orc.weno(a, 0, 1e200, 1e-20)
        np.testing.assert_allclose(d1["omega"], d2["omega"], rtol=1e-12)


@pytest.mark.parametrize("weights", [W_IS, W_IS_B01])
def test_comparison_weights_fifth_order_on_smooth_data(orc, weights):
    """Away from critical points tau5 / beta_k = O(dx^4) (Eq.(13)), so the
    reconstruction keeps fifth order."""
    errs = []
    for h in [0.1 / 2 ** k for k in range(4)]:
        x0 = 0.37
        a = [(np.cos(x0 + (o - 0.5) * h) - np.cos(x0 + (o + 0.5) * h)) / h for o in range(-2, 3)]
        f, _ = orc.weno(a, weights)
        errs.append(abs(f - np.sin(x0 + 0.5 * h)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 4.6, rates


def test_beta01_weights_favour_two_point_stencils_next_to_a_shock(orc):
    """The case of Eq.(14a) in Sec. 2.4: a jump inside S3 only, smooth data in
    S0, S1, S2.  tau5 = O(1) while beta_0, beta_1, beta_01, beta_2 are small,
    so the product of Eq.(14) gives the 2-point stencils far more weight,
    relative to their optimal weights, than the 3-point stencil S2; the
    original Eq.(8) weights do not."""
    h = 0.01
    smooth = [np.sin(1.0 + o * h) for o in range(-2, 3)]
    a = np.array(smooth)
    a[0] += 1.0  # the jump between f_{j-2} and f_{j-1}
    _, db = orc.weno(a, W_IS_B01)
    _, di = orc.weno(a, W_IS)
    rel_b = (db["omega"][0] / D[0]) / (db["omega"][2] / D[2])
    rel_i = (di["omega"][0] / D[0]) / (di["omega"][2] / D[2])
    assert rel_b > 1e3 * rel_i and rel_b > 1e3, (rel_b, rel_i)
