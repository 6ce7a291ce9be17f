"""Pins of the oracle's host thermodynamics against what the paper and the mathematics fix.

Each test uses an independent route (closed-form antiderivatives, scipy adaptive
quadrature, finite differences, printed values) -- never the oracle's own Simpson or
bisection code -- so that a dropped term or wrong sign in the oracle fails here.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def cs(Tr, a=0.5, **kw):
    e, s = O.eos_build(O.make_eos(base=O.BASE_CS, a=a, b=4.0, R=1.0, Tr=Tr, **kw))
    return e, s


def pr(Tr, **kw):
    e, s = O.eos_build(O.make_eos(base=O.BASE_PR, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, Tr=Tr, **kw))
    return e, s


# ---------------------------------------------------------------- critical point
def test_cs_critical_point_matches_printed_constant_and_definition():
    g = _gold("maxwell.json")["Tc_over_a_bR"]["value"]
    e, _ = cs(0.5)
    assert e.Tc * e.b * e.R / e.a == pytest.approx(g, rel=1e-3)
    # definition: dp/drho = d2p/drho2 = 0 at (rho_c, Tc); check with finite differences of p
    ec = O.cs_critical_eta()
    rc = 4 * ec / e.b
    crit = O.make_eos(base=O.BASE_CS, a=0.5, b=4.0, R=1.0, Tr=0.5)
    O.eos_build(crit)
    crit.T = crit.Tc  # evaluate the base EOS at the critical temperature
    h = 1e-4
    p = lambda r: float(O.base_p(crit, r)[0])
    d1 = (p(rc + h) - p(rc - h)) / (2 * h)
    d2 = (p(rc + h) - 2 * p(rc) + p(rc - h)) / h**2
    scale = p(rc) / rc
    assert abs(d1) < 1e-7 * scale / 1e-3
    assert abs(d2) < 1e-5 * scale / rc


def test_pr_critical_point_matches_textbook_ratio():
    # textbook PR: a = 0.45724 R^2 Tc^2/pc, b = 0.07780 R Tc/pc  =>  Tc = 0.07780 a /(0.45724 b R)
    e, _ = pr(0.5)
    assert e.Tc == pytest.approx(0.07780 * e.a / (0.45724 * e.b * e.R), rel=2e-4)


def test_base_derivative_matches_finite_difference():
    for e, _ in (cs(0.5), pr(0.6)):
        for r in np.linspace(0.05, 0.9, 7) * (e.rho_l):
            h = 1e-6 * r
            fd = (O.base_p(e, r + h)[0] - O.base_p(e, r - h)[0]) / (2 * h)
            assert O.base_dp(e, r)[0] == pytest.approx(fd, rel=1e-6, abs=1e-10)


# ---------------------------------------------------------------- Maxwell rule
def _cs_antiderivative(e, r):
    """closed form of int p/rho^2 for C-S: RT[ln rho + (4eta-3eta^2)/(1-eta)^2] - a rho"""
    eta = e.b * r / 4
    return e.scale * (e.R * e.T * (math.log(r) + (4 * eta - 3 * eta**2) / (1 - eta) ** 2) - e.a * r)


def _pr_antiderivative(e, r):
    kappa = 0.37464 + 1.54226 * e.omega - 0.26992 * e.omega**2
    al = (1 + kappa * (1 - math.sqrt(e.T / e.Tc))) ** 2
    b = e.b
    s2 = math.sqrt(2.0)
    return e.scale * (e.R * e.T * math.log(r / (1 - b * r))
                      - e.a * al / (2 * s2 * b) * math.log((s2 - 1 + b * r) / (s2 + 1 - b * r)))


@pytest.mark.parametrize("Tr", [0.9, 0.7, 0.5, 0.35])
def test_cs_maxwell_equal_area_closed_form(Tr):
    e, _ = cs(Tr)
    # equal pressures
    assert O.base_p(e, e.rho_v)[0] == pytest.approx(e.p_sat, rel=1e-9)
    assert O.base_p(e, e.rho_l)[0] == pytest.approx(e.p_sat, rel=1e-6, abs=1e-12)
    # Eq. MaxwellRule with the closed-form antiderivative
    lhs = e.p_sat * (1 / e.rho_v - 1 / e.rho_l)
    rhs = _cs_antiderivative(e, e.rho_l) - _cs_antiderivative(e, e.rho_v)
    assert lhs == pytest.approx(rhs, rel=1e-9)


@pytest.mark.parametrize("Tr", [0.8, 0.6, 0.5, 0.47])
def test_pr_maxwell_equal_area_closed_form(Tr):
    e, _ = pr(Tr)
    assert O.base_p(e, e.rho_v)[0] == pytest.approx(e.p_sat, rel=1e-9)
    lhs = e.p_sat * (1 / e.rho_v - 1 / e.rho_l)
    rhs = _pr_antiderivative(e, e.rho_l) - _pr_antiderivative(e, e.rho_v)
    assert lhs == pytest.approx(rhs, rel=1e-9)


def test_printed_saturation_values():
    g = _gold("maxwell.json")
    e, _ = cs(0.5)
    assert e.p_sat == pytest.approx(g["p_sat_Tr05"]["value"], rel=0.05)
    assert O.base_p(e, 1.001 * e.rho_l)[0] == pytest.approx(g["p_liq_plus_0p1pct_Tr05"]["value"], rel=0.1)
    for key, Tr, tol in (("ratio_Tr06", 0.6, 0.01), ("ratio_Tr05", 0.5, 0.005),
                         ("ratio_Tr035", 0.35, 0.005), ("ratio_Tr065", 0.65, 0.01)):
        e, _ = cs(Tr)
        assert e.rho_l / e.rho_v == pytest.approx(g[key]["value"], rel=tol), key


def test_standard_procedure_keeps_coexistence():
    """Sec. III.B: scaling a at fixed Tr (or multiplying the EOS) leaves rho_v, rho_l unchanged."""
    e1, _ = cs(0.5, a=0.5)
    e2, _ = cs(0.5, a=0.141)
    e3, _ = cs(0.5, a=0.5, scale=0.3)
    for e in (e2, e3):
        assert e.rho_v == pytest.approx(e1.rho_v, rel=1e-8)
        assert e.rho_l == pytest.approx(e1.rho_l, rel=1e-10)
    assert e2.p_sat == pytest.approx(e1.p_sat * 0.141 / 0.5, rel=1e-8)


# ---------------------------------------------------------------- Smooth loop
SMOOTH_CASES = [
    dict(Tr=0.5, alpha=0.610), dict(Tr=0.5, alpha=0.342), dict(Tr=0.5, alpha=0.216),
    dict(Tr=0.5, alpha=0.554, k_vap=4.0), dict(Tr=0.5, alpha=0.207, k_vap=4.0),
    dict(Tr=0.5, a=0.363, alpha=0.775, k_vap=2 / 0.363), dict(Tr=0.6, a=0.387, alpha=0.834, k_vap=2 / 0.387),
    dict(Tr=0.7, alpha=0.5), dict(Tr=0.35, a=0.363, alpha=0.4, k_vap=4.0),
]


def _smooth(c):
    c = dict(c)
    return cs(c.pop("Tr"), a=c.pop("a", 0.5), shape=O.SHAPE_SMOOTH, **c)


def _check_knot_continuity(e):
    knots = [(e.rho_v, e.p_sat_new, e.slope_v), (e.rho_max, e.p_max, 0.0),
             (e.rho_min, e.p_min, 0.0), (e.rho_l, e.p_sat_new, e.slope_l)]
    for r, pk, sk in knots:
        h = 1e-9 * r
        left, right = O.eos_p(e, r - h)[0], O.eos_p(e, r + h)[0]
        assert left == pytest.approx(pk, abs=1e-8 * max(abs(pk), e.p_sat_new) + abs(sk) * 2 * h + 1e-15)
        assert right == pytest.approx(pk, abs=1e-8 * max(abs(pk), e.p_sat_new) + abs(sk) * 2 * h + 1e-15)
        # one-sided finite-difference slopes on both sides agree with the prescribed slope
        # (the ellipse arcs can be sharply curved next to the saturated densities, so the
        # step is tiny; two step sizes are combined by Richardson extrapolation)
        d = 1e-8 * r
        one = lambda dd: ((O.eos_p(e, r)[0] - O.eos_p(e, r - dd)[0]) / dd,
                          (O.eos_p(e, r + dd)[0] - O.eos_p(e, r)[0]) / dd)
        (l1, r1), (l2, r2) = one(d), one(d / 2)
        sl, sr = 2 * l2 - l1, 2 * r2 - r1
        tol = 1e-3 * max(abs(e.slope_v), abs(e.slope_l)) + 1e-9
        assert sl == pytest.approx(sk, abs=tol)
        assert sr == pytest.approx(sk, abs=tol)


@pytest.mark.parametrize("case", SMOOTH_CASES)
def test_smooth_loop_knots_and_sound_speed_continuity(case):
    e, _ = _smooth(case)
    _check_knot_continuity(e)
    # vapor and liquid branch slopes as prescribed (Sec. III.D): vapor scaled by k_vap, liquid unchanged
    assert e.slope_v == pytest.approx(e.k_vap * O.base_dp(e, e.rho_v)[0], rel=1e-12)
    assert e.slope_l == pytest.approx(O.base_dp(e, e.rho_l)[0], rel=1e-12)
    # p_min rule
    assert e.p_min == pytest.approx(e.p_sat_new - e.alpha * (e.p_sat - e.p_min_base), rel=1e-12)
    # bulk branches unchanged up to the offsets
    for r in (0.5 * e.rho_v, 0.9 * e.rho_v):
        assert O.eos_p(e, r)[0] == pytest.approx(e.k_vap * O.base_p(e, r)[0], rel=1e-12)
    for r in (1.01 * e.rho_l, 1.05 * e.rho_l):
        assert O.eos_p(e, r)[0] == pytest.approx(O.base_p(e, r)[0] + (e.k_vap - 1) * e.p_sat, rel=1e-12)


@pytest.mark.parametrize("case", SMOOTH_CASES[5:8])
def test_moved_knots_keep_the_loop_continuous(case):
    """Knots treated as free parameters (finite-difference gradients): after moving each one the
    refitted ellipses still meet the saturated branches with their slopes and the knots flat."""
    e, _ = _smooth(case)
    k = [e.rho_max, e.p_max, e.rho_min, e.p_min]
    assert O.eos_set_knots(e, *k).a1sq == e.a1sq and O.eos_set_knots(e, *k).b3 == e.b3
    for j, rel in ((0, 0.01), (1, 0.02), (2, -0.01), (3, 0.03)):
        kk = list(k)
        kk[j] += rel * abs(kk[j])
        _check_knot_continuity(O.eos_set_knots(e, *kk))
    with pytest.raises(O.OracleError):
        O.eos_set_knots(e, e.rho_min, e.p_max, e.rho_max, e.p_min)


@pytest.mark.parametrize("case", SMOOTH_CASES)
def test_smooth_loop_obeys_maxwell(case):
    """p_max makes the shaped EOS satisfy Eq. MaxwellRule at the base Maxwell densities."""
    e, _ = _smooth(case)
    f = lambda r: (e.p_sat_new - O.eos_p(e, r)[0]) / r**2
    pts = [e.rho_v, e.rho_max, e.rho_min, e.rho_l]
    total = 0.0
    scale = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        # adaptive quadrature in ln(rho), independent of the oracle's Simpson rule
        val, err = integrate.quad(lambda s: f(math.exp(s)) * math.exp(s), math.log(a), math.log(b),
                                  epsabs=0, epsrel=1e-12, limit=400)
        total += val
        scale += abs(val)
    assert abs(total) < 1e-8 * scale


@pytest.mark.parametrize("Tr", [0.9, 0.7, 0.5])
def test_eps_solves_mechanical_stability(Tr):
    """eps from Newton/Simpson (Sec. III.A) zeroes Eq. VaporLiqEq under an independent quadrature."""
    e, sigma = cs(Tr)
    G = -1.0

    def integrand(s, eps):
        r = math.exp(s)
        p = O.eos_p(e, r)[0]
        dp = O.eos_dp(e, r)[0]
        psi = math.sqrt(2 * (p - r / 3) / G)
        dpsi = (dp - 1 / 3) / (G * psi)
        return (e.p_sat - p) * dpsi * psi ** (-1 - eps) * r

    pts = [e.rho_v, e.rho_max, e.rho_min, e.rho_l]
    tot, scale = 0.0, 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        v, _ = integrate.quad(integrand, math.log(a), math.log(b), args=(e.eps,), epsrel=1e-12, epsabs=0, limit=400)
        tot += v
        scale += abs(v)
    assert abs(tot) < 1e-8 * scale
    assert sigma == pytest.approx(e.eps / 16.0, rel=1e-14)  # eps = -16 G sigma with G = -1


def test_eps_near_linear_in_Tr():
    """Sec. III.A / Fig. e_CS: for C-S a=0.5 the eps(Tr) curve approaches a straight line."""
    trs = np.array([0.5, 0.6, 0.7, 0.8, 0.9])
    eps = np.array([cs(t)[0].eps for t in trs])
    assert np.all(np.diff(eps) < 0)
    second = np.abs(np.diff(eps, 2)).max()
    first = np.abs(np.diff(eps)).mean()
    assert second < 0.1 * first


def test_eps_independent_of_G():
    e1, s1 = O.eos_build(O.make_eos(Tr=0.6), G=-1.0)
    e2, s2 = O.eos_build(O.make_eos(Tr=0.6), G=-2.5)
    assert e2.eps == pytest.approx(e1.eps, rel=1e-9)
    assert s2 == pytest.approx(s1 / 2.5, rel=1e-9)


def test_peng_loop_satisfies_shan_condition_and_theta():
    e, _ = cs(0.6, a=0.387, shape=O.SHAPE_PENG, r_theta=0.45)
    assert e.rho_v < e.rho_m < e.rho_l
    # Eq. PengEOS: value p0 at both saturated densities and at rho_m
    for r in (e.rho_v, e.rho_m, e.rho_l):
        inside = e.p_sat + e.theta * (r - e.rho_v) * (r - e.rho_l) * (r - e.rho_m)
        assert inside == pytest.approx(e.p_sat, rel=1e-12)
    # Eq. PengTheta: slopes blend the bulk slopes with weights (1-r, r)
    th_v = e.slope_v / ((e.rho_v - e.rho_m) * (e.rho_v - e.rho_l))
    th_l = e.slope_l / ((e.rho_l - e.rho_m) * (e.rho_l - e.rho_v))
    assert e.theta == pytest.approx((1 - e.r_theta) * th_v + e.r_theta * th_l, rel=1e-12)
    # Eq. ShanVaporLiqEq (eps = 0) by independent quadrature
    G = -1.0

    def integrand(s):
        r = math.exp(s)
        p = O.eos_p(e, r)[0]
        dp = O.eos_dp(e, r)[0]
        psi = math.sqrt(2 * (p - r / 3) / G)
        return (e.p_sat - p) * (dp - 1 / 3) / (G * psi) / psi * r

    v1, _ = integrate.quad(integrand, math.log(e.rho_v), math.log(e.rho_m), epsrel=1e-12, limit=400)
    v2, _ = integrate.quad(integrand, math.log(e.rho_m), math.log(e.rho_l), epsrel=1e-12, limit=400)
    assert abs(v1 + v2) < 1e-8 * (abs(v1) + abs(v2))


def test_pr_stiffness_reported():
    """With the textbook PR at Tr=0.5 psi^2 turns negative for a compressed liquid."""
    e, _ = pr(0.5)
    r = np.linspace(e.rho_l, 1.1 * e.rho_l, 50)
    assert (O.base_p(e, r) - r / 3).max() > 0
