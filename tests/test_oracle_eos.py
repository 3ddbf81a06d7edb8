"""Pins of the oracle's Peng-Robinson EOS (Eq. (21)) against the paper's printed
coexistence densities and against textbook properties of the EOS.

Nothing here re-derives a formula the oracle uses: the checks are independent
numerical quadrature and differentiation, the critical-point conditions, and
the numbers the paper prints.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle as O

A2, A3, B, R, OMEGA = 2.0 / 49.0, 3.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def _p(a):
    tc, k = O.Tc(a, B, R), O.kappa(OMEGA)
    return (lambda rho, T: O.p_eos(rho, T, a, B, R, tc, k)), tc, k


def test_critical_point_conditions(golden):
    """At T = T_c the isotherm has a horizontal inflection, and the critical
    compressibility p_c/(rho_c R T_c) is the Peng-Robinson value 0.3074."""
    for a in (A2, A3):
        p, tc, k = _p(a)
        rho = np.linspace(0.2, 8.0, 200001)
        dp = np.array([O.dp_drho(r, tc, a, B, R, tc, k) for r in rho[::100]])
        i = int(np.argmin(dp))
        # the minimum of dp/drho along the critical isotherm is ~0 (the rounded
        # coefficients 0.45724 and 0.0778 shift it by ~1e-5 of R T_c)
        assert abs(dp[i]) < 1e-4 * R * tc
        rho_c = rho[::100][i]
        zc = p(rho_c, tc) / (rho_c * R * tc)
        ref = golden["pr_critical_compressibility"]
        assert abs(zc - ref["value"]) < ref["tolerance"]
        # phi(T_c) = 1 for any kappa
        assert O.phi(tc, tc, k) == pytest.approx(1.0, abs=1e-15)


def test_maxwell_matches_paper(golden):
    ref = golden["coexistence_086Tc"]
    e = ref["eos"]
    tc = O.Tc(e["a"], e["b"], e["R"])
    rv, rl, ps = O.maxwell(e["a"], e["b"], e["R"], e["omega"], ref["Ts_over_Tc"] * tc)
    assert abs(rl - ref["rho_L"]) < ref["rho_L_digits"]
    assert abs(rv - ref["rho_V"]) < ref["rho_V_digits"]


@pytest.mark.parametrize("a", [A2, A3])
@pytest.mark.parametrize("theta", [0.7, 0.86, 0.95])
def test_maxwell_equal_area_by_quadrature(a, theta):
    """Equal pressures and equal areas, checked with adaptive quadrature of the
    oracle's p_EOS (the oracle itself uses a closed-form antiderivative)."""
    p, tc, k = _p(a)
    T = theta * tc
    rv, rl, ps = O.maxwell(a, B, R, OMEGA, T)
    assert rv < rl
    assert abs(p(rv, T) - ps) < 1e-11 * ps
    assert abs(p(rl, T) - ps) < 1e-11 * ps
    area, _ = integrate.quad(lambda r: (p(r, T) - ps) / r ** 2, rv, rl, limit=400, epsabs=1e-14, epsrel=1e-13)
    scale = integrate.quad(lambda r: abs(p(r, T) - ps) / r ** 2, rv, rl, limit=400)[0]
    assert abs(area) < 1e-9 * scale
    # both roots sit on stable branches
    assert O.dp_drho(rv, T, a, B, R, tc, k) > 0 and O.dp_drho(rl, T, a, B, R, tc, k) > 0


def test_coexistence_independent_of_a():
    """At fixed T/T_c and b, p scales with a, so the coexistence densities do not depend on a."""
    r2 = O.maxwell(A2, B, R, OMEGA, 0.86 * O.Tc(A2, B, R))
    r3 = O.maxwell(A3, B, R, OMEGA, 0.86 * O.Tc(A3, B, R))
    assert r2[0] == pytest.approx(r3[0], rel=1e-10)
    assert r2[1] == pytest.approx(r3[1], rel=1e-10)
    assert r3[2] / r2[2] == pytest.approx(1.5, rel=1e-10)


@pytest.mark.parametrize("rho", [0.05, 0.38, 2.0, 6.5, 8.0])
@pytest.mark.parametrize("theta", [0.5, 0.86, 1.1])
def test_eos_derivatives_by_differences(rho, theta):
    """(dp/dT)_rho and (dp/drho)_T against 4th-order central differences of p."""
    for a in (A2, A3):
        p, tc, k = _p(a)
        T = theta * tc
        hT, hr = 1e-4 * T, 1e-4 * rho
        dT_num = (-p(rho, T + 2 * hT) + 8 * p(rho, T + hT) - 8 * p(rho, T - hT) + p(rho, T - 2 * hT)) / (12 * hT)
        dr_num = (-p(rho + 2 * hr, T) + 8 * p(rho + hr, T) - 8 * p(rho - hr, T) + p(rho - 2 * hr, T)) / (12 * hr)
        scale_T = abs(rho * R / (1 - B * rho)) + 1e-300
        scale_r = abs(R * T / (1 - B * rho) ** 2)
        assert abs(O.dp_dT(rho, T, a, B, R, tc, k) - dT_num) < 1e-8 * scale_T
        assert abs(O.dp_drho(rho, T, a, B, R, tc, k) - dr_num) < 1e-8 * scale_r
        # dphi/dT against differences of phi
        dphi_num = (O.phi(T + hT, tc, k) - O.phi(T - hT, tc, k)) / (2 * hT)
        assert O.dphi_dT(T, tc, k) == pytest.approx(dphi_num, rel=1e-7)


def test_ideal_gas_limit():
    """With a = 0 and b -> 0 the EOS reduces to p = rho R T (Sec. 2 after Eq. (15))."""
    tc, k = 0.1, O.kappa(OMEGA)
    for rho in (0.1, 1.0, 5.0):
        assert O.p_eos(rho, 0.07, 0.0, 1e-14, R, tc, k) == pytest.approx(rho * R * 0.07, rel=1e-12)
        assert O.dp_dT(rho, 0.07, 0.0, 1e-14, R, tc, k) == pytest.approx(rho * R, rel=1e-12)


def test_physical_ratios(golden):
    """Viscosity and conductivity ratios the paper quotes for the coexistence densities."""
    rv, rl, _ = O.maxwell(A3, B, R, OMEGA, 0.86 * O.Tc(A3, B, R))
    v = golden["viscosity_ratio"]
    assert abs(rl * v["nu_L"] / (rv * v["nu_V"]) - v["value"]) < v["tolerance"]
    c = golden["conductivity_ratio"]
    assert abs((c["cv_chi"] * rl) / (c["cv_chi"] * rv) - c["value"]) < c["tolerance"]
