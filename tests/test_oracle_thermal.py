"""Pins of the oracle's temperature solver (Eqs. (18)-(20)) and heat flux.

* K(T) on polynomial fields equals the continuum right-hand side of Eq. (18)
  (the stencils are exact on quadratics), with (dp/dT)_rho taken by numerical
  differentiation of the EOS.
* Whole RK4 steps in test modes match discrete closed forms: 1-D conduction
  between Dirichlet walls, periodic advection-diffusion of a Fourier mode
  (both evolve each mode by the RK4 stability polynomial R(z)), and the
  pressure-work term on a uniform temperature in a uniformly diverging flow.
* The wall heat flux is exact on linear and quadratic profiles.
"""
import numpy as np
import pytest

import oracle as O
from oracle import Params, State, THERMAL_ONLY


def R4(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def _dpdT_num(rho, T, p: Params):
    tc, k = O.Tc(p.a, p.b, p.R), O.kappa(p.omega)
    h = 1e-4 * T
    f = lambda t: O.p_eos(rho, t, p.a, p.b, p.R, tc, k)
    return (-f(T + 2 * h) + 8 * f(T + h) - 8 * f(T - h) + f(T - 2 * h)) / (12 * h)


def test_thermal_rhs_on_polynomials():
    """K = -v.grad T + chi (lap T + grad rho.grad T/rho) - T/(rho c_v) (dp/dT) div v."""
    p = Params(nx=14, ny=11)
    y, x = np.mgrid[0:p.ny, 0:p.nx].astype(float)
    tc = O.Tc(p.a, p.b, p.R)
    T = 0.86 * tc * (1 + 1e-3 * x - 2e-3 * y + 3e-5 * x * x - 1e-5 * x * y + 2e-5 * y * y)
    rho = 3.0 + 0.05 * x + 0.08 * y
    vx = 0.01 + 1e-3 * x - 2e-3 * y
    vy = -0.02 + 3e-3 * x + 1.5e-3 * y
    K = O.thermal_rhs(p, rho, vx, vy, T)
    s = 0.86 * tc
    Tx = s * (1e-3 + 6e-5 * x - 1e-5 * y)
    Ty = s * (-2e-3 - 1e-5 * x + 4e-5 * y)
    lapT = s * (6e-5 + 4e-5)
    div = 1e-3 + 1.5e-3
    chi = p.cv_chi / p.cv
    dpdT = np.vectorize(lambda r, t: _dpdT_num(r, t, p))(rho, T)
    expect = -(vx * Tx + vy * Ty) + chi * (lapT + (0.05 * Tx + 0.08 * Ty) / rho) - T / (rho * p.cv) * dpdT * div
    sl = (slice(1, -1), slice(1, -1))
    scale = np.max(np.abs(expect[sl]))
    assert np.max(np.abs(K[sl] - expect[sl])) < 1e-9 * scale
    assert np.all(K[[0, -1]] == 0)




@pytest.mark.parametrize("cv_chi", [0.028, 0.2])
def test_conduction_1d_closed_form(cv_chi):
    """THERMAL_ONLY, v = 0, uniform rho, x-uniform T between Dirichlet walls.
    The deviation from the linear steady profile decays mode by mode as
    R(chi * lambda_k)^n with lambda_k = -4 sin^2(k pi / 2H)."""
    p = Params(nx=5, ny=17, cv_chi=cv_chi, thermal_mode=THERMAL_ONLY)
    H = p.ny - 1
    tc = O.Tc(p.a, p.b, p.R)
    Ts, Tb = 0.86 * tc, 0.93 * tc
    rho = np.full((p.ny, p.nx), 2.0)
    r = np.random.default_rng(0)
    prof = Ts + 0.01 * tc * r.uniform(-1, 1, p.ny)
    T0 = np.tile(prof[:, None], (1, p.nx))
    s = State(p, rho, T0=T0, T_bottom=np.full(p.nx, Tb))
    n = 37
    s.step(n)
    got = s.fields()["T"][:, 0]
    j = np.arange(p.ny)
    lin = Tb + (Ts - Tb) * j / H
    e0 = prof - lin
    e0[0] = e0[-1] = 0.0
    chi = p.cv_chi / p.cv
    en = np.zeros(p.ny)
    for k in range(1, H):
        mode = np.sin(k * np.pi * j / H)
        bk = 2.0 / H * np.sum(e0 * mode)
        en += bk * mode * R4(chi * -4 * np.sin(k * np.pi / (2 * H)) ** 2) ** n
    expect = lin + en
    assert np.max(np.abs(got - expect)) < 1e-13 * np.max(np.abs(expect))
    # x-uniform stays x-uniform
    assert np.max(np.abs(s.fields()["T"] - got[:, None])) < 1e-15


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("U,cv_chi", [(0.05, 0.028), (0.08, 0.0), (-0.03, 0.1)])
def test_advection_diffusion_fourier_mode(axis, U, cv_chi):
    """THERMAL_ONLY, periodic box, uniform rho and velocity U along one axis,
    T = T_s + A sin(k s): the discrete operator maps e^{iks} to
    z e^{iks} with z = -i U sin k - 4 chi sin^2(k/2), so
    T^n = T_s + A Im(R(z)^n e^{iks})."""
    p = Params(nx=24, ny=20, cv_chi=cv_chi, periodic_y=1, thermal_mode=THERMAL_ONLY)
    L = p.nx if axis == "x" else p.ny
    m = 3
    k = 2 * np.pi * m / L
    y, x = np.mgrid[0:p.ny, 0:p.nx].astype(float)
    sgrid = x if axis == "x" else y
    tc = O.Tc(p.a, p.b, p.R)
    Ts, A = 0.86 * tc, 1e-3 * tc
    T0 = Ts + A * np.sin(k * sgrid)
    rho = np.full((p.ny, p.nx), 1.7)
    ux = np.full_like(rho, U if axis == "x" else 0.0)
    uy = np.full_like(rho, U if axis == "y" else 0.0)
    s = State(p, rho, ux0=ux, uy0=uy, T0=T0)
    n = 25
    s.step(n)
    chi = p.cv_chi / p.cv
    z = -1j * U * np.sin(k) - 4 * chi * np.sin(k / 2) ** 2
    expect = Ts + A * np.imag(R4(z) ** n * np.exp(1j * k * sgrid))
    got = s.fields()["T"]
    assert np.max(np.abs(got - expect)) < 1e-13 * Ts


def test_pressure_work_uniform_expansion():
    """Uniform T and rho with v_y = alpha (y - y0): away from the walls (radius
    4 per step) T stays uniform and follows one RK4 step of the scalar ODE
    dT/dt = -T/(rho c_v) (dp/dT)_rho(rho, T) alpha."""
    p = Params(nx=6, ny=24, thermal_mode=THERMAL_ONLY)
    tc = O.Tc(p.a, p.b, p.R)
    rho0 = 3.0
    alpha = 2e-3
    y, x = np.mgrid[0:p.ny, 0:p.nx].astype(float)
    rho = np.full((p.ny, p.nx), rho0)
    uy = alpha * (y - p.ny / 2)
    T0 = np.full((p.ny, p.nx), 0.9 * tc)
    # velocity in THERMAL_ONLY mode is sum_a e_a f_a / rho
    s = State(p, rho, uy0=uy, T0=T0, T_bottom=np.full(p.nx, 0.9 * tc))
    s.step(1)
    g = lambda T: -T / (rho0 * p.cv) * _dpdT_num(rho0, T, p) * alpha
    Tn = 0.9 * tc
    h1 = g(Tn)
    h2 = g(Tn + h1 / 2)
    h3 = g(Tn + h2 / 2)
    h4 = g(Tn + h3)
    expect = Tn + (h1 + 2 * h2 + 2 * h3 + h4) / 6
    got = s.fields()["T"][6:-6]
    assert abs(expect - Tn) > 1e-6 * Tn  # the term is exercised
    assert np.max(np.abs(got - expect)) < 1e-12 * Tn


@pytest.mark.parametrize("quad", [0.0, 3e-6])
def test_heat_flux_exact_on_low_order_profiles(quad):
    """q_w = -lambda dT/dy|_0 with lambda = c_v chi rho: the one-sided
    second-order difference is exact on linear and quadratic profiles
    (Sec. 3.2).  The linear profile with v = 0 is also the steady state, so
    a step leaves it (and q) unchanged: q = c_v chi rho dT / (ny - 1)."""
    p = Params(nx=7, ny=12, thermal_mode=THERMAL_ONLY)
    tc = O.Tc(p.a, p.b, p.R)
    Ts, Tb = 0.86 * tc, 0.95 * tc
    H = p.ny - 1
    j = np.arange(p.ny, dtype=float)
    prof = Tb + (Ts - Tb) * j / H + quad * j * (j - H)
    rho = np.full((p.ny, p.nx), 4.2)
    s = State(p, rho, T0=np.tile(prof[:, None], (1, p.nx)), T_bottom=np.full(p.nx, Tb))
    hf = s.heat_flux()
    slope = (Ts - Tb) / H + quad * (-H)
    assert hf["q_now"] == pytest.approx(-p.cv_chi * 4.2 * slope, rel=1e-12)
    assert np.allclose(hf["q_local"], -p.cv_chi * 4.2 * slope, rtol=1e-12)
    if quad == 0.0:
        s.step(3)
        hf = s.heat_flux()
        assert hf["q_now"] == pytest.approx(p.cv_chi * 4.2 * (Tb - Ts) / H, rel=1e-12)
        assert hf["n_samples"] == 3
        assert hf["q_mean"] == pytest.approx(hf["q_now"], rel=1e-12)
