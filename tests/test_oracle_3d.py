"""Pins of the oracle's three-dimensional (D3Q19) extension of the model, the
extension the paper names as future work (Sec. 4).  Each pin is fixed by
something other than the oracle's own formulas:

* The moment basis is orthogonal (M M^T diagonal), and M f_eq and M F' of
  the Guo term equal the closed-form D3Q19 equilibrium and forcing moments
  of the literature (e_eq = -11 rho + 19 rho v^2, epsilon_eq = 3 rho -
  11/2 rho v^2, q_eq = -2/3 rho v, pi_eq = -p_eq/2, m_eq = 0; S_e = 38 v.F,
  S_epsilon = -11 v.F, S_q = -2/3 F, ...).
* The collision equals a dense M^-1 (m - L(m - m_eq) + (I - L/2) S) built
  here from those closed forms with numpy's inverse, and its sigma part is
  the mass- and momentum-free equal increment s sigma Q / 60 of every moving
  population that gives each diagonal stress component the same s sigma Q/6
  as the two-dimensional term of Eq. (8).
* Mass and momentum are conserved in a fully periodic box; a uniform state
  stays uniform; the Zou-He wall nodes carry no momentum.
* The thermal stencils are exact on quadratics; 1-D conduction across the
  walls follows the discrete closed form R(z)^n of the RK4 step.
* A flat liquid slab relaxes to the same coexistence densities as the
  two-dimensional model (the same pressure tensor to fourth order), close to
  the Maxwell construction (Sec. 3.1: 6.5 / 0.38).
* A static drop obeys Laplace's law with the sphere's 2 gamma / R against the
  cylinder's gamma / R of the two-dimensional model.
* The wall heat flux of a linear temperature profile is c_v chi rho dT/dy.
"""
import numpy as np
import pytest

import oracle as O
from oracle import ISOTHERMAL, THERMAL_ONLY, Params, State, State3

A3, B, R, OMEGA = 3.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def _coex(a=A3):
    tc = O.Tc(a, B, R)
    rv, rl, _ = O.maxwell(a, B, R, OMEGA, 0.86 * tc)
    return tc, rv, rl


def _closed_form_moments(rho, v, F):
    """D3Q19 equilibrium and Guo forcing moments in the standard basis."""
    vx, vy, vz = v
    v2 = float(np.dot(v, v))
    vF = float(np.dot(v, F))
    p_xx, p_ww = rho * (3 * vx * vx - v2), rho * (vy * vy - vz * vz)
    meq = np.array([rho, -11 * rho + 19 * rho * v2, 3 * rho - 5.5 * rho * v2,
                    rho * vx, -2 / 3 * rho * vx, rho * vy, -2 / 3 * rho * vy, rho * vz, -2 / 3 * rho * vz,
                    p_xx, -0.5 * p_xx, p_ww, -0.5 * p_ww, rho * vx * vy, rho * vy * vz, rho * vx * vz, 0, 0, 0])
    S_xx = 2 * (3 * vx * F[0] - vF)
    S_ww = 2 * (vy * F[1] - vz * F[2])
    S = np.array([0, 38 * vF, -11 * vF, F[0], -2 / 3 * F[0], F[1], -2 / 3 * F[1], F[2], -2 / 3 * F[2],
                  S_xx, -0.5 * S_xx, S_ww, -0.5 * S_ww, vx * F[1] + vy * F[0], vy * F[2] + vz * F[1],
                  vx * F[2] + vz * F[0], 0, 0, 0])
    return meq, S


def test_basis_orthogonal_and_closed_form_moments():
    e, W, M = O.lattice3()
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert list(np.diag(G)) == [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    assert abs(W.sum() - 1) < 1e-15 and np.allclose(np.einsum("a,ai,aj->ij", W, e, e), np.eye(3) / 3)
    rng = np.random.default_rng(4)
    for _ in range(5):
        rho, v, F = rng.uniform(0.3, 7), rng.normal(size=3) * 0.05, rng.normal(size=3) * 0.01
        feq = O.feq3(rho, v)
        meq, S = _closed_form_moments(rho, v, F)
        assert np.allclose(M @ feq, meq, rtol=0, atol=1e-14 * rho * 40)
        eu, eF = e @ v, e @ F
        Fp = W * (3 * (e @ F - v @ F) + 9 * eu * eF)
        assert np.allclose(M @ Fp, S, rtol=0, atol=1e-16 * 40)


def test_collision_matches_dense_inverse_and_sigma_increment():
    e, W, M = O.lattice3()
    tc, rv, rl = _coex()
    p = Params(a=A3, rho_L=rl, rho_V=rv, sigma=1.2, s_e=0.8, s_zeta=0.8, s_q=1.1)
    rng = np.random.default_rng(5)
    Minv = np.linalg.inv(M)
    for _ in range(6):
        rho = rng.uniform(0.4, 6.5)
        v, F, Q = rng.normal(size=3) * 0.03, rng.normal(size=3) * 0.01, rng.uniform(0, 1e-3)
        f = O.feq3(rho, v) * (1 + 0.05 * rng.normal(size=19))
        meq, S = _closed_form_moments(rho, v, F)
        tau_nu = (3 * p.nu_V + 0.5) + (rho - rv) * (3 * (p.nu_L - p.nu_V)) / (rl - rv)
        sn = 1 / tau_nu
        L = np.array([p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q, p.s_j, p.s_q, p.s_j, p.s_q, sn, p.s_zeta, sn,
                      p.s_zeta, sn, sn, sn, p.s_q, p.s_q, p.s_q])
        m = M @ f
        want0 = Minv @ (m - L * (m - meq) + (1 - L / 2) * S)
        got0 = O.collide_site3(Params(**{**p.__dict__, "sigma": 0.0}), f, rho, v, F, Q)
        assert np.max(np.abs(got0 - want0)) < 1e-14 * rho
        # the sigma part: with s_e = s_zeta = s, an equal increment s sigma Q / 60
        # of every moving population (and -18 times it on the rest population)
        got = O.collide_site3(p, f, rho, v, F, Q)
        k = p.s_e * p.sigma * Q / 60
        assert np.max(np.abs(got - got0 - np.r_[-18 * k, np.full(18, k)])) < 1e-14 * rho
        # which adds s sigma Q / 6 to each diagonal component of the second moment
        d = np.einsum("a,ai,aj->ij", got - got0, e, e)
        assert np.max(np.abs(d - np.eye(3) * p.s_e * p.sigma * Q / 6)) < 1e-13 * rho


def _momentum(f):
    e, _, _ = O.lattice3()
    return np.array([np.einsum("a,azyx->", e[:, d].astype(float), f) for d in range(3)])


def test_periodic_box_conserves_mass_and_momentum():
    tc, rv, rl = _coex()
    p = Params(nx=12, ny=14, a=A3, rho_L=rl, rho_V=rv, periodic_y=1, g=3e-5)
    rng = np.random.default_rng(3)
    nz = 10
    y = np.arange(p.ny)[None, :, None]
    rho0 = rv + (rl - rv) * (np.abs(y - 7) < 3.5) + 0.05 * (rng.random((nz, p.ny, p.nx)) - 0.5)
    z, yy, x = np.mgrid[0:nz, 0:p.ny, 0:p.nx]
    T0 = 0.86 * tc * (1 + 0.02 * np.sin(2 * np.pi * x / p.nx) * np.cos(2 * np.pi * z / nz))
    s = State3(p, nz, rho0, T0=T0)
    f0 = s.fields()
    m0, j0 = f0["rho"].sum(), _momentum(f0["f"])
    s.step(150)
    f1 = s.fields()
    assert abs(f1["rho"].sum() / m0 - 1) < 1e-13
    assert np.max(np.abs(_momentum(f1["f"]) - j0)) < 1e-12 * m0
    assert np.max(np.abs(f1["rho"] - f0["rho"])) > 0.1  # the state moved


def test_uniform_state_stationary_and_wall_nodes_carry_no_momentum():
    tc, rv, rl = _coex()
    p = Params(nx=8, ny=9, a=A3, rho_L=rl, rho_V=rv, g=3e-5)
    s = State3(p, 6, np.full((6, 9, 8), 3.0))
    f0 = s.fields()
    s.step(30)
    f1 = s.fields()
    assert np.max(np.abs(f1["f"] - f0["f"])) < 1e-14 and np.max(np.abs(f1["T"] - f0["T"])) < 1e-17
    # a layered, noisy state with a hot wall and a wettable bottom: the Zou-He
    # rows have zero momentum in every direction after every step
    p = Params(nx=10, ny=12, a=A3, rho_L=rl, rho_V=rv, Gw_bottom=0.08, Gw_top=-0.03)
    rng = np.random.default_rng(6)
    y = np.arange(12)[None, :, None]
    rho0 = np.where(y < 6, rl, rv) + 1e-2 * rng.random((7, 12, 10))
    Tb = 0.86 * tc + 0.01 * rng.random((7, 10))
    s = State3(p, 7, rho0, T_bottom=Tb)
    e, _, _ = O.lattice3()
    for _ in range(3):
        s.step(20)
        f = s.fields()["f"]
        for row in (0, -1):
            j = np.einsum("ad,azx->dzx", e.astype(float), f[:, :, row, :])
            assert np.max(np.abs(j)) < 1e-14


def test_stencils_exact_on_quadratics():
    nz, ny, nx = 9, 10, 11
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    rng = np.random.default_rng(8)
    c = rng.normal(size=10)
    phi = (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * x + c[5] * y * y + c[6] * z * z + c[7] * x * y
           + c[8] * y * z + c[9] * x * z)
    dx, dy, dz, lap = O.grad_iso3(phi)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    want = [c[1] + 2 * c[4] * x + c[7] * y + c[9] * z, c[2] + 2 * c[5] * y + c[7] * x + c[8] * z,
            c[3] + 2 * c[6] * z + c[8] * y + c[9] * x]
    for got, w in zip((dx, dy, dz), want):
        assert np.max(np.abs(got[inner] - w[inner])) < 1e-11
    assert np.max(np.abs(lap[inner] - 2 * (c[4] + c[5] + c[6]))) < 1e-11
    assert np.all(dy[:, 0] == 0) and np.all(lap[:, -1] == 0)  # wall rows carry no stencil


def test_conduction_across_the_walls_follows_the_rk4_closed_form():
    """THERMAL_ONLY with v = 0 and a temperature that depends on y only: the
    3-D stencils reduce to the 3-point Laplacian along y, so each sine mode of
    the deviation from the linear profile is multiplied by R(z) = 1 + z +
    z^2/2 + z^3/6 + z^4/24, z = -4 chi sin^2(k pi / 2H), every step."""
    tc, rv, rl = _coex()
    ny, nx, nz = 17, 4, 3
    H = ny - 1
    p = Params(nx=nx, ny=ny, a=A3, rho_L=rl, rho_V=rv, thermal_mode=THERMAL_ONLY, cv_chi=0.15)
    chi = p.cv_chi / p.cv
    Ts, dT = 0.86 * tc, 0.01
    j = np.arange(ny)
    base = Ts + dT * (1 - j / H)
    b = {1: 0.004, 3: -0.002}
    T0 = base + sum(bk * np.sin(k * np.pi * j / H) for k, bk in b.items())
    T3 = np.broadcast_to(T0[None, :, None], (nz, ny, nx)).copy()
    s = State3(p, nz, np.full((nz, ny, nx), 2.0), T0=T3, T_bottom=np.full((nz, nx), Ts + dT))
    n = 40
    s.step(n)
    Rz = lambda zz: 1 + zz + zz ** 2 / 2 + zz ** 3 / 6 + zz ** 4 / 24
    want = base + sum(bk * Rz(-4 * chi * np.sin(k * np.pi / (2 * H)) ** 2) ** n * np.sin(k * np.pi * j / H)
                      for k, bk in b.items())
    got = s.fields()["T"]
    assert np.max(np.abs(got - want[None, :, None])) < 1e-13


def test_linear_profile_heat_flux():
    tc, rv, rl = _coex()
    ny, nx, nz = 12, 5, 4
    p = Params(nx=nx, ny=ny, a=A3, rho_L=rl, rho_V=rv, thermal_mode=THERMAL_ONLY)
    Ts, dT = 0.86 * tc, 0.02
    T0 = Ts + dT * (1 - np.arange(ny) / (ny - 1))
    s = State3(p, nz, np.full((nz, ny, nx), 4.0), T0=np.broadcast_to(T0[None, :, None], (nz, ny, nx)).copy(),
               T_bottom=np.full((nz, nx), Ts + dT))
    q = s.heat_flux()
    assert abs(q["q_now"] / (p.cv_chi * 4.0 * dT / (ny - 1)) - 1) < 1e-12
    assert np.allclose(q["q_local"], q["q_now"], rtol=1e-12)


def test_flat_slab_coexistence_matches_two_dimensions_and_maxwell():
    """Sec. 3.1 (rho_L ~ 6.5, rho_V ~ 0.38 at T_s = 0.86 T_c, a = 3/49,
    sigma = 1.2): a flat slab in a periodic box relaxes to the densities the
    two-dimensional model gives, and close to the Maxwell construction."""
    tc, rv, rl = _coex()
    ny = 64
    p = Params(nx=4, ny=ny, a=A3, rho_L=rl, rho_V=rv, periodic_y=1, g=0.0, thermal_mode=ISOTHERMAL)
    y = np.arange(ny)
    prof = rv + (rl - rv) * 0.5 * (np.tanh((y - 16) / 2) - np.tanh((y - 48) / 2))
    s2 = State(p, np.tile(prof[:, None], (1, 4))).step(4000)
    s3 = State3(p, 4, np.tile(prof[None, :, None], (4, 1, 4))).step(4000)
    r2, r3 = s2.fields()["rho"][:, 0], s3.fields()["rho"][0, :, 0]
    assert abs(r3[32] / r2[32] - 1) < 1e-4 and abs(r3[0] / r2[0] - 1) < 2e-3
    assert abs(r3[32] / rl - 1) < 2e-3 and abs(r3[0] / rv - 1) < 3e-2


@pytest.mark.slow
def test_static_drop_obeys_laplace_with_twice_the_cylinder_pressure():
    """A static drop (isothermal, no gravity): the pressure jump of a sphere,
    2 gamma / R, against gamma / R of a cylinder of the same model in two
    dimensions (Laplace's law, which the paper invokes in Sec. 3.2).  The
    finite interface width shifts both by a few per cent at R ~ 8."""
    tc, rv, rl = _coex()
    Ts, kap = 0.86 * tc, O.kappa(OMEGA)

    def pe(r):
        return O.p_eos(r, Ts, A3, B, R, tc, kap)

    n3 = 24
    p3 = Params(nx=n3, ny=n3, a=A3, rho_L=rl, rho_V=rv, periodic_y=1, g=0.0, thermal_mode=ISOTHERMAL)
    z, y, x = np.mgrid[0:n3, 0:n3, 0:n3] - (n3 - 1) / 2
    s3 = State3(p3, n3, rv + (rl - rv) * 0.5 * (1 - np.tanh((np.sqrt(x * x + y * y + z * z) - 8.0) / 1.5)))
    r = s3.step(1500).fields()["rho"]
    c = n3 // 2
    rin, rout = r[c, c, c], r[0, 0, 0]
    R3 = (3 * np.sum((r - rout) / (rin - rout)) / (4 * np.pi)) ** (1 / 3)
    k3 = (pe(rin) - pe(rout)) * R3
    n2 = 48
    p2 = Params(nx=n2, ny=n2, a=A3, rho_L=rl, rho_V=rv, periodic_y=1, g=0.0, thermal_mode=ISOTHERMAL)
    y, x = np.mgrid[0:n2, 0:n2] - (n2 - 1) / 2
    s2 = State(p2, rv + (rl - rv) * 0.5 * (1 - np.tanh((np.sqrt(x * x + y * y) - 8.0) / 1.5)))
    r = s2.step(3000).fields()["rho"]
    c = n2 // 2
    rin, rout = r[c, c], r[0, 0]
    R2 = np.sqrt(np.sum((r - rout) / (rin - rout)) / np.pi)
    k2 = (pe(rin) - pe(rout)) * R2
    assert 6.5 < R3 < 9.5 and k2 > 0
    assert 1.7 < k3 / k2 < 2.2, (k3, k2)
