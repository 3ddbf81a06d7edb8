"""Pins of the oracle's lattice pieces: moment basis, equilibrium, forcing,
single-site MRT collision, interaction force and stencils.

Each check compares the oracle with an independent object: the moments the
paper prints (Eq. (5), Eq. (8)), Guo's velocity-space forcing term, a dense
numpy inverse of M, or exactness of the discrete operators on polynomials.
"""
import numpy as np
import pytest

import oracle as O
from paper_1501_03857_amd import workloads as WL

EX, EY, W, WPSI, M = O.lattice()
E = np.stack([EX, EY], axis=1).astype(float)


def test_moment_basis_orthogonal():
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=0)
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4], atol=0)
    # the rows are the standard D2Q9 moments of the velocity set
    ex, ey = EX.astype(float), EY.astype(float)
    e2 = ex ** 2 + ey ** 2
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[1], -4 + 3 * e2)
    assert np.array_equal(M[3], ex) and np.array_equal(M[5], ey)
    assert np.array_equal(M[7], ex ** 2 - ey ** 2) and np.array_equal(M[8], ex * ey)


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0, 0), (6.5, 0.03, -0.02), (0.38, -0.1, 0.07)])
def test_equilibrium_moments_eq5(rho, ux, uy):
    """M f_eq reproduces the equilibrium moments printed in Eq. (5)."""
    feq = O.feq(rho, ux, uy)
    v2 = ux * ux + uy * uy
    eq5 = rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, ux, -ux, uy, -uy, ux * ux - uy * uy, ux * uy])
    assert np.allclose(M @ feq, eq5, rtol=0, atol=1e-14 * rho)
    # hydrodynamic moments of the discrete equilibrium
    assert feq.sum() == pytest.approx(rho, rel=1e-15)
    assert E.T @ feq == pytest.approx(rho * np.array([ux, uy]), abs=1e-15 * rho)
    Pi = np.einsum("a,ai,aj->ij", feq, E, E)
    assert np.allclose(Pi, rho * (np.eye(2) / 3 + np.outer([ux, uy], [ux, uy])), atol=1e-14 * rho)


def _guo(vx, vy, Fx, Fy):
    """Guo et al.'s velocity-space forcing W_a [3 (e - v).F + 9 (e.v)(e.F)]."""
    out = np.zeros(9)
    for a in range(9):
        ev = E[a, 0] * vx + E[a, 1] * vy
        eF = E[a, 0] * Fx + E[a, 1] * Fy
        out[a] = W[a] * (3 * ((E[a, 0] - vx) * Fx + (E[a, 1] - vy) * Fy) + 9 * ev * eF)
    return out


@pytest.mark.parametrize("seed", range(5))
def test_forcing_term_is_guo_projection(seed):
    """At sigma = 0, S of Eq. (8) is the moment projection of Guo's forcing term."""
    r = np.random.default_rng(seed)
    vx, vy, Fx, Fy = r.uniform(-0.1, 0.1, 4)
    p = O.Params(sigma=0.0)
    S = O.forcing_moments(p, vx, vy, Fx, Fy, 0.37)
    assert np.allclose(M @ _guo(vx, vy, Fx, Fy), S, rtol=0, atol=1e-16)


def test_sigma_term_shifts_e_equilibrium():
    """The sigma term of Eq. (8) acts on e and zeta only.  Since
    (1 - s_e/2)/(tau_e - 1/2) = s_e, it is the same as relaxing e towards
    e_eq + sigma Q (and zeta towards zeta_eq - sigma Q): the post-collision
    moments move by s_e sigma Q and -s_zeta sigma Q, every other moment (and
    so mass and momentum) is untouched."""
    r = np.random.default_rng(7)
    f = O.feq(2.0, 0.02, -0.01) + r.uniform(-1e-3, 1e-3, 9)
    p0 = O.Params(sigma=0.0, s_e=0.8, s_zeta=1.3)
    p1 = O.Params(sigma=1.2, s_e=0.8, s_zeta=1.3)
    args = (f.sum(), 0.01, -0.02, 1e-3, -2e-3, 0.05)
    d = M @ (O.collide_site(p1, f, *args) - O.collide_site(p0, f, *args))
    expect = np.zeros(9)
    expect[1] = 0.8 * 1.2 * 0.05
    expect[2] = -1.3 * 1.2 * 0.05
    assert np.allclose(d, expect, atol=1e-15)


@pytest.mark.parametrize("seed", range(8))
def test_collide_site_dense_bruteforce(seed):
    """Oracle collision against Eq. (1) in velocity space with a dense
    numpy inverse of M: f* = f - M^-1 L M (f - f_eq) + M^-1 (I - L/2) S."""
    r = np.random.default_rng(100 + seed)
    rho = r.uniform(0.3, 7.0)
    u = r.uniform(-0.05, 0.05, 2)
    f = O.feq(rho, *u) * (1 + r.uniform(-0.05, 0.05, 9))
    Fx, Fy, Q = r.uniform(-0.02, 0.02), r.uniform(-0.02, 0.02), r.uniform(0, 0.01)
    p = O.Params(sigma=r.uniform(0, 1.5), s_e=r.uniform(0.6, 1.4), s_zeta=r.uniform(0.6, 1.4),
                 s_q=r.uniform(0.8, 1.6), s_j=r.uniform(0.8, 1.4), s_rho=r.uniform(0.8, 1.2))
    dens = f.sum()
    j = E.T @ f
    vx, vy = (j + 0.5 * np.array([Fx, Fy])) / dens
    tau_L, tau_V = 3 * p.nu_L + 0.5, 3 * p.nu_V + 0.5
    tau_nu = tau_V + (dens - p.rho_V) * (tau_L - tau_V) / (p.rho_L - p.rho_V)
    Lam = np.diag([p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q, p.s_j, p.s_q, 1 / tau_nu, 1 / tau_nu])
    Minv = np.linalg.inv(M)
    S = M @ _guo(vx, vy, Fx, Fy)
    S[1] += p.sigma * Q / (1 / p.s_e - 0.5)
    S[2] -= p.sigma * Q / (1 / p.s_zeta - 0.5)
    fs = f - Minv @ Lam @ M @ (f - O.feq(dens, vx, vy)) + Minv @ (np.eye(9) - 0.5 * Lam) @ S
    got = O.collide_site(p, f, dens, vx, vy, Fx, Fy, Q)
    assert np.max(np.abs(got - fs)) <= 1e-14 * np.max(np.abs(fs))
    # mass conserved, momentum gains exactly F (j* = j + F)
    assert got.sum() == pytest.approx(f.sum(), rel=1e-14)
    assert np.allclose(E.T @ got, j + np.array([Fx, Fy]), atol=1e-14 * dens)


def _poly_field(nx, ny, c):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y, x, y


@pytest.mark.parametrize("wall", ["bottom", "top"])
@pytest.mark.parametrize("cx,cxx,cyy", [(0.01, 0.0, 0.02), (-0.02, 1e-3, -0.01), (0.0, -2e-3, 0.03)])
def test_ghost_layer_force_on_mirror_quadratic(wall, cx, cxx, cyy):
    """Ghost-layer variant (Sec. 3.2): a ghost row that mirrors the first
    fluid row about the wall row continues any field that is even about the
    wall row.  For psi = c0 + cx x + cxx x^2 + cyy (y - y_w)^2 the stencil
    sum on the wall row y_w is therefore exactly grad psi = (cx + 2 cxx x, 0),
    so F_m = -G psi grad psi (no normal part) and Q = G^2 |grad psi|^2 there;
    without the ghost layer both are zero."""
    nx, ny = 10, 8
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    j = 0 if wall == "bottom" else ny - 1
    psi = 3.0 + cx * x + cxx * x * x + cyy * (y - j) ** 2
    p = O.Params(nx=nx, ny=ny, G=-1.0, ghost_layer=1)
    Fx, Fy, Q = O.interaction_force(p, psi)
    gx = cx + 2 * cxx * x[j]
    cols = slice(1, -1)  # x wraps, which a polynomial does not
    assert np.allclose(Fx[j, cols], (-p.G * psi[j] * gx)[cols], atol=1e-13)
    assert np.allclose(Fy[j, cols], 0.0, atol=1e-13)
    assert np.allclose(Q[j, cols], (p.G ** 2 * gx ** 2)[cols], atol=1e-13)
    F0 = O.interaction_force(O.Params(nx=nx, ny=ny, G=-1.0), psi)
    assert all(np.all(a[[0, -1]] == 0) for a in F0)
    # off the wall rows the two variants agree exactly
    for a, b in zip((Fx, Fy, Q), F0):
        assert np.array_equal(a[1:-1], b[1:-1])


def test_ghost_layer_force_matches_padded_lattice():
    """On a random positive psi the ghost-layer force on every row equals the
    plain stencil evaluated on psi padded by one ghost row on each side (the
    mirror images of rows 1 and ny-2) and wrapped in x; on the wall rows its
    normal component is zero to rounding for any psi."""
    rng = np.random.default_rng(7)
    nx, ny = 9, 7
    psi = 1.0 + rng.random((ny, nx))
    pad = np.pad(psi, ((1, 1), (0, 0)), mode="reflect")
    pad = np.pad(pad, ((0, 0), (1, 1)), mode="wrap")
    sx = np.zeros_like(psi)
    sy = np.zeros_like(psi)
    for a in range(1, 9):
        nb = pad[1 + EY[a]:1 + EY[a] + ny, 1 + EX[a]:1 + EX[a] + nx]
        sx += WPSI[a] * EX[a] * nb
        sy += WPSI[a] * EY[a] * nb
    G = -1.0
    Fx, Fy, Q = O.interaction_force(O.Params(nx=nx, ny=ny, G=G, ghost_layer=1), psi)
    assert np.allclose(Fx, -G * psi * sx, rtol=0, atol=1e-14)
    assert np.allclose(Fy, -G * psi * sy, rtol=0, atol=1e-14)
    assert np.allclose(Q, G * G * (sx * sx + sy * sy), rtol=0, atol=1e-14)
    assert np.max(np.abs(Fy[[0, -1]])) < 1e-14


@pytest.mark.parametrize("k", range(6))
def test_isotropic_stencils_exact_on_quadratics(k):
    c = np.zeros(6)
    c[k] = 1.0
    c[0] += 2.0
    phi, x, y = _poly_field(12, 9, c)
    dx, dy, lap = O.grad_iso(phi)
    ex = c[1] + 2 * c[3] * x + c[4] * y
    ey = c[2] + c[4] * x + 2 * c[5] * y
    el = 2 * c[3] + 2 * c[5]
    sl = (slice(1, -1), slice(1, -1))  # interior rows, away from the x-wrap
    assert np.allclose(dx[sl], ex[sl], atol=1e-12)
    assert np.allclose(dy[sl], ey[sl], atol=1e-12)
    assert np.allclose(lap[sl], el, atol=1e-12)


def test_stencils_reduce_to_three_point_in_1d():
    r = np.random.default_rng(3)
    row = r.uniform(size=16)
    phi = np.tile(row, (6, 1))
    dx, dy, lap = O.grad_iso(phi, periodic_y=1)
    assert np.allclose(dx, (np.roll(phi, -1, 1) - np.roll(phi, 1, 1)) / 2, atol=1e-15)
    assert np.allclose(lap, np.roll(phi, -1, 1) + np.roll(phi, 1, 1) - 2 * phi, atol=1e-14)
    assert np.allclose(dy, 0, atol=1e-15)


@pytest.mark.parametrize("k", range(6))
def test_interaction_force_on_quadratic_psi(k):
    """sum_a w_a psi(x+e_a) e_a = grad psi exactly for quadratic psi (the
    weights satisfy sum w e e = I), so F_m = -G psi grad psi and
    Q = G^2 |grad psi|^2 on the interior rows; zero on the wall rows."""
    c = np.array([3.0, 0.01, -0.02, 1e-3, 2e-3, -1e-3])
    c[k] *= 2
    psi, x, y = _poly_field(10, 8, c)
    p = O.Params(nx=10, ny=8, G=-1.0)
    Fx, Fy, Q = O.interaction_force(p, psi)
    gx = c[1] + 2 * c[3] * x + c[4] * y
    gy = c[2] + c[4] * x + 2 * c[5] * y
    sl = (slice(1, -1), slice(1, -1))
    assert np.allclose(Fx[sl], (-p.G * psi * gx)[sl], atol=1e-13)
    assert np.allclose(Fy[sl], (-p.G * psi * gy)[sl], atol=1e-13)
    assert np.allclose(Q[sl], (p.G ** 2 * (gx ** 2 + gy ** 2))[sl], atol=1e-13)
    assert np.all(Fx[[0, -1]] == 0) and np.all(Fy[[0, -1]] == 0) and np.all(Q[[0, -1]] == 0)
    # Q equals |F_m|^2 / psi^2 wherever F_m is applied
    assert np.allclose(Q[sl], ((Fx ** 2 + Fy ** 2) / psi ** 2)[sl], rtol=1e-12)


@pytest.mark.parametrize("bits", [24, 52, 40])
def test_storage_rounding_model(bits):
    """The rounding model behind the parity bars of v and q: after a step of a
    fully periodic box (every population streamed, none completed by a wall
    rule) each stored population has at most `bits` significant bits (24:
    exactly a float), and so has T when the model also rounds psi and T
    (bits != 24).  The state stays within a small multiple of that rounding
    of the unrounded one: a population rounding alone (24) moves f by at
    most half a unit in the last kept place; rounding psi as well moves F,
    and f through it, by a few tens of those units."""
    tc = O.Tc(2.0 / 49.0, 2.0 / 21.0, 1.0)
    rv, rl, _ = O.maxwell(2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344, 0.86 * tc)
    p = O.Params(nx=20, ny=12, rho_L=rl, rho_V=rv, periodic_y=1)
    rho0 = WL.layered_density(p.nx, p.ny, rl, rv, 6, 1e-2, seed=3)
    y, x = np.mgrid[0:p.ny, 0:p.nx]
    T0 = 0.86 * tc * (1 + 0.01 * np.sin(2 * np.pi * x / p.nx))
    a = O.State(p, rho0, T0=T0).step(1).fields()
    bf = O.State(p, rho0, T0=T0).store_bits(bits).step(1).fields()
    b = bf["f"]

    def kept(v, n):
        m, _ = np.frexp(v)
        scaled = np.ldexp(m, n)
        return np.array_equal(scaled, np.round(scaled))

    assert kept(b, bits)
    if bits == 24:
        assert np.array_equal(b, b.astype(np.float32).astype(np.float64))
        assert np.max(np.abs(b - a["f"]) / np.abs(a["f"])) <= 2.0 ** -bits * 1.0001
        assert np.array_equal(bf["T"], a["T"])
    else:
        assert kept(bf["T"], bits)
        assert np.max(np.abs(b - a["f"]) / np.abs(a["f"])) <= 2.0 ** -(bits - 6)
    assert np.max(np.abs(b - a["f"])) > 0
    with pytest.raises(O.OracleError):
        O.State(p, rho0).store_bits(53)
