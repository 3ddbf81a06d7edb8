"""Batched adjoint: the adjoint of every batch member in shared launches must
equal each member's adjoint alone bitwise (and so, through the single-lattice
adjoint tests, the oracle's), leave every member's state unchanged and the
batch in phase."""
import numpy as np
import pytest

import oracle as O
from paper_1501_03857_amd import lbboil as L
from paper_1501_03857_amd import workloads as WL
from parity_utils import make_pair, normwise

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _members(precision):
    base = WL.PLAIN_128x64
    specs = [
        base.resized(100, 37, heater=(10, 60), Gw_bottom=0.065, seed=5),
        base.resized(130, 17, dT_over_Tc=0.10, heater=(0, -1), Gw_bottom=0.154, seed=6),
        base.resized(70, 40, dT_over_Tc=0.2, heater=(3, 40), Gw_bottom=-0.04, seed=7),
        base.resized(62, 8, heater=(0, 31), seed=8),
    ]
    out = []
    for w in specs:
        tc = O.Tc(w.a, w.b, w.R)
        rv, rl, _ = O.maxwell(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * tc)
        p = L.Params(nx=w.nx, ny=w.ny, precision=precision, liquid_rows=w.liquid_rows, sigma=w.sigma, g=w.g,
                     Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv)
        out.append((p, w.heater_T(tc), w.density(rl, rv)))
    return out


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_batch_adjoint_equals_member_adjoints_bitwise(precision):
    _say("batch adjoint vs single", precision)
    mem = _members(precision)
    b = L.Batch([m[0] for m in mem], [m[1] for m in mem], [m[2] for m in mem])
    b.step(9)
    before = [b.domain(i).fields() for i in range(len(mem))]
    J, g, gw = b.adjoint(23, K=6)  # four segments, the last one ragged
    for i, (p, Tb, rho0) in enumerate(mem):
        d = L.Domain(p, T_bottom=Tb, rho0=rho0).step(9)
        Js, gs, gws = d.adjoint(23, K=6)
        assert J[i] == Js and np.array_equal(g[i], gs) and gw[i] == gws, i
        after = b.domain(i).fields()
        for k in ("f", "T"):
            assert np.array_equal(before[i][k], after[k]), (i, k)
    # still in phase: the batch steps on, members as when stepped alone
    b.step(5)
    for i, (p, Tb, rho0) in enumerate(mem):
        d = L.Domain(p, T_bottom=Tb, rho0=rho0).step(14)
        assert np.array_equal(b.domain(i).fields()["f"], d.fields()["f"]), i


def test_batch_adjoint_member_matches_oracle():
    _say("batch adjoint member vs oracle")
    w = WL.PLAIN_128x64.resized(100, 37, heater=(10, 60), Gw_bottom=0.065, seed=5)
    o, _, _ = make_pair(w)
    mem = _members(L.FP64)
    b = L.Batch([m[0] for m in mem], [m[1] for m in mem], [m[2] for m in mem])
    J, g, gw = b.adjoint(20, K=7)
    Jo, go, gwo = o.adjoint(20, K=7)
    assert abs(J[0] / Jo - 1) < 1e-9
    assert normwise(g[0], go) < 1e-9
    assert abs(gw[0] / gwo - 1) < 1e-9


def test_adjoint_automatic_checkpoint_interval():
    """K <= 0 lets the library choose (every state kept for a lattice this
    small); the result does not depend on K."""
    _say("adjoint automatic K")
    _, d, _ = make_pair(WL.PLAIN_128x64.resized(80, 30, heater=(20, 50), seed=9))
    a = d.adjoint(17, K=0)
    for K in (17, 4):
        r = d.adjoint(17, K=K)
        assert a[0] == r[0] and np.array_equal(a[1], r[1]) and a[2] == r[2], K


def test_temperature_adjoint_tile_height_does_not_change_the_gradient():
    """16 lattices of 400x200 give the batch enough temperature-adjoint tiles
    for 24-row tiles, while one lattice alone uses 8-row tiles: the gradients
    must be bitwise equal (the per-node arithmetic of the transposed RK4 step
    does not depend on the tiling)."""
    _say("batch adjoint 16 x 400x200: 24-row vs 8-row temperature-adjoint tiles")
    base = WL.PLAIN_128x64
    mem = []
    for i in range(16):
        w = base.resized(400, 200, dT_over_Tc=0.04 + 0.01 * i, heater=(0, -1), Gw_bottom=0.065, seed=30 + i,
                         g=WL.scaled_gravity(200, 2.0 / 49.0))
        tc = O.Tc(w.a, w.b, w.R)
        rv, rl, _ = O.maxwell(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * tc)
        p = L.Params(nx=w.nx, ny=w.ny, precision=L.FP32, liquid_rows=w.liquid_rows, sigma=w.sigma, g=w.g,
                     Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv)
        mem.append((p, w.heater_T(tc), w.density(rl, rv)))
    b = L.Batch([m[0] for m in mem], [m[1] for m in mem], [m[2] for m in mem])
    b.step(5)
    J, g, gw = b.adjoint(8, K=4)  # two segments: the recompute stream and both buffers
    b.close()
    for i in (0, 9):
        p, Tb, rho0 = mem[i]
        d = L.Domain(p, T_bottom=Tb, rho0=rho0).step(5)
        Js, gs, gws = d.adjoint(8, K=4)
        assert J[i] == Js and np.array_equal(g[i], gs) and gw[i] == gws, i
        d.close()
