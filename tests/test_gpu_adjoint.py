"""GPU discrete adjoint vs the oracle's adjoint (and through it, central
finite differences): J = time-averaged bottom-wall heat flux, gradient with
respect to T_b(x) and G_w.  FP64 storage: gradients within 1e-9 normwise of
the oracle's (the two differ only in rounding order); FP32 storage: the
error against the FP64 adjoint is reported and bounded (FP32 state
trajectories) within 1e-5."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1501_03857_amd import lbboil as L
from paper_1501_03857_amd import workloads as WL
from parity_utils import make_pair, normwise

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


SMALL = WL.PLAIN_128x64.resized(48, 24, heater=(10, 30), Gw_bottom=0.06, dT_over_Tc=0.08, seed=21)


def test_adjoint_fp64_matches_oracle_small():
    _say("adjoint small fp64")
    o, d, _ = make_pair(SMALL, Gw_top=-0.02)
    o.step(20)
    d.step(20)
    Jo, go, gwo = o.adjoint(30, K=7)
    before = d.fields()
    Jd, gd, gwd = d.adjoint(30, K=7)
    after = d.fields()
    assert abs(Jd - Jo) <= 1e-12 * abs(Jo)
    assert normwise(gd, go) <= 1e-9, normwise(gd, go)
    assert abs(gwd - gwo) <= 1e-9 * abs(gwo)
    for k in ("f", "T"):
        assert np.array_equal(before[k], after[k])  # state restored
    assert d.heat_flux()["n_samples"] == 20


def test_adjoint_checkpoint_interval_bitwise():
    _say("adjoint K")
    _, d, _ = make_pair(SMALL)
    ref = d.adjoint(24, K=24)
    for K in (1, 5):
        J, g, gw = d.adjoint(24, K=K)
        assert J == ref[0] and np.array_equal(g, ref[1]) and gw == ref[2]


@pytest.mark.slow
@pytest.mark.parametrize("precision,tol", [(L.FP64, 1e-6), (L.FP32, 1e-5)])
def test_adjoint_256x128_heater_gradient(precision, tol):
    """The adjoint workload: 256x128, heater i in [96, 160) at 0.10 T_c,
    G_w = 0.065, 400 steps, checkpoints every 50."""
    _say("adjoint 256x128", precision)
    w = WL.ADJOINT_256x128
    o, d, _ = make_pair(w, precision=precision)
    Jo, go, gwo = o.adjoint(w.steps, K=50)
    Jd, gd, gwd = d.adjoint(w.steps, K=50)
    lo, hi = w.heater_range
    err_T = normwise(gd[lo:hi], go[lo:hi])
    err_G = abs(gwd - gwo) / abs(gwo)
    print(f"[adjoint] precision={precision} J rel err {abs(Jd / Jo - 1):.3e}, dJ/dT_b normwise {err_T:.3e}, "
          f"dJ/dG_w rel {err_G:.3e}", flush=True)
    assert err_T <= tol and err_G <= tol


def test_autograd_function_matches_library_gradient():
    _say("autograd")
    from paper_1501_03857_amd.autograd import HeatFluxFn

    _, d, info = make_pair(SMALL)
    lo, hi = SMALL.heater_range
    idx = np.arange(lo, hi)
    Tb0 = d.bottom_temperature()
    T_heater = torch.tensor(Tb0[idx], dtype=torch.float64, requires_grad=True)
    Gw = torch.tensor(SMALL.Gw_bottom, dtype=torch.float64, requires_grad=True)
    J = HeatFluxFn.apply(T_heater, Gw, d, idx, 25, 6)
    (2.0 * J).backward()
    J2, g, gw = d.adjoint(25, K=6)
    assert float(J) == J2
    assert np.allclose(T_heater.grad.numpy(), 2.0 * g[idx], rtol=0, atol=0)
    assert float(Gw.grad) == 2.0 * gw


def test_adjoint_refused_by_device_budget_leaves_domain_usable():
    """A budget below what the adjoint workspace needs: ENOMEM, no partial
    allocation held, the domain's state untouched and the adjoint working
    again once the budget is lifted; all bytes given back on destruction."""
    _say("adjoint budget")
    import gc

    gc.collect()  # earlier tests' domains are released now, not midway
    gc.disable()
    try:
        _budget_case()
    finally:
        gc.enable()


def _budget_case():
    held0 = L.device_bytes_held()
    _, d, _ = make_pair(SMALL)
    d.step(5)
    held1 = L.device_bytes_held()
    assert held1 > held0
    before = d.fields()
    L.set_device_budget(held1 + 4096)
    try:
        with pytest.raises(L.LbbError) as e:
            d.adjoint(24, K=6)
        assert e.value.code == L.LBB_ENOMEM
        assert L.device_bytes_held() == held1
    finally:
        L.set_device_budget(0)
    after = d.fields()
    assert np.array_equal(before["f"], after["f"]) and np.array_equal(before["T"], after["T"])
    J, g, gw = d.adjoint(24, K=6)
    assert np.isfinite(J) and np.all(np.isfinite(g))
    assert L.device_bytes_held() > held1
    d.close()
    assert L.device_bytes_held() == held0


def test_adjoint_heater_index_selection():
    """dJ_dTb for a list of heater nodes (any order, repeats allowed) is the
    full bottom-wall gradient at those nodes, bit for bit, and J is the same;
    an index outside [0, nx) is EINVAL and leaves the domain usable."""
    _say("adjoint heater_idx")
    _, d, _ = make_pair(SMALL)
    J, g, gw = d.adjoint(20, K=5)
    idx = [7, 3, 3, SMALL.nx - 1, 0]
    Js, gs, gws = d.adjoint(20, K=5, heater_idx=idx)
    assert Js == J and gws == gw
    assert np.array_equal(gs, g[idx])
    with pytest.raises(L.LbbError) as e:
        d.adjoint(20, K=5, heater_idx=[SMALL.nx])
    assert e.value.code == L.LBB_EINVAL
    J2, g2, _ = d.adjoint(20, K=5)
    assert J2 == J and np.array_equal(g2, g)
