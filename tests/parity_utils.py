"""Shared set-up for GPU-vs-oracle parity tests: the same seeded inputs and
parameters go to the CPU oracle and to the HIP library.

Error measures (all against the oracle b):
  fields rho, T, f : normwise relative, max |a - b| / max |b|;
  velocity         : Eq. (6) makes v the small difference of sum_a e_a f_a
                     and -F/2 (they nearly cancel near mechanical
                     equilibrium), so its error is measured against the size
                     of those terms, max(|v| + |sum_a e_a f_a| / rho);
  heat flux q      : q_w = -c_v chi rho (-3 T_0 + 4 T_1 - T_2)/2 is a small
                     difference of temperatures, so its error is measured
                     against c_v chi max(rho_0) (3|T_0| + 4|T_1| + |T_2|)/2.
"""
import numpy as np

import oracle as O
from paper_1501_03857_amd import lbboil as L
from paper_1501_03857_amd import workloads as WL

FIELDS = ("rho", "ux", "uy", "T", "f")
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def normwise(a, b, scale=None):
    """max |a - b| / scale, scale = max |b| by default."""
    den = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def velocity_scale(fields):
    f, rho = fields["f"], fields["rho"]
    jx = np.einsum("a,ajk->jk", EX, f)
    jy = np.einsum("a,ajk->jk", EY, f)
    jn = np.hypot(jx, jy) / rho
    return float(np.max(np.hypot(fields["ux"], fields["uy"]) + jn))


def heat_flux_scale(o):
    fl = o.fields()
    T = fl["T"]
    return float(o.p.cv_chi * np.max(fl["rho"][0]) * np.max(3 * np.abs(T[0]) + 4 * np.abs(T[1]) + np.abs(T[2])) / 2)


def make_pair(w: WL.Workload, *, precision=None, mode=O.COUPLED, periodic_y=0, Gw_top=0.0, g=None,
              rho0=None, T0=None, ux0=None, uy0=None, **extra):
    """Oracle state and GPU domain of workload w with identical inputs;
    extra: further model parameters (relaxation rates, viscosities, c_v ...)
    given to both sides."""
    tc = O.Tc(w.a, w.b, w.R)
    rv, rl, _ = O.maxwell(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * tc)
    if rho0 is None:
        rho0 = w.density(rl, rv)
    Tb = w.heater_T(tc)
    g = w.g if g is None else g
    common = dict(nx=w.nx, ny=w.ny, a=w.a, b=w.b, R=w.R, omega=w.omega, Ts_over_Tc=w.Ts_over_Tc,
                  sigma=w.sigma, g=g, Gw_bottom=w.Gw_bottom, Gw_top=Gw_top, rho_L=rl, rho_V=rv,
                  periodic_y=periodic_y, thermal_mode=mode, **extra)
    o = O.State(O.Params(**common), rho0, ux0=ux0, uy0=uy0, T0=T0, T_bottom=Tb)
    prec = {"fp64": L.FP64, "fp32": L.FP32}[w.precision] if precision is None else precision
    d = L.Domain(L.Params(precision=prec, liquid_rows=w.liquid_rows, **common), T_bottom=Tb, rho0=rho0)
    if T0 is not None or ux0 is not None or uy0 is not None:
        d.set_fields(rho0, ux0, uy0, T0)
    return o, d, dict(Tc=tc, rho_L=rl, rho_V=rv, Tb=Tb)


def compare(o, d, tol, fields=FIELDS):
    a, b = d.fields(), o.fields()
    vs = velocity_scale(b)
    errs = {k: normwise(a[k], b[k], vs if k in ("ux", "uy") else None) for k in fields}
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
