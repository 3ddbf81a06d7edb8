"""GPU (HIP, gfx950) vs CPU oracle parity of the three-dimensional (D3Q19)
time step, the extension of the model to three dimensions that the paper
names as its future work (Sec. 4).  Same measures and bars as the
two-dimensional parity tests: normwise max |gpu - oracle| / max |oracle| per
field and for the heat flux; rho, T, f at 1e-12 (FP64) or 1e-5 (FP32); v
and q against the oracle's rounding twin (State3.store_bits: 52 bits of f,
psi and T in FP64, FP32 populations in FP32), four times its own error or
the tolerance, whichever is larger.  Sizes span several 256-node blocks with
ragged tails, walls and fully periodic boxes, every test mode."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1501_03857_amd import lbboil as L
from paper_1501_03857_amd import workloads as WL
from parity_utils import STORE_FACTOR, normwise

pytestmark = pytest.mark.gpu

A, B = 2.0 / 49.0, 2.0 / 21.0
TOL = {L.FP64: 1e-12, L.FP32: 1e-5}
TWIN = {L.FP64: 52, L.FP32: 24}


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _pair(nx, ny, nz, precision=L.FP64, periodic_y=0, mode=O.COUPLED, seed=3, Gw=0.06, Gw_top=-0.02, dT=0.08,
          noise=1e-2, rho0=None, u0=None, T0=None, **extra):
    tc = O.Tc(A, B, 1.0)
    rv, rl, _ = O.maxwell(A, B, 1.0, 0.344, 0.86 * tc)
    liquid = int(0.6 * ny)
    if rho0 is None:
        rho0 = WL.layered_density3(nx, ny, nz, rl, rv, liquid, noise, seed)
    Tb = np.full((nz, nx), 0.86 * tc)
    Tb[:, nx // 4: nx // 4 + max(1, nx // 2)] += dT * tc
    common = dict(nx=nx, ny=ny, a=A, b=B, rho_L=rl, rho_V=rv, Gw_bottom=Gw, Gw_top=Gw_top, periodic_y=periodic_y,
                  thermal_mode=mode, **extra)
    op = O.Params(**common)
    ux0 = uy0 = uz0 = None
    if u0 is not None:
        ux0, uy0, uz0 = u0
    o = O.State3(op, nz, rho0, ux0=ux0, uy0=uy0, uz0=uz0, T0=T0, T_bottom=Tb)
    tw = O.State3(op, nz, rho0, ux0=ux0, uy0=uy0, uz0=uz0, T0=T0, T_bottom=Tb).store_bits(TWIN[precision])
    d = L.Domain3(L.Params(precision=precision, liquid_rows=liquid, **common), nz, T_bottom=Tb, rho0=rho0)
    if u0 is not None or T0 is not None:
        d.set_fields(rho0, None if u0 is None else np.stack(u0), T0)
    return o, tw, d


def _compare(o, tw, d, precision, with_q=True):
    tol = TOL[precision]
    a, b, t = d.fields(), o.fields(), tw.fields()
    errs, bars = {}, {}
    for k in ("rho", "ux", "uy", "uz", "T", "f"):
        errs[k] = normwise(a[k], b[k])
        bars[k] = tol
        if k in ("ux", "uy", "uz"):
            errs["twin:" + k] = normwise(t[k], b[k])
            bars[k] = max(tol, STORE_FACTOR * errs["twin:" + k])
    if with_q:
        ha, hb, ht = d.heat_flux(), o.heat_flux(), tw.heat_flux()
        for k in ("q_local", "q_now", "q_mean"):
            if k == "q_mean" and not hb["n_samples"]:
                continue
            errs[k] = normwise(ha[k], hb[k])
            errs["twin:" + k] = normwise(ht[k], hb[k])
            bars[k] = max(tol, STORE_FACTOR * errs["twin:" + k])
        assert ha["n_samples"] == hb["n_samples"]
    print("[parity]", " ".join(f"{k}={v:.3g}" for k, v in errs.items()), flush=True)
    bad = {k: (errs[k], bars[k]) for k in bars if not errs[k] <= bars[k]}
    return errs, bad


@pytest.mark.parametrize("steps", [0, 1, 60])
def test_walls_fp64(steps):
    _say("3d walls fp64 29x21x11", steps)
    o, tw, d = _pair(29, 21, 11)
    for s in (o, tw, d):
        s.step(steps)
    errs, bad = _compare(o, tw, d, L.FP64)
    assert not bad, bad


@pytest.mark.parametrize("nx,ny,nz", [(3, 4, 3), (17, 9, 5), (64, 13, 7)])
def test_ragged_sizes_fp64(nx, ny, nz):
    _say("3d ragged", nx, ny, nz)
    o, tw, d = _pair(nx, ny, nz, seed=nx + ny)
    for s in (o, tw, d):
        s.step(40)
    errs, bad = _compare(o, tw, d, L.FP64)
    assert not bad, bad


def test_fp32_storage():
    _say("3d fp32 29x21x11")
    o, tw, d = _pair(29, 21, 11, precision=L.FP32)
    for s in (o, tw, d):
        s.step(60)
    errs, bad = _compare(o, tw, d, L.FP32)
    assert not bad, bad


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_periodic_box_conserves_mass(precision):
    _say("3d periodic", precision)
    tc = O.Tc(A, B, 1.0)
    nx, ny, nz = 20, 18, 12
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    T0 = 0.86 * tc * (1 + 0.01 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * z / nz))
    o, tw, d = _pair(nx, ny, nz, precision=precision, periodic_y=1, noise=5e-2, T0=T0)
    for s in (o, tw, d):
        s.step(60)
    errs, bad = _compare(o, tw, d, precision, with_q=False)
    assert not bad, bad
    m = d.fields(f=False)["rho"].sum() / o.fields()["rho"].sum()
    assert abs(m - 1) < (1e-13 if precision == L.FP64 else 1e-6)


@pytest.mark.parametrize("mode", [O.ISOTHERMAL, O.THERMAL_ONLY])
def test_test_modes_fp64(mode):
    _say("3d mode", mode)
    nx, ny, nz = 24, 16, 9
    u0 = T0 = None
    if mode == O.THERMAL_ONLY:
        z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
        s = np.sin(np.pi * y / (ny - 1))
        u0 = (0.02 * np.sin(2 * np.pi * x / nx) * s, 0.01 * np.cos(2 * np.pi * z / nz) * s,
              0.015 * np.cos(2 * np.pi * x / nx) * s)
    o, tw, d = _pair(nx, ny, nz, mode=mode, u0=u0, T0=T0)
    for s_ in (o, tw, d):
        s_.step(50)
    errs, bad = _compare(o, tw, d, L.FP64)
    assert not bad, bad


def test_parameter_variants_fp64():
    """sigma, relaxation rates, viscosities, thermal constants and gravity
    other than the defaults, in one run on a ragged lattice."""
    _say("3d parameter variant")
    o, tw, d = _pair(23, 15, 8, sigma=0.7, s_e=1.2, s_zeta=1.4, s_q=1.6, nu_L=0.05, nu_V=0.25, cv=4.0,
                     cv_chi=0.05, g=1e-4, seed=9)
    for s in (o, tw, d):
        s.step(50)
    errs, bad = _compare(o, tw, d, L.FP64)
    assert not bad, bad


def test_heater_change_and_average_reset():
    _say("3d heater change")
    o, tw, d = _pair(30, 16, 6)
    for s in (o, tw, d):
        s.step(33)
    tc = O.Tc(A, B, 1.0)
    Tb2 = np.full((6, 30), 0.98 * tc)
    for s in (o, tw, d):
        s.set_heater(Tb2)
        s.reset_average()
        s.step(41)
    errs, bad = _compare(o, tw, d, L.FP64)
    assert not bad, bad
    assert d.heat_flux()["n_samples"] == 41


def test_chunked_stepping_bitwise_and_builtin_initial_state():
    """Graph replays (32-step chunks) and single launches give the same bits;
    the built-in layered state equals the shared generator's bitwise."""
    _say("3d chunks")
    tc = O.Tc(A, B, 1.0)
    rv, rl, _ = O.maxwell(A, B, 1.0, 0.344, 0.86 * tc)
    p = L.Params(nx=21, ny=12, precision=L.FP32, liquid_rows=7, a=A, b=B, rho_L=rl, rho_V=rv, noise_amp=1e-3,
                 seed=5)
    runs = []
    for chunks in ([70], [3, 33, 34], [1] * 6 + [64]):
        d = L.Domain3(p, 5)
        for c in chunks:
            d.step(c)
        runs.append((d.fields(), d.heat_flux(local=False)))
        d.close()
    for f, h in runs[1:]:
        assert np.array_equal(f["f"], runs[0][0]["f"]) and np.array_equal(f["T"], runs[0][0]["T"])
        assert h["q_mean"] == runs[0][1]["q_mean"] and h["n_samples"] == 70
    p64 = L.Params(nx=21, ny=12, precision=L.FP64, liquid_rows=7, a=A, b=B, rho_L=rl, rho_V=rv, noise_amp=1e-3,
                   seed=5)
    d = L.Domain3(p64, 5)
    o = O.State3(O.Params(nx=21, ny=12, a=A, b=B, rho_L=rl, rho_V=rv), 5,
                 WL.layered_density3(21, 12, 5, rl, rv, 7, 1e-3, 5))
    assert np.array_equal(d.fields()["f"], o.fields()["f"])


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_larger_ragged_lattice(precision):
    """62x60x51: ragged first-stage column tiles in x and y (30x14
    interiors; runs of one plane in FP32, of 2 in FP64 with a last run of
    one), about 740 per-node blocks, walls."""
    _say("3d ragged 62x60x51", precision)
    o, tw, d = _pair(62, 60, 51, precision=precision, seed=9)
    for s in (o, tw, d):
        s.step(12)
    errs, bad = _compare(o, tw, d, precision)
    assert not bad, bad


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_first_stage_plane_runs(precision):
    """301x155x41: the first RK4 stage marches its 30x14 column tiles along z
    in runs of several planes (11 x 12 tiles; runs of 2 planes in FP32, 14 in
    FP64, the last one shorter), ragged in x, y and z, walls, 2 steps."""
    _say("3d plane runs 301x155x41", precision)
    o, tw, d = _pair(301, 155, 41, precision=precision, seed=11)
    for s in (o, tw, d):
        s.step(2)
    errs, bad = _compare(o, tw, d, precision)
    assert not bad, bad


def test_benchmarked_pool_full_size_fp32():
    """The benchmarked 3-D pool at its full size and launch shapes: 150x151x150
    nodes, FP32 storage, a = 3/49, liquid below 0.6 ny, heater 0.10 T_c over
    the whole bottom wall, G_w = 0.065, g = 3e-5; 2 steps against the oracle
    and its FP32 twin (every node and field compared)."""
    _say("3d benchmarked pool 150x151x150 fp32, 2 steps")
    a = 3.0 / 49.0
    nx, ny, nz = 150, 151, 150
    tc = O.Tc(a, B, 1.0)
    rv, rl, _ = O.maxwell(a, B, 1.0, 0.344, 0.86 * tc)
    liquid = int(0.6 * ny)
    rho0 = WL.layered_density3(nx, ny, nz, rl, rv, liquid, 1e-3, 7)
    Tb = np.full((nz, nx), 0.96 * tc)
    common = dict(nx=nx, ny=ny, a=a, b=B, rho_L=rl, rho_V=rv, g=3e-5, Gw_bottom=0.065)
    o = O.State3(O.Params(**common), nz, rho0, T_bottom=Tb)
    tw = O.State3(O.Params(**common), nz, rho0, T_bottom=Tb).store_bits(TWIN[L.FP32])
    d = L.Domain3(L.Params(precision=L.FP32, liquid_rows=liquid, seed=7, **common), nz, T_bottom=Tb, rho0=rho0)
    for s in (o, tw, d):
        s.step(2)
    errs, bad = _compare(o, tw, d, L.FP32)
    assert not bad, bad


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_long_run_heat_flux_matches_stored_oracle_run(precision):
    """A 40x51x20 pool with vapour on the heater (a = 3/49, T_s = 0.86 T_c,
    heater 0.14 T_c above T_s, G_w = 0.065, g = 3e-5), 16000 steps, against
    the oracle's FP64 run of the same pool stored by
    tests/golden/make_oracle_pool3d_long_run.py: the time average of q over
    steps 8001-16000 within 2% (the long-run bar), q every 2000 steps within
    a factor 1.5, the mass to 1e-5 and the vapour fraction at the heater to
    0.05."""
    _say("3d long run 40x51x20, 16000 steps vs stored oracle run", precision)
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_pool3d_40x51x20.json")) as fh:
        ref = json.load(fh)
    nx, ny, nz = ref["nx"], ref["ny"], ref["nz"]
    a, theta = ref["a"], ref["Ts_over_Tc"]
    tc = O.Tc(a, B, 1.0)
    rv, rl, _ = O.maxwell(a, B, 1.0, 0.344, theta * tc)
    liquid = int(0.6 * ny)
    rho0 = WL.layered_density3(nx, ny, nz, rl, rv, liquid, 1e-3, ref["seed"])
    p = L.Params(nx=nx, ny=ny, precision=precision, liquid_rows=liquid, a=a, b=B, Ts_over_Tc=theta, rho_L=rl,
                 rho_V=rv, g=ref["g"], Gw_bottom=ref["Gw_bottom"], seed=ref["seed"])
    d = L.Domain3(p, nz, T_bottom=np.full((nz, nx), (theta + ref["dT_over_Tc"]) * tc), rho0=rho0)
    trace = []
    for k in range(ref["steps"] // 2000):
        if k * 2000 == ref["steps"] // 2:
            d.reset_average()
        d.step(2000)
        trace.append(d.heat_flux()["q_now"])
    hf = d.heat_flux()
    rho = d.fields()["rho"]
    d.close()
    assert hf["n_samples"] == ref["n_samples"] == ref["steps"] // 2
    rel = abs(hf["q_mean"] / ref["q_mean"] - 1.0)
    vap = float(np.mean(rho[:, 1:3, :] < 0.5 * (rl + rv)))
    _say(f"q_mean gpu {hf['q_mean']:.6e} oracle {ref['q_mean']:.6e} rel {rel:.2e}; vapour at heater gpu {vap:.3f} "
         f"oracle {ref['vapour_at_heater']:.3f}")
    assert rel < 0.02
    q_ref = np.array([q for _, q in ref["q_trace"]])
    assert np.all(np.array(trace) > 0) and np.all(q_ref > 0)
    assert np.all(np.abs(np.log(np.array(trace) / q_ref)) < np.log(1.5))
    assert abs(float(np.sum(rho)) / ref["mass_final"] - 1.0) < 1e-5
    assert abs(vap - ref["vapour_at_heater"]) < 0.05
