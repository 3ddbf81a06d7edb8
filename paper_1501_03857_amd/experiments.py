"""The paper's boiling experiments on the batched GPU path (Sec. 3.1-3.3 of
arXiv:1501.03857): the 600 x 150 pool with the superheat-step protocol, the
transient and time-averaged bottom-wall heat flux, the heat transfer
coefficient, and the pressure at the centre of the top wall.

Every lattice step runs in the library's kernels; this module only builds
the inputs, switches heaters at the protocol's step time and records the
library's read-backs.  Run ``python -m paper_1501_03857_amd.experiments`` for
the boiling curves of Figs. 7 and 13 (the paper's curves are not reproduced
in its text, so the comparison is with its stated regimes), and with
``--calibrate`` for the contact angle against the wall strength G_w from
sessile drops (Sec. 3.2, 3.3), which turns contact-angle labels into G_w.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import lbboil as L
from .workloads import layered_density, smooth_layered_density, smooth_layered_density3

# Sec. 2 and Sec. 3.1: a = 3/49, b = 2/21, R = 1, omega = 0.344, sigma = 1.2,
# T_s = 0.86 T_c, nu_L = 0.1, nu_V = 0.5/3, c_v = 6, c_v chi = 0.028,
# g = 3e-5; a 600 x 150 domain between walls at y = 0 and y = 150 (151 wet
# node rows), liquid for y < 90.
PAPER_A, PAPER_B, PAPER_R, PAPER_OMEGA = 3.0 / 49.0, 2.0 / 21.0, 1.0, 0.344
PAPER_NX, PAPER_NY, PAPER_LIQUID_ROWS = 600, 151, 90
# Sec. 3.2: the superheat before the step at t = 20000 (Figs. 1-6)
PAPER_DT0, PAPER_T_STEP = 0.0137, 20000
# Sec. 3.2-3.3: the superheats of the boiling curves (lattice units) and the
# wall strengths of Sec. 3.3 (contact angles about 44.5, 50 and 55.5 deg)
PAPER_SUPERHEATS = (0.008, 0.01, 0.0137, 0.0165, 0.019, 0.021, 0.023, 0.025, 0.029, 0.032, 0.035)
PAPER_GW = (0.0, 0.065, 0.105)


def saturation(a: float = PAPER_A, b: float = PAPER_B, R: float = PAPER_R, omega: float = PAPER_OMEGA,
               Ts_over_Tc: float = 0.86) -> Tuple[float, float, float]:
    """(T_s, rho_V, rho_L) of the EOS at T_s = Ts_over_Tc T_c."""
    Tc, _ = L.eos_constants(a, b, R, omega)
    Ts = Ts_over_Tc * Tc
    rv, rl = L.coexistence(a, b, R, omega, Ts)
    return Ts, rv, rl


def paper_case(dT: float, Gw: float = 0.0, precision: int = L.FP32, seed: int = 1,
               nx: int = PAPER_NX, ny: int = PAPER_NY, coexistence: Optional[Tuple[float, float]] = None):
    """Params, bottom-wall temperature and initial density of the paper's pool
    at wall superheat dT (lattice units) and bottom wall strength Gw.
    `coexistence` = (rho_V, rho_L) replaces the library's Maxwell densities
    (the initial layers and the ends of tau_nu(rho))."""
    Ts, rv, rl = saturation()
    if coexistence is not None:
        rv, rl = coexistence
    liquid = int(round(PAPER_LIQUID_ROWS * (ny - 1) / (PAPER_NY - 1)))
    p = L.Params(nx=nx, ny=ny, precision=precision, liquid_rows=liquid, a=PAPER_A, b=PAPER_B, R=PAPER_R,
                 omega=PAPER_OMEGA, sigma=1.2, g=3e-5, Gw_bottom=Gw, rho_L=rl, rho_V=rv, seed=seed)
    Tb = np.full(nx, Ts + dT)
    rho0 = layered_density(nx, ny, rl, rv, liquid, p.noise_amp, seed)
    return p, Tb, rho0


def top_centre_pressure(dom: L.Domain) -> float:
    """p_EOS at the centre node of the top wall (Fig. 3)."""
    f = dom.fields(f=False)
    i, j = dom.p.nx // 2, dom.p.ny - 1
    return L.eos_pressure(dom.p.a, dom.p.b, dom.p.R, dom.p.omega, f["rho"][j, i], f["T"][j, i])


@dataclass
class BoilingRun:
    """One (superheat, wall strength) member of a boiling-curve batch."""
    dT: float
    Gw: float
    t: np.ndarray                      # sample times
    q: np.ndarray                      # q(t), Sec. 3.2
    q_mean: float = 0.0                # time average over the averaging window
    n_avg: int = 0
    p_top: Optional[np.ndarray] = None  # top-wall-centre pressure at the sample times

    @property
    def h_c(self) -> float:
        """Heat transfer coefficient q_mean / dT (Fig. 8)."""
        return self.q_mean / self.dT

    def summary(self) -> dict:
        return {"dT": self.dT, "Gw": self.Gw, "q_mean": self.q_mean, "h_c": self.h_c, "n_avg": self.n_avg,
                "q_std_window": float(np.std(self.q[self.t >= self.t[-1] - self._win])) if len(self.q) else 0.0}

    _win: int = field(default=0, repr=False)


def boiling_curve(superheats: Sequence[float] = PAPER_SUPERHEATS, wall_strengths: Sequence[float] = PAPER_GW,
                  t_end: int = 60000, t_avg: int = 30000, t_step: int = PAPER_T_STEP, dT0: float = PAPER_DT0,
                  sample_every: int = 200, probe: Sequence[Tuple[float, float]] = (),
                  precision: int = L.FP32, seed: int = 1, nx: int = PAPER_NX, ny: int = PAPER_NY,
                  tune_steps: int = 10, log=None, coexistence: Optional[Tuple[float, float]] = None,
                  inspect=None) -> Tuple[List[BoilingRun], dict]:
    """Every (dT, Gw) pair as one member of a single batch.

    Protocol (Sec. 3.2): members whose superheat exceeds dT0 heat at dT0 until
    t_step and then at their own superheat; the others heat at their own
    superheat throughout.  q(t) is sampled every `sample_every` steps and
    q_mean is the library's average over the last t_avg steps.  Members listed
    in `probe` as (dT, Gw) also record the top-wall-centre pressure.
    `coexistence` is passed to paper_case; `inspect(batch, cases)`, if given,
    is called on the batch after the last step, before it is released.
    Returns the runs and the wall time of the stepping (read-backs included)
    with the lattice-update rate it amounts to."""
    cases = [(dT, Gw) for Gw in wall_strengths for dT in superheats]
    params, Tbs, rhos = [], [], []
    Ts, _, _ = saturation()
    for dT, Gw in cases:
        p, Tb, rho0 = paper_case(min(dT, dT0) if t_step > 0 else dT, Gw, precision, seed, nx, ny, coexistence)
        params.append(p)
        Tbs.append(Tb)
        rhos.append(rho0)
    b = L.Batch(params, Tbs, rhos)
    try:
        if tune_steps > 0:
            b.autotune(tune_steps)
        probes = {i for i, c in enumerate(cases) if any(abs(c[0] - d) < 1e-12 and abs(c[1] - g) < 1e-12
                                                         for d, g in probe)}
        ts, qs = [], []
        ps: Dict[int, list] = {i: [] for i in probes}
        wall0 = time.perf_counter()
        t = 0
        stepped = t_step <= 0
        reset = False
        while t < t_end:
            if not stepped and t >= t_step:
                for i, (dT, _) in enumerate(cases):
                    if dT > dT0:
                        b.domain(i).set_heater(np.full(nx, Ts + dT))
                stepped = True
            if not reset and t >= t_end - t_avg:
                for i in range(len(cases)):
                    b.domain(i).reset_average()
                reset = True
            n = sample_every
            for edge in (t_step, t_end - t_avg):
                if t < edge < t + n:
                    n = edge - t
            n = min(n, t_end - t)
            b.step(n)
            t += n
            hf = b.heat_flux()
            ts.append(t)
            qs.append(hf["q_now"].copy())
            for i in probes:
                ps[i].append(top_centre_pressure(b.domain(i)))
            if log and len(ts) % 50 == 0:
                log(f"[boiling] t = {t}")
        hf = b.heat_flux()
        seconds = time.perf_counter() - wall0
        if inspect is not None:
            inspect(b, cases)
        updates = float(t_end) * sum(p.nx * p.ny for p in params)
        info = {"members": len(cases), "nx": nx, "ny": ny, "steps": t_end, "seconds": seconds,
                "mlups": updates / seconds / 1e6, "tiles": list(b.domain(0).tiles)}
        q = np.array(qs)
        out = []
        for i, (dT, Gw) in enumerate(cases):
            r = BoilingRun(dT=dT, Gw=Gw, t=np.array(ts), q=q[:, i], q_mean=float(hf["q_mean"][i]),
                           n_avg=int(hf["n_samples"][i]), p_top=np.array(ps[i]) if i in ps else None)
            r._win = t_avg
            out.append(r)
        return out, info
    finally:
        b.close()


def drop_angle(rho: np.ndarray, rho_L: float, rho_V: float, base_row: int = 1, plane: float = 1.0) -> float:
    """Contact angle (liquid side, degrees) of a drop resting on the bottom
    wall, from its circular cap: base width w on `base_row`, apex height h
    above the contact plane y = `plane` on the centre column,
    tan(theta / 2) = 2 h / w.  With the fluid-solid force the wall row is the
    solid and the plane is row 1, the first fluid row; with the ghost-layer
    wall the wall row, about which the ghost layer mirrors the fluid, is the
    contact plane (y = 0) and the base is read on it.  The interface is
    where the density crosses (rho_L + rho_V) / 2, located between nodes by
    linear interpolation.  NaN when the drop has left the wall (no liquid on
    the base row or on the centre column) or spread over the whole width."""
    mid = 0.5 * (rho_L + rho_V)
    ny, nx = rho.shape
    col = rho[:, nx // 2]
    inside = np.nonzero(col > mid)[0]
    base = rho[base_row]
    wet = np.nonzero(base > mid)[0]
    if len(inside) == 0 or len(wet) == 0:
        return float("nan")
    j = int(inside.max())
    apex = j + (col[j] - mid) / (col[j] - col[j + 1])
    i0, i1 = int(wet.min()), int(wet.max())
    if i0 == 0 or i1 == nx - 1 or j + 1 >= ny:
        return float("nan")
    w = (i1 - i0) + (base[i0] - mid) / (base[i0] - base[i0 - 1]) + (base[i1] - mid) / (base[i1] - base[i1 + 1])
    return float(2.0 * np.degrees(np.arctan(2.0 * (apex - plane) / w)))


def sessile_drops(wall_strengths: Sequence[float], a: float = PAPER_A, nx: int = 160, ny: int = 60,
                  radius: float = 22.0, steps: int = 5000, precision: int = L.FP64, ghost_layer: int = 0,
                  centre_y: float = 0.0) -> List[float]:
    """Equilibrium contact angles of a drop on the bottom wall for each wall
    strength G_w (Eq. (22)), all drops in one batch: isothermal at T_s, no
    gravity, a disc of liquid of the given radius centred at height
    `centre_y` above the wall row (0: a half-disc, 90 degrees to start with),
    relaxed for `steps` steps (Sec. 3.2, 3.3).  ghost_layer = 1 runs the wall
    variant with the fluid-fluid force on the wall rows through a ghost fluid
    layer (Sec. 3.2), whose contact plane is the wall row."""
    Ts, rv, rl = saturation(a=a)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    rho0 = rv + (rl - rv) * 0.5 * (1.0 - np.tanh((np.hypot(x - nx / 2, y - centre_y) - radius) / 2.0))
    params = [L.Params(nx=nx, ny=ny, precision=precision, a=a, rho_L=rl, rho_V=rv, g=0.0, Gw_bottom=float(Gw),
                       thermal_mode=L.ISOTHERMAL, liquid_rows=1, ghost_layer=ghost_layer) for Gw in wall_strengths]
    geom = dict(base_row=0, plane=0.0) if ghost_layer else {}
    b = L.Batch(params, None, [rho0] * len(params))
    try:
        b.step(steps)
        return [drop_angle(b.domain(i).fields(f=False)["rho"], rl, rv, **geom) for i in range(len(params))]
    finally:
        b.close()


def calibrate_wall_strength(targets_deg: Sequence[float], a: float = PAPER_A,
                            grid: Sequence[float] = tuple(np.round(np.arange(-0.10, 0.901, 0.05), 3)),
                            **drop_kw) -> dict:
    """The wall strength G_w that gives each target contact angle: theta(G_w)
    measured by sessile drops on `grid`, then inverted by linear
    interpolation on the monotone part of the curve.  Targets outside the
    measured range map to None."""
    angles = np.array(sessile_drops(grid, a=a, **drop_kw))
    g = np.asarray(grid, dtype=float)
    # keep the increasing run of the curve from its smallest angle on
    if not np.any(np.isfinite(angles)):
        return {"a": a, "grid": g.tolist(), "angles": angles.tolist(), "Gw": {float(t): None for t in targets_deg}}
    k0 = int(np.nanargmin(angles))
    gs, th = [g[k0]], [angles[k0]]
    for gi, ti in zip(g[k0 + 1:], angles[k0 + 1:]):
        if not np.isfinite(ti) or ti <= th[-1]:
            break
        gs.append(gi)
        th.append(ti)
    out = {}
    for t in targets_deg:
        out[float(t)] = float(np.interp(t, th, gs)) if th[0] <= t <= th[-1] else None
    return {"a": a, "grid": g.tolist(), "angles": angles.tolist(), "Gw": out}


# ---------------------------------------------------------------------------
# Larger density ratios (Sec. 4 names boiling at large density ratios as the
# model's next step).  Lowering T_s / T_c raises rho_L / rho_V along the
# Peng-Robinson coexistence curve: 17 at 0.86 T_c, 71 at 0.75, 145 at 0.70,
# 853 at 0.60 (a drops out of these reduced densities).  The model is
# unchanged; only the initial layers start smooth.

def large_ratio_pool(Ts_over_Tc: float, dT_over_Tc: float, a: float = 2.0 / 49.0, Gw: float = 0.0,
                     precision: int = L.FP32, seed: int = 1, nx: int = PAPER_NX, ny: int = PAPER_NY,
                     width: float = 2.5):
    """The paper's pool at T_s = Ts_over_Tc T_c with the whole bottom wall at
    T_s + dT_over_Tc T_c, liquid below row 90 (of 151) at the coexistence
    densities of T_s with a tanh interface of half-width `width`, gravity
    scaled with a from the paper's 3e-5 at a = 3/49 (the hydrostatic load then
    keeps its ratio to the pressure scale).  Returns (Params, T_bottom, rho0,
    rho_L / rho_V)."""
    Tc, _ = L.eos_constants(a, PAPER_B, PAPER_R, PAPER_OMEGA)
    Ts = Ts_over_Tc * Tc
    rv, rl = L.coexistence(a, PAPER_B, PAPER_R, PAPER_OMEGA, Ts)
    liquid = int(round(PAPER_LIQUID_ROWS * (ny - 1) / (PAPER_NY - 1)))
    p = L.Params(nx=nx, ny=ny, precision=precision, liquid_rows=liquid, a=a, b=PAPER_B, R=PAPER_R,
                 omega=PAPER_OMEGA, Ts_over_Tc=Ts_over_Tc, sigma=1.2, g=3e-5 * a / PAPER_A, Gw_bottom=Gw,
                 rho_L=rl, rho_V=rv, seed=seed)
    Tb = np.full(nx, Ts + dT_over_Tc * Tc)
    rho0 = smooth_layered_density(nx, ny, rl, rv, liquid, width, p.noise_amp, seed)
    return p, Tb, rho0, rl / rv


def large_ratio_boiling(cases: Sequence[Tuple[float, float, float]], steps: int = 40000, t_avg: int = 20000,
                        sample_every: int = 200, precision: int = L.FP32, nx: int = PAPER_NX,
                        ny: int = PAPER_NY) -> List[dict]:
    """Boiling pools of large_ratio_pool, one per (Ts_over_Tc, dT_over_Tc, a)
    case, in one batch: q(t) sampled every `sample_every` steps, its mean over
    the last t_avg steps, and at the end the vapour fraction of the two
    fluid rows next to the heater (near 1 once a vapour film covers it)."""
    built = [large_ratio_pool(th, dT, a, precision=precision, nx=nx, ny=ny) for th, dT, a in cases]
    b = L.Batch([x[0] for x in built], [x[1] for x in built], [x[2] for x in built])
    qs = [[] for _ in cases]
    ts = []
    try:
        for t in range(sample_every, steps + 1, sample_every):
            b.step(sample_every)
            hf = b.heat_flux()
            ts.append(t)
            for i in range(len(cases)):
                qs[i].append(float(hf["q_now"][i]))
        out = []
        for i, ((th, dT, a), (p, _, _, ratio)) in enumerate(zip(cases, built)):
            rho = b.domain(i).fields(f=False)["rho"]
            t_arr, q_arr = np.array(ts), np.array(qs[i])
            win = t_arr > steps - t_avg
            out.append({"Ts_over_Tc": th, "dT_over_Tc": dT, "a": a, "density_ratio": ratio, "t": t_arr, "q": q_arr,
                        "q_mean": float(q_arr[win].mean()),
                        "vapour_at_heater": float(np.mean(rho[1:3] < 0.5 * (p.rho_L + p.rho_V)))})
        return out
    finally:
        b.close()


def large_ratio_boiling3(cases: Sequence[Tuple[float, float, float]], nx: int = 120, ny: int = 81, nz: int = 60,
                         steps: int = 20000, t_avg: int = 10000, sample_every: int = 500,
                         precision: int = L.FP32) -> List[dict]:
    """Three-dimensional pools (the D3Q19 path), one per (Ts_over_Tc,
    dT_over_Tc, a) case, run one after another: liquid below row 0.6 ny with
    a smooth interface, the whole bottom wall dT above T_s, gravity scaled
    with a.  Per case: q(t) sampled every `sample_every` steps, the mean of
    q over the last t_avg steps (the library's running average, restarted
    there), and the vapour fraction of the two fluid rows next to the heater
    at every sample."""
    out = []
    for th, dT, a in cases:
        Tc, _ = L.eos_constants(a, PAPER_B, PAPER_R, PAPER_OMEGA)
        Ts = th * Tc
        rv, rl = L.coexistence(a, PAPER_B, PAPER_R, PAPER_OMEGA, Ts)
        liquid = int(0.6 * ny)
        p = L.Params(nx=nx, ny=ny, precision=precision, liquid_rows=liquid, a=a, b=PAPER_B, R=PAPER_R,
                     omega=PAPER_OMEGA, Ts_over_Tc=th, sigma=1.2, g=3e-5 * a / PAPER_A, rho_L=rl, rho_V=rv)
        rho0 = smooth_layered_density3(nx, ny, nz, rl, rv, liquid, 2.5, p.noise_amp, p.seed)
        d = L.Domain3(p, nz, T_bottom=np.full((nz, nx), Ts + dT * Tc), rho0=rho0)
        ts, qs, vap = [], [], []
        try:
            for t in range(sample_every, steps + 1, sample_every):
                if t - sample_every == steps - t_avg:
                    d.reset_average()
                d.step(sample_every)
                ts.append(t)
                qs.append(d.heat_flux(local=False)["q_now"])
                rho = d.fields(f=False)["rho"]
                vap.append(float(np.mean(rho[:, 1:3, :] < 0.5 * (rl + rv))))
            q_mean = d.heat_flux(local=False)["q_mean"]
        finally:
            d.close()
        out.append({"Ts_over_Tc": th, "dT_over_Tc": dT, "a": a, "density_ratio": rl / rv, "t": np.array(ts),
                    "q": np.array(qs), "q_mean": float(q_mean), "vapour_at_heater": np.array(vap)})
    return out


def flat_interfaces(thetas: Sequence[float], a: float = 2.0 / 49.0, sigma: float = 1.2, steps: int = 20000,
                    ny: int = 100, precision: int = L.FP64) -> List[dict]:
    """Coexistence on the lattice: one periodic 4 x ny slab per T_s / T_c
    (liquid in the middle half, smooth interfaces, no gravity, T fixed), all
    in one batch; the densities at the slab centre and half a period away
    after `steps` steps against the Maxwell densities."""
    params, rhos, maxwell = [], [], []
    for th in thetas:
        Tc, _ = L.eos_constants(a, PAPER_B, PAPER_R, PAPER_OMEGA)
        rv, rl = L.coexistence(a, PAPER_B, PAPER_R, PAPER_OMEGA, th * Tc)
        params.append(L.Params(nx=4, ny=ny, precision=precision, a=a, b=PAPER_B, R=PAPER_R, omega=PAPER_OMEGA,
                               Ts_over_Tc=th, sigma=sigma, g=0.0, rho_L=rl, rho_V=rv, periodic_y=1,
                               thermal_mode=L.ISOTHERMAL))
        j = np.abs(np.arange(ny) + 0.5 - ny / 2)
        rhos.append((rv + (rl - rv) * 0.5 * (1 - np.tanh((j - ny / 4) / 2.5)))[:, None] * np.ones((1, 4)))
        maxwell.append((rv, rl))
    b = L.Batch(params, None, rhos)
    try:
        b.step(steps)
        out = []
        for i, th in enumerate(thetas):
            r = b.domain(i).fields(f=False)["rho"]
            out.append({"Ts_over_Tc": th, "rho_V": float(r[0, 0]), "rho_L": float(r[ny // 2, 0]),
                        "maxwell": maxwell[i], "rho": r})
        return out
    finally:
        b.close()


def regimes(runs: Sequence[BoilingRun]) -> Dict[float, dict]:
    """Per wall strength: the superheat of the largest q_mean (critical heat
    flux), of the largest h_c, and the curve itself."""
    out = {}
    for Gw in sorted({r.Gw for r in runs}):
        rs = sorted((r for r in runs if r.Gw == Gw), key=lambda r: r.dT)
        q = np.array([r.q_mean for r in rs])
        h = np.array([r.h_c for r in rs])
        out[Gw] = {"dT": [r.dT for r in rs], "q_mean": q.tolist(), "h_c": h.tolist(),
                   "dT_chf": rs[int(np.argmax(q))].dT, "q_chf": float(q.max()), "dT_hmax": rs[int(np.argmax(h))].dT}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="Boiling curves of the paper's pool on the batched GPU path.")
    ap.add_argument("--t-end", type=int, default=60000)
    ap.add_argument("--t-avg", type=int, default=30000)
    ap.add_argument("--sample-every", type=int, default=200)
    ap.add_argument("--gw", type=float, nargs="*", default=list(PAPER_GW))
    ap.add_argument("--dt", type=float, nargs="*", default=list(PAPER_SUPERHEATS))
    ap.add_argument("--out", default=None, help="write the curves and q(t) as JSON")
    ap.add_argument("--calibrate", action="store_true",
                    help="contact angle against G_w for a = 2/49 and 3/49 instead of the boiling curves")
    args = ap.parse_args(argv)
    if args.calibrate:
        res = [calibrate_wall_strength((40, 44.5, 50, 55.5, 60, 90, 120), a=a) for a in (2.0 / 49.0, PAPER_A)]
        for r in res:
            print(f"a = {r['a']:.6f}: " + " ".join(f"{g:+.2f}:{t:.1f}" for g, t in zip(r["grid"], r["angles"])))
            print("   G_w for " + ", ".join(f"{t:g} deg -> {'out of range' if v is None else f'{v:.4f}'}"
                                           for t, v in r["Gw"].items()))
        if args.out:
            with open(args.out, "w") as fh:
                json.dump(res, fh)
        return
    runs, info = boiling_curve(args.dt, args.gw, t_end=args.t_end, t_avg=args.t_avg, sample_every=args.sample_every,
                               probe=[(PAPER_DT0, 0.0), (0.0165, 0.0)],
                               log=lambda s: print(s, file=sys.stderr, flush=True))
    reg = regimes(runs)
    print(f"{info['members']} lattices of {info['nx']}x{info['ny']}, {info['steps']} steps in {info['seconds']:.2f} s "
          f"({info['mlups']:.0f} MLUPS with the read-backs), tiles {info['tiles']}")
    for Gw, r in reg.items():
        print(f"G_w = {Gw}: CHF {r['q_chf']:.4e} at dT = {r['dT_chf']}, max h_c at dT = {r['dT_hmax']}")
        for dT, q, h in zip(r["dT"], r["q_mean"], r["h_c"]):
            print(f"   dT = {dT:.4f}  q_mean = {q:.4e}  h_c = {h:.4e}")
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"info": info, "regimes": {str(k): v for k, v in reg.items()},
                       "runs": [dict(r.summary(), t=r.t.tolist(), q=r.q.tolist(),
                                     p_top=None if r.p_top is None else r.p_top.tolist()) for r in runs]}, fh)


if __name__ == "__main__":
    main()
