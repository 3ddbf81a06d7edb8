#!/usr/bin/env python3
"""Write the oracle's long-horizon heat flux of two boiling pools at larger
density ratios.

Runs the CPU oracle (FP64) on 200x151 pools (liquid below row 90 at the
coexistence densities of T_s, smooth interfaces of half-width 2.5 with seeded
1e-3 noise, the whole bottom wall 0.35 T_c above T_s, G_w = 0, sigma = 1.2,
gravity 3e-5 a / (3/49)) for 20000 steps:
  * T_s = 0.75 T_c with a = 3/49 (rho_L / rho_V = 71),
  * T_s = 0.70 T_c with a = 2/49 (rho_L / rho_V = 145),
and stores for each: q (Sec. 3.2) after every 1000th step, the time average
of q over steps 10001-20000 (average reset after step 10000) and the total
mass after step 20000.  Only the oracle and the seeded input generator are
used.  Takes a few minutes on 8 cores.

    python tests/golden/make_oracle_ratio_long_runs.py
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1501_03857_amd import workloads as WL  # noqa: E402

NX, NY, LIQUID, WIDTH, NOISE, SEED = 200, 151, 90, 2.5, 1e-3, 1
B, OMEGA, A3 = 2.0 / 21.0, 0.344, 3.0 / 49.0
CASES = [(0.75, 0.35, 3.0 / 49.0), (0.70, 0.35, 2.0 / 49.0)]


def pool(theta, dT, a):
    """Oracle parameters, initial density and heater of one pool."""
    tc = O.Tc(a, B, 1.0)
    rv, rl, _ = O.maxwell(a, B, 1.0, OMEGA, theta * tc)
    p = O.Params(nx=NX, ny=NY, a=a, b=B, omega=OMEGA, Ts_over_Tc=theta, sigma=1.2, g=3e-5 * a / A3,
                 Gw_bottom=0.0, rho_L=rl, rho_V=rv)
    rho0 = WL.smooth_layered_density(NX, NY, rl, rv, LIQUID, WIDTH, NOISE, SEED)
    return p, rho0, np.full(NX, (theta + dT) * tc), rl / rv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", default=os.path.join(HERE, "oracle_ratio_pools_200x151.json"))
    args = ap.parse_args()
    runs = []
    t0 = time.time()
    for theta, dT, a in CASES:
        p, rho0, Tb, ratio = pool(theta, dT, a)
        s = O.State(p, rho0, T_bottom=Tb)
        half = args.steps // 2
        q_trace = []
        for k in range(args.steps // 1000):
            if k * 1000 == half:
                s.reset_average()
            s.step(1000)
            q_trace.append([s.t, s.heat_flux()["q_now"]])
        hf = s.heat_flux()
        runs.append({"Ts_over_Tc": theta, "dT_over_Tc": dT, "a": a, "density_ratio": ratio, "q_trace": q_trace,
                     "q_mean_window": [half + 1, args.steps], "q_mean": hf["q_mean"], "n_samples": hf["n_samples"],
                     "mass_final": float(np.sum(s.fields()["rho"]))})
        print(f"T_s = {theta} T_c, ratio {ratio:.1f}: q_mean {hf['q_mean']:.6e}  ({time.time() - t0:.0f} s)",
              flush=True)
    out = {"nx": NX, "ny": NY, "liquid_rows": LIQUID, "width": WIDTH, "noise_amp": NOISE, "seed": SEED,
           "steps": args.steps, "runs": runs, "oracle_threads": O.num_threads(), "seconds": round(time.time() - t0, 1)}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
