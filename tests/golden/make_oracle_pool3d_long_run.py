#!/usr/bin/env python3
"""Write the oracle's long-horizon heat flux of a small boiling 3-D pool.

Runs the CPU oracle (FP64, D3Q19) on a 40x51x20 pool (a = 3/49, T_s = 0.86
T_c, liquid below row 30 with seeded 1e-3 noise, the whole bottom wall at
T_s + 0.14 T_c, where vapour forms on the heater, G_w = 0.065, g = 3e-5) for
16000 steps, and stores:
  * q (Sec. 3.2) of the state after every 2000th step,
  * the time average of q over steps 8001-16000 (average reset after step
    8000), the window the GPU test compares with,
  * the total mass and the vapour fraction of the two fluid rows next to the
    heater after step 16000.
Only the oracle and the seeded input generator are used.  Takes about twelve
minutes on 8 cores.

    python tests/golden/make_oracle_pool3d_long_run.py
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

NX, NY, NZ = 40, 51, 20
A, B, OMEGA = 3.0 / 49.0, 2.0 / 21.0, 0.344
THETA, DT, GW, G, SEED = 0.86, 0.14, 0.065, 3e-5, 7


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=16000)
    ap.add_argument("--out", default=os.path.join(HERE, "oracle_pool3d_40x51x20.json"))
    args = ap.parse_args()
    tc = O.Tc(A, B, 1.0)
    rv, rl, _ = O.maxwell(A, B, 1.0, OMEGA, THETA * tc)
    liquid = int(0.6 * NY)
    p = O.Params(nx=NX, ny=NY, a=A, b=B, omega=OMEGA, Ts_over_Tc=THETA, g=G, Gw_bottom=GW, rho_L=rl, rho_V=rv)
    rho0 = WL.layered_density3(NX, NY, NZ, rl, rv, liquid, 1e-3, SEED)
    s = O.State3(p, NZ, rho0, T_bottom=np.full((NZ, NX), (THETA + DT) * tc))
    half = args.steps // 2
    q_trace = []
    t0 = time.time()
    for k in range(args.steps // 2000):
        if k * 2000 == half:
            s.reset_average()
        s.step(2000)
        q_trace.append([s.t, s.heat_flux()["q_now"]])
        print(f"step {s.t}: q = {q_trace[-1][1]:.6e}  ({time.time() - t0:.0f} s)", flush=True)
    hf = s.heat_flux()
    rho = s.fields()["rho"]
    out = {"nx": NX, "ny": NY, "nz": NZ, "a": A, "Ts_over_Tc": THETA, "dT_over_Tc": DT, "Gw_bottom": GW, "g": G,
           "seed": SEED, "steps": args.steps, "q_trace": q_trace, "q_mean_window": [half + 1, args.steps],
           "q_mean": hf["q_mean"], "n_samples": hf["n_samples"], "mass_final": float(np.sum(rho)),
           "vapour_at_heater": float(np.mean(rho[:, 1:3, :] < 0.5 * (rl + rv))),
           "oracle_threads": O.num_threads(), "seconds": round(time.time() - t0, 1)}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: out[k] for k in ("q_mean", "n_samples", "mass_final", "vapour_at_heater", "seconds")}))


if __name__ == "__main__":
    main()
