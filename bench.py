#!/usr/bin/env python3
"""Benchmark of the coupled LB + thermal time step on one MI355X.

Workload: the 1024x512 boiling lattice (a = 2/49, T_s = 0.86 T_c,
full-width heater at 0.10 T_c, G_w = 0.107 for a 60 deg contact angle), FP32 storage, inputs
resident in HBM before the timed region.  A "step" is one time step of the
whole hot path (LB launch + thermal launch, with the mass and heat-flux
reductions) over the lattice.  --steps K steps are timed with HIP events on
the library's stream around graph replays; value = nx*ny*K / time in MLUPS.

Prints ONE JSON line.  --gpus N > 1 exits: the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update of the method in FP32 storage: the nine
# populations and T, each read once and written once.
ALG_BYTES_STEP = {"f32": 80, "f64": 160}
# The LB launch's share of it: the nine populations read and written; the
# thermal launch's: T read and written.
ALG_BYTES_LB = {"f32": 72, "f64": 144}
ALG_BYTES_TH = {"f32": 8, "f64": 16}


def _kernel_roofline(alg_bytes, ms, traffic, per_update):
    """One launch priced against HBM: algorithmic bytes over its mean
    duration (events recorded by the dispatches)."""
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "kernel_ms": round(ms, 6), "alg_bytes_per_update": per_update, "traffic": traffic,
            "traffic_unit": "bytes per launch"}

# HBM traffic of each launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch, mean over the dispatches of a --profile run with the
# given tiles), each scaled by what the same counter reads for an
# elementwise kernel that reads 1 GiB and writes 1 GiB (FETCH_SIZE 524297.8
# KiB -> factor 2.00, WRITE_SIZE 1048576 KiB -> factor 1.0).  The factor is
# the one under which the 3-D kernels whose reads are fixed by their design
# fetch exactly those bytes; a copy whose input sits partly in the
# last-level cache reads less (one session read 436918.5 KiB), since
# FETCH_SIZE does not count those hits.  Valid for the kernel source whose
# hash is recorded and the same tile shape; null otherwise.
MEASURED_TRAFFIC = {
    "source_hash": "7f926bdeb6b7b8bd",
    "fetch_factor": 1048576.0 / 524297.8,
    "write_factor": 1048576.0 / 1048576.0,
    "k_lb": {
        "large_1024x512_fp32": [
            {"tiles": [62, 4, 4], "fetch_kib": 10725.0, "write_kib": 24620.1},
            {"tiles": [62, 8, 8], "fetch_kib": 10719.3, "write_kib": 24640.2},
        ],
        "large_4096x2048_fp32": [
            {"tiles": [62, 4, 4], "fetch_kib": 166708.7, "write_kib": 395598.9},
        ],
    },
    "k_thermal": {
        "large_1024x512_fp32": [
            {"tiles": [56, 24, 16], "fetch_kib": 4838.3, "write_kib": 2040.2},
        ],
        "large_4096x2048_fp32": [
            {"tiles": [56, 40, 16], "fetch_kib": 68760.1, "write_kib": 32749.2},
        ],
    },
}

# The same counters for the seven launches of one 3-D step (150x151x150 pool,
# FP32 storage; KiB per dispatch), valid for the 3-D kernel and host sources
# whose hash is recorded (the host source sets the first stage's plane runs).
MEASURED_TRAFFIC_3D = {
    "source_hash": "c97ad07e51234cee",
    "pool3d_150x151x150_fp32": {
        "k3_psi": (132765.1, 40023.5), "k3_reduce": (108.5, 0.1), "k3_lb": (146640.1, 294904.3),
        "k3_stage0": (37460.4, 93766.5), "k3_stage1": (53429.2, 26544.7), "k3_stage2": (53429.4, 26543.0),
        "k3_stage3": (53351.1, 13271.5),
    },
}


def measured_traffic_3d(workload: str):
    """HBM bytes of one 3-D step from the recorded counters, or None when
    the 3-D kernel source or the workload differ."""
    m = MEASURED_TRAFFIC_3D
    if m.get("source_hash") != source_hash("lbb3_device.hpp", "lbb3_host.hpp") or workload not in m:
        return None
    f = MEASURED_TRAFFIC["fetch_factor"]
    return int(round(sum(fe * f + wr for fe, wr in m[workload].values()) * 1024))


def measured_traffic(kernel: str, workload: str, tiles):
    """HBM bytes per launch of `kernel` from the recorded counters, or None
    when the kernel source, the workload or the tile shape differ."""
    m = MEASURED_TRAFFIC
    if not m or m.get("source_hash") != source_hash():
        return None
    for c in m.get(kernel, {}).get(workload, []):
        if list(c["tiles"]) == list(tiles):
            return int(round((c["fetch_kib"] * m["fetch_factor"] + c["write_kib"] * m["write_factor"]) * 1024))
    return None


def arithmetic(store: str) -> str:
    """The arithmetic types of the step for a storage precision."""
    if store == "f64":
        return "f64"
    return "mixed: f32 storage; f64 LB, EOS and reductions; f32 RK4 stages (pressure-work coefficients formed in f64)"


def source_hash(*names: str) -> str:
    """Hash of kernel source files (the recorded counters depend on them and,
    in 2-D, on the tile shape; the 3-D launch shapes are set in the 3-D host
    source, which is hashed with its kernels)."""
    h = hashlib.sha256()
    for name in names or ("lbb_device.hpp",):
        with open(os.path.join(ROOT, "paper_1501_03857_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """HBM bandwidth a plain elementwise kernel reaches on this GPU: torch.neg
    reading and writing nbytes each, timed with events over `reps` launches
    after two untimed ones; GB/s of read + write traffic."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        torch.neg(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps):
    """The oracle, as it stands, on the host cores over a bounded sample."""
    import oracle as O

    tc = O.Tc(w.a, w.b, w.R)
    rv, rl, _ = O.maxwell(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * tc)
    p = O.Params(nx=w.nx, ny=w.ny, a=w.a, b=w.b, sigma=w.sigma, g=w.g, Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv)
    s = O.State(p, w.density(rl, rv), T_bottom=w.heater_T(tc))
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(w.nx * w.ny * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle", "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"first {steps} steps of the {w.nx}x{w.ny} workload in FP64 "
                      f"({w.nx * w.ny * steps:.3g} lattice updates, {dt:.1f} s)"}


def sweep_bench(steps, warmup=50, tune_steps=10):
    """The 48-lattice boiling-curve sweep: aggregate MLUPS of one batch
    (shared launches, autotuned) against the same lattices run one after
    another through the single-lattice path with its default tiles ("plain"),
    and again with each lattice autotuned; each timed with HIP events on its
    stream."""
    import torch
    from paper_1501_03857_amd import lbboil as L
    from paper_1501_03857_amd import workloads as WL

    ws = WL.sweep_workloads(steps)
    params, tbs, rhos = [], [], []
    for w in ws:
        Tc, _ = L.eos_constants(w.a, w.b, w.R, w.omega)
        rv, rl = L.coexistence(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * Tc)
        params.append(L.Params(nx=w.nx, ny=w.ny, precision=L.FP32, liquid_rows=w.liquid_rows, a=w.a, b=w.b,
                               R=w.R, omega=w.omega, Ts_over_Tc=w.Ts_over_Tc, sigma=w.sigma, g=w.g,
                               Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv))
        tbs.append(w.heater_T(Tc))
        rhos.append(w.density(rl, rv))
    cells = sum(w.nx * w.ny for w in ws)

    def timed(obj, n):
        st = torch.cuda.ExternalStream(obj.stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        obj.step_async(n)
        e1.record(st)
        obj.sync()
        return e0.elapsed_time(e1)

    b = L.Batch(params, tbs, rhos)
    tb_tiles = b.autotune(tune_steps)
    b.step(warmup)
    ms_batch = timed(b, steps)
    q_batch = b.heat_flux()["q_mean"]
    b.close()
    ms_plain = ms_tuned = 0.0
    for p, tb, rho in zip(params, tbs, rhos):
        d = L.Domain(p, T_bottom=tb, rho0=rho)
        d.step(warmup)
        ms_plain += timed(d, steps)
        d.close()
        d = L.Domain(p, T_bottom=tb, rho0=rho)
        d.autotune(tune_steps)
        d.step(warmup)
        ms_tuned += timed(d, steps)
        d.close()
    mb = cells * steps / (ms_batch * 1e-3) / 1e6
    mp = cells * steps / (ms_plain * 1e-3) / 1e6
    mt = cells * steps / (ms_tuned * 1e-3) / 1e6
    sizes = {}
    for w in ws:
        sizes[f"{w.nx}x{w.ny}"] = sizes.get(f"{w.nx}x{w.ny}", 0) + 1
    return {"instances": len(ws), "cells": cells, "steps": steps, "sizes": sizes,
            "batched_mlups": round(mb, 1), "plain_sequential_mlups": round(mp, 1),
            "speedup": round(mb / mp, 2), "batched_ms": round(ms_batch, 3), "plain_ms": round(ms_plain, 3),
            "sequential_autotuned_mlups": round(mt, 1), "speedup_vs_autotuned": round(mb / mt, 2),
            "batch_tiles": [tb_tiles["shape_lb"], tb_tiles["shape_thermal"]],
            "q_mean_range": [float(min(q_batch)), float(max(q_batch))]}


def adjoint_bench():
    """Cost of the adjoint against the forward on the adjoint workload
    (256x128, heater i in [96, 160) at 0.10 T_c, G_w = 0.065, 400 steps),
    autotuned tiles, wall time of synchronous calls: checkpoints every 50
    with recompute, and with the interval the library picks (K <= 0)."""
    from paper_1501_03857_amd import lbboil as L
    from paper_1501_03857_amd import workloads as WL

    w = WL.ADJOINT_256x128
    out = {"workload": w.name, "steps": w.steps, "K": 50}
    Tc, _ = L.eos_constants(w.a, w.b, w.R, w.omega)
    rv, rl = L.coexistence(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * Tc)
    for name, prec in (("f64", L.FP64), ("f32", L.FP32)):
        p = L.Params(nx=w.nx, ny=w.ny, precision=prec, liquid_rows=w.liquid_rows, sigma=w.sigma, g=w.g,
                     Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv)
        d = L.Domain(p, T_bottom=w.heater_T(Tc), rho0=w.density(rl, rv))
        d.autotune(20)
        d.step(8)
        blob = d.save()
        t0 = time.perf_counter()
        d.step(w.steps)
        fwd = time.perf_counter() - t0
        d.load(blob)
        d.adjoint(w.steps, 50)  # warm-up: the workspace for this interval, first launches
        t0 = time.perf_counter()
        J, g, gw = d.adjoint(w.steps, 50)
        adj = time.perf_counter() - t0
        d.adjoint(w.steps, 0)  # warm-up for the interval the library picks
        t0 = time.perf_counter()
        d.adjoint(w.steps, 0)
        adj_auto = time.perf_counter() - t0
        out[name] = {"forward_ms": round(fwd * 1e3, 3), "adjoint_ms": round(adj * 1e3, 3),
                     "ratio": round(adj / fwd, 2), "adjoint_auto_K_ms": round(adj_auto * 1e3, 3),
                     "ratio_auto_K": round(adj_auto / fwd, 2), "J": J, "dJ_dGw": gw,
                     "tiles": list(d.tiles)}
        d.close()
    return out


def batch_adjoint_bench(steps=600):
    """Batched adjoint: 16 lattices of 384x192 (FP32), 600 steps, checkpoint
    interval chosen by the library.  Forward = the same 600 steps of the batch
    (graph replays); adjoint = one lbb_batch_adjoint call; device memory as
    the library's own count and the drop of hipMemGetInfo's free bytes."""
    import torch
    from paper_1501_03857_amd import lbboil as L
    from paper_1501_03857_amd import workloads as WL

    ws = WL.batch_adjoint_workloads(steps)
    params, tbs, rhos = [], [], []
    for w in ws:
        Tc, _ = L.eos_constants(w.a, w.b, w.R, w.omega)
        rv, rl = L.coexistence(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * Tc)
        params.append(L.Params(nx=w.nx, ny=w.ny, precision=L.FP32, liquid_rows=w.liquid_rows, a=w.a, b=w.b,
                               R=w.R, omega=w.omega, Ts_over_Tc=w.Ts_over_Tc, sigma=w.sigma, g=w.g,
                               Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv))
        tbs.append(w.heater_T(Tc))
        rhos.append(w.density(rl, rv))
    b = L.Batch(params, tbs, rhos)
    b.autotune(10)
    b.step(64)  # graph instantiation and first launches
    free0 = torch.cuda.mem_get_info()[0]
    blob = [b.domain(i).save() for i in range(len(ws))]
    t0 = time.perf_counter()
    b.step(steps)
    fwd = time.perf_counter() - t0
    for i, x in enumerate(blob):
        b.domain(i).load(x)
    t0 = time.perf_counter()
    J, g, gw = b.adjoint(steps, 0)
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    J2, g2, gw2 = b.adjoint(steps, 0)
    adj = time.perf_counter() - t0
    free1 = torch.cuda.mem_get_info()[0]
    dev = b.device_bytes()
    b.close()
    return {"instances": len(ws), "nx": 384, "ny": 192, "storage": "f32", "steps": steps, "K": "auto",
            "forward_ms": round(fwd * 1e3, 3), "adjoint_ms": round(adj * 1e3, 3),
            "adjoint_first_call_ms": round(first * 1e3, 3), "ratio": round(adj / fwd, 2),
            "repeat_bitwise": bool(np.array_equal(J, J2) and all(np.array_equal(a, c) for a, c in zip(g, g2))),
            "J_range": [float(J.min()), float(J.max())], "dJ_dGw_range": [float(gw.min()), float(gw.max())],
            "library_device_bytes": int(dev), "hip_free_bytes_drop": int(free0 - free1)}


def three_d_bench(steps=300, warmup=64, nx=150, ny=151, nz=150):
    """The three-dimensional (D3Q19) step on a pool of nx x ny x nz nodes in
    FP32 storage (a = 3/49, liquid below 0.6 ny, full-width heater at
    0.10 T_c, G_w = 0.065): MLUPS over graph replays timed with HIP events on
    the library's stream, and the step priced against HBM with its
    algorithmic 160 B/update (19 populations and T read and written)."""
    import torch
    from paper_1501_03857_amd import lbboil as L
    from paper_1501_03857_amd import workloads as WL

    a = 3.0 / 49.0
    Tc, _ = L.eos_constants(a, 2.0 / 21.0, 1.0, 0.344)
    rv, rl = L.coexistence(a, 2.0 / 21.0, 1.0, 0.344, 0.86 * Tc)
    liquid = int(0.6 * ny)
    p = L.Params(nx=nx, ny=ny, precision=L.FP32, liquid_rows=liquid, a=a, rho_L=rl, rho_V=rv, g=3e-5,
                 Gw_bottom=0.065, seed=7)
    d = L.Domain3(p, nz, T_bottom=np.full((nz, nx), 0.96 * Tc),
                  rho0=WL.layered_density3(nx, ny, nz, rl, rv, liquid, 1e-3, 7))
    d.step(warmup)
    st = torch.cuda.ExternalStream(d.stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    d.step_async(steps)
    e1.record(st)
    d.sync()
    ms = e0.elapsed_time(e1) / steps
    cells = nx * ny * nz
    gbs = 160 * cells / (ms * 1e-3) / 1e9
    q = d.heat_flux(local=False)
    name = f"pool3d_{nx}x{ny}x{nz}_fp32"
    traffic = measured_traffic_3d(name)
    d.close()
    return {"workload": name, "nodes": cells, "steps": steps, "ms_per_step": round(ms, 4),
            "mlups": round(cells / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_update": 160,
                         "traffic": traffic, "traffic_unit": "bytes per step",
                         "traffic_gbs": None if traffic is None else round(traffic / (ms * 1e-3) / 1e9, 1)},
            "launches_per_step": 7, "q_mean": q["q_mean"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="large", choices=["large", "large4096", "plain"])
    ap.add_argument("--kernel-steps", type=int, default=400, help="steps timed per launch for the roofline")
    ap.add_argument("--tune-steps", type=int, default=30,
                    help="steps per tile shape for the autotuner before timing (0: default shapes)")
    ap.add_argument("--tiles", default=None,
                    help="LB,thermal tile shape indices to use instead of the autotuner (profiling runs)")
    ap.add_argument("--cpu-steps", type=int, default=300, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=10000, help="steps of the 48-lattice sweep comparison (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--three-d-steps", type=int, default=300, help="steps of the 3-D pool measurement (0: skip)")
    ap.add_argument("--three-d-only", action="store_true", help="only the 3-D pool measurement (profiling)")
    ap.add_argument("--adjoint-only", action="store_true", help="only the adjoint/forward cost measurement (profiling)")
    ap.add_argument("--profile", action="store_true", help="timed region only (for rocprofv3 runs)")
    ap.add_argument("--copy-probe", action="store_true", help="run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(batches would shard by lattice, a single lattice by x-slabs with halo exchange)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_probe:
        # An elementwise kernel that reads 1 GiB and writes 1 GiB (a same-type
        # copy_ may go to a DMA engine, which the shader counters never see).
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}))
        return

    if args.three_d_only:
        print(json.dumps({"three_d": three_d_bench(args.three_d_steps or 300)}), flush=True)
        return

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_bench(), "batch_adjoint": batch_adjoint_bench()}), flush=True)
        return

    from paper_1501_03857_amd import lbboil as L
    from paper_1501_03857_amd import workloads as WL

    w = {"large": WL.LARGE_1024x512, "large4096": WL.LARGE_4096x2048, "plain": WL.PLAIN_128x64}[args.workload]
    store = "f32" if w.precision == "fp32" else "f64"
    Tc, _ = L.eos_constants(w.a, w.b, w.R, w.omega)
    rv, rl = L.coexistence(w.a, w.b, w.R, w.omega, w.Ts_over_Tc * Tc)
    p = L.Params(nx=w.nx, ny=w.ny, precision=L.FP32 if store == "f32" else L.FP64, liquid_rows=w.liquid_rows,
                 a=w.a, b=w.b, R=w.R, omega=w.omega, Ts_over_Tc=w.Ts_over_Tc, sigma=w.sigma, g=w.g,
                 Gw_bottom=w.Gw_bottom, rho_L=rl, rho_V=rv)
    d = L.Domain(p, T_bottom=w.heater_T(Tc), rho0=w.density(rl, rv))
    cells = w.nx * w.ny
    tune = None
    if args.tiles:
        d.set_tiles(*(int(x) for x in args.tiles.split(",")))
    elif args.tune_steps > 0:
        tune = d.autotune(args.tune_steps)
    shapes_lb, shapes_th = L.tile_shapes()
    tiles = {"lb": list(shapes_lb[d.tiles[0]]), "thermal": list(shapes_th[d.tiles[1]]),
             "autotuned": tune is not None}
    print(f"[bench] {w.name}: {w.nx}x{w.ny} {store} storage, tiles {tiles}, warmup {args.warmup}, "
          f"timed {args.steps}", file=sys.stderr, flush=True)

    d.step(args.warmup)
    stream = torch.cuda.ExternalStream(d.stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    d.step_async(args.steps)
    e1.record(stream)
    d.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    mlups = cells * args.steps / (ms / 1e3) / 1e6
    hf = d.heat_flux(local=False)
    print(f"[bench] timed {args.steps} steps: {ms:.2f} ms (host wall {wall * 1e3:.1f} ms), {mlups:.1f} MLUPS, "
          f"q_mean {hf['q_mean']:.6e}", file=sys.stderr, flush=True)
    if args.profile:
        print(json.dumps({"metric": "MLUPS", "value": round(mlups, 2), "ms_per_step": ms_step}))
        return

    ms_lb, ms_th, ms_seq = d.time_kernels(args.kernel_steps)
    step_bytes = ALG_BYTES_STEP[store] * cells
    achieved = step_bytes / (ms_step * 1e-3) / 1e9
    tr_lb = measured_traffic("k_lb", w.name, tiles["lb"])
    tr_th = measured_traffic("k_thermal", w.name, tiles["thermal"])
    traffic = None if tr_lb is None or tr_th is None else tr_lb + tr_th
    sweep = sweep_bench(args.sweep_steps) if args.sweep_steps > 0 else None
    if sweep:
        print(f"[bench] sweep: batched {sweep['batched_mlups']} MLUPS vs sequential {sweep['plain_sequential_mlups']} "
              f"MLUPS ({sweep['speedup']}x)", file=sys.stderr, flush=True)
    adj = None if args.no_adjoint else adjoint_bench()
    badj = None if args.no_adjoint else batch_adjoint_bench()
    if adj:
        print(f"[bench] adjoint/forward: f64 {adj['f64']['ratio']}x, f32 {adj['f32']['ratio']}x; "
              f"batch of {badj['instances']}: {badj['ratio']}x", file=sys.stderr, flush=True)
    three = three_d_bench(args.three_d_steps) if args.three_d_steps > 0 else None
    if three:
        print(f"[bench] 3-D pool {three['workload']}: {three['mlups']} MLUPS, {three['ms_per_step']} ms/step, "
              f"{three['roofline']['frac']} of HBM peak", file=sys.stderr, flush=True)
    cpu = cpu_baseline(w, args.cpu_steps) if args.cpu_steps > 0 else None
    copy_gbs = copy_bandwidth()

    line = {
        "metric": "MLUPS of coupled LB+thermal step, % HBM peak; batched vs plain; adjoint/fwd",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": arithmetic(store),
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "storage": store, "global_batch": 1,
                   "parallelism": "none", "launches_per_step": 2, "graph_steps": 32, "tiles": tiles},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per step",
                     "traffic_gbs": None if traffic is None else round(traffic / (ms_step * 1e-3) / 1e9, 1),
                     "kernel": "step (k_lb + k_thermal)", "step_ms": round(ms_step, 6),
                     "alg_bytes_per_update": ALG_BYTES_STEP[store],
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "kernel_rooflines": {
            "k_lb": _kernel_roofline(ALG_BYTES_LB[store] * cells, ms_lb, tr_lb, ALG_BYTES_LB[store]),
            "k_thermal": _kernel_roofline(ALG_BYTES_TH[store] * cells, ms_th, tr_th, ALG_BYTES_TH[store]),
        },
        "kernels_ms": {"k_lb": round(ms_lb, 6), "k_thermal": round(ms_th, 6), "step_single_launch": round(ms_seq, 6)},
        "heat_flux_mean": hf["q_mean"],
        "batched_sweep": sweep,
        "adjoint": adj,
        "batch_adjoint": badj,
        "three_d": three,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
