#!/usr/bin/env python3
"""Throughput of the two-phase LBGK step on one MI355X: D3Q27, 256^3 static drop.

Workload (synthetic, shaped like the paper's 3D drop tests): Peng-Robinson EOS,
acentric factor 0.344, T/Tc = 0.6 (liquid/vapour density ratio 853), b = 2/21,
kappa~ = 0.02 and a chosen so that the flat equilibrium interface is 5 nodes wide,
drop radius 50 at the centre with a tanh profile of width 5 between the Maxwell
densities, multiplicative density noise 1e-5 (seed 1003), tau = 0.8, periodic.

Timed: K steps of lbm_step with the state resident in HBM, bracketed by device
synchronisation. One JSON line on stdout. The FP32 leg stores populations as
FP32 deviations from w_i rho_v; the FP64 leg is reported alongside, with the
maximum relative density difference between the two after the same steps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor peak
B21 = 2.0 / 21.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(P, n, precision, check_every=-1):
    """Params and initial fields of the static-drop workload at n^3."""
    base = P.Params(P.LBM_D3Q27, n, n, n, P.LBM_EOS_PR, 2.0 / 49.0, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
    k_ref = P.lbm_kappa_for_width(base, 5.0)          # kappa(W=5) scales linearly with a
    a = base.a * 0.02 / k_ref
    p = P.Params(P.LBM_D3Q27, n, n, n, P.LBM_EOS_PR, a, B21, 1.0, 0.344, 0.6, 0.02, 0.8,
                 precision=precision, check_every=check_every)
    rv, rl, _, _ = P.lbm_coexistence(p)
    p.rho_ref = rv if precision == P.LBM_FP32_DEV else 0.0
    import lbm_inputs as L
    radius = 50.0 * n / 256.0
    rho0 = L.drop(n, n, n, radius, rl, rv, 5.0, noise=1e-5, seed=1003)
    return p, rho0, (rv, rl, a)


def time_leg(P, torch, n, precision, steps, warmup):
    p, rho0, (rv, rl, a) = workload(P, n, precision)
    sim = P.Simulation(p)
    sim.init(rho0)
    stream = torch.cuda.current_stream()
    P.lbm_set_stream(sim.ctx, stream.cuda_stream)
    P.lbm_step(sim.ctx, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-kernel device time from HIP events on the same stream
    kt = max(5, min(steps, 20))
    ms, nl = P.lbm_step_timed(sim.ctx, kt)
    N = n ** 3
    s = 4 if precision == P.LBM_FP32_DEV else 8
    Q, D = 27, 3
    res = {
        "mlups": N * steps / dt / 1e6,
        "ms_per_step": dt * 1e3 / steps,
        "kernel_ms": {"moments": ms[0] / nl[0], "collide": ms[1] / nl[1]},
        "bytes_min_per_lup": 2 * Q * s,
        "bytes_collide_per_lup": (2 * Q + D + 1) * s,
        "steps_total": warmup + steps + kt,
    }
    return sim, res, (rv, rl, a)


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload (48^3, same physics)."""
    from oracle import oracle as O
    from oracle import thermo as T
    import lbm_inputs as L
    n = 48
    fl0 = T.Fluid(T.PR, 2.0 / 49.0, B21, 0.6, 1.0, 0.344)
    a = fl0.a * 0.02 / T.kappa_for_width(fl0, 5.0)
    fl = T.Fluid(T.PR, a, B21, 0.6, 1.0, 0.344)
    rv, rl, _ = T.coexistence(fl)
    cfg = O.Config(3, n, n, n, T.PR, a, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
    orc = O.Oracle(cfg).init(L.drop(n, n, n, 50.0 * n / 256, rl, rv, 5.0, noise=1e-5, seed=1003))
    orc.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        orc.step(2)
        steps += 2
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"D3Q27 {n}^3 drop (same EOS, T/Tc, kappa, tau; radius scaled), {steps} FP64 steps, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: the step runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2112_01975_amd as P
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    n = args.size
    N = n ** 3
    log(f"[bench] FP32-dev leg {n}^3 warmup={args.warmup} steps={args.steps}")
    sim32, r32, (rv, rl, a) = time_leg(P, torch, n, P.LBM_FP32_DEV, args.steps, args.warmup)
    log(f"[bench] FP32-dev {r32['mlups']:.0f} MLUPS, kernels {r32['kernel_ms']}")
    fp64 = None
    dens_err = None
    if not args.no_fp64:
        log("[bench] FP64 leg")
        sim64, r64, _ = time_leg(P, torch, n, P.LBM_FP64, args.steps, args.warmup)
        log(f"[bench] FP64 {r64['mlups']:.0f} MLUPS, kernels {r64['kernel_ms']}")
        rho32, _, t32 = sim32.moments()
        rho64, _, t64 = sim64.moments()
        dens_err = float(np.max(np.abs(rho32 - rho64) / rho64))
        t_c = r64["kernel_ms"]["collide"] * 1e-3
        fp64 = {"value": r64["mlups"], "unit": "MLUPS", "ms_per_step": r64["ms_per_step"],
                "roofline": {"bound": "hbm", "achieved": N * r64["bytes_collide_per_lup"] / t_c / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s"},
                "useful_frac_step": r64["mlups"] * 1e6 * r64["bytes_min_per_lup"] / (HBM_PEAK_GBS * 1e9),
                "mass_rel_diff_vs_fp32": abs(t32[0] - t64[0]) / t64[0]}
        fp64["roofline"]["frac"] = fp64["roofline"]["achieved"] / HBM_PEAK_GBS
        sim64.close()
    sim32.close()
    t_c = r32["kernel_ms"]["collide"] * 1e-3
    achieved = N * r32["bytes_collide_per_lup"] / t_c / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline()
    out = {
        "metric": "MLUPS and % of HBM roofline, FP32 vs FP64 at stated density error, D3Q27 256³",
        "value": r32["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"D3Q27 {n}^3 periodic static drop R={50 * n // 256}, Peng-Robinson "
                               f"omega'=0.344 T/Tc=0.6 (rho_l/rho_v={rl / rv:.0f}), kappa=0.02, a={a:.6g}, "
                               f"b=2/21, W=5, tau=0.8, FP32 deviation storage rho_ref=rho_v",
                   "nodes": N, "lattice": "D3Q27", "precision": "fp32-dev"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "collide-stream pass",
                     "bytes_per_lup": r32["bytes_collide_per_lup"]},
        "useful_frac_step": r32["mlups"] * 1e6 * r32["bytes_min_per_lup"] / (HBM_PEAK_GBS * 1e9),
        "kernel_ms": r32["kernel_ms"],
        "fp64": fp64,
        "density_error_fp32_vs_fp64": dens_err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
