#!/usr/bin/env python3
"""Throughput of the two-phase LBGK step on one MI355X: D3Q27, 256^3 static drop.

Workload (synthetic, shaped like the paper's 3D drop tests): Peng-Robinson EOS,
acentric factor 0.344, T/Tc = 0.6 (liquid/vapour density ratio 853), b = 2/21,
kappa~ = 0.02 with `a` chosen so that the flat equilibrium interface is 5 nodes
wide, drop radius 50 at the centre with a tanh profile of width 5 between the
Maxwell densities, multiplicative density noise 1e-5 (seed 1003), at rest,
tau = 0.8, periodic.

Timed: K steps of lbm_step with the state resident in HBM, bracketed by device
synchronisation; one JSON line on stdout. The headline leg stores populations
as FP32 deviations from w_i rho_v (single-pass z-march kernel); the FP64 leg runs
the same workload and the line states the density difference between the two
after the same number of steps. `roofline` is for the dominant kernel: algorithmic
bytes per launch (27 populations read and written, 4 B each, per node) over its
average launch time from HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor peak
B21 = 2.0 / 21.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused3_d3q27_256_fp32_traffic.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(P, n, precision, check_every=-1, box=None):
    """Params and initial density of the static-drop workload at n^3 (or at box = (nx, ny,
    nz), the drop radius scaled with the smallest side)."""
    nx, ny, nz = box or (n, n, n)
    base = P.Params(P.LBM_D3Q27, nx, ny, nz, P.LBM_EOS_PR, 2.0 / 49.0, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
    a = base.a * 0.02 / P.lbm_kappa_for_width(base, 5.0)   # kappa(W) is linear in a at fixed b, T/Tc
    p = P.Params(P.LBM_D3Q27, nx, ny, nz, P.LBM_EOS_PR, a, B21, 1.0, 0.344, 0.6, 0.02, 0.8,
                 precision=precision, check_every=check_every)
    rv, rl, _, _ = P.lbm_coexistence(p)
    p.rho_ref = rv if precision == P.LBM_FP32_DEV else 0.0
    import lbm_inputs as L
    rho0 = L.drop(nx, ny, nz, 50.0 * min(nx, ny, nz) / 256.0, rl, rv, 5.0, noise=1e-5, seed=1003)
    return p, rho0, (rv, rl, a)


def density_error(rho32, rho64, n):
    """FP32 against FP64 density of the n^3 drop: largest pointwise relative difference, and
    the relative differences of the mean densities of a 4^3 block at the liquid centre and
    at the vapour corner."""
    c = n // 2
    a, b = rho32.reshape(n, n, n), rho64.reshape(n, n, n)
    centre = (slice(c - 2, c + 2),) * 3
    corner = (slice(0, 4),) * 3
    return {"max_pointwise_rel": float(np.max(np.abs(rho32 - rho64) / rho64)),
            "liquid_centre_rel": float(abs(a[centre].mean() / b[centre].mean() - 1)),
            "vapour_corner_rel": float(abs(a[corner].mean() / b[corner].mean() - 1))}


def size_sweep(P, torch, boxes, steps=10, warmup=3):
    """The FP32 drop's fused step at other lattice sizes: ms per step from HIP events
    (lbm_step_timed) and GLUPS; ends with the copy probe so that counter runs of this leg
    carry their own scale."""
    out = {}
    for box in boxes:
        p, rho0, _ = workload(P, 0, P.LBM_FP32_DEV, box=box)
        with P.Simulation(p) as sim:
            sim.init(rho0)
            del rho0
            P.lbm_step(sim.ctx, warmup)
            ms, nl = P.lbm_step_timed(sim.ctx, steps)
            _, _, tot = sim.moments(want_fields=False)
        name = "x".join(str(v) for v in box)
        out[name] = {"ms_per_step": round(ms[1] / steps, 4), "GLUPS": round(p.N * steps / ms[1] / 1e6, 2),
                     "fused": bool(nl[0] == 0), "finite": bool(np.isfinite(tot).all())}
        log(f"[bench] size {name}: {out[name]}")
    out["copy_probe_GBs"] = round(copy_probe(P, torch)["GBs"], 1)
    return out


def time_leg(P, torch, n, precision, steps, warmup, check_every=1000):
    """Time `steps` steps of lbm_step with the FP64 watchdog every `check_every` steps (and at
    the end of the call); then the per-launch kernel time from HIP events, and the cost of one
    watchdog check: K calls of one step (each ending in a check) against one call of K steps."""
    p, rho0, meta = workload(P, n, precision, check_every)
    sim = P.Simulation(p)
    sim.init(rho0)
    _, _, tot0 = sim.moments(want_fields=False)
    P.lbm_set_stream(sim.ctx, torch.cuda.current_stream().cuda_stream)
    P.lbm_step(sim.ctx, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = max(5, min(steps, 20))
    ms, nl = P.lbm_step_timed(sim.ctx, kt)   # HIP events around every launch
    kern = {"moment_pass": ms[0] / nl[0] if nl[0] else 0.0, "step_kernel": ms[1] / nl[1]}
    K = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.lbm_step(sim.ctx, K)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(K):
        P.lbm_step(sim.ctx, 1)
    torch.cuda.synchronize()
    t_each = time.perf_counter() - t0
    check_ms = max(0.0, (t_each - t_one) / (K - 1)) * 1e3
    return sim, {"mlups": n ** 3 * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps, "kernel_ms": kern,
                 "fused": nl[0] == 0, "steps_total": warmup + steps + kt + 2 * K, "mass0": tot0[0],
                 "check_ms": check_ms, "check_every": check_every}, meta


def copy_probe(P, torch, nbytes=1 << 32, reps=5):
    """Attainable copy bandwidth: the library's hand-written streaming copy (16-byte accesses,
    non-temporal loads and stores, the fastest of a few launch shapes) over two 4 GiB device
    buffers; also the counter scale of the traffic profiles."""
    x = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    gbs, ms, shape = P.lbm_copy_probe(y.data_ptr(), x.data_ptr(), nbytes, reps,
                                      torch.cuda.current_stream().cuda_stream)
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "GBs": gbs, "ms": ms,
            "shape": f"{shape // 100000} x 16 B in flight per lane, {shape % 100000} workgroups"}


def traffic_from_profile():
    """HBM bytes per launch of the fused kernel from the committed counter summary, if it
    was taken on the current kernel sources; otherwise None."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    from paper_2112_01975_amd import profsum
    d = profsum.read_traffic(TRAFFIC_SUMMARY)
    if d.get("source_fingerprint") != profsum.source_fingerprint():
        return None
    return float(d["traffic_bytes_per_launch"])


def batch_sweep(P, torch, steps):
    """64 D2Q9 flat-interface cases, 4 x L with L log-spaced 128..2048 increasing with T/Tc in
    0.55..0.99 (vdW, kappa 0.02, a set for W = 4 at T/Tc = 0.55, tau 0.8; FP32 below T/Tc = 0.95,
    FP64 above): the batch (a HIP graph per chunk of steps; its layout, e.g. tiles of several
    steps per launch, chosen by the library's tuner) against the same cases stepped one by one
    through lbm_step."""
    import lbm_inputs as L
    base = P.Params(P.LBM_D2Q9, 8, 4, 1, P.LBM_EOS_VDW, 9 / 49, B21, 1.0, 0.0, 0.55, 0.02, 0.8)
    a = base.a * 0.02 / P.lbm_kappa_for_width(base, 4.0)
    cases, inits = [], []
    for sc in L.temperature_sweep(64, 0.55, 0.99, 128, 2048, 4):
        prec = P.LBM_FP64 if sc.fp64 else P.LBM_FP32_DEV
        p = P.Params(P.LBM_D2Q9, sc.nx, sc.ny, 1, P.LBM_EOS_VDW, a, B21, 1.0, 0.0, sc.T_reduced, 0.02, 0.8,
                     precision=prec, check_every=0)
        rv, rl, _, _ = P.lbm_coexistence(p)
        p.rho_ref = rv if prec == P.LBM_FP32_DEV else 0.0
        W = max(4.0, 4.0 * (P.lbm_kappa_for_width(p, 4.0) / 0.02) ** -0.5)
        cases.append(p)
        inits.append(L.flat_slab(sc.nx, sc.ny, 1, rl, rv, W, noise=1e-4, seed=3000 + sc.index))
    nodes = sum(c.N for c in cases)
    b = P.lbm_batch_create(cases)
    for i, r in enumerate(inits):
        P.lbm_batch_init_fields(b, i, r)
    P.lbm_batch_step(b, 20)                       # autotune + graph capture + warm-up
    layout = P.lbm_batch_layout(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.lbm_batch_step(b, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    P.lbm_batch_destroy(b)
    t_seq = 0.0
    for p, r in zip(cases, inits):
        with P.Simulation(p) as s:
            s.init(r).step(10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(steps)
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - t0
    return {"cases": len(cases), "nodes": nodes, "steps": steps, "batched_s": t_batch, "one_by_one_s": t_seq,
            "speedup": t_seq / t_batch, "batched_MLUPS": nodes * steps / t_batch / 1e6, "layout": layout,
            "one_by_one_MLUPS": nodes * steps / t_seq / 1e6,
            "fp64_cases": sum(1 for c in cases if c.precision == P.LBM_FP64)}


def timed_mlups(P, torch, p, rho0, U0, steps, warmup):
    """MLUPS of lbm_step on one workload (state resident in HBM, synchronised both sides)."""
    with P.Simulation(p) as sim:
        sim.init(rho0, U0)
        P.lbm_set_stream(sim.ctx, torch.cuda.current_stream().cuda_stream)
        P.lbm_step(sim.ctx, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.lbm_step(sim.ctx, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, _, tot = sim.moments(want_fields=False)
    return p.N * steps / dt / 1e6, bool(np.isfinite(tot).all())


def d2q9_drop_leg(P, torch, steps=1000, n=512):
    """D2Q9 n^2 static drop R = 60 n / 512 (van der Waals T/Tc = 0.8, kappa 0.02, a for W = 4,
    tau 0.8), MLUPS in both storage precisions. At the workload's 512^2 the whole lattice fits
    in the MALL, so only MLUPS are meaningful; larger n stream from HBM."""
    import lbm_inputs as L
    base = P.Params(P.LBM_D2Q9, 8, 4, 1, P.LBM_EOS_VDW, 9 / 49, B21, 1.0, 0.0, 0.8, 0.02, 0.8)
    a2 = base.a * 0.02 / P.lbm_kappa_for_width(base, 4.0)
    d2 = {}
    for prec, name in ((P.LBM_FP32_DEV, "fp32"), (P.LBM_FP64, "fp64")):
        p = P.Params(P.LBM_D2Q9, n, n, 1, P.LBM_EOS_VDW, a2, B21, 1.0, 0.0, 0.8, 0.02, 0.8, precision=prec,
                     check_every=-1)
        rv, rl, _, _ = P.lbm_coexistence(p)
        p.rho_ref = rv if prec == P.LBM_FP32_DEV else 0.0
        rho0 = L.drop(n, n, 1, 60.0 * n / 512, rl, rv, 4.0, noise=1e-4, seed=1003)
        d2[name], ok = timed_mlups(P, torch, p, rho0, None, steps, 50)
        d2[name + "_finite"] = ok
    return {"unit": "MLUPS", "steps": steps, **d2}


def other_workloads(P, torch):
    """The other full-size workloads of the path, MLUPS in both storage precisions:
    - the D2Q9 512^2 static drop (d2q9_drop_leg);
    - D3Q27 512 x 256 x 256 drop impact on a textured wall (floor plus 8 x 8 pillars of
      height 16 every 16 nodes; Peng-Robinson T/Tc = 0.6, a for W = 5, kappa 0.02;
      nu_vapour = 15 nu_liquid with tau_liquid = 0.55 (and 0.51, FP32); wall density = vapour density;
      drop R = 40 at (256, 128, 77) moving at -0.05 along z): MLUPS over all nodes and
      MFLUPS over fluid nodes."""
    import lbm_inputs as L
    out = {"d2q9_512x512_drop": d2q9_drop_leg(P, torch)}
    nx, ny, nz = 512, 256, 256
    base = P.Params(P.LBM_D3Q27, 8, 8, 8, P.LBM_EOS_PR, 2.0 / 49.0, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
    a3 = base.a * 0.02 / P.lbm_kappa_for_width(base, 5.0)
    mask = L.pillar_mask(nx, ny, nz, 8, 8, 16)
    fluid = int((mask == 0).sum())
    d3 = {}
    for prec, name, tau in ((P.LBM_FP32_DEV, "fp32", 0.55), (P.LBM_FP64, "fp64", 0.55),
                            (P.LBM_FP32_DEV, "fp32_tau_liquid_0.51", 0.51)):
        p = P.Params(P.LBM_D3Q27, nx, ny, nz, P.LBM_EOS_PR, a3, B21, 1.0, 0.344, 0.6, 0.02, tau,
                     tau_vapour=0.5 + 15 * (tau - 0.5), mask=mask, precision=prec, check_every=-1)
        rv, rl, _, _ = P.lbm_coexistence(p)
        p.rho_liquid, p.rho_vapour, p.rho_wall = rl, rv, rv
        p.rho_ref = rv if prec == P.LBM_FP32_DEV else 0.0
        if name == "fp32":
            rho0 = L.drop(nx, ny, nz, 40.0, rl, rv, 5.0, centre=(256.0, 128.0, 77.0), noise=1e-5, seed=1005)
            rho0 = np.where(mask.astype(bool), rv, rho0)
            U0 = L.impact_drop_velocity(rho0, rl, rv, 3, -0.05, 2)
        mlups, ok = timed_mlups(P, torch, p, rho0, U0, 50, 5)
        d3[name] = {"MLUPS": mlups, "MFLUPS": mlups * fluid / p.N, "finite": ok}
    out["d3q27_512x256x256_impact"] = {"steps": 50, "fluid_nodes": fluid, "nodes": nx * ny * nz, **d3}
    out["d3q27_256_tapered_posts"] = tapered_posts_workload(P, torch, a3)
    return out


def tapered_posts_workload(P, torch, a3, d0=64):
    """Drop impact on tapered posts with curved walls: a 4 D0 box (256^3 at D0 = 64), solid
    floor 2 nodes thick, 8 x 8 cone-frustum posts every D0/2 (base radius 0.15 D0, tip
    0.05 D0, height D0/2), a drop of diameter D0 whose lowest point is 10 nodes above the
    post tops, moving at -0.05 along z; Peng-Robinson T/Tc = 0.6 as the impact workload,
    wall density = vapour density. Interpolated bounce-back with the exact cut fraction of
    every wall link (two-pass step), FP32 and FP64; the same geometry with halfway
    bounce-back (fused step) for comparison."""
    import lbm_inputs as L
    n = 4 * d0
    t0 = time.perf_counter()
    mask, lq_cube = L.tapered_posts(n, n, n, 2, 0.15 * d0, 0.05 * d0, 0.5 * d0, d0 // 2)
    t_geom = time.perf_counter() - t0
    cl = P.lbm_velocities(P.LBM_D3Q27)
    link_q = np.stack([lq_cube[int(c[0]) + 1, int(c[1]) + 1, int(c[2]) + 1] for c in cl])
    del lq_cube
    fluid = int((mask == 0).sum())
    wall_links = int((link_q > 0).sum())
    top = 1.5 + 0.5 * d0
    res = {"nodes": n ** 3, "fluid_nodes": fluid, "wall_links": wall_links, "steps": 50,
           "geometry_s": t_geom}
    rho0 = U0 = None
    for prec, name, lq in ((P.LBM_FP32_DEV, "fp32", link_q), (P.LBM_FP64, "fp64", link_q),
                           (P.LBM_FP32_DEV, "fp32_halfway", None)):
        p = P.Params(P.LBM_D3Q27, n, n, n, P.LBM_EOS_PR, a3, B21, 1.0, 0.344, 0.6, 0.02, 0.55,
                     tau_vapour=0.5 + 15 * 0.05, mask=mask, precision=prec, check_every=-1, link_q=lq)
        rv, rl, _, _ = P.lbm_coexistence(p)
        p.rho_liquid, p.rho_vapour, p.rho_wall = rl, rv, rv
        p.rho_ref = rv if prec == P.LBM_FP32_DEV else 0.0
        if rho0 is None:
            rho0 = L.drop(n, n, n, 0.5 * d0, rl, rv, 5.0, centre=(n / 2, n / 2, top + 10.0 + 0.5 * d0),
                          noise=1e-5, seed=1007)
            rho0 = np.where(mask.astype(bool), rv, rho0)
            U0 = L.impact_drop_velocity(rho0, rl, rv, 3, -0.05, 2)
        mlups, ok = timed_mlups(P, torch, p, rho0, U0, 50, 5)
        res[name] = {"MLUPS": mlups, "MFLUPS": mlups * fluid / p.N, "finite": ok}
    return res


def pressure_tensor_leg(P, torch, n, reps=3):
    """The discrete pressure tensor (Appendix E) of the drop workload after 20 steps, FP32 and
    FP64: wall time per lbm_pressure_tensor call (moment pass, tensor kernel, and the copy of
    6 FP64 components per node to the host)."""
    out = {}
    for prec, name in ((P.LBM_FP32_DEV, "fp32"), (P.LBM_FP64, "fp64")):
        p, rho0, _ = workload(P, n, prec)
        with P.Simulation(p) as s:
            s.init(rho0)
            s.step(20)
            P.lbm_pressure_tensor(s.ctx, n ** 3, P.LBM_D3Q27)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Pt = P.lbm_pressure_tensor(s.ctx, n ** 3, P.LBM_D3Q27)
            dt = (time.perf_counter() - t0) / reps
            c = n // 2
            centre = Pt[:, c + n * (c + n * c)]
        out[name] = {"call_s": dt, "centre_xx_yy_zz": [float(v) for v in centre[:3]],
                     "finite": bool(np.isfinite(Pt).all())}
    return out


def cpu_baseline(n=256, budget_s=15.0):
    """The FP64 oracle on the headline workload itself (n^3 drop, same physics): a bounded
    sample of whole oracle steps after one untimed step, timed on the host's cores."""
    from oracle import oracle as O
    from oracle import thermo as T
    import lbm_inputs as L
    fl0 = T.Fluid(T.PR, 2.0 / 49.0, B21, 0.6, 1.0, 0.344)
    a = fl0.a * 0.02 / T.kappa_for_width(fl0, 5.0)
    fl = T.Fluid(T.PR, a, B21, 0.6, 1.0, 0.344)
    rv, rl, _ = T.coexistence(fl)
    cfg = O.Config(3, n, n, n, T.PR, a, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
    orc = O.Oracle(cfg).init(L.drop(n, n, n, 50.0 * n / 256, rl, rv, 5.0, noise=1e-5, seed=1003))
    orc.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        orc.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    orc.close()
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"the D3Q27 {n}^3 drop workload itself (same EOS, T/Tc, kappa, tau, radius "
                      f"{50.0 * n / 256:g}), {steps} FP64 oracle steps in {dt:.1f} s after one untimed step",
            "host": host_cpu()}


def host_cpu():
    """The host the CPU baseline ran on: CPU model, logical CPUs, and those this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--error-steps", type=int, default=5000,
                    help="steps after which the FP32 state is compared with the FP64 state (untimed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-case batched sweep (with its case-by-case comparison)")
    ap.add_argument("--no-other", action="store_true", help="skip the D2Q9 512^2, drop-impact and posts legs")
    ap.add_argument("--posts-only", action="store_true",
                    help="run only the tapered-posts leg (curved walls) and print its JSON line")
    ap.add_argument("--posts-d0", type=int, default=64,
                    help="post spacing scale D0 of the posts leg; the box is 4 D0 (150: the paper's 600^3)")
    ap.add_argument("--d2q9-only", action="store_true",
                    help="time only the D2Q9 drop (512^2, or --d2q9-size) in both precisions and print its JSON line")
    ap.add_argument("--d2q9-size", type=int, default=512, help="grid side of the --d2q9-only leg")
    ap.add_argument("--pressure-only", action="store_true",
                    help="time only the discrete pressure tensor of the 256^3 drop and print its JSON line")
    ap.add_argument("--sizes-only", default=None, metavar="NXxNYxNZ,...",
                    help="time only the FP32 drop's fused step at these lattice sizes and print their JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: the step runs on one GPU, --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2112_01975_amd as P
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.sizes_only:
        boxes = [tuple(int(v) for v in b.split("x")) for b in args.sizes_only.split(",")]
        print(json.dumps({"fp32_drop_sizes": size_sweep(P, torch, boxes)}), flush=True)
        return
    if args.pressure_only:
        print(json.dumps({"pressure_tensor_256": pressure_tensor_leg(P, torch, args.size)}), flush=True)
        return
    if args.d2q9_only:
        n = args.d2q9_size
        steps = max(20, min(1000, int(1000 * (512 / n) ** 2)))
        # the copy probe first: its kernel is the scale of HBM counters taken on this leg
        print(json.dumps({"attainable_copy": copy_probe(P, torch),
                          f"d2q9_{n}x{n}_drop": d2q9_drop_leg(P, torch, steps, n)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch_sweep": batch_sweep(P, torch, args.batch_steps)}), flush=True)
        return
    if args.posts_only:
        base = P.Params(P.LBM_D3Q27, 8, 8, 8, P.LBM_EOS_PR, 2.0 / 49.0, B21, 1.0, 0.344, 0.6, 0.02, 0.8)
        a3 = base.a * 0.02 / P.lbm_kappa_for_width(base, 5.0)
        d0 = args.posts_d0
        print(json.dumps({f"d3q27_{4 * d0}_tapered_posts": tapered_posts_workload(P, torch, a3, d0)}), flush=True)
        return
    n = args.size
    N = n ** 3
    log(f"[bench] FP32 deviation-storage leg {n}^3 warmup={args.warmup} steps={args.steps}")
    sim32, r32, (rv, rl, a) = time_leg(P, torch, n, P.LBM_FP32_DEV, args.steps, args.warmup)
    log(f"[bench] FP32 {r32['mlups']:.0f} MLUPS, kernels {r32['kernel_ms']}, check {r32['check_ms']:.3f} ms")
    probe = copy_probe(P, torch)
    log(f"[bench] copy probe {probe['GBs']:.0f} GB/s ({probe['shape']})")
    fp64 = None
    dens = None
    _, _, t32_timed = sim32.moments(want_fields=False)
    if not args.no_fp64:
        log("[bench] FP64 leg")
        sim64, r64, _ = time_leg(P, torch, n, P.LBM_FP64, args.steps, args.warmup)
        log(f"[bench] FP64 {r64['mlups']:.0f} MLUPS, kernels {r64['kernel_ms']}, check {r64['check_ms']:.3f} ms")
        _, _, t64_timed = sim64.moments(want_fields=False)
        # the precision comparison at the workload's full length: both states continued to
        # `error_steps` steps in all (untimed)
        total = max(args.error_steps, r32["steps_total"])
        log(f"[bench] FP32 and FP64 continued to {total} steps")
        sim32.step(total - r32["steps_total"])
        sim64.step(total - r64["steps_total"])
        rho32, _, t32 = sim32.moments()
        rho64, _, t64 = sim64.moments()
        dens = {"after_steps": total, "rho_ref": "rho_vapour", **density_error(rho32, rho64, n),
                "mass_rel_drift_fp32": abs(t32[0] / r32["mass0"] - 1),
                "mass_rel_drift_fp64": abs(t64[0] / r64["mass0"] - 1)}
        del rho32
        # the other references the deviation storage could take (liquid density, mean of the two)
        alt = {}
        for name, ref in (("rho_liquid", rl), ("mean", 0.5 * (rl + rv))):
            p_alt, rho0_alt, _ = workload(P, n, P.LBM_FP32_DEV)
            p_alt.rho_ref = ref
            with P.Simulation(p_alt) as s_alt:
                s_alt.init(rho0_alt)
                del rho0_alt
                s_alt.step(total)
                rho_alt, _, _ = s_alt.moments()
            alt[name] = density_error(rho_alt, rho64, n)
            del rho_alt
        dens["other_rho_ref"] = alt
        del rho64
        log(f"[bench] FP32 density error {dens}")
        t_k = r64["kernel_ms"]["step_kernel"] * 1e-3
        b64 = (2 * 27 + 4) * 8 if not r64["fused"] else 2 * 27 * 8
        fp64 = {"value": r64["mlups"], "unit": "MLUPS", "ms_per_step": r64["ms_per_step"],
                "kernel": "collide-stream pass (two-pass step)" if not r64["fused"] else "fused step",
                "kernel_ms": r64["kernel_ms"], "watchdog_check_ms": r64["check_ms"],
                "roofline": {"bound": "hbm", "achieved": N * b64 / t_k / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": N * b64 / t_k / 1e9 / HBM_PEAK_GBS, "bytes_per_lup": b64,
                             "frac_of_attainable_copy": N * b64 / t_k / 1e9 / probe["GBs"]},
                "useful_frac_step": r64["mlups"] * 1e6 * 432 / (HBM_PEAK_GBS * 1e9),
                "mass_rel_drift_timed": abs(t64_timed[0] / r64["mass0"] - 1)}
        sim64.close()
    sim32.close()
    t_k = r32["kernel_ms"]["step_kernel"] * 1e-3
    bytes_lup = 2 * 27 * 4
    achieved = N * bytes_lup / t_k / 1e9
    traffic = traffic_from_profile() if r32["fused"] else None
    batch = None
    if not args.no_batch:
        log("[bench] batched temperature sweep vs one-by-one")
        batch = batch_sweep(P, torch, args.batch_steps)
        log(f"[bench] batch {batch['batched_s']:.3f} s vs one-by-one {batch['one_by_one_s']:.3f} s")
    other = None
    if not args.no_other:
        log("[bench] other workloads (D2Q9 512^2, D3Q27 512x256x256 impact, 256^3 tapered posts)")
        other = other_workloads(P, torch)
        log(f"[bench] other {json.dumps(other)}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline()
    out = {
        "metric": "MLUPS and % of HBM roofline, FP32 vs FP64 at stated density error, D3Q27 256³",
        "value": r32["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"D3Q27 {n}^3 periodic static drop R={50 * n / 256:g} at rest, Peng-Robinson "
                               f"omega'=0.344 T/Tc=0.6 (rho_l/rho_v={rl / rv:.0f}), kappa=0.02, a={a:.6g}, "
                               f"b=2/21, W=5, tau=0.8, FP32 deviation storage (rho_ref=rho_v), FP64 watchdog "
                               f"every {r32['check_every']} steps and at the end of each lbm_step call",
                   "nodes": N, "lattice": "D3Q27", "precision": "fp32-deviation", "kernel": "fused z-march"
                   if r32["fused"] else "two-pass"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fused3 (single-pass step)" if r32["fused"] else "collide-stream pass",
                     "bytes_per_lup": bytes_lup, "launch_ms": r32["kernel_ms"]["step_kernel"],
                     # the counted HBM bytes over the same launch time (null without a current profile)
                     "traffic_GBs": (traffic / (r32["kernel_ms"]["step_kernel"] * 1e-3) / 1e9
                                     if traffic else None),
                     "traffic_frac": (traffic / (r32["kernel_ms"]["step_kernel"] * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None)},
        "useful_frac_step": r32["mlups"] * 1e6 * bytes_lup / (HBM_PEAK_GBS * 1e9),
        "attainable_copy_GBs": probe["GBs"],
        "attainable_copy": probe,
        "frac_of_attainable_copy": achieved / probe["GBs"],
        "watchdog": {"check_every": r32["check_every"], "check_ms": r32["check_ms"],
                     "check_frac_of_step": r32["check_ms"] / r32["ms_per_step"]},
        "mass_rel_drift_fp32": abs(t32_timed[0] / r32["mass0"] - 1),
        "density_error_fp32_vs_fp64": dens,
        "fp64": fp64,
        "batch_sweep": batch,
        "other_workloads": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
