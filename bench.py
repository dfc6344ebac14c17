#!/usr/bin/env python3
"""Benchmark of the DG SSP-RK3 step on one MI355X.

A step is one pass of the whole hot path over the state: CFL time step (FP64
reduction), driving-mode update when due (host Ornstein-Uhlenbeck + table upload),
and one SSP-RK3 step (projection, three right-hand sides with viscosity, driving and
Rusanov faces, three stage combinations with the positivity limiter).  The metric is
DG degree-of-freedom updates per second per Runge-Kutta stage: 3 * 4 * nb * N^3 per
step divided by the wall time of the timed steps.

Default workload: 64^3 cells, degree 2 (10 modes per variable, 27 Gauss points),
FP64, artificial viscosity + primitive projection + positivity limiter, mean-free
solenoidal OU driving on 1 <= |n| <= 2 aimed at RMS Mach ~3 (t_c = T = 1/(2 Mach)).
The input state is a seeded synthetic turbulence-like modal field (log-normal density,
RMS velocity 3), resident in HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c4|c5]
                       [--precision fp64|fp32] [--no-compare] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG DOF-updates/sec per RK stage (3D, order p) + % HBM/MFMA roofline vs FP64"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector = matrix FP64 peak
PEAK_FP32_VALU_TFLOPS = 78.6  # unpacked FP32 vector rate (packed FP32 is disabled in this build)

WORKLOADS = {
    # name: (N, degree, default precision, target Mach, driving sigma)
    "c2": (64, 2, "fp64", 3.0, 3.0),
    "c3": (128, 3, "fp32", 10.0, 25.0),
    "c4": (128, 2, "fp32", 10.0, 25.0),
    "c5": (256, 2, "fp32", 10.0, 25.0),
}


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_06841_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload, precision, launches_unit):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def run_gpu(args, precision, measure_profile=True):
    import numpy as np
    import torch

    import synthetic
    from paper_2401_06841_amd import dg, model

    N, k, _, mach, sigma = WORKLOADS[args.workload]
    prec = dg.DG_FP64 if precision == "fp64" else dg.DG_FP32
    flags = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER | dg.DG_FORCING | dg.DG_FORCE_MEANFREE
    cfg = dg.Config(N, N, N, degree=k, precision=prec, flags=flags)
    ctx = dg.dg_init(cfg)
    u0 = synthetic.turbulent_like(N, N, N, k, mach=mach, seed=args.seed)
    u = torch.as_tensor(u0, device="cuda").to(ctx.dtype).contiguous()
    del u0
    assert dg.dg_limit(ctx, u) == 0
    t_c = 1.0 / (2.0 * mach)           # eddy turnover time T = L/(2 cs Mach), t_c = T
    dt_drive = t_c / 100.0
    dg.dg_forcing_ou_init(ctx, t_c, sigma)
    nd = dg.dg_forcing_ou_ndraws()
    dg.dg_forcing_ou_advance(ctx, synthetic.gaussian_draws(args.seed, 0, nd), 1e30)   # stationary start
    state = {"t": 0.0, "next": dt_drive, "n_drive": 1, "retries": 0, "dt_ms": 0.0, "dt0": None, "dtmin": 1e300}

    def step():
        t0 = time.perf_counter()
        dt = dg.dg_dt_max(ctx, u)
        state["dt_ms"] += 1e3 * (time.perf_counter() - t0)
        if state["dt0"] is None:
            state["dt0"] = dt
        state["dtmin"] = min(state["dtmin"], dt)
        if not (dt > 1e-3 * state["dt0"]):
            raise RuntimeError(f"time step collapsed ({dt:.3e} vs {state['dt0']:.3e} at the start): "
                               "the flow state is not physical")
        while state["t"] + dt >= state["next"]:
            dg.dg_forcing_ou_advance(ctx, synthetic.gaussian_draws(args.seed, state["n_drive"], nd), dt_drive)
            state["n_drive"] += 1
            state["next"] += dt_drive
        while dg.dg_rk_step(ctx, u, dt) == dg.DG_RETRY:
            state["retries"] += 1
            dt *= 0.5
        state["t"] += dt

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    state["dt_ms"] = 0.0
    state["retries"] = 0
    if measure_profile:
        dg.dg_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = dg.dg_profile_read(ctx) if measure_profile else None
    dg.dg_profile(ctx, False)

    dof = 4 * cfg.nb * cfg.ncell
    value = 3.0 * dof * args.steps / wall
    out = {"precision": precision, "value": value, "wall_s": wall, "ms_per_step": 1e3 * wall / args.steps,
           "dt_reduction_ms_per_step": state["dt_ms"] / args.steps, "retries": state["retries"],
           "sim_time": state["t"], "drive_updates": state["n_drive"], "dt_first": state["dt0"],
           "dt_min": state["dtmin"]}
    # RMS Mach number of the cell means (diagnostic of the synthetic state)
    rho = u[0, 0].double()
    v2 = ((u[1:, 0].double() / rho) ** 2).sum(0)
    out["rms_mach_cell_means"] = float(torch.sqrt(v2.mean()))
    if prof:
        rhs_ms, rhs_n, st_ms, st_n = prof
        avg = rhs_ms / max(rhs_n, 1)
        flops = model.rhs_flops_per_cell(k, av=True, proj=True, forcing=True) * cfg.ncell
        achieved = flops / (avg * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_VALU_TFLOPS
        out["kernels"] = {"k_rhs_avg_ms": avg, "k_rhs_launches": rhs_n,
                          "k_stage_avg_ms": st_ms / max(st_n, 1), "k_stage_launches": st_n,
                          "k_rhs_share_of_step": rhs_ms / (1e3 * wall)}
        out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                           "frac": achieved / peak,
                           "traffic": traffic_from_profiles("k_rhs", args.workload, precision, 1)}
        out["algorithmic_flops_per_launch"] = flops
    ctx.close()
    return out


def run_cpu_baseline(args):
    """The oracle as it stands, timed on the host cores on a bounded sample: 3 SSP-RK3
    steps (9 stages) of the same workload from the same synthetic input."""
    import numpy as np

    import oracle
    import synthetic

    N, k, _, mach, sigma = WORKLOADS[args.workload]
    flags = oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER | oracle.FORCING | oracle.FORCE_MEANFREE
    cfg = oracle.Cfg(N, N, N, k, flags=flags)
    u = synthetic.turbulent_like(N, N, N, k, mach=mach, seed=args.seed)
    modes = synthetic.forcing_table(args.seed, amp=sigma)
    nsteps = args.cpu_steps
    t0 = time.perf_counter()
    for _ in range(nsteps):
        dt = oracle.dt_max(cfg, u)
        u, st = oracle.rk_step(cfg, u, dt, modes)
    wall = time.perf_counter() - t0
    dof = 4 * cfg.nb * cfg.ncell
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 3.0 * dof * nsteps / wall, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{nsteps} SSP-RK3 steps ({3 * nsteps} stages) of the {N}^3 degree-{k} workload, "
                      f"FP64 C oracle with OpenMP over cells, {wall:.1f} s"}


def copy_calibration():
    """A plain device copy of known size (512 MiB read + 512 MiB written per launch), used
    to scale the FETCH_SIZE / WRITE_SIZE counters of the DG kernels to bytes."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    p.add_argument("--precision", default=None, choices=["fp64", "fp32"])
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=3)
    p.add_argument("--copy-calibration", action="store_true")
    args = p.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the method's multi-GPU path (domain decomposition with "
              "a face-trace halo exchange) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    N, k, default_prec, mach, sigma = WORKLOADS[args.workload]
    precision = args.precision or default_prec
    main_run = run_gpu(args, precision)
    compare = None
    if not args.no_compare:
        other = "fp32" if precision == "fp64" else "fp64"
        try:
            r = run_gpu(args, other)
            compare = {other: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                               "roofline_frac": r.get("roofline", {}).get("frac"),
                               "k_rhs_avg_ms": r.get("kernels", {}).get("k_rhs_avg_ms"),
                               "retries": r["retries"]}}
        except Exception as exc:  # report, do not hide the main measurement
            compare = {other: {"error": str(exc)}}
    cpu = None if args.no_cpu else run_cpu_baseline(args)
    rec = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}^3 cells, degree {k} ({(k + 1) * (k + 2) * (k + 3) // 6} modes/var, "
                               f"{(k + 1) ** 3} Gauss points), isothermal Euler, AV + primitive projection + "
                               f"positivity limiter, mean-free OU driving (target RMS Mach {mach:g})",
                   "cells": N ** 3, "degree": k, "dof": 4 * ((k + 1) * (k + 2) * (k + 3) // 6) * N ** 3,
                   "parallelism": "single GPU"},
        "roofline": main_run.get("roofline"),
        "cpu_baseline": cpu,
        "kernels": main_run.get("kernels"),
        "dt_reduction_ms_per_step": main_run["dt_reduction_ms_per_step"],
        "retries": main_run["retries"],
        "rms_mach_cell_means": main_run["rms_mach_cell_means"],
        "compare": compare,
        "source_hash": source_hash(),
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
