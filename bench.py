#!/usr/bin/env python3
"""Benchmark of the DG SSP-RK3 step on one MI355X.

A step is one pass of the whole hot path over the state: time step (CFL and viscous
bound, FP64 reduction on the GPU), driving-mode update when due (host Ornstein-Uhlenbeck
+ table upload), and one SSP-RK3 step (projection, three right-hand sides with viscosity,
driving and Rusanov faces, three stage combinations with the positivity limiter).  The
metric is DG degree-of-freedom updates per second per Runge-Kutta stage: 3 * 4 * nb * N^3
per step divided by the wall time of the timed steps.

Default workload (c5): 256^3 cells, degree 2 (10 modes per variable, 27 Gauss points),
FP64, artificial viscosity + primitive projection + positivity limiter, mean-free
solenoidal OU driving on 1 <= |n| <= 2 aimed at RMS Mach ~10 (t_c = T = 1/(2 Mach)).
A warm-up as long as the workload's spin-up (c5: 1500 steps) starts from density 1 at
rest; a shorter one (the default 5) starts from the seeded turbulence-like state of the
CPU leg (velocity RMS at the target Mach, log-normal density) and runs the warm-up steps
from there.  Then exactly K steps are timed with the state resident in HBM.

Comparison legs, from the same state and driving, timed the same way:
  * the other precision with the plain sensor (FP32 bulk mode for the FP64 workloads);
  * FP32 with the learned sensor (degree 2), whose network is trained by the library's
    kernels on sensor snapshots taken during the warm-up (at least its last state).
Each leg reports its throughput, its k_rhs roofline and the difference of its final state
from the main run's: per-field relative L2, density-PDF L1 distance and velocity-spectrum
log distance (the FP32 legs' statistics error against the FP64 path).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c2|c3|c4|c5]
                       [--precision fp64|fp32] [--no-compare] [--no-learned] [--no-cpu]
                       [--no-stats] [--rho-floor-rel R]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG DOF-updates/sec per RK stage (3D, order p) + % HBM/MFMA roofline vs FP64"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector = matrix FP64 peak
PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak (packed issue)
FP32_UNPACKED_TFLOPS = 78.6  # issue limit without packed FP32, which the library's kernels do not emit
PEAK_HBM_TBPS = 8.0          # MI355X HBM3E

WORKLOADS = {
    # name: (N, degree, default precision, target Mach, driving sigma, spin-up steps from rest)
    # sigma: stationary standard deviation of each OU component, from spin-up runs at 64^3
    # (RMS Mach grows as (sigma^2 t_c)^(1/3), Sec. 4.2; the calibration is statistical):
    # sigma 2.5 gives Mach 3.07 at t = 2.7 t_c, sigma 28 gives Mach 9.1 at t = 2.4 t_c
    # (sigma 40 reached Mach 11 and then stalled in positivity retries)
    "c1": (16, 1, "fp64", 0.0, 0.0, 20),
    "c2": (64, 2, "fp64", 3.0, 2.5, 4000),
    "c3": (128, 3, "fp32", 10.0, 28.0, 1000),
    "c4": (128, 2, "fp32", 10.0, 28.0, 1000),
    "c5": (256, 2, "fp64", 10.0, 28.0, 1500),
}
DEFAULT_WORKLOAD = "c5"
DEFAULT_WARMUP = 5
# log-normal width of the seeded start state's density: that of Mach 3 (a wider one puts
# cell means of the 256^3 mesh below the density floor, which no time step can repair)
START_DENSITY_MACH = 3.0


def start_state(workload, seed):
    """The seeded turbulence-like start state of a driven workload (numpy, FP64), shared by
    the GPU run (short warm-up) and the CPU leg."""
    import synthetic
    N, k, _, mach, _, _ = WORKLOADS[workload]
    return synthetic.turbulent_like(N, N, N, k, mach=mach, seed=seed, high_amp=0.02, kmax_frac=0.125,
                                    density_mach=min(mach, START_DENSITY_MACH))


# workloads without driving, artificial viscosity or projection: the 16^3 degree-1 sound wave
# (positivity limiter only).  At 4,096 cells it is bound by launch latency, not by the
# kernels' arithmetic or memory traffic.
UNDRIVEN = {"c1"}


def workload_flags(workload):
    from paper_2401_06841_amd import dg
    if workload in UNDRIVEN:
        return dg.DG_POS_LIMITER
    return dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER | dg.DG_FORCING | dg.DG_FORCE_MEANFREE


def source_hash():
    """Hash of the step kernels' sources (the counters in profiles/ are valid while it holds)."""
    from paper_2401_06841_amd.profiling import source_hash as h
    return h()


def _profile_record(kernel, workload, precision, what):
    """A committed rocprofv3 counter summary (profiles/<kernel>_<workload>_<precision>_<what>.json),
    or None when it is missing or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_{what}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec


def traffic_from_profiles(kernel, workload, precision, launches_unit=1):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, calibrated with a plain copy)."""
    rec = _profile_record(kernel, workload, precision, "traffic")
    return rec.get("bytes_per_launch") if rec else None


def executed_flops_from_profiles(kernel, workload, precision):
    """Floating-point operations the kernel executes per launch, from the SQ counters of its
    VALU additions, multiplications, fused multiply-adds (2) and transcendentals, 64 lanes
    per wave instruction."""
    rec = _profile_record(kernel, workload, precision, "flops")
    return rec.get("flops_per_launch") if rec else None


def _log(msg):
    """Progress on stderr (the JSON line is the only output on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _timed(sim, steps, measure_profile):
    import torch

    from paper_2401_06841_amd import dg
    t_dt = 0.0
    retries0 = sim.retries
    if measure_profile:
        dg.dg_profile(sim.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt_min = 1e300
    for _ in range(steps):
        dt = sim.step()
        dt_min = min(dt_min, dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = dg.dg_profile_read(sim.ctx) if measure_profile else None
    dg.dg_profile(sim.ctx, False)
    return wall, prof, sim.retries - retries0, dt_min


def _summary(args, sim, precision, wall, prof, retries, dt_min):
    from paper_2401_06841_amd import dg, model
    cfg = sim.cfg
    k = cfg.degree
    dof = 4 * cfg.nb * cfg.ncell
    out = {"precision": precision, "value": 3.0 * dof * args.steps / wall, "wall_s": wall,
           "ms_per_step": 1e3 * wall / args.steps, "retries": retries, "dt_min": dt_min,
           "sim_time": sim.t, "rms_mach": sim.rms_mach()}
    if prof:
        rhs_ms, rhs_n, st_ms, st_n = prof
        avg = rhs_ms / max(rhs_n, 1)
        fl = cfg.flags
        rhs_flops = model.rhs_flops_per_cell(k, av=bool(fl & dg.DG_AV), proj=bool(fl & dg.DG_PRIM_PROJ),
                                             forcing=bool(fl & dg.DG_FORCING)) * cfg.ncell
        # with split stages the timed kernel (the first stage's right-hand side) also forms the
        # stage's combination
        split = dg.dg_split_stages(sim.ctx)
        flops = rhs_flops + (model.combination_flops_per_cell(k) * cfg.ncell if split else 0)
        achieved = flops / (avg * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
        out["kernels"] = {"k_rhs_avg_ms": avg, "k_rhs_launches": rhs_n,
                          "k_rhs_forms_stage_combination": split,
                          "k_stage_avg_ms": st_ms / st_n if st_n else None, "k_stage_launches": st_n}
        if not split:
            out["kernels"]["k_rhs_share_of_step"] = avg * 3 * args.steps / (1e3 * wall)
        out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                           "frac": achieved / peak,
                           "kernel": "k_rhs: right-hand side and stage combination" if split else "k_rhs",
                           "traffic": traffic_from_profiles("k_rhs", args.workload, precision, 1)}
        if precision == "fp32":
            out["roofline"]["frac_of_unpacked_fp32"] = achieved / FP32_UNPACKED_TFLOPS
        executed = executed_flops_from_profiles("k_rhs", args.workload, precision)
        if executed:
            # the flops the kernel issues (counted), beside the model count of Sec. 7
            out["roofline"]["executed_flops_per_launch"] = executed
            out["roofline"]["executed_TFLOP_s"] = executed / (avg * 1e-3) / 1e12
            out["roofline"]["executed_frac"] = out["roofline"]["executed_TFLOP_s"] / peak
        traffic = out["roofline"]["traffic"]
        if traffic:
            # HBM rate implied by the counted bytes per launch over the live launch time
            gbps = traffic / (avg * 1e-3) / 1e9
            out["roofline"]["traffic_GB_per_s"] = gbps
            out["roofline"]["traffic_frac_of_hbm"] = gbps / (PEAK_HBM_TBPS * 1e3)
        out["algorithmic_flops_per_launch"] = flops
        out["rhs_flops_per_launch"] = rhs_flops
    return out


def _rhs_alone(sim, calls, summary):
    """With split stages every stage's right-hand-side kernel also forms the stage's
    combination: the right-hand side alone (stored, dg_rhs on the run's final state) timed over
    a few calls, its roofline beside the dominant kernel's."""
    import torch

    from paper_2401_06841_amd import dg
    out = torch.empty_like(sim.u)
    dt = dg.dg_dt_max(sim.ctx, sim.u)
    dg.dg_rhs(sim.ctx, sim.u, out, dt)            # untimed: the first call after the steps
    torch.cuda.synchronize()
    dg.dg_profile(sim.ctx, 1)
    for _ in range(calls):
        dg.dg_rhs(sim.ctx, sim.u, out, dt)
    torch.cuda.synchronize()
    ms, n, _, _ = dg.dg_profile_read(sim.ctx)
    dg.dg_profile(sim.ctx, False)
    avg = ms / max(n, 1)
    rf = summary["roofline"]
    achieved = summary["rhs_flops_per_launch"] / (avg * 1e-3) / 1e12
    summary["kernels"]["k_rhs_stored_avg_ms"] = avg
    rf["rhs_alone"] = {"kernel": "k_rhs alone (right-hand side stored, dg_rhs)", "avg_ms": avg,
                       "achieved": achieved, "frac": achieved / rf["peak"], "launches": n}


def _statistics(sim):
    """Flow statistics of the final state on the GPU (Sec. 4.3), timed: the structure
    function with 100 bins of 1e5 pairs and the spectrum on the N p grid (p = k+1).  Each
    is run once untimed (hipFFT plan set-up) and then timed on the host clock around the
    synchronising call.  The pair kernel reads two cell records of 4 nb doubles per pair."""
    import numpy as np
    import torch

    from paper_2401_06841_amd import analysis, dg
    ctx, u, k = sim.ctx, sim.u, sim.cfg.degree
    nbins, npairs, p = analysis.SF_BINS, analysis.SF_PAIRS, k + 1
    scr = torch.empty(dg.dg_stats_scratch_bytes(ctx, nbins, p), dtype=torch.uint8, device=ctx.device)
    out = {}
    for rep in range(2):
        t0 = time.perf_counter()
        s2 = dg.dg_structure_function(ctx, u, nbins, npairs, analysis.SF_SEED, scratch=scr)
        t_sf = time.perf_counter() - t0
        t0 = time.perf_counter()
        e = dg.dg_velocity_spectrum(ctx, u, p, scratch=scr)
        t_sp = time.perf_counter() - t0
    l = dg.dg_sf_bins(ctx, nbins)
    mach_l = np.sqrt(0.5 * s2) / sim.cfg.cs
    rec_bytes = 4 * sim.cfg.nb * 8
    pairs = nbins * npairs
    out["structure_function"] = {
        "bins": nbins, "pairs_per_bin": npairs, "ms": 1e3 * t_sf, "pairs_per_s": pairs / t_sf,
        "record_bytes_per_pair": 2 * rec_bytes, "record_GB_per_s": 2 * rec_bytes * pairs / t_sf / 1e9,
        "l_min": float(l[0]), "l_max": float(l[-1]),
        "mach_at_l_min": float(mach_l[0]), "mach_at_l_max": float(mach_l[-1]),
        "sonic_scale": analysis.sonic_scale(l, mach_l)}
    npts = (sim.cfg.nx * p) * (sim.cfg.ny * p) * (sim.cfg.nz * p)
    out["spectrum"] = {"samples_per_cell": p, "grid_points": npts, "ms": 1e3 * t_sp, "shells": len(e),
                       "half_v2": float(e.sum())}
    del scr
    torch.cuda.synchronize()
    return out


def _train_sensor(args, sim, ds):
    """Fit the learned sensor on the snapshots taken during the warm-up (library kernels)."""
    from paper_2401_06841_amd import sensor
    x, t = ds.rows
    tr = sensor.Trainer(sim.ctx, sensor.init_params(args.seed))
    t0 = time.perf_counter()
    batch = min(sim.cfg.ncell, 262144)
    losses = tr.fit(x, t, args.train_steps, lr=3e-3, lr_final=3e-4, batch=batch, seed=args.seed,
                    log_every=max(args.train_steps // 4, 1))
    full = tr.loss(x, t)
    info = {"rows": int(ds.n), "snapshots": int(ds.n // sim.cfg.ncell), "adam_steps": args.train_steps,
            "minibatch_rows": batch, "loss_first": losses[0], "loss_last_batch": losses[-1],
            "loss_all_rows": full, "train_s": time.perf_counter() - t0}
    return tr.P.detach().cpu(), info


def run_gpu(args, precision, measure_profile=True):
    """Spin up from rest (untimed warm-up, taking sensor snapshots near its end), then time
    exactly args.steps steps.  The comparison legs (the other precision with the plain
    sensor, and FP32 with the learned sensor trained on the warm-up snapshots) start from
    the same state with the same driving, are timed the same way, and their final states
    are compared with the main run's (per-field L2, density PDF, velocity spectrum)."""
    import torch

    from paper_2401_06841_amd import analysis, dg, sensor
    from paper_2401_06841_amd.driver import Driving, Simulation

    N, k, _, mach, sigma, spinup = WORKLOADS[args.workload]
    flags = workload_flags(args.workload)
    prec = dg.DG_FP64 if precision == "fp64" else dg.DG_FP32
    cfg = dg.Config(N, N, N, degree=k, precision=prec, flags=flags, rho_floor_rel=args.rho_floor_rel)
    dtype = torch.float64 if prec == dg.DG_FP64 else torch.float32
    if args.workload in UNDRIVEN:
        import synthetic
        drv = None
        u = torch.as_tensor(synthetic.c1_modal_state(args.seed, N), device="cuda").to(dtype).contiguous()
        sim = Simulation(cfg, u=u, driving=None)
    elif args.start_state is not None:
        drv = Driving(mach, sigma, seed=args.seed)
        sim = Simulation(cfg, u=torch.as_tensor(args.start_state, device="cuda").to(dtype).contiguous(), driving=drv)
    else:
        drv = Driving(mach, sigma, seed=args.seed)
        sim = Simulation(cfg, driving=drv)
    learned = (not args.no_compare) and (not args.no_learned) and k == 2
    # snapshots for the sensor training: at most about 1e7 cells (at least one snapshot)
    nsnap = max(1, min(args.snapshots, args.warmup // args.snapshot_every, int(1e7) // cfg.ncell)) if learned else 0
    ds = sensor.Dataset(nsnap * cfg.ncell) if nsnap else None
    first = args.warmup - nsnap * args.snapshot_every
    for i in range(args.warmup):
        sim.step()
        if ds is not None and i + 1 > first and (i + 1 - first) % args.snapshot_every == 0:
            ds.add(sim.ctx, sim.u)
        if args.verbose and (i + 1) % 1000 == 0:
            print(f"warm-up step {i + 1}: t={sim.t:.4f} rms Mach {sim.rms_mach():.3f}", file=sys.stderr, flush=True)
    _log(f"warm-up done: {args.warmup} steps, t = {sim.t:.4g}, rms Mach {sim.rms_mach():.3f}")
    u0 = sim.u.clone()
    drive0 = sim.driving_state() if drv is not None else None
    wall, prof, retries, dt_min = _timed(sim, args.steps, measure_profile)
    main = _summary(args, sim, precision, wall, prof, retries, dt_min)
    _log(f"timed {args.steps} steps ({precision}): {main['ms_per_step']:.3f} ms per step")
    if not args.no_stats:
        main["statistics"] = _statistics(sim)
        _log("flow statistics done")
    compare = None
    if not args.no_compare:
        compare = {}
        ref = sim.u.detach().clone()
        legs = [("fp32" if precision == "fp64" else "fp64", False)]
        if learned:
            legs.append(("fp32", True))
        params, train_info = (None, None)
        for other, use_learned in legs:
            name = other + ("_learned" if use_learned else "")
            try:
                if use_learned and params is None:
                    params, train_info = _train_sensor(args, sim, ds)
                fl = flags | (dg.DG_LEARNED_SENSOR if use_learned else 0)
                cfg2 = dataclasses.replace(cfg, precision=dg.DG_FP32 if other == "fp32" else dg.DG_FP64, flags=fl)
                dtype = torch.float32 if other == "fp32" else torch.float64
                sim2 = Simulation(cfg2, u=u0.to(dtype).contiguous(), driving=drv,
                                  sensor_params=params if use_learned else None)
                if drive0 is not None:
                    sim2.set_driving_state(drive0)
                w2, p2, r2, d2 = _timed(sim2, args.steps, measure_profile)
                rec = _summary(args, sim2, other, w2, p2, r2, d2)
                rec["vs_main"] = analysis.compare(sim2.u, ref, k, (N, N, N), sim2.ctx, sim.ctx)
                if use_learned:
                    rec["training"] = train_info
                    rec["fallback_fraction_mean"] = float(sum(sim2.fallback_counts)) / max(
                        len(sim2.fallback_counts), 1) / cfg.ncell
                    rec["judge_every"] = sim2.judge_every
                compare[name] = rec
                sim2.ctx.close()
                _log(f"leg {name}: {rec['ms_per_step']:.3f} ms per step")
            except Exception as exc:  # report, do not hide the main measurement
                compare[name] = {"error": str(exc)}
    if measure_profile and main.get("kernels", {}).get("k_rhs_forms_stage_combination"):
        # after the statistics and the legs, which compare against the timed run's final state
        _rhs_alone(sim, 3, main)
    sim.ctx.close()
    return main, compare


def _omp_threads(n=None):
    """The OpenMP thread count of the oracle's parallel loops (set when n is given)."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def run_cpu_baseline(args):
    """The oracle as it stands, timed on the host cores on a bounded sample of the same
    workload (same mesh, degree, flags and driving), from the seeded start state the GPU run
    uses for short warm-ups (the oracle's cost does not depend on the flow): whole SSP-RK3
    steps where they take seconds (64^3 and below), otherwise one right-hand side of the whole
    mesh (the dominant work of one stage; the stage combination is a few operations per DOF).
    Also on one core: the per-cell right-hand side over a seeded sample of cells, timed with
    one thread and with all of them (the per-cell form also projects the velocity of the six
    neighbours, so its rate is below the whole-mesh form's)."""
    import numpy as np

    import oracle
    import synthetic

    N, k, _, mach, sigma, _ = WORKLOADS[args.workload]
    if args.workload in UNDRIVEN:
        cfg = oracle.Cfg(N, N, N, k, flags=oracle.POS_LIMITER)
        u = synthetic.c1_modal_state(args.seed, N)
        modes = None
    else:
        flags = oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER | oracle.FORCING | oracle.FORCE_MEANFREE
        cfg = oracle.Cfg(N, N, N, k, flags=flags, rho_floor_rel=args.rho_floor_rel)
        u = args.start_state if args.start_state is not None else start_state(args.workload, args.seed)
        modes = synthetic.forcing_table(args.seed, amp=sigma)
    oracle.lib()
    cores = _omp_threads()
    dof = 4 * cfg.nb * cfg.ncell
    if N <= 64:
        # the 16^3 workload takes milliseconds per step: time enough steps for a stable figure
        nsteps = max(args.cpu_steps, 200) if args.workload in UNDRIVEN else args.cpu_steps
        t0 = time.perf_counter()
        for _ in range(nsteps):
            dt = oracle.dt_max(cfg, u)
            u, st = oracle.rk_step(cfg, u, dt, modes)
        wall = time.perf_counter() - t0
        rec = {"value": 3.0 * dof * nsteps / wall, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
               "sample": f"{nsteps} SSP-RK3 steps ({3 * nsteps} stages) of the {N}^3 degree-{k} workload, "
                         f"FP64 C oracle with OpenMP over cells, {wall:.1f} s"}
    else:
        t0 = time.perf_counter()
        oracle.rhs(cfg, u, 1e-5, modes)
        wall = time.perf_counter() - t0
        rec = {"value": dof / wall, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
               "sample": f"one right-hand side of the whole {N}^3 degree-{k} mesh (the work of one stage without "
                         f"the stage combination), FP64 C oracle with OpenMP over cells, {wall:.1f} s"}
    ns = min(cfg.ncell, args.cpu_cells)
    cells = np.sort(np.random.default_rng(args.seed).choice(cfg.ncell, ns, replace=False))
    abar = oracle.forcing_mean(cfg, u, modes) if modes is not None else None
    rates = {}
    for threads in (1, cores):
        _omp_threads(threads)
        t0 = time.perf_counter()
        oracle.rhs_cells(cfg, u, cells, 1e-5, modes, abar)
        rates[threads] = 4 * cfg.nb * ns / (time.perf_counter() - t0)
    _omp_threads(cores)
    rec["one_core"] = {"value": rates[1], "unit": "DOF-updates/s", "cores": 1,
                       "all_cores_same_sample": rates[cores],
                       "sample": f"per-cell right-hand side (orc_rhs_cells) of {ns} seeded cells of the same state, "
                                 f"with its six neighbours' projections; 1 thread and {cores} threads"}
    return rec


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
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=DEFAULT_WARMUP)
    p.add_argument("--verbose", action="store_true")
    p.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    p.add_argument("--start", default="auto", choices=["auto", "rest", "turbulent"],
                   help="driven workloads: start at rest, or from the seeded turbulence-like state "
                        "(auto: the latter when the warm-up is shorter than the workload's spin-up)")
    p.add_argument("--rho-floor-rel", type=float, default=0.1,
                   help="relative part of the limiter's target density max(1e-3, R * cell mean)")
    p.add_argument("--cpu-cells", type=int, default=50000)
    p.add_argument("--precision", default=None, choices=["fp64", "fp32"])
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=10)
    p.add_argument("--no-learned", action="store_true")
    p.add_argument("--no-stats", action="store_true", help="skip the flow-statistics timing")
    p.add_argument("--snapshots", type=int, default=16)
    p.add_argument("--snapshot-every", type=int, default=100)
    p.add_argument("--train-steps", type=int, default=2000)
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
    N, k, default_prec, mach, sigma, spinup = WORKLOADS[args.workload]
    precision = args.precision or default_prec
    turbulent_start = args.workload not in UNDRIVEN and (
        args.start == "turbulent" or (args.start == "auto" and args.warmup < spinup))
    args.start_state = start_state(args.workload, args.seed) if turbulent_start else None
    _log(f"workload {args.workload}, {precision}, start {'seeded turbulence-like state' if turbulent_start else 'rest'}")
    try:
        main_run, compare = run_gpu(args, precision)
    except RuntimeError as exc:        # e.g. positivity retries exhausted: report, no figure
        print(json.dumps({"metric": METRIC, "value": None, "unit": "DOF-updates/s", "n_gpus": 1,
                          "workload": args.workload, "rho_floor_rel": args.rho_floor_rel, "error": str(exc)}))
        sys.exit(1)
    cpu = None if args.no_cpu else run_cpu_baseline(args)
    if cpu:
        _log(f"CPU oracle: {cpu['value']:.3e} DOF-updates/s on {cpu['cores']} threads")
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
                               f"{(k + 1) ** 3} Gauss points), isothermal Euler, " + (
                                   "sound wave of amplitude 1e-3, positivity limiter only (launch-latency bound: "
                                   "the roofline fraction does not measure the kernels)" if args.workload in UNDRIVEN
                                   else f"AV + primitive projection + positivity limiter (target max(1e-3, "
                                        f"{args.rho_floor_rel:g} x cell mean)), mean-free OU driving (target RMS "
                                        f"Mach {mach:g}), " + (
                                            f"timed after {args.warmup} warm-up steps from a seeded turbulence-like "
                                            f"state (velocity RMS Mach {mach:g}, log-normal density of the Mach "
                                            f"{min(mach, START_DENSITY_MACH):g} width)" if turbulent_start else
                                            f"timed after a spin-up of {args.warmup} steps from rest")),
                   "cells": N ** 3, "degree": k, "dof": 4 * ((k + 1) * (k + 2) * (k + 3) // 6) * N ** 3,
                   "parallelism": "single GPU"},
        "roofline": main_run.get("roofline"),
        "cpu_baseline": cpu,
        "kernels": main_run.get("kernels"),
        "statistics": main_run.get("statistics"),
        "retries": main_run["retries"],
        "rms_mach": main_run["rms_mach"],
        "sim_time": main_run["sim_time"],
        "compare": compare,
        "source_hash": source_hash(),
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
