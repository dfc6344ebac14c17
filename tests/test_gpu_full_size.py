"""Parity at the full sizes of the larger workloads, on sampled cells.

The GPU evaluates the right-hand side of the whole mesh in the configuration the
benchmark times; the oracle computes a seeded sample of cells one by one (with the
periodic corner cells always included).  Cases:
  * 128^3, degree 3, FP32 and FP64, Mach-10-like state with viscosity, projection, driving;
  * 128^3, degree 2, FP32, learned sensor with prescribed per-cell viscosity and fallback;
  * 256^3, degree 2, FP32 and FP64, Mach-10-like state with viscosity, projection, driving;
  * 256^3, degree 3, FP64 (the driving field is evaluated inside the right-hand side from a
    table of about 1 KB per y-z pencil, so no per-point field of 4 x 64 x 16.8M values is
    stored and every variable block stays below the 4 GiB of a buffer descriptor).
The mean-free driving correction needs a sum over the whole mesh (too slow for the oracle's
one-by-one cells at these sizes); whole-mesh steps with it are compared in
test_gpu_step_paths.py (up to 128^3), so the driving here is plain.
Bar: 1e-12 (FP64) / 1e-5 (FP32) state-relative per cell, as everywhere.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from gpu_util import dev, host, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
ALL = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER
DRIVE = ALL | dg.DG_FORCING
TOL = {dg.DG_FP64: 1e-12, dg.DG_FP32: 1e-5}

CASES = {
    "128-k3-fp32": (128, 3, dg.DG_FP32, DRIVE, False),
    "128-k3-fp64": (128, 3, dg.DG_FP64, DRIVE, False),
    "128-k2-learned-fp32": (128, 2, dg.DG_FP32, ALL | dg.DG_LEARNED_SENSOR, True),
    "256-k2-fp32": (256, 2, dg.DG_FP32, DRIVE, False),
    "256-k2-fp64": (256, 2, dg.DG_FP64, DRIVE, False),
    "256-k3-fp64": (256, 3, dg.DG_FP64, DRIVE, False),
}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", list(CASES))
def test_full_size_sampled(case):
    n, k, precision, flags, learned = CASES[case]
    print(f"full-size sampled case {case}", flush=True)
    u = synthetic.turbulent_like(n, n, n, k, mach=10.0, seed=31, high_amp=0.02, kmax_frac=0.125)
    if precision == dg.DG_FP32:
        u = u.astype(np.float32).astype(np.float64)
    nc = n ** 3
    modes = synthetic.forcing_table(4, amp=30.0) if flags & dg.DG_FORCING else None
    dt = 2e-5                                   # the Pi_max cap binds in strongly compressed cells
    ctx = make(n, n, n, k, flags, precision)
    if modes is not None:
        dg.dg_set_forcing(ctx, modes)
    nu = fb = None
    if learned:
        nu = synthetic.random_nu(nc, 5) * 1e-2
        fb = synthetic.random_fallback(nc, 6)
        if precision == dg.DG_FP32:
            nu = nu.astype(np.float32).astype(np.float64)
        dg.dg_sensor_set_nu(ctx, torch.as_tensor(nu, device=ctx.device).to(ctx.dtype),
                            torch.as_tensor(fb, device=ctx.device))
    ud = dev(u, ctx)
    out = torch.full_like(ud, float("nan"))
    dg.dg_rhs(ctx, ud, out, dt)
    rng = np.random.default_rng(1)
    cells = np.unique(np.concatenate([rng.integers(0, nc, 256), [0, n - 1, n * n - 1, nc - n * n, nc - 1]]))
    got = host(out[:, :, torch.as_tensor(cells, device=ctx.device)])          # [4][nb][s]
    del out, ud
    ctx.close()
    ocfg = oracle.Cfg(n, n, n, k, flags=(flags & ~dg.DG_LEARNED_SENSOR) | (oracle.LEARNED if learned else 0))
    ref = oracle.rhs_cells(ocfg, u, cells, dt, modes, None, nu, fb)            # [s][4][nb]
    g = np.transpose(got, (2, 0, 1))
    assert np.all(np.isfinite(g))
    scale = np.linalg.norm(u[:, :, cells].transpose(2, 0, 1).reshape(len(cells), 4, -1), axis=2)
    err = np.linalg.norm(dt * (g - ref), axis=2) / np.maximum(scale, 1e-30)
    assert err.max() < TOL[precision], (case, err.max())
