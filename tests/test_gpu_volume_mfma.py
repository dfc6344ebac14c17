"""The FP32 degree-2 volume integral on the matrix cores (DG_VOLUME_MFMA) against the oracle
and against the vector-unit kernel it can replace.

The variant evaluates the state at the points and contracts the point fluxes and the driving
source with the weighted basis tables on v_mfma_f32_16x16x4f32, 16 cells per product; the
pointwise physics and the face pass are the vector kernel's.  Cases: meshes whose waves share
a y-z pencil (the staged driving table) and meshes where they do not, ragged tails (cells past
the mesh in the last tiles), viscosity with the Pi_max cap, the learned viscosity with its
fallback flags, mean-free driving, whole steps, and whole-line meshes where faces are shared.
Bar: the FP32 tolerance 1e-5 against the oracle; against the vector kernel the two differ only
by the order of their FP32 sums.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from gpu_util import assert_state_close, dev, field_rel, host, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
ALL = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER
FORCE = ALL | dg.DG_FORCING | dg.DG_FORCE_MEANFREE
MFMA = dg.DG_VOLUME_MFMA


def _rhs(shape, flags, u, dt, modes=None, nu=None, fb=None):
    ctx = make(*shape, 2, flags, dg.DG_FP32)
    if modes is not None:
        dg.dg_set_forcing(ctx, modes)
    if nu is not None:
        dg.dg_sensor_set_nu(ctx, torch.as_tensor(nu, device=ctx.device).to(ctx.dtype), torch.as_tensor(fb, device=ctx.device))
    ud = dev(u, ctx)
    out = torch.full_like(ud, float("nan"))
    dg.dg_rhs(ctx, ud, out, dt)
    got = host(out)
    ctx.close()
    return got


@pytest.mark.parametrize("shape", [(12, 10, 9), (64, 4, 6), (7, 1, 3), (128, 2, 3), (64, 5, 1)])
@pytest.mark.parametrize("flags", [FORCE, ALL, dg.DG_POS_LIMITER, FORCE | dg.DG_HLLC])
def test_rhs_matches_the_oracle_and_the_vector_kernel(shape, flags):
    print(f"volume on the matrix cores: {shape} flags {flags}", flush=True)
    u = synthetic.turbulent_like(*shape, 2, mach=4.0, seed=sum(shape) + flags, high_amp=0.1)
    u = u.astype(np.float32).astype(np.float64)
    modes = synthetic.forcing_table(3, amp=8.0) if flags & dg.DG_FORCING else None
    ocfg = oracle.Cfg(*shape, 2, flags=flags)
    dt = 0.5 * oracle.dt_max(ocfg, u)                 # the Pi_max cap binds in compressed points
    ref = oracle.rhs(ocfg, u, dt, modes)
    got = _rhs(shape, flags | MFMA, u, dt, modes)
    vec = _rhs(shape, flags, u, dt, modes)
    assert np.all(np.isfinite(got))
    e = field_rel(dt * got, dt * ref, u)
    assert max(e) < 1e-5, e
    ev = field_rel(dt * got, dt * vec, u)
    print(f"  vs oracle {e}, vs vector kernel {ev}", flush=True)
    assert max(ev) < 1e-6, ev


def test_rhs_with_the_learned_viscosity_and_fallback():
    shape = (64, 4, 4)
    flags = ALL | dg.DG_LEARNED_SENSOR
    u = synthetic.turbulent_like(*shape, 2, mach=4.0, seed=7, high_amp=0.1).astype(np.float32).astype(np.float64)
    nc = int(np.prod(shape))
    nu = (synthetic.random_nu(nc, 5) * 1e-2).astype(np.float32).astype(np.float64)
    fb = synthetic.random_fallback(nc, 6)
    ocfg = oracle.Cfg(*shape, 2, flags=(flags & ~dg.DG_LEARNED_SENSOR) | oracle.LEARNED)
    dt = 0.5 * oracle.dt_max(ocfg, u, nu, fb)
    ref = oracle.rhs(ocfg, u, dt, None, nu, fb)
    got = _rhs(shape, flags | MFMA, u, dt, nu=nu, fb=fb)
    assert max(field_rel(dt * got, dt * ref, u)) < 1e-5


def test_driven_steps_match_the_oracle():
    n = 16
    u = synthetic.turbulent_like(n, n, n, 2, mach=3.0, seed=8, high_amp=0.05).astype(np.float32).astype(np.float64)
    modes = synthetic.forcing_table(9, amp=10.0)
    ocfg = oracle.Cfg(n, n, n, 2, flags=FORCE)
    ctx = make(n, n, n, 2, FORCE | MFMA, dg.DG_FP32)
    dg.dg_set_forcing(ctx, modes)
    ud = dev(u, ctx)
    for i in range(3):
        dt = oracle.dt_max(ocfg, u)
        u, st = oracle.rk_step(ocfg, u, dt, modes)
        assert st == oracle.OK
        rc, _ = dg.dg_rk_step_next(ctx, ud, dt, i > 0)
        assert rc == dg.DG_OK
    assert_state_close(host(ud), u, 1e-5, "matrix-core volume, 3 driven steps")


def test_flag_needs_fp32_degree_2():
    for precision, k in ((dg.DG_FP64, 2), (dg.DG_FP32, 1), (dg.DG_FP32, 3)):
        with pytest.raises(dg.DGError) as err:
            make(8, 8, 8, k, ALL | MFMA, precision)
        assert err.value.rc == dg.DG_EUNSUPPORTED
