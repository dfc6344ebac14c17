"""The host time loop: checkpoint and resume, copying a run's driving state, and the fused
step that returns the next time step (one read-back per step).

A driven run interrupted by a checkpoint and resumed in a fresh context must continue
bitwise identically to the uninterrupted run (same OU state, same update counters, same
kernels in the same order)."""
import os

import numpy as np
import pytest
import torch

import synthetic
from gpu_util import dev, make
from paper_2401_06841_amd import dg
from paper_2401_06841_amd.driver import Driving, Simulation

pytestmark = pytest.mark.gpu
FLAGS = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER | dg.DG_FORCING | dg.DG_FORCE_MEANFREE


def test_checkpoint_resume_is_bitwise(tmp_path):
    n = 12
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP64, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=4)
    a = Simulation(cfg, driving=drv)
    for _ in range(60):
        a.step()
    path = os.path.join(tmp_path, "ck")
    a.save(path)
    for _ in range(40):
        a.step()
    b = Simulation.load(path)
    for _ in range(40):
        b.step()
    assert b.nstep == a.nstep and b.t == a.t and b.n_drive == a.n_drive
    assert torch.equal(a.u, b.u)
    assert np.array_equal(dg.dg_forcing_ou_get(a.ctx), dg.dg_forcing_ou_get(b.ctx))


def test_driving_state_copy_gives_identical_runs():
    n = 10
    cfg = dg.Config(n, n, n, degree=1, precision=dg.DG_FP64, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=2)
    a = Simulation(cfg, driving=drv)
    for _ in range(30):
        a.step()
    b = Simulation(cfg, u=a.u.clone(), driving=drv)
    b.set_driving_state(a.driving_state())
    for _ in range(30):
        a.step()
        b.step()
    assert torch.equal(a.u, b.u)


# ------------------------------------------------- fused next time step and reuse

@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_fused_next_time_step_equals_dt_max(precision):
    n, k = 12, 2
    flags = FLAGS
    ctx = make(n, n, n, k, flags, precision)
    dg.dg_set_forcing(ctx, synthetic.forcing_table(3, amp=2.0))
    u = dev(synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=5, high_amp=0.02, kmax_frac=0.125), ctx)
    dt = dg.dg_dt_max(ctx, u)
    for _ in range(3):
        rc, dn = dg.dg_rk_step_next(ctx, u, dt, True)
        assert rc == dg.DG_OK
        assert dn == dg.dg_dt_max(ctx, u)        # same kernels' arithmetic, same reduction
        dt = dn


@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_fused_steps_match_plain_steps_bitwise(precision):
    n, k = 10, 2
    u0 = synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=8, high_amp=0.02, kmax_frac=0.125)
    modes = synthetic.forcing_table(2, amp=2.0)
    a, b = make(n, n, n, k, FLAGS, precision), make(n, n, n, k, FLAGS, precision)
    for c in (a, b):
        dg.dg_set_forcing(c, modes)
    ua, ub = dev(u0, a), dev(u0, b)
    dtb = dg.dg_dt_max(b, ub)
    for i in range(8):
        dta = dg.dg_dt_max(a, ua)
        assert dg.dg_rk_step(a, ua, dta) == dg.DG_OK
        assert dta == dtb
        rc, dtb = dg.dg_rk_step_next(b, ub, dtb, i > 0)
        assert rc == dg.DG_OK
    assert torch.equal(ua, ub)


def test_reuse_is_dropped_after_state_changes():
    """After an intervening state-changing call the kept projection is not used: a state
    perturbed in between and then passed through dg_limit (which invalidates) gives the
    plain step's result."""
    n, k = 8, 2
    u0 = synthetic.turbulent_like(n, n, n, k, mach=2.0, seed=3, high_amp=0.02, kmax_frac=0.125)
    a, b = make(n, n, n, k, FLAGS & ~dg.DG_FORCING), make(n, n, n, k, FLAGS & ~dg.DG_FORCING)
    ua, ub = dev(u0, a), dev(u0, b)
    rc, dn = dg.dg_rk_step_next(b, ub, dg.dg_dt_max(b, ub), False)
    assert rc == dg.DG_OK
    ua.copy_(ub)
    for t in (ua, ub):
        t[1:, 1] += 0.01                          # perturb the momentum's linear x mode
    dg.dg_limit(b, ub)                            # a state-changing library call
    dg.dg_limit(a, ua)
    rc, _ = dg.dg_rk_step_next(b, ub, dn, True)
    assert rc == dg.DG_OK
    assert dg.dg_rk_step(a, ua, dn) == dg.DG_OK
    assert torch.equal(ua, ub)


def test_fused_step_retry_restores_state():
    k = 1
    ctx = make(4, 3, 2, k, dg.DG_POS_LIMITER)
    u = np.zeros((4, ctx.cfg.nb, ctx.cfg.ncell))
    u[0, 0] = 5e-4
    u[1, 0] = 2e-4
    ud = dev(u, ctx)
    rc, dn = dg.dg_rk_step_next(ctx, ud, 1e-3, False)
    assert rc == dg.DG_RETRY and dn is None
    assert np.array_equal(ud.cpu().numpy(), u)


def test_driver_detects_torch_writes_between_steps():
    n = 8
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP64, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=6)
    a = Simulation(cfg, driving=drv)
    for _ in range(5):
        a.step()
    b = Simulation(cfg, u=a.u.clone(), driving=drv)
    b.set_driving_state(a.driving_state())
    a.u[1:, 2] += 1e-3                            # in-place torch write: the driver must notice
    b.u[1:, 2] += 1e-3
    b.invalidate()
    for _ in range(3):
        a.step()
        b.step()
    assert torch.equal(a.u, b.u)


def _flat_params(seed):
    params = synthetic.mlp_params(seed)
    flat = np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)
    return torch.as_tensor(flat, device="cuda")


def test_learned_fused_step_needs_a_stored_viscosity():
    ctx = make(4, 4, 4, 2, FLAGS | dg.DG_LEARNED_SENSOR)
    u = ctx.empty_state()
    u.zero_()
    u[0, 0] = 1.0
    with pytest.raises(dg.DGError):
        dg.dg_rk_step_next(ctx, u, 1e-3, False)


@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_learned_fused_steps_match_plain_steps_bitwise(precision):
    """The fused learned step runs the network on the new state and returns the time step
    of dg_sensor_infer + dg_dt_max; the next fused step uses that viscosity."""
    n, k = 8, 2
    flags = FLAGS | dg.DG_LEARNED_SENSOR
    u0 = synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=12, high_amp=0.02, kmax_frac=0.125)
    modes = synthetic.forcing_table(4, amp=2.0)
    a, b = make(n, n, n, k, flags, precision), make(n, n, n, k, flags, precision)
    P = _flat_params(3)
    for c in (a, b):
        dg.dg_set_forcing(c, modes)
        dg.dg_sensor_set_params(c, P)
    ua, ub = dev(u0, a), dev(u0, b)
    dg.dg_sensor_infer(b, ub)
    dtb = dg.dg_dt_max(b, ub)
    for i in range(6):
        dg.dg_sensor_infer(a, ua)
        dta = dg.dg_dt_max(a, ua)
        assert dg.dg_rk_step(a, ua, dta) == dg.DG_OK
        assert dta == dtb
        rc, dtb = dg.dg_rk_step_next(b, ub, dtb, i > 0)
        assert rc == dg.DG_OK
    assert torch.equal(ua, ub)


@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_learned_fused_step_failure_keeps_state_and_viscosity(precision):
    """A fused learned step that fails its positivity check leaves u^n in place, and the
    viscosity the step stores is that of u^n (the network runs on u after the stages; with
    the failure flag raised it projects u afresh instead of reading the stage's projection):
    the time step afterwards equals dg_sensor_infer + dg_dt_max of u^n."""
    n, k = 8, 2
    flags = FLAGS | dg.DG_LEARNED_SENSOR
    u0 = synthetic.turbulent_like(n, n, n, k, mach=4.0, seed=13, high_amp=0.05, kmax_frac=0.25)
    ctx = make(n, n, n, k, flags, precision)
    dg.dg_set_forcing(ctx, synthetic.forcing_table(5, amp=2.0))
    dg.dg_sensor_set_params(ctx, _flat_params(6))
    u = dev(u0, ctx)
    before = u.clone()
    dg.dg_sensor_infer(ctx, u)
    dt_ref = dg.dg_dt_max(ctx, u)
    rc, dt_next = dg.dg_rk_step_next(ctx, u, 300.0 * dt_ref, False)
    assert rc == dg.DG_RETRY and dt_next is None
    assert torch.equal(u, before)
    assert dg.dg_dt_max(ctx, u) == dt_ref
    rc, _ = dg.dg_rk_step_next(ctx, u, dt_ref, False)
    assert rc == dg.DG_OK


def test_learned_driver_run_with_judge():
    """Driver with the learned sensor: judge every 3 steps, fused steps in between; the run
    stays finite and the judge keeps a count per judgement."""
    n = 8
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP32, flags=FLAGS | dg.DG_LEARNED_SENSOR)
    sim = Simulation(cfg, driving=Driving(3.0, 2.5, seed=1), sensor_params=_flat_params(4), judge_every=3)
    for _ in range(10):
        dt = sim.step()
        assert dt > 0 and np.isfinite(dt)
    assert len(sim.fallback_counts) == 4
    assert torch.all(torch.isfinite(sim.u))


# ------------------------------------------------------------- instrumentation levels

def test_profile_levels_count_the_bracketed_launches():
    """Level 1 times the first stage's right-hand side of each step, level 2 every
    right-hand-side and stage launch; the timed steps give the same state as untimed ones."""
    n = 8
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP64, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=1)
    plain = Simulation(cfg, driving=drv)
    timed = Simulation(cfg, driving=drv)
    for level, steps in ((1, 5), (2, 4)):
        dg.dg_profile(timed.ctx, level)
        r0 = timed.retries
        for _ in range(steps):
            plain.step()
            timed.step()
        attempts = steps + timed.retries - r0
        rhs_ms, rhs_n, st_ms, st_n = dg.dg_profile_read(timed.ctx)
        dg.dg_profile(timed.ctx, 0)
        if level == 1:
            assert (rhs_n, st_n) == (attempts, 0)
        else:
            assert (rhs_n, st_n) == (3 * attempts, 3 * attempts)
            assert st_ms > 0.0
        assert rhs_ms > 0.0
    assert torch.equal(plain.u, timed.u) and plain.t == timed.t
