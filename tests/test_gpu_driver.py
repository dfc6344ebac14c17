"""The host time loop: checkpoint and resume, copying a run's driving state, and the fused
step that returns the next time step (one read-back per step).

A driven run interrupted by a checkpoint and resumed in a fresh context must continue
bitwise identically to the uninterrupted run (same OU state, same update counters, same
kernels in the same order)."""
import ctypes
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


# ------------------------------------------------ next step's first stage launched ahead

@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_launched_ahead_runs_match_plain_runs_bitwise(precision):
    """Driven runs with and without the first stage launched ahead: same states, times and
    driving updates, bit for bit (12^3 at Mach 3 updates the driving every few steps, so many
    launched stages are continued and some are not launched)."""
    n = 12
    cfg = dg.Config(n, n, n, degree=2, precision=precision, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=7)
    a = Simulation(cfg, driving=drv, speculate=True)
    b = Simulation(cfg, driving=drv, speculate=False)
    for _ in range(40):
        assert a.step() == b.step()
    assert torch.equal(a.u, b.u) and a.t == b.t and a.n_drive == b.n_drive


def test_launched_ahead_learned_run_with_judge_matches_plain_run():
    n = 8
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP32, flags=FLAGS | dg.DG_LEARNED_SENSOR)
    runs = [Simulation(cfg, driving=Driving(3.0, 2.5, seed=1), sensor_params=_flat_params(4), judge_every=3,
                       speculate=s) for s in (True, False)]
    for _ in range(12):
        assert runs[0].step() == runs[1].step()
    assert torch.equal(runs[0].u, runs[1].u)
    assert runs[0].fallback_counts == runs[1].fallback_counts


def test_launched_stage_is_dropped_when_its_inputs_change():
    """A stage launched ahead is continued only by the same array with the returned time
    step; a new driving table in between, another time step or a torch write all discard it
    and the step is computed afresh (compared with a context that never launches ahead)."""
    n, k = 10, 2
    u0 = synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=14, high_amp=0.02, kmax_frac=0.125)
    t1, t2 = synthetic.forcing_table(1, amp=3.0), synthetic.forcing_table(2, amp=3.0)
    ctx_a, ctx_b = make(n, n, n, k, FLAGS), make(n, n, n, k, FLAGS)
    for c in (ctx_a, ctx_b):
        dg.dg_set_forcing(c, t1)
    ua, ub = dev(u0, ctx_a), dev(u0, ctx_b)
    dta = dg.dg_dt_max(ctx_a, ua)
    dtb = dta
    reuse = False
    for i in range(8):
        rc, dta_n = dg.dg_rk_step_next_ahead(ctx_a, ua, dta, reuse, float("inf"))
        rcb, dtb_n = dg.dg_rk_step_next(ctx_b, ub, dtb, reuse)
        assert rc == rcb == dg.DG_OK and dta_n == dtb_n
        dta, dtb = dta_n, dtb_n
        reuse = True
        if i == 2:                                   # new table: the launched stage is stale
            for c in (ctx_a, ctx_b):
                dg.dg_set_forcing(c, t2)
        if i == 4:                                   # another time step than the returned one
            dta = dtb = 0.5 * dta
        if i == 6:                                   # a write the library does not see: reuse = 0
            ua.mul_(1.0)
            ub.mul_(1.0)
            reuse = False
    assert torch.equal(ua, ub)


def test_launched_ahead_argument_errors():
    n, k = 6, 2
    ctx = make(n, n, n, k, FLAGS)
    u = dev(synthetic.turbulent_like(n, n, n, k, mach=2.0, seed=3), ctx)
    with pytest.raises(dg.DGError):
        dg.dg_rk_step_next_ahead(ctx, u, 1e-4, False, float("nan"))
    with pytest.raises(dg.DGError):
        dg.dg_rk_step_next_ahead(ctx, u, 0.0, False, 1.0)
    st = ctypes.c_int(0)
    assert dg._lib.dg_rk_step_next_ahead(ctx.h, ctypes.c_void_p(u.data_ptr()), 1e-4, 0, 1.0, ctypes.byref(st),
                                         None) == dg.DG_EINVAL
    rc, dt_next = dg.dg_rk_step_next_ahead(ctx, u, 1e-5, False, 0.0)     # horizon 0: plain step
    assert rc == dg.DG_OK and dt_next > 0


# ------------------------------------------------------------- instrumentation levels

def test_profile_levels_count_the_bracketed_launches():
    """Level 1 times the first stage's right-hand side of each step, level 2 every
    right-hand-side and stage launch; the timed steps give the same state as untimed ones."""
    n = 8
    cfg = dg.Config(n, n, n, degree=2, precision=dg.DG_FP64, flags=FLAGS)
    drv = Driving(3.0, 2.5, seed=1)
    plain = Simulation(cfg, driving=drv, speculate=False)
    timed = Simulation(cfg, driving=drv, speculate=False)
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
