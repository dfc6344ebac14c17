"""Host control flow of the time-stepping driver, with the library calls replaced by stubs
(no GPU): the horizon passed to dg_rk_step_next_ahead is the time left before the next
driving update, infinite without driving and zero before a judgement; retries halve the
time step and drop the reuse of the kept projection."""
import math
import types

import pytest

from paper_2401_06841_amd import dg, driver


class _Stub:
    """Records the fused-step calls; returns a fixed next time step, failing on demand."""

    def __init__(self, dt_next, fail_calls=()):
        self.calls = []
        self.dt_next = dt_next
        self.fail_calls = set(fail_calls)
        self.judged = []
        self.drives = 0

    def step(self, ctx, u, dt, reuse, horizon):
        self.calls.append((dt, reuse, horizon))
        if len(self.calls) - 1 in self.fail_calls:
            return dg.DG_RETRY, None
        return dg.DG_OK, self.dt_next


def _sim(monkeypatch, stub, driving=None, learned=False, judge_every=10):
    u = types.SimpleNamespace(_version=0)
    sim = driver.Simulation.__new__(driver.Simulation)
    sim.cfg, sim.ctx, sim.u = None, None, u
    sim.t, sim.nstep, sim.retries, sim.retry_limit = 0.0, 0, 0, 5
    sim.driving, sim.n_drive = driving, 0
    sim.next_drive = driving.dt_drive if driving else 0.0
    sim._dt_next, sim._u_version = None, None
    sim.learned, sim.judge_every, sim.tau, sim.fallback_counts = learned, judge_every, 0.5, []
    sim.speculate = True
    monkeypatch.setattr(dg, "dg_rk_step_next_ahead", stub.step)
    monkeypatch.setattr(dg, "dg_dt_max", lambda ctx, u: stub.dt_next)
    monkeypatch.setattr(dg, "dg_sensor_judge", lambda ctx, u, tau: stub.judged.append(sim.nstep) or 0)
    monkeypatch.setattr(dg, "dg_sensor_infer", lambda ctx, u: None)

    def _drive(dt_drive):
        stub.drives += 1
        sim.n_drive += 1
    sim._drive = _drive
    return sim


def test_horizon_is_the_time_left_before_the_next_driving_update(monkeypatch):
    stub = _Stub(dt_next=0.3)
    drv = driver.Driving(mach=1.0 / (2.0 * 100.0), sigma=1.0)     # t_c = 100, dt_drive = 1
    sim = _sim(monkeypatch, stub, driving=drv)
    for _ in range(7):
        sim.step()
    for i, (dt, reuse, horizon) in enumerate(stub.calls):
        t_before = 0.3 * i
        # the updates the step needed were applied before it: next_drive is past t + dt
        next_drive = math.floor((t_before + dt) / 1.0) + 1.0
        assert horizon == pytest.approx(next_drive - (t_before + dt))
        assert horizon > 0
        assert reuse == (i > 0)
    assert stub.drives == math.floor(0.3 * 7 / 1.0)


def test_horizon_is_infinite_without_driving(monkeypatch):
    stub = _Stub(dt_next=0.01)
    sim = _sim(monkeypatch, stub)
    for _ in range(3):
        sim.step()
    assert all(h == math.inf for _, _, h in stub.calls)


def test_no_launch_ahead_before_a_judgement(monkeypatch):
    stub = _Stub(dt_next=0.01)
    sim = _sim(monkeypatch, stub, learned=True, judge_every=3)
    for _ in range(7):
        sim.step()
    assert stub.judged == [0, 3, 6]
    for n, (_, _, horizon) in enumerate(stub.calls):
        assert (horizon == 0.0) == ((n + 1) % 3 == 0)


def test_retry_halves_the_step_and_drops_reuse(monkeypatch):
    stub = _Stub(dt_next=0.02, fail_calls=(1,))
    sim = _sim(monkeypatch, stub)
    sim.step()
    sim.step()
    dts = [c[0] for c in stub.calls]
    reuses = [c[1] for c in stub.calls]
    assert dts == [0.02, 0.02, 0.01] and reuses == [False, True, False]
    assert sim.retries == 1 and sim.t == pytest.approx(0.03)


def test_time_step_cap_lands_on_an_output_time(monkeypatch):
    """step(dt_cap) takes the smaller of the stable step and the cap, so a run can stop
    exactly at an output time."""
    stub = _Stub(dt_next=0.3)
    sim = _sim(monkeypatch, stub)
    t_end = 1.0
    while sim.t < t_end * (1 - 1e-12):
        sim.step(dt_cap=t_end - sim.t)
    assert [c[0] for c in stub.calls] == pytest.approx([0.3, 0.3, 0.3, 0.1])
    assert sim.t == pytest.approx(1.0, abs=1e-15)
