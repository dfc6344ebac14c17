"""Time-stepping driver around libdg (host control flow only; all arithmetic on the GPU).

One driver step: CFL time step (FP64 reduction on the GPU: the value dg_rk_step_next
returned with the previous step, so that a step costs one read-back, else dg_dt_max),
Ornstein-Uhlenbeck driving updates on the host whenever the simulation time crosses the
next update time (every t_c/100, Sec. 4.2), then the fused step; when the step reports a
positivity failure the state is still u^n and the step is retried with half the time step
(Sec. 3.1).  With the learned sensor the network's viscosity of u^n enters the viscous
bound and serves the stages (the previous fused step ran the network on this state), and
every judge_every steps the judge recomputes the plain labels and the fallback flags, after
which the time step is taken again.  With speculate (the default) each step also has the
library launch the next step's first stage ahead (dg_rk_step_next_ahead) unless a driving
update or a judgement comes first, so the GPU does not wait for the host between steps; the
results are the same.  Checkpoints are the raw [var][mode][cell] array plus a JSON record of
the run parameters, the simulation time and the driving state.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import numpy as np

from . import dg


@dataclasses.dataclass
class Driving:
    mach: float               # target RMS Mach number
    sigma: float              # stationary standard deviation of each OU component
    seed: int = 0

    @property
    def t_c(self) -> float:   # eddy turnover time T = L / (2 cs Mach) with L = cs = 1 (Sec. 4.2)
        return 1.0 / (2.0 * self.mach)

    @property
    def dt_drive(self) -> float:
        return self.t_c / 100.0


def gaussian_draws(seed: int, update: int, n: int):
    """Standard normal draws for OU update number ``update`` of stream ``seed``."""
    return np.random.default_rng([seed, update]).standard_normal(n)


class Simulation:
    def __init__(self, cfg: dg.Config, u=None, driving: Driving | None = None, retry_limit: int = 30,
                 sensor_params=None, judge_every: int = 10, tau: float = 0.5, speculate: bool = True):
        import torch
        self.cfg = cfg
        self.ctx = dg.dg_init(cfg)
        self.u = self.ctx.empty_state() if u is None else u
        if u is None:
            self.u.zero_()
            self.u[0, 0] = 1.0                      # density 1, at rest (mode 0 is the mean)
        self.t = 0.0
        self.nstep = 0
        self.retries = 0
        self.retry_limit = retry_limit
        self.speculate = speculate
        self.driving = driving
        self.n_drive = 0
        self.next_drive = 0.0
        if driving is not None:
            dg.dg_forcing_ou_init(self.ctx, driving.t_c, driving.sigma)
            self._drive(1e30)                       # start from the stationary distribution
            self.next_drive = driving.dt_drive
        self._torch = torch
        # next time step returned by the fused step (plain sensor), valid while u is unchanged
        self._dt_next = None
        self._u_version = None
        # learned sensor (DG_LEARNED_SENSOR): network parameters, judge cadence and threshold
        self.learned = bool(cfg.flags & dg.DG_LEARNED_SENSOR)
        self.judge_every = judge_every
        self.tau = tau
        self.fallback_counts = []
        if self.learned:
            if sensor_params is None:
                raise ValueError("a learned-sensor run needs network parameters")
            dg.dg_sensor_set_params(self.ctx, sensor_params.to(self.ctx.device, torch.float32).contiguous())

    def _drive(self, dt_drive):
        z = gaussian_draws(self.driving.seed, self.n_drive, dg.dg_forcing_ou_ndraws())
        dg.dg_forcing_ou_advance(self.ctx, z, dt_drive)
        self.n_drive += 1

    def invalidate(self):
        """Forget the time step and projection kept from the last step (call after writing
        to self.u by other means than torch in-place operations, which are detected)."""
        self._dt_next = None

    def step(self, dt_cap: float | None = None):
        """One step; dt_cap (optional) shortens the time step, e.g. to land on an output time."""
        reuse = self._dt_next is not None and self._u_version == self.u._version
        if self.learned:
            # the network's viscosity of u^n serves the time step and the stages: the fused
            # step of the previous call already ran it on this state; the judge (which also
            # runs the network) refreshes the fallback flags, which changes the time step
            if self.nstep % self.judge_every == 0:
                self.fallback_counts.append(dg.dg_sensor_judge(self.ctx, self.u, self.tau))
                self._dt_next = None
            elif not reuse:
                dg.dg_sensor_infer(self.ctx, self.u)
        dt = self._dt_next if (reuse and self._dt_next is not None) else dg.dg_dt_max(self.ctx, self.u)
        if dt_cap is not None:
            dt = min(dt, dt_cap)
        if not (dt > 0.0 and np.isfinite(dt)):
            raise RuntimeError(f"invalid time step {dt} at step {self.nstep}")
        if self.driving is not None:
            while self.t + dt >= self.next_drive:
                self._drive(self.driving.dt_drive)
                self.next_drive += self.driving.dt_drive
        tries = 0
        self._dt_next = None
        while True:
            # launch the next step's first stage ahead unless the next step starts with a
            # driving update (its time step reaches the next update time) or a judgement
            horizon = 0.0
            if self.speculate and not (self.learned and (self.nstep + 1) % self.judge_every == 0):
                horizon = math.inf if self.driving is None else self.next_drive - (self.t + dt)
            rc, dt_next = dg.dg_rk_step_next_ahead(self.ctx, self.u, dt, reuse, horizon)
            if rc == dg.DG_OK:
                break
            self.retries += 1
            tries += 1
            if tries > self.retry_limit:
                raise RuntimeError(f"positivity retries exhausted at step {self.nstep}")
            dt *= 0.5
            reuse = False
        self._dt_next = dt_next
        self._u_version = self.u._version
        self.t += dt
        self.nstep += 1
        return dt

    def driving_state(self):
        """Everything that determines the future driving: time, update counters, OU state."""
        d = {"t": self.t, "n_drive": self.n_drive, "next_drive": self.next_drive}
        if self.driving is not None:
            d["ou_x"] = dg.dg_forcing_ou_get(self.ctx).tolist()
        return d

    def set_driving_state(self, d):
        self.t, self.n_drive, self.next_drive = d["t"], d["n_drive"], d["next_drive"]
        if self.driving is not None and "ou_x" in d:
            dg.dg_forcing_ou_set(self.ctx, np.asarray(d["ou_x"]))

    def rms_mach(self):
        """Volume-weighted RMS Mach number from the cell means (Sec. 4.1 definition with the
        velocity of each cell's mean state)."""
        u = self.u
        rho = u[0, 0].double()
        v2 = ((u[1:, 0].double() / rho) ** 2).sum(0)
        return float(self._torch.sqrt(v2.mean()) / self.cfg.cs)

    def save(self, path: str):
        np.save(path + ".npy", self.u.detach().cpu().numpy())
        meta = {"cfg": dataclasses.asdict(self.cfg), "nstep": self.nstep,
                "driving": dataclasses.asdict(self.driving) if self.driving else None,
                "state": self.driving_state()}
        with open(path + ".json", "w") as fh:
            json.dump(meta, fh)

    @classmethod
    def load(cls, path: str, precision: int | None = None):
        import torch
        with open(path + ".json") as fh:
            meta = json.load(fh)
        cfg = dg.Config(**meta["cfg"])
        if precision is not None:
            cfg = dataclasses.replace(cfg, precision=precision)
        arr = np.load(path + ".npy")
        dtype = torch.float64 if cfg.precision == dg.DG_FP64 else torch.float32
        u = torch.as_tensor(arr, device="cuda").to(dtype).contiguous()
        drv = Driving(**meta["driving"]) if meta["driving"] else None
        sim = cls(cfg, u=u, driving=drv)
        sim.nstep = meta["nstep"]
        sim.set_driving_state(meta["state"])
        return sim
