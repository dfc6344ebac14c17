"""Learned viscosity sensor: data collection, training and use (host control flow only).

The network (20 -> 64 -> 64 -> 1, GELU, bf16 matrix-core arithmetic) stands in for the
compression sensor of Sec. 3.1.  Every operation runs in libdg kernels:
  * data   - per-cell features (dg_sensor_features) and targets t = log(1 + nu/1e-3) of
             the plain sensor's labels (dg_sensor_targets), taken from snapshots of runs
             with the plain method;
  * fit    - mean-squared error on the full batch or on contiguous minibatches, gradient
             by dg_mlp_grad (fixed-order reduction, so training is deterministic), Adam by
             dg_mlp_adam;
  * use    - a Simulation with DG_LEARNED_SENSOR runs the network on u^n once per step
             (dg_sensor_infer) before the time step; the per-cell bulk viscosity serves the
             viscous time-step bound and the three stages.  Every `judge_every` steps
             dg_sensor_judge recomputes the plain labels and sends the cells whose
             prediction is off by more than tau (relative to nu + 1e-3) back to the plain
             sensor until the next judgement.
Parameters are one FP32 vector in the order W1[64][20], b1, W2[64][64], b2, W3[1][64], b3.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dg

SIZES = ((64, 20), (64, 64), (1, 64))


def init_params(seed: int) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; FP32 host tensor."""
    rng = np.random.default_rng(seed)
    parts = []
    for fo, fi in SIZES:
        parts.append(rng.standard_normal(fo * fi) * math.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == dg.DG_MLP_NPARAM
    return torch.from_numpy(p)


class Dataset:
    """Feature rows and targets gathered on the device from snapshots."""

    def __init__(self, capacity: int, device=None):
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.x = torch.empty((capacity, dg.DG_MLP_NIN), dtype=torch.float32, device=device)
        self.t = torch.empty(capacity, dtype=torch.float32, device=device)
        self.n = 0

    def add(self, ctx: dg.Context, u):
        nc = ctx.cfg.ncell
        if self.n + nc > self.x.shape[0]:
            raise ValueError("dataset capacity exceeded")
        dg.dg_sensor_features(ctx, u, self.x[self.n:self.n + nc])
        dg.dg_sensor_targets(ctx, u, self.t[self.n:self.n + nc])
        self.n += nc

    @property
    def rows(self):
        return self.x[:self.n], self.t[:self.n]


class Trainer:
    """Adam; the context only supplies the stream and the scratch for the per-wave
    gradient partials."""

    def __init__(self, ctx: dg.Context, params: torch.Tensor):
        dev = ctx.device
        self.ctx = ctx
        self.P = params.to(device=dev, dtype=torch.float32).contiguous().clone()
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.g = torch.empty_like(self.P)
        self.loss_dev = torch.empty(1, dtype=torch.float32, device=dev)
        self.step = 0

    def loss(self, x, t) -> float:
        dg.dg_mlp_grad(self.ctx, self.P, x, t, self.g, self.loss_dev)
        return float(self.loss_dev.item())

    def fit(self, x, t, steps: int, lr: float = 3e-3, lr_final: float = 3e-4, log_every: int = 0,
            batch: int = 0, seed: int = 0):
        """`steps` Adam updates with the learning rate decaying geometrically from lr to
        lr_final; returns the losses read back every log_every steps (and the last).  With
        0 < batch < rows each step uses one contiguous block of `batch` rows at a seeded
        random offset, otherwise the full batch."""
        losses = []
        ratio = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
        n = x.shape[0]
        rng = np.random.default_rng(seed)
        for i in range(steps):
            if 0 < batch < n:
                o = int(rng.integers(0, n - batch + 1))
                xb, tb = x[o:o + batch], t[o:o + batch]
            else:
                xb, tb = x, t
            dg.dg_mlp_grad(self.ctx, self.P, xb, tb, self.g, self.loss_dev)
            if (log_every and i % log_every == 0) or i == steps - 1:
                losses.append(float(self.loss_dev.item()))
            self.step += 1
            dg.dg_mlp_adam(self.ctx, self.P, self.g, self.m, self.v, self.step, lr * ratio ** i)
        return losses

    def predict(self, x) -> torch.Tensor:
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        dg.dg_mlp_forward(self.ctx, self.P, x, y)
        return y


def collect_from_run(sim, dataset: Dataset, snapshots: int, every: int):
    """Advance a plain-method Simulation and add a snapshot every `every` steps."""
    for _ in range(snapshots):
        for _ in range(every):
            sim.step()
        dataset.add(sim.ctx, sim.u)


def train_from_run(sim, snapshots: int, every: int, steps: int, seed: int = 0, lr: float = 3e-3,
                   lr_final: float = 3e-4):
    """Collect `snapshots` snapshots from a plain-method run and fit a network on them;
    returns (trainer, dataset, losses)."""
    ds = Dataset(snapshots * sim.cfg.ncell)
    collect_from_run(sim, ds, snapshots, every)
    tr = Trainer(sim.ctx, init_params(seed))
    x, t = ds.rows
    losses = tr.fit(x, t, steps, lr=lr, lr_final=lr_final, log_every=max(steps // 10, 1))
    return tr, ds, losses
