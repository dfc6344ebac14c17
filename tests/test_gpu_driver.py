"""The host time loop: checkpoint and resume, and copying a run's driving state.

A driven run interrupted by a checkpoint and resumed in a fresh context must continue
bitwise identically to the uninterrupted run (same OU state, same update counters, same
kernels in the same order)."""
import os

import numpy as np
import pytest
import torch

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
