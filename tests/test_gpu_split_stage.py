"""Split Runge-Kutta stages against separate stage kernels.

With DG_SPLIT_STAGE every stage of a step without a side combination is split: once a cell's
right-hand side is formed, the right-hand-side kernel combines it with the cell's input weights
(and u^n) and stores the result, and a second kernel limits it (Sec. 3.1) and projects its
velocity (Sec. 3.2) for the next stage.  The last stage stores its combination into a free
workspace buffer, raises the failure flag from its mean density, and the stage kernel writes
the caller's array from there unless a cell failed.  DG_SEPARATE_STAGE stores
the right-hand side and runs the stage kernel instead.  Every combination has the same
roundings in both, so they give the same bits, except with mean-free driving (Sec. 4.2) and a
table on the driving shell: the split path then forms the mean-acceleration partials of a
stage input (in the previous split stage, or in a kernel of their own before a step's first
stage) in the modal form of the pencil table, the same sums as the right-hand side's point
sums up to rounding, and the two paths agree to the parity bars (1e-12 FP64, 1e-5 FP32, in
the field norms and weight by weight, and the time steps).  Each case steps one seeded state in
two contexts.  Without either flag the split is used on meshes of at least 2^21 cells; the parity of
both paths with the oracle is checked by the step tests of the other files.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from gpu_util import assert_state_close, dev, host, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
BASE = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER
FORCE = BASE | dg.DG_FORCING | dg.DG_FORCE_MEANFREE
FP64, FP32 = dg.DG_FP64, dg.DG_FP32

# (label, cells, degree, precision, flags, forcing table: "shell", "general" or None)
CASES = [
    ("k1 fp64", (16, 16, 16), 1, FP64, FORCE, "shell"),
    ("k2 fp64", (24, 16, 16), 2, FP64, FORCE, "shell"),
    ("k2 fp64 hllc", (24, 16, 16), 2, FP64, FORCE | dg.DG_HLLC, "shell"),
    ("k2 fp64 undriven", (16, 16, 16), 2, FP64, BASE, None),
    ("k2 fp64 driven, mean kept", (16, 16, 16), 2, FP64, BASE | dg.DG_FORCING, "shell"),
    ("k2 fp64 general table", (16, 16, 16), 2, FP64, FORCE, "general"),
    ("k2 fp64 plain traces", (16, 16, 16), 2, FP64, FORCE & ~dg.DG_PRIM_PROJ, "shell"),
    # a last block with inactive lanes, and waves spanning several pencils (x lines of 20)
    ("k2 fp64 ragged", (20, 15, 13), 2, FP64, FORCE, "shell"),
    ("k2 fp32 ragged", (20, 15, 13), 2, FP32, FORCE, "shell"),
    ("k3 fp32 ragged", (9, 7, 5), 3, FP32, FORCE, "shell"),
    ("k1 fp64 two-stage scheme", (16, 16, 16), 1, FP64, FORCE | dg.DG_RK_BY_ORDER, "shell"),
    ("k2 fp32", (16, 16, 16), 2, FP32, FORCE, "shell"),
    ("k3 fp32", (12, 12, 12), 3, FP32, FORCE, "shell"),
    ("k3 fp32 five-stage scheme", (12, 12, 12), 3, FP32, FORCE | dg.DG_RK_BY_ORDER, "shell"),
    # above 1,024 blocks the mean acceleration goes through its own reduction kernel
    ("k2 fp64 1,152 blocks", (72, 64, 64), 2, FP64, FORCE, "shell"),
    ("k2 fp32 1,280 blocks", (128, 64, 40), 2, FP32, FORCE, "shell"),
]


def _pair(shape, k, precision, flags, table, seed, split=dg.DG_SPLIT_STAGE, **kw):
    """Two contexts of one configuration: split stages (or the default choice, split=0) and
    separate ones."""
    a = make(*shape, k, flags | split, precision, **kw)
    b = make(*shape, k, flags | dg.DG_SEPARATE_STAGE, precision, **kw)
    if table:
        modes = (synthetic.forcing_table if table == "shell" else synthetic.forcing_table_general)(seed, amp=2.5)
        for c in (a, b):
            dg.dg_set_forcing(c, modes)
    return a, b


TOL = {FP64: 1e-12, FP32: 1e-5}


def _exact(flags, table):
    """Whether the two paths form the same partial sums (see the module text)."""
    return not (flags & dg.DG_FORCE_MEANFREE and flags & dg.DG_FORCING and table == "shell")


def _compare(ua, ub, da, db, exact, tol, label):
    if exact:
        assert da == db, (label, da, db)
        assert torch.equal(ua, ub), f"{label}: largest difference {(ua - ub).abs().max().item():.3e}"
    else:
        assert abs(da - db) <= tol * abs(db), (label, da, db)
        assert_state_close(host(ua), host(ub), tol, label)


def _steps_equal(a, b, ua, ub, nsteps, ahead=False, exact=True, tol=0.0):
    dt = dg.dg_dt_max(a, ua)
    assert dt == dg.dg_dt_max(b, ub)
    for i in range(nsteps):
        if ahead:
            ra, da = dg.dg_rk_step_next_ahead(a, ua, dt, i > 0, float("inf"))
            rb, db = dg.dg_rk_step_next_ahead(b, ub, dt, i > 0, float("inf"))
        else:
            ra, da = dg.dg_rk_step_next(a, ua, dt, i > 0)
            rb, db = dg.dg_rk_step_next(b, ub, dt, i > 0)
        assert ra == rb == dg.DG_OK, (i, ra, rb)
        _compare(ua, ub, da, db, exact, tol, f"step {i}")
        dt = da


@pytest.mark.parametrize("label,shape,k,precision,flags,table", CASES, ids=[c[0] for c in CASES])
def test_split_stage_equals_separate_stage(label, shape, k, precision, flags, table):
    print(f"split vs separate stages: {label} {shape}", flush=True)
    u0 = synthetic.turbulent_like(*shape, k, mach=3.0, seed=70 + k, high_amp=0.02, kmax_frac=0.125)
    a, b = _pair(shape, k, precision, flags, table, 30 + k)
    ua, ub = dev(u0, a), dev(u0, b)
    _steps_equal(a, b, ua, ub, 3, exact=_exact(flags, table), tol=TOL[precision])


def test_split_stage_launched_ahead():
    """The first stage of the next step queued behind the step (time step read from device
    memory, failure flag cleared by the mean-acceleration kernel) is split too."""
    shape, k = (24, 16, 16), 2
    print(f"split stages, launched ahead {shape}", flush=True)
    u0 = synthetic.turbulent_like(*shape, k, mach=3.0, seed=75, high_amp=0.02, kmax_frac=0.125)
    a, b = _pair(shape, k, FP64, FORCE, "shell", 35)
    ua, ub = dev(u0, a), dev(u0, b)
    _steps_equal(a, b, ua, ub, 4, ahead=True, exact=False, tol=TOL[FP64])


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_split_stage_limits_cells(precision):
    """A rough state whose first stage the limiter acts on (checked with the oracle's limiter
    on the oracle's first stage): the limited split stages equal the separate ones."""
    shape, k = (12, 12, 12), 2
    print(f"split stages with limited cells {shape} precision={precision}", flush=True)
    u0 = synthetic.turbulent_like(*shape, k, mach=4.0, seed=76, high_amp=0.35, kmax_frac=0.25)
    flags = FORCE
    modes = synthetic.forcing_table(36, amp=2.5)
    ocfg = oracle.Cfg(*shape, k, flags=flags)
    dt = 0.5 * oracle.dt_max(ocfg, u0)
    w1 = u0 + dt * oracle.rhs(ocfg, u0, dt, modes)
    _, nfail, theta = oracle.limit(ocfg, w1)
    print(f"oracle first stage: {int((theta < 1.0).sum())} limited cells, {nfail} failing", flush=True)
    assert nfail == 0 and (theta < 1.0).sum() > 0
    a, b = _pair(shape, k, precision, flags, "shell", 36)
    ua, ub = dev(u0, a), dev(u0, b)
    ra, da = dg.dg_rk_step_next(a, ua, dt, False)
    rb, db = dg.dg_rk_step_next(b, ub, dt, False)
    assert ra == rb == dg.DG_OK
    _compare(ua, ub, da, db, False, TOL[precision], "limited step")
    # without mean-free driving the two paths give the same bits
    a, b = _pair(shape, k, precision, BASE | dg.DG_FORCING, "shell", 36)
    ua, ub = dev(u0, a), dev(u0, b)
    ra, da = dg.dg_rk_step_next(a, ua, dt, False)
    rb, db = dg.dg_rk_step_next(b, ub, dt, False)
    assert ra == rb == dg.DG_OK
    _compare(ua, ub, da, db, True, 0.0, "limited step, mean kept")


def test_split_stage_failure_keeps_state():
    """A positivity failure raised in a split stage (first-stage cell means below the floor:
    a uniform state, whose right-hand side is zero, under the floor) fails the step in both
    forms, and u keeps u^n bit for bit."""
    k = 1
    u = np.zeros((4, 4, 8 * 6 * 4))
    u[0, 0] = 5e-4
    u[1, 0] = 2e-4
    for flags in (BASE | dg.DG_SPLIT_STAGE, BASE | dg.DG_SEPARATE_STAGE):
        ctx = make(8, 6, 4, k, flags)
        ud = dev(u, ctx)
        rc, dn = dg.dg_rk_step_next(ctx, ud, 1e-3, False)
        assert rc == dg.DG_RETRY and dn is None
        assert np.array_equal(ud.cpu().numpy(), u)


def _flat_params(seed):
    params = synthetic.mlp_params(seed)
    flat = np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)
    return torch.as_tensor(flat, device="cuda")


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_split_stage_learned_sensor(precision):
    """With the learned viscosity (the network's value per cell, plain sensor where it falls
    back) the split stages equal the separate ones."""
    n, k = 12, 2
    print(f"split stages, learned sensor {n}^3 precision={precision}", flush=True)
    flags = FORCE | dg.DG_LEARNED_SENSOR
    u0 = synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=77, high_amp=0.02, kmax_frac=0.125)
    a, b = _pair((n, n, n), k, precision, flags, "shell", 37)
    P = _flat_params(5)
    for c in (a, b):
        dg.dg_sensor_set_params(c, P)
    ua, ub = dev(u0, a), dev(u0, b)
    for c, ud in ((a, ua), (b, ub)):
        dg.dg_sensor_infer(c, ud)
    _steps_equal(a, b, ua, ub, 3, exact=False, tol=TOL[precision])


def test_split_stage_partials_across_a_table_upload():
    """A driving-table upload between two steps: the partials of the next step's first stage
    are formed from the new table (a stale sum would change the removed mean and the bits)."""
    shape, k = (16, 16, 16), 2
    print(f"split stages across a driving-table upload {shape}", flush=True)
    u0 = synthetic.turbulent_like(*shape, k, mach=3.0, seed=78, high_amp=0.02, kmax_frac=0.125)
    a, b = _pair(shape, k, FP64, FORCE, "shell", 38)
    ua, ub = dev(u0, a), dev(u0, b)
    _steps_equal(a, b, ua, ub, 2, exact=False, tol=TOL[FP64])
    modes = synthetic.forcing_table(39, amp=4.0)
    for c in (a, b):
        dg.dg_set_forcing(c, modes)
    dt = dg.dg_dt_max(a, ua)
    ra, da = dg.dg_rk_step_next(a, ua, dt, True)
    rb, db = dg.dg_rk_step_next(b, ub, dt, True)
    assert ra == rb == dg.DG_OK
    _compare(ua, ub, da, db, False, TOL[FP64], "after the upload")


def test_default_splits_large_fp64_meshes():
    """Without either flag a mesh of 2^22 cells in FP64 takes the split stages; they agree with
    the separate path."""
    shape, k = (256, 128, 128), 1
    print(f"default stage choice {shape} k={k} FP64", flush=True)
    u0 = synthetic.turbulent_like(64, 64, 64, k, mach=3.0, seed=79, high_amp=0.02, kmax_frac=0.125)
    u0 = np.tile(u0.reshape(4, -1, 64, 64, 64), (1, 1, 2, 2, 4)).reshape(4, u0.shape[1], -1)
    a, b = _pair(shape, k, FP64, FORCE, "shell", 40, split=0)
    ua, ub = dev(u0, a), dev(u0, b)
    del u0
    dg.dg_profile(a, 2)
    dg.dg_profile(b, 2)
    _steps_equal(a, b, ua, ub, 2, exact=False, tol=TOL[FP64])
    pa, pb = dg.dg_profile_read(a), dg.dg_profile_read(b)
    ta, tb = pa[2] / pa[3], pb[2] / pb[3]
    print(f"mean stage-kernel times: default {ta:.3f} ms, separate {tb:.3f} ms", flush=True)
    # the split's second kernel moves about a third of the stage kernel's bytes
    assert ta < 0.9 * tb


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_split_stage_step_matches_oracle(k, precision):
    """Split stages with mean-free driving on the driving shell (the modal partials) against
    the oracle's SSP-RK3 step, whole mesh (the two-lane FP64 degree-3 kernel keeps separate
    stages: that case checks the flag is accepted)."""
    shape = (24, 16, 16)
    print(f"split step vs oracle {shape} k={k} precision={precision}", flush=True)
    u0 = synthetic.turbulent_like(*shape, k, mach=3.0, seed=80 + k, high_amp=0.02, kmax_frac=0.125)
    if precision == FP32:
        u0 = u0.astype(np.float32).astype(np.float64)
    modes = synthetic.forcing_table(41 + k, amp=2.5)
    ocfg = oracle.Cfg(*shape, k, flags=FORCE)
    ctx = make(*shape, k, FORCE | dg.DG_SPLIT_STAGE, precision)
    dg.dg_set_forcing(ctx, modes)
    ud = dev(u0, ctx)
    dt = oracle.dt_max(ocfg, u0)
    rc, dt_next = dg.dg_rk_step_next(ctx, ud, dt, False)
    assert rc == dg.DG_OK
    ref, st = oracle.rk_step(ocfg, u0, dt, modes)
    assert st == oracle.OK
    assert_state_close(host(ud), ref, TOL[precision], "split step")
    d1 = oracle.dt_max(ocfg, ref)
    assert abs(dt_next - d1) <= TOL[precision] * d1


def test_default_stage_choice_by_mesh_size():
    """The default splits meshes of at least 2^21 cells in either precision, never the two-lane
    FP64 degree-3 configuration; the flags force either path."""
    for shape, k, precision, flags, want in [((64, 64, 64), 2, FP64, FORCE, False),
                                             ((128, 128, 128), 2, FP64, FORCE, True),
                                             ((128, 128, 128), 2, FP32, FORCE, True),
                                             ((128, 128, 127), 1, FP32, BASE, False),
                                             ((128, 128, 128), 3, FP64, FORCE, False),
                                             ((128, 128, 128), 3, FP32, FORCE, True),
                                             ((64, 64, 64), 2, FP64, FORCE | dg.DG_SPLIT_STAGE, True),
                                             ((128, 128, 128), 2, FP64, FORCE | dg.DG_SEPARATE_STAGE, False)]:
        ctx = make(*shape, k, flags, precision)
        assert dg.dg_split_stages(ctx) == want, (shape, k, precision, flags)
        ctx.close()
