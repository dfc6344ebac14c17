"""Pin of the oracle's per-cell right-hand side (``orc_rhs_cells``) to its whole-mesh one.

``orc_rhs_cells`` is what every full-size parity test compares against: it rebuilds the
projected velocity of each cell and of its six neighbours on demand and takes the removed
mean acceleration as an argument.  ``orc_rhs`` (pinned by the closed forms, conservation,
free-stream, convergence and shock-tube tests) projects the whole mesh first and computes
the mean acceleration itself.  Both evaluate the weight evolution of Sec. 2.2 cell by cell
with the same per-cell arithmetic, so on every cell of small meshes the two must agree bit
for bit: with mean-free driving (Sec. 4.2), viscosity (Sec. 3.1), projected or plain face
traces (Sec. 3.2), the HLLC-type flux, and the learned sensor's prescribed viscosity with
its fallback flags.  A stale neighbour projection, a wrong sign of the mean acceleration or
a dropped learned/fallback argument fails one of these cases.
"""
import numpy as np
import pytest

import oracle
import synthetic

FORCE = oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER | oracle.FORCING | oracle.FORCE_MEANFREE
MESH = (7, 5, 4)


def _state(k, seed, mach=4.0):
    return synthetic.turbulent_like(*MESH, k, mach=mach, seed=seed, high_amp=0.2)


def _all_cells_shuffled(cfg, seed):
    return np.random.default_rng(seed).permutation(cfg.ncell)


def _as_cells(full, cells):
    return np.transpose(full[:, :, cells], (2, 0, 1))         # [s][4][nb]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_rhs_cells_equals_rhs_with_meanfree_driving(k):
    cfg = oracle.Cfg(*MESH, k, flags=FORCE)
    u = _state(k, 100 + k)
    modes = synthetic.forcing_table(40 + k, amp=8.0)
    dt = 0.5 * oracle.dt_max(cfg, u)
    full = oracle.rhs(cfg, u, dt, modes)
    abar = oracle.forcing_mean(cfg, u, modes)
    assert np.abs(abar).max() > 1e-3                      # the removal is not a no-op here
    cells = _all_cells_shuffled(cfg, k)
    got = oracle.rhs_cells(cfg, u, cells, dt, modes, abar)
    assert np.array_equal(got, _as_cells(full, cells))
    # the mean acceleration is used, with its sign: a flipped or missing one differs
    assert not np.array_equal(oracle.rhs_cells(cfg, u, cells, dt, modes, -abar), got)
    assert not np.array_equal(oracle.rhs_cells(cfg, u, cells, dt, modes, None), got)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("flags", [oracle.AV | oracle.POS_LIMITER,
                                   oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER | oracle.HLLC,
                                   oracle.PRIM_PROJ | oracle.POS_LIMITER])
def test_rhs_cells_equals_rhs_without_driving(k, flags):
    cfg = oracle.Cfg(*MESH, k, flags=flags)
    u = _state(k, 200 + k + flags)
    dt = 0.5 * oracle.dt_max(cfg, u)
    full = oracle.rhs(cfg, u, dt)
    cells = _all_cells_shuffled(cfg, flags)
    assert np.array_equal(oracle.rhs_cells(cfg, u, cells, dt), _as_cells(full, cells))


def test_rhs_cells_equals_rhs_with_learned_viscosity_and_fallback():
    k = 2
    cfg = oracle.Cfg(*MESH, k, flags=oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER | oracle.LEARNED)
    u = _state(k, 300)
    nu = synthetic.random_nu(cfg.ncell, 7) * 1e-2
    fb = synthetic.random_fallback(cfg.ncell, 8)
    assert 0 < fb.sum() < cfg.ncell
    dt = 0.5 * oracle.dt_max(cfg, u, nu, fb)
    full = oracle.rhs(cfg, u, dt, None, nu, fb)
    cells = _all_cells_shuffled(cfg, 3)
    got = oracle.rhs_cells(cfg, u, cells, dt, None, None, nu, fb)
    assert np.array_equal(got, _as_cells(full, cells))
    # both arguments matter: without the flags every cell is learned, without nu none is
    assert not np.array_equal(oracle.rhs_cells(cfg, u, cells, dt, None, None, nu, None), got)
    assert not np.array_equal(oracle.rhs_cells(cfg, u, cells, dt, None, None, None, fb), got)


def test_rhs_cells_sample_with_repeats_and_corners():
    """A sample with repeated cells and the periodic corners, as the full-size tests draw."""
    k = 2
    cfg = oracle.Cfg(*MESH, k, flags=FORCE)
    u = _state(k, 400)
    modes = synthetic.forcing_table(9, amp=8.0)
    dt = 0.5 * oracle.dt_max(cfg, u)
    full = oracle.rhs(cfg, u, dt, modes)
    nx, ny, nz = MESH
    cells = np.array([0, nx - 1, nx * ny - 1, cfg.ncell - nx * ny, cfg.ncell - 1, 3, 3, 0])
    got = oracle.rhs_cells(cfg, u, cells, dt, modes, oracle.forcing_mean(cfg, u, modes))
    assert np.array_equal(got, _as_cells(full, cells))
