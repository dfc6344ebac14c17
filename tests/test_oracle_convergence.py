"""Accuracy pins of the oracle that need time evolution (CPU).

* Smooth flow: a small plane sound wave converges as L1 ~ h^(k+1) (Sec. 2.2, eq. l1_norm
  and the statement that degree k gives spatial order k+1).  Amplitude 1e-6 keeps the
  O(A^2) nonlinearity below the discretisation error; meshes are quasi-1D (N x 1 x 1).
  For k = 3 the finest mesh is N = 16: at N = 32 the error (~5e-7 A) meets the
  nonlinear/round-off floor.
* Shocks: the isothermal shock tube (a dense slab in a periodic box) against the exact
  isothermal Riemann solution; L1 ~ N^-1 is expected for discontinuities (Sec. 7), with
  artificial viscosity and primitive projection on and no positivity retry.
Both with the Rusanov flux and with the HLLC-type flux, and with the per-order
Runge-Kutta choice (two stages at degree 1, five at degree 3).
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers.isothermal_riemann import sample, star_state


def _evolve(cfg, u, tend):
    t = 0.0
    nsteps = 0
    while t < tend - 1e-14:
        dt = min(oracle.dt_max(cfg, u), tend - t)
        u, st = oracle.rk_step(cfg, u, dt)
        assert st == oracle.OK
        t += dt
        nsteps += 1
    return u


@pytest.mark.parametrize("k,Ns,riemann", [(1, [8, 16, 32, 64], 0), (2, [8, 16, 32, 64], 0), (3, [4, 8, 16], 0),
                                          (1, [8, 16, 32, 64], oracle.HLLC), (2, [8, 16, 32], oracle.HLLC),
                                          (1, [8, 16, 32, 64], oracle.RK_BY_ORDER),
                                          (3, [4, 8, 16], oracle.RK_BY_ORDER)])
def test_sound_wave_convergence_order(k, Ns, riemann):
    amp, tend = 1e-6, 0.25
    errs = []
    f = synthetic.sound_wave(0, amp)
    for N in Ns:
        cfg = oracle.Cfg(N, 1, 1, k, flags=oracle.POS_LIMITER | riemann)
        u = oracle.project_function(cfg, f)
        u = _evolve(cfg, u, tend)
        nq = k + 3
        ex = f(oracle.points(cfg, nq), tend)
        errs.append(oracle.l1_error(cfg, nq, u, ex)[0] / amp)
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(slopes) >= k + 1 - 0.2, (errs, slopes)


def test_exact_riemann_helper_jump_conditions():
    rs, vs = star_state(1.0, 0.0, 0.1, 0.0)
    # right-moving shock into rho = 0.1: mass and momentum fluxes continuous in its frame
    S = 0.0 + np.sqrt(rs / 0.1)
    j1 = 0.1 * (0.0 - S)
    j2 = rs * (vs - S)
    assert abs(j1 - j2) < 1e-12
    assert abs((0.1 * (0 - S) ** 2 + 0.1) - (rs * (vs - S) ** 2 + rs)) < 1e-12
    # left rarefaction into rho = 1: Riemann invariant v + cs ln(rho) constant
    assert abs((vs + np.log(rs)) - (0.0 + np.log(1.0))) < 1e-12


@pytest.mark.parametrize("k,riemann", [(1, 0), (2, 0), (1, oracle.HLLC)])
def test_isothermal_shock_tube(k, riemann):
    tend = 0.1      # the two shocks meet at x = 0 only at t = 0.25/1.75
    errs = []
    for N in [32, 64, 128]:
        cfg = oracle.Cfg(N, 1, 1, k, flags=oracle.POS_LIMITER | oracle.AV | oracle.PRIM_PROJ | riemann)

        def ic(x):
            out = np.zeros((4,) + x.shape[:-1])
            xx = x[..., 0]
            out[0] = np.where((xx > 0.25) & (xx < 0.75), 1.0, 0.1)
            return out

        u = oracle.project_function(cfg, ic)
        u = _evolve(cfg, u, tend)
        nq = k + 3
        x = oracle.points(cfg, nq)[..., 0]
        r1, v1 = sample((x - 0.25) / tend, 0.1, 0.0, 1.0, 0.0)
        r2, v2 = sample((x - 0.75) / tend, 1.0, 0.0, 0.1, 0.0)
        rho = np.where(x < 0.5, r1, r2)
        v = np.where(x < 0.5, v1, v2)
        ex = np.zeros((4,) + x.shape)
        ex[0] = rho
        ex[1] = rho * v
        errs.append(oracle.l1_error(cfg, nq, u, ex))
        assert oracle.eval_points(cfg, nq, u[:1]).min() > 0.05
    e = [x[0] for x in errs]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(rates) > 0.8, (e, rates)
    assert e[-1] < 0.006
    em = [x[1] for x in errs]
    assert em[-1] < em[0]
