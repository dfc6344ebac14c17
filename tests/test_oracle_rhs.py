"""Pins of the oracle's right-hand side, limiter, time step and stage update (CPU).

Each test checks the oracle against something other than itself: a closed form, an
invariant, a hand-computed example or a textbook identity, chosen so that a dropped
term, a wrong sign or index, or a transposed operand fails at least one of them.
Paper: Sec. 2.2 (weight evolution, numerical flux), Sec. 3.1 (von Neumann-Richtmyer
viscosity, Pi_max, positivity), Sec. 3.2 (primitive projection), Sec. 4.2 (driving),
Sec. 7 (CFL scaling, Runge-Kutta stages).
"""
import math
import os

import numpy as np
import pytest
from scipy.special import spherical_jn

import oracle
import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL = oracle.AV | oracle.PRIM_PROJ | oracle.POS_LIMITER


def _mode_index(k):
    return {tuple(e): i for i, e in enumerate(oracle.basis_exps(k))}


# ---------------------------------------------------------------- free stream
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("flags", [oracle.POS_LIMITER, ALL])
def test_uniform_state_is_preserved(k, flags):
    cfg = oracle.Cfg(3, 4, 5, k, flags=flags)
    u = np.zeros(cfg.shape)
    u[0, 0] = 1.7
    u[1:, 0] = np.array([0.9, -2.3, 0.4])[:, None]
    L = oracle.rhs(cfg, u, dt=1e-3)
    assert np.abs(L).max() < 1e-12


# -------------------------------------------------------------- conservation
@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_and_momentum_conserved_with_av(k):
    cfg = oracle.Cfg(6, 5, 4, k, flags=ALL)
    u = synthetic.turbulent_like(6, 5, 4, k, mach=3.0, seed=11)
    L = oracle.rhs(cfg, u, dt=2e-3)
    scale = np.abs(L[:, 0]).sum(axis=1)
    tot = L[:, 0].sum(axis=1)
    assert np.all(np.abs(tot) < 1e-13 * scale), (tot, scale)
    # the AV really acted: the same state without AV gives a different RHS
    cfg2 = oracle.Cfg(6, 5, 4, k, flags=oracle.PRIM_PROJ | oracle.POS_LIMITER)
    assert np.abs(oracle.rhs(cfg2, u, dt=2e-3) - L).max() > 1e-3


def test_forcing_mean_removal_conserves_momentum():
    k = 2
    flags = ALL | oracle.FORCING
    u = synthetic.turbulent_like(6, 6, 6, k, mach=2.0, seed=3)
    modes = synthetic.forcing_table(5, amp=3.0)
    raw = oracle.rhs(oracle.Cfg(6, 6, 6, k, flags=flags), u, 1e-3, modes)
    free = oracle.rhs(oracle.Cfg(6, 6, 6, k, flags=flags | oracle.FORCE_MEANFREE), u, 1e-3, modes)
    scale = np.abs(free[:, 0]).sum(axis=1)
    assert np.all(np.abs(free[:, 0].sum(axis=1)) < 1e-13 * scale)
    # without removal the driving injects net momentum rho a (mass-weighted mean != 0)
    assert np.abs(raw[1:, 0].sum(axis=1)).max() > 1e-3 * scale[1:].max()
    # the difference is exactly -abar * W_rho (the removed constant acceleration)
    abar = oracle.forcing_mean(oracle.Cfg(6, 6, 6, k, flags=flags), u, modes)
    for d in range(3):
        np.testing.assert_allclose(free[1 + d] - raw[1 + d], -abar[d] * u[0], atol=1e-12)
    np.testing.assert_allclose(free[0], raw[0], atol=0)


# ------------------------------------------------------------------- Rusanov
def test_rusanov_worked_example():
    vals = {}
    with open(os.path.join(GOLDEN, "rusanov_example.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, *v = line.split()
                vals[name] = np.array([float(x) for x in v])
    np.testing.assert_allclose(oracle.rusanov(0, 1.0, vals["uL"], vals["uR"]), vals["Fhat"], atol=1e-15)


def test_rusanov_consistency_and_reflection():
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = int(rng.integers(3))
        u = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        F = np.zeros(4)
        F[0] = u[1 + d]
        F[1:] = u[1 + d] * u[1:] / u[0]
        F[1 + d] += u[0]
        np.testing.assert_allclose(oracle.rusanov(d, 1.0, u, u), F, atol=1e-14)
        uL = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        uR = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        R = np.ones(4)
        R[1 + d] = -1.0
        a = oracle.rusanov(d, 1.0, uL, uR)
        b = oracle.rusanov(d, 1.0, R * uR, R * uL)
        np.testing.assert_allclose(b, -R * a, atol=1e-13)


# ------------------------------------------------------------- projection
@pytest.mark.parametrize("k", [1, 2, 3])
def test_projection_constant_density(k):
    """With rho constant the projected velocity is exactly W_m / rho (Sec. 3.2)."""
    cfg = oracle.Cfg(3, 3, 3, k, flags=ALL)
    u = synthetic.turbulent_like(3, 3, 3, k, mach=1.0, seed=1)
    u[0, 1:] = 0.0
    u[0, 0] = 2.5
    vh = oracle.project_primitive(cfg, u)
    np.testing.assert_allclose(vh, u[1:] / 2.5, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_projection_of_linear_field_closed_form(k):
    """Projecting f(x) = x gives W_0 = cell centre, W_(1,0,0) = (h/2)/sqrt(3), rest 0."""
    cfg = oracle.Cfg(4, 2, 3, k)
    w = oracle.project_function(cfg, lambda x: x[..., 0][None])
    idx = _mode_index(k)[(1, 0, 0)]
    i = np.arange(cfg.ncell) % 4
    np.testing.assert_allclose(w[0, 0], (i + 0.5) * cfg.h, atol=1e-15)
    np.testing.assert_allclose(w[0, idx], 0.5 * cfg.h / math.sqrt(3), atol=1e-15)
    rest = np.delete(w[0], [0, idx], axis=0)
    assert np.abs(rest).max() < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3])
def test_density_projection_is_identity(k):
    """Projecting a representable polynomial returns its coefficients (Sec. 3.2)."""
    cfg = oracle.Cfg(2, 3, 2, k)
    rng = np.random.default_rng(k)
    w = rng.normal(size=(1, cfg.nb, cfg.ncell))
    vals = oracle.eval_points(cfg, k + 1, w)
    back = oracle.project_values(cfg, k + 1, vals)
    np.testing.assert_allclose(back, w, atol=1e-13)


# --------------------------------------------------------- artificial viscosity
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("dt", [1.0, 1e-4])
def test_vnr_uniform_compression_closed_form(k, dt):
    """v = -gamma (x - x_K) inside every cell, rho const: div v = -3 gamma, Pi constant;
    the RHS difference AV-on minus AV-off is the volume term of Pi alone:
    dL_{m_d,(1,0,0)-like} = (1/(4h)) Pi Int d(phi)/dxi_d = 2 sqrt(2a+1) Pi / h for odd a."""
    N = 4
    gamma = 3.0
    rho0 = 1.3
    cfg_on = oracle.Cfg(N, N, N, k, flags=ALL)
    cfg_off = oracle.Cfg(N, N, N, k, flags=oracle.PRIM_PROJ | oracle.POS_LIMITER)
    u = np.zeros(cfg_on.shape)
    u[0, 0] = rho0
    idx = _mode_index(k)
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        u[1 + d, idx[e]] = -gamma * rho0 * 0.5 * cfg_on.h / math.sqrt(3)
    dL = oracle.rhs(cfg_on, u, dt) - oracle.rhs(cfg_off, u, dt)
    h = cfg_on.h
    hp = h / (k + 1)
    s = 3.0 * gamma
    pi = cfg_on.alpha * rho0 * hp * hp * s * s + cfg_on.beta * rho0 * cfg_on.cs * hp * s
    pi = min(pi, 0.5 * rho0 * hp * hp * s / dt)
    assert abs(oracle.vnr_pi(cfg_on, rho0, -s, dt) - pi) < 1e-14 * pi
    expect = np.zeros_like(dL)
    for d in range(3):
        for a in range(1, k + 1, 2):
            e = [0, 0, 0]
            e[d] = a
            expect[1 + d, idx[tuple(e)]] = 2.0 * math.sqrt(2 * a + 1) * pi / h
    np.testing.assert_allclose(dL, expect, atol=1e-10 * np.abs(expect).max())
    # expansion: no viscosity at all
    u2 = u.copy()
    u2[1:] *= -1.0
    assert np.abs(oracle.rhs(cfg_on, u2, dt) - oracle.rhs(cfg_off, u2, dt)).max() == 0.0


def test_vnr_pi_pieces():
    cfg = oracle.Cfg(8, 8, 8, 2)
    hp = cfg.h / 3
    # quadratic term alone (beta = 0) and linear term alone (alpha = 0)
    c = oracle.Cfg(8, 8, 8, 2, beta=0.0)
    assert abs(oracle.vnr_pi(c, 2.0, -5.0, 0.0) - 2.0 * 2.0 * hp * hp * 25.0) < 1e-15
    c = oracle.Cfg(8, 8, 8, 2, alpha=0.0)
    assert abs(oracle.vnr_pi(c, 2.0, -5.0, 0.0) - 0.2 * 2.0 * 1.0 * hp * 5.0) < 1e-15
    assert oracle.vnr_pi(cfg, 2.0, 5.0, 0.0) == 0.0
    assert oracle.vnr_pi(cfg, 2.0, 0.0, 1e-3) == 0.0
    # cap Pi_max = 0.5 rho (h/p)^2 |div v| / dt (Sec. 3.1)
    assert abs(oracle.vnr_pi(cfg, 2.0, -5.0, 1.0) - 0.5 * 2.0 * hp * hp * 5.0 / 1.0) < 1e-15
    assert oracle.vnr_pi(cfg, 2.0, -5.0, 1e-6) > 0.25


# ---------------------------------------------------------------- forcing
@pytest.mark.parametrize("n", [(1, 0, 0), (1, 1, 0), (0, -1, 2), (1, -1, 1)])
def test_forcing_source_matches_exact_projection(n):
    """rho uniform, m = 0, one driving mode: the momentum source is rho0 times the
    projection of a(x) = Re[ahat e^{2 pi i n.x}], whose exact value factorises into
    spherical Bessel functions: (1/2) Int e^{i w xi} Lt_a(xi) dxi = sqrt(2a+1) i^a j_a(w).
    The (k+1)-point rule approximates it: the 1D Gauss remainder for n = 3 points is
    2^7 (3!)^4 / (7 (6!)^3) max|f^(6)| ~ 6.4e-5 max|f^(6)|, and with w = pi h |n_a| <= 0.4
    and Lt_2 derivatives up to 3 sqrt(5) that stays below ~1e-3 of the amplitude; a
    wrong phase, sign or scale is an O(1) error."""
    k, N = 2, 16
    rho0 = 1.7
    cfg_f = oracle.Cfg(N, N, N, k, flags=oracle.FORCING | oracle.POS_LIMITER)
    cfg_0 = oracle.Cfg(N, N, N, k, flags=oracle.POS_LIMITER)
    nv = np.array(n, dtype=float)
    ahat = np.cross(nv, [0.3, -1.1, 0.7]) + 1j * np.cross(nv, [0.5, 0.2, -0.4])
    tab = np.zeros((1, 9))
    tab[0, :3] = nv
    tab[0, 3::2] = ahat.real
    tab[0, 4::2] = ahat.imag
    u = np.zeros(cfg_f.shape)
    u[0, 0] = rho0
    S = oracle.rhs(cfg_f, u, 0.0, tab) - oracle.rhs(cfg_0, u, 0.0)
    assert np.abs(S[0]).max() == 0.0
    h = cfg_f.h
    ijk = np.stack(np.unravel_index(np.arange(cfg_f.ncell), (N, N, N), order="F"), axis=1)
    xc = (ijk + 0.5) * h
    ph = np.exp(2j * np.pi * xc @ nv)
    exps = oracle.basis_exps(k)
    exact = np.zeros((3, cfg_f.nb, cfg_f.ncell))
    for l, e in enumerate(exps):
        fac = np.prod([math.sqrt(2 * e[a] + 1) * (1j ** e[a]) * spherical_jn(e[a], math.pi * h * nv[a])
                       for a in range(3)])
        for d in range(3):
            exact[d, l] = rho0 * np.real(ahat[d] * ph * fac)
    err = np.abs(S[1:] - exact).max()
    assert err < 1e-3 * np.abs(exact).max(), err
    assert np.abs(exact).max() > 0.5


# ------------------------------------------------------------------ time step
@pytest.mark.parametrize("k", [1, 2, 3])
def test_cfl_uniform_closed_form(k):
    cfg = oracle.Cfg(4, 4, 4, k, cfl=0.3)
    v0 = np.array([0.7, -1.9, 0.2])
    u = np.zeros(cfg.shape)
    u[0, 0] = 2.0
    u[1:, 0] = 2.0 * v0[:, None]
    dt = oracle.dt_max(cfg, u)
    assert abs(dt - 0.3 * cfg.h / ((k + 1) * (np.abs(v0).sum() + 3.0))) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("gamma", [0.5, 50.0])
def test_dt_viscous_bound_closed_form(k, gamma):
    """Uniform compression v = -gamma (x - x_K), rho const: the viscous pressure acts as a
    bulk viscosity nu = alpha (h/p)^2 (3 gamma) + beta cs (h/p); dt = min(advective CFL step
    (largest interior |v| sits at the outermost Gauss points), cfl_visc (h/p)^2 / nu)."""
    N = 4
    cfg = oracle.Cfg(N, N, N, k, flags=ALL, cfl_visc=0.1)
    idx = _mode_index(k)
    rho0 = 1.7
    u = np.zeros(cfg.shape)
    u[0, 0] = rho0
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        u[1 + d, idx[e]] = -gamma * rho0 * 0.5 * cfg.h / math.sqrt(3)
    h = cfg.h
    hp = h / (k + 1)
    gmax = oracle.gauss(k + 1)[0].max()
    dt_adv = 0.3 * h / ((k + 1) * 3 * (gamma * 0.5 * h * gmax + 1.0))
    nu = 2.0 * hp * hp * 3 * gamma + 0.2 * 1.0 * hp
    dt_visc = 0.1 * hp * hp / nu
    assert abs(oracle.dt_max(cfg, u) - min(dt_adv, dt_visc)) < 1e-14 * min(dt_adv, dt_visc)
    # expansion: no viscous bound; AV off: no viscous bound
    ue = u.copy()
    ue[1:] *= -1.0
    assert abs(oracle.dt_max(cfg, ue) - dt_adv) < 1e-14 * dt_adv
    cfg0 = oracle.Cfg(N, N, N, k, flags=oracle.PRIM_PROJ | oracle.POS_LIMITER, cfl_visc=0.1)
    assert abs(oracle.dt_max(cfg0, u) - dt_adv) < 1e-14 * dt_adv
    if gamma > 10:
        assert dt_visc < dt_adv


def test_ssprk3_stability_polynomial():
    cfg = oracle.Cfg(4, 4, 4, 2)
    assert oracle.rk_stages(cfg) == 3
    for k in (1, 2, 3):                              # third order for every degree by default
        assert oracle.rk_stages(oracle.Cfg(4, 4, 4, k)) == 3
    for lam in [-1.0, -7.3, 2.1, 0.0]:
        for dt in [0.01, 0.2, 0.4]:
            z = lam * dt
            assert abs(oracle.rk_linear(cfg, lam, dt, 1.3) - 1.3 * (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14


def test_rk_by_order_stability_polynomials():
    """With the per-order choice (k+1 evaluations per step, Sec. 7): degree 1 uses a
    two-stage scheme whose amplification factor is exactly 1 + z + z^2/2; degree 3 a
    five-stage scheme of order four, so its factor agrees with exp(z) up to z^4 and the
    remainder scales as z^5 (and is not zero: five stages cannot match exp(z) exactly)."""
    c1 = oracle.Cfg(4, 4, 4, 1, flags=oracle.RK_BY_ORDER)
    c2 = oracle.Cfg(4, 4, 4, 2, flags=oracle.RK_BY_ORDER)
    c3 = oracle.Cfg(4, 4, 4, 3, flags=oracle.RK_BY_ORDER)
    assert [oracle.rk_stages(c) for c in (c1, c2, c3)] == [2, 3, 5]
    for z in [-0.9, -0.3, 0.05, 0.7]:
        assert abs(oracle.rk_linear(c1, z, 1.0, 2.0) - 2.0 * (1 + z + z * z / 2)) < 1e-14
        assert abs(oracle.rk_linear(c2, z, 1.0, 2.0) - 2.0 * (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14

    def rem(z):
        taylor4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        return oracle.rk_linear(c3, z, 1.0, 1.0) - taylor4

    for z in [0.02, -0.02, 0.05]:
        ratio = rem(2 * z) / rem(z)
        assert abs(ratio - 32.0) < 0.5, (z, ratio)           # remainder ~ c z^5
    assert 1e-5 < abs(rem(0.05) / 0.05 ** 5) < 0.01


# -------------------------------------------------------------------- limiter
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("rel", [0.0, 0.1, 0.3])
def test_limiter_theta_closed_form(k, rel):
    """theta = (mean - target)/(mean - rho_min), target = max(floor, rel * mean): the mean is
    untouched, every high-order weight of all four variables is scaled by theta and the new
    minimum sits exactly on the target (linear x-profile: minimum on the low-x face)."""
    cfg = oracle.Cfg(2, 1, 1, k, flags=oracle.POS_LIMITER, rho_floor_rel=rel)
    idx = _mode_index(k)
    u = np.zeros(cfg.shape)
    u[0, 0] = 0.5
    u[1, 0] = 0.3
    u[0, idx[(1, 0, 0)], 0] = 0.4                 # rho = 0.5 + 0.4 sqrt(3) xi: min at the face
    u[1, idx[(1, 0, 0)], 0] = 0.2
    u[0, idx[(1, 0, 0)], 1] = 0.02                # second cell stays above every target
    lim, nfail, theta = oracle.limit(cfg, u)
    assert nfail == 0
    target = max(1e-3, rel * 0.5)
    rmin = 0.5 - 0.4 * math.sqrt(3)
    th = (0.5 - target) / (0.5 - rmin)
    assert abs(theta[0] - th) < 1e-15 and theta[1] == 1.0
    np.testing.assert_allclose(lim[:, 1:, 0], th * u[:, 1:, 0], atol=1e-16)
    assert np.all(lim[:, 0] == u[:, 0])           # means untouched
    assert np.all(lim[:, :, 1] == u[:, :, 1])
    vals = oracle.eval_points(cfg, k + 1, lim[:1])
    assert vals.min() >= target - 1e-15
    face = 0.5 - th * 0.4 * math.sqrt(3)          # new minimum sits exactly on the target
    assert abs(face - target) < 1e-15


def test_limiter_retry_and_step_restore():
    k = 1
    cfg = oracle.Cfg(4, 1, 1, k, flags=oracle.POS_LIMITER)
    u = np.zeros(cfg.shape)
    u[0, 0] = 1.0
    u[0, 0, 2] = 5e-4                              # mean below the floor
    _, nfail, _ = oracle.limit(cfg, u)
    assert nfail == 1
    out, st = oracle.rk_step(cfg, u, 1e-3)
    assert st == oracle.OK                        # inflow lifts the mean above the floor
    # a uniform state below the floor stays there: the step must ask for a retry
    low = np.zeros(cfg.shape)
    low[0, 0] = 5e-4
    low[1, 0] = 2e-4
    out, st = oracle.rk_step(cfg, low, 1e-3)
    assert st == oracle.RETRY
    assert np.array_equal(out, low)


# ------------------------------------------------------------------- symmetry
@pytest.mark.parametrize("k", [1, 2])
def test_axis_permutation_symmetry(k):
    """A sound wave along x, y or z gives RHS that are permutations of each other."""
    N = 6
    res = {}
    for axis in range(3):
        cfg = oracle.Cfg(N, N, N, k, flags=ALL)
        f = synthetic.sound_wave(axis, amp=0.05)
        u = oracle.project_function(cfg, f)
        res[axis] = (u, oracle.rhs(cfg, u, 1e-3))
    exps = oracle.basis_exps(k)
    idx = _mode_index(k)
    for axis in (1, 2):
        perm = [0, 1, 2]
        perm[0], perm[axis] = perm[axis], perm[0]   # swap x and the wave axis
        ux, Lx = res[0]
        ua, La = res[axis]
        cell = np.arange(N ** 3)
        ijk = np.stack(np.unravel_index(cell, (N, N, N), order="F"), axis=1)
        pc = np.ravel_multi_index(ijk[:, perm].T, (N, N, N), order="F")
        for v in range(4):
            vp = 0 if v == 0 else 1 + perm[v - 1]
            for l, e in enumerate(exps):
                lp = idx[tuple(np.array(e)[perm])]
                np.testing.assert_allclose(La[vp, lp, pc], Lx[v, l, cell], atol=1e-13)
                np.testing.assert_allclose(ua[vp, lp, pc], ux[v, l, cell], atol=1e-15)


def test_learned_mode_reduces_to_prescribed_viscosity():
    """With the learned flag, a compressed point uses Pi = rho nu s (s = -div v, nu the cell's
    bulk viscosity) capped by Pi_max of its own compression, an expanding point none, and a
    cell whose fallback flag is set the plain sensor."""
    k = 2
    cfg_l = oracle.Cfg(4, 4, 4, k, flags=ALL | oracle.LEARNED)
    cfg_p = oracle.Cfg(4, 4, 4, k, flags=ALL)
    cfg_0 = oracle.Cfg(4, 4, 4, k, flags=oracle.PRIM_PROJ | oracle.POS_LIMITER)
    u = synthetic.turbulent_like(4, 4, 4, k, mach=2.0, seed=9)
    nc = cfg_l.ncell
    L_plain = oracle.rhs(cfg_p, u, 1e-3)
    # everything on fallback -> plain sensor
    np.testing.assert_array_equal(oracle.rhs(cfg_l, u, 1e-3, nu=np.ones(nc), fallback=np.ones(nc)), L_plain)
    # anisotropic linear compression with a prescribed nu, no fallback: the divergence is
    # uniform, so Pi is constant in every cell and the RHS difference has the closed form
    # of the vNR test above
    idx = _mode_index(k)
    rho0 = 1.3
    gam = [3.0, -1.0, 0.5]                     # dv_d/dx_d = -gam_d, divergence -2.5
    uc = np.zeros(cfg_l.shape)
    uc[0, 0] = rho0
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        uc[1 + d, idx[e]] = -gam[d] * rho0 * 0.5 * cfg_l.h / math.sqrt(3)
    hp = cfg_l.h / (k + 1)
    s = sum(gam)
    for nu0, dt in [(0.01, 0.1), (0.01, 1.0), (5e-4, 0.1)]:   # the cap binds at dt = 1
        nu = np.full(nc, nu0)
        dL = oracle.rhs(cfg_l, uc, dt, nu=nu, fallback=np.zeros(nc)) - oracle.rhs(cfg_0, uc, dt)
        pi = min(rho0 * nu0 * s, 0.5 * rho0 * hp * hp * s / dt)
        expect = 2.0 * math.sqrt(3) * pi / cfg_l.h
        for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            np.testing.assert_allclose(dL[1 + d, idx[e]], expect, rtol=1e-10)
    # expanding everywhere: no viscosity whatever nu is
    ue = uc.copy()
    ue[1:] *= -1.0
    for nu0 in (5e-4, 0.05):
        dL = oracle.rhs(cfg_l, ue, 0.1, nu=np.full(nc, nu0), fallback=np.zeros(nc)) - oracle.rhs(cfg_0, ue, 0.1)
        assert np.abs(dL).max() == 0.0
    # zero mean divergence, compressed on one side: V_x = c phi_(200) gives
    # div v = (2/h) 3 sqrt(5) c xi_1, so (c > 0) only the Gauss layer xi_1 = -sqrt(3/5)
    # (1D weight 5/9) is compressed, at s = (2/h) 3 sqrt(5) c sqrt(3/5).  Without the cap
    # (dt = 0) Pi = rho0 nu s there; being a pressure it enters every momentum flux, so m_d
    # gains (1/(4h)) * 4 (5/9) Pi * d/dxi_d phi_l at that layer: sqrt(3) for the unit mode
    # e_d, 3 sqrt(5) xi_1 for (200) in m_x, 3 xi_1 for (110) in m_y and (101) in m_z.
    c, nu0 = 0.02, 0.03
    uz = np.zeros(cfg_l.shape)
    uz[0, 0] = rho0
    uz[1, idx[(2, 0, 0)]] = rho0 * c
    dL = oracle.rhs(cfg_l, uz, 0.0, nu=np.full(nc, nu0), fallback=np.zeros(nc)) - oracle.rhs(cfg_0, uz, 0.0)
    xm = math.sqrt(0.6)
    s_layer = (2.0 / cfg_l.h) * 3 * math.sqrt(5) * c * xm
    layer = 4.0 * (5.0 / 9.0) * rho0 * nu0 * s_layer / (4.0 * cfg_l.h)
    expect = np.zeros((4, cfg_l.nb))
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        expect[1 + d, idx[e]] = layer * math.sqrt(3)
    expect[1, idx[(2, 0, 0)]] = layer * 3 * math.sqrt(5) * (-xm)
    expect[2, idx[(1, 1, 0)]] = layer * 3 * (-xm)
    expect[3, idx[(1, 0, 1)]] = layer * 3 * (-xm)
    np.testing.assert_allclose(dL, np.broadcast_to(expect[:, :, None], dL.shape), rtol=0, atol=1e-12 * layer)
    # the same state with the cap binding: Pi = 1/2 rho0 (h/p)^2 s / dt at the layer
    dt = 1.0
    pcap = 0.5 * rho0 * hp * hp * s_layer / dt
    assert pcap < rho0 * nu0 * s_layer
    dL = oracle.rhs(cfg_l, uz, dt, nu=np.full(nc, nu0), fallback=np.zeros(nc)) - oracle.rhs(cfg_0, uz, dt)
    np.testing.assert_allclose(dL[1, idx[(1, 0, 0)]], layer * math.sqrt(3) * pcap / (rho0 * nu0 * s_layer),
                               rtol=1e-12)


def test_sensor_features_and_labels_closed_form():
    """Features of a cell with constant density and a linear velocity field v = v0 + G (x - x_K):
    the density-shape entries are W_rho,l / W_rho,0, the gradient block is G (h/p)/cs, the
    divergence slopes vanish and the last entry is |v0|/cs.  A quadratic velocity gives the
    slopes from the Legendre derivatives d/dxi Lt_2 = 3 sqrt(5) xi, Lt_1 d/dxi Lt_1 = 3 xi.
    The label of a uniformly compressing cell is the vNR bulk viscosity alpha (h/p)^2 s +
    beta cs (h/p); with slopes it is the omega s weighted mean of that viscosity over the
    compressed Gauss points, summed here by brute force over numpy's 3-point rule."""
    k, N = 2, 3
    cfg = oracle.Cfg(N, N, N, k, flags=ALL)
    idx = _mode_index(k)
    rng = np.random.default_rng(4)
    G = rng.normal(size=(3, 3))
    v0 = np.array([0.4, -1.2, 2.0])
    rho0 = 0.8
    u = np.zeros(cfg.shape)
    u[0, 0] = rho0
    for d in range(3):
        u[1 + d, 0] = rho0 * v0[d]
        for e, ex in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            u[1 + d, idx[ex]] = rho0 * G[d, e] * 0.5 * cfg.h / math.sqrt(3)
    x = oracle.sensor_features(cfg, u)
    hp = cfg.h / 3
    assert np.abs(x[:, :6]).max() == 0.0
    np.testing.assert_allclose(x[:, 6], math.log10(rho0), atol=1e-15)
    np.testing.assert_allclose(x[:, 7:16], np.tile((G * hp).reshape(-1), (cfg.ncell, 1)), atol=1e-14)
    assert np.abs(x[:, 16:19]).max() < 1e-14
    np.testing.assert_allclose(x[:, 19], np.linalg.norm(v0), atol=1e-14)
    u2 = u.copy()
    u2[0, 1:] = rng.normal(size=(cfg.nb - 1, cfg.ncell)) * 0.01
    x2 = oracle.sensor_features(cfg, u2)
    sel = [idx[e] for e in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2)]]
    np.testing.assert_allclose(x2[:, :6], (u2[0, sel] / rho0).T, atol=1e-15)
    # quadratic velocity modes (coefficients of V = m / rho0 in the basis)
    c = rng.normal(size=9)
    uq = u.copy()
    uq[1, idx[(2, 0, 0)]] = rho0 * c[0]
    uq[2, idx[(1, 1, 0)]] = rho0 * c[1]
    uq[3, idx[(1, 0, 1)]] = rho0 * c[2]
    uq[1, idx[(1, 1, 0)]] = rho0 * c[3]
    uq[2, idx[(0, 2, 0)]] = rho0 * c[4]
    uq[3, idx[(0, 1, 1)]] = rho0 * c[5]
    uq[1, idx[(1, 0, 1)]] = rho0 * c[6]
    uq[2, idx[(0, 1, 1)]] = rho0 * c[7]
    uq[3, idx[(0, 0, 2)]] = rho0 * c[8]
    r5 = 3 * math.sqrt(5)
    slopes = np.array([r5 * c[0] + 3 * c[1] + 3 * c[2], 3 * c[3] + r5 * c[4] + 3 * c[5],
                       3 * c[6] + 3 * c[7] + r5 * c[8]]) * 2.0 / cfg.h
    xq = oracle.sensor_features(cfg, uq)
    np.testing.assert_allclose(xq[:, 16:19], np.tile(slopes * hp, (cfg.ncell, 1)), rtol=1e-12)
    np.testing.assert_allclose(xq[:, 7:16], x[:, 7:16], atol=1e-14)
    trace = np.trace(G)
    xg, wg = np.polynomial.legendre.leggauss(3)
    num = den = 0.0
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                sq = -(trace + slopes[0] * xg[a] + slopes[1] * xg[b] + slopes[2] * xg[cc])
                if sq > 0:
                    w = wg[a] * wg[b] * wg[cc]
                    num += w * sq * (2.0 * hp * hp * sq + 0.2 * hp)
                    den += w * sq
    assert den > 0
    np.testing.assert_allclose(oracle.sensor_labels(cfg, uq), num / den, rtol=1e-10)
    # label: uniform compression at rate s per direction
    gamma = 2.0
    uc = np.zeros(cfg.shape)
    uc[0, 0] = rho0
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        uc[1 + d, idx[e]] = -gamma * rho0 * 0.5 * cfg.h / math.sqrt(3)
    s = 3 * gamma
    nu = 2.0 * hp * hp * s + 0.2 * hp
    np.testing.assert_allclose(oracle.sensor_labels(cfg, uc), nu, rtol=1e-12)
    ue = uc.copy()
    ue[1:] *= -1.0
    assert np.abs(oracle.sensor_labels(cfg, ue)).max() == 0.0


def test_learned_time_step_uses_the_cell_viscosity():
    """Uniform state with prescribed per-cell bulk viscosities: the viscous bound takes the
    largest nu of the learned cells; a fallback cell contributes its own (here none, the
    state is uniform)."""
    k, n = 2, 4
    cfg = oracle.Cfg(n, n, n, k, flags=ALL | oracle.LEARNED)
    u = np.zeros(cfg.shape)
    v0 = np.array([0.3, -0.2, 0.1])
    u[0, 0] = 1.0
    u[1:, 0] = v0[:, None]
    hp = cfg.h / (k + 1)
    dt_adv = cfg.cfl * cfg.h / ((k + 1) * (np.abs(v0).sum() + 3 * cfg.cs))
    assert oracle.dt_max(cfg, u) == pytest.approx(dt_adv, rel=1e-14)
    nu = np.zeros(cfg.ncell)
    nu[5] = 0.02
    nu[9] = 0.05
    fb = np.zeros(cfg.ncell)
    assert oracle.dt_max(cfg, u, nu, fb) == pytest.approx(min(dt_adv, cfg.cfl_visc * hp * hp / 0.05), rel=1e-14)
    fb[9] = 1
    assert oracle.dt_max(cfg, u, nu, fb) == pytest.approx(min(dt_adv, cfg.cfl_visc * hp * hp / 0.02), rel=1e-14)
