"""Pins of the oracle's HLLC-type interface flux (Sec. 2.2 uses Toro's HLLC; here its
isothermal counterpart: HLL for density and normal momentum, tangential momentum carried
by the mass flux with the upwind tangential velocity).

Checked against properties that fix it independently of its formula:
  * consistency F(u, u) = F(u);
  * supersonic upwinding: all waves moving right (left) give exactly F(u_L) (F(u_R));
  * reflection symmetry across the face;
  * a stationary shear layer (equal density, no normal velocity, a jump of the tangential
    velocity across cell faces) is an exact steady state of the whole scheme: the
    right-hand side vanishes, while the Rusanov flux diffuses the jump.
"""
import numpy as np
import pytest

import oracle


def _flux(d, u):
    F = np.zeros(4)
    F[0] = u[1 + d]
    F[1:] = u[1 + d] * u[1:] / u[0]
    F[1 + d] += u[0]
    return F


def test_consistency_and_reflection():
    rng = np.random.default_rng(1)
    for _ in range(30):
        d = int(rng.integers(3))
        u = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        np.testing.assert_allclose(oracle.hllc(d, 1.0, u, u), _flux(d, u), atol=1e-13)
        uL = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        uR = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3)])
        R = np.ones(4)
        R[1 + d] = -1.0
        a = oracle.hllc(d, 1.0, uL, uR)
        b = oracle.hllc(d, 1.0, R * uR, R * uL)
        np.testing.assert_allclose(b, -R * a, atol=1e-13)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_supersonic_upwinding(sign):
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = int(rng.integers(3))
        uL = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=3)])
        uR = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=3)])
        uL[1 + d] = sign * uL[0] * rng.uniform(1.1, 4.0)     # |v_n| > cs on both sides
        uR[1 + d] = sign * uR[0] * rng.uniform(1.1, 4.0)
        up = uL if sign > 0 else uR
        np.testing.assert_allclose(oracle.hllc(d, 1.0, uL, uR), _flux(d, up), atol=1e-13)


@pytest.mark.parametrize("k", [1, 2])
def test_stationary_shear_layer_is_steady(k):
    n = 6
    cfg_h = oracle.Cfg(n, n, 1, k, flags=oracle.POS_LIMITER | oracle.HLLC)
    cfg_r = oracle.Cfg(n, n, 1, k, flags=oracle.POS_LIMITER)

    def state(x):
        out = np.zeros((4,) + x.shape[:-1])
        out[0] = 1.3
        out[2] = 1.3 * np.where(x[..., 0] < 0.5, 0.7, -0.4)   # v_y jumps across x = 0.5 and x = 0
        return out

    u = oracle.project_function(cfg_h, state)
    Lh = oracle.rhs(cfg_h, u, 1e-3)
    assert np.abs(Lh).max() < 1e-12
    Lr = oracle.rhs(cfg_r, u, 1e-3)
    assert np.abs(Lr[2]).max() > 0.1            # Rusanov diffuses the tangential momentum
