"""Pins of the FP64 reference of the learned-sensor network (CPU)."""
import math

import numpy as np

import synthetic
from oracle import mlp


def test_gelu_values():
    # GELU(z) = z Phi(z): Phi(0) = 1/2, Phi(1) = 0.8413447460685429 (normal CDF table)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + (1 - 0.8413447460685429)) < 1e-15
    z = np.linspace(-4, 4, 33)
    fd = (mlp.gelu(z + 1e-6) - mlp.gelu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(mlp.gelu_prime(z), fd, atol=1e-8)


def test_backward_matches_finite_differences():
    params = synthetic.mlp_params(3)
    rng = np.random.default_rng(0)
    x = rng.normal(size=(17, 20))
    t = rng.normal(size=17)
    grads = mlp.backward(params, x, t)
    worst = 0.0
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
                old = flat[idx]
                eps = 1e-4
                vals = []
                for sh in (2, 1, -1, -2):
                    flat[idx] = old + sh * eps
                    vals.append(mlp.loss(params, x, t))
                flat[idx] = old
                fd = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * eps)   # 4th-order central
                worst = max(worst, abs(fd - gf[idx]) / max(1e-6, abs(fd) + abs(gf[idx])))
    assert worst < 1e-7


def test_target_transform_roundtrip():
    nu = np.array([0.0, 1e-4, 1e-3, 0.3])
    np.testing.assert_allclose(mlp.inverse_target(mlp.target_transform(nu)), nu, atol=1e-15)
    assert abs(mlp.target_transform(np.array([1e-3]))[0] - math.log(2.0)) < 1e-15
