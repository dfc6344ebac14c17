"""FP64 numpy reference of the learned shock-sensor network (test infrastructure only).

Network: Linear(20,64) -> GELU -> Linear(64,64) -> GELU -> Linear(64,1), exact (erf)
GELU, mean-squared-error loss.  The network is not part of the paper; it stands in for
the compression sensor of Sec. 3.1 and is trained on that sensor's output.
Parameters are a list [(W [out, in], b [out]), ...] (y = W x + b per layer).
"""
from __future__ import annotations

import math

import numpy as np

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(params, x):
    """x [n, 20] -> (y [n], cache)."""
    a = np.asarray(x, dtype=np.float64)
    cache = [a]
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        if i < len(params) - 1:
            cache.append(z)
            a = gelu(z)
            cache.append(a)
        else:
            a = z
    return a[:, 0], cache


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, x, t):
    """Gradients of the mean-squared error: [(dW, db), ...] in the layout of params."""
    y, cache = forward(params, x)
    n = y.shape[0]
    g = (2.0 / n) * (y - t)[:, None]          # dL/dz of the last layer
    grads = [None] * len(params)
    # cache: [x, z1, a1, z2, a2]
    acts = [cache[0]] + [cache[2 * i + 2] for i in range(len(params) - 1)]
    pre = [cache[2 * i + 1] for i in range(len(params) - 1)]
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        a_in = acts[i]
        grads[i] = (g.T @ a_in, g.sum(axis=0))
        if i > 0:
            g = (g @ W) * gelu_prime(pre[i - 1])
    return grads


def target_transform(nu, nu0: float = 1e-3):
    """Training target t = log(1 + nu/nu0)."""
    return np.log1p(np.asarray(nu) / nu0)


def inverse_target(t, nu0: float = 1e-3):
    """Viscosity from a network output: nu = nu0 (exp(t) - 1), clipped at zero."""
    return np.maximum(nu0 * np.expm1(np.asarray(t)), 0.0)


def adam_update(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of array p in place; returns (m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return m, v
