"""Exact solution of the isothermal Riemann problem (textbook isothermal gas dynamics).

Each wave is a shock when the star density exceeds the state it faces (jump relation
v* - v_K = -/+ cs (rho* - rho_K)/sqrt(rho* rho_K), speed v_K -/+ cs sqrt(rho*/rho_K)) or
a rarefaction otherwise (v* - v_K = -/+ cs ln(rho*/rho_K); inside the fan
rho = rho_K exp(-/+ (v - v_K)/cs)).  rho* solves f_L(rho*) + f_R(rho*) + v_R - v_L = 0.
Used only to pin the oracle's shock handling.
"""
import math

import numpy as np


def _f(rho, rk, cs):
    if rho > rk:
        return cs * (rho - rk) / math.sqrt(rho * rk)
    return cs * math.log(rho / rk)


def _df(rho, rk, cs):
    if rho > rk:
        return cs * (0.5 / math.sqrt(rho * rk) + 0.5 * rk / (rho * math.sqrt(rho * rk)))
    return cs / rho


def star_state(rl, vl, rr, vr, cs=1.0):
    rho = math.sqrt(rl * rr)
    for _ in range(200):
        g = _f(rho, rl, cs) + _f(rho, rr, cs) + vr - vl
        dg = _df(rho, rl, cs) + _df(rho, rr, cs)
        step = g / dg
        rho_new = rho - step
        if rho_new <= 0:
            rho_new = 0.5 * rho
        if abs(rho_new - rho) < 1e-15 * rho:
            rho = rho_new
            break
        rho = rho_new
    v = 0.5 * (vl + vr) + 0.5 * (_f(rho, rr, cs) - _f(rho, rl, cs))
    return rho, v


def sample(xi, rl, vl, rr, vr, cs=1.0):
    """(rho, v) at similarity coordinate xi = (x - x0)/t (array)."""
    rs, vs = star_state(rl, vl, rr, vr, cs)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    v = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= vs:  # left of contact: left wave
            if rs > rl:
                sl = vl - cs * math.sqrt(rs / rl)
                r, w = (rl, vl) if s < sl else (rs, vs)
            else:
                head, tail = vl - cs, vs - cs
                if s < head:
                    r, w = rl, vl
                elif s > tail:
                    r, w = rs, vs
                else:
                    w = s + cs
                    r = rl * math.exp(-(w - vl) / cs)
        else:
            if rs > rr:
                sr = vr + cs * math.sqrt(rs / rr)
                r, w = (rr, vr) if s > sr else (rs, vs)
            else:
                head, tail = vr + cs, vs + cs
                if s > head:
                    r, w = rr, vr
                elif s < tail:
                    r, w = rs, vs
                else:
                    w = s - cs
                    r = rr * math.exp((w - vr) / cs)
        rho[idx] = r
        v[idx] = w
    return rho, v
