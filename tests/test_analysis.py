"""The flow statistics used to compare runs (density PDF, velocity spectrum), checked on
states with known answers built by the oracle's projection."""
import numpy as np
import pytest

import oracle
from paper_2401_06841_amd import analysis


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mode_order_matches_the_oracle(k):
    assert [tuple(e) for e in oracle.basis_exps(k)] == analysis.modes(k)


def _state(n, k, f):
    cfg = oracle.Cfg(n, n, n, k)
    return oracle.project_function(cfg, f)


def test_density_pdf_of_uniform_and_two_level_states():
    n, k = 4, 2
    u = _state(n, k, lambda x: np.stack([np.full(x.shape[:-1], 10.0)] + [np.zeros(x.shape[:-1])] * 3))
    p = analysis.density_pdf(u, k)
    assert abs(p.sum() - 1) < 1e-12
    edges = np.linspace(-4, 3, 201)
    assert p[np.searchsorted(edges, 1.0, side="right") - 1] == pytest.approx(1.0)
    # half the box at rho = 0.1, half at rho = 1 (cell-aligned, so each cell is uniform)
    u2 = _state(n, k, lambda x: np.stack([np.where(x[..., 0] < 0.5, 0.1, 1.0)] + [np.zeros(x.shape[:-1])] * 3))
    p2 = analysis.density_pdf(u2, k)
    assert p2[np.searchsorted(edges, -1.0 + 1e-9, side="right") - 1] == pytest.approx(0.5)
    assert p2[np.searchsorted(edges, 0.0 + 1e-9, side="right") - 1] == pytest.approx(0.5)
    assert analysis.pdf_distance(p, p) == 0.0
    assert analysis.pdf_distance(p, p2) == pytest.approx(2.0)


def test_velocity_grid_reproduces_a_linear_field():
    n, k = 3, 2
    # rho = 1, m = (x, 2y, -z): linear, so representable exactly and v = m on the sub-grid
    u = _state(n, k, lambda x: np.stack([np.ones(x.shape[:-1]), x[..., 0], 2 * x[..., 1], -x[..., 2]]))
    v = analysis.velocity_grid(u, k, (n, n, n))
    p = k + 1
    g = (np.arange(n * p) + 0.5) / (n * p)
    assert np.allclose(v[0], g[None, None, :], atol=1e-12)
    assert np.allclose(v[1], 2 * g[None, :, None], atol=1e-12)
    assert np.allclose(v[2], -g[:, None, None], atol=1e-12)


def test_power_spectrum_single_mode_and_parseval():
    m = 24
    z, y, x = np.meshgrid(*(np.arange(m) / m,) * 3, indexing="ij")
    v = np.zeros((3, m, m, m))
    v[0] = 0.7 * np.sin(2 * np.pi * 3 * y)
    e = analysis.power_spectrum(v)
    assert e[3] == pytest.approx(0.25 * 0.49)
    assert abs(e.sum() - e[3]) < 1e-14
    rng = np.random.default_rng(0)
    w = rng.standard_normal((3, m, m, m))
    assert analysis.power_spectrum(w).sum() == pytest.approx(0.5 * (w ** 2).sum(0).mean())
    assert analysis.spectrum_distance(e + 1e-30, e + 1e-30, 5) == 0.0


def test_compare_of_a_state_with_itself():
    n, k = 4, 1
    u = _state(n, k, lambda x: np.stack([1 + 0.1 * np.sin(2 * np.pi * x[..., 0]), np.cos(2 * np.pi * x[..., 1]),
                                         0 * x[..., 0], 0 * x[..., 0]]))
    c = analysis.compare(u, u, k, (n, n, n))
    assert c["l2_rel_rho"] == 0.0 and c["density_pdf_l1"] == 0.0 and c["spectrum_log10_mean_abs"] == 0.0


def test_loglog_slope_of_power_laws():
    l = np.geomspace(0.01, 0.5, 40)
    assert analysis.loglog_slope(l, 3.0 * l ** 0.5, 0.1, 0.25) == pytest.approx(0.5, abs=1e-12)
    assert analysis.loglog_slope(l, 0.2 * l ** (1 / 3), 0.1, 0.25) == pytest.approx(1 / 3, abs=1e-12)
    assert np.isnan(analysis.loglog_slope(l, l, 0.3, 0.31))          # fewer than two points


def test_sonic_scale_of_a_power_law():
    l = np.geomspace(0.005, 0.5, 100)
    v = 4.0 * (l / 0.5) ** 0.5                       # M(l) = 1 at l = 0.5 / 16
    assert analysis.sonic_scale(l, v) == pytest.approx(0.5 / 16, rel=1e-12)
    assert analysis.sonic_scale(l, 0.5 * np.ones_like(l)) is None    # subsonic everywhere
    assert analysis.sonic_scale(l, 2.0 * np.ones_like(l)) is None    # supersonic at every bin


def test_spectrum_distance_ignores_shells_at_the_rounding_level():
    """Two velocity fields that agree to FP32 rounding: the smooth field has power in a few
    shells only, every other shell holds rounding noise (about 1e-30 of the peak in FP64,
    about 1e-14 after FP32 rounding).  Over all shells the mean log distance is of order 1;
    over the shells above the floor it is near 0, and so is the energy-weighted one.  A
    real difference (a mode's amplitude 10 % off) still shows."""
    m = 32
    z, y, x = np.meshgrid(*(np.arange(m) / m,) * 3, indexing="ij")
    v = np.zeros((3, m, m, m))
    v[0] = np.sin(2 * np.pi * y) + 0.3 * np.sin(2 * np.pi * 4 * z)
    v[1] = 0.5 * np.cos(2 * np.pi * 2 * x)
    w = v.astype(np.float32).astype(np.float64)
    ev, ew = analysis.power_spectrum(v), analysis.power_spectrum(w)
    a, b = ew[1:m // 2 + 1], ev[1:m // 2 + 1]
    ok = (a > 0) & (b > 0)
    assert np.mean(np.abs(np.log10(a[ok]) - np.log10(b[ok]))) > 0.5      # the unfiltered mean
    assert analysis.spectrum_distance(ew, ev, m // 2) < 1e-6
    assert analysis.spectrum_distance_energy_weighted(ew, ev, m // 2) < 1e-6
    assert analysis.spectrum_shells_used(ev, m // 2) == 3
    v2 = v.copy()
    v2[1] *= 1.1
    d = analysis.spectrum_distance(analysis.power_spectrum(v2), ev, m // 2)
    assert abs(d - np.log10(1.21) / 3) < 1e-9                                # one shell of three
