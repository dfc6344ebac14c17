"""Pins of the oracle's flow statistics (Sec. 4.3: the velocity structure function of the
scale-dependent velocity v(l), and the velocity power spectrum on the N p grid).

Each check compares the oracle with something it does not compute itself:
  * the published reference outputs of the SplitMix64 generator;
  * geometry of the pairs (periodic distance l, points inside the box) and isotropy of
    the directions (moments of the uniform distribution on the sphere);
  * exact zero for a uniform flow, and the closed form A^2 (1 - sin(2 pi l)/(2 pi l)) of a
    single sine wave averaged over positions and directions;
  * an independent evaluation (numpy Legendre polynomials) of the velocity of a few
    pairs on a small non-cubic mesh;
  * the grid layout and sub-point positions for per-cell linear velocities;
  * single Fourier modes and Parseval's identity for the shell spectrum.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import synthetic

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_splitmix64_reference_sequence():
    # first outputs of SplitMix64 seeded with 0 (Steele, Lea & Flood 2014, reference code)
    assert [oracle.splitmix64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                           0x06C45D188009454F]


def test_bins_span_resolution_limit_to_half_box():
    cfg = oracle.Cfg(16, 16, 16, 2)
    l = oracle.sf_bins(cfg, 100)
    lmin, lmax = (1.0 / 16) / 3, 0.5
    edges = lmin * (lmax / lmin) ** (np.arange(101) / 100.0)
    assert np.all(l > edges[:-1]) and np.all(l < edges[1:])
    assert np.allclose(l, np.sqrt(edges[:-1] * edges[1:]), rtol=1e-13)


def test_pairs_lie_at_distance_l_in_the_periodic_box():
    cfg = oracle.Cfg(6, 4, 5, 1)                     # box 1 x 2/3 x 5/6
    L = np.array([1.0, 4 / 6, 5 / 6])
    for pair, l in [(0, 0.01), (17, 0.2), (12345, 0.33), (99, 1e-4)]:
        x1, x2 = oracle.sf_pair(cfg, 11, pair, l)
        assert np.all((x1 >= 0) & (x1 < L)) and np.all((x2 >= 0) & (x2 < L))
        d = x2 - x1
        d -= L * np.round(d / L)                    # minimum image
        assert abs(np.linalg.norm(d) - l) < 1e-13


def test_directions_are_isotropic():
    cfg = oracle.Cfg(4, 4, 4, 1)
    n = 20000
    dirs = np.zeros((n, 3))
    for j in range(n):
        x1, x2 = oracle.sf_pair(cfg, 5, j, 0.1)
        d = x2 - x1
        dirs[j] = (d - np.round(d)) / 0.1
    sig = 1.0 / np.sqrt(n)
    assert np.all(np.abs(dirs.mean(0)) < 5 * sig * np.sqrt(1 / 3))
    second = dirs.T @ dirs / n
    # <n_i n_i> = 1/3 (variance of n_i^2 is 4/45), <n_i n_j> = 0 (variance 1/15)
    assert np.all(np.abs(np.diag(second) - 1 / 3) < 5 * sig * np.sqrt(4 / 45))
    off = second[~np.eye(3, dtype=bool)]
    assert np.all(np.abs(off) < 5 * sig * np.sqrt(1 / 15))


def test_uniform_flow_has_zero_structure_function():
    cfg = oracle.Cfg(5, 5, 5, 2)
    u = np.zeros(cfg.shape)
    u[0, 0] = 2.0
    u[1, 0], u[2, 0], u[3, 0] = 0.4, -1.0, 3.0
    s2 = oracle.structure_function(cfg, u, 8, 500, 3)
    assert np.all(s2 == 0.0)


def test_sine_wave_matches_closed_form():
    """v_x = A sin(2 pi x), rho = 1: <|dv|^2> over x is A^2 (1 - cos(2 pi l n_x)), and n_x of a
    uniform direction is uniform on [-1, 1], so S2 = A^2 (1 - sin(2 pi l) / (2 pi l))."""
    A = 0.7
    cfg = oracle.Cfg(16, 16, 16, 3)

    def f(x):
        one = np.ones(x.shape[:-1])
        return np.stack([one, A * np.sin(2 * np.pi * x[..., 0]), 0 * one, 0 * one])

    u = oracle.project_function(cfg, f)
    npairs, nbins = 40000, 12
    l = oracle.sf_bins(cfg, nbins)
    s2 = oracle.structure_function(cfg, u, nbins, npairs, 21)
    exact = A ** 2 * (1 - np.sin(2 * np.pi * l) / (2 * np.pi * l))
    # per-pair values 4 A^2 sin^2(theta/2) cos^2(.) have second moment <= 6 A^4
    tol = 5 * np.sqrt(6.0) * A ** 2 / np.sqrt(npairs) + 1e-4
    assert np.all(np.abs(s2 - exact) < tol), np.abs(s2 - exact).max()


# ---------------------------------------------------- independent evaluation of pairs
_G = 0x9E3779B97F4A7C15
_M = 2 ** 64 - 1


def _sm64(seed, i):
    z = (seed + (i + 1) * _G) & _M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M
    return z ^ (z >> 31)


def _u01(seed, i):
    return (_sm64(seed, i) >> 11) * 2.0 ** -53


def _pair(seed, pair, l, L):
    base = pair * 256
    x1 = np.array([_u01(seed, base + a) * L[a] for a in range(3)])
    n = np.array([0.0, 0.0, 1.0])
    for t in range(84):
        c = np.array([2.0 * _u01(seed, base + 3 + 3 * t + a) - 1.0 for a in range(3)])
        r2 = float(c @ c)
        if 1e-12 < r2 <= 1.0:
            n = c / np.sqrt(r2)
            break
    return x1, np.mod(x1 + l * n, L)


def _velocity(u, k, nxyz, h, x, floor):
    idx = [min(int(np.floor(x[a] / h)), nxyz[a] - 1) for a in range(3)]
    xi = [2.0 * (x[a] / h - idx[a]) - 1.0 for a in range(3)]
    c = idx[0] + nxyz[0] * (idx[1] + nxyz[1] * idx[2])
    vals = []
    for v in range(4):
        s = 0.0
        for l, (a, b, cc) in enumerate(oracle.basis_exps(k)):
            p = 1.0
            for e, t in zip((a, b, cc), xi):
                p *= np.sqrt(2 * e + 1) * npleg.legval(t, [0] * e + [1])
            s += u[v, l, c] * p
        vals.append(s)
    return np.array(vals[1:]) / max(vals[0], floor)


def test_pairs_match_an_independent_evaluation():
    nx, ny, nz, k = 4, 3, 5, 2
    cfg = oracle.Cfg(nx, ny, nz, k)                  # h = 1/4: box 1 x 3/4 x 5/4
    u = synthetic.turbulent_like(nx, ny, nz, k, mach=2.0, seed=9)
    nbins, npairs, seed = 4, 3, 77
    s2 = oracle.structure_function(cfg, u, nbins, npairs, seed)
    L = np.array([nx, ny, nz]) * cfg.h
    for b, l in enumerate(oracle.sf_bins(cfg, nbins)):
        acc = 0.0
        for j in range(npairs):
            x1, x2 = _pair(seed, b * npairs + j, l, L)
            d = _velocity(u, k, (nx, ny, nz), cfg.h, x1, 1e-3) - _velocity(u, k, (nx, ny, nz), cfg.h, x2, 1e-3)
            acc += float(d @ d)
        assert abs(s2[b] - acc / npairs) <= 1e-12 * max(1.0, acc / npairs)


def test_selected_bins_equal_the_full_measurement():
    cfg = oracle.Cfg(6, 6, 6, 1)
    u = synthetic.turbulent_like(6, 6, 6, 1, mach=1.0, seed=2)
    full = oracle.structure_function(cfg, u, 10, 300, 4)
    part = oracle.structure_function(cfg, u, 10, 300, 4, b0=3, nsel=4)
    assert np.array_equal(full[3:7], part)


# ------------------------------------------------------------------- grid and spectrum
def test_velocity_grid_layout_and_sub_points():
    nx, ny, nz, k, p = 3, 2, 4, 1, 3
    cfg = oracle.Cfg(nx, ny, nz, k)
    rng = np.random.default_rng(0)
    nc = nx * ny * nz
    c0, c1, c2 = rng.normal(size=(3, nc))
    u = np.zeros(cfg.shape)
    u[0, 0] = 1.5                                      # modes (000), (100), (010), (001)
    u[1, 0] = 1.5 * c0                                 # v_x = c0 + c1 sqrt(3) xi_x
    u[1, 1] = 1.5 * c1
    u[3, 2] = 1.5 * c2                                 # v_z = c2 sqrt(3) xi_y
    g = oracle.velocity_grid(cfg, u, p)
    assert g.shape == (3, nz * p, ny * p, nx * p)
    xs = -1.0 + (2.0 * np.arange(p) + 1.0) / p
    for gz in range(nz * p):
        for gy in range(ny * p):
            for gx in range(nx * p):
                c = gx // p + nx * (gy // p + ny * (gz // p))
                assert abs(g[0, gz, gy, gx] - (c0[c] + c1[c] * np.sqrt(3) * xs[gx % p])) < 1e-13
                assert abs(g[2, gz, gy, gx] - c2[c] * np.sqrt(3) * xs[gy % p]) < 1e-13
    assert np.all(g[1] == 0.0)


def test_spectrum_of_single_modes():
    Z, Y, X = 10, 8, 12
    z, y, x = np.meshgrid(np.arange(Z) / Z, np.arange(Y) / Y, np.arange(X) / X, indexing="ij")
    g = np.zeros((3, Z, Y, X))
    A, B = 0.8, 0.3
    g[0] = A * np.cos(2 * np.pi * 3 * x)                   # |kappa| = 3
    g[2] = B * np.sin(2 * np.pi * (2 * y + z))             # |kappa| = sqrt 5 -> shell 2
    e = oracle.power_spectrum(g)
    assert len(e) == oracle.spectrum_nshell(X, Y, Z)
    assert abs(e[3] - A ** 2 / 4) < 1e-14 and abs(e[2] - B ** 2 / 4) < 1e-14
    e[2] = e[3] = 0.0
    assert np.all(np.abs(e) < 1e-28)


def test_spectrum_parseval():
    rng = np.random.default_rng(3)
    g = rng.normal(size=(3, 7, 6, 9))
    e = oracle.power_spectrum(g)
    assert abs(e.sum() - 0.5 * (g ** 2).sum(0).mean()) < 1e-12
