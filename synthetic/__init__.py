"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and lays them out; it holds none of the DG method's
arithmetic (no basis, no quadrature, no fluxes, no projection), so a mistake here
cannot cancel between the two implementations that consume its arrays.

Workload recipes (the paper's runs are 3D periodic boxes of isothermal gas driven to
RMS Mach 0.1-12.8, Sec. 5 table of simulations; its data is not public, so these
stand in for it):
  * ``sound_wave``        -- small-amplitude plane sound wave (pointwise field).
  * ``turbulent_like``    -- modal state with log-normal density (width from the
                             Mach number) and a smooth random velocity field of the
                             requested RMS Mach number, with random high-order modes
                             of decaying amplitude (some cells dip below the density
                             floor at their Gauss points, some compress strongly).
  * ``forcing_table``     -- random driving modes on the shell 1 <= |n| <= 2, one per
                             +/- pair, with complex amplitudes perpendicular to n.
  * ``gaussian_draws``    -- standard normal numbers for the Ornstein-Uhlenbeck update.
  * ``mlp_params``        -- random sensor-network parameters rounded to bfloat16.
"""
from __future__ import annotations

import numpy as np


def nbasis(k: int) -> int:
    """Number of modes per variable of a total-degree-k expansion in 3D."""
    return (k + 1) * (k + 2) * (k + 3) // 6


def sound_wave(axis: int, amp: float = 1e-3, cs: float = 1.0, rho0: float = 1.0):
    """Plane sound wave rho = rho0 + amp sin(2 pi x_axis), m_axis = cs amp sin(2 pi x_axis).

    Returns f(x[..., 3], t=0) -> array [4, ...]; the exact linear solution travels at +cs.
    """
    def f(x, t=0.0):
        s = np.sin(2.0 * np.pi * (x[..., axis] - cs * t))
        out = np.zeros((4,) + x.shape[:-1])
        out[0] = rho0 + amp * s
        out[1 + axis] = cs * amp * s
        return out
    return f


def c1_axis(seed: int) -> int:
    """Propagation axis of the 16^3 sound-wave workload for a seed."""
    return int(np.random.default_rng(seed).integers(3))


def c1_modal_state(seed: int, n: int = 16, amp: float = 1e-3, cs: float = 1.0):
    """Degree-1 modal state [4][4][n^3] of the 16^3 sound-wave workload for throughput runs:
    each cell takes the wave's value at its centre as the mean and its local slope as the
    linear mode along the propagation axis (first-order Taylor form, not a projection).
    Cells are x fastest; modes in graded order (000), (100), (010), (001)."""
    axis = c1_axis(seed)
    h = 1.0 / n
    idx = np.indices((n, n, n))                          # [z, y, x] grids
    xc = (idx[2 - axis].reshape(-1) + 0.5) * h          # centre coordinate along the axis
    s = amp * np.sin(2.0 * np.pi * xc)
    ds = amp * 2.0 * np.pi * np.cos(2.0 * np.pi * xc) * h / (2.0 * np.sqrt(3.0))
    u = np.zeros((4, 4, n ** 3))
    u[0, 0] = 1.0 + s
    u[0, 1 + axis] = ds
    u[1 + axis, 0] = cs * s
    u[1 + axis, 1 + axis] = cs * ds
    return u


def _smooth(rng, shape, kmax: float, slope: float):
    """Unit-variance periodic random field on a grid (nz, ny, nx) with power ~ |k|^-slope, |k| <= kmax."""
    nz, ny, nx = shape
    noise = rng.standard_normal(shape)
    F = np.fft.rfftn(noise)
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    filt = np.where((kk > 0) & (kk <= kmax), np.maximum(kk, 1.0) ** (-slope / 2.0), 0.0)
    f = np.fft.irfftn(F * filt, s=shape, axes=(0, 1, 2))
    sd = f.std()
    return f / sd if sd > 0 else f


def turbulent_like(nx: int, ny: int, nz: int, k: int, mach: float, seed: int,
                   high_amp: float = 0.08, kmax_frac: float = 0.25, dtype=np.float64,
                   density_mach: float | None = None):
    """Random modal state [4][nb][ncell] resembling driven isothermal turbulence.

    Cell means: log-normal density with variance ln(1 + (M_rho/3)^2) (solenoidal driving),
    M_rho = density_mach if given else mach, velocity of RMS |v| = mach.  (A narrower
    density than the target Mach's keeps every cell mean of a large mesh above a density
    floor: at Mach 10 on 256^3 cells the full width reaches means of 1e-4.)  Higher modes: random density modes of relative amplitude
    high_amp/(1 + l/4) scaled by the local contrast, random velocity modes of amplitude
    high_amp/(1 + l/4) times the local speed, and momentum modes built as the first-order
    product of the two (m_l = v_mean rho_l + rho_mean v_l), so that the velocity m/rho stays
    bounded inside every cell while the point values vary.
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    kmax = max(2.0, min(nx, ny, nz) * kmax_frac)
    sig2 = np.log(1.0 + ((mach if density_mach is None else density_mach) / 3.0) ** 2)
    s = np.sqrt(sig2) * _smooth(rng, shape, kmax, 2.0)
    rho = np.exp(s - 0.5 * sig2)
    vel = [mach / np.sqrt(3.0) * _smooth(rng, shape, kmax, 2.0) for _ in range(3)]
    nb = nbasis(k)
    nc = nx * ny * nz
    u = np.zeros((4, nb, nc))
    r0 = rho.reshape(-1)
    v0 = [v.reshape(-1) for v in vel]
    u[0, 0] = r0
    for d in range(3):
        u[1 + d, 0] = r0 * v0[d]
    # local contrast: neighbour differences of the mean fields
    def contrast(f):
        c = np.zeros_like(f)
        for ax in range(3):
            c += np.abs(np.roll(f, 1, ax) - np.roll(f, -1, ax))
        return c.reshape(-1)
    crho = np.minimum(contrast(np.log(rho)) + 0.05, 1.0)
    vmag = np.sqrt(sum(v * v for v in vel)).reshape(-1) + 0.1
    for l in range(1, nb):
        a = high_amp / (1.0 + l / 4.0)
        rl = a * r0 * crho * rng.standard_normal(nc)
        u[0, l] = rl
        for d in range(3):
            vl = a * vmag * rng.standard_normal(nc)
            u[1 + d, l] = v0[d] * rl + r0 * vl
    return u.astype(dtype)


def shell_vectors():
    """Integer wave vectors with 1 <= |n| <= 2, one of each +/- pair (first non-zero component > 0)."""
    out = []
    for nx in range(-2, 3):
        for ny in range(-2, 3):
            for nz in range(-2, 3):
                n2 = nx * nx + ny * ny + nz * nz
                if not (1 <= n2 <= 4):
                    continue
                first = nx if nx != 0 else (ny if ny != 0 else nz)
                if first > 0:
                    out.append((nx, ny, nz))
    return np.array(out, dtype=np.float64)


def forcing_table(seed: int, amp: float = 1.0):
    """Driving-mode table [nmodes][9] = (n, Re/Im a_x, Re/Im a_y, Re/Im a_z) with a perpendicular to n."""
    rng = np.random.default_rng(seed)
    n = shell_vectors()
    tab = np.zeros((len(n), 9))
    tab[:, :3] = n
    for i, nv in enumerate(n):
        re = np.cross(nv, rng.standard_normal(3))
        im = np.cross(nv, rng.standard_normal(3))
        re *= amp / np.linalg.norm(nv)
        im *= amp / np.linalg.norm(nv)
        tab[i, 3::2] = re
        tab[i, 4::2] = im
    return tab


def forcing_table_general(seed: int, amp: float = 1.0):
    """Driving-mode table with wavevectors off the integer shell |n_a| <= 2: components of
    magnitude 3 and a non-integer one (a perpendicular to n as in forcing_table)."""
    rng = np.random.default_rng(seed)
    n = np.array([[3.0, 0.0, 1.0], [1.0, -3.0, 2.0], [0.5, 1.0, 0.0], [-2.0, 2.0, -3.0], [0.0, 1.0, -1.0]])
    tab = np.zeros((len(n), 9))
    tab[:, :3] = n
    for i, nv in enumerate(n):
        re = np.cross(nv, rng.standard_normal(3))
        im = np.cross(nv, rng.standard_normal(3))
        tab[i, 3::2] = re * amp / np.linalg.norm(nv)
        tab[i, 4::2] = im * amp / np.linalg.norm(nv)
    return tab


def gaussian_draws(seed: int, step: int, n: int):
    """n standard normal numbers for OU update number ``step`` of stream ``seed``."""
    rng = np.random.default_rng([seed, step])
    return rng.standard_normal(n)


def to_bf16(a):
    """Round float values to the nearest bfloat16 (ties to even); returns float32 values."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def mlp_params(seed: int, sizes=(20, 64, 64, 1)):
    """Random network parameters [(W [out,in], b [out]), ...] with bf16-representable weights."""
    rng = np.random.default_rng(seed)
    out = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = to_bf16(rng.standard_normal((fo, fi)) / np.sqrt(fi)).astype(np.float64)
        b = (0.1 * rng.standard_normal(fo)).astype(np.float32).astype(np.float64)
        out.append((W, b))
    return out


def random_nu(ncell: int, seed: int):
    """Per-cell learned-sensor viscosity values (mix of zeros, small and large)."""
    rng = np.random.default_rng(seed)
    nu = np.exp(rng.uniform(np.log(1e-5), np.log(0.5), ncell))
    nu[rng.random(ncell) < 0.3] = 0.0
    return nu


def random_fallback(ncell: int, seed: int, frac: float = 0.2):
    rng = np.random.default_rng(seed)
    return (rng.random(ncell) < frac).astype(np.int32)
