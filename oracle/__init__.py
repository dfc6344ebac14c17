"""Plain FP64 CPU oracle for the modal DG right-hand side of 3D isothermal Euler.

TEST INFRASTRUCTURE ONLY.  The arithmetic lives in ``orc.c`` (plain C loops, double
precision) and in ``mlp.py`` (numpy FP64 reference of the learned sensor network).
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library and never imports it.

Paper: Cernetic, Springel, Guillet & Pakmor (2024), "Supersonic turbulence
simulations with GPU-based high-order Discontinuous Galerkin hydrodynamics";
Sec. 2 (DG discretisation), Sec. 3 (artificial viscosity, primitive projection,
positivity), Sec. 4.2 (driving), Sec. 7 (cost model).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.environ.get("ORC_SO") or os.path.join(_HERE, "liborc.so")

AV = 1
PRIM_PROJ = 2
FORCING = 4
POS_LIMITER = 8
LEARNED = 16
FORCE_MEANFREE = 32
HLLC = 64
RK_BY_ORDER = 128

OK = 0
RETRY = 1


def build(verbose: bool = False) -> str:
    """Compile ``orc.c`` into ``liborc.so`` (gcc, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", _SO, os.path.join(_HERE, "orc.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, "orc.c")):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        cp = ctypes.POINTER(_Cfg)
        L.orc_leg.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_gauss.argtypes = [ctypes.c_int, dp, dp]
        L.orc_nbasis.argtypes = [ctypes.c_int]
        L.orc_basis_exps.argtypes = [ctypes.c_int, ip]
        L.orc_basis_eval.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_accel.argtypes = [dp, ctypes.c_int, dp, dp]
        L.orc_rusanov.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.orc_hllc.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.orc_vnr_pi.argtypes = [cp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_vnr_pi.restype = ctypes.c_double
        L.orc_project_primitive.argtypes = [cp, dp, dp]
        L.orc_forcing_mean.argtypes = [cp, dp, dp, ctypes.c_int, dp]
        L.orc_rhs.argtypes = [cp, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp, ip]
        L.orc_rhs_cells.argtypes = [cp, dp, ctypes.c_double, dp, ctypes.c_int, dp, dp, ip,
                                    ctypes.c_long, lp, dp]
        L.orc_dt_max.argtypes = [cp, dp]
        L.orc_dt_max.restype = ctypes.c_double
        L.orc_dt_max_learned.argtypes = [cp, dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.orc_dt_max_learned.restype = ctypes.c_double
        L.orc_limit.argtypes = [cp, dp, dp]
        L.orc_limit.restype = ctypes.c_long
        L.orc_rk_linear.argtypes = [cp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_rk_linear.restype = ctypes.c_double
        L.orc_rk_stages.argtypes = [cp]
        L.orc_rk_step.argtypes = [cp, dp, ctypes.c_double, dp, ctypes.c_int, dp, ip]
        L.orc_conserved_sums.argtypes = [cp, dp, dp]
        L.orc_points.argtypes = [cp, ctypes.c_int, dp]
        L.orc_project_values.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_eval_points.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_l1_error.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_sensor_features.argtypes = [cp, dp, dp]
        L.orc_sensor_labels.argtypes = [cp, dp, dp]
        u64 = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_splitmix64.restype = u64
        L.orc_sf_bins.argtypes = [cp, ctypes.c_int, dp]
        L.orc_sf_pair.argtypes = [cp, u64, u64, ctypes.c_double, dp, dp]
        L.orc_sf_pair.restype = None
        L.orc_velocity_at.argtypes = [cp, dp, dp, dp]
        L.orc_velocity_at.restype = None
        L.orc_structure_function.argtypes = [cp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_long,
                                             u64, dp]
        L.orc_velocity_grid.argtypes = [cp, dp, ctypes.c_int, dp]
        _lib = L
    return _lib


class _Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("k", ctypes.c_int),
                ("h", ctypes.c_double), ("cs", ctypes.c_double), ("cfl", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("rho_floor", ctypes.c_double),
                ("flags", ctypes.c_int), ("rho_floor_rel", ctypes.c_double), ("cfl_visc", ctypes.c_double)]


@dataclasses.dataclass
class Cfg:
    """Mesh and method parameters (defaults: Sec. 3.1 alpha=2, beta=0.2; floor 1e-3; the
    limiter aims at max(floor, rho_floor_rel * cell mean))."""
    nx: int
    ny: int
    nz: int
    k: int
    h: float = None
    cs: float = 1.0
    cfl: float = 0.3
    alpha: float = 2.0
    beta: float = 0.2
    rho_floor: float = 1e-3
    flags: int = POS_LIMITER
    rho_floor_rel: float = 0.1
    cfl_visc: float = 0.1

    def __post_init__(self):
        if self.h is None:
            self.h = 1.0 / self.nx

    @property
    def nb(self) -> int:
        return (self.k + 1) * (self.k + 2) * (self.k + 3) // 6

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (4, self.nb, self.ncell)

    def c(self):
        return ctypes.byref(_Cfg(self.nx, self.ny, self.nz, self.k, self.h, self.cs, self.cfl,
                                 self.alpha, self.beta, self.rho_floor, self.flags, self.rho_floor_rel,
                                 self.cfl_visc))


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _modes(modes):
    if modes is None:
        return None, 0
    m = _f64(modes).reshape(-1, 9)
    return m, m.shape[0]


# ------------------------------------------------------------------ 1D pieces
def leg(n: int, x: float):
    v, d = ctypes.c_double(), ctypes.c_double()
    lib().orc_leg(n, x, ctypes.byref(v), ctypes.byref(d))
    return v.value, d.value


def gauss(n: int):
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gauss(n, _d(x), _d(w))
    return x, w


def nbasis(k: int) -> int:
    return lib().orc_nbasis(k)


def basis_exps(k: int):
    e = np.zeros(3 * nbasis(k), dtype=np.int32)
    lib().orc_basis_exps(k, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return e.reshape(-1, 3)


def basis_eval(k: int, l: int, xi):
    xi = _f64(xi)
    phi = ctypes.c_double()
    d = np.zeros(3)
    lib().orc_basis_eval(k, l, _d(xi), ctypes.byref(phi), _d(d))
    return phi.value, d


def accel(modes, x):
    m, nm = _modes(modes)
    a = np.zeros(3)
    lib().orc_accel(_d(m), nm, _d(_f64(x)), _d(a))
    return a


def rusanov(d: int, cs: float, uL, uR):
    out = np.zeros(4)
    lib().orc_rusanov(d, cs, _d(_f64(uL)), _d(_f64(uR)), _d(out))
    return out


def hllc(d: int, cs: float, uL, uR):
    out = np.zeros(4)
    lib().orc_hllc(d, cs, _d(_f64(uL)), _d(_f64(uR)), _d(out))
    return out


def vnr_pi(cfg: Cfg, rho: float, divv: float, dt: float) -> float:
    return lib().orc_vnr_pi(cfg.c(), rho, divv, dt)


# ---------------------------------------------------------------- field ops
def project_primitive(cfg: Cfg, u):
    u = _f64(u)
    out = np.zeros((3, cfg.nb, cfg.ncell))
    _check(lib().orc_project_primitive(cfg.c(), _d(u), _d(out)))
    return out


def forcing_mean(cfg: Cfg, u, modes):
    m, nm = _modes(modes)
    out = np.zeros(3)
    _check(lib().orc_forcing_mean(cfg.c(), _d(_f64(u)), _d(m), nm, _d(out)))
    return out


def _nu_args(nu, fallback):
    nu_p = _d(_f64(nu)) if nu is not None else None
    fb = None
    if fallback is not None:
        fb_arr = np.ascontiguousarray(fallback, dtype=np.int32)
        fb = fb_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        return nu_p, fb, fb_arr
    return nu_p, fb, None


def rhs(cfg: Cfg, u, dt: float = 0.0, modes=None, nu=None, fallback=None):
    u = _f64(u)
    out = np.zeros(cfg.shape)
    m, nm = _modes(modes)
    nu_c = _f64(nu) if nu is not None else None
    fb = np.ascontiguousarray(fallback, dtype=np.int32) if fallback is not None else None
    _check(lib().orc_rhs(cfg.c(), _d(u), _d(out), dt, _d(m) if m is not None else None, nm,
                         _d(nu_c) if nu_c is not None else None,
                         fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if fb is not None else None))
    return out


def rhs_cells(cfg: Cfg, u, cells, dt: float = 0.0, modes=None, abar=None, nu=None, fallback=None):
    u = _f64(u)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 4, cfg.nb))
    m, nm = _modes(modes)
    ab = _f64(abar) if abar is not None else None
    nu_c = _f64(nu) if nu is not None else None
    fb = np.ascontiguousarray(fallback, dtype=np.int32) if fallback is not None else None
    _check(lib().orc_rhs_cells(cfg.c(), _d(u), dt, _d(m) if m is not None else None, nm,
                               _d(ab) if ab is not None else None,
                               _d(nu_c) if nu_c is not None else None,
                               fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if fb is not None else None,
                               len(cells), cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _d(out)))
    return out


def dt_max(cfg: Cfg, u, nu=None, fallback=None) -> float:
    """Time step; with the LEARNED flag and a per-cell viscosity nu, cells whose fallback
    flag is 0 use nu in the viscous bound."""
    if nu is None:
        return lib().orc_dt_max(cfg.c(), _d(_f64(u)))
    nu = _f64(nu)
    fb = np.ascontiguousarray(np.zeros(cfg.ncell) if fallback is None else fallback, dtype=np.int32)
    return lib().orc_dt_max_learned(cfg.c(), _d(_f64(u)), _d(nu), fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))


def limit(cfg: Cfg, u):
    """Returns (limited copy, number of failing cells, theta per cell)."""
    u = _f64(u).copy()
    theta = np.zeros(cfg.ncell)
    nfail = lib().orc_limit(cfg.c(), _d(u), _d(theta))
    return u, nfail, theta


def rk_linear(cfg: Cfg, lam: float, dt: float, u0: float) -> float:
    """One step of the configuration's Runge-Kutta scheme on du/dt = lam u."""
    return lib().orc_rk_linear(cfg.c(), lam, dt, u0)


def rk_stages(cfg: Cfg) -> int:
    return lib().orc_rk_stages(cfg.c())


def rk_step(cfg: Cfg, u, dt: float, modes=None, nu=None, fallback=None):
    """One SSP-RK3 step; returns (new state, status)."""
    u = _f64(u).copy()
    m, nm = _modes(modes)
    nu_c = _f64(nu) if nu is not None else None
    fb = np.ascontiguousarray(fallback, dtype=np.int32) if fallback is not None else None
    st = lib().orc_rk_step(cfg.c(), _d(u), dt, _d(m) if m is not None else None, nm,
                           _d(nu_c) if nu_c is not None else None,
                           fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if fb is not None else None)
    _check(st if st < 0 else 0)
    return u, st


def conserved_sums(cfg: Cfg, u):
    out = np.zeros(4)
    _check(lib().orc_conserved_sums(cfg.c(), _d(_f64(u)), _d(out)))
    return out


def points(cfg: Cfg, nq: int):
    out = np.zeros((cfg.ncell, nq ** 3, 3))
    _check(lib().orc_points(cfg.c(), nq, _d(out)))
    return out


def project_values(cfg: Cfg, nq: int, vals):
    vals = _f64(vals)
    nvar = vals.shape[0]
    out = np.zeros((nvar, cfg.nb, cfg.ncell))
    _check(lib().orc_project_values(cfg.c(), nq, nvar, _d(vals), _d(out)))
    return out


def eval_points(cfg: Cfg, nq: int, w):
    w = _f64(w)
    nvar = w.shape[0]
    out = np.zeros((nvar, cfg.ncell, nq ** 3))
    _check(lib().orc_eval_points(cfg.c(), nq, nvar, _d(w), _d(out)))
    return out


def l1_error(cfg: Cfg, nq: int, w, exact):
    w = _f64(w)
    exact = _f64(exact)
    nvar = w.shape[0]
    out = np.zeros(nvar)
    _check(lib().orc_l1_error(cfg.c(), nq, nvar, _d(w), _d(exact), _d(out)))
    return out


def project_function(cfg: Cfg, f, nq: int = None):
    """Project f(x[...,3]) -> array[nvar, ...] onto the basis with a (k+3)-point rule."""
    nq = nq or cfg.k + 3
    x = points(cfg, nq)
    vals = np.asarray(f(x), dtype=np.float64)  # [nvar, ncell, nq^3]
    return project_values(cfg, nq, vals)


def sensor_features(cfg: Cfg, u):
    out = np.zeros((cfg.ncell, 20))
    _check(lib().orc_sensor_features(cfg.c(), _d(_f64(u)), _d(out)))
    return out


def sensor_labels(cfg: Cfg, u):
    out = np.zeros(cfg.ncell)
    _check(lib().orc_sensor_labels(cfg.c(), _d(_f64(u)), _d(out)))
    return out


# ------------------------------------------------------------- flow statistics
# Sec. 4.3: velocity structure function S2(l) = <|v(x) - v(x + l n)|^2>, v(l) = sqrt(S2/2),
# and the velocity power spectrum on the N p grid (the readings are listed in orc.c).

def splitmix64(seed: int, i: int) -> int:
    """Draw i of the counter-based SplitMix64 stream `seed` (64-bit unsigned)."""
    return int(lib().orc_splitmix64(seed & (2 ** 64 - 1), i & (2 ** 64 - 1)))


def sf_bins(cfg: Cfg, nbins: int):
    out = np.zeros(nbins)
    _check(lib().orc_sf_bins(cfg.c(), nbins, _d(out)))
    return out


def sf_pair(cfg: Cfg, seed: int, pair: int, l: float):
    x1, x2 = np.zeros(3), np.zeros(3)
    lib().orc_sf_pair(cfg.c(), seed, pair, float(l), _d(x1), _d(x2))
    return x1, x2


def velocity_at(cfg: Cfg, u, x):
    u = _f64(u)
    x = _f64(x)
    v = np.zeros(3)
    lib().orc_velocity_at(cfg.c(), _d(u), _d(x), _d(v))
    return v


def structure_function(cfg: Cfg, u, nbins: int, npairs: int, seed: int, b0: int = 0, nsel: int = None):
    """S2 of bins b0 .. b0+nsel-1 (default all) of an nbins-bin measurement."""
    nsel = nbins - b0 if nsel is None else nsel
    l = sf_bins(cfg, nbins)
    out = np.zeros(nsel)
    _check(lib().orc_structure_function(cfg.c(), _d(_f64(u)), nbins, b0, nsel, _d(l), npairs, seed, _d(out)))
    return out


def velocity_grid(cfg: Cfg, u, p: int):
    out = np.zeros((3, cfg.nz * p, cfg.ny * p, cfg.nx * p))
    _check(lib().orc_velocity_grid(cfg.c(), _d(_f64(u)), p, _d(out)))
    return out


def power_spectrum(grid):
    """Shell sums of 1/2 |v_hat|^2 with v_hat = FFT(v) / (number of points) over integer
    shells |kappa| in [K - 1/2, K + 1/2) (kappa in box wavenumber units); index K of the
    result; sum over K = 1/2 <|v|^2>."""
    grid = np.asarray(grid, dtype=np.float64)
    Z, Y, X = grid.shape[1:]
    vh = np.fft.fftn(grid, axes=(1, 2, 3)) / (X * Y * Z)
    e = 0.5 * (np.abs(vh) ** 2).sum(0)
    fz = np.fft.fftfreq(Z, 1.0 / Z)[:, None, None]
    fy = np.fft.fftfreq(Y, 1.0 / Y)[None, :, None]
    fx = np.fft.fftfreq(X, 1.0 / X)[None, None, :]
    shell = np.floor(np.sqrt(fx ** 2 + fy ** 2 + fz ** 2) + 0.5).astype(np.int64)
    return np.bincount(shell.reshape(-1), weights=e.reshape(-1), minlength=spectrum_nshell(X, Y, Z))


def spectrum_nshell(X: int, Y: int, Z: int) -> int:
    """Number of integer shells K = 0 .. Kmax of an X x Y x Z grid."""
    return int(np.floor(np.sqrt((X // 2) ** 2 + (Y // 2) ** 2 + (Z // 2) ** 2) + 0.5)) + 1


def velocity_spectrum(cfg: Cfg, u, p: int):
    return power_spectrum(velocity_grid(cfg, u, p))


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed with status {rc}")
