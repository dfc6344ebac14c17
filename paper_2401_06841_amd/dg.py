"""Thin ctypes binding of libdg (the C ABI in include/dg.h), same entry-point names.

Argument marshalling only: every step of the method runs in the HIP kernels of
libdg.so.  Device arrays are torch tensors on the current HIP device; the library
launches on torch's current stream.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg.so")

DG_OK, DG_RETRY = 0, 1
DG_EINVAL, DG_EUNSUPPORTED, DG_EHIP, DG_ENOMEM, DG_ESTATE = -1, -2, -3, -4, -5
DG_FP64, DG_FP32 = 0, 1
DG_AV, DG_PRIM_PROJ, DG_FORCING, DG_POS_LIMITER, DG_LEARNED_SENSOR, DG_FORCE_MEANFREE = 1, 2, 4, 8, 16, 32
DG_HLLC, DG_RK_BY_ORDER, DG_VOLUME_MFMA, DG_SEPARATE_STAGE, DG_SPLIT_STAGE = 64, 128, 256, 512, 1024
DG_MLP_NIN, DG_MLP_NHID = 20, 64
DG_MLP_NPARAM = 64 * 20 + 64 + 64 * 64 + 64 + 64 + 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdg.so not found at {LIB_PATH}: build it with `python -m paper_2401_06841_amd.build`")


class dg_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("degree", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("h", ctypes.c_double), ("cs", ctypes.c_double), ("cfl", ctypes.c_double),
                ("alpha_visc", ctypes.c_double), ("beta_visc", ctypes.c_double),
                ("rho_floor", ctypes.c_double), ("rho_floor_rel", ctypes.c_double), ("cfl_visc", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


_lib = ctypes.CDLL(LIB_PATH)
_vp, _dp, _ip, _lp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), \
    ctypes.POINTER(ctypes.c_long)
_SIGS = {
    "dg_config_default": (None, [ctypes.POINTER(dg_config), ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "dg_init": (ctypes.c_int, [ctypes.POINTER(dg_config), ctypes.POINTER(_vp)]),
    "dg_free": (None, [_vp]),
    "dg_last_error": (ctypes.c_char_p, [_vp]),
    "dg_set_wait_limit": (ctypes.c_int, [_vp, ctypes.c_double]),
    "dg_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "dg_split_stages": (ctypes.c_int, [_vp]),
    "dg_set_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "dg_set_forcing": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
    "dg_rhs": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double]),
    "dg_rk_step": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _ip]),
    "dg_dt_max": (ctypes.c_int, [_vp, _vp, _dp, ctypes.c_int]),
    "dg_dt_max_noalloc": (ctypes.c_int, [_vp, _vp, _dp, ctypes.c_int]),
    "dg_rk_step_next": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int, _ip, _dp]),
    "dg_rk_step_next_ahead": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_double, _ip, _dp]),
    "dg_project_primitive": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_limit": (ctypes.c_int, [_vp, _vp, _lp]),
    "dg_conserved_sums": (ctypes.c_int, [_vp, _vp, _dp]),
    "dg_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_profile_read": (ctypes.c_int, [_vp, _dp]),
    "dg_forcing_ou_ndraws": (ctypes.c_int, []),
    "dg_forcing_ou_init": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
    "dg_forcing_ou_advance": (ctypes.c_int, [_vp, _dp, ctypes.c_double]),
    "dg_forcing_get": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
    "dg_forcing_ou_get": (ctypes.c_int, [_vp, _dp]),
    "dg_forcing_ou_set": (ctypes.c_int, [_vp, _dp]),
    "dg_sensor_features": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_sensor_labels": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_sensor_targets": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_sensor_set_params": (ctypes.c_int, [_vp, _vp]),
    "dg_sensor_infer": (ctypes.c_int, [_vp, _vp]),
    "dg_sensor_judge": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _lp]),
    "dg_sensor_set_nu": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "dg_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "dg_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float]),
    "dg_sf_bins": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "dg_stats_scratch_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int]),
    "dg_structure_function": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_longlong, ctypes.c_ulonglong, _vp,
                                             ctypes.c_size_t, _dp]),
    "dg_spectrum_nshell": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_velocity_spectrum": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t, _dp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class DGError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"libdg error {rc}: {msg}")
        self.rc = rc


@dataclasses.dataclass
class Config:
    """Mirror of dg_config (defaults: alpha 2, beta 0.2, floor 1e-3 from Sec. 3.1; CFL 0.3)."""
    nx: int
    ny: int
    nz: int
    degree: int = 2
    precision: int = DG_FP64
    flags: int = DG_AV | DG_PRIM_PROJ | DG_POS_LIMITER
    h: float = 0.0
    cs: float = 1.0
    cfl: float = 0.3
    alpha_visc: float = 2.0
    beta_visc: float = 0.2
    rho_floor: float = 1e-3
    rho_floor_rel: float = 0.1
    cfl_visc: float = 0.1

    @property
    def nb(self):
        k = self.degree
        return (k + 1) * (k + 2) * (k + 3) // 6

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (4, self.nb, self.ncell)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(ctx, t, dtype, numel, name):
    """Reject a device buffer the kernels could overrun or misread: wrong dtype or device,
    not contiguous, or fewer than numel elements."""
    if t is None or t.dtype != dtype or not t.is_contiguous() or t.device != ctx.device or t.numel() < numel:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {ctx.device} with at least {numel} elements")


class Context:
    """Owns one dg_ctx and its workspace (a torch uint8 tensor on the current device)."""

    def __init__(self, cfg: Config, stream=None):
        import torch
        self.cfg = cfg
        self.dtype = torch.float64 if cfg.precision == DG_FP64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        c = dg_config(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.precision, cfg.flags, cfg.h, cfg.cs, cfg.cfl,
                      cfg.alpha_visc, cfg.beta_visc, cfg.rho_floor, cfg.rho_floor_rel, cfg.cfl_visc,
                      ctypes.c_void_p(stream.cuda_stream))
        h = ctypes.c_void_p()
        rc = _lib.dg_init(ctypes.byref(c), ctypes.byref(h))
        if rc != DG_OK:
            raise DGError(rc, "dg_init rejected the configuration")
        self.h = h
        n = _lib.dg_workspace_bytes(h)
        self.ws = torch.zeros(max(n, 256), dtype=torch.uint8, device=self.device)
        self._chk(_lib.dg_set_workspace(h, _ptr(self.ws), self.ws.numel()))

    def _chk(self, rc, ok=(DG_OK,)):
        if rc not in ok:
            raise DGError(rc, _lib.dg_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            _lib.dg_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_state(self, u, nvar=4):
        cfg = self.cfg
        if u.dtype != self.dtype or not u.is_contiguous() or u.device != self.device or \
                u.numel() != nvar * cfg.nb * cfg.ncell:
            raise ValueError("state must be a contiguous device tensor of shape [%d][nb][ncell] and dtype %s"
                             % (nvar, self.dtype))

    def empty_state(self, nvar=4):
        import torch
        return torch.empty((nvar, self.cfg.nb, self.cfg.ncell), dtype=self.dtype, device=self.device)


# ----------------------------------------------------------- C ABI mirror
def dg_init(cfg: Config, stream=None) -> Context:
    return Context(cfg, stream)


def dg_free(ctx: Context):
    ctx.close()


def dg_set_wait_limit(ctx: Context, seconds: float):
    """Wall-clock bound of the host wait for a fused step's published status (DG_EHIP when
    exceeded; synchronise the stream before using the state then)."""
    ctx._chk(_lib.dg_set_wait_limit(ctx.h, float(seconds)))


def dg_set_forcing(ctx: Context, modes):
    import numpy as np
    m = np.ascontiguousarray(modes, dtype=np.float64).reshape(-1, 9)
    ctx._chk(_lib.dg_set_forcing(ctx.h, m.ctypes.data_as(_dp), m.shape[0]))


def dg_rhs(ctx: Context, u, dudt, dt: float):
    ctx._check_state(u)
    ctx._check_state(dudt)
    ctx._chk(_lib.dg_rhs(ctx.h, _ptr(u), _ptr(dudt), float(dt)))


def dg_rk_step(ctx: Context, u, dt: float) -> int:
    """One SSP-RK3 step in place; returns DG_OK or DG_RETRY (u restored)."""
    ctx._check_state(u)
    st = ctypes.c_int(0)
    return ctx._chk(_lib.dg_rk_step(ctx.h, _ptr(u), float(dt), ctypes.byref(st)), ok=(DG_OK, DG_RETRY))


def dg_rk_step_next(ctx: Context, u, dt: float, reuse: bool):
    """One SSP-RK3 step in place that also returns the next time step; returns
    (DG_OK, dt_next) or (DG_RETRY, None) with u restored."""
    ctx._check_state(u)
    st = ctypes.c_int(0)
    dn = ctypes.c_double(0.0)
    rc = ctx._chk(_lib.dg_rk_step_next(ctx.h, _ptr(u), float(dt), 1 if reuse else 0, ctypes.byref(st),
                                       ctypes.byref(dn)), ok=(DG_OK, DG_RETRY))
    return rc, (dn.value if rc == DG_OK else None)


def dg_rk_step_next_ahead(ctx: Context, u, dt: float, reuse: bool, horizon: float):
    """dg_rk_step_next that, when the returned time step is below horizon, also launches the
    next step's first stage ahead (continued by the next call with that time step);
    returns (DG_OK, dt_next) or (DG_RETRY, None)."""
    ctx._check_state(u)
    st = ctypes.c_int(0)
    dn = ctypes.c_double(0.0)
    rc = ctx._chk(_lib.dg_rk_step_next_ahead(ctx.h, _ptr(u), float(dt), 1 if reuse else 0, float(horizon),
                                             ctypes.byref(st), ctypes.byref(dn)), ok=(DG_OK, DG_RETRY))
    return rc, (dn.value if rc == DG_OK else None)


def dg_dt_max(ctx: Context, u, out_dev=None) -> float:
    ctx._check_state(u)
    if out_dev is not None:
        ctx._chk(_lib.dg_dt_max(ctx.h, _ptr(u), ctypes.cast(ctypes.c_void_p(out_dev.data_ptr()), _dp), 0))
        return None
    v = ctypes.c_double()
    ctx._chk(_lib.dg_dt_max(ctx.h, _ptr(u), ctypes.byref(v), 1))
    return v.value


def dg_dt_max_noalloc(ctx: Context, u, out_dev=None) -> float:
    """dg_dt_max without the workspace: the library's static device scratch instead."""
    ctx._check_state(u)
    if out_dev is not None:
        _need(ctx, out_dev, torch.float64, 1, "out_dev")
        ctx._chk(_lib.dg_dt_max_noalloc(ctx.h, _ptr(u), ctypes.cast(ctypes.c_void_p(out_dev.data_ptr()), _dp), 0))
        return None
    v = ctypes.c_double()
    ctx._chk(_lib.dg_dt_max_noalloc(ctx.h, _ptr(u), ctypes.byref(v), 1))
    return v.value


def dg_project_primitive(ctx: Context, u, vhat):
    ctx._check_state(u)
    ctx._check_state(vhat, 3)
    ctx._chk(_lib.dg_project_primitive(ctx.h, _ptr(u), _ptr(vhat)))


def dg_limit(ctx: Context, u) -> int:
    ctx._check_state(u)
    n = ctypes.c_long()
    ctx._chk(_lib.dg_limit(ctx.h, _ptr(u), ctypes.byref(n)))
    return n.value


def dg_conserved_sums(ctx: Context, u):
    ctx._check_state(u)
    out = (ctypes.c_double * 4)()
    ctx._chk(_lib.dg_conserved_sums(ctx.h, _ptr(u), out))
    return list(out)


def dg_profile(ctx: Context, enable):
    """enable: False/0 off, True/1 the first stage's right-hand side of each step, 3 the last
    stage's right-hand side of each step, 2 every right-hand-side and stage launch."""
    ctx._chk(_lib.dg_profile(ctx.h, int(enable)))


def dg_split_stages(ctx: Context) -> bool:
    """Whether the context's steps split their stages (DG_SPLIT_STAGE or the default)."""
    r = _lib.dg_split_stages(ctx.h)
    if r < 0:
        ctx._chk(r)
    return bool(r)


def dg_profile_read(ctx: Context):
    """(rhs_ms_total, rhs_launches, stage_ms_total, stage_launches)."""
    out = (ctypes.c_double * 4)()
    ctx._chk(_lib.dg_profile_read(ctx.h, out))
    return out[0], int(out[1]), out[2], int(out[3])


def dg_forcing_ou_ndraws() -> int:
    return _lib.dg_forcing_ou_ndraws()


def dg_forcing_ou_init(ctx: Context, t_c: float, sigma: float):
    ctx._chk(_lib.dg_forcing_ou_init(ctx.h, float(t_c), float(sigma)))


def dg_forcing_ou_advance(ctx: Context, z, dt_drive: float):
    import numpy as np
    z = np.ascontiguousarray(z, dtype=np.float64)
    if z.size != dg_forcing_ou_ndraws():
        raise ValueError("wrong number of draws")
    ctx._chk(_lib.dg_forcing_ou_advance(ctx.h, z.ctypes.data_as(_dp), float(dt_drive)))


def dg_forcing_ou_get(ctx: Context):
    import numpy as np
    x = np.zeros(dg_forcing_ou_ndraws())
    ctx._chk(_lib.dg_forcing_ou_get(ctx.h, x.ctypes.data_as(_dp)))
    return x


def dg_forcing_ou_set(ctx: Context, x):
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != dg_forcing_ou_ndraws():
        raise ValueError("wrong OU state size")
    ctx._chk(_lib.dg_forcing_ou_set(ctx.h, x.ctypes.data_as(_dp)))


def dg_forcing_get(ctx: Context):
    import numpy as np
    out = np.zeros((64, 9))
    n = _lib.dg_forcing_get(ctx.h, out.ctypes.data_as(_dp), 64)
    return out[:n].copy()


def dg_sensor_features(ctx: Context, u, x):
    ctx._check_state(u)
    _need(ctx, x, torch.float32, ctx.cfg.ncell * DG_MLP_NIN, "x")
    ctx._chk(_lib.dg_sensor_features(ctx.h, _ptr(u), _ptr(x)))


def dg_sensor_labels(ctx: Context, u, nu):
    ctx._check_state(u)
    _need(ctx, nu, torch.float64, ctx.cfg.ncell, "nu")
    ctx._chk(_lib.dg_sensor_labels(ctx.h, _ptr(u), _ptr(nu)))


def dg_sensor_targets(ctx: Context, u, t):
    """Training targets log(1 + nu/1e-3) of the plain labels, float32 [ncell]."""
    ctx._check_state(u)
    _need(ctx, t, torch.float32, ctx.cfg.ncell, "t")
    ctx._chk(_lib.dg_sensor_targets(ctx.h, _ptr(u), _ptr(t)))


def dg_sensor_set_params(ctx: Context, params):
    _need(ctx, params, torch.float32, DG_MLP_NPARAM, "params")
    ctx._chk(_lib.dg_sensor_set_params(ctx.h, _ptr(params)))


def dg_sensor_infer(ctx: Context, u):
    ctx._check_state(u)
    ctx._chk(_lib.dg_sensor_infer(ctx.h, _ptr(u)))


def dg_sensor_judge(ctx: Context, u, tau: float) -> int:
    ctx._check_state(u)
    n = ctypes.c_long()
    ctx._chk(_lib.dg_sensor_judge(ctx.h, _ptr(u), float(tau), ctypes.byref(n)))
    return n.value


def dg_sensor_set_nu(ctx: Context, nu=None, fallback=None):
    if nu is not None:
        _need(ctx, nu, ctx.dtype, ctx.cfg.ncell, "nu")
    if fallback is not None:
        _need(ctx, fallback, torch.int32, ctx.cfg.ncell, "fallback")
    ctx._chk(_lib.dg_sensor_set_nu(ctx.h, _ptr(nu), _ptr(fallback)))


def dg_mlp_forward(ctx: Context, params, x, y):
    n = x.shape[0]
    _need(ctx, params, torch.float32, DG_MLP_NPARAM, "params")
    _need(ctx, x, torch.float32, n * DG_MLP_NIN, "x")
    _need(ctx, y, torch.float32, n, "y")
    ctx._chk(_lib.dg_mlp_forward(ctx.h, _ptr(params), _ptr(x), x.shape[0], _ptr(y)))


def dg_mlp_grad(ctx: Context, params, x, t, grad, loss):
    n = x.shape[0]
    _need(ctx, params, torch.float32, DG_MLP_NPARAM, "params")
    _need(ctx, x, torch.float32, n * DG_MLP_NIN, "x")
    _need(ctx, t, torch.float32, n, "t")
    _need(ctx, grad, torch.float32, DG_MLP_NPARAM, "grad")
    _need(ctx, loss, torch.float32, 1, "loss")
    ctx._chk(_lib.dg_mlp_grad(ctx.h, _ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(grad), _ptr(loss)))


def dg_mlp_adam(ctx: Context, params, grad, m, v, step: int, lr: float):
    for name, b in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _need(ctx, b, torch.float32, DG_MLP_NPARAM, name)
    ctx._chk(_lib.dg_mlp_adam(ctx.h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr)))


# ------------------------------------------------------------------ flow statistics
def _scratch(ctx: Context, nbytes: int, scratch):
    import torch
    if scratch is None:
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=ctx.device)
    _need(ctx, scratch, torch.uint8, nbytes, "scratch")
    return scratch


def dg_sf_bins(ctx: Context, nbins: int):
    out = np.zeros(nbins)
    ctx._chk(_lib.dg_sf_bins(ctx.h, int(nbins), out.ctypes.data_as(_dp)))
    return out


def dg_stats_scratch_bytes(ctx: Context, nbins: int = 0, p: int = 0) -> int:
    return int(_lib.dg_stats_scratch_bytes(ctx.h, int(nbins), int(p)))


def dg_structure_function(ctx: Context, u, nbins: int, npairs: int, seed: int, scratch=None):
    """S2(l_b) for the bins of dg_sf_bins (numpy array [nbins]); v(l) = sqrt(S2 / 2)."""
    ctx._check_state(u)
    scr = _scratch(ctx, dg_stats_scratch_bytes(ctx, nbins, 0), scratch)
    out = np.zeros(nbins)
    ctx._chk(_lib.dg_structure_function(ctx.h, _ptr(u), int(nbins), int(npairs), int(seed) & (2 ** 64 - 1),
                                        _ptr(scr), scr.numel(), out.ctypes.data_as(_dp)))
    return out


def dg_spectrum_nshell(ctx: Context, p: int) -> int:
    n = _lib.dg_spectrum_nshell(ctx.h, int(p))
    if n < 1:
        raise DGError(n, f"no spectrum for p = {p}")
    return n


def dg_velocity_spectrum(ctx: Context, u, p: int, scratch=None):
    """Shell-summed velocity power spectrum on the p-sample grid (numpy array)."""
    ctx._check_state(u)
    n = dg_spectrum_nshell(ctx, p)
    scr = _scratch(ctx, dg_stats_scratch_bytes(ctx, 0, p), scratch)
    out = np.zeros(n)
    ctx._chk(_lib.dg_velocity_spectrum(ctx.h, _ptr(u), int(p), _ptr(scr), scr.numel(), out.ctypes.data_as(_dp)))
    return out
