"""Helpers shared by the GPU tests (marshalling only)."""
import numpy as np
import torch

from paper_2401_06841_amd import dg


def make(nx, ny, nz, k, flags, precision=dg.DG_FP64, **kw):
    cfg = dg.Config(nx, ny, nz, degree=k, precision=precision, flags=flags, **kw)
    return dg.dg_init(cfg)


def dev(a, ctx):
    return torch.as_tensor(np.ascontiguousarray(a), device=ctx.device).to(ctx.dtype).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy()


def field_rel(a, b, ref):
    """Per-field relative L2 error (rho, |m| as a 3-vector) of a - b against ref."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    e_rho = np.linalg.norm(d[0]) / np.linalg.norm(r[0])
    e_m = np.linalg.norm(d[1:]) / np.linalg.norm(r[1:])
    return e_rho, e_m


def dof_rel(a, b, ref):
    """Per-field element-wise error: the largest |a - b| over the degrees of freedom of each
    field (rho; m over its three components) divided by the largest |ref| of that field."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    r = np.abs(np.asarray(ref, dtype=np.float64))
    return d[0].max() / r[0].max(), d[1:].max() / r[1:].max()


def assert_state_close(got, ref, tol, label=""):
    """Both bars of a state comparison: the per-field relative L2 norm and the per-DOF
    element-wise error (relative to the field's largest magnitude) are below tol, so that
    no single weight can be off by more than the tolerance of the whole field."""
    e = field_rel(got, ref, ref)
    m = dof_rel(got, ref, ref)
    print(f"{label} field L2 (rho, m) = {e[0]:.3e}, {e[1]:.3e}; per-DOF max = {m[0]:.3e}, {m[1]:.3e}", flush=True)
    assert max(e) < tol, (label, e)
    assert max(m) < tol, (label, m)
    return e, m
