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
