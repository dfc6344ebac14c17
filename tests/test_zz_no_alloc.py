"""dg_dt_max_noalloc (the time step without a workspace, static device scratch) against
dg_dt_max, through the C ABI: two calls in a row, the second on a smaller mesh, in both
precisions, with the result on the host and in device memory; and from a context that has
no workspace at all, where dg_dt_max itself refuses."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic
from gpu_util import dev, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
FLAGS = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER


@pytest.mark.parametrize("precision", [dg.DG_FP64, dg.DG_FP32])
def test_noalloc_time_step_equals_dt_max_twice_in_a_row(precision):
    for shape, seed in (((40, 36, 30), 1), ((12, 10, 9), 2)):      # the second call is smaller
        print(f"no-alloc dt {shape} precision {precision}", flush=True)
        k = 2
        ctx = make(*shape, k, FLAGS, precision)
        u = dev(synthetic.turbulent_like(*shape, k, mach=4.0, seed=seed), ctx)
        want = dg.dg_dt_max(ctx, u)
        got = dg.dg_dt_max_noalloc(ctx, u)
        assert got == want, (got, want)
        dbuf = torch.full((1,), -1.0, dtype=torch.float64, device=ctx.device)
        dg.dg_dt_max_noalloc(ctx, u, out_dev=dbuf)
        torch.cuda.synchronize()
        assert float(dbuf.cpu()[0]) == want
        ctx.close()


def test_noalloc_time_step_without_a_workspace():
    """A context created through the C ABI with no workspace: dg_dt_max returns DG_ENOMEM,
    dg_dt_max_noalloc returns the time step of a context that has one, for two meshes."""
    L = dg._lib
    for shape, k, seed in (((33, 17, 9), 3, 4), ((7, 5, 3), 1, 5)):
        cfg = dg.dg_config()
        L.dg_config_default(ctypes.byref(cfg), *shape)
        cfg.degree = k
        cfg.flags = FLAGS
        cfg.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        h = ctypes.c_void_p()
        assert L.dg_init(ctypes.byref(cfg), ctypes.byref(h)) == dg.DG_OK
        try:
            ref = make(*shape, k, FLAGS)
            u = dev(synthetic.turbulent_like(*shape, k, mach=3.0, seed=seed), ref)
            want = dg.dg_dt_max(ref, u)
            out = ctypes.c_double(0.0)
            up = ctypes.c_void_p(u.data_ptr())
            assert L.dg_dt_max(h, up, ctypes.byref(out), 1) == dg.DG_ENOMEM
            assert L.dg_dt_max_noalloc(h, up, ctypes.byref(out), 1) == dg.DG_OK
            assert out.value == want, (out.value, want)
            ref.close()
        finally:
            L.dg_free(h)


def test_noalloc_rejects_what_it_cannot_do():
    L = dg._lib
    out = ctypes.c_double(0.0)
    assert L.dg_dt_max_noalloc(None, None, ctypes.byref(out), 1) == dg.DG_EINVAL
    ctx = make(8, 8, 8, 2, FLAGS | dg.DG_LEARNED_SENSOR)
    u = dev(synthetic.turbulent_like(8, 8, 8, 2, mach=3.0, seed=6), ctx)
    with pytest.raises(dg.DGError) as err:
        dg.dg_dt_max_noalloc(ctx, u)
    assert err.value.rc == dg.DG_EUNSUPPORTED
    ctx.close()
    # a mesh beyond the static scratch (65,536 blocks): refused before any launch
    big = dg.dg_config()
    L.dg_config_default(ctypes.byref(big), 256, 256, 257)
    big.degree = 1
    h = ctypes.c_void_p()
    assert L.dg_init(ctypes.byref(big), ctypes.byref(h)) == dg.DG_OK
    try:
        fake = torch.empty(8, dtype=torch.float64, device="cuda")     # never read: the size is refused first
        assert L.dg_dt_max_noalloc(h, ctypes.c_void_p(fake.data_ptr()), ctypes.byref(out), 1) == dg.DG_EINVAL
        assert b"static scratch" in L.dg_last_error(h)
    finally:
        L.dg_free(h)
    assert np.isfinite(out.value)
