"""The C ABI checks each device array it is handed against the allocation that holds it.

An array that would run past the end of its allocation is rejected with DG_EINVAL before
anything is launched, so the kernels never reach memory outside it; an array that ends
exactly at the allocation's end is accepted.  The calls go straight to the library
(no binding-side size check in between).  The arrays live in an allocation of the test's own
(hipMalloc), and every pointer handed over lies inside it, so nothing here can touch memory
that another array owns or that is not mapped.
"""
import ctypes

import numpy as np
import pytest
import torch

import synthetic
from gpu_util import dev, host, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
L = dg._lib


def _hip():
    # the HIP runtime already loaded in this process (shared with torch and the library)
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMemGetAddressRange.restype = ctypes.c_int
    h.hipMemGetAddressRange.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.c_void_p]
    h.hipMalloc.restype = ctypes.c_int
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.restype = ctypes.c_int
    h.hipFree.argtypes = [ctypes.c_void_p]
    return h


class Allocation:
    """One hipMalloc of `nbytes` and the extent the runtime reports for it."""

    def __init__(self, nbytes):
        self.hip = _hip()
        p = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(p), nbytes) == 0
        self.ptr = p.value
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        assert self.hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(self.ptr)) == 0
        assert base.value == self.ptr and size.value >= nbytes
        self.end = self.ptr + size.value

    def free(self):
        torch.cuda.synchronize()
        assert self.hip.hipFree(ctypes.c_void_p(self.ptr)) == 0


def test_state_arrays_past_the_end_of_their_allocation_are_rejected():
    n, k = 8, 2
    print("ABI extent checks 8^3 k=2 FP64", flush=True)
    ctx = make(n, n, n, k, dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER)
    sb = 4 * ctx.cfg.nb * ctx.cfg.ncell * 8
    a = Allocation(4 * sb)
    torch.cuda.synchronize()
    try:
        end = a.end - sb                        # a state that ends exactly at the allocation's end
        over = end + 512                        # the same state 512 bytes further: 512 bytes past it
        out = (ctypes.c_double * 4)()
        assert L.dg_conserved_sums(ctx.h, ctypes.c_void_p(end), out) == dg.DG_OK
        torch.cuda.synchronize()
        assert L.dg_conserved_sums(ctx.h, ctypes.c_void_p(over), out) == dg.DG_EINVAL
        msg = L.dg_last_error(ctx.h).decode()
        assert "overrun" in msg and "u:" in msg, msg

        # a state array that fits, with an output array that does not
        u = dev(synthetic.turbulent_like(n, n, n, k, mach=1.0, seed=61, high_amp=0.02), ctx)
        assert L.dg_rhs(ctx.h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(over), 1e-3) == dg.DG_EINVAL
        assert "dudt" in L.dg_last_error(ctx.h).decode()
        vhat = a.end - 3 * ctx.cfg.nb * ctx.cfg.ncell * 8
        assert L.dg_project_primitive(ctx.h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(vhat)) == dg.DG_OK
        assert L.dg_project_primitive(ctx.h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(vhat + 64)) \
            == dg.DG_EINVAL

        # a step on an array past the end is refused and writes nothing
        torch.cuda.synchronize()
        u_before = u.clone()
        st, dtn = ctypes.c_int(), ctypes.c_double()
        assert L.dg_rk_step_next(ctx.h, ctypes.c_void_p(over), 1e-3, 0, ctypes.byref(st), ctypes.byref(dtn)) \
            == dg.DG_EINVAL
        # the time step into a device scalar at the very end of the allocation
        dto = a.end - 8
        assert L.dg_dt_max(ctx.h, ctypes.c_void_p(u.data_ptr()), ctypes.cast(ctypes.c_void_p(dto), dg._dp), 0) \
            == dg.DG_OK
        torch.cuda.synchronize()
        assert torch.equal(u, u_before)

        # the context carries on: the same call with arrays that fit agrees with the binding's
        ref = dg.dg_conserved_sums(ctx, u)
        got = (ctypes.c_double * 4)()
        assert L.dg_conserved_sums(ctx.h, ctypes.c_void_p(u.data_ptr()), got) == dg.DG_OK
        assert list(got) == ref
        assert dg.dg_rk_step_next(ctx, u, dg.dg_dt_max(ctx, u), False)[0] == dg.DG_OK
        assert np.isfinite(host(u)).all()
    finally:
        a.free()


def test_workspace_shorter_than_its_stated_size_is_rejected():
    n, k = 8, 2
    ctx = make(n, n, n, k, dg.DG_AV)
    need = L.dg_workspace_bytes(ctx.h)
    a = Allocation(need + 4096)
    try:
        tail = (a.end - need // 2) & ~255       # 256-byte aligned, about half the workspace left
        assert L.dg_set_workspace(ctx.h, ctypes.c_void_p(tail), need) == dg.DG_EINVAL
        assert "workspace" in L.dg_last_error(ctx.h).decode()
        # the whole allocation is accepted
        assert L.dg_set_workspace(ctx.h, ctypes.c_void_p(a.ptr), need) == dg.DG_OK
        # and the context steps on it
        u = dev(synthetic.turbulent_like(n, n, n, k, mach=1.0, seed=62, high_amp=0.02), ctx)
        dt = dg.dg_dt_max(ctx, u)
        assert dg.dg_rk_step_next(ctx, u, dt, False)[0] == dg.DG_OK
        assert np.isfinite(host(u)).all()
        ctx.close()
    finally:
        a.free()
