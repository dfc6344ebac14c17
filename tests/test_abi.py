"""The C ABI library loads on the CPU host and exports every symbol include/dg.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_all_declared_symbols():
    so = os.path.join(ROOT, "paper_2401_06841_amd", "libdg.so")
    assert os.path.exists(so), "build libdg.so first (python -m paper_2401_06841_amd.build)"
    lib = ctypes.CDLL(so)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_abi():
    from paper_2401_06841_amd import dg
    assert sorted(dg.EXPORTED) == _declared()


def test_config_default_and_rejections_without_gpu():
    from paper_2401_06841_amd import dg
    c = dg.dg_config()
    dg._lib.dg_config_default(ctypes.byref(c), 16, 16, 16)
    assert (c.degree, c.precision, c.cfl, c.alpha_visc, c.beta_visc, c.rho_floor) == (2, 0, 0.3, 2.0, 0.2, 1e-3)
    h = ctypes.c_void_p()
    c.degree = 4
    assert dg._lib.dg_init(ctypes.byref(c), ctypes.byref(h)) == dg.DG_EUNSUPPORTED
    c.degree = 2
    c.nx = 0
    assert dg._lib.dg_init(ctypes.byref(c), ctypes.byref(h)) == dg.DG_EINVAL
    c.nx = 16
    c.flags = 2048                                # no such flag
    assert dg._lib.dg_init(ctypes.byref(c), ctypes.byref(h)) == dg.DG_EINVAL
    c.flags = dg.DG_SEPARATE_STAGE | dg.DG_SPLIT_STAGE   # separate and split stages at once
    assert dg._lib.dg_init(ctypes.byref(c), ctypes.byref(h)) == dg.DG_EINVAL
    assert dg._lib.dg_forcing_ou_ndraws() == 96


def test_entry_points_reject_a_null_context_without_gpu():
    """Every entry point that takes a context returns DG_EINVAL for a null one (no device
    call is made), including the flow-statistics calls."""
    from paper_2401_06841_amd import dg
    L = dg._lib
    buf = (ctypes.c_double * 8)()
    dp = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    assert L.dg_sf_bins(None, 4, dp) == dg.DG_EINVAL
    assert L.dg_stats_scratch_bytes(None, 100, 3) == 0
    assert L.dg_spectrum_nshell(None, 3) == dg.DG_EINVAL
    assert L.dg_structure_function(None, None, 4, 10, 1, None, 0, dp) == dg.DG_EINVAL
    assert L.dg_velocity_spectrum(None, None, 3, None, 0, dp) == dg.DG_EINVAL
    assert L.dg_rk_step_next(None, None, 1e-3, 0, None, dp) == dg.DG_EINVAL
    assert L.dg_rk_step_next_ahead(None, None, 1e-3, 0, 1.0, None, dp) == dg.DG_EINVAL
    assert L.dg_rhs(None, None, None, 1e-3) == dg.DG_EINVAL
    assert L.dg_set_wait_limit(None, 1.0) == dg.DG_EINVAL
    assert L.dg_workspace_bytes(None) == 0


def test_oversized_variable_blocks_are_rejected_without_gpu():
    """Each variable block is addressed with 32-bit offsets: a mesh whose largest block
    reaches 4 GiB is refused before anything is allocated."""
    from paper_2401_06841_amd import dg
    c = dg.dg_config()
    dg._lib.dg_config_default(ctypes.byref(c), 512, 512, 512)      # 27 points x 134M cells x 8 B
    h = ctypes.c_void_p()
    c.degree = 2
    assert dg._lib.dg_init(ctypes.byref(c), ctypes.byref(h)) == dg.DG_EINVAL
    assert not h.value
