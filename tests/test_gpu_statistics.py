"""GPU flow statistics (Sec. 4.3) against the oracle: the velocity structure function of
random pairs evaluated through the cell expansions, and the shell spectrum of the p-sample
velocity grid.

The pairs are drawn from the same counter-based generator on both sides, so the GPU and
the oracle evaluate the same pairs: the bar is the FP64 one (1e-12 relative per bin), also
for FP32 states (both sides evaluate the FP32 coefficients in FP64).  At the benchmark's
full sizes (100 bins of 1e5 pairs at 64^3 and 128^3) the oracle recomputes a sample of
bins alone.  Spectra: per shell within 1e-12 of the total energy plus 1e-9 relative (the
two FFTs round differently)."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from gpu_util import dev, make
from paper_2401_06841_amd import dg

pytestmark = pytest.mark.gpu
FLAGS = dg.DG_AV | dg.DG_PRIM_PROJ | dg.DG_POS_LIMITER


def _state(nx, ny, nz, k, precision, seed, mach=3.0):
    u = synthetic.turbulent_like(nx, ny, nz, k, mach=mach, seed=seed, high_amp=0.05, kmax_frac=0.25)
    if precision == dg.DG_FP32:
        u = u.astype(np.float32).astype(np.float64)
    return u


SF_CASES = {
    "8c-k2-fp64": (8, 8, 8, 2, dg.DG_FP64, 12, 3000),
    "8c-k2-fp32": (8, 8, 8, 2, dg.DG_FP32, 12, 3000),
    "8c-k1-fp64": (8, 8, 8, 1, dg.DG_FP64, 7, 2000),
    "8c-k3-fp64": (8, 8, 8, 3, dg.DG_FP64, 7, 2000),            # records staged in two halves
    "8c-k1-fp32": (8, 8, 8, 1, dg.DG_FP32, 7, 2000),
    "8c-k3-fp32": (8, 8, 8, 3, dg.DG_FP32, 7, 2000),
    "noncubic-k2": (6, 5, 4, 2, dg.DG_FP64, 9, 1500),
    "strided-pairs": (10, 10, 10, 2, dg.DG_FP64, 3, 40000),     # > 256 one-wave blocks x 64 pairs per bin
    "one-pair-one-bin": (4, 4, 4, 2, dg.DG_FP64, 1, 1),
}


@pytest.mark.parametrize("case", list(SF_CASES))
def test_structure_function_matches_oracle(case):
    nx, ny, nz, k, prec, nbins, npairs = SF_CASES[case]
    print(f"structure function case {case}", flush=True)
    u = _state(nx, ny, nz, k, prec, seed=4)
    ctx = make(nx, ny, nz, k, FLAGS, prec)
    assert np.allclose(dg.dg_sf_bins(ctx, nbins), oracle.sf_bins(oracle.Cfg(nx, ny, nz, k), nbins), rtol=1e-15)
    got = dg.dg_structure_function(ctx, dev(u, ctx), nbins, npairs, 12345)
    ref = oracle.structure_function(oracle.Cfg(nx, ny, nz, k), u, nbins, npairs, 12345)
    assert np.all(np.isfinite(got)) and np.all(got >= 0)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(ref, 1e-300)), (case, np.abs(got / ref - 1).max())


def test_structure_function_is_deterministic_and_seeded():
    n, k = 8, 2
    ctx = make(n, n, n, k, FLAGS)
    u = dev(_state(n, n, n, k, dg.DG_FP64, seed=1), ctx)
    a = dg.dg_structure_function(ctx, u, 10, 5000, 7)
    b = dg.dg_structure_function(ctx, u, 10, 5000, 7)
    c = dg.dg_structure_function(ctx, u, 10, 5000, 8)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_uniform_flow_gives_zero():
    n, k = 6, 2
    ctx = make(n, n, n, k, FLAGS)
    u = np.zeros(ctx.cfg.shape)
    u[0, 0] = 1.3
    u[1, 0], u[2, 0], u[3, 0] = 0.2, -0.7, 1.1
    assert np.all(dg.dg_structure_function(ctx, dev(u, ctx), 8, 1000, 3) == 0.0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,prec", [(64, dg.DG_FP64), (128, dg.DG_FP32)])
def test_structure_function_full_size_sampled_bins(n, prec):
    """100 bins of 1e5 pairs on the GPU; the oracle recomputes the first, a middle and the
    last bin."""
    k = 2
    print(f"full-size structure function {n}^3", flush=True)
    u = synthetic.turbulent_like(n, n, n, k, mach=5.0, seed=3, high_amp=0.02, kmax_frac=0.125)
    if prec == dg.DG_FP32:
        u = u.astype(np.float32).astype(np.float64)
    ctx = make(n, n, n, k, FLAGS, prec)
    got = dg.dg_structure_function(ctx, dev(u, ctx), 100, 100000, 2024)
    cfg = oracle.Cfg(n, n, n, k)
    for b in (0, 57, 99):
        ref = oracle.structure_function(cfg, u, 100, 100000, 2024, b0=b, nsel=1)[0]
        assert abs(got[b] - ref) <= 1e-12 * ref, (b, got[b], ref)


SP_CASES = {
    "8c-k2-p3": (8, 8, 8, 2, dg.DG_FP64, 3),
    "8c-k2-p3-fp32": (8, 8, 8, 2, dg.DG_FP32, 3),
    "noncubic-odd-k1-p3": (6, 5, 4, 1, dg.DG_FP64, 3),            # 18 x 15 x 12: odd Y
    "odd-all-k3-p1": (7, 5, 3, 3, dg.DG_FP64, 1),
    "8c-k3-p4": (8, 8, 8, 3, dg.DG_FP64, 4),
}


def _spectrum_close(got, ref):
    assert got.shape == ref.shape
    tol = 1e-12 * ref.sum() + 1e-9 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= tol), np.abs(got - ref).max()


@pytest.mark.parametrize("case", list(SP_CASES))
def test_spectrum_matches_oracle(case):
    nx, ny, nz, k, prec, p = SP_CASES[case]
    print(f"spectrum case {case}", flush=True)
    u = _state(nx, ny, nz, k, prec, seed=6)
    ctx = make(nx, ny, nz, k, FLAGS, prec)
    got = dg.dg_velocity_spectrum(ctx, dev(u, ctx), p)
    ref = oracle.velocity_spectrum(oracle.Cfg(nx, ny, nz, k), u, p)
    _spectrum_close(got, ref)


@pytest.mark.timeout(600)
def test_spectrum_full_size():
    """64^3 cells, degree 2, 3 samples per cell: the 192^3 grid of the benchmark workload."""
    n, k, p = 64, 2, 3
    print("full-size spectrum 64^3 p=3", flush=True)
    u = synthetic.turbulent_like(n, n, n, k, mach=3.0, seed=8, high_amp=0.02, kmax_frac=0.125)
    ctx = make(n, n, n, k, FLAGS)
    got = dg.dg_velocity_spectrum(ctx, dev(u, ctx), p)
    ref = oracle.velocity_spectrum(oracle.Cfg(n, n, n, k), u, p)
    _spectrum_close(got, ref)


def test_statistics_reject_bad_arguments():
    n, k = 4, 2
    ctx = make(n, n, n, k, FLAGS)
    u = dev(_state(n, n, n, k, dg.DG_FP64, seed=2), ctx)
    small = torch.empty(256, dtype=torch.uint8, device=ctx.device)
    with pytest.raises(ValueError):
        dg.dg_structure_function(ctx, u, 4, 10, 1, scratch=small)
    with pytest.raises(dg.DGError):
        dg.dg_structure_function(ctx, u, 0, 10, 1)
    with pytest.raises(dg.DGError):
        dg.dg_structure_function(ctx, u, 4, 0, 1)
    with pytest.raises(dg.DGError):
        dg.dg_spectrum_nshell(ctx, 0)
    one = make(1, 4, 4, 1, FLAGS)                   # 1 x 4 x 4 grid at p = 1: too thin
    with pytest.raises(dg.DGError):
        dg.dg_velocity_spectrum(one, dev(np.zeros(one.cfg.shape) + 1.0, one), 1)


def test_statistics_series_mean_and_spread():
    """Measurement i of a series uses pair stream seed + i; the mean and spread are those of
    the individual calls."""
    from paper_2401_06841_amd import analysis
    n, k = 8, 2
    ctx = make(n, n, n, k, FLAGS)
    u = dev(_state(n, n, n, k, dg.DG_FP64, seed=5), ctx)
    ser = analysis.StatisticsSeries(ctx, nbins=6, npairs=2000, seed=40)
    for _ in range(3):
        ser.measure(u)
    s = ser.summary()
    single = [np.sqrt(0.5 * dg.dg_structure_function(ctx, u, 6, 2000, 40 + i)) for i in range(3)]
    assert s["n"] == 3
    assert np.allclose(s["v_mean"], np.mean(single, 0), rtol=1e-14)
    assert np.allclose(s["v_std"], np.std(single, 0), rtol=1e-12, atol=1e-15)
    assert np.all(s["v_std"] > 0)                   # fresh pairs per measurement
    assert np.all(s["E_std"] <= 1e-12 * s["E_mean"].sum())   # same state: same spectrum
