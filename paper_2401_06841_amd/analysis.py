"""Flow statistics of DG states for comparing runs (host numpy, measurement only).

* Density PDF: volume-weighted histogram of log10(rho) over the interior Gauss-Legendre
  points of every cell (weight omega_q h^3 / 8), the quantity shown in the paper's density
  PDFs (Sec. 5); distance between two PDFs = L1 norm of the difference of the normalised
  histograms.
* Velocity power spectrum: v = m/rho evaluated on a uniform grid of p = k+1 points per cell
  per dimension (N p points per dimension, Sec. 4.3; rho clipped at the 1e-3 floor there,
  since positivity is enforced only at the Gauss points), FFT, energy 1/2 |v_hat|^2 summed over
  integer shells |kappa| in [K - 1/2, K + 1/2); distance between two spectra = mean
  |log10 E_a - log10 E_b| over 1 <= K <= N p / 2 (all sampled scales) and over
  1 <= K <= N / 2 (scales resolved by the cells).  On meshes above 85^3 cells p is reduced
  so that the sampling grid has at most 256 points per dimension.
The basis (orthonormal total-degree Legendre, graded order) is evaluated here with numpy's
Legendre routines; nothing here runs in a simulation step.

With library contexts for the two states, compare() instead takes the statistics from the
GPU (dg_velocity_spectrum on the full N p grid with p = k+1, and dg_structure_function
with 100 bins of 1e5 pairs, the same pairs for both states, so the difference reflects the
states and not the sampling).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

RHO_FLOOR = 1e-3    # density floor of the method (Sec. 3.1)


def modes(k: int):
    """Exponent triples in graded order: total degree ascending, then a, then b descending."""
    out = []
    for n in range(k + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def _leg1d(k: int, x):
    """Normalised Legendre values sqrt(2n+1) P_n(x), shape [k+1][len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([np.sqrt(2 * n + 1) * npleg.legval(x, [0] * n + [1]) for n in range(k + 1)])


def _basis_tensor(k: int, pts1d):
    """phi_l at the tensor points (x fastest), shape [nb][npts^3]."""
    L = _leg1d(k, pts1d)
    P = len(pts1d)
    out = []
    for a, b, c in modes(k):
        out.append(np.einsum("z,y,x->zyx", L[c], L[b], L[a]).reshape(P ** 3))
    return np.array(out)


def _as_numpy(u):
    if hasattr(u, "detach"):
        u = u.detach().to("cpu").double().numpy()
    return np.asarray(u, dtype=np.float64)


def density_pdf(u, k: int, bins: int = 200, lo: float = -4.0, hi: float = 3.0):
    """Normalised volume-weighted histogram of log10(rho) at the Gauss points."""
    u = _as_numpy(u)
    x, w = npleg.leggauss(k + 1)
    phi = _basis_tensor(k, x)                                   # [nb][q]
    wq = np.einsum("z,y,x->zyx", w, w, w).reshape(-1) / 8.0     # sums to 1 per cell
    rho = phi.T @ u[0]                                          # [q][cells]
    lr = np.log10(np.clip(rho, 1e-300, None))
    hist, _ = np.histogram(lr.reshape(-1), bins=bins, range=(lo, hi),
                           weights=np.broadcast_to(wq[:, None], rho.shape).reshape(-1))
    return hist / max(hist.sum(), 1e-300)


def pdf_distance(p, q) -> float:
    return float(np.abs(np.asarray(p) - np.asarray(q)).sum())


def velocity_grid(u, k: int, n: tuple[int, int, int], p: int = 0):
    """v = m / rho on the uniform sub-grid of p points per cell per dimension (default
    k+1; cell-centred sub-cells); returns [3][nz p][ny p][nx p]."""
    u = _as_numpy(u)
    nx, ny, nz = n
    p = p or (k + 1)
    xi = -1.0 + (2.0 * np.arange(p) + 1.0) / p
    phi = _basis_tensor(k, xi)                                  # [nb][p^3], sub-point (a,b,c) x fastest
    vals = np.einsum("lq,vlc->vqc", phi, u)                     # [4][p^3][cells]
    # the limiter keeps rho positive at the Gauss points only; at the sampling points the
    # density is clipped at the method's floor so that near-vacuum points cannot dominate
    v = vals[1:] / np.maximum(vals[0], RHO_FLOOR)[None]
    v = v.reshape(3, p, p, p, nz, ny, nx)                       # [d][sz][sy][sx][cz][cy][cx]
    v = v.transpose(0, 4, 1, 5, 2, 6, 3).reshape(3, nz * p, ny * p, nx * p)
    return v


def power_spectrum(v):
    """Shell-summed kinetic energy spectrum of a periodic velocity field [3][Z][Y][X] on the
    unit box; sum over shells = 1/2 <|v|^2>."""
    v = np.asarray(v, dtype=np.float64)
    shape = v.shape[1:]
    npts = np.prod(shape)
    vh = np.fft.fftn(v, axes=(1, 2, 3)) / npts
    e = 0.5 * (np.abs(vh) ** 2).sum(0)
    kz = np.fft.fftfreq(shape[0], 1.0 / shape[0])
    ky = np.fft.fftfreq(shape[1], 1.0 / shape[1])
    kx = np.fft.fftfreq(shape[2], 1.0 / shape[2])
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    shell = np.floor(kk + 0.5).astype(np.int64)
    return np.bincount(shell.reshape(-1), weights=e.reshape(-1))


# shells whose reference power is below this fraction of the spectrum's peak hold rounding
# noise, not flow (FP32 rounding of the velocity leaves about 1e-14 of the peak power there)
SPECTRUM_FLOOR = 1e-10


def _spectrum_shells(e_test, e_ref, kmax: int, floor: float):
    a = np.asarray(e_test, dtype=np.float64)[1:kmax + 1]
    b = np.asarray(e_ref, dtype=np.float64)[1:kmax + 1]
    ok = (a > 0) & (b > 0) & (b >= floor * b.max()) if b.size else np.zeros(0, bool)
    return a[ok], b[ok]


def spectrum_distance(e_test, e_ref, kmax: int, floor: float = SPECTRUM_FLOOR) -> float:
    """Mean |log10 E_test - log10 E_ref| over the shells 1..kmax whose reference power is at
    least floor times the reference peak (shells at the rounding level are left out)."""
    a, b = _spectrum_shells(e_test, e_ref, kmax, floor)
    return float(np.mean(np.abs(np.log10(a) - np.log10(b)))) if a.size else float("nan")


def spectrum_distance_energy_weighted(e_test, e_ref, kmax: int, floor: float = SPECTRUM_FLOOR) -> float:
    """|log10 E_test - log10 E_ref| averaged over the same shells with the reference power as
    the weight (the error where the kinetic energy is)."""
    a, b = _spectrum_shells(e_test, e_ref, kmax, floor)
    return float(np.sum(b * np.abs(np.log10(a) - np.log10(b))) / np.sum(b)) if a.size else float("nan")


def spectrum_shells_used(e_ref, kmax: int, floor: float = SPECTRUM_FLOOR) -> int:
    return int(_spectrum_shells(e_ref, e_ref, kmax, floor)[0].size)


SF_BINS, SF_PAIRS, SF_SEED = 100, 100000, 0x5F3759DF


def gpu_structure_function(ctx, u, nbins: int = SF_BINS, npairs: int = SF_PAIRS, seed: int = SF_SEED):
    """(l, v(l)) of Sec. 4.3 on the GPU: v(l) = sqrt(S2(l) / 2)."""
    from . import dg
    return dg.dg_sf_bins(ctx, nbins), np.sqrt(0.5 * dg.dg_structure_function(ctx, u, nbins, npairs, seed))


def loglog_slope(x, y, lo: float, hi: float) -> float:
    """Least-squares slope of log y against log x over lo <= x <= hi (the paper fits v(l)
    between 0.1 and 0.25 of the box, Sec. 5)."""
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    sel = (x >= lo) & (x <= hi) & (y > 0)
    if sel.sum() < 2:
        return float("nan")
    return float(np.polyfit(np.log(x[sel]), np.log(y[sel]), 1)[0])


def sonic_scale(l, v, cs: float = 1.0):
    """Separation where M(l) = v(l)/cs first reaches 1 from below, interpolated linearly in
    log l and log M between bins; None when M(l) does not cross 1 inside the bins."""
    l, m = np.asarray(l, dtype=np.float64), np.asarray(v, dtype=np.float64) / cs
    up = np.nonzero(m >= 1.0)[0]
    if up.size == 0 or up[0] == 0:
        return None
    i = up[0]
    t = np.log(1.0 / m[i - 1]) / np.log(m[i] / m[i - 1])
    return float(np.exp(np.log(l[i - 1]) + t * np.log(l[i] / l[i - 1])))


class StatisticsSeries:
    """Structure functions and spectra of one run measured on the GPU at the caller's
    output times, summarised as the mean and the 1-sigma spread over the measurements (the
    paper averages 96 measurements over five eddy turnover times, Sec. 4.3).  Measurement i
    draws its pairs from stream seed + i, so every measurement uses fresh pairs."""

    def __init__(self, ctx, nbins: int = SF_BINS, npairs: int = SF_PAIRS, p: int | None = None,
                 seed: int = SF_SEED):
        import torch

        from . import dg
        self.ctx, self.nbins, self.npairs, self.seed = ctx, nbins, npairs, seed
        self.p = p or ctx.cfg.degree + 1
        self.l = dg.dg_sf_bins(ctx, nbins)
        self.scratch = torch.empty(dg.dg_stats_scratch_bytes(ctx, nbins, self.p), dtype=torch.uint8,
                                   device=ctx.device)
        self.v, self.e = [], []

    def measure(self, u):
        from . import dg
        s2 = dg.dg_structure_function(self.ctx, u, self.nbins, self.npairs, self.seed + len(self.v),
                                      scratch=self.scratch)
        self.v.append(np.sqrt(0.5 * s2))
        self.e.append(dg.dg_velocity_spectrum(self.ctx, u, self.p, scratch=self.scratch))

    def summary(self):
        """{"l", "v_mean", "v_std", "E_mean", "E_std", "n"} over the measurements so far."""
        v, e = np.array(self.v), np.array(self.e)
        return {"l": self.l, "v_mean": v.mean(0), "v_std": v.std(0), "E_mean": e.mean(0), "E_std": e.std(0),
                "n": len(self.v)}


def log_distance(a, b) -> float:
    """Mean |log10 a - log10 b| over the entries where both are positive."""
    a, b = np.asarray(a), np.asarray(b)
    ok = (a > 0) & (b > 0)
    return float(np.mean(np.abs(np.log10(a[ok]) - np.log10(b[ok])))) if ok.any() else float("nan")


def compare(u_test, u_ref, k: int, n: tuple[int, int, int], ctx_test=None, ctx_ref=None):
    """Per-field relative L2 difference, density-PDF distance, spectrum distance (and, with
    contexts, structure-function distance) of two states on the same mesh."""
    a, b = _as_numpy(u_test), _as_numpy(u_ref)
    rho = float(np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0]))
    mom = float(np.linalg.norm(a[1:] - b[1:]) / np.linalg.norm(b[1:]))
    pa, pb = density_pdf(a, k), density_pdf(b, k)
    if ctx_test is not None and ctx_ref is not None:
        from . import dg
        p = k + 1
        ea, eb = dg.dg_velocity_spectrum(ctx_test, u_test, p), dg.dg_velocity_spectrum(ctx_ref, u_ref, p)
        _, va = gpu_structure_function(ctx_test, u_test)
        _, vb = gpu_structure_function(ctx_ref, u_ref)
        return {"l2_rel_rho": rho, "l2_rel_m": mom, "density_pdf_l1": pdf_distance(pa, pb),
                "spectrum_samples_per_cell": p,
                "spectrum_log10_mean_abs": spectrum_distance(ea, eb, min(n) * p // 2),
                "spectrum_log10_energy_weighted": spectrum_distance_energy_weighted(ea, eb, min(n) * p // 2),
                "spectrum_shells_used": spectrum_shells_used(eb, min(n) * p // 2),
                "spectrum_log10_mean_abs_cell_scales": spectrum_distance(ea, eb, min(n) // 2),
                "structure_function_log10_mean_abs": log_distance(va, vb)}
    # k+1 samples per cell (the paper's N p grid), fewer on large meshes so that the grid
    # stays at most 256 points per dimension
    p = max(1, min(k + 1, 256 // max(n)))
    kmax = min(n) * p // 2
    ea = power_spectrum(velocity_grid(a, k, n, p))
    eb = power_spectrum(velocity_grid(b, k, n, p))
    return {"l2_rel_rho": rho, "l2_rel_m": mom, "density_pdf_l1": pdf_distance(pa, pb),
            "spectrum_samples_per_cell": p,
            "spectrum_log10_mean_abs": spectrum_distance(ea, eb, kmax),
            "spectrum_log10_energy_weighted": spectrum_distance_energy_weighted(ea, eb, kmax),
            "spectrum_shells_used": spectrum_shells_used(eb, kmax),
            "spectrum_log10_mean_abs_cell_scales": spectrum_distance(ea, eb, min(n) // 2)}
