"""Algorithmic work counts of the DG stage (used for roofline fractions).

The paper's operation-count model (Sec. 7, "Discussion on computational cost") per cell
and per evaluation of the weight derivative:
    volume  v_k (10 b_k f + c_F),  surface  6 s_k (5 b_k f + c_F),
with v_k = (k+1)^3 interior points, s_k = (k+1)^2 points per face, b_k modes per field,
f fields and c_F ~ 15 operations per flux / Riemann evaluation.  This module adds the
pieces this method runs beside it, counted the same way (one multiply-add = 2):
    primitive projection  6 b v + 3 v   (Sec. 3.2: m/rho at v points, 3 projections)
    compression sensor+AV 6 b v + 20 v  (Sec. 3.1: divergence from the projected velocity)
    driving source        12 b v        (Sec. 4.2: rho a at v points projected on 3 rows)
    positivity limiter    2 b (v + 6 s) (Sec. 3.1: density at every volume and face point)
    stage combination     5 per DOF     (Sec. 2.2 / 7: SSP Runge-Kutta)
Kernels that do fewer operations (e.g. exploiting zero derivative entries) are still
measured against these counts.
"""


def nbasis(k: int) -> int:
    return (k + 1) * (k + 2) * (k + 3) // 6


def nvol(k: int) -> int:
    return (k + 1) ** 3


def nface(k: int) -> int:
    return (k + 1) ** 2


def paper_rhs_flops_per_cell(k: int, f: int = 4, cF: int = 15) -> int:
    b, v, s = nbasis(k), nvol(k), nface(k)
    return v * (10 * b * f + cF) + 6 * s * (5 * b * f + cF)


def stage_flops_per_cell(k: int, av: bool = True, proj: bool = True, forcing: bool = True,
                         limiter: bool = True) -> int:
    """Algorithmic operations of one full RK stage (RHS + extras + combine) per cell, f = 4."""
    b, v, s = nbasis(k), nvol(k), nface(k)
    n = paper_rhs_flops_per_cell(k, 4, 15)
    if proj or av:
        n += 6 * b * v + 3 * v
    if av:
        n += 6 * b * v + 20 * v
    if forcing:
        n += 12 * b * v
    if limiter:
        n += 2 * b * (v + 6 * s)
    n += 5 * 4 * b
    return n


def rhs_flops_per_cell(k: int, av: bool = True, proj: bool = True, forcing: bool = True) -> int:
    """Algorithmic operations of the right-hand-side part alone (no limiter, no combine)."""
    b, v = nbasis(k), nvol(k)
    n = paper_rhs_flops_per_cell(k, 4, 15)
    if av:
        n += 6 * b * v + 20 * v
    if forcing:
        n += 12 * b * v
    return n


def combination_flops_per_cell(k: int) -> int:
    """The stage combination alone (5 per DOF, f = 4): the extra work of a right-hand-side
    kernel that forms its stage's combination (split stages)."""
    return 5 * 4 * nbasis(k)


def stage_bytes_per_cell(k: int, elem_bytes: int) -> float:
    """Minimum HBM bytes of one stage averaged over the three SSP-RK3 stages:
    read u^(i) (and u^n for stages 2 and 3), write u^(i+1)."""
    dof = 4 * nbasis(k)
    return dof * elem_bytes * (2 + 3 + 3) / 3.0
