"""Pins of the oracle's 1D pieces, basis and quadrature (CPU).

Paper: Sec. 2.1 (tensor-product Legendre basis), Sec. 2.2 (orthonormality, Gaussian
quadrature), Sec. 3.2 footnote and Sec. 7 (total-degree truncation, b_k, v_k, s_k).
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_gl():
    rows = {}
    with open(os.path.join(GOLDEN, "gauss_legendre.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, xe, we = line.split()
            rows.setdefault(int(n), []).append((eval(xe, {"math": math}), eval(we, {"math": math})))
    return rows


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_gauss_closed_forms(n):
    x, w = oracle.gauss(n)
    ref = _golden_gl()[n]
    np.testing.assert_allclose(x, [r[0] for r in ref], atol=1e-15)
    np.testing.assert_allclose(w, [r[1] for r in ref], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_matches_numpy_and_is_exact(n):
    x, w = oracle.gauss(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, atol=1e-14)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(2 * n):
        exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** p) - exact) < 1e-14
    # degree 2n is not integrated exactly
    assert abs(np.sum(w * x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def test_legendre_closed_forms():
    for x in np.linspace(-1, 1, 11):
        for n, p, dp in [(0, 1.0, 0.0), (1, x, 1.0), (2, 1.5 * x * x - 0.5, 3 * x),
                         (3, 2.5 * x ** 3 - 1.5 * x, 7.5 * x * x - 1.5),
                         (4, (35 * x ** 4 - 30 * x * x + 3) / 8, (140 * x ** 3 - 60 * x) / 8)]:
            v, d = oracle.leg(n, x)
            s = math.sqrt(2 * n + 1)
            assert abs(v - s * p) < 1e-14
            assert abs(d - s * dp) < 1e-13


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_basis_count_and_order(k):
    e = oracle.basis_exps(k)
    assert len(e) == (k + 1) * (k + 2) * (k + 3) // 6 == oracle.nbasis(k)
    # graded: total degree ascending, then a descending, then b descending
    keys = [(a + b + c, -a, -b) for a, b, c in e]
    assert keys == sorted(keys)
    assert len({tuple(r) for r in e}) == len(e)
    assert all(a + b + c <= k for a, b, c in e)
    if k == 2:
        assert [tuple(r) for r in e] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0),
                                        (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_orthonormality_on_gauss_points(k):
    """(1/8) sum_q w_q phi_l phi_m = delta_lm with the (k+1)-point rule (Sec. 2.2)."""
    g, w = oracle.gauss(k + 1)
    nb = oracle.nbasis(k)
    M = np.zeros((nb, nb))
    for qz in range(k + 1):
        for qy in range(k + 1):
            for qx in range(k + 1):
                xi = [g[qx], g[qy], g[qz]]
                phi = np.array([oracle.basis_eval(k, l, xi)[0] for l in range(nb)])
                M += 0.125 * w[qx] * w[qy] * w[qz] * np.outer(phi, phi)
    np.testing.assert_allclose(M, np.eye(nb), atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_tensor_quadrature_exact_on_polynomials(k):
    """The (k+1)^3 rule integrates x^a y^b z^c exactly for a, b, c <= 2k+1."""
    g, w = oracle.gauss(k + 1)
    rng = np.random.default_rng(k)
    for _ in range(10):
        a, b, c = rng.integers(0, 2 * k + 2, 3)
        q = sum(w[i] * w[j] * w[l] * g[i] ** a * g[j] ** b * g[l] ** c
                for i in range(k + 1) for j in range(k + 1) for l in range(k + 1))
        ex = np.prod([2.0 / (p + 1) if p % 2 == 0 else 0.0 for p in (a, b, c)])
        assert abs(q - ex) < 1e-13


def test_basis_values_closed_form():
    xi = np.array([0.3, -0.7, 0.45])
    phi, d = oracle.basis_eval(2, 5, xi)            # mode (1,1,0)
    assert abs(phi - 3.0 * xi[0] * xi[1]) < 1e-15
    np.testing.assert_allclose(d, [3.0 * xi[1], 3.0 * xi[0], 0.0], atol=1e-15)
    phi, d = oracle.basis_eval(2, 9, xi)            # mode (0,0,2)
    assert abs(phi - math.sqrt(5) * (1.5 * xi[2] ** 2 - 0.5)) < 1e-15
    np.testing.assert_allclose(d, [0.0, 0.0, math.sqrt(5) * 3 * xi[2]], atol=1e-14)
