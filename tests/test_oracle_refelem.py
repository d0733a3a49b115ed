"""Pins of the oracle's reference element against closed forms and library rules."""
from fractions import Fraction
from math import comb, factorial, sqrt

import numpy as np
import pytest
from scipy.special import roots_jacobi, roots_legendre

from oracle import refelem as R


def test_lgl_closed_forms():
    # roots of (1 - x^2) P_P'(x): textbook closed forms for P = 2, 3, 4
    np.testing.assert_allclose(R.lgl_nodes(1), [-1, 1], atol=1e-15)
    np.testing.assert_allclose(R.lgl_nodes(2), [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(R.lgl_nodes(3), [-1, -1 / sqrt(5), 1 / sqrt(5), 1], atol=1e-15)
    np.testing.assert_allclose(R.lgl_nodes(4), [-1, -sqrt(3 / 7), 0, sqrt(3 / 7), 1], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_rules_match_library(n):
    x, w = R.gauss_legendre(n)
    xs, ws = roots_legendre(n)
    np.testing.assert_allclose(x, xs, atol=1e-14)
    np.testing.assert_allclose(w, ws, atol=1e-14)
    assert abs(w.sum() - 2) < 1e-14
    x, w = R.gauss_jacobi(n, 1.0, 0.0)
    xs, ws = roots_jacobi(n, 1.0, 0.0)
    np.testing.assert_allclose(x, xs, atol=1e-14)
    np.testing.assert_allclose(w, ws, atol=1e-14)
    assert abs(w.sum() - 2) < 1e-14   # int (1 - x) dx over [-1, 1]


@pytest.mark.parametrize("P", range(1, 9))
def test_triangle_nodes(P):
    r, s = R.tri_nodes(P)
    assert r.size == (P + 1) * (P + 2) // 2
    ijk = R.tri_node_ijk(P)
    lgl = R.lgl_nodes(P)
    # edge nodes are exactly the 1D LGL nodes
    for a, (i, j, k) in enumerate(ijk):
        if j == 0:
            assert abs(r[a] - lgl[i]) < 1e-15 and abs(s[a] + 1) < 1e-15
        if i == 0:
            assert abs(s[a] - lgl[j]) < 1e-15 and abs(r[a] + 1) < 1e-15
    # invariant under the vertex permutations of the triangle (barycentric symmetry)
    lam = np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2], 1)
    key = lambda L: np.round(L, 12)
    base = {tuple(x) for x in key(lam)}
    for perm in [(1, 2, 0), (2, 0, 1), (0, 2, 1), (1, 0, 2), (2, 1, 0)]:
        assert {tuple(x) for x in key(lam[:, perm])} == base


@pytest.mark.parametrize("P", [1, 2])
def test_triangle_nodes_equispaced_low_order(P):
    r, s = R.tri_nodes(P)
    for a, (i, j, k) in enumerate(R.tri_node_ijk(P)):
        assert abs(r[a] - (-1 + 2 * i / P)) < 1e-15
        assert abs(s[a] - (-1 + 2 * j / P)) < 1e-15


def _exact_monomial_integral(a, b):
    """int_T r^a s^b dr ds, T = {r, s >= -1, r + s <= 0}, with r = 2x-1, s = 2y-1."""
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = comb(a, i) * comb(b, j) * 2 ** i * 2 ** j * (-1) ** (a - i) * (-1) ** (b - j)
            tot += c * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return 4 * tot


@pytest.mark.parametrize("P", range(1, 9))
def test_cubature_exactness(P):
    r, s, w = R.tri_cubature(P)
    for a in range(2 * P + 2):
        for b in range(2 * P + 2 - a):
            ex = float(_exact_monomial_integral(a, b))
            assert abs(np.sum(w * r ** a * s ** b) - ex) < 1e-13 * max(1, abs(ex))


@pytest.mark.parametrize("P", range(1, 9))
def test_basis_orthonormal(P):
    r, s, w = R.tri_cubature(P)
    V, _, _ = R.vandermonde_tri(r, s, P)
    M = V.T @ (w[:, None] * V)
    np.testing.assert_allclose(M, np.eye(M.shape[0]), atol=1e-13)


@pytest.mark.parametrize("P", range(1, 9))
def test_basis_derivatives_by_finite_differences(P):
    rng = np.random.default_rng(1)
    r = rng.uniform(-0.9, 0.3, 20)
    s = rng.uniform(-0.9, 0.3, 20)
    m = r + s < -0.1
    r, s = r[m], s[m]
    _, Vr, Vs = R.vandermonde_tri(r, s, P)
    h = 1e-6
    Vp, _, _ = R.vandermonde_tri(r + h, s, P)
    Vm, _, _ = R.vandermonde_tri(r - h, s, P)
    np.testing.assert_allclose(Vr, (Vp - Vm) / (2 * h), atol=1e-6)
    Vp, _, _ = R.vandermonde_tri(r, s + h, P)
    Vm, _, _ = R.vandermonde_tri(r, s - h, P)
    np.testing.assert_allclose(Vs, (Vp - Vm) / (2 * h), atol=1e-6)


@pytest.mark.parametrize("P", range(1, 9))
def test_reference_matrices_reproduce_polynomials(P):
    re = R.ref(P)
    # a degree-P polynomial p(r,s) t^P: interpolate at nodes, evaluate/derive at cubature points
    c = 1.0 if P >= 2 else 0.0
    p = lambda r, s: (0.3 + r - 0.5 * s) ** P + c * r * s
    pr = lambda r, s: P * (0.3 + r - 0.5 * s) ** (P - 1) + c * s
    ps = lambda r, s: -0.5 * P * (0.3 + r - 0.5 * s) ** (P - 1) + c * r
    u = p(re.r, re.s)
    np.testing.assert_allclose(re.B @ u, p(re.cr, re.cs), atol=1e-12)
    np.testing.assert_allclose(re.Dr @ u, pr(re.cr, re.cs), atol=1e-11)
    np.testing.assert_allclose(re.Ds @ u, ps(re.cr, re.cs), atol=1e-11)
    ut = re.t ** P
    np.testing.assert_allclose(re.Bz @ ut, re.zq ** P, atol=1e-13)
    np.testing.assert_allclose(re.Dz @ ut, P * re.zq ** (P - 1), atol=1e-11)
