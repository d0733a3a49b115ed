"""Pins of the oracle's numbering, geometry and stiffness operator."""
import math
from fractions import Fraction
from math import comb, factorial
from types import SimpleNamespace

import numpy as np
import pytest
import sympy as sp

from oracle import mesh as M
from oracle import refelem as R
from oracle.mg import Hierarchy
from oracle.operator import LevelGeometry, StiffnessOperator, element_node_xyz
from paper_2009_00705_amd import workloads as W


# ---------------------------------------------------------------------------
# exact stiffness of affine prisms by symbolic integration (P = 1, 2)
# ---------------------------------------------------------------------------

def _tri_monomial(a, b):
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = comb(a, i) * comb(b, j) * 2 ** (i + j) * (-1) ** (a - i + b - j)
            tot += c * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return 4 * tot


def _line_monomial(c):
    return Fraction(0) if c % 2 else Fraction(2, c + 1)


def _exact_affine_stiffness(P, Jmat):
    """Lagrange basis on rational nodes (P <= 2) and exact int grad N_i . grad N_j."""
    r, s, t = sp.symbols("r s t")
    ijk = R.tri_node_ijk(P)
    tri_rs = [(Fraction(-1) + Fraction(2 * i, P), Fraction(-1) + Fraction(2 * j, P)) for (i, j, k) in ijk]
    tz = [Fraction(-1) + Fraction(2 * c, P) for c in range(P + 1)]
    nodes = [(a_rs[0], a_rs[1], tc) for tc in tz for a_rs in tri_rs]
    monos = [(i, j, k) for k in range(P + 1) for i in range(P + 1) for j in range(P + 1 - i)]
    V = sp.Matrix([[sp.Rational(n[0]) ** m[0] * sp.Rational(n[1]) ** m[1] * sp.Rational(n[2]) ** m[2]
                    for m in monos] for n in nodes])
    C = V.inv()   # column n holds the monomial coefficients of N_n
    Jm = sp.Matrix(Jmat)
    Kt = Jm.inv().T                     # physical gradient = J^-T reference gradient
    detJ = abs(Jm.det())
    np_ = len(nodes)
    grads = []
    for n in range(np_):
        Nn = sum(C[q, n] * r ** monos[q][0] * s ** monos[q][1] * t ** monos[q][2] for q in range(np_))
        g = sp.Matrix([sp.diff(Nn, r), sp.diff(Nn, s), sp.diff(Nn, t)])
        grads.append(Kt * g)
    A = np.zeros((np_, np_))
    for i in range(np_):
        for j in range(i, np_):
            poly = sp.Poly(sp.expand((grads[i].T * grads[j])[0, 0] * detJ), r, s, t)
            val = Fraction(0)
            for (a, b, c), coef in poly.terms():
                val += Fraction(str(coef)) * _tri_monomial(a, b) * _line_monomial(c)
            A[i, j] = A[j, i] = float(val)
    return A, nodes


@pytest.mark.parametrize("P", [1, 2])
@pytest.mark.parametrize("shear", [False, True])
def test_affine_element_stiffness_exact(P, shear):
    if shear:
        Jmat = [[sp.Rational(3, 5), sp.Rational(1, 5), 0],
                [sp.Rational(-1, 10), sp.Rational(7, 10), 0],
                [sp.Rational(1, 10), sp.Rational(-1, 5), sp.Rational(1, 4)]]
    else:
        Jmat = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    A_ex, nodes = _exact_affine_stiffness(P, Jmat)
    J = np.array(Jmat, dtype=float)
    re = R.ref(P)
    ref_nodes = np.array([[re.r[a], re.s[a], re.t[c]] for c in range(P + 1) for a in range(re.np_tri)])
    xyz = (ref_nodes @ J.T)[None] + np.array([0.5, -0.25, 2.0])
    geo = LevelGeometry(P, P, xyz)
    op = StiffnessOperator(SimpleNamespace(P=P), geo)
    A = op.element_matrices()[0]
    np.testing.assert_allclose(A, A_ex, atol=1e-13 * np.abs(A_ex).max())
    # matrix-free apply equals the element matrix
    u = np.random.default_rng(0).standard_normal(re.np)
    np.testing.assert_allclose(op.element_apply(u[None])[0], A_ex @ u, atol=1e-12)


# ---------------------------------------------------------------------------
# numbering
# ---------------------------------------------------------------------------

def _small_cyl():
    return W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=2)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 6])
def test_box_counts_and_multiplicity(P):
    m = W.box_mesh(3, 2)
    n = M.Numbering(m, P)
    assert n.n_dof == (3 * P + 1) ** 2 * (2 * P + 1)
    assert n.n2d == m["xy"].shape[0] + n.ne * (P - 1) + n.nt * max(0, (P - 1) * (P - 2) // 2)
    assert n.mult.sum() == n.n_elem * n.np
    assert set(np.unique(n.map)) == set(range(n.n_dof))
    assert np.all(n.map[:, np.arange(n.np)] >= 0)


@pytest.mark.parametrize("meshname", ["box", "cyl"])
@pytest.mark.parametrize("P", [2, 3, 5])
def test_numbering_is_geometrically_consistent(meshname, P):
    """Every (element, local node) mapped to one global id sits at one physical point."""
    m = W.box_mesh(3, 2) if meshname == "box" else _small_cyl()
    n = M.Numbering(m, P)
    eta = 0.05 * np.cos(np.arange(n.n2d))
    X = element_node_xyz(m, n, eta)                       # (E, Np, 3)
    pts = np.full((n.n_dof, 3), np.nan)
    flat_g = n.map.ravel()
    flat_x = X.reshape(-1, 3)
    pts[flat_g] = flat_x
    np.testing.assert_allclose(flat_x, pts[flat_g], atol=1e-13)
    # distinct ids are distinct points
    key = np.round(pts, 9)
    assert np.unique(key, axis=0).shape[0] == n.n_dof


@pytest.mark.parametrize("P", [1, 3])
def test_colouring_valid(P):
    for m in (W.box_mesh(3, 2), _small_cyl()):
        n = M.Numbering(m, P)
        col = n.colours()
        for c in np.unique(col):
            nodes = n.map[col == c].ravel()
            assert np.unique(nodes).size == nodes.size
        np.testing.assert_array_equal(col, n.colours())


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def test_volume_flat_box():
    m = W.config_mesh("c1")
    h = Hierarchy(m, 4, omega=0.3)
    for lv in h.levels:
        assert abs(lv.geo.wdet.sum() - 4 * math.pi ** 2) < 1e-12


def test_volume_curved_surface():
    m = W.box_mesh(8, 2)
    n = M.Numbering(m, 6)
    xy = M.unique_xy_2d(m, n)
    eta = W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    X = element_node_xyz(m, n, eta)
    geo = LevelGeometry(6, 6, X)
    # int (eta + h) over full periods is the flat volume
    assert abs(geo.wdet.sum() - 4 * math.pi ** 2) < 1e-8


def test_volume_cylinder_mesh():
    m = W.cylinder_mesh(spacing=0.5, half=2.0, radius=0.5, n_layers=1)
    n = M.Numbering(m, 4)
    X = element_node_xyz(m, n, np.zeros(n.n2d))
    geo = LevelGeometry(4, 4, X)
    assert abs(geo.wdet.sum() - (16 - math.pi * 0.25)) < 1e-7


# ---------------------------------------------------------------------------
# operator invariants
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1_curved():
    m = W.box_mesh(2, 2)
    n = M.Numbering(m, 3)
    xy = M.unique_xy_2d(m, n)
    eta = W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    return Hierarchy(m, 3, eta2d=eta, omega=0.3)


def test_operator_invariants(c1_curved):
    lv = c1_curved.levels[0]
    A = lv.op.assembled()
    ones = np.ones(A.shape[0])
    assert np.abs(A @ ones).max() < 1e-13 * abs(A).max()          # constant nullspace
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()               # symmetric
    x = np.random.default_rng(3).standard_normal(A.shape[0])
    np.testing.assert_allclose(lv.op.apply(x), A @ x, atol=1e-12 * abs(A).max())
    free = np.flatnonzero(lv.free)
    ev = np.linalg.eigvalsh(A[free][:, free].toarray())
    assert ev.min() > 0
    np.testing.assert_allclose(lv.diag, A.diagonal(), atol=1e-14 * abs(A).max())


def test_patch_test_exact_on_extruded_mesh():
    """phi = 1 + 0.3 x - 0.7 y with Dirichlet walls and top is reproduced exactly."""
    from oracle.krylov import direct_solve
    m = W.box_mesh(3, 2)
    n = M.Numbering(m, 4)
    xy = M.unique_xy_2d(m, n)
    eta = W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    h = Hierarchy(m, 4, eta2d=eta, omega=0.3, dirichlet_tags=0b11110)
    xyz = M.node_xyz(m, h.levels[0].num, eta)
    phi = 1 + 0.3 * xyz[:, 0] - 0.7 * xyz[:, 1]
    sol = direct_solve(h, phi)
    assert np.abs(sol - phi).max() < 1e-10


def test_spectral_convergence_in_P():
    from oracle.krylov import direct_solve
    m = W.config_mesh("c1")
    errs = []
    for P in range(1, 7):
        h = Hierarchy(m, P, omega=0.3)
        xyz = M.node_xyz(m, h.levels[0].num, np.zeros(h.levels[0].num.n2d))
        ex = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
        errs.append(np.abs(direct_solve(h, ex) - ex).max())
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs)) < -1.0), errs    # at least a factor e per order
    assert errs[-1] < 1e-6


def test_h_convergence_rate():
    from oracle.krylov import direct_solve
    P = 2
    errs = []
    for N in (2, 4, 8):
        m = W.box_mesh(N, max(1, N // 2))
        h = Hierarchy(m, P, omega=0.3)
        xyz = M.node_xyz(m, h.levels[0].num, np.zeros(h.levels[0].num.n2d))
        ex = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
        errs.append(np.sqrt(np.mean((direct_solve(h, ex) - ex) ** 2)))
    rates = -np.diff(np.log2(errs))
    assert np.all(rates >= P + 0.5), rates
