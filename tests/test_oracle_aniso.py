"""Pins of the oracle's anisotropic orders (triangle order P, vertical order PZ)
and of the in-plane-first and equal-order (semi-coarsening) sequences.

The paper's 3D test coarsens (5,3) -> (3,3) -> (1,1) (Sec. 6.2, Table
BTcoarse3D): prisms may carry different orders in the plane and along the
extrusion.  What pins them here: exact cubature of monomials, exact
reproduction of polynomials by the transfers, operator invariants, the weak
Laplacian of linear fields, and the direct solution.
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from oracle.mg import Hierarchy, Level, level_orders
from oracle.operator import element_node_xyz
from oracle.refelem import RefElement
from paper_2009_00705_amd import workloads as W


def _tri_monomial(a, b):
    """int_T r^a s^b, T = {r, s >= -1, r + s <= 0} (binomial expansion in x = (1+r)/2)."""
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = comb(a, i) * comb(b, j) * 2 ** i * 2 ** j * (-1) ** (a - i) * (-1) ** (b - j)
            tot += c * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return 4 * tot


def test_in_plane_first_sequence():
    assert level_orders(6, "xy") == [(6, 6), (3, 6), (1, 6), (1, 3), (1, 1)]
    assert level_orders(8, "xy") == [(8, 8), (4, 8), (2, 8), (1, 8), (1, 4), (1, 2), (1, 1)]
    assert level_orders(3, "xy") == [(3, 3), (1, 3), (1, 1)]
    assert level_orders(1, "xy") == [(1, 1)]
    assert level_orders(6, "both") == [6, 3, 1]


def test_equal_order_sequence():
    """Semi-coarsening of the higher-order direction until the orders agree, then
    both together (Sec. 6.2, Table BTcoarse3D); the finest pairs of the scaling
    study (Sec. 6.3) and a vertical-first case (vertical order above the
    triangle order)."""
    assert level_orders(5, "equal", 3) == [(5, 3), (3, 3), (1, 1)]
    assert level_orders(2, "equal", 2) == [(2, 2), (1, 1)]
    assert level_orders(4, "equal", 2) == [(4, 2), (2, 2), (1, 1)]
    assert level_orders(6, "equal", 4) == [(6, 4), (4, 4), (2, 2), (1, 1)]
    assert level_orders(9, "equal", 7) == [(9, 7), (7, 7), (3, 3), (1, 1)]
    assert level_orders(8, "equal", 2) == [(8, 2), (4, 2), (2, 2), (1, 1)]
    assert level_orders(3, "equal", 6) == [(3, 6), (3, 3), (1, 1)]
    assert level_orders(6, "equal") == [(6, 6), (3, 3), (1, 1)]
    assert level_orders(5, "both", 3) == [(5, 3), (2, 1), (1, 1)]
    assert level_orders(5, "xy", 3) == [(5, 3), (2, 3), (1, 3), (1, 1)]
    # every step lowers an order to no less than its floor half and never raises one
    for P in range(1, 9):
        for PZ in range(1, 9):
            seq = level_orders(P, "equal", PZ)
            assert seq[0] == (P, PZ) and seq[-1] == (1, 1)
            for (a, b), (c, d) in zip(seq, seq[1:]):
                assert c <= a and d <= b and (c, d) != (a, b) and c >= max(1, a // 2) and d >= max(1, b // 2)


@pytest.fixture(scope="module")
def fpso_like():
    """(5, 3) -> (3, 3) -> (1, 1) on a curved 2 x 2 x 2 box: the order pairs of the
    paper's 3D case."""
    m = W.box_mesh(2, 2)
    num = M.Numbering(m, 5)
    eta = 0.05 * np.sin(M.unique_xy_2d(m, num)[:, 0])
    return m, Hierarchy(m, 5, eta2d=eta, nu1=3, nu2=3, smoother="chebyshev", coarsening="equal", PZ=3)


def test_anisotropic_finest_level_is_the_fine_space(fpso_like):
    """The finest level carries triangle order 5 and vertical order 3: node and
    cubature counts, the isoparametric geometry of the order-5 map (its volume
    equals that of the same map at (5, 5): the sigma map is affine along the
    extrusion, so the vertical order does not change it), and the weak
    Laplacian of linear fields vanishing at nodes away from the boundary."""
    m, h = fpso_like
    assert [(lv.num.P, lv.num.PZ) for lv in h.levels] == [(5, 3), (3, 3), (1, 1)]
    lv = h.levels[0]
    assert lv.num.n_dof == (2 * 5 + 1) ** 2 * (2 * 3 + 1)
    iso = Hierarchy(m, 5, eta2d=h.eta2d, omega=0.3, coarsening="both")
    assert abs(lv.geo.wdet.sum() - iso.levels[0].geo.wdet.sum()) < 1e-12 * lv.geo.wdet.sum()
    xyz = M.node_xyz(m, lv.num, h.eta2d)
    lin = 0.7 + 0.3 * xyz[:, 0] - 0.2 * xyz[:, 1] + 0.5 * xyz[:, 2]
    y = lv.op.apply(lin)
    z = np.arange(lv.num.n_dof) % lv.num.nz
    x, yy = xyz[:, 0], xyz[:, 1]
    inner = (x > 1e-9) & (x < 2 * np.pi - 1e-9) & (yy > 1e-9) & (yy < 2 * np.pi - 1e-9) & (z > 0) & \
            (z < lv.num.nz - 1)
    assert inner.any() and np.abs(y[inner]).max() < 1e-10 * np.abs(lv.diag).max()


def test_equal_order_transfers_reproduce_coarse_polynomials():
    """Flat box: fields of the coarse space prolongate to their fine interpolant
    on both steps of (5, 3) -> (3, 3) -> (1, 1); P 1 = 1; R = P^T."""
    m = W.box_mesh(2, 2)
    h = Hierarchy(m, 5, omega=0.3, coarsening="equal", PZ=3, top_neumann=True, coarse="chebyshev",
                  cheb=(2, 0.1, 2.0))
    rng = np.random.default_rng(5)
    for i in range(len(h.levels) - 1):
        lf, lc = h.levels[i], h.levels[i + 1]
        ct, cz = lc.num.P, lc.num.PZ
        xf = M.node_xyz(m, lf.num, np.zeros(lf.num.n2d))
        xc = M.node_xyz(m, lc.num, np.zeros(lc.num.n2d))
        f = lambda X: (0.2 + 0.1 * X[:, 0] - 0.3 * X[:, 1]) ** ct * (X[:, 2] + 0.4) ** cz
        np.testing.assert_allclose(h.prolong(i, f(xc)), f(xf), atol=1e-12)
        np.testing.assert_allclose(h.prolong(i, np.ones(lc.num.n_dof)), 1.0, atol=1e-14)
        x = rng.standard_normal(lc.num.n_dof)
        y = rng.standard_normal(lf.num.n_dof)
        assert abs(h.prolong(i, x) @ y - x @ h.restrict(i, y)) < 1e-12 * np.abs(x).sum() * np.abs(y).max()


def test_equal_order_solve_equals_direct(fpso_like):
    """PCG with (5, 3) -> (3, 3) -> (1, 1) V-cycles reaches the direct solution
    of the (5, 3) problem, with a V-cycle contraction well below one."""
    m, h = fpso_like
    xyz = M.node_xyz(m, h.levels[0].num, h.eta2d)
    phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    ref = K.direct_solve(h, phi)
    r = K.solve(h, phi, method="pcg", rtol=1e-11, imax=100)
    assert np.abs(r.phi - ref).max() < 1e-9 * np.abs(ref).max()
    q = r.res_hist[1:] / r.res_hist[:-1]
    assert np.exp(np.mean(np.log(q))) < 0.3, q


@pytest.mark.parametrize("P,PZ", [(3, 6), (1, 6), (2, 8), (6, 2)])
def test_anisotropic_cubature_exact(P, PZ):
    re = RefElement(P, PZ)
    assert re.np == (P + 1) * (P + 2) // 2 * (PZ + 1) and re.nq == (P + 1) ** 2 * (PZ + 1)
    t = np.kron(re.zq, np.ones(re.nq_tri))
    r = np.tile(re.cr, PZ + 1)
    s = np.tile(re.cs, PZ + 1)
    for a in range(2 * P + 2):
        for b in range(2 * P + 2 - a):
            for c in (0, 1, 2 * PZ, 2 * PZ + 1):
                ex = float(_tri_monomial(a, b)) * (0.0 if c % 2 else 2.0 / (c + 1))
                got = np.sum(re.w * r ** a * s ** b * t ** c)
                assert abs(got - ex) < 1e-13 * max(1.0, abs(ex)), (a, b, c)


def _flat_box_hierarchy(coarsening, eta_amp=0.0, **kw):
    m = W.box_mesh(2, 2)
    num = M.Numbering(m, 6)
    xy = M.unique_xy_2d(m, num)
    eta = eta_amp * np.sin(xy[:, 0]) * np.cos(xy[:, 1])
    return m, Hierarchy(m, 6, eta2d=eta, omega=0.3, coarsening=coarsening, **kw)


def test_transfers_reproduce_polynomials_of_the_coarse_space():
    """Flat box (affine sigma map): a field of triangle degree <= Pc_t and
    vertical degree <= Pc_z interpolated on the coarse level and prolongated
    equals its interpolant on the fine level; P 1 = 1; R = P^T."""
    m, h = _flat_box_hierarchy("xy", top_neumann=True, coarse="chebyshev", cheb=(2, 0.1, 2.0))
    rng = np.random.default_rng(2)
    for i in range(len(h.levels) - 1):
        lf, lc = h.levels[i], h.levels[i + 1]
        ct, cz = lc.num.P, lc.num.PZ
        xf = M.node_xyz(m, lf.num, np.zeros(lf.num.n2d))
        xc = M.node_xyz(m, lc.num, np.zeros(lc.num.n2d))
        f = lambda X: (0.2 + 0.1 * X[:, 0] - 0.3 * X[:, 1]) ** ct * (X[:, 2] + 0.4) ** cz
        np.testing.assert_allclose(h.prolong(i, f(xc)), f(xf), atol=1e-12)
        np.testing.assert_allclose(h.prolong(i, np.ones(lc.num.n_dof)), 1.0, atol=1e-14)
        x = rng.standard_normal(lc.num.n_dof)
        y = rng.standard_normal(lf.num.n_dof)
        assert abs(h.prolong(i, x) @ y - x @ h.restrict(i, y)) < 1e-12 * np.abs(x).sum() * np.abs(y).max()


@pytest.mark.parametrize("order", [(3, 6), (1, 6), (1, 3)])
def test_anisotropic_operator_invariants(order):
    """Curved surface, pure Neumann: symmetric, constants in the kernel,
    matrix-free = assembled, positive on the free nodes with a Dirichlet top,
    diagonal = assembled diagonal."""
    m = W.box_mesh(2, 2)
    num_f = M.Numbering(m, 6)
    xy = M.unique_xy_2d(m, num_f)
    eta = W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    xyz_f = element_node_xyz(m, num_f, eta)
    lv = Level(m, order, 6, xyz_f, None, False)
    A = lv.op.assembled()
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-13 * abs(A).max()
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    x = np.random.default_rng(3).standard_normal(A.shape[0])
    np.testing.assert_allclose(lv.op.apply(x), A @ x, atol=1e-12 * abs(A).max())
    free = np.flatnonzero(lv.free)
    assert np.linalg.eigvalsh(A[free][:, free].toarray()).min() > 0
    np.testing.assert_allclose(lv.diag, A.diagonal(), atol=1e-14 * abs(A).max())


def test_weak_laplacian_of_linear_fields_vanishes_inside():
    """A applied to the nodal values of a + bx + cy + dz is zero at nodes away
    from the boundary: on every level of the in-plane-first sequence when the
    map is affine (flat surface: linear fields lie in every level's space), and
    on the isoparametric fine level of a curved surface.  (Coarser levels keep
    the fine map, so on a curved surface their spaces do not hold linear fields.)"""
    for amp, levels in ((0.0, None), (0.05, [0])):
        m, h = _flat_box_hierarchy("xy", eta_amp=amp)
        for i, lv in enumerate(h.levels):
            if levels is not None and i not in levels:
                continue
            eta = h.eta2d if i == 0 else np.zeros(lv.num.n2d)
            xyz = M.node_xyz(m, lv.num, eta)
            lin = 0.7 + 0.3 * xyz[:, 0] - 0.2 * xyz[:, 1] + 0.5 * xyz[:, 2]
            y = lv.op.apply(lin)
            z = np.arange(lv.num.n_dof) % lv.num.nz
            x, yy = xyz[:, 0], xyz[:, 1]
            inner = (x > 1e-9) & (x < 2 * np.pi - 1e-9) & (yy > 1e-9) & (yy < 2 * np.pi - 1e-9) & (z > 0) & \
                    (z < lv.num.nz - 1)
            if inner.any():
                assert np.abs(y[inner]).max() < 1e-10 * np.abs(lv.diag).max(), (amp, lv.num.P, lv.num.PZ)


def test_in_plane_first_solve_equals_direct():
    m, h = _flat_box_hierarchy("xy", eta_amp=0.05)
    xyz = M.node_xyz(m, h.levels[0].num, h.eta2d)
    phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    ref = K.direct_solve(h, phi)
    r = K.solve(h, phi, method="pcg", rtol=1e-11, imax=200)
    assert np.abs(r.phi - ref).max() < 1e-9 * np.abs(ref).max()


def test_in_plane_first_coarsening_fixes_flat_in_plane_elements():
    """Prisms 5x taller than their in-plane size (the 128 x 128 box's aspect):
    coarsening in every direction leaves the vertically oscillating error to
    neither the point smoother nor the coarse levels; coarsening the plane
    first restores a small convergence factor."""
    dx = 2 * np.pi / 128
    m = W.box_mesh(4, 2, lx=4 * dx, ly=4 * dx, depth=0.5)
    num = M.Numbering(m, 6)
    xy = M.unique_xy_2d(m, num)
    eta = 0.01 * np.sin(2 * np.pi * xy[:, 0] / (4 * dx))
    xyz = M.node_xyz(m, num, eta)
    k = 2 * np.pi / (4 * dx)
    phi = np.cosh(k * (xyz[:, 2] + 0.5)) / np.cosh(k * 0.5) * np.cos(k * xyz[:, 0])
    it = {}
    for c in ("both", "xy"):
        h = Hierarchy(m, 6, eta2d=eta, nu1=3, nu2=3, smoother="chebyshev", coarsening=c)
        it[c] = K.solve(h, phi, method="pcg", rtol=1e-8, imax=200).iters
    assert it["xy"] <= 0.5 * it["both"], it
