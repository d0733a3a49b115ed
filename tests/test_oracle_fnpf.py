"""Pins of the oracle's free-surface time stepping (eq. FSeta, eq. FSphi, ERK4).

What fixes it independently of its own code:
* surface gradients are exact for fields in the nodal space: quadratics on
  straight triangles, linear fields on the curved (isoparametric) cylinder mesh;
* w~ of phi = 3 z + 2 is exactly 3 under any surface (linear along every
  column), and w~ of the discrete linear wave is k tanh(k h) phi~ (the
  Dirichlet-to-Neumann map of eq. laplaceproblem) to discretisation accuracy;
* a raised flat surface at rest: eta_t = 0, phi~_t = -g a exactly;
* the quadratic terms of eq. FSphi on a linear wave: phi~_t = -1/2 eps^2 k^2
  (sin^2 kx - tanh^2(kh) cos^2 kx);
* ERK4 on a small-amplitude standing wave follows the linear solution with
  omega^2 = g k tanh(k h), and its error falls 16x when dt halves.
"""
import math

import numpy as np
import pytest

from oracle import mesh as M
from oracle.fnpf import Surface
from paper_2009_00705_amd import workloads as W

G = 9.81


def _box(nq=4, L=2, depth=1.0):
    return W.box_mesh(nq, L, depth=depth)


@pytest.mark.parametrize("P", [2, 3, 6])
def test_gradient_exact_for_quadratics_on_straight_triangles(P):
    s = Surface(_box(3, 1), P)
    xy = M.unique_xy_2d(s.mesh, s.num)
    x, y = xy[:, 0], xy[:, 1]
    f = 1 + 2 * x - y + 0.3 * x * x - 0.2 * x * y + 0.1 * y * y
    fx, fy = s.grad(f)
    np.testing.assert_allclose(fx, 2 + 0.6 * x - 0.2 * y, atol=1e-11)
    np.testing.assert_allclose(fy, -1 - 0.2 * x + 0.2 * y, atol=1e-11)


def test_gradient_exact_for_linear_fields_on_curved_triangles():
    m = W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=1)
    s = Surface(m, 4)
    xy = M.unique_xy_2d(m, s.num)
    fx, fy = s.grad(0.5 - 1.5 * xy[:, 0] + 0.25 * xy[:, 1])
    np.testing.assert_allclose(fx, -1.5, atol=1e-11)
    np.testing.assert_allclose(fy, 0.25, atol=1e-11)


def test_w_of_a_field_linear_in_z_is_exact_under_any_surface():
    s = Surface(_box(3, 3), 4)
    xy = M.unique_xy_2d(s.mesh, s.num)
    eta = 0.1 * np.sin(xy[:, 0]) * np.cos(xy[:, 1])
    xyz = M.node_xyz(s.mesh, s.num, eta)
    np.testing.assert_allclose(s.w(3 * xyz[:, 2] + 2, eta), 3.0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2])
def test_w_is_the_dirichlet_to_neumann_map_of_the_linear_wave(k):
    h = 1.0
    s = Surface(_box(4 * k, 2, depth=h), 6)          # same resolution per wavelength
    x = M.unique_xy_2d(s.mesh, s.num)[:, 0]
    phis = np.cos(k * x)
    phi = s.laplace(np.zeros_like(x), phis)
    w = s.w(phi, np.zeros_like(x))
    # pointwise boundary derivative of the Galerkin solution: ~3e-5 at this resolution
    np.testing.assert_allclose(w, k * math.tanh(k * h) * phis, atol=1e-4 * k)


def test_flat_raised_surface_at_rest():
    s = Surface(_box(3, 2), 3)
    a = 0.05
    eta = np.full(s.num.n2d, a)
    deta, dphis, phi = s.rhs(eta, np.zeros(s.num.n2d), G)
    assert np.abs(phi).max() == 0.0
    np.testing.assert_allclose(deta, 0.0, atol=1e-15)
    np.testing.assert_allclose(dphis, -G * a, rtol=1e-15)


def test_quadratic_terms_of_the_dynamic_condition():
    k, h, eps = 1, 1.0, 1e-2
    s = Surface(_box(4, 2, depth=h), 6)
    x = M.unique_xy_2d(s.mesh, s.num)[:, 0]
    eta = np.zeros_like(x)
    deta, dphis, _ = s.rhs(eta, eps * np.cos(k * x), G)
    th = math.tanh(k * h)
    # both to 1e-4 of their size (the discrete w~ carries ~3e-5 relative error here)
    np.testing.assert_allclose(deta, eps * k * th * np.cos(k * x), atol=1e-4 * eps)
    want = -0.5 * eps ** 2 * k ** 2 * (np.sin(k * x) ** 2 - th ** 2 * np.cos(k * x) ** 2)
    np.testing.assert_allclose(dphis, want, atol=1e-4 * eps ** 2)


def _standing_wave_error(n_steps):
    k, h, eps = 1, 1.0, 1e-6
    s = Surface(_box(4, 2, depth=h), 6)
    x = M.unique_xy_2d(s.mesh, s.num)[:, 0]
    om = math.sqrt(G * k * math.tanh(k * h))
    t_end = 0.2 * (2 * math.pi / om)
    dt = t_end / n_steps
    eta, phis = eps * np.cos(k * x), np.zeros_like(x)
    for _ in range(n_steps):
        eta, phis = s.erk4(eta, phis, dt, G)
    eta_ex = eps * np.cos(k * x) * math.cos(om * t_end)
    phis_ex = -G * eps / om * np.cos(k * x) * math.sin(om * t_end)
    return max(np.abs(eta - eta_ex).max() / eps, np.abs(phis - phis_ex).max() * om / (G * eps))


def test_erk4_standing_wave_and_order():
    e1 = _standing_wave_error(2)
    e2 = _standing_wave_error(4)
    assert e2 < 1e-4, (e1, e2)
    assert 12.0 < e1 / e2 < 20.0, (e1, e2)
