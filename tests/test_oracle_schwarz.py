"""Pins of the oracle's overlapping additive Schwarz smoother (Sec. 5.2,
eq. Mass, eq. weights; refined overlap of Sec. 6.3).

What pins it, independently of its own code:
* on the split-quad box every node has integer lattice coordinates; the
  subdomain of an element must be the lattice ball of radius dt around its
  triangle (hexagonal metric max(|dx|, |dy|, |dx - dy|) of the (1,1)-cut
  lattice) times the vertical band of radius dz around its layer;
* overlap 0 is block Jacobi: the weights are the node multiplicities;
* when every subdomain holds every free node, one sweep is the direct solve;
* post-smoothing is the transpose of pre-smoothing;
* the paper's statements on convergence: overlap 1 beats block Jacobi, and
  both beat point Jacobi.
"""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from oracle.mg import Hierarchy
from oracle.schwarz import Schwarz, overlap_of, subdomains
from paper_2009_00705_amd import workloads as W


def _lattice_xy(num, nq):
    """Integer lattice coordinates of every 2D node of box_mesh(nq, .) at order P."""
    from oracle.refelem import tri_node_ijk
    P = num.P
    gxy = -np.ones((num.n2d, 2), dtype=np.int64)
    for t in range(num.nt):
        q = t // 2
        qi, qj = q % nq, q // nq
        for a, (i, j, k) in enumerate(tri_node_ijk(P)):
            # (v00, v10, v11): lambda1 = i, lambda2 = j; (v00, v11, v01): lambda1 = i, lambda2 = j
            x, y = (i + j, j) if t % 2 == 0 else (i, i + j)
            xy = (qi * P + x, qj * P + y)
            g = num.map2d[t, a]
            assert gxy[g, 0] < 0 or tuple(gxy[g]) == xy
            gxy[g] = xy
    return gxy


def _hex(d):
    return np.maximum(np.maximum(np.abs(d[..., 0]), np.abs(d[..., 1])), np.abs(d[..., 0] - d[..., 1]))


@pytest.mark.parametrize("P,PZ,dt,dz", [(3, 3, 1, 1), (3, 3, 2, 2), (4, 2, 1, 1), (3, 3, 0, 0), (3, 3, 2, 1),
                                        (2, 3, 1, 3)])
def test_subdomains_are_lattice_balls(P, PZ, dt, dz):
    nq, L = 4, 3
    m = W.box_mesh(nq, L)
    num = M.Numbering(m, P, PZ)
    gxy = _lattice_xy(num, nq)
    free = np.ones(num.n_dof, dtype=bool)
    sub = subdomains(num, free, dt, dz)
    g2 = np.arange(num.n_dof) // num.nz
    gz = np.arange(num.n_dof) % num.nz
    for e in range(num.n_elem):
        t, layer = divmod(e, L)
        tri_xy = gxy[num.map2d[t]]                                       # (Np_tri, 2)
        d2 = _hex(gxy[g2][:, None, :] - tri_xy[None, :, :]).min(axis=1)  # distance to the triangle
        lo, hi = layer * PZ, (layer + 1) * PZ
        dv = np.maximum(np.maximum(lo - gz, gz - hi), 0)
        expect = np.flatnonzero((d2 <= dt) & (dv <= dz))
        np.testing.assert_array_equal(sub[e], expect, err_msg=str(e))


def test_block_jacobi_weights_are_multiplicities():
    m = W.box_mesh(3, 2)
    h = Hierarchy(m, 3, smoother="schwarz", overlap=0, dirichlet_tags=0b10)
    lv = h.levels[0]
    s = lv.schwarz
    for e in range(lv.num.n_elem):
        own = np.unique(lv.num.map[e])
        np.testing.assert_array_equal(s.sub[e], own[lv.free[own]])
    np.testing.assert_array_equal(s.count[lv.free], lv.num.mult[lv.free])
    assert np.all(s.count[~lv.free] == 0)


def test_refined_overlap_orders():
    assert overlap_of((6, 6), -1) == (4, 4)
    assert overlap_of((5, 3), -1) == (3, 2)
    assert overlap_of((1, 1), -1) == (1, 1)
    assert overlap_of((6, 3), 1) == (1, 1)


def test_one_sweep_is_exact_when_subdomains_cover_everything():
    """Two prisms at P = 2 and overlap 2: both subdomains hold every free node,
    W = 1/2, so S^-1 = A_FF^-1 and one undamped sweep from zero is the direct solve."""
    m = W.box_mesh(1, 1)
    h = Hierarchy(m, 2, smoother="schwarz", overlap=2, eta2d=None, omega=1.0)
    lv = h.levels[0]
    s = lv.schwarz
    assert all(np.array_equal(x, np.flatnonzero(lv.free)) for x in s.sub)
    f = np.where(lv.free, np.random.default_rng(0).standard_normal(lv.num.n_dof), 0.0)
    u = h.smooth(0, np.zeros_like(f), f, 1)
    A = lv.op.assembled().tocsr()
    idx = np.flatnonzero(lv.free)
    ref = np.zeros_like(f)
    ref[idx] = np.linalg.solve(A[idx][:, idx].toarray(), f[idx])
    np.testing.assert_allclose(u, ref, atol=1e-12 * np.abs(ref).max())


def test_post_smoother_is_the_transpose():
    m = W.box_mesh(2, 2)
    num = M.Numbering(m, 3)
    eta = 0.05 * np.sin(M.unique_xy_2d(m, num)[:, 0])
    h = Hierarchy(m, 3, eta2d=eta, smoother="schwarz", overlap=1)
    s = h.levels[0].schwarz
    rng = np.random.default_rng(1)
    free = h.levels[0].free
    x = np.where(free, rng.standard_normal(free.size), 0.0)
    y = np.where(free, rng.standard_normal(free.size), 0.0)
    a, b = s.apply(x) @ y, x @ s.apply(y, transpose=True)
    assert abs(a - b) < 1e-12 * np.abs(s.apply(x)).sum() * np.abs(y).max()
    # the symmetric V-cycle: <V x, y> = <x, V y>
    a, b = h.vcycle(x) @ y, x @ h.vcycle(y)
    assert abs(a - b) < 1e-11 * abs(a)


def test_local_solves_are_principal_submatrix_inverses():
    m = W.box_mesh(2, 1)
    h = Hierarchy(m, 3, smoother="schwarz", overlap=1)
    lv = h.levels[0]
    A = lv.op.assembled().toarray()
    for s, inv in zip(lv.schwarz.sub, lv.schwarz.inv):
        np.testing.assert_allclose(inv @ A[np.ix_(s, s)], np.eye(s.size), atol=1e-9)


def test_overlap_beats_block_jacobi_beats_point_jacobi():
    """Sec. 5.2: one overlapping node converges faster than block Jacobi
    (overlap 0), and element-block smoothers beat point Jacobi."""
    m = W.box_mesh(4, 2)
    num = M.Numbering(m, 4)
    xy = M.unique_xy_2d(m, num)
    eta = W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    xyz = M.node_xyz(m, num, eta)
    phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    it = {}
    for name, kw in (("jacobi", dict(smoother="jacobi")), ("block", dict(smoother="schwarz", overlap=0)),
                     ("asm1", dict(smoother="schwarz", overlap=1))):
        h = Hierarchy(m, 4, eta2d=eta, nu1=2, nu2=2, **kw)
        it[name] = K.solve(h, phi, method="pcg", rtol=1e-10, imax=200).iters
    assert it["asm1"] < it["block"] < it["jacobi"], it


def test_damping_estimate_is_the_spectral_radius():
    """The automatic damping 4/(3 rho) uses rho = 1.05 x the power estimate of
    the spectral radius of S^-1 A; on a small case it equals 1.05 x the largest
    eigenvalue modulus of the dense S^-1 A_FF (to 3%: 30 power steps on a
    non-normal matrix; a dropped weight W would be off by a factor 2-3)."""
    m = W.box_mesh(2, 1)
    num = M.Numbering(m, 3)
    eta = 0.05 * np.sin(M.unique_xy_2d(m, num)[:, 0])
    h = Hierarchy(m, 3, eta2d=eta, smoother="schwarz", overlap=1)
    lv = h.levels[0]
    idx = np.flatnonzero(lv.free)
    A = lv.op.assembled().toarray()[np.ix_(idx, idx)]
    S = np.zeros((idx.size, idx.size))
    for c, g in enumerate(idx):
        e = np.zeros(lv.num.n_dof)
        e[g] = 1.0
        S[:, c] = lv.schwarz.apply(e)[idx]
    rho = np.abs(np.linalg.eigvals(S @ A)).max()
    assert abs(h.schwarz_rho(0) / 1.05 - rho) < 3e-2 * rho
    assert abs(lv.omega - 4.0 / (3.0 * h.schwarz_rho(0))) < 1e-14
