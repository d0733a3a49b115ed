"""Pins of the oracle's p-multigrid pieces and outer solvers."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from oracle.mg import Hierarchy, chebyshev, level_orders, splitmix64_unit
from paper_2009_00705_amd import workloads as W


def test_level_orders_match_paper_table():
    # Table BTcoarse (Sec. 6.1): P = 6 coarsens 6 -> 3 -> 1; Table BTcoarse3D
    # (Sec. 6.2): (5, 3) -> (3, 3) -> (1, 1)
    pair = lambda txt: tuple(int(v) for v in txt.split(","))
    with open("tests/golden/coarsening_tables.txt") as fh:
        rows = [l for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for row in rows:
        head, rest = row.split(":")
        seq, fine = head.split()
        P, PZ = pair(fine)
        want = [pair(v) for v in rest.split()]
        got = [o if isinstance(o, tuple) else (o, o) for o in level_orders(P, seq, PZ)]
        assert got == want, (row, got)
    assert level_orders(4) == [4, 2, 1]
    assert level_orders(8) == [8, 4, 2, 1]


def test_splitmix64_reference_values():
    # published splitmix64 outputs for state 0 (first three draws)
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = splitmix64_unit(3, 0)
    np.testing.assert_array_equal(got, [(v >> 11) * 2.0 ** -53 for v in ref])


@pytest.fixture(scope="module")
def hier_neumann():
    m = W.box_mesh(3, 2)
    return Hierarchy(m, 4, omega=0.3, top_neumann=True, coarse="chebyshev", cheb=(2, 0.1, 2.0))


def test_prolongation_reproduces_coarse_polynomials(hier_neumann):
    h = hier_neumann
    m = h.mesh
    for i in range(len(h.levels) - 1):
        lf, lc = h.levels[i], h.levels[i + 1]
        Pc = lc.P
        xf = M.node_xyz(m, lf.num, np.zeros(lf.num.n2d))
        xc = M.node_xyz(m, lc.num, np.zeros(lc.num.n2d))
        f = lambda X: (0.2 + 0.1 * X[:, 0] - 0.3 * X[:, 1]) ** Pc + (X[:, 2] + 0.5) ** Pc
        np.testing.assert_allclose(h.prolong(i, f(xc)), f(xf), atol=1e-12)
        np.testing.assert_allclose(h.prolong(i, np.ones(lc.num.n_dof)), 1.0, atol=1e-14)


def test_restriction_is_transpose(c1_hier):
    h = c1_hier
    rng = np.random.default_rng(5)
    for i in range(len(h.levels) - 1):
        nf, nc = h.levels[i].num.n_dof, h.levels[i + 1].num.n_dof
        x = np.where(h.levels[i + 1].free, rng.standard_normal(nc), 0)
        y = np.where(h.levels[i].free, rng.standard_normal(nf), 0)
        assert abs(h.prolong(i, x) @ y - x @ h.restrict(i, y)) < 1e-12 * np.abs(x).sum()


@pytest.fixture(scope="module")
def c1_hier():
    return Hierarchy(W.config_mesh("c1"), 4, omega=None)


def test_vcycle_symmetric_and_contractive(c1_hier):
    h = c1_hier
    lv = h.levels[0]
    rng = np.random.default_rng(7)
    x = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    y = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    assert abs(h.vcycle(x) @ y - x @ h.vcycle(y)) < 1e-10 * np.linalg.norm(x) * np.linalg.norm(y)
    # spectral radius of I - M^-1 A by power iteration
    e = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    for _ in range(40):
        e = e - h.vcycle(lv.A(e))
        nrm = np.linalg.norm(e)
        e = e / nrm
    assert nrm < 1.0


def test_auto_omega_is_below_jacobi_bound(c1_hier):
    for i, lv in enumerate(c1_hier.levels[:-1]):
        # omega = 4/(3 lambda) with lambda >= lambda_max(D^-1 A) keeps the smoother convergent
        A = lv.op.assembled()
        free = np.flatnonzero(lv.free)
        Aff = A[free][:, free].toarray()
        d = lv.diag[free]
        lam = np.linalg.eigvalsh(Aff / np.sqrt(np.outer(d, d))).max()
        assert lv.omega * lam < 4.0 / 3.0 + 1e-9
        assert lv.omega * lam > 1.0


def test_chebyshev_matches_closed_form():
    rng = np.random.default_rng(11)
    n = 30
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T
    d = np.diag(A).copy()
    dinv = 1 / d
    f = rng.standard_normal(n)
    k, lmin, lmax = 7, 0.05, 3.0
    x = chebyshev(lambda v: A @ v, dinv, f, k, lmin, lmax)
    # error after k steps from zero: e_k = p_k(D^-1 A) e_0 with p_k = T_k((th - l)/de) / T_k(th/de)
    S = A / np.sqrt(np.outer(d, d))
    lam, V = np.linalg.eigh(S)
    th, de = (lmax + lmin) / 2, (lmax - lmin) / 2
    T = np.polynomial.chebyshev.chebval
    c = np.zeros(k + 1)
    c[k] = 1
    p = T((th - lam) / de, c) / T(th / de, c)
    e0 = np.linalg.solve(A, f)
    ek = (V @ (p * (V.T @ (np.sqrt(d) * e0)))) / np.sqrt(d)
    np.testing.assert_allclose(e0 - x, ek, atol=1e-12 * np.abs(e0).max())


def test_solvers_agree_with_direct(c1_hier):
    h = c1_hier
    lv = h.levels[0]
    xyz = M.node_xyz(h.mesh, lv.num, np.zeros(lv.num.n2d))
    phi_ex = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    ref = K.direct_solve(h, phi_ex)
    for meth in ("pcg", "fpcg", "pdc", "mg"):
        r = K.solve(h, phi_ex, method=meth, rtol=1e-10, imax=400)
        assert r.rel_res <= 1e-10
        assert abs(r.res_hist[-1] / r.norm_f - r.rel_res) < 1e-12
        assert np.abs(r.phi - ref).max() < 1e-8 * np.abs(ref).max(), meth
    # the exact potential is reproduced to discretisation accuracy
    assert np.abs(ref - phi_ex).max() < 1e-3


def test_pcg_converges_in_finite_steps_without_preconditioner():
    # with M = I, PCG is CG: at most n_free steps in exact arithmetic
    m = W.box_mesh(1, 1)
    h = Hierarchy(m, 2, omega=0.3)
    lv = h.levels[0]
    phi = np.linspace(0, 1, lv.num.n_dof)
    r = K.solve(h, phi, method="pcg", precond=lambda v: v.copy(), rtol=1e-12, imax=200)
    assert r.iters <= int(lv.free.sum()) + 2


@pytest.mark.slow
def test_convergence_factor_flat_in_element_count():
    """O(n) claim (Sec. 6.3): mean q stays flat as elements grow at fixed aspect ratio."""
    qs = []
    for N, L in ((4, 1), (8, 2), (16, 4)):
        h = Hierarchy(W.box_mesh(N, L), 4)
        lv = h.levels[0]
        xyz = M.node_xyz(h.mesh, lv.num, np.zeros(lv.num.n2d))
        phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
        r = K.solve(h, phi, rtol=1e-8)
        qs.append(np.exp(np.mean(np.log(r.q))))
    assert max(qs) / min(qs) <= 1.25, qs


def test_chebyshev_smoother_is_symmetric_and_beats_jacobi():
    """Polynomial (Chebyshev-Jacobi) smoothing keeps the V-cycle symmetric and
    damps the anisotropic prism problem better than damped Jacobi."""
    import math
    m = W.box_mesh(8, 4, lx=math.pi / 4, ly=math.pi / 4)       # dx = 0.098, dz = 0.25
    hj = Hierarchy(m, 4)
    hc = Hierarchy(m, 4, smoother="chebyshev", nu1=3, nu2=3, omega=[lv.omega for lv in hj.levels[:-1]])
    lv = hc.levels[0]
    rng = np.random.default_rng(2)
    x = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    y = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    assert abs(hc.vcycle(x) @ y - x @ hc.vcycle(y)) < 1e-10 * np.linalg.norm(x) * np.linalg.norm(y)
    xyz = M.node_xyz(m, lv.num, np.zeros(lv.num.n2d))
    phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    rj = K.solve(hj, phi, rtol=1e-8)
    rc = K.solve(hc, phi, rtol=1e-8)
    assert rc.iters < rj.iters
    np.testing.assert_allclose(rc.phi, rj.phi, atol=1e-7 * np.abs(rj.phi).max())

def test_chebyshev_smoother_closed_form():
    # one pre-smoothing from zero equals the closed-form polynomial p(D^-1 A) D^-1 f
    m = W.box_mesh(2, 2)
    hc = Hierarchy(m, 2, smoother="chebyshev", nu1=3, nu2=3)
    lv = hc.levels[0]
    rng = np.random.default_rng(4)
    f = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    u = hc.smooth(0, np.zeros_like(f), f, 3)
    lmax = 4.0 / (3.0 * lv.omega)
    lmin = lmax / hc.smooth_ratio
    free = np.flatnonzero(lv.free)
    A = lv.op.assembled()[free][:, free].toarray()
    d = lv.diag[free]
    S = A / np.sqrt(np.outer(d, d))
    lam, V = np.linalg.eigh(S)
    th, de = (lmax + lmin) / 2, (lmax - lmin) / 2
    c = np.zeros(4)
    c[3] = 1
    p = np.polynomial.chebyshev.chebval((th - lam) / de, c) / np.polynomial.chebyshev.chebval(th / de, c)
    e0 = np.linalg.solve(A, f[free])
    want = e0 - (V @ (p * (V.T @ (np.sqrt(d) * e0)))) / np.sqrt(d)
    np.testing.assert_allclose(u[free], want, atol=1e-10 * np.abs(want).max())


def test_coarse_level_sweep_counts():
    """Sweep counts of the levels below the finest (a tuning beside Alg. 1,
    which passes one (nu1, nu2) pair down the recursion): they act only on the
    levels strictly between the finest and the coarsest, the V-cycle stays a
    symmetric operator when every level's pre and post counts agree (and not
    when they differ), and the preconditioned solve still reaches the direct
    solution."""
    import math
    m = W.box_mesh(4, 2, lx=math.pi / 4, ly=math.pi / 4)
    # two levels (2 -> 1, exact coarse solve): no level below the finest smooths
    h2 = Hierarchy(m, 2, smoother="chebyshev", nu1=3, nu2=3, smooth_ratio=8.0)
    h2c = Hierarchy(m, 2, smoother="chebyshev", nu1=3, nu2=3, smooth_ratio=8.0, nu1_coarse=0, nu2_coarse=5)
    lv = h2.levels[0]
    rng = np.random.default_rng(21)
    x = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    y = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    np.testing.assert_array_equal(h2.vcycle(x), h2c.vcycle(x))
    # three levels (4 -> 2 -> 1): the middle level's counts change the cycle
    kw = dict(smoother="chebyshev", nu1=3, nu2=3, smooth_ratio=8.0)
    h3 = Hierarchy(m, 4, **kw)
    lv = h3.levels[0]
    x = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    y = np.where(lv.free, rng.standard_normal(lv.num.n_dof), 0)
    nxy = np.linalg.norm(x) * np.linalg.norm(y)
    hs = Hierarchy(m, 4, nu1_coarse=2, nu2_coarse=2, omega=[l.omega for l in h3.levels[:-1]], **kw)
    ha = Hierarchy(m, 4, nu1_coarse=1, nu2_coarse=3, omega=[l.omega for l in h3.levels[:-1]], **kw)
    assert hs.sweeps(0) == (3, 3) and hs.sweeps(1) == (2, 2)
    z3, zs = h3.vcycle(x), hs.vcycle(x)
    assert np.linalg.norm(zs - z3) > 1e-3 * np.linalg.norm(z3)
    assert abs(zs @ y - x @ hs.vcycle(y)) < 1e-10 * nxy
    assert abs(ha.vcycle(x) @ y - x @ ha.vcycle(y)) > 1e-6 * nxy
    xyz = M.node_xyz(m, lv.num, np.zeros(lv.num.n2d))
    phi_ex = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    ref = K.direct_solve(hs, phi_ex)
    r = K.solve(hs, phi_ex, method="pcg", rtol=1e-10, imax=200)
    assert r.rel_res <= 1e-10
    assert np.abs(r.phi - ref).max() < 1e-8 * np.abs(ref).max()
