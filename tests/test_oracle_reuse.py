"""Pins of the oracle's operator-reuse modes (Sec. 6, Fig. simstrats), each
against a hierarchy built from scratch at the surface the mode should use:
strategy III ("none"): every level at the new surface; strategy I ("t0"):
coarse levels and the finest diagonal of the first surface, the finest
operator of the new one; strategy II ("lin"): coarse levels on the flat
surface, the finest level (diagonal included) at the new one.  Under every
mode the outer iteration solves the new surface's problem."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from oracle.mg import Hierarchy
from paper_2009_00705_amd import workloads as W


def _setup():
    m = W.box_mesh(3, 2)
    num = M.Numbering(m, 4)
    xy = M.unique_xy_2d(m, num)
    return m, num, 0.05 * np.sin(xy[:, 0]), 0.08 * np.cos(xy[:, 1])


def _same_ops(la, lb, x):
    np.testing.assert_allclose(la.op.apply(x), lb.op.apply(x), rtol=0, atol=1e-12 * np.abs(lb.op.apply(x)).max())


@pytest.mark.parametrize("mode", ["none", "t0", "lin"])
def test_reuse_modes_against_fresh_hierarchies(mode):
    m, num, e1, e2 = _setup()
    kw = dict(smoother="chebyshev", nu1=3, nu2=3, omega=0.3)
    h = Hierarchy(m, 4, eta2d=e1, **kw)
    h.set_reuse(mode)
    h.set_surface(e2)
    first, new, flat = (Hierarchy(m, 4, eta2d=e, **kw) for e in (e1, e2, np.zeros_like(e1)))
    rng = np.random.default_rng(0)
    coarse_ref = {"none": new, "t0": first, "lin": flat}[mode]
    diag_ref = first if mode == "t0" else new
    for i, lv in enumerate(h.levels):
        x = rng.standard_normal(lv.num.n_dof)
        _same_ops(lv, (new if i == 0 else coarse_ref).levels[i], x)
        ref = diag_ref if i == 0 else coarse_ref
        np.testing.assert_allclose(lv.diag, ref.levels[i].diag, rtol=1e-13)
    xyz = M.node_xyz(m, num, e2)
    phi = W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)
    r = K.solve(h, phi, rtol=1e-11, imax=100)
    d = K.direct_solve(new, phi)
    assert np.abs(r.phi - d).max() < 1e-8 * np.abs(d).max()
