"""GPU parity of the operator-reuse modes (Sec. 6, Fig. simstrats: strategies
I, II, III) against the oracle, through the C-ABI: after a surface change
every level's operator and diagonal, the V-cycle (1e-11) and the PCG solve
(equal iteration counts, 1e-10) match the oracle hierarchy under the same
mode.  FP64 differences are summation order only."""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from paper_2009_00705_amd import workloads as W

from gpu_common import dev, host, make_pair, rel_err

pytestmark = pytest.mark.gpu

CASES = {
    "box5x5_L3_P6_xy": (lambda: W.box_mesh(5, 3), 6, dict(coarsening="xy")),
    "cyl_P3": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3), 3, {}),
}


def _eta2(xy):
    return 0.08 * np.cos(xy[:, 1]) - 0.03 * np.sin(2 * xy[:, 0] + xy[:, 1])


@pytest.mark.parametrize("mode", ["none", "t0", "lin"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_reuse_mode_parity(case, mode):
    import torch
    mk, P, kw = CASES[case]
    mesh = mk()
    print(f"\n[reuse {case} {mode}]", flush=True)
    h, ctx = make_pair(mesh, P, omega="auto", smoother="chebyshev", nu1=3, nu2=3, **kw)
    h.set_reuse(mode)
    ctx.set_reuse(mode)
    num = M.Numbering(mesh, P)
    h.set_surface(_eta2(M.unique_xy_2d(mesh, num)))
    ctx.set_surface(dev(_eta2(ctx.surface_xy())))
    torch.cuda.synchronize()
    for lvl, lv in enumerate(h.levels):
        x = W.random_vector(lv.num.n_dof, 11 + lvl)
        y = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
        ctx.apply(lvl, dev(x), y, "fp64", masked=False)
        assert rel_err(host(y), lv.op.apply(x)) < 1e-12, (case, mode, lvl)
        d = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
        ctx.diagonal(lvl, d)
        assert rel_err(host(d), lv.diag) < 1e-12, (case, mode, lvl)
    lv = h.levels[0]
    r = np.where(lv.free, W.random_vector(lv.num.n_dof, 3), 0.0)
    z = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
    ctx.vcycle(dev(r), z)
    assert rel_err(host(z), h.vcycle(r)) < 1e-11
    xyz_o = M.node_xyz(mesh, num, h.eta2d)
    phi_o = W.linear_wave(xyz_o[:, 0], xyz_o[:, 1], xyz_o[:, 2], 1.0)
    xyz_l = ctx.node_xyz(0)
    surf = W.linear_wave(xyz_l[:, 0], xyz_l[:, 1], xyz_l[:, 2], 1.0)[num.surface_nodes]
    ref = K.solve(h, phi_o, method="pcg", rtol=1e-10, imax=300)
    phi = torch.zeros(num.n_dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(phi, phi_surf=dev(surf), rtol=1e-10, imax=300)
    assert rc == 0 and st["iters"] == ref.iters, (st["iters"], ref.iters)
    assert rel_err(host(phi), ref.phi) < 1e-10
    ctx.close()
