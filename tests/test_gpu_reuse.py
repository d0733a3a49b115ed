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


@pytest.mark.parametrize("prec", ["bf16g", "fp32", "bf16x3", "bf16"])
def test_t0_keeps_the_finest_low_precision_operator(prec):
    """Strategy I keeps the finest level's low-precision factors of the surface
    current when the mode is set (the native BF16 copies are built lazily, so
    setting the mode must build the pending ones first), while its FP64
    factors follow every surface: after a surface change the low-precision
    operator is bitwise the one of a context left at the first surface, and
    the FP64 operator that of a context set to the new one."""
    import torch
    from gpu_common import surface_eta
    from paper_2009_00705_amd import pmg
    mk, P, kw = CASES["box5x5_L3_P6_xy"]
    mesh = mk()
    a, b, c = (pmg.Context(mesh, P=P, **kw) for _ in range(3))
    xy = a.surface_xy()
    eta1, eta2 = dev(surface_eta(xy, "wavy")), dev(_eta2(xy))
    a.set_surface(eta1)
    b.set_surface(eta1)
    c.set_surface(eta2)
    a.set_reuse("t0")
    a.set_surface(eta2)
    n = a.levels[0]["n_dof"]
    x32 = dev(W.random_vector(n, 21), torch.float32)
    ya, yb = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(2))
    a.apply(0, x32, ya, prec)
    b.apply(0, x32, yb, prec)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb), prec
    x64 = dev(W.random_vector(n, 22))
    za, zc = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2))
    a.apply(0, x64, za, "fp64")
    c.apply(0, x64, zc, "fp64")
    assert rel_err(host(za), host(zc)) < 1e-13
    for ctx in (a, b, c):
        ctx.close()
