"""GPU parity of the overlapping additive Schwarz smoother (Sec. 5.2,
eq. Mass, eq. weights) against the FP64 oracle, through the C-ABI.

Tolerances: the local inverses come from a blocked Gauss-Jordan elimination
on the GPU and from LAPACK in the oracle; the local matrices have condition
numbers of about 1e3 at P = 6, so the FP64 results agree to ~1e-13 and are
checked at 1e-10 (smoothing, V-cycle, solve; equal iteration counts).  FP32
inverses carry 2^-24 relative rounding per entry (checked at 1e-4); BF16
inverses 2^-9 per entry, summed over subdomains of a few hundred nodes
(checked at 5e-2), and their V-cycle must still converge the Krylov loop in
about the FP64 iteration count.
"""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from paper_2009_00705_amd import workloads as W

from gpu_common import dev, host, make_pair, rel_err

pytestmark = pytest.mark.gpu

CASES = {
    # name: (mesh factory, P, coarsening, overlap)
    "box5x5_L3_P6": (lambda: W.box_mesh(5, 3), 6, "both", 1),
    "box5x5_L3_P6_xy": (lambda: W.box_mesh(5, 3), 6, "xy", 1),
    "cyl_P3": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3), 3, "both", 1),
    "cyl_P3_block": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3), 3, "both", 0),
    "box3_L2_P4_refined_xy": (lambda: W.box_mesh(3, 2), 4, "xy", -1),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    mk, P, seq, ov = CASES[request.param]
    print(f"\n[schwarz case {request.param}]", flush=True)
    h, ctx = make_pair(mk(), P, omega="auto", smoother="schwarz", overlap=ov, coarsening=seq, nu1=1, nu2=1)
    yield request.param, h, ctx
    ctx.close()


def _rand(n, seed):
    return W.random_vector(n, seed)


def test_automatic_damping_matches_oracle():
    """omega = 4/(3 rho), rho the power estimate of the spectral radius of S^-1 A
    (same counter-based start vector and steps as the oracle)."""
    mk, P, seq, ov = CASES["cyl_P3"]
    h, ctx = make_pair(mk(), P, omega="lib", smoother="schwarz", overlap=ov, coarsening=seq)
    om, _, _ = ctx.params()
    for i, lv in enumerate(h.levels[:-1]):
        assert abs(om[i] - lv.omega) < 1e-9 * lv.omega, (i, om[i], lv.omega)
    ctx.close()


def test_subdomain_sizes_match(pair):
    name, h, ctx = pair
    for i, lv in enumerate(h.levels[:-1]):
        info = ctx.schwarz_info(i)
        assert info["total"] == sum(s.size for s in lv.schwarz.sub)
        assert info["max_size"] == max(s.size for s in lv.schwarz.sub)


def test_smoothing_fp64_every_level(pair):
    import torch
    name, h, ctx = pair
    for i, lv in enumerate(h.levels[:-1]):
        n = lv.num.n_dof
        f = np.where(lv.free, _rand(n, 70 + i), 0.0)
        u = np.where(lv.free, _rand(n, 80 + i), 0.0)
        ud = dev(u)
        ctx.smooth(i, dev(f), ud, sweeps=2)
        torch.cuda.synchronize()
        assert rel_err(host(ud), h.smooth(i, u, f, 2)) < 1e-10, (name, i)


def test_vcycle_fp64(pair):
    import torch
    name, h, ctx = pair
    lv = h.levels[0]
    r = np.where(lv.free, _rand(lv.num.n_dof, 90), 0.0)
    z = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
    ctx.vcycle(dev(r), z)
    assert rel_err(host(z), h.vcycle(r)) < 1e-10


def test_pcg_solve_fp64(pair):
    import torch
    name, h, ctx = pair
    num = h.levels[0].num
    xyz_o = M.node_xyz(h.mesh, num, h.eta2d)
    phi_o = W.linear_wave(xyz_o[:, 0], xyz_o[:, 1], xyz_o[:, 2], 1.0)
    xyz_l = ctx.node_xyz(0)
    surf = W.linear_wave(xyz_l[:, 0], xyz_l[:, 1], xyz_l[:, 2], 1.0)[num.surface_nodes]
    ref = K.solve(h, phi_o, method="pcg", rtol=1e-10, imax=300)
    phi = torch.zeros(num.n_dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(phi, phi_surf=dev(surf), rtol=1e-10, imax=300)
    assert rc == 0 and st["iters"] == ref.iters, (st["iters"], ref.iters)
    np.testing.assert_allclose(st["res_hist"], ref.res_hist, rtol=1e-7, atol=1e-10 * ref.res_hist[0])
    assert rel_err(host(phi), ref.phi) < 1e-9


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16g", 5e-2)])
def test_smoothing_low_precision(pair, prec, tol):
    import torch
    name, h, ctx = pair
    for i, lv in enumerate(h.levels[:-1]):
        n = lv.num.n_dof
        f = np.where(lv.free, _rand(n, 100 + i), 0.0)
        ud = torch.zeros(n, dtype=torch.float32, device="cuda")
        ctx.smooth(i, dev(f, torch.float32), ud, sweeps=1, precision=prec)
        want = h.smooth(i, np.zeros(n), f.astype(np.float32).astype(np.float64), 1)
        assert rel_err(host(ud), want) < tol, (name, i, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16g"])
def test_mixed_precision_solve_converges(pair, prec):
    import torch
    name, h, ctx = pair
    num = h.levels[0].num
    xyz_l = ctx.node_xyz(0)
    surf = W.linear_wave(xyz_l[:, 0], xyz_l[:, 1], xyz_l[:, 2], 1.0)[num.surface_nodes]
    phi64 = torch.zeros(num.n_dof, dtype=torch.float64, device="cuda")
    rc, st64 = ctx.solve(phi64, phi_surf=dev(surf), rtol=1e-10, imax=300)
    ctx.set_solver(precision=prec, krylov="fpcg")
    try:
        phi = torch.zeros(num.n_dof, dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(phi, phi_surf=dev(surf), rtol=1e-10, imax=300)
    finally:
        ctx.set_solver(precision="fp64", krylov="pcg")
    assert rc == 0 and st["rel_res"] <= 1e-10
    assert st["iters"] <= st64["iters"] + 3, (st["iters"], st64["iters"])
    assert rel_err(host(phi), host(phi64)) < 1e-8


def test_schwarz_kernel_timing_runs(pair):
    name, h, ctx = pair
    for prec in ("fp64", "fp32", "bf16g"):
        ms = ctx.time_kernel("schwarz", level=0, precision=prec, reps=2)
        assert ms > 0


def test_chunked_setup_and_partial_storage_are_bitwise_equal():
    """Inverses kept only in FP32 and BF16, built in many small FP64 chunks,
    give bitwise the FP32 / BF16 smoothing of a context that keeps every copy
    (the per-subdomain arithmetic does not depend on the chunking); a step in
    a precision whose copy is not kept is refused."""
    import torch
    from paper_2009_00705_amd import pmg
    mesh = W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3)
    kw = dict(P=3, smoother="schwarz", overlap=1, nu1=1, nu2=1, omega=[0.8] * 8)
    full = pmg.Context(mesh, **kw)
    part = pmg.Context(mesh, schwarz_store="fp32,bf16", schwarz_chunk=5000, **kw)
    xy = full.surface_xy()
    eta = dev(W.surface_elevation_c2(xy[:, 0], xy[:, 1]))
    full.set_surface(eta)
    part.set_surface(eta)
    for lvl in range(full.n_levels - 1):
        n = full.levels[lvl]["n_dof"]
        mask = torch.from_numpy(full.dirichlet_mask(lvl) == 0).cuda()
        f = dev(_rand(n, 7 + lvl), torch.float32) * mask
        for prec in ("fp32", "bf16g"):
            a = torch.zeros(n, dtype=torch.float32, device="cuda")
            b = torch.zeros_like(a)
            full.smooth(lvl, f, a, sweeps=2, precision=prec)
            part.smooth(lvl, f, b, sweeps=2, precision=prec)
            assert torch.equal(a, b), (lvl, prec)
    with pytest.raises(pmg.PmgError):
        part.smooth(0, dev(np.zeros(full.levels[0]["n_dof"])),
                    torch.zeros(full.levels[0]["n_dof"], dtype=torch.float64, device="cuda"), sweeps=1)
    full.close()
    part.close()
