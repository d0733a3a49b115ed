"""GPU parity of every hot-path step against the FP64 oracle, through the C-ABI.

Floating-point tolerances: FP64 steps 1e-12 relative to the output's max
(different summation orders only); the FP64 solve 1e-10 (residual history
and potential, equal iteration counts).  FP32 steps carry G and vectors
rounded to 2^-24: 2e-5.  Split-BF16 products (hi/lo halves, about 16
significant bits, FP32 G from the column factors): 2e-4.  BF16 geometric
factors or reference tables carry 2^-9 relative rounding: 1e-2.  Integer
maps are bit-exact (tests/test_lib_host.py).
"""
import numpy as np
import pytest

from oracle import krylov as K
from oracle import mesh as M
from paper_2009_00705_amd import workloads as W

from gpu_common import dev, host, make_pair, rel_err

pytestmark = pytest.mark.gpu

CASES = {
    # name: (mesh factory, P)
    "c1": (lambda: W.config_mesh("c1"), 4),
    "box5x5_L3_P6": (lambda: W.box_mesh(5, 3), 6),        # several blocks + ragged tail
    "cyl_P3": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3), 3),
    "box2_L1_P8": (lambda: W.box_mesh(2, 1), 8),
    # four layers: batches of 16 prisms hold whole columns; these cases run
    # with pmg_options.fused_sum = 1 (the MFMA levels write column sums and a
    # node kernel finishes them), so every check below covers that path too
    "box5x5_L4_P6": (lambda: W.box_mesh(5, 4), 6),
    "cyl_L4_P3": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=4), 3),
}
# in-plane-first hierarchies (anisotropic orders, e.g. (6,6) (3,6) (1,6) (1,3) (1,1))
XY_CASES = {k + "_xy": v for k, v in CASES.items() if k != "c1"}
# anisotropic finest levels with the equal-order sequence (Sec. 6.2, Table
# BTcoarse3D): (5,3) (3,3) (1,1), and vertical-first (3,6) (3,3) (1,1)
EQ_CASES = {
    "box5x5_L3_P5_eq53": (lambda: W.box_mesh(5, 3), 5),
    "cyl_P3_eq36": (CASES["cyl_P3"][0], 3),
}
EQ_PZ = {"box5x5_L3_P5_eq53": 3, "cyl_P3_eq36": 6}
ALL = dict(CASES, **XY_CASES, **EQ_CASES)


def _opts(name):
    o = {"fused_sum": 1} if "_L4_" in name else {}
    if name in EQ_PZ:
        o.update({"coarsening": "equal", "PZ": EQ_PZ[name]})
    elif name.endswith("_xy"):
        o["coarsening"] = "xy"
    return o


@pytest.fixture(scope="module", params=sorted(ALL))
def pair(request):
    mk, P = ALL[request.param]
    h, ctx = make_pair(mk(), P, **_opts(request.param))
    yield request.param, h, ctx
    ctx.close()


def _rand(n, seed):
    return W.random_vector(n, seed)


def test_operator_fp64_all_levels(pair):
    name, h, ctx = pair
    import torch
    for lvl, lv in enumerate(h.levels):
        n = lv.num.n_dof
        x = _rand(n, 10 + lvl)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.apply(lvl, dev(x), y, "fp64", masked=False)
        ref = lv.op.apply(x)
        assert rel_err(host(y), ref) < 1e-12, (name, lvl)
        ctx.apply(lvl, dev(x), y, "fp64", masked=True)
        assert rel_err(host(y), lv.A(x)) < 1e-12, (name, lvl)


# (precision, bar on levels of in-plane order 6, bar elsewhere).  bf16x3 runs its
# split-BF16 products (about 16 significant bits, G formed in FP32 from the
# column factors) at in-plane order 6 and FP32 arithmetic on BF16-stored G
# (2^-9 relative rounding of G) elsewhere; bf16x2 rounds the reference tables
# to BF16 (2^-9) on the split levels.
LOWP_BARS = [("fp32", 2e-5, 2e-5), ("bf16", 1e-2, 1e-2), ("bf16g", 1e-2, 1e-2), ("bf16x3", 2e-4, 1e-2),
             ("bf16x2", 1e-2, 1e-2)]


@pytest.mark.parametrize("prec,tol6,tol", LOWP_BARS)
def test_operator_low_precision(pair, prec, tol6, tol):
    name, h, ctx = pair
    import torch
    for lvl, lv in enumerate(h.levels):
        n = lv.num.n_dof
        x = _rand(n, 3 + lvl)
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        ctx.apply(lvl, dev(x, torch.float32), y, prec, masked=True)
        bar = tol6 if ctx.levels[lvl]["order"] == 6 else tol
        assert rel_err(host(y), lv.A(x.astype(np.float32).astype(np.float64))) < bar, (name, lvl)


@pytest.fixture(scope="module")
def multi_batch():
    """A mesh with more prisms than the element operators keep resident
    workgroups for 16-prism batches (53 x 53 split quads x 3 layers = 16854
    prisms = 1053 full batches and a ragged one of 6): every workgroup of the
    resident grids (256 FP64, 512 FP32 / BF16 / split) strides over two or
    more batches, reusing its LDS tables, and the last batch is partial.  The
    oracle's unmasked operator of every in-plane-first level is computed once."""
    import torch
    from types import SimpleNamespace
    from oracle.mg import level_orders
    from oracle.operator import LevelGeometry, StiffnessOperator, element_node_xyz
    from paper_2009_00705_amd import pmg
    from gpu_common import surface_eta
    mesh = W.box_mesh(53, 3)
    num_f = M.Numbering(mesh, 6)
    assert num_f.n_elem == 16854 and num_f.n_elem % 16 == 6
    eta = surface_eta(M.unique_xy_2d(mesh, num_f), "wavy")
    xyz = element_node_xyz(mesh, num_f, eta)
    ref = []
    for lvl, order in enumerate(level_orders(6, "xy")):
        num = M.Numbering(mesh, *order)
        op = StiffnessOperator(num, LevelGeometry(order, 6, xyz))
        x = _rand(num.n_dof, 70 + lvl)
        x32 = x.astype(np.float32).astype(np.float64)
        ref.append((order, x, op.apply(x), op.apply(x32)))
        del op
    ctxs = {}
    for g in ("column", "stored"):
        c = pmg.Context(mesh, P=6, geometry=g, coarsening="xy", smoother="chebyshev", nu1=3, nu2=3,
                        coarse="chebyshev")
        c.set_surface(dev(surface_eta(c.surface_xy(), "wavy")))
        ctxs[g] = c
    torch.cuda.synchronize()
    yield ref, ctxs
    for c in ctxs.values():
        c.close()


@pytest.mark.parametrize("geometry", ["column", "stored"])
def test_multi_batch_operator_parity(multi_batch, geometry):
    """Every level, every precision, element by element at all nodes against the
    oracle on the multi-batch mesh: FP64 1e-12, FP32 2e-5, split BF16 2e-4 at
    in-plane order 6, 1e-2 for BF16-rounded factors or tables (bars of
    test_operator_low_precision).  With stored G the BF16 and split-BF16 kernels
    take their prefetch path (the next q tile's G words loaded under the
    current tile's products); the split kernel then reads BF16-rounded G, so its
    bar is the BF16 one."""
    import torch
    ref, ctxs = multi_batch
    ctx = ctxs[geometry]
    for lvl, (order, x, y64, y32) in enumerate(ref):
        assert ctx.levels[lvl]["n_dof"] == x.size and ctx.levels[lvl]["order"] == order[0]
        y = torch.empty(x.size, dtype=torch.float64, device="cuda")
        ctx.apply(lvl, dev(x), y, "fp64", masked=False)
        assert rel_err(host(y), y64) < 1e-12, (geometry, order, "fp64")
        for prec, tol6, tol in LOWP_BARS:
            y = torch.empty(x.size, dtype=torch.float32, device="cuda")
            ctx.apply(lvl, dev(x, torch.float32), y, prec, masked=False)
            bar = tol6 if (order[0] == 6 and geometry == "column") else tol
            err = rel_err(host(y), y32)
            assert err < bar, (geometry, order, prec, err)


def test_split_bf16_products_match_fp32_products(pair):
    """On levels of in-plane order 6 bf16x3 and fp32 form the same FP32 G from
    the column factors; their products differ only by the split's rounding
    (about 2^-16 relative), far below the 2^-9 of a single BF16 product: 1e-4.
    The other levels run bf16x3 as bf16g (the same kernel: equal)."""
    name, h, ctx = pair
    import torch
    for lvl, lv in enumerate(h.levels):
        n = lv.num.n_dof
        split = ctx.levels[lvl]["order"] == 6
        x = dev(_rand(n, 7 + lvl), torch.float32)
        y3 = torch.empty(n, dtype=torch.float32, device="cuda")
        yr = torch.empty_like(y3)
        ctx.apply(lvl, x, y3, "bf16x3", masked=True)
        ctx.apply(lvl, x, yr, "fp32" if split else "bf16g", masked=True)
        assert rel_err(host(y3), host(yr)) < (1e-4 if split else 1e-15), (name, lvl)


def test_diagonal(pair):
    name, h, ctx = pair
    import torch
    for lvl, lv in enumerate(h.levels):
        d = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
        ctx.diagonal(lvl, d)
        assert rel_err(host(d), lv.diag) < 1e-12


def test_transfers(pair):
    name, h, ctx = pair
    import torch
    for i in range(len(h.levels) - 1):
        lf, lc = h.levels[i], h.levels[i + 1]
        xc = np.where(lc.free, _rand(lc.num.n_dof, 20 + i), 0)
        yf = torch.empty(lf.num.n_dof, dtype=torch.float64, device="cuda")
        ctx.prolong(i, dev(xc), yf)
        assert rel_err(host(yf), h.prolong(i, xc)) < 1e-12
        xf = _rand(lf.num.n_dof, 30 + i)
        yc = torch.empty(lc.num.n_dof, dtype=torch.float64, device="cuda")
        ctx.restrict(i, dev(xf), yc)
        assert rel_err(host(yc), h.restrict(i, xf)) < 1e-12


def test_smoother_and_coarse_solve(pair):
    name, h, ctx = pair
    import torch
    lv = h.levels[0]
    f = np.where(lv.free, _rand(lv.num.n_dof, 40), 0)
    u = np.where(lv.free, _rand(lv.num.n_dof, 41), 0)
    ud = dev(u)
    ctx.smooth(0, dev(f), ud, sweeps=3)
    assert rel_err(host(ud), h.smooth(0, u, f, 3)) < 1e-12
    lc = h.levels[-1]
    fc = np.where(lc.free, _rand(lc.num.n_dof, 42), 0)
    uc = torch.empty(lc.num.n_dof, dtype=torch.float64, device="cuda")
    ctx.coarse_solve(dev(fc), uc)
    assert rel_err(host(uc), h.coarse_solve(fc)) < 1e-11


def test_vcycle(pair):
    name, h, ctx = pair
    import torch
    lv = h.levels[0]
    r = np.where(lv.free, _rand(lv.num.n_dof, 50), 0)
    z = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
    ctx.vcycle(dev(r), z)
    assert rel_err(host(z), h.vcycle(r)) < 1e-11


def _dirichlet(h, ctx, k=1.0):
    num = h.levels[0].num
    xyz_o = M.node_xyz(h.mesh, num, h.eta2d)
    phi_o = W.linear_wave(xyz_o[:, 0], xyz_o[:, 1], xyz_o[:, 2], k)
    xyz_l = ctx.node_xyz(0)
    phi_l = W.linear_wave(xyz_l[:, 0], xyz_l[:, 1], xyz_l[:, 2], k)
    surf_l = phi_l[num.surface_nodes]
    return phi_o, surf_l


@pytest.fixture(scope="module", params=sorted(ALL))
def solve_pair(request):
    mk, P = ALL[request.param]
    h, ctx = make_pair(mk(), P, omega="auto", **_opts(request.param))
    yield request.param, h, ctx
    ctx.close()


def test_auto_omega_matches_oracle():
    h, ctx = make_pair(W.config_mesh("c1"), 4, omega="lib")
    om, _, _ = ctx.params()
    for i, lv in enumerate(h.levels[:-1]):
        assert abs(om[i] - lv.omega) < 1e-9 * lv.omega
    ctx.close()


def test_pcg_solve_parity(solve_pair):
    name, h, ctx = solve_pair
    import torch
    phi_o, surf_l = _dirichlet(h, ctx)
    ref = K.solve(h, phi_o, method="pcg", rtol=1e-10, imax=300)
    phi = torch.zeros(h.levels[0].num.n_dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(phi, phi_surf=dev(surf_l), rtol=1e-10, imax=300)
    assert rc == 0
    assert st["iters"] == ref.iters
    np.testing.assert_allclose(st["res_hist"], ref.res_hist, rtol=1e-10 * 10, atol=1e-10 * ref.res_hist[0])
    assert rel_err(host(phi), ref.phi) < 1e-10
    assert st["rel_res"] <= 1e-10
    # a second solve is bitwise identical
    phi2 = torch.zeros_like(phi)
    ctx.solve(phi2, phi_surf=dev(surf_l), rtol=1e-10, imax=300)
    assert torch.equal(phi, phi2)


@pytest.fixture(scope="module", params=["box5x5_L3_P6", "cyl_P3", "box5x5_L3_P6_nu22"])
def cheb_pair(request):
    # the last case smooths the levels below the finest with 2 + 2 sweeps
    name = request.param.replace("_nu22", "")
    kw = dict(nu1_coarse=2, nu2_coarse=2) if request.param.endswith("_nu22") else {}
    mk, P = CASES[name]
    h, ctx = make_pair(mk(), P, omega="auto", smoother="chebyshev", nu1=3, nu2=3, **kw)
    yield request.param, h, ctx
    ctx.close()


def test_chebyshev_smoother_vcycle_and_solve(cheb_pair):
    name, h, ctx = cheb_pair
    import torch
    lv = h.levels[0]
    f = np.where(lv.free, _rand(lv.num.n_dof, 60), 0)
    u = np.where(lv.free, _rand(lv.num.n_dof, 61), 0)
    ud = dev(u)
    ctx.smooth(0, dev(f), ud, sweeps=3)
    assert rel_err(host(ud), h.smooth(0, u, f, 3)) < 1e-12
    z = torch.empty(lv.num.n_dof, dtype=torch.float64, device="cuda")
    ctx.vcycle(dev(f), z)
    assert rel_err(host(z), h.vcycle(f)) < 1e-11
    phi_o, surf_l = _dirichlet(h, ctx)
    ref = K.solve(h, phi_o, method="pcg", rtol=1e-10, imax=300)
    phi = torch.zeros(lv.num.n_dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(phi, phi_surf=dev(surf_l), rtol=1e-10, imax=300)
    assert rc == 0 and st["iters"] == ref.iters
    np.testing.assert_allclose(st["res_hist"], ref.res_hist, rtol=1e-9, atol=1e-10 * ref.res_hist[0])
    assert rel_err(host(phi), ref.phi) < 1e-10


@pytest.mark.parametrize("case", ["box5x5_L3_P6", "cyl_P3"])
def test_coarse_chebyshev_parity(case):
    """Chebyshev coarse solve (assembled P = 1 matrix, fused step) against the
    oracle's Chebyshev iteration on the same interval and degree: coarse solve
    and V-cycle to 1e-11, PCG solve with equal iteration counts to 1e-10."""
    import torch
    from paper_2009_00705_amd import pmg
    from oracle.mg import Hierarchy
    mk, P = CASES[case]
    mesh = mk()
    ctx = pmg.Context(mesh, P=P, coarse="chebyshev")
    xy = ctx.surface_xy()
    ctx.set_surface(dev(W.surface_elevation_c2(xy[:, 0], xy[:, 1])))
    info = ctx.coarse_info()
    assert info["mode"] == "chebyshev" and info["degree"] >= 4
    assert 0 < info["lmin"] < info["lmax"]
    om, _, _ = ctx.params()
    num = M.Numbering(mesh, P)
    eta_o = W.surface_elevation_c2(*M.unique_xy_2d(mesh, num).T)
    h = Hierarchy(mesh, P, eta2d=eta_o, omega=list(om), coarse="chebyshev",
                  cheb=(info["degree"], info["lmin"], info["lmax"]))
    nc = h.levels[-1].num.n_dof
    fc = np.where(h.levels[-1].free, _rand(nc, 31), 0.0)
    uc = torch.zeros(nc, dtype=torch.float64, device="cuda")
    ctx.coarse_solve(dev(fc), uc)
    assert rel_err(host(uc), h.coarse_solve(fc)) < 1e-11
    n0 = h.levels[0].num.n_dof
    r = np.where(h.levels[0].free, _rand(n0, 32), 0.0)
    z = torch.zeros(n0, dtype=torch.float64, device="cuda")
    ctx.vcycle(dev(r), z)
    assert rel_err(host(z), h.vcycle(r)) < 1e-11
    phi_o, surf_l = _dirichlet(h, ctx)
    ref = K.solve(h, phi_o, method="pcg", rtol=1e-10, imax=300)
    phi = torch.zeros(n0, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(phi, phi_surf=dev(surf_l), rtol=1e-10, imax=300)
    assert rc == 0 and st["iters"] == ref.iters
    assert rel_err(host(phi), ref.phi) < 1e-10
    # FP32 coarse solve: same result to single precision
    u32 = torch.zeros(nc, dtype=torch.float32, device="cuda")
    ctx.coarse_solve(dev(fc, torch.float32), u32, precision="fp32")
    assert rel_err(host(u32), h.coarse_solve(fc)) < 1e-4
    ctx.close()


@pytest.mark.parametrize("case", ["box5x5_L3_P6", "cyl_P3_xy", "box2_L1_P8_xy"])
def test_column_geometry_matches_stored_factors(case):
    """The element operators that form G from the per-column factors (the
    sigma-transform shares x_r .. y_s and eta across a column) give the same
    product as those that stream the stored G: FP64 to 1e-13 relative (a
    different rounding order of the same factors), FP32 to 2e-6 (one more
    rounding of the factors).  The split-BF16 products read a BF16 copy of
    the stored G (2^-9 relative rounding) but form G from FP32 column
    factors: 1e-2."""
    import torch
    from paper_2009_00705_amd import pmg
    from gpu_common import surface_eta
    mk, P = ALL[case]
    mesh = mk()
    ctxs = {g: pmg.Context(mesh, P=P, geometry=g, **_opts(case)) for g in ("stored", "column")}
    for c in ctxs.values():
        c.set_surface(dev(surface_eta(c.surface_xy(), "wavy")))
    for lvl in range(ctxs["column"].n_levels):
        n = ctxs["column"].levels[lvl]["n_dof"]
        for prec, tol in (("fp64", 1e-13), ("fp32", 2e-6), ("bf16x3", 1e-2)):
            dt = torch.float64 if prec == "fp64" else torch.float32
            x = dev(_rand(n, 40 + lvl), dt)
            ys = {g: torch.empty(n, dtype=dt, device="cuda") for g in ctxs}
            for g, c in ctxs.items():
                c.apply(lvl, x, ys[g], prec, masked=True)
            assert rel_err(host(ys["column"]), host(ys["stored"])) < tol, (case, lvl, prec)
    for c in ctxs.values():
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_stored_geometry_solves_match_column_solves(prec):
    """The whole solve (FP64 outer iteration, V-cycle in each precision) with
    stored G and with the column factors: FP64 iteration counts and residual
    histories agree to 1e-10, the mixed ones to the rounding of their
    geometric factors (iteration counts within one, potentials within 1e-8 of
    each other at rtol 1e-10)."""
    import torch
    from gpu_common import surface_eta
    from paper_2009_00705_amd import pmg
    mk, P = CASES["box5x5_L3_P6"]
    mesh = mk()
    out = {}
    for g in ("stored", "column"):
        ctx = pmg.Context(mesh, P=P, geometry=g, coarsening="xy", smoother="chebyshev", nu1=3, nu2=3)
        xy = ctx.surface_xy()
        ctx.set_surface(dev(surface_eta(xy, "wavy")))
        ctx.set_solver(prec, "pcg" if prec == "fp64" else "fpcg")
        phi = torch.zeros(ctx.levels[0]["n_dof"], dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(phi, phi_surf=dev(np.cos(xy[:, 0]) * np.cos(xy[:, 1])), rtol=1e-10, imax=300)
        assert rc == 0, (g, prec)
        out[g] = (st, host(phi))
        ctx.close()
    (ss, ps), (sc, pc) = out["stored"], out["column"]
    # the mixed V-cycles differ by their factors' rounding (BF16-stored G for bf16x3)
    assert abs(ss["iters"] - sc["iters"]) <= (0 if prec == "fp64" else 1)
    if prec == "fp64":
        np.testing.assert_allclose(sc["res_hist"], ss["res_hist"], rtol=1e-9, atol=1e-10 * ss["res_hist"][0])
    assert rel_err(pc, ps) < (1e-10 if prec == "fp64" else 1e-8)


@pytest.fixture(scope="module", params=["box5x5_L4_P6", "box5x5_L4_P6_xy", "cyl_L4_P3_xy", "c1"])
def fused_pair(request):
    """The same hierarchy with the direct-stiffness sum inside the element
    operators (default) and through the element-layout buffer and node-centric
    sum kernel (fused_sum = 0)."""
    import torch
    from paper_2009_00705_amd import pmg
    from gpu_common import surface_eta
    mk, P = ALL[request.param]
    mesh = mk()
    ctxs = []
    for fused in (1, 0):
        opts = dict(_opts(request.param), fused_sum=fused)
        c = pmg.Context(mesh, P=P, omega=[0.3] * 8, **opts)
        c.set_surface(dev(surface_eta(c.surface_xy(), "wavy")))
        ctxs.append(c)
    torch.cuda.synchronize()
    yield request.param, ctxs[0], ctxs[1]
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16g", "bf16x3"])
def test_fused_sum_equals_node_sum(fused_pair, prec):
    """y = A x on every level: the fused summation and the node-centric one add
    the same contributions in different orders (FP64 1e-13, FP32 2e-6 of the
    output's max), both masked and bitwise reproducible."""
    import torch
    name, cf, cu = fused_pair
    dt = torch.float64 if prec == "fp64" else torch.float32
    for lvl, info in enumerate(cf.levels):
        n = info["n_dof"]
        x = dev(_rand(n, 90 + lvl), dt)
        yf = torch.empty(n, dtype=dt, device="cuda")
        yf2 = torch.empty_like(yf)
        yu = torch.empty_like(yf)
        cf.apply(lvl, x, yf, prec, masked=True)
        cf.apply(lvl, x, yf2, prec, masked=True)
        cu.apply(lvl, x, yu, prec, masked=True)
        assert torch.equal(yf, yf2), (name, lvl, prec)
        assert rel_err(host(yf), host(yu)) < (1e-13 if prec == "fp64" else 2e-6), (name, lvl, prec)


def test_fused_sum_smoother_vcycle_and_solve(fused_pair):
    """Chebyshev smoothing, V-cycle and PCG solve with the fused summation match
    the node-centric summation (the FP64 Chebyshev steps, residual and the
    outer iteration's q = A p with its dot product all take the fused path)."""
    import torch
    name, cf, cu = fused_pair
    lv0 = cf.levels[0]
    n = lv0["n_dof"]
    nz = n // lv0["n_surface"]
    top = np.arange(n) % nz == nz - 1
    mask = ~top
    f = np.where(mask, _rand(n, 61), 0.0)
    outs = []
    for c in (cf, cu):
        c.set_solver("fp64", "pcg")
        u = torch.zeros(n, dtype=torch.float64, device="cuda")
        c.smooth(0, dev(f), u, sweeps=3)
        z = torch.empty(n, dtype=torch.float64, device="cuda")
        c.vcycle(dev(f), z)
        outs.append((host(u), host(z)))
    assert rel_err(outs[0][0], outs[1][0]) < 1e-12 and rel_err(outs[0][1], outs[1][1]) < 1e-11, name
    xyz = cf.node_xyz(0)
    surf = dev(np.ascontiguousarray(W.linear_wave(xyz[:, 0], xyz[:, 1], xyz[:, 2], 1.0)[top]))
    sols = []
    for c in (cf, cu):
        for prec in ("fp64", "bf16x3"):
            c.set_solver(prec, "pcg" if prec == "fp64" else "fpcg")
            phi = torch.zeros(n, dtype=torch.float64, device="cuda")
            rc, st = c.solve(phi, phi_surf=surf, rtol=1e-10, imax=300)
            assert rc == 0 and st["rel_res"] <= 1e-10, (name, prec, rc, st["rel_res"])
            sols.append((prec, st["iters"], host(phi)))
    for k in range(2):
        (_, it_f, pf), (_, it_u, pu) = sols[k], sols[k + 2]
        assert abs(it_f - it_u) <= 1, (name, sols[k][0], it_f, it_u)
        assert rel_err(pf, pu) < 1e-9, (name, sols[k][0])
