"""Coloured direct-stiffness sum (pmg_options.dss = 1) against the
node-centric sum (the default) on the same context settings.

The two add the same element values (Sec. 3.1's assembly sum) in different
orders, so every operator apply, transfer and smoothing step agrees to the
rounding of the summation order; the solves converge in the same number of
iterations to the same tolerance, and a coloured solve is bitwise
reproducible (no atomics).  The node-centric path itself is pinned to the
oracle by the parity tests.
"""
import numpy as np
import pytest

from gpu_common import host, rel_err
from paper_2009_00705_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    # name: (mesh factory, P, coarsening)
    "box5x5_L3_P6_xy": (lambda: W.box_mesh(5, 3), 6, "xy"),
    "cyl_P3_both": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3), 3, "both"),
    "box2_L1_P8_xy": (lambda: W.box_mesh(2, 1), 8, "xy"),
}
# summation-order rounding of one apply, relative to the output's max
TOL = {"fp64": 1e-13, "fp32": 2e-6, "bf16g": 2e-6, "bf16x3": 2e-6}


def _ctx(mesh, P, coarsening, dss):
    import torch
    from paper_2009_00705_amd import pmg
    ctx = pmg.Context(mesh, P=P, coarse="chebyshev", smoother="chebyshev", nu1=3, nu2=3, coarsening=coarsening,
                      smooth_ratio=8.0, dss=dss)
    xy = ctx.surface_xy()
    ctx.set_surface(torch.from_numpy(0.5 * W.surface_elevation_c2(xy[:, 0], xy[:, 1])).cuda())
    return ctx


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    mk, P, co = CASES[request.param]
    mesh = mk()
    a, b = _ctx(mesh, P, co, 0), _ctx(mesh, P, co, 1)
    yield request.param, a, b
    a.close()
    b.close()


def test_colours_cover_every_triangle_once(pair):
    name, a, b = pair
    col = b.dss_colours(0)
    assert col.shape == (a.n_tri,) and col.min() == 0
    assert np.bincount(col).min() > 0, name  # no empty colour


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16g"])
def test_apply_matches_node_centric_sum(pair, prec):
    import torch
    name, a, b = pair
    rng = np.random.default_rng(11)
    dt = torch.float64 if prec == "fp64" else torch.float32
    for lvl, info in enumerate(a.levels):
        x = torch.from_numpy(rng.standard_normal(info["n_dof"])).to(dt).cuda()
        ya = torch.zeros_like(x)
        yb = torch.zeros_like(x)
        for rep in range(2):  # the accumulator is back at zero after every sum
            a.apply(lvl, x, ya, precision=prec)
            b.apply(lvl, x, yb, precision=prec)
            err = np.abs(host(ya) - host(yb)).max() / np.abs(host(ya)).max()
            assert err < TOL[prec], (name, lvl, prec, rep, err)


def test_transfers_match_node_centric_sum(pair):
    import torch
    name, a, b = pair
    rng = np.random.default_rng(12)
    for lvl in range(a.n_levels - 1):
        nf, nc = a.levels[lvl]["n_dof"], a.levels[lvl + 1]["n_dof"]
        xf = torch.from_numpy(rng.standard_normal(nf)).cuda()
        xc = torch.from_numpy(rng.standard_normal(nc)).cuda()
        outs = []
        for ctx in (a, b):
            yc = torch.zeros(nc, dtype=torch.float64, device="cuda")
            yf = torch.zeros(nf, dtype=torch.float64, device="cuda")
            ctx.restrict(lvl, xf, yc)
            ctx.prolong(lvl, xc, yf)
            outs.append((host(yc), host(yf)))
        assert rel_err(outs[0][0], outs[1][0]) < 1e-13, (name, lvl, "restrict")
        assert rel_err(outs[0][1], outs[1][1]) < 1e-13, (name, lvl, "prolong")


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_solves_match_and_repeat_bitwise(pair, prec):
    import torch
    name, a, b = pair
    if prec == "bf16x3" and a.levels[0]["order"] != 6:
        pytest.skip("split-BF16 operators at in-plane order 6 only")
    xy = a.surface_xy()
    eta = 0.5 * W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    surf = torch.from_numpy(W.mode_sum(xy[:, 0], xy[:, 1], eta, W.mode_amplitudes(3), W.mode_pairs())).cuda()
    n = a.levels[0]["n_dof"]
    res = {}
    for key, ctx in (("node", a), ("colour", b), ("colour2", b)):
        ctx.set_solver(prec, "pcg" if prec == "fp64" else "fpcg")
        phi = torch.zeros(n, dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(phi, phi_surf=surf, rtol=1e-8, imax=200)
        assert rc == 0 and st["rel_res"] <= 1e-8, (name, key, st["rel_res"])
        res[key] = (host(phi), st["iters"], np.asarray(st["res_hist"]))
    assert abs(res["node"][1] - res["colour"][1]) <= 1, (name, res["node"][1], res["colour"][1])
    assert rel_err(res["node"][0], res["colour"][0]) < 1e-7, name
    np.testing.assert_array_equal(res["colour"][0], res["colour2"][0])
    np.testing.assert_array_equal(res["colour"][2], res["colour2"][2])


def test_time_kernel_runs_the_coloured_sum(pair):
    name, a, b = pair
    for ctx in (a, b):
        assert ctx.time_kernel("assemble", 0, "fp32", reps=3) > 0.0, name
