"""GPU parity of the free-surface time stepping (eq. FSeta, eq. FSphi, ERK4)
against the FP64 oracle, through the C-ABI.

Tolerances: gradients and w~ are the same formulas in a different summation
order (1e-12 relative).  The right-hand side and the ERK4 steps contain the
Laplace solve, exact (sparse LU) in the oracle and iterative (PCG to rtol
1e-12) in the library, so they agree to about 1e-10; checked at 1e-8.
"""
import math

import numpy as np
import pytest

from oracle import mesh as M
from oracle.fnpf import Surface
from paper_2009_00705_amd import workloads as W

from gpu_common import dev, host, rel_err

pytestmark = pytest.mark.gpu
G = 9.81

MESHES = {
    "box_P4": (lambda: W.box_mesh(4, 2), 4),
    "box_P6": (lambda: W.box_mesh(3, 2), 6),
    "cyl_P4": (lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=2), 4),
}


def _ctx(mesh, P):
    from paper_2009_00705_amd import pmg
    return pmg.Context(mesh, P=P, coarse="exact", smoother="chebyshev", nu1=3, nu2=3)


def _state(xy, amp=0.05):
    x, y = xy[:, 0], xy[:, 1]
    eta = amp * np.cos(x) * np.cos(0.5 * y) + 0.3 * amp * np.sin(2 * x + y)
    phis = 2 * amp * np.sin(x) * np.cos(y) - amp * np.cos(2 * y)
    return eta, phis


@pytest.fixture(scope="module", params=sorted(MESHES))
def pair(request):
    mk, P = MESHES[request.param]
    mesh = mk()
    print(f"\n[fnpf case {request.param}]", flush=True)
    s = Surface(mesh, P)
    ctx = _ctx(mesh, P)
    yield request.param, s, ctx
    ctx.close()


def test_surface_gradient(pair):
    name, s, ctx = pair
    xy = ctx.surface_xy()
    eta, phis = _state(xy)
    for f in (eta, phis):
        fx, fy = ctx.surface_grad(dev(f))
        ox, oy = s.grad(f)
        assert rel_err(host(fx), ox) < 1e-12 and rel_err(host(fy), oy) < 1e-12, name


def test_surface_w(pair):
    import torch
    name, s, ctx = pair
    xy = ctx.surface_xy()
    eta, _ = _state(xy)
    ctx.set_surface(dev(eta))
    phi = W.random_vector(s.num.n_dof, 5)
    w = ctx.surface_w(dev(phi))
    torch.cuda.synchronize()
    assert rel_err(host(w), s.w(phi, eta)) < 1e-12


def test_rhs(pair):
    import torch
    name, s, ctx = pair
    xy = ctx.surface_xy()
    eta, phis = _state(xy)
    phi = torch.zeros(s.num.n_dof, dtype=torch.float64, device="cuda")
    deta, dphis, rc, st = ctx.fnpf_rhs(dev(eta), dev(phis), phi, g=G, rtol=1e-12, imax=400)
    assert rc == 0
    oe, op, ophi = s.rhs(eta, phis, G)
    assert rel_err(host(phi), ophi) < 1e-10
    assert rel_err(host(deta), oe) < 1e-8 and rel_err(host(dphis), op) < 1e-8


def test_erk4_steps_match_oracle(pair):
    import torch
    name, s, ctx = pair
    xy = ctx.surface_xy()
    eta0, phis0 = _state(xy)
    dt = 0.05
    eta, phis = dev(eta0), dev(phis0)
    phi = torch.zeros(s.num.n_dof, dtype=torch.float64, device="cuda")
    oe, op = eta0.copy(), phis0.copy()
    for step in range(3):
        rc, st = ctx.fnpf_erk4(eta, phis, phi, dt, g=G, warm=step > 0, rtol=1e-12, imax=400)
        assert rc == 0 and st["status"] == 0 and max(st["rel_res"]) <= 1e-12
        oe, op = s.erk4(oe, op, dt, G)
    assert rel_err(host(eta), oe) < 1e-8 and rel_err(host(phis), op) < 1e-8


def test_warm_stages_need_fewer_iterations():
    """Stage solves after the first start from the previous stage's solution,
    and need fewer iterations than a stage solved from zero; so does the next
    step's first stage when warm."""
    import torch
    mk, P = MESHES["box_P4"]
    ctx = _ctx(mk(), P)
    eta0, phis0 = _state(ctx.surface_xy())
    eta, phis = dev(eta0), dev(phis0)
    phi = torch.zeros(ctx.levels[0]["n_dof"], dtype=torch.float64, device="cuda")
    rc, s1 = ctx.fnpf_erk4(eta, phis, phi, 0.05, g=G, warm=False, rtol=1e-8)
    rc, s2 = ctx.fnpf_erk4(eta, phis, phi, 0.05, g=G, warm=True, rtol=1e-8)
    assert max(s1["iters"][1:]) < s1["iters"][0], s1["iters"]
    assert s2["iters"][0] < s1["iters"][0], (s1["iters"], s2["iters"])
    ctx.close()


def test_errors_leave_the_state_unchanged():
    import torch
    from paper_2009_00705_amd import pmg
    mk, P = MESHES["box_P4"]
    ctx = _ctx(mk(), P)
    n2 = ctx.levels[0]["n_surface"]
    eta = torch.full((n2,), -2.0, dtype=torch.float64, device="cuda")   # below the bottom: inverted prisms
    phis = torch.zeros(n2, dtype=torch.float64, device="cuda")
    phi = torch.zeros(ctx.levels[0]["n_dof"], dtype=torch.float64, device="cuda")
    with pytest.raises(pmg.PmgError) as e:
        ctx.fnpf_erk4(eta, phis, phi, 0.05)
    assert e.value.code == -6
    assert torch.all(eta == -2.0) and torch.all(phis == 0.0)
    with pytest.raises(pmg.PmgError) as e:
        ctx.fnpf_erk4(torch.zeros_like(eta), phis, phi, 0.0)
    assert e.value.code == -1
    ctx.close()


def test_small_amplitude_standing_wave_follows_linear_theory():
    """eps = 1e-5 standing wave, k = 1, h = 1: after 0.2 periods (8 steps)
    eta and phi~ match eps cos(kx) cos(wt) and -(g eps / w) cos(kx) sin(wt)."""
    import torch
    mesh = W.box_mesh(4, 2)
    ctx = _ctx(mesh, 6)
    x = ctx.surface_xy()[:, 0]
    eps, k, h = 1e-5, 1.0, 1.0
    om = math.sqrt(G * k * math.tanh(k * h))
    t_end = 0.2 * 2 * math.pi / om
    eta, phis = dev(eps * np.cos(k * x)), dev(np.zeros_like(x))
    phi = torch.zeros(ctx.levels[0]["n_dof"], dtype=torch.float64, device="cuda")
    for step in range(8):
        ctx.fnpf_erk4(eta, phis, phi, t_end / 8, g=G, warm=step > 0, rtol=1e-12)
    e_ex = eps * np.cos(k * x) * math.cos(om * t_end)
    p_ex = -G * eps / om * np.cos(k * x) * math.sin(om * t_end)
    assert np.abs(host(eta) - e_ex).max() < 1e-4 * eps
    assert np.abs(host(phis) - p_ex).max() < 1e-4 * G * eps / om
    ctx.close()
