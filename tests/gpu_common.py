"""Shared helpers of the GPU parity tests (oracle vs library on equal inputs)."""
from __future__ import annotations

import numpy as np

from oracle import mesh as M
from oracle.mg import Hierarchy
from paper_2009_00705_amd import workloads as W


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().double().cpu().numpy()


def surface_eta(xy, kind):
    if kind == "flat":
        return np.zeros(xy.shape[0])
    if kind == "wavy":
        return W.surface_elevation_c2(xy[:, 0], xy[:, 1])
    raise KeyError(kind)


def make_pair(mesh, P, eta_kind="wavy", omega=0.3, **kw):
    """(oracle Hierarchy, library Context) for the same mesh, order, surface and options."""
    import torch
    from paper_2009_00705_amd import pmg
    num = M.Numbering(mesh, P)
    eta_o = surface_eta(M.unique_xy_2d(mesh, num), eta_kind)
    okw = {}
    if "dirichlet_tags" in kw:
        okw["dirichlet_tags"] = kw["dirichlet_tags"]
    if kw.get("top_neumann"):
        okw["top_neumann"] = True
    if "smoother" in kw:
        okw["smoother"] = kw["smoother"]
        okw["smooth_ratio"] = kw.get("smooth_ratio", 15.0)
    if "coarsening" in kw:
        okw["coarsening"] = kw["coarsening"]
    if "PZ" in kw:
        okw["PZ"] = kw["PZ"]
    if "overlap" in kw:
        okw["overlap"] = kw["overlap"]
    for k in ("nu1_coarse", "nu2_coarse"):
        if k in kw:
            okw[k] = kw[k]
    if kw.get("coarse") == "chebyshev":
        okw["coarse"] = "chebyshev"
        okw["cheb"] = (kw["cheb_degree"], kw["cheb_lmin"], kw["cheb_lmax"])
    h = Hierarchy(mesh, P, eta2d=eta_o, nu1=kw.get("nu1", 2), nu2=kw.get("nu2", 2),
                  omega=None if omega in ("auto", "lib") else omega, **okw)
    lkw = dict(kw)
    if omega == "auto":
        # the oracle's automatic weights, passed to the library as explicit values
        lkw["omega"] = [lv.omega for lv in h.levels[:-1]]
    elif omega != "lib":
        lkw["omega"] = [omega] * 8
    ctx = pmg.Context(mesh, P=P, **lkw)
    eta_l = surface_eta(ctx.surface_xy(), eta_kind)
    ctx.set_surface(dev(eta_l))
    torch.cuda.synchronize()
    return h, ctx


def rel_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale
