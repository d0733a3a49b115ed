"""Host-side checks of libpmg.so (no GPU): exports, numbering and colouring.

The gather maps and colours of the library are a bit-exact contract with the
oracle's numbering; node coordinates agree to rounding.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mesh as M
from paper_2009_00705_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pmg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2009_00705_amd import pmg
    L = pmg.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in pmg.SIGNATURES, f"binding lacks {n}"
    assert L.pmg_abi_version() == 7
    # the binding's struct ends where the header's does: the last fields' defaults
    o = pmg.default_options()
    assert (o.dss, o.nu1_coarse, o.nu2_coarse) == (0, -1, -1)
    assert pmg.default_options(nu1_coarse=2).nu1_coarse == 2


def _host_ctx(mesh, P, **kw):
    from paper_2009_00705_amd import pmg
    return pmg.Context(mesh, P=P, host_only=1, **kw)


MESHES = {
    "box": lambda: W.box_mesh(3, 2),
    "cyl": lambda: W.cylinder_mesh(spacing=0.45, half=2.0, radius=0.5, n_layers=3),
}


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P", [1, 2, 3, 4, 6, 8])
def test_gather_maps_bit_exact(meshname, P):
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P)
    orders = [P]
    while orders[-1] > 1:
        orders.append(max(1, orders[-1] // 2))
    assert ctx.n_levels == len(orders)
    for lvl, p in enumerate(orders):
        num = M.Numbering(m, p)
        info = ctx.levels[lvl]
        assert info["order"] == p and info["n_dof"] == num.n_dof and info["n_elem"] == num.n_elem
        assert info["n_surface"] == num.n2d
        np.testing.assert_array_equal(ctx.gather_map(lvl), num.map.astype(np.int32))
    ctx.close()


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P", [1, 3])
def test_colours_bit_exact(meshname, P):
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P)
    np.testing.assert_array_equal(ctx.colours(0), M.Numbering(m, P).colours().astype(np.int32))


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P", [1, 3, 6])
def test_dss_colours_bit_exact(meshname, P):
    """Triangle colours of the coloured direct-stiffness sum: greedy over
    ascending triangles, each taking the smallest colour of no lower triangle
    that shares a 2D node with it (brute force over the 2D gather map), so no
    two triangles of a colour share a node; the same on every level."""
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P)
    for lvl in range(ctx.n_levels):
        p = ctx.levels[lvl]["order"]
        m2 = M.Numbering(m, p).map2d
        nt = m2.shape[0]
        node_tris = {}
        for t in range(nt):
            for g in set(m2[t].tolist()):
                node_tris.setdefault(g, []).append(t)
        want = -np.ones(nt, dtype=np.int32)
        for t in range(nt):
            used = {int(want[u]) for g in set(m2[t].tolist()) for u in node_tris[g] if u < t}
            c = 0
            while c in used:
                c += 1
            want[t] = c
        got = ctx.dss_colours(lvl)
        np.testing.assert_array_equal(got, want, err_msg=f"level {lvl}")
        for g, ts in node_tris.items():
            assert len({int(got[t]) for t in ts}) == len(ts), (lvl, g)
    ctx.close()


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P", [2, 3, 5, 6, 8])
def test_in_plane_first_levels_bit_exact(meshname, P):
    """Levels of the in-plane-first sequence (triangle order coarsened first,
    then the vertical order): orders, sizes and gather maps equal the oracle's
    numbering of the same (triangle, vertical) orders."""
    from oracle.mg import level_orders
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P, coarsening="xy")
    orders = level_orders(P, "xy")
    assert ctx.n_levels == len(orders)
    for lvl, (pt, pz) in enumerate(orders):
        num = M.Numbering(m, pt, pz)
        info = ctx.levels[lvl]
        assert (info["order"], info["order_z"]) == (pt, pz)
        assert info["n_dof"] == num.n_dof and info["np"] == num.np and info["n_surface"] == num.n2d
        np.testing.assert_array_equal(ctx.gather_map(lvl), num.map.astype(np.int32))
    ctx.close()


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P,PZ,coarsening", [(5, 3, "equal"), (4, 2, "equal"), (6, 4, "equal"), (3, 6, "equal"),
                                             (2, 4, "equal"), (4, 8, "equal"), (6, 6, "equal"), (3, 6, "xy"),
                                             (4, 4, "both")])
def test_anisotropic_finest_levels_bit_exact(meshname, P, PZ, coarsening):
    """Finest vertical order PZ (pmg_options.PZ) with the equal-order sequence
    (Sec. 6.2, Table BTcoarse3D) or the others: orders, sizes and gather maps of
    every level equal the oracle's numbering of the same orders."""
    from oracle.mg import level_orders
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P, PZ=PZ, coarsening=coarsening)
    orders = [o if isinstance(o, tuple) else (o, o) for o in level_orders(P, coarsening, PZ)]
    assert ctx.n_levels == len(orders)
    for lvl, (pt, pz) in enumerate(orders):
        num = M.Numbering(m, pt, pz)
        info = ctx.levels[lvl]
        assert (info["order"], info["order_z"]) == (pt, pz)
        assert info["n_dof"] == num.n_dof and info["np"] == num.np and info["n_surface"] == num.n2d
        np.testing.assert_array_equal(ctx.gather_map(lvl), num.map.astype(np.int32))
    ctx.close()


def test_unbuilt_order_sequences_are_rejected():
    from paper_2009_00705_amd import pmg
    m = W.box_mesh(2, 1)
    for kw in (dict(P=5, PZ=3, coarsening="xy"), dict(P=7, PZ=2, coarsening="equal"), dict(P=3, PZ=9)):
        with pytest.raises(pmg.PmgError) as e:
            pmg.Context(m, host_only=1, **kw)
        assert e.value.code == -1, kw


@pytest.mark.parametrize("meshname", sorted(MESHES))
@pytest.mark.parametrize("P,coarsening,overlap,tags,top_neumann", [
    (3, "both", 1, 0, 0), (4, "xy", 1, 0b10, 0), (3, "both", 0, 0b10, 1), (4, "both", -1, 0, 0),
    (3, "xy", 2, 0, 1), (2, "xy", -1, 0b110, 0)])
def test_schwarz_subdomains_bit_exact(meshname, P, coarsening, overlap, tags, top_neumann):
    """Subdomains of the Schwarz smoother (library: distance to the shared
    entity of touching prisms; oracle: brute force over shared nodes) are the
    same node lists on every non-coarsest level, and the query reports them."""
    from oracle.mg import level_orders
    from oracle.refelem import order_pair
    from oracle.schwarz import overlap_of, subdomains
    m = MESHES[meshname]()
    ctx = _host_ctx(m, P, coarsening=coarsening, smoother="schwarz", overlap=overlap, dirichlet_tags=tags,
                    top_neumann=top_neumann)
    orders = level_orders(P, coarsening)
    for lvl, p in enumerate(orders[:-1]):
        pt, pz = order_pair(p)
        num = M.Numbering(m, pt, pz)
        free = np.ones(num.n_dof, dtype=bool)
        if not top_neumann:
            free[num.surface_nodes] = False
        if tags:
            for g2 in M.lateral_dirichlet_2d(m, num, tags):
                free[g2 * num.nz:(g2 + 1) * num.nz] = False
        dt, dz = overlap_of((pt, pz), overlap)
        want = subdomains(num, free, dt, dz)
        got = ctx.schwarz_nodes(lvl)
        info = ctx.schwarz_info(lvl)
        assert (info["dt"], info["dz"]) == (dt, dz) and info["n_sub"] == num.n_elem
        assert info["max_size"] == max(w.size for w in want)
        assert info["total"] == sum(w.size for w in want)
        nt = [(w.size + 31) // 32 for w in want]
        assert info["inv_entries"] == sum(t * (t + 1) // 2 * 1024 for t in nt)
        assert len(got) == len(want)
        for e in range(num.n_elem):
            np.testing.assert_array_equal(got[e], want[e].astype(np.int32), err_msg=f"level {lvl} element {e}")
    with pytest.raises(Exception):
        ctx.schwarz_info(len(orders) - 1)
    ctx.close()


@pytest.mark.parametrize("meshname", sorted(MESHES))
def test_surface_xy_and_node_xyz(meshname):
    m = MESHES[meshname]()
    P = 4
    ctx = _host_ctx(m, P)
    num = M.Numbering(m, P)
    np.testing.assert_allclose(ctx.surface_xy(), M.unique_xy_2d(m, num), atol=1e-14)
    np.testing.assert_allclose(ctx.node_xyz(0), M.node_xyz(m, num, np.zeros(num.n2d)), atol=1e-14)


def test_dirichlet_mask_and_free_counts():
    m = W.box_mesh(3, 2)
    ctx = _host_ctx(m, 3, dirichlet_tags=0b00110)
    num = M.Numbering(m, 3)
    lat = M.lateral_dirichlet_2d(m, num, 0b00110)
    want = np.zeros(num.n_dof, np.uint8)
    want[num.surface_nodes] = 1
    for g2 in lat:
        want[g2 * num.nz:(g2 + 1) * num.nz] = 1
    np.testing.assert_array_equal(ctx.dirichlet_mask(0), want)
    assert ctx.levels[0]["n_free"] == int((want == 0).sum())


def test_create_rejects_bad_input():
    from paper_2009_00705_amd import pmg
    m = W.box_mesh(2, 1)
    with pytest.raises(pmg.PmgError) as e:
        pmg.Context(m, P=9, host_only=1)
    assert e.value.code == -1
    big = dict(m)
    big["n_layers"] = (1 << 31) // len(m["tri"]) + 1   # 2^31 or more prisms
    with pytest.raises(pmg.PmgError) as e:
        pmg.Context(big, P=2, host_only=1)
    assert e.value.code == -1
    bad = dict(m)
    bad["tri"] = m["tri"][:, [0, 2, 1]]       # clockwise triangles
    with pytest.raises(pmg.PmgError) as e:
        pmg.Context(bad, P=2, host_only=1)
    assert e.value.code == -6
    ctx = pmg.Context(m, P=2, host_only=1)
    import torch
    with pytest.raises(pmg.PmgError) as e:   # device call on a host-only context
        ctx._c(pmg.lib().pmg_set_surface(ctx.h, ctypes.c_void_p(1), None))
    assert e.value.code == -7


def test_frozen_cylinder_mesh():
    """The unstructured workloads read the cylinder mesh from the committed
    fixture: 12015 counter-clockwise triangles in [-4, 4]^2, none inside the
    cylinder of radius 0.5, curved edges with both ends on that circle, and
    every boundary edge tagged; the library numbers it like the oracle."""
    m = W.config_mesh("c4")
    xy, tri = m["xy"], m["tri"]
    assert tri.shape == (12015, 3) and m["n_layers"] == 4 and m["depth"] == 1.0
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    assert area2.min() > 0
    cen = (p0 + p1 + p2) / 3
    assert np.hypot(cen[:, 0], cen[:, 1]).min() > 0.5 and np.abs(xy).max() <= 4.0 + 1e-12
    ends = xy[m["curved_edge"].ravel()]
    assert len(ends) > 0 and np.abs(np.hypot(ends[:, 0], ends[:, 1]) - 0.5).max() < 1e-12
    # boundary edges (held by one triangle) carry a tag, interior edges none
    from collections import Counter
    cnt = Counter(tuple(sorted((int(t[i]), int(t[(i + 1) % 3])))) for t in tri for i in range(3))
    for t, tags in zip(tri, m["edge_tag"]):
        for i in range(3):
            e = tuple(sorted((int(t[i]), int(t[(i + 1) % 3]))))
            assert (tags[i] != 0) == (cnt[e] == 1)
    ctx = _host_ctx(m, 1)
    np.testing.assert_array_equal(ctx.gather_map(0), M.Numbering(m, 1).map.astype(np.int32))
    ctx.close()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus above 1 ends with exit code 2 and a
    JSON line that says so, before anything touches a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2, r.stderr[-2000:]
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises; there is no fallback path."""
    from paper_2009_00705_amd import pmg
    monkeypatch.setattr(pmg, "_lib", None)
    monkeypatch.setattr(pmg, "LIB_PATH", str(tmp_path / "libpmg.so"))
    with pytest.raises(ImportError, match="not built"):
        pmg.lib()
    with pytest.raises(ImportError):
        pmg.Context(W.box_mesh(2, 1), P=2, host_only=1)
