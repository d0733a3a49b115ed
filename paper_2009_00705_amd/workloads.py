"""Seeded synthetic inputs: meshes, exact potentials and wave histories.

This module only produces *inputs* (vertex coordinates, triangles, boundary
tags, closed-form fields evaluated at caller-supplied points).  It holds none
of the discretisation's arithmetic: node placement, numbering, geometry,
operators and solvers live in the library (and, independently, in the CPU
oracle used by the tests).

The paper's own workloads (the submerged-bar bathymetry, the FPSO hull and the
measured gauge series of Sec. 6) are not available; these generators stand in
for them with the same structure: unstructured triangle meshes of the
xy-plane extruded into prism layers (Sec. 3.1 and Sec. 6.2), flat bottom,
free-surface Dirichlet data and no-flux walls (eq. laplaceproblem).

Random draws use ``numpy.random.default_rng(20090705 + config_no)``.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 20090705
GRAVITY = 9.81  # Sec. 2: g = 9.81 m/s^2

# Boundary tags of lateral edges (0 = interior edge).
TAG_XMIN, TAG_XMAX, TAG_YMIN, TAG_YMAX, TAG_CYL = 1, 2, 3, 4, 5


def rng_for(config_no: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(config_no))


def _boundary_edge_tags(xy, tri, box, circle=None, tol=1e-9):
    """Tag each triangle edge (tri[i], tri[(i+1)%3]) that lies on the boundary."""
    x0, x1, y0, y1 = box
    nt = tri.shape[0]
    tags = np.zeros((nt, 3), dtype=np.int32)
    # count edge occurrences to find boundary edges
    e = np.stack([tri, np.roll(tri, -1, axis=1)], axis=2).reshape(-1, 2)
    key = np.sort(e, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    on_bnd = (cnt[inv.ravel()] == 1).reshape(nt, 3)
    for t in range(nt):
        for i in range(3):
            if not on_bnd[t, i]:
                continue
            a, b = tri[t, i], tri[t, (i + 1) % 3]
            pa, pb = xy[a], xy[b]
            if abs(pa[0] - x0) < tol and abs(pb[0] - x0) < tol:
                tags[t, i] = TAG_XMIN
            elif abs(pa[0] - x1) < tol and abs(pb[0] - x1) < tol:
                tags[t, i] = TAG_XMAX
            elif abs(pa[1] - y0) < tol and abs(pb[1] - y0) < tol:
                tags[t, i] = TAG_YMIN
            elif abs(pa[1] - y1) < tol and abs(pb[1] - y1) < tol:
                tags[t, i] = TAG_YMAX
            elif circle is not None:
                cx, cy, R = circle
                ra = math.hypot(pa[0] - cx, pa[1] - cy)
                rb = math.hypot(pb[0] - cx, pb[1] - cy)
                if abs(ra - R) < 1e-9 and abs(rb - R) < 1e-9:
                    tags[t, i] = TAG_CYL
                else:
                    raise ValueError("boundary edge not on any known boundary")
            else:
                raise ValueError("boundary edge not on the box")
    return tags


def box_mesh(nq: int, n_layers: int, lx: float = 2 * math.pi,
             ly: float = 2 * math.pi, depth: float = 1.0) -> dict:
    """Split-quad box [0,lx]x[0,ly] with nq x nq quads, each cut along (v00,v11).

    Quads are taken row-major with i fastest; vertex (i, j) has id
    j*(nq+1)+i; the two counter-clockwise triangles of quad (i, j) are
    (v00, v10, v11) and (v00, v11, v01).
    """
    n1 = nq + 1
    xs = np.linspace(0.0, lx, n1)
    ys = np.linspace(0.0, ly, n1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # X[j, i]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    tris = []
    for j in range(nq):
        for i in range(nq):
            v00 = j * n1 + i
            v10 = v00 + 1
            v01 = v00 + n1
            v11 = v01 + 1
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    tri = np.asarray(tris, dtype=np.int32)
    tags = _boundary_edge_tags(xy, tri, (0.0, lx, 0.0, ly))
    return dict(xy=xy, tri=tri, edge_tag=tags,
                curved_edge=np.zeros((0, 2), np.int32),
                circle=np.zeros((0, 3), np.float64),
                n_layers=int(n_layers), depth=float(depth))


def cylinder_mesh(spacing: float = 0.1026, half: float = 4.0, radius: float = 0.5,
                  jitter: float = 0.1, n_layers: int = 4, depth: float = 1.0,
                  seed_offset: int = 4) -> dict:
    """Seeded Delaunay mesh of [-half,half]^2 minus a cylinder of given radius.

    Interior points lie on a jittered square lattice (jitter uniform in
    [-jitter, jitter] * spacing per coordinate); the square boundary and the
    circle carry points at the same spacing.  Triangles whose centroid falls
    inside the cylinder are removed.  Cylinder edges are listed in
    ``curved_edge`` with the circle (cx, cy, R) so that the discretisation
    can place their nodes on the exact circle.
    """
    from scipy.spatial import Delaunay

    rng = rng_for(seed_offset)
    h = float(spacing)
    nside = int(round(2 * half / h))
    s = np.linspace(-half, half, nside + 1)
    bnd = []
    for v in s:
        bnd.append((v, -half))
        bnd.append((v, half))
    for v in s[1:-1]:
        bnd.append((-half, v))
        bnd.append((half, v))
    ncirc = int(round(2 * math.pi * radius / h))
    th = 2 * math.pi * np.arange(ncirc) / ncirc
    circ = np.stack([radius * np.cos(th), radius * np.sin(th)], axis=1)
    g = np.linspace(-half, half, nside + 1)[1:-1]
    X, Y = np.meshgrid(g, g, indexing="xy")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    pts = pts + rng.uniform(-jitter, jitter, size=pts.shape) * h
    r = np.hypot(pts[:, 0], pts[:, 1])
    keep = r > radius + 0.5 * h
    keep &= np.all(np.abs(pts) < half - 0.5 * h, axis=1)
    pts = pts[keep]
    allp = np.concatenate([np.asarray(bnd), circ, pts], axis=0)
    allp = np.unique(np.round(allp, 14), axis=0)
    dt = Delaunay(allp)
    tri = dt.simplices.astype(np.int64)
    cen = allp[tri].mean(axis=1)
    tri = tri[np.hypot(cen[:, 0], cen[:, 1]) > radius]
    # counter-clockwise orientation
    p0, p1, p2 = allp[tri[:, 0]], allp[tri[:, 1]], allp[tri[:, 2]]
    area2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    flip = area2 < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    area2 = np.abs(area2)
    if area2.min() < 1e-6 * h * h:
        raise ValueError("degenerate triangle in cylinder mesh")
    # drop unused vertices and renumber
    used = np.unique(tri)
    newid = -np.ones(allp.shape[0], dtype=np.int64)
    newid[used] = np.arange(used.size)
    xy = allp[used].astype(np.float64)
    tri = newid[tri].astype(np.int32)
    tags = _boundary_edge_tags(xy, tri, (-half, half, -half, half), (0.0, 0.0, radius))
    ce = []
    for t in range(tri.shape[0]):
        for i in range(3):
            if tags[t, i] == TAG_CYL:
                ce.append((tri[t, i], tri[t, (i + 1) % 3]))
    curved = np.asarray(ce, dtype=np.int32).reshape(-1, 2)
    circle = np.tile(np.array([[0.0, 0.0, radius]]), (curved.shape[0], 1))
    return dict(xy=xy, tri=tri, edge_tag=tags, curved_edge=curved, circle=circle,
                n_layers=int(n_layers), depth=float(depth))


# ---------------------------------------------------------------------------
# closed-form potentials (inputs: Dirichlet data and exact references)
# ---------------------------------------------------------------------------

def linear_wave(x, y, z, kx: float, ky: float = 0.0, depth: float = 1.0):
    """cosh(k(z+h))/cosh(kh) cos(kx x) cos(ky y), k = |(kx, ky)|: harmonic."""
    k = math.hypot(kx, ky)
    return np.cosh(k * (np.asarray(z) + depth)) / math.cosh(k * depth) * \
        np.cos(kx * np.asarray(x)) * np.cos(ky * np.asarray(y))


def mode_pairs(kmax: float = 4.0):
    """Non-negative integer (kx, ky) with 1 <= |k| <= kmax (16 pairs for 4)."""
    out = []
    for kx in range(int(kmax) + 1):
        for ky in range(int(kmax) + 1):
            k = math.hypot(kx, ky)
            if 1.0 <= k <= kmax + 1e-12:
                out.append((kx, ky))
    return out


def mode_amplitudes(config_no: int = 3, n: int = 16, hi: float = 0.05):
    return rng_for(config_no).uniform(0.0, hi, size=n)


def mode_sum(x, y, z, amps, pairs, depth: float = 1.0):
    out = np.zeros(np.broadcast(np.asarray(x), np.asarray(z)).shape)
    for a, (kx, ky) in zip(amps, pairs):
        out = out + a * linear_wave(x, y, z, kx, ky, depth)
    return out


def surface_elevation_c2(x, y):
    """Free-surface elevation 0.1 sin(x) cos(y) of the box workloads."""
    return 0.1 * np.sin(np.asarray(x)) * np.cos(np.asarray(y))


def uniform_flow_cylinder(x, y, z=None, radius: float = 0.5, speed: float = 1.0):
    """Potential of uniform flow past a circular cylinder: U x (1 + R^2/r^2)."""
    x = np.asarray(x)
    y = np.asarray(y)
    return speed * x * (1.0 + radius * radius / (x * x + y * y))


class WaveGroup:
    """Unidirectional linear focusing group of 16 components (steepness <= 0.1).

    Component m has wavenumber k_m = linspace(1, 4, 16)[m], frequency from
    the linear dispersion relation omega^2 = g k tanh(k h), amplitude drawn
    uniform in [0.5, 1.5] and scaled so that max(k) * sum(a) = steepness,
    and all phases align at x = 0 at the focus time t_f.
    """

    def __init__(self, config_no: int = 5, n: int = 16, depth: float = 1.0,
                 steepness: float = 0.1, n_steps: int = 300):
        rng = rng_for(config_no)
        self.depth = depth
        self.k = np.linspace(1.0, 4.0, n)
        self.omega = np.sqrt(GRAVITY * self.k * np.tanh(self.k * depth))
        a = rng.uniform(0.5, 1.5, size=n)
        self.a = a * steepness / (self.k.max() * a.sum())
        kp = 2.5
        self.Tp = 2 * math.pi / math.sqrt(GRAVITY * kp * math.tanh(kp * depth))
        self.dt = self.Tp / 16.0
        self.t_focus = 0.0
        self.n_steps = n_steps

    def time(self, n: int) -> float:
        return self.t_focus + (n - self.n_steps // 2) * self.dt

    def eta(self, x, n: int):
        t = self.time(n) - self.t_focus
        x = np.asarray(x)[..., None]
        return np.sum(self.a * np.cos(self.k * x - self.omega * t), axis=-1)

    def phi(self, x, z, n: int):
        """Linear-theory potential at (x, z)."""
        t = self.time(n) - self.t_focus
        x = np.asarray(x)[..., None]
        z = np.asarray(z)[..., None]
        c = GRAVITY / self.omega * np.cosh(self.k * (z + self.depth)) / np.cosh(self.k * self.depth)
        return np.sum(self.a * c * np.sin(self.k * x - self.omega * t), axis=-1)

    def surface(self, x, n: int):
        """(eta, phi_tilde) at surface points with abscissa x."""
        eta = self.eta(x, n)
        return eta, self.phi(x, eta, n)


# ---------------------------------------------------------------------------
# named configurations of the measured workloads
# ---------------------------------------------------------------------------

def config_mesh(name: str) -> dict:
    """Meshes of the five workloads (see the module docstring)."""
    if name == "c1":
        return box_mesh(4, 2)
    if name == "c2":
        return box_mesh(32, 4)
    if name == "c3":
        return box_mesh(128, 4)
    if name in ("c4", "c5"):
        return frozen_cylinder_mesh()
    raise KeyError(name)


def frozen_cylinder_mesh() -> dict:
    """The default cylinder_mesh() as written to fixtures/cyl_mesh.npz by
    fixtures/make_cyl_mesh.py (plain arrays, no pickles), so that the
    unstructured workloads keep one numbering whatever Delaunay implementation
    the running machine has."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixtures", "cyl_mesh.npz")
    with np.load(path, allow_pickle=False) as f:
        return dict(xy=f["xy"].astype(np.float64), tri=f["tri"].astype(np.int32),
                    edge_tag=f["edge_tag"].astype(np.int32), curved_edge=f["curved_edge"].astype(np.int32),
                    circle=f["circle"].astype(np.float64), n_layers=int(f["n_layers"]), depth=float(f["depth"]))


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded uniform(-1, 1) vector (parity inputs)."""
    return np.random.default_rng(SEED_BASE + 1000 + int(seed)).uniform(-1.0, 1.0, n).astype(dtype)
