"""Numbering of the nodal space V^p on an extruded prism mesh (FP64 / int64).

Sec. 3.1: the xy-plane is tessellated into triangles; the fluid volume is the
triangles extruded into prism layers; V^p is continuous with a cardinal nodal
basis, so nodes shared by elements carry one global unknown.

Global numbering (the bit-exact contract shared with the library):
* edges: every (min, max) vertex pair, sorted lexicographically -> edge id;
* 2D node id: vertex v -> v; edge-interior node m = 1..P-1 counted from the
  lower-id vertex -> nv + e (P-1) + m - 1; triangle-interior node of rank k in
  local order -> nv + ne (P-1) + t (P-1)(P-2)/2 + k;
* vertical level z = layer * P + c in [0, L P]; global node
  g = id2d * (L P + 1) + z (columns contiguous); element e = t L + layer;
* gather map M[e, c Np_tri + a] = g; surface nodes have z = L P.
Colouring: greedy over e ascending, smallest colour unused by any lower
element sharing a global node.
"""
from __future__ import annotations

import numpy as np

from .refelem import ref, tri_node_ijk


def edges_of(tri: np.ndarray):
    """Sorted unique (min, max) edges and, per triangle, the id of edge (v_i, v_{i+1})."""
    nt = tri.shape[0]
    e = np.stack([tri, np.roll(tri, -1, axis=1)], axis=2).reshape(-1, 2)
    key = np.sort(e, axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    return uniq, inv.reshape(nt, 3)


class Numbering:
    """Global numbering of order P (triangle) and PZ (vertical, default P) on
    the extruded mesh."""

    def __init__(self, mesh: dict, P: int, PZ: int = None):
        PZ = P if PZ is None else PZ
        self.P = P
        self.PZ = PZ
        re = ref(P, PZ)
        tri = np.asarray(mesh["tri"], dtype=np.int64)
        self.nv = int(np.asarray(mesh["xy"]).shape[0])
        self.nt = tri.shape[0]
        self.L = int(mesh["n_layers"])
        edges, tedge = edges_of(tri)
        self.edges = edges
        self.ne = edges.shape[0]
        self.nint = (P - 1) * (P - 2) // 2 if P >= 3 else 0
        self.n2d = self.nv + self.ne * max(P - 1, 0) + self.nt * self.nint
        self.nz = self.L * PZ + 1
        self.n_dof = self.n2d * self.nz
        self.np_tri = re.np_tri
        self.np = re.np
        ijk = tri_node_ijk(P)
        # local triangle node -> 2D global id, per triangle
        m2 = np.empty((self.nt, self.np_tri), dtype=np.int64)
        for a, (i, j, k) in enumerate(ijk):
            if (i, j) == (0, 0):
                m2[:, a] = tri[:, 0]
            elif (i, j) == (P, 0):
                m2[:, a] = tri[:, 1]
            elif (i, j) == (0, P):
                m2[:, a] = tri[:, 2]
            elif j == 0:          # edge v0 -> v1, position i from v0
                m2[:, a] = self._edge_node(tri[:, 0], tri[:, 1], tedge[:, 0], i)
            elif k == 0:          # edge v1 -> v2, position j from v1
                m2[:, a] = self._edge_node(tri[:, 1], tri[:, 2], tedge[:, 1], j)
            elif i == 0:          # edge v2 -> v0, position P - j from v2
                m2[:, a] = self._edge_node(tri[:, 2], tri[:, 0], tedge[:, 2], P - j)
        rank = 0
        for a, (i, j, k) in enumerate(ijk):
            if i >= 1 and j >= 1 and k >= 1:
                m2[:, a] = self.nv + self.ne * (P - 1) + np.arange(self.nt) * self.nint + rank
                rank += 1
        self.map2d = m2
        # 3D gather map
        E = self.nt * self.L
        self.n_elem = E
        layer = np.tile(np.arange(self.L), self.nt)
        t_of_e = np.repeat(np.arange(self.nt), self.L)
        c = np.repeat(np.arange(PZ + 1), self.np_tri)       # local node n -> c
        a = np.tile(np.arange(self.np_tri), PZ + 1)         # local node n -> a
        z = layer[:, None] * PZ + c[None, :]
        self.map = m2[t_of_e][:, a] * self.nz + z
        self.surface_nodes = np.arange(self.n2d) * self.nz + self.L * PZ
        self.mult = np.bincount(self.map.ravel(), minlength=self.n_dof).astype(np.float64)

    def _edge_node(self, va, vb, eid, m):
        P = self.P
        mg = np.where(va < vb, m, P - m)
        return self.nv + eid * (P - 1) + mg - 1

    def colours(self) -> np.ndarray:
        """Greedy element colouring: no two elements of a colour share a node."""
        E = self.n_elem
        node_elems = [[] for _ in range(self.n_dof)]
        for e in range(E):
            for g in np.unique(self.map[e]):
                node_elems[g].append(e)
        col = -np.ones(E, dtype=np.int64)
        for e in range(E):
            used = set()
            for g in np.unique(self.map[e]):
                for f in node_elems[g]:
                    if f < e:
                        used.add(int(col[f]))
            c = 0
            while c in used:
                c += 1
            col[e] = c
        return col


def lateral_dirichlet_2d(mesh: dict, num: Numbering, tag_mask: int) -> np.ndarray:
    """2D node ids lying on edges whose tag bit is set in ``tag_mask``."""
    P = num.P
    tri = np.asarray(mesh["tri"])
    tags = np.asarray(mesh["edge_tag"])
    ijk = tri_node_ijk(P)
    out = set()
    for t in range(num.nt):
        for le in range(3):
            tg = int(tags[t, le])
            if tg == 0 or not (tag_mask >> tg) & 1:
                continue
            for a, (i, j, k) in enumerate(ijk):
                on = (le == 0 and j == 0) or (le == 1 and k == 0) or (le == 2 and i == 0)
                if on:
                    out.add(int(num.map2d[t, a]))
    return np.array(sorted(out), dtype=np.int64)


def node_xy_2d(mesh: dict, num: Numbering) -> np.ndarray:
    """Per-triangle xy of the P-th order triangle nodes, shape (nt, Np_tri, 2).

    Straight triangles use the affine vertex map.  A triangle with an edge
    listed in ``curved_edge`` has that edge's nodes moved onto the circle
    (linear in angle along the short arc) and every node displaced by the
    edge displacement blended with (lambda_A + lambda_B):
    x = x_lin + (lA + lB) (X_arc(s) - X_chord(s)), s = lB / (lA + lB).
    """
    P = num.P
    re = ref(P)
    xy = np.asarray(mesh["xy"], dtype=np.float64)
    tri = np.asarray(mesh["tri"], dtype=np.int64)
    l1 = (1 + re.r) / 2
    l2 = (1 + re.s) / 2
    l0 = -(re.r + re.s) / 2
    lam = np.stack([l0, l1, l2], axis=1)          # (Np_tri, 3)
    X = np.einsum("av,tvd->tad", lam, xy[tri])     # (nt, Np_tri, 2)
    curved = {}
    ce = np.asarray(mesh.get("curved_edge", np.zeros((0, 2))), dtype=np.int64)
    circ = np.asarray(mesh.get("circle", np.zeros((0, 3))), dtype=np.float64)
    for k in range(ce.shape[0]):
        curved[(min(ce[k]), max(ce[k]))] = circ[k]
    if not curved:
        return X
    for t in range(tri.shape[0]):
        for le in range(3):
            va, vb = int(tri[t, le]), int(tri[t, (le + 1) % 3])
            key = (min(va, vb), max(va, vb))
            if key not in curved:
                continue
            cx, cy, R = curved[key]
            A, Bv = xy[va], xy[vb]
            thA = np.arctan2(A[1] - cy, A[0] - cx)
            thB = np.arctan2(Bv[1] - cy, Bv[0] - cx)
            dth = thB - thA
            dth = (dth + np.pi) % (2 * np.pi) - np.pi
            lA = lam[:, le]
            lB = lam[:, (le + 1) % 3]
            ssum = lA + lB
            for a in range(re.np_tri):
                if ssum[a] < 1e-14:
                    continue
                sp = lB[a] / ssum[a]
                arc = np.array([cx + R * np.cos(thA + sp * dth), cy + R * np.sin(thA + sp * dth)])
                chord = (1 - sp) * A + sp * Bv
                X[t, a] += ssum[a] * (arc - chord)
    return X


def unique_xy_2d(mesh: dict, num: Numbering) -> np.ndarray:
    """xy of every 2D global node (n2d, 2)."""
    X = node_xy_2d(mesh, num)
    out = np.zeros((num.n2d, 2))
    out[num.map2d.ravel()] = X.reshape(-1, 2)
    return out


def node_xyz(mesh: dict, num: Numbering, eta2d: np.ndarray) -> np.ndarray:
    """xyz of every global node: z = -h + sigma (eta + h), sigma of level layer PZ + c in LGL spacing."""
    PZ, L = num.PZ, num.L
    re = ref(num.P, PZ)
    h = float(mesh["depth"])
    xy = unique_xy_2d(mesh, num)
    # sigma of vertical level zl = layer PZ + c
    sig = np.empty(num.nz)
    for layer in range(L):
        for c in range(PZ + 1):
            sig[layer * PZ + c] = (layer + (1 + re.t[c]) / 2) / L
    out = np.empty((num.n_dof, 3))
    g2 = np.repeat(np.arange(num.n2d), num.nz)
    zl = np.tile(np.arange(num.nz), num.n2d)
    out[:, 0] = xy[g2, 0]
    out[:, 1] = xy[g2, 1]
    out[:, 2] = -h + sig[zl] * (np.asarray(eta2d)[g2] + h)
    return out
