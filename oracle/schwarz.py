"""Overlapping additive Schwarz smoother (Sec. 5.2, eq. sec_form, eq. Mass,
eq. weights), FP64, test infrastructure.

S^-1 = W sum_k R_k^T (R_k A R_k^T)^-1 R_k,   W = (sum_k R_k R_k^T)^-1.

Subdomain k is element k's nodes plus an overlap zone in the elements that
touch it (share at least one node with it).  Overlap reading (Sec. 5.2 and
Sec. 6.3): a node x of a touching element e is in the zone when some node y
that e shares with k lies within ``dt`` lattice steps of x in the triangle
(the hexagonal distance of the barycentric indices, max |d lambda_i|) and
within ``dz`` steps along the extrusion.  dt = dz = 1 is the paper's "one
overlapping node in each spatial direction"; dt = dz = 0 is block Jacobi; the
"refined" variant takes ceil((P + 1)/2) per direction with P that direction's
order on the level.  Dirichlet nodes are left out of every subdomain (their
correction is zero), so R_k A R_k^T is a principal submatrix of A_FF.

The distance test is a brute force over the shared nodes of every touching
element; local inverses come from numpy.  Post-smoothing uses the transpose
sum_k R_k^T A_k^-1 R_k W, so the V-cycle stays symmetric for PCG.
"""
from __future__ import annotations

import math

import numpy as np

from .refelem import tri_node_ijk


def overlap_of(order, overlap):
    """(dt, dz) for a level of (triangle, vertical) order; overlap < 0 is refined."""
    pt, pz = order
    if overlap < 0:
        return math.ceil((pt + 1) / 2), math.ceil((pz + 1) / 2)
    return int(overlap), int(overlap)


def _within(num, dt, dz):
    """C[x, y]: local prism node x lies within (dt, dz) lattice steps of y."""
    ijk = np.asarray(tri_node_ijk(num.P))
    dtri = np.abs(ijk[:, None, :] - ijk[None, :, :]).max(axis=2)        # hexagonal distance
    c = np.arange(num.PZ + 1)
    dver = np.abs(c[:, None] - c[None, :])
    a = np.tile(np.arange(num.np_tri), num.PZ + 1)
    cc = np.repeat(c, num.np_tri)
    return (dtri[a][:, a] <= dt) & (dver[cc][:, cc] <= dz)


def subdomains(num, free, dt, dz):
    """Sorted free global nodes of every subdomain (list over elements)."""
    m = num.map
    node_elems = {}
    for e in range(num.n_elem):
        for g in m[e]:
            node_elems.setdefault(int(g), set()).add(e)
    C = _within(num, dt, dz)
    out = []
    for k in range(num.n_elem):
        own = set(int(g) for g in m[k])
        touching = set()
        for g in own:
            touching |= node_elems[g]
        nodes = set(own)
        for e in touching:
            shared = np.array([int(g) in own for g in m[e]])
            keep = C[:, shared].any(axis=1)
            nodes.update(int(g) for g in m[e][keep])
        idx = np.array(sorted(nodes), dtype=np.int64)
        out.append(idx[free[idx]])
    return out


class Schwarz:
    """Local inverses and weights of one level (``level`` has num, op, free)."""

    def __init__(self, level, dt, dz):
        self.dt, self.dz = dt, dz
        self.sub = subdomains(level.num, level.free, dt, dz)
        A = level.op.assembled().tocsr()
        self.inv = [np.linalg.inv(A[s][:, s].toarray()) if s.size else np.zeros((0, 0)) for s in self.sub]
        count = np.zeros(level.num.n_dof)
        for s in self.sub:
            count[s] += 1.0
        self.count = count
        self.w = np.where(count > 0, 1.0 / np.where(count > 0, count, 1.0), 0.0)

    def apply(self, r, transpose=False):
        """W sum_k R_k^T A_k^-1 R_k r, or its transpose sum_k R_k^T A_k^-1 R_k W r."""
        x = self.w * r if transpose else r
        z = np.zeros_like(r)
        for s, inv in zip(self.sub, self.inv):
            z[s] += inv @ x[s]
        return z if transpose else self.w * z
