"""Free-surface time stepping of the FNPF equations (FP64), test infrastructure.

eq. FSeta:  eta_t  = -grad eta . grad phi~ + w~ (1 + grad eta . grad eta)
eq. FSphi:  phi~_t = -g eta - 1/2 (grad phi~ . grad phi~ - w~^2 (1 + grad eta . grad eta))

closed by the Laplace problem (eq. laplaceproblem): phi = phi~ at z = eta,
zero flux at the bottom and walls; w~ is the vertical velocity d phi / dz at
the surface.  Time integration: the classical fourth-order explicit
Runge-Kutta method (ERK4, Sec. 6.1 and 6.2), one Laplace solve per stage.

Readings (the paper does not spell these out):
* grad of a surface field: the x and y derivatives of its order-P nodal
  interpolant on each triangle (isoparametric map of the fine order), taken at
  the nodes and averaged over the triangles sharing a node;
* w~ at a surface node: the derivative of phi along its column in the top
  prism, at the top node, divided by dz/dt = (eta + h) / (2L) (the sigma map
  z = -h + sigma (eta + h), sigma = (layer + (1 + t)/2) / L, leaves x and y
  independent of t, so the derivative along the column is d/dz at fixed x, y);
* the Laplace problem of each stage is solved exactly here (sparse LU); the
  library solves it iteratively to a given tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .mesh import Numbering, node_xy_2d
from .mg import Level
from .operator import element_node_xyz
from .refelem import ref


class Surface:
    """Surface operators of one mesh at order P (triangle and vertical)."""

    def __init__(self, mesh: dict, P: int):
        self.mesh = mesh
        self.P = P
        self.num = Numbering(mesh, P)
        self.h = float(mesh["depth"])
        re = ref(P)
        _, self.Dr, self.Ds = re.tri_eval(re.r, re.s)
        _, D1 = re.line_eval(re.t)
        self.d_top = D1[P]                               # d/dt at the top node t = +1
        X = node_xy_2d(mesh, self.num)                   # (nt, Np_tri, 2)
        xr, xs = X[:, :, 0] @ self.Dr.T, X[:, :, 0] @ self.Ds.T
        yr, ys = X[:, :, 1] @ self.Dr.T, X[:, :, 1] @ self.Ds.T
        det = xr * ys - xs * yr
        self.rx, self.ry = ys / det, -xs / det
        self.sx, self.sy = -yr / det, xr / det
        self.count = np.bincount(self.num.map2d.ravel(), minlength=self.num.n2d).astype(np.float64)

    def grad(self, f):
        """(f_x, f_y) at the surface nodes: element derivatives averaged over triangles."""
        m2 = self.num.map2d
        F = np.asarray(f)[m2]
        fr, fs = F @ self.Dr.T, F @ self.Ds.T
        fx = fr * self.rx + fs * self.sx
        fy = fr * self.ry + fs * self.sy
        n2 = self.num.n2d
        return (np.bincount(m2.ravel(), fx.ravel(), n2) / self.count,
                np.bincount(m2.ravel(), fy.ravel(), n2) / self.count)

    def w(self, phi, eta):
        """w~ = d phi / dz at the surface nodes (top prism of every column)."""
        n = self.num
        col = np.asarray(phi).reshape(n.n2d, n.nz)[:, (n.L - 1) * n.PZ:]
        return (col @ self.d_top) * (2.0 * n.L) / (np.asarray(eta) + self.h)

    def laplace(self, eta, phis):
        """phi with phi = phi~ at the surface nodes (exact solve on the fine level)."""
        n = self.num
        lv = Level(self.mesh, self.P, self.P, element_node_xyz(self.mesh, n, eta), None, False)
        A = lv.op.assembled().tocsr()
        free = np.flatnonzero(lv.free)
        phiD = np.zeros(n.n_dof)
        phiD[n.surface_nodes] = phis
        f = -(A @ phiD)
        phi = phiD.copy()
        phi[free] = spla.spsolve(A[free][:, free].tocsc(), f[free])
        return phi

    def rhs(self, eta, phis, g: float):
        """(eta_t, phi~_t, phi) of eq. FSeta and eq. FSphi at the state (eta, phi~)."""
        phi = self.laplace(eta, phis)
        w = self.w(phi, eta)
        ex, ey = self.grad(eta)
        px, py = self.grad(phis)
        s = 1.0 + ex * ex + ey * ey
        deta = -(ex * px + ey * py) + w * s
        dphis = -g * eta - 0.5 * ((px * px + py * py) - w * w * s)
        return deta, dphis, phi

    def erk4(self, eta, phis, dt: float, g: float):
        """One classical Runge-Kutta step of (eta, phi~)."""
        k1e, k1p, _ = self.rhs(eta, phis, g)
        k2e, k2p, _ = self.rhs(eta + 0.5 * dt * k1e, phis + 0.5 * dt * k1p, g)
        k3e, k3p, _ = self.rhs(eta + 0.5 * dt * k2e, phis + 0.5 * dt * k2p, g)
        k4e, k4p, _ = self.rhs(eta + dt * k3e, phis + dt * k3p, g)
        return (eta + dt / 6.0 * (k1e + 2 * k2e + 2 * k3e + k4e),
                phis + dt / 6.0 * (k1p + 2 * k2p + 2 * k3p + k4p))
