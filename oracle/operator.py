"""Isoparametric geometry and the SEM stiffness operator (FP64).

eq. laplaceproblemdiscrete: L_ij = -sum_k int K grad N_j . grad N_i; we solve
with A = -L (the SPD stiffness, Sec. 3.1's SPD remark).  For the non-sigma
form (Sec. 3.1, used for wave-body problems) K is the identity in physical
coordinates, so on element e

    A_e[i, j] = sum_q w_q detJ_q grad N_i(x_q) . grad N_j(x_q),

with physical gradients obtained from reference ones through K = J^-1.  The
geometry is the fine (order P) isoparametric map x(r, s, t) = sum_n x_n N_n,
evaluated at the level's own cubature points on every level.
"""
from __future__ import annotations

import numpy as np

from .mesh import Numbering, node_xy_2d
from .refelem import order_pair, ref


def element_node_xyz(mesh: dict, num_f: Numbering, eta2d: np.ndarray, elements=None) -> np.ndarray:
    """Nodal xyz of every prism (or of the listed prisms, in that order) at the
    fine order, shape (E, Np, 3)."""
    P, L = num_f.P, num_f.L
    re = ref(P)
    h = float(mesh["depth"])
    X2 = node_xy_2d(mesh, num_f)                            # (nt, Np_tri, 2)
    eta_t = np.asarray(eta2d, dtype=np.float64)[num_f.map2d]  # (nt, Np_tri)
    els = np.arange(num_f.n_elem) if elements is None else np.asarray(elements)
    out = np.empty((els.size, re.np, 3))
    for i, e in enumerate(els):
        t, layer = divmod(int(e), L)
        for c in range(P + 1):
            sig = (layer + (1 + re.t[c]) / 2) / L
            sl = slice(c * re.np_tri, (c + 1) * re.np_tri)
            out[i, sl, 0] = X2[t, :, 0]
            out[i, sl, 1] = X2[t, :, 1]
            out[i, sl, 2] = -h + sig * (eta_t[t] + h)
    return out


class LevelGeometry:
    """Geometric factors of one level: G[e, ab, q] = w_q detJ_q (K K^T)_ab.

    ab runs over (rr, rs, rt, ss, st, tt).  ``detJ`` and ``K`` are kept for
    tests (volume, physical gradients).
    """

    def __init__(self, Pl, Pf: int, xyz_f: np.ndarray):
        rl = ref(*order_pair(Pl))
        rf = ref(Pf)
        # fine-order map, differentiated at this level's cubature points
        _, Dr, Ds, Dt = rf.prism_mats(rl.cr, rl.cs, rl.zq)
        J = np.empty((xyz_f.shape[0], rl.nq, 3, 3))  # J[e, q, c, a] = d x_c / d r_a
        for a, D in enumerate((Dr, Ds, Dt)):
            J[:, :, :, a] = np.einsum("qn,enc->eqc", D, xyz_f)
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ <= 0):
            raise ValueError("non-positive Jacobian")
        K = np.linalg.inv(J)                          # K[e, q, a, c] = d r_a / d x_c
        self.K = K
        KK = np.einsum("eqac,eqbc->eqab", K, K)
        wd = rl.w[None, :] * self.detJ
        idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        self.G = np.stack([wd * KK[:, :, a, b] for (a, b) in idx], axis=1)  # (E, 6, Nq)
        self.P = Pl
        self.wdet = wd

    def full(self) -> np.ndarray:
        """Symmetric 3x3 G per point: (E, Nq, 3, 3)."""
        G = self.G
        out = np.empty((G.shape[0], G.shape[2], 3, 3))
        idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        for m, (a, b) in enumerate(idx):
            out[:, :, a, b] = G[:, m]
            out[:, :, b, a] = G[:, m]
        return out


class StiffnessOperator:
    """Matrix-free y = A x on one level (all nodes; masking is the caller's)."""

    def __init__(self, num: Numbering, geo: LevelGeometry):
        self.num = num
        self.geo = geo
        rl = ref(num.P, getattr(num, "PZ", num.P))
        self.Dr = np.kron(rl.Bz, rl.Dr)
        self.Ds = np.kron(rl.Bz, rl.Ds)
        self.Dt = np.kron(rl.Dz, rl.B)
        self.Gf = geo.full()

    def element_apply(self, U: np.ndarray) -> np.ndarray:
        """Y_e = sum_ab D_a^T diag(G_ab) D_b U_e for all elements; U is (E, Np)."""
        D = (self.Dr, self.Ds, self.Dt)
        dU = [U @ Db.T for Db in D]                       # (E, Nq) each
        Y = np.zeros_like(U)
        for a in range(3):
            Va = sum(self.Gf[:, :, a, b] * dU[b] for b in range(3))
            Y += Va @ D[a]
        return Y

    def apply(self, x: np.ndarray) -> np.ndarray:
        m = self.num.map
        Y = self.element_apply(x[m])
        return np.bincount(m.ravel(), weights=Y.ravel(), minlength=self.num.n_dof)

    def element_matrices(self) -> np.ndarray:
        """Dense A_e (E, Np, Np): physical-gradient form sum_c Dphys_c^T W Dphys_c."""
        K = self.geo.K
        wd = self.geo.wdet
        D = np.stack([self.Dr, self.Ds, self.Dt], axis=0)   # (3, Nq, Np)
        # physical gradient matrices: Dp[e, c, q, n] = sum_a K[e,q,a,c] D[a,q,n]
        Dp = np.einsum("eqac,aqn->ecqn", K, D)
        # sum over (c, q) of Dp[e,c,q,i] wd[e,q] Dp[e,c,q,j], as one product per prism
        E, _, nq, n = Dp.shape
        Dpf = Dp.reshape(E, 3 * nq, n)
        return np.matmul(Dpf.transpose(0, 2, 1), Dpf * np.tile(wd, (1, 3))[:, :, None])

    def assembled(self):
        """Global sparse matrix Q^T blockdiag(A_e) Q (scipy CSR)."""
        import scipy.sparse as sp
        Ae = self.element_matrices()
        m = self.num.map
        E, n = m.shape
        rows = np.repeat(m, n, axis=1).ravel()
        cols = np.tile(m, (1, n)).ravel()
        A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(self.num.n_dof,) * 2)
        return A.tocsr()

    def diagonal(self) -> np.ndarray:
        """diag(A) = Q^T diag(A_e): sum over points of D_a[q,n] G_ab[q] D_b[q,n]."""
        D = (self.Dr, self.Ds, self.Dt)
        de = np.zeros((self.num.n_elem, self.num.np))
        for a in range(3):
            for b in range(3):
                de += (self.Gf[:, :, a, b]) @ (D[a] * D[b])
        m = self.num.map
        return np.bincount(m.ravel(), weights=de.ravel(), minlength=self.num.n_dof)
