"""Geometric p-multigrid on one fixed prism mesh (FP64).

* Levels (Sec. 5, "N^p ~ 2 N^{p-1}"): orders P, floor(P/2), ..., 1, all on the
  same mesh and layer count; every level is rediscretised with the fine
  isoparametric map at its own cubature points.
* Prolongation (Sec. 5.1): the coarse space is nested in the fine one, so
  P_{p-1}^p interpolates: per element, the coarse nodal basis evaluated at
  the fine nodes (Pi = Pi_z (x) Pi_tri), then one value per shared fine node
  (the average over the elements holding it).  Restriction is its transpose
  (eq. rest).
* Smoother (eq. sec_form): damped Jacobi, S^-1 = omega D^-1, or a
  Chebyshev-accelerated Jacobi polynomial of the same degree as the sweep
  count on [lambda/ratio, lambda] with lambda = 4/(3 omega) (the power
  estimate of lambda_max(D^-1 A)); both are linear and symmetric.  Or the
  overlapping additive Schwarz smoother of eq. Mass (``oracle.schwarz``),
  its transpose in post-smoothing, damped by omega = 4/(3 rho) with rho the
  power estimate of the spectral radius of S^-1 A (the paper's undamped form
  is omega = 1; on tall prisms one undamped sweep makes the V-cycle
  indefinite).
* Coarsest level (P = 1): exact solve (dense Cholesky or sparse LU), or a
  fixed-degree Jacobi-preconditioned Chebyshev iteration on a given interval.
* V-cycle: Alg. 1 with zero initial guess below the top.
* Operator reuse across surfaces (Sec. 6, Fig. simstrats): "none" rebuilds
  every level from each new surface (strategy III); "t0" keeps the
  preconditioner and moves only the finest level's operator (strategy I);
  "lin" puts the coarse levels on the flat surface eta = 0 once and moves the
  finest level with its diagonal (strategy II).  Weights stay as they are.
Dirichlet nodes carry homogeneous corrections on every level.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .mesh import Numbering, lateral_dirichlet_2d
from .operator import LevelGeometry, StiffnessOperator, element_node_xyz
from .refelem import order_pair, ref, vandermonde_1d, vandermonde_tri
from .schwarz import Schwarz, overlap_of


def level_orders(P: int, coarsening: str = "both", PZ: int = None):
    """Orders of the levels, finest first, for the finest triangle order P and
    vertical order PZ (default P); a level is (triangle order, vertical order),
    or the plain int P for the isotropic all-direction sequence.

    "both": both orders halve together, max(1, floor(p/2)) (Sec. 5, Table
    BTcoarse: 6 -> 3 -> 1).  "xy": the triangle order is coarsened first with
    the vertical order kept, then the vertical order, (P, PZ) -> ... -> (1, PZ)
    -> (1, floor(PZ/2)) -> ... -> (1, 1) (in-plane semi-coarsening, for prisms
    whose in-plane node spacing is much finer than the vertical one).
    "equal": semi-coarsening of the direction of higher order until the two
    orders agree, each step to max(lower order, floor(higher/2)), then both
    together (Sec. 6.2 and Table BTcoarse3D: (5, 3) -> (3, 3) -> (1, 1); with
    PZ > P the vertical order is the one coarsened first)."""
    PZ = P if PZ is None else int(PZ)
    half = lambda p: max(1, p // 2)

    def seq(p):
        out = [p]
        while out[-1] > 1:
            out.append(half(out[-1]))
        return out
    if coarsening == "both":
        if PZ == P:
            return seq(P)
        out = [(P, PZ)]
        while out[-1] != (1, 1):
            out.append((half(out[-1][0]), half(out[-1][1])))
        return out
    if coarsening == "xy":
        return [(pt, PZ) for pt in seq(P)] + [(1, pz) for pz in seq(PZ)[1:]]
    if coarsening == "equal":
        out = [(P, PZ)]
        pt, pz = P, PZ
        while pt != pz:
            if pt > pz:
                pt = max(pz, half(pt))
            else:
                pz = max(pt, half(pz))
            out.append((pt, pz))
        for p in seq(pt)[1:]:
            out.append((p, p))
        return out
    raise ValueError(coarsening)


def element_prolongation(Pf, Pc) -> np.ndarray:
    """Pi (Np_f x Np_c): coarse nodal basis evaluated at the fine nodes,
    Pi = Pi_z (x) Pi_tri (each factor the identity where that order is kept)."""
    (ft, fz), (ct, cz) = order_pair(Pf), order_pair(Pc)
    rf, rc = ref(ft, fz), ref(ct, cz)
    Vt, _, _ = vandermonde_tri(rf.r, rf.s, ct)
    Pi_tri = Vt @ rc.Vinv
    V1, _ = vandermonde_1d(rf.t, cz)
    Pi_z = V1 @ rc.V1inv
    return np.kron(Pi_z, Pi_tri)


def splitmix64_unit(n: int, seed: int) -> np.ndarray:
    """Counter-based uniform [0,1) numbers: splitmix64(seed + i + 1), top 53 bits."""
    M = (1 << 64) - 1
    out = np.empty(n)
    for i in range(n):
        z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z = z ^ (z >> 31)
        out[i] = (z >> 11) * (1.0 / (1 << 53))
    return out


class Level:
    def __init__(self, mesh, P, Pf, xyz_f, dir2d, top_neumann):
        self.P = P
        self.num = Numbering(mesh, *order_pair(P))
        self.geo = LevelGeometry(P, Pf, xyz_f)
        self.op = StiffnessOperator(self.num, self.geo)
        n = self.num
        mask = np.ones(n.n_dof, dtype=bool)
        if not top_neumann:
            mask[n.surface_nodes] = False
        if dir2d is not None and len(dir2d):
            # lateral Dirichlet 2D nodes at this order
            for g2 in dir2d:
                mask[g2 * n.nz:(g2 + 1) * n.nz] = False
        self.free = mask
        self.diag = self.op.diagonal()
        self.dinv = np.where(mask, 1.0 / np.where(mask, self.diag, 1.0), 0.0)
        self.omega = None

    def A(self, x):
        """A_FF x on free nodes (x is zero-extended; output zero on Dirichlet)."""
        return np.where(self.free, self.op.apply(np.where(self.free, x, 0.0)), 0.0)


class Hierarchy:
    """All levels of the p-multigrid preconditioner for one surface state."""

    def __init__(self, mesh: dict, P: int, eta2d=None, nu1=2, nu2=2, omega=None,
                 dirichlet_tags: int = 0, top_neumann: bool = False,
                 coarse: str = "exact", cheb=None, seed: int = 0,
                 smoother: str = "jacobi", smooth_ratio: float = 15.0, coarsening: str = "both",
                 overlap: int = 1, PZ: int = None, nu1_coarse: int = None, nu2_coarse: int = None):
        self.mesh = mesh
        # P: triangle order of the finest level, which is also the order of the
        # isoparametric map every level's geometry comes from (the sigma map is
        # affine along the extrusion inside a layer, so the map's vertical order
        # does not change it); PZ: vertical order of the finest level
        self.P = P
        self.PZ = P if PZ is None else int(PZ)
        self.dirichlet_tags, self.top_neumann = dirichlet_tags, top_neumann
        self.reuse = "none"
        self.orders = level_orders(P, coarsening, self.PZ)
        num_f = Numbering(mesh, P)
        if eta2d is None:
            eta2d = np.zeros(num_f.n2d)
        self.eta2d = np.asarray(eta2d, dtype=np.float64)
        xyz_f = element_node_xyz(mesh, num_f, self.eta2d)
        self.levels = []
        for p in self.orders:
            nl = Numbering(mesh, *order_pair(p))
            d2 = lateral_dirichlet_2d(mesh, nl, dirichlet_tags) if dirichlet_tags else None
            self.levels.append(Level(mesh, p, P, xyz_f, d2, top_neumann))
        self.nu1, self.nu2 = nu1, nu2
        # sweeps on the levels below the finest (None: nu1, nu2 on every level,
        # as in Alg. 1, which passes one pair down the recursion)
        self.nu1_coarse, self.nu2_coarse = nu1_coarse, nu2_coarse
        self.Pi = [element_prolongation(self.orders[i], self.orders[i + 1])
                   for i in range(len(self.orders) - 1)]
        if smoother not in ("jacobi", "chebyshev", "schwarz"):
            raise ValueError(smoother)
        if smoother == "schwarz":
            for lv in self.levels[:-1]:
                lv.schwarz = Schwarz(lv, *overlap_of(order_pair(lv.P), overlap))
        # smoothing weights
        for i, lv in enumerate(self.levels[:-1]):
            if omega is None and smoother == "schwarz":
                lv.omega = 4.0 / (3.0 * self.schwarz_rho(i, seed=seed))
            elif omega is None:
                lv.omega = 4.0 / (3.0 * self.lambda_max(i, seed=seed))
            elif np.isscalar(omega):
                lv.omega = float(omega)
            else:
                lv.omega = float(omega[i])
        self.smoother = smoother
        self.overlap = int(overlap)
        self.smooth_ratio = float(smooth_ratio)
        self.coarse_mode = coarse
        self.cheb = cheb
        self._coarse_setup()

    # -- operator reuse across surfaces
    def _rebuild(self, i, xyz_f):
        old = self.levels[i]
        nl = Numbering(self.mesh, *order_pair(old.P))
        d2 = lateral_dirichlet_2d(self.mesh, nl, self.dirichlet_tags) if self.dirichlet_tags else None
        lv = Level(self.mesh, old.P, self.P, xyz_f, d2, self.top_neumann)
        lv.omega = old.omega
        if self.smoother == "schwarz" and i < len(self.levels) - 1:
            lv.schwarz = Schwarz(lv, *overlap_of(order_pair(lv.P), self.overlap))
        self.levels[i] = lv

    def set_reuse(self, mode: str):
        if mode not in ("none", "t0", "lin"):
            raise ValueError(mode)
        if mode == "lin":
            num_f = Numbering(self.mesh, self.P)
            xyz0 = element_node_xyz(self.mesh, num_f, np.zeros(num_f.n2d))
            for i in range(1, len(self.levels)):
                self._rebuild(i, xyz0)
            self._coarse_setup()
        self.reuse = mode

    def set_surface(self, eta2d):
        self.eta2d = np.asarray(eta2d, dtype=np.float64)
        num_f = Numbering(self.mesh, self.P)
        xyz_f = element_node_xyz(self.mesh, num_f, self.eta2d)
        if self.reuse == "none":
            for i in range(len(self.levels)):
                self._rebuild(i, xyz_f)
            self._coarse_setup()
        elif self.reuse == "t0":
            lv = self.levels[0]
            lv.geo = LevelGeometry(lv.P, self.P, xyz_f)
            lv.op = StiffnessOperator(lv.num, lv.geo)
        else:
            self._rebuild(0, xyz_f)

    # -- eigenvalue estimate of D^-1 A (power iteration, Rayleigh quotient in the D inner product)
    def lambda_max(self, i: int, steps: int = 30, seed: int = 0) -> float:
        lv = self.levels[i]
        x = np.where(lv.free, splitmix64_unit(lv.num.n_dof, seed), 0.0)
        for _ in range(steps):
            y = lv.dinv * lv.A(x)
            x = y / np.linalg.norm(y)
        Ax = lv.A(x)
        rq = float(x @ Ax) / float(np.sum(np.where(lv.free, lv.diag, 0.0) * x * x))
        return 1.05 * rq

    # -- spectral radius of S^-1 A for the Schwarz preconditioner (power iteration, 2-norm)
    def schwarz_rho(self, i: int, steps: int = 30, seed: int = 0) -> float:
        lv = self.levels[i]
        x = np.where(lv.free, splitmix64_unit(lv.num.n_dof, seed), 0.0)
        for _ in range(steps):
            y = lv.schwarz.apply(lv.A(x))
            x = y / np.linalg.norm(y)
        return 1.05 * float(np.linalg.norm(lv.schwarz.apply(lv.A(x))))

    def _coarse_setup(self):
        lv = self.levels[-1]
        self.coarse_idx = np.flatnonzero(lv.free)
        if self.coarse_mode == "exact":
            A = lv.op.assembled()
            Aff = A[self.coarse_idx][:, self.coarse_idx]
            if Aff.shape[0] <= 6000:
                self._cho = sla.cho_factor(Aff.toarray())
                self._lu = None
            else:
                self._cho = None
                self._lu = spla.splu(Aff.tocsc())
        elif self.coarse_mode == "chebyshev":
            if self.cheb is None:
                raise ValueError("chebyshev coarse solve needs (degree, lmin, lmax)")
        else:
            raise ValueError(self.coarse_mode)

    def coarse_solve(self, f: np.ndarray) -> np.ndarray:
        lv = self.levels[-1]
        out = np.zeros_like(f)
        if self.coarse_mode == "exact":
            b = f[self.coarse_idx]
            x = sla.cho_solve(self._cho, b) if self._cho is not None else self._lu.solve(b)
            out[self.coarse_idx] = x
            return out
        k, lmin, lmax = self.cheb
        return chebyshev(lv.A, lv.dinv, f, int(k), float(lmin), float(lmax))

    # -- transfers
    def prolong(self, i: int, uc: np.ndarray) -> np.ndarray:
        """Fine level i from coarse level i+1: W_f Q_f^T (I (x) Pi) Q_c u_c, zero on Dirichlet."""
        lf, lc = self.levels[i], self.levels[i + 1]
        Uf = uc[lc.num.map] @ self.Pi[i].T
        uf = np.bincount(lf.num.map.ravel(), Uf.ravel(), lf.num.n_dof) / lf.num.mult
        return np.where(lf.free, uf, 0.0)

    def restrict(self, i: int, rf: np.ndarray) -> np.ndarray:
        """Transpose of ``prolong``: Q_c^T (I (x) Pi^T) Q_f W_f r_f, zero on Dirichlet."""
        lf, lc = self.levels[i], self.levels[i + 1]
        r = np.where(lf.free, rf, 0.0) / lf.num.mult
        Rc = r[lf.num.map] @ self.Pi[i]
        rc = np.bincount(lc.num.map.ravel(), Rc.ravel(), lc.num.n_dof)
        return np.where(lc.free, rc, 0.0)

    # -- Alg. 1
    def smooth(self, i: int, u: np.ndarray, f: np.ndarray, sweeps: int, post: bool = False) -> np.ndarray:
        lv = self.levels[i]
        if self.smoother == "schwarz":
            for _ in range(sweeps):
                u = u + lv.omega * lv.schwarz.apply(f - lv.A(u), transpose=post)
            return u
        if self.smoother == "chebyshev":
            if sweeps <= 0:
                return u
            lmax = 4.0 / (3.0 * lv.omega)
            return u + chebyshev(lv.A, lv.dinv, f - lv.A(u), sweeps, lmax / self.smooth_ratio, lmax)
        for _ in range(sweeps):
            u = u + lv.omega * lv.dinv * (f - lv.A(u))
        return u

    def sweeps(self, i: int):
        """(pre, post) smoothing sweeps of level i: nu1, nu2 on the finest level,
        nu1_coarse, nu2_coarse (where given) on the levels below it."""
        if i == 0:
            return self.nu1, self.nu2
        return (self.nu1 if self.nu1_coarse is None else self.nu1_coarse,
                self.nu2 if self.nu2_coarse is None else self.nu2_coarse)

    def vcycle(self, f: np.ndarray, i: int = 0, u0=None) -> np.ndarray:
        if i == len(self.levels) - 1:
            return self.coarse_solve(f)
        lv = self.levels[i]
        pre, post = self.sweeps(i)
        u = np.zeros_like(f) if u0 is None else u0.copy()
        u = self.smooth(i, u, f, pre)
        r = f - lv.A(u)
        rc = self.restrict(i, r)
        uc = self.vcycle(rc, i + 1)
        u = u + self.prolong(i, uc)
        u = self.smooth(i, u, f, post, post=True)
        return u


def chebyshev(A, dinv, f, k: int, lmin: float, lmax: float) -> np.ndarray:
    """k steps of Jacobi-preconditioned Chebyshev iteration from x = 0 on [lmin, lmax].

    Three-term recurrence of the shifted-and-scaled Chebyshev polynomials
    (theta = (lmax+lmin)/2, delta = (lmax-lmin)/2, sigma = theta/delta):
    rho_0 = 1/sigma, d_0 = z_0/theta;  rho_j = 1/(2 sigma - rho_{j-1}),
    d_j = rho_j rho_{j-1} d_{j-1} + 2 rho_j/delta z_j, with z = D^-1 r.
    """
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    x = np.zeros_like(f)
    r = f.copy()
    rho = 1.0 / sigma
    d = dinv * r / theta
    for j in range(k):
        x = x + d
        if j == k - 1:
            break
        r = r - A(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + 2.0 * rho_new / delta * (dinv * r)
        rho = rho_new
    return x
