"""Reference prism of order P: nodes, cubature, basis and matrices (FP64).

Sec. 3.1 builds V^p from continuous piecewise polynomials with a nodal
(cardinal) basis; Fig. pcoarse places LGL nodes along edges.  The prism is a
triangle (r, s) in T = {r, s >= -1, r + s <= 0} times t in [-1, 1].  Local node
n = c * Np_tri + a pairs vertical LGL node c (bottom to top) with triangle
node a.  Cubature point q = k * Nq_tri + qt pairs vertical Gauss point k with
triangle point qt = j * (P + 1) + i.
"""
from __future__ import annotations

from functools import lru_cache
from math import gamma, sqrt

import numpy as np
from scipy.special import eval_jacobi


# ---------------------------------------------------------------------------
# 1D rules
# ---------------------------------------------------------------------------

def gauss_jacobi(n: int, alpha: float, beta: float):
    """n-point Gauss-Jacobi rule for weight (1-x)^alpha (1+x)^beta (Golub-Welsch)."""
    a, b = float(alpha), float(beta)
    k = np.arange(n, dtype=np.float64)
    # three-term recurrence of the monic Jacobi polynomials
    denom = (2 * k + a + b) * (2 * k + a + b + 2)
    diag = np.where(denom == 0, (b - a) / (a + b + 2), (b * b - a * a) / np.where(denom == 0, 1, denom))
    kk = np.arange(1, n, dtype=np.float64)
    num = 4 * kk * (kk + a) * (kk + b) * (kk + a + b)
    den = (2 * kk + a + b) ** 2 * (2 * kk + a + b + 1) * (2 * kk + a + b - 1)
    off = np.sqrt(num / den)
    J = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    mu0 = 2.0 ** (a + b + 1) * gamma(a + 1) * gamma(b + 1) / gamma(a + b + 2)
    w = mu0 * V[0, :] ** 2
    return x, w


def gauss_legendre(n: int):
    return gauss_jacobi(n, 0.0, 0.0)


def lgl_nodes(P: int) -> np.ndarray:
    """P+1 Legendre-Gauss-Lobatto nodes: -1, 1 and the roots of P_P'."""
    if P == 0:
        return np.zeros(1)
    if P == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(P + 1)
    c[P] = 1.0
    inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    # polish with Newton on P_P'(x) = 0
    dc = np.polynomial.legendre.legder(c)
    ddc = np.polynomial.legendre.legder(dc)
    for _ in range(3):
        inner = inner - np.polynomial.legendre.legval(inner, dc) / np.polynomial.legendre.legval(inner, ddc)
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


# ---------------------------------------------------------------------------
# orthonormal polynomials
# ---------------------------------------------------------------------------

def jacobi_normalized(x, alpha: float, beta: float, n: int):
    """Jacobi polynomial P_n^(alpha,beta), orthonormal for its weight on [-1,1]."""
    x = np.asarray(x, dtype=np.float64)
    h = 2.0 ** (alpha + beta + 1) / (2 * n + alpha + beta + 1) * \
        gamma(n + alpha + 1) * gamma(n + beta + 1) / (gamma(n + alpha + beta + 1) * gamma(n + 1))
    return eval_jacobi(n, alpha, beta, x) / sqrt(h)


def jacobi_normalized_deriv(x, alpha: float, beta: float, n: int):
    """d/dx of ``jacobi_normalized`` via d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    h = 2.0 ** (alpha + beta + 1) / (2 * n + alpha + beta + 1) * \
        gamma(n + alpha + 1) * gamma(n + beta + 1) / (gamma(n + alpha + beta + 1) * gamma(n + 1))
    return 0.5 * (n + alpha + beta + 1) * eval_jacobi(n - 1, alpha + 1, beta + 1, x) / sqrt(h)


def vandermonde_1d(x, P: int):
    """V[i, n] = orthonormal Legendre p_n(x_i), n = 0..P, and its derivative."""
    x = np.asarray(x, dtype=np.float64)
    V = np.stack([jacobi_normalized(x, 0, 0, n) for n in range(P + 1)], axis=1)
    Vx = np.stack([jacobi_normalized_deriv(x, 0, 0, n) for n in range(P + 1)], axis=1)
    return V, Vx


def tri_modes(P: int):
    """Mode list (i, j), i + j <= P, of the triangle basis."""
    return [(i, j) for i in range(P + 1) for j in range(P + 1 - i)]


def vandermonde_tri(r, s, P: int):
    """Orthonormal PKD/Dubiner basis on T and its r, s derivatives.

    psi_ij = sqrt(2) p_i(a) p_j^(2i+1,0)(b) (1-b)^i with collapsed
    coordinates a = 2(1+r)/(1-s) - 1 and b = s.
    """
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    one_m_s = 1.0 - s
    safe = np.where(np.abs(one_m_s) < 1e-14, 1.0, one_m_s)
    a = np.where(np.abs(one_m_s) < 1e-14, -1.0, 2.0 * (1.0 + r) / safe - 1.0)
    b = s
    cols, cr, cs = [], [], []
    for (i, j) in tri_modes(P):
        f = jacobi_normalized(a, 0, 0, i)
        fd = jacobi_normalized_deriv(a, 0, 0, i)
        g = jacobi_normalized(b, 2 * i + 1, 0, j)
        gd = jacobi_normalized_deriv(b, 2 * i + 1, 0, j)
        pw = (1.0 - b) ** i
        pwm1 = (1.0 - b) ** (i - 1) if i >= 1 else np.zeros_like(b)
        cols.append(sqrt(2.0) * f * g * pw)
        # d/dr: da/dr = 2/(1-b)
        cr.append(sqrt(2.0) * fd * g * 2.0 * pwm1)
        # d/ds: da/ds = (1+a)/(1-b), db/ds = 1
        cs.append(sqrt(2.0) * (fd * (1.0 + a) * g * pwm1 + f * gd * pw - i * f * g * pwm1))
    return np.stack(cols, 1), np.stack(cr, 1), np.stack(cs, 1)


# ---------------------------------------------------------------------------
# triangle nodes and cubature
# ---------------------------------------------------------------------------

def tri_node_ijk(P: int):
    """Lattice indices (i, j, k), i + j + k = P, in local order (j outer, i inner)."""
    return [(i, j, P - i - j) for j in range(P + 1) for i in range(P + 1 - j)]


def tri_nodes(P: int):
    """Blyth-Pozrikidis nodes built from the 1D LGL nodes v = (1 + xi)/2.

    x = (1 + 2 v_i - v_j - v_k)/3, y = (1 + 2 v_j - v_i - v_k)/3, then
    (r, s) = (2x - 1, 2y - 1); vertices v0=(-1,-1), v1=(1,-1), v2=(-1,1).
    """
    if P == 0:
        return np.array([-1.0 / 3]), np.array([-1.0 / 3])
    v = (1.0 + lgl_nodes(P)) / 2.0
    rs = []
    for (i, j, k) in tri_node_ijk(P):
        x = (1.0 + 2 * v[i] - v[j] - v[k]) / 3.0
        y = (1.0 + 2 * v[j] - v[i] - v[k]) / 3.0
        rs.append((2 * x - 1, 2 * y - 1))
    rs = np.asarray(rs)
    return rs[:, 0], rs[:, 1]


def tri_cubature(P: int):
    """Collapsed (P+1)^2 rule: Gauss-Legendre in a, Gauss-Jacobi(1,0) in b.

    r = (1+a)(1-b)/2 - 1, s = b, w = w_a w_b / 2; point index j*(P+1)+i.
    """
    n = P + 1
    a, wa = gauss_legendre(n)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    r = np.empty(n * n)
    s = np.empty(n * n)
    w = np.empty(n * n)
    for j in range(n):
        for i in range(n):
            q = j * n + i
            r[q] = (1 + a[i]) * (1 - b[j]) / 2 - 1
            s[q] = b[j]
            w[q] = wa[i] * wb[j] / 2
    return r, s, w


# ---------------------------------------------------------------------------
# reference element
# ---------------------------------------------------------------------------

class RefElement:
    """Reference prism of order P in the triangle and PZ (default P) along the
    extrusion, with matrices at its own cubature points: (P+1)^2 collapsed
    points on the triangle times PZ+1 Gauss points vertically (exact for the
    stiffness of affine prisms in each direction)."""

    def __init__(self, P: int, PZ: int = None):
        PZ = P if PZ is None else PZ
        self.P = P
        self.PZ = PZ
        self.n1 = PZ + 1
        self.np_tri = (P + 1) * (P + 2) // 2
        self.np = self.np_tri * (PZ + 1)
        self.nq_tri = (P + 1) ** 2
        self.nq = self.nq_tri * (PZ + 1)
        self.r, self.s = tri_nodes(P)
        self.t = lgl_nodes(PZ)
        self.V, _, _ = vandermonde_tri(self.r, self.s, P)
        self.Vinv = np.linalg.inv(self.V)
        self.V1, _ = vandermonde_1d(self.t, PZ)
        self.V1inv = np.linalg.inv(self.V1)
        self.cr, self.cs, self.cw = tri_cubature(P)
        self.zq, self.zw = gauss_legendre(PZ + 1)
        self.B, self.Dr, self.Ds = self.tri_eval(self.cr, self.cs)
        self.Bz, self.Dz = self.line_eval(self.zq)
        self.w = np.kron(self.zw, self.cw)  # prism cubature weights

    # nodal interpolation/derivative matrices of this order at given points
    def tri_eval(self, r, s):
        Vq, Vr, Vs = vandermonde_tri(r, s, self.P)
        return Vq @ self.Vinv, Vr @ self.Vinv, Vs @ self.Vinv

    def line_eval(self, t):
        Vq, Vt = vandermonde_1d(t, self.PZ)
        return Vq @ self.V1inv, Vt @ self.V1inv

    def prism_mats(self, cr, cs, zq):
        """Interpolation and r/s/t derivative matrices (Nq x Np) at a tensor point set."""
        B, Dr, Ds = self.tri_eval(cr, cs)
        Bz, Dz = self.line_eval(zq)
        return np.kron(Bz, B), np.kron(Bz, Dr), np.kron(Bz, Ds), np.kron(Dz, B)


@lru_cache(maxsize=None)
def ref(P: int, PZ: int = None) -> RefElement:
    return RefElement(P, P if PZ is None else PZ)


def order_pair(order):
    """(triangle order, vertical order) of a level order given as P or (P, PZ)."""
    if isinstance(order, (tuple, list)):
        return int(order[0]), int(order[1])
    return int(order), int(order)
