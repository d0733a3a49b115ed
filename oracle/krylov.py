"""Outer iterations around the p-multigrid V-cycle (FP64).

The Laplace problem (eq. laplaceproblem) is discretised into A phi = b
(eq. laplaceproblemdiscrete, A = -L).  Dirichlet values phi_D at z = eta
(and at lateral nodes chosen by tests) are imposed by lifting:
f = (b_N - A phi_D) on the free nodes, A_FF phi_F = f_F, phi = phi_D + phi_F.
With no-flux walls and bottom b_N = 0.

Stop test (Sec. 5, after Alg. 1): ||r||_2 <= rtol ||f||_2 + atol, checked
before every iteration.  The convergence factor q_m = ||r_m|| / ||r_{m-1}||
(eq. convrate) is recorded.

* ``pcg``  -- Alg. 3 with q <- A p (the printed "A delta" is read as A p) and
              Fletcher-Reeves beta = z^T r / delta.
* ``fpcg`` -- the same with Polak-Ribiere beta = z_{k+1}^T (r_{k+1} - r_k) / delta_k
              (flexible: tolerates a preconditioner that changes between calls).
* ``pdc``  -- Alg. 2, u <- u - MG(-r) = u + MG(r), residual recomputed after
              every correction so that the test uses the current residual.
* ``mg``   -- stand-alone V-cycles on the full problem with the current iterate
              as initial guess (Alg. 1 at the top level with u != 0).
"""
from __future__ import annotations

import numpy as np

from .mg import Hierarchy


class SolveResult:
    def __init__(self, phi, iters, res_hist, rel_res, norm_f):
        self.phi = phi
        self.iters = iters
        self.res_hist = np.asarray(res_hist)
        self.rel_res = rel_res
        self.norm_f = norm_f

    @property
    def q(self):
        h = self.res_hist
        return h[1:] / h[:-1] if h.size > 1 else np.zeros(0)


def lifted_rhs(h: Hierarchy, phi_dir: np.ndarray):
    """phi_D (values at Dirichlet nodes, zero elsewhere) and f = -A phi_D on free nodes."""
    lv = h.levels[0]
    phiD = np.where(lv.free, 0.0, phi_dir)
    f = np.where(lv.free, -lv.op.apply(phiD), 0.0)
    return phiD, f


def solve(h: Hierarchy, phi_dir: np.ndarray, guess=None, method: str = "pcg",
          rtol: float = 1e-8, atol: float = 0.0, imax: int = 200,
          precond=None) -> SolveResult:
    """Solve for phi with Dirichlet values ``phi_dir`` (full-length, read at Dirichlet nodes)."""
    lv = h.levels[0]
    A = lv.A
    M = precond if precond is not None else (lambda r: h.vcycle(r))
    phiD, f = lifted_rhs(h, phi_dir)
    u = np.zeros_like(f) if guess is None else np.where(lv.free, guess, 0.0)
    nf = float(np.linalg.norm(f))
    tol = rtol * nf + atol
    r = f - A(u)
    hist = [float(np.linalg.norm(r))]
    i = 0
    if method in ("pcg", "fpcg"):
        p = M(r)
        delta = float(p @ r)
        while i < imax and hist[-1] > tol:
            q = A(p)
            alpha = delta / float(p @ q)
            u = u + alpha * p
            r_old = r
            r = r - alpha * q
            hist.append(float(np.linalg.norm(r)))
            z = M(r)
            if method == "pcg":
                beta = float(z @ r) / delta
            else:
                beta = float(z @ (r - r_old)) / delta
            p = z + beta * p
            delta = float(z @ r)
            i += 1
    elif method == "pdc":
        while i < imax and hist[-1] > tol:
            u = u + M(r)
            r = f - A(u)
            hist.append(float(np.linalg.norm(r)))
            i += 1
    elif method == "mg":
        while i < imax and hist[-1] > tol:
            u = h.vcycle(f, 0, u0=u)
            r = f - A(u)
            hist.append(float(np.linalg.norm(r)))
            i += 1
    else:
        raise ValueError(method)
    phi = phiD + u
    rel = float(np.linalg.norm(f - A(u))) / nf if nf > 0 else 0.0
    return SolveResult(phi, i, hist, rel, nf)


def direct_solve(h: Hierarchy, phi_dir: np.ndarray) -> np.ndarray:
    """The discrete solution by definition: sparse LU of A_FF (small meshes)."""
    import scipy.sparse.linalg as spla
    lv = h.levels[0]
    A = lv.op.assembled()
    free = np.flatnonzero(lv.free)
    phiD, f = lifted_rhs(h, phi_dir)
    Aff = A[free][:, free].tocsc()
    u = np.zeros_like(f)
    u[free] = spla.spsolve(Aff, f[free])
    return phiD + u


def relative_residual(h: Hierarchy, phi: np.ndarray, phi_dir: np.ndarray) -> float:
    """||f - A_FF phi_F|| / ||f|| for a full-length phi (definition of the stop test)."""
    lv = h.levels[0]
    phiD, f = lifted_rhs(h, phi_dir)
    u = np.where(lv.free, phi, 0.0)
    return float(np.linalg.norm(f - lv.A(u))) / float(np.linalg.norm(f))
