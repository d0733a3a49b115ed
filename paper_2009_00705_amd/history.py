"""Time history of Laplace solves along a focusing wave group (learned warm start).

Each time level n sets the free surface eta_n and solves with the surface
potential phi~_n as Dirichlet data (Sec. 2: one Laplace solve per stage of
the free-surface time stepping).  The history supplies the training set of
the warm-start network (features of the coarsest nodes, target = correction
of the extrapolated guess) and the test steps on which the guesses are
compared: zero, previous solution, extrapolation 2 phi_{n-1} - phi_{n-2},
and extrapolation plus the learned correction.
"""
from __future__ import annotations

import time

import numpy as np

from . import pmg
from .workloads import WaveGroup


class History:
    def __init__(self, ctx: "pmg.Context", wave: WaveGroup):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.wave = wave
        xy = ctx.surface_xy()
        self.x = xy[:, 0]
        self.n_dof = ctx.levels[0]["n_dof"]
        self.n1 = ctx.levels[ctx.net_level]["n_dof"]
        self._surf = {}

    def surface(self, n: int):
        """(eta_n, phi~_n) as device tensors (cached)."""
        if n not in self._surf:
            eta, phis = self.wave.surface(self.x, n)
            t = self.torch
            self._surf[n] = (t.from_numpy(eta).cuda(), t.from_numpy(phis).cuda())
        return self._surf[n]

    def set_step(self, n: int):
        eta, phis = self.surface(n)
        self.ctx.set_surface(eta)
        return phis

    def solve_sequence(self, steps, guess="extrap", sols=None, net=None, rtol=1e-8, imax=500):
        """Solve the given steps in order; returns {n: solution} and per-step stats.

        ``sols`` holds earlier solutions (needed by the previous / extrapolated /
        learned guesses).  The solve time excludes pmg_set_surface.
        """
        t = self.torch
        sols = {} if sols is None else dict(sols)
        stats = []
        for n in steps:
            phis = self.set_step(n)
            phi = t.zeros(self.n_dof, dtype=t.float64, device="cuda")
            mode, hist = guess, None
            if guess == "prev" and (n - 1) in sols:
                phi.copy_(sols[n - 1])
                mode = "given"
            elif guess in ("extrap", "learned") and (n - 1) in sols and (n - 2) in sols:
                hist = [sols[n - 1], sols[n - 2]]
            elif guess in ("extrap3", "learned3") and all((n - k) in sols for k in (1, 2, 3)):
                hist = [sols[n - 1], sols[n - 2], sols[n - 3]]
            elif guess in ("extrap3", "learned3") and (n - 1) in sols and (n - 2) in sols:
                mode, hist = "extrap", [sols[n - 1], sols[n - 2]]
            elif guess != "zero":
                mode = "given" if (n - 1) in sols else "zero"
                if mode == "given":
                    phi.copy_(sols[n - 1])
            t.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = self.ctx.solve(phi, phi_surf=phis, guess=mode, hist=hist,
                                    net=net if mode in ("learned", "learned3") else None,
                                    rtol=rtol, imax=imax)
            t.cuda.synchronize()
            st["wall_ms"] = (time.perf_counter() - t0) * 1e3
            st["status"] = rc
            st["step"] = n
            stats.append(st)
            sols[n] = phi
        return sols, stats

    def training_set(self, sols, steps, third=False):
        """Features and targets of the coarsest nodes for the given steps (device
        float32), relative to the second- or (third=True) third-order extrapolation."""
        t = self.torch
        Xs, Ts = [], []
        for n in steps:
            _, phis = self.surface(n)
            X = t.empty((self.n1, 7), dtype=t.float32, device="cuda")
            T = t.empty(self.n1, dtype=t.float32, device="cuda")
            self.ctx.features(phis, sols[n - 1], sols[n - 2], X, pnow=sols[n], T=T,
                              p3=sols[n - 3] if third else None)
            Xs.append(X)
            Ts.append(T)
        return t.cat(Xs).contiguous(), t.cat(Ts).contiguous()


def summarize(stats):
    it = np.array([s["iters"] for s in stats])
    ms = np.array([s["wall_ms"] for s in stats])
    r0 = np.array([s["res_hist"][0] / s["norm_f"] if s["norm_f"] > 0 else 0 for s in stats])
    return {"solves_per_s": float(len(stats) / (ms.sum() / 1e3)), "ms_per_solve": float(ms.mean()),
            "iters_mean": float(it.mean()), "iters_max": int(it.max()),
            "initial_rel_res_median": float(np.median(r0)),
            "guess_ms_mean": float(np.mean([s.get("t_guess_ms", 0.0) for s in stats])),
            "fallbacks": int(sum(1 for s in stats if s.get("fallback"))),
            "max_rel_res": float(max(s["rel_res"] for s in stats))}
