"""Thin ctypes binding of libpmg.so (include/pmg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device arrays are torch tensors on the context's GPU (their
``data_ptr()`` is passed through); host arrays are numpy arrays.  The binding
raises ``PmgError`` on negative status codes and never falls back to any other
implementation: without the built library nothing here works.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmg.so")

PMG_OK, PMG_NOT_CONVERGED, PMG_FALLBACK_USED = 0, 1, 2
PMG_FP64, PMG_MIXED_FP32, PMG_MIXED_BF16, PMG_MIXED_BF16G, PMG_MIXED_BF16X3, PMG_MIXED_BF16X2 = 0, 1, 2, 3, 4, 5
PMG_PCG, PMG_FPCG, PMG_PDC, PMG_MG = 0, 1, 2, 3
PMG_GUESS_GIVEN, PMG_GUESS_ZERO, PMG_GUESS_LEARNED, PMG_GUESS_EXTRAP, PMG_GUESS_EXTRAP3, PMG_GUESS_LEARNED3 = \
    0, 1, 2, 3, 4, 5
PMG_COARSE_EXACT, PMG_COARSE_CHEBYSHEV = 0, 1
PMG_COARSEN_BOTH, PMG_COARSEN_XY_FIRST, PMG_COARSEN_EQUAL = 0, 1, 2

STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "FALLBACK_USED", -1: "EINVAL", -2: "ENOMEM",
          -3: "EDEVICE", -4: "EBREAKDOWN", -5: "ENONFINITE", -6: "EMESH", -7: "ESTATE"}
STATUS_CODES = {v: k for k, v in STATUS.items()}
PRECISIONS = {"fp64": PMG_FP64, "fp32": PMG_MIXED_FP32, "bf16": PMG_MIXED_BF16, "bf16g": PMG_MIXED_BF16G,
              "bf16x3": PMG_MIXED_BF16X3, "bf16x2": PMG_MIXED_BF16X2}
KRYLOV = {"pcg": PMG_PCG, "fpcg": PMG_FPCG, "pdc": PMG_PDC, "mg": PMG_MG}


class PmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("xy", C.POINTER(C.c_double)), ("nt", C.c_int32),
                ("tri", C.POINTER(C.c_int32)), ("edge_tag", C.POINTER(C.c_int32)),
                ("ncurved", C.c_int32), ("curved_edge", C.POINTER(C.c_int32)),
                ("circle", C.POINTER(C.c_double)), ("n_layers", C.c_int32), ("depth", C.c_double)]


class Options(C.Structure):
    _fields_ = [("P", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32), ("omega", C.c_double * 8),
                ("precision", C.c_int32), ("krylov", C.c_int32), ("dirichlet_tags", C.c_uint32),
                ("top_neumann", C.c_int32), ("coarse", C.c_int32), ("cheb_degree", C.c_int32),
                ("cheb_lmin", C.c_double), ("cheb_lmax", C.c_double), ("cheb_ratio", C.c_double),
                ("exact_max", C.c_int32), ("seed", C.c_uint64), ("host_only", C.c_int32),
                ("kernel_variant", C.c_int32), ("smoother", C.c_int32), ("smooth_ratio", C.c_double),
                ("coarsening", C.c_int32), ("overlap", C.c_int32), ("schwarz_store", C.c_int32),
                ("schwarz_chunk", C.c_int64), ("geometry", C.c_int32), ("PZ", C.c_int32),
                ("fused_sum", C.c_int32), ("graphs", C.c_int32), ("dss", C.c_int32),
                ("nu1_coarse", C.c_int32), ("nu2_coarse", C.c_int32)]


class FnpfStats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 4), ("rel_res", C.c_double * 4), ("t_step_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("status", C.c_int32)]

    def as_dict(self):
        return dict(iters=list(self.iters), rel_res=list(self.rel_res), t_step_ms=self.t_step_ms,
                    t_solve_ms=self.t_solve_ms, status=self.status)


class SchwarzInfo(C.Structure):
    _fields_ = [("dt", C.c_int32), ("dz", C.c_int32), ("n_sub", C.c_int64), ("max_size", C.c_int32),
                ("total", C.c_int64), ("inv_entries", C.c_int64)]


class LevelInfo(C.Structure):
    _fields_ = [("order", C.c_int32), ("np", C.c_int32), ("nq", C.c_int32), ("n_colours", C.c_int32),
                ("n_dof", C.c_int64), ("n_free", C.c_int64), ("n_elem", C.c_int64),
                ("n_surface", C.c_int64), ("order_z", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_hist", C.c_int32), ("rel_res", C.c_double),
                ("norm_f", C.c_double), ("res_hist", C.c_double * 512), ("t_solve_ms", C.c_double),
                ("t_guess_ms", C.c_double), ("fallback", C.c_int32), ("n_vcycles", C.c_int32),
                ("n_fine_applies", C.c_int32), ("n_graph_vcycles", C.c_int32)]

    def as_dict(self):
        h = np.array(self.res_hist[: self.n_hist])
        return dict(iters=self.iters, rel_res=self.rel_res, norm_f=self.norm_f, res_hist=h,
                    q=h[1:] / h[:-1] if h.size > 1 else np.zeros(0), t_solve_ms=self.t_solve_ms,
                    t_guess_ms=self.t_guess_ms, fallback=self.fallback, n_vcycles=self.n_vcycles,
                    n_fine_applies=self.n_fine_applies, n_graph_vcycles=self.n_graph_vcycles)


_lib = None

# name -> (restype, argtypes); every symbol include/pmg.h declares
_VP, _I, _D = C.c_void_p, C.c_int, C.c_double
SIGNATURES = {
    "pmg_options_default": (None, [C.POINTER(Options)]),
    "pmg_create": (_I, [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(_VP)]),
    "pmg_destroy": (None, [_VP]),
    "pmg_last_error": (C.c_char_p, [_VP]),
    "pmg_global_error": (C.c_char_p, []),
    "pmg_abi_version": (_I, []),
    "pmg_n_levels": (_I, [_VP]),
    "pmg_level_info_get": (_I, [_VP, _I, C.POINTER(LevelInfo)]),
    "pmg_gather_map": (_I, [_VP, _I, _VP]),
    "pmg_colours": (_I, [_VP, _I, _VP]),
    "pmg_dss_colours": (_I, [_VP, _I, _VP]),
    "pmg_surface_xy": (_I, [_VP, _VP]),
    "pmg_dirichlet_mask": (_I, [_VP, _I, _VP]),
    "pmg_set_surface": (_I, [_VP, _VP, _VP]),
    "pmg_node_xyz": (_I, [_VP, _I, _VP]),
    "pmg_apply": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "pmg_diagonal": (_I, [_VP, _I, _VP, _VP]),
    "pmg_smooth": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "pmg_prolong": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "pmg_restrict": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "pmg_coarse_solve": (_I, [_VP, _I, _VP, _VP, _VP]),
    "pmg_vcycle": (_I, [_VP, _I, _VP, _VP, _VP]),
    "pmg_get_params": (_I, [_VP, _VP, _VP, _VP]),
    "pmg_set_params": (_I, [_VP, _VP, _D, _D]),
    "pmg_solve": (_I, [_VP, _VP, _VP, _VP, _I, _VP, _VP, _D, _D, C.c_int32, C.POINTER(Stats), _VP]),
    "pmg_set_solver": (_I, [_VP, _I, _I]),
    "pmg_coarse_info": (_I, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pmg_schwarz_info_get": (_I, [_VP, _I, C.POINTER(SchwarzInfo)]),
    "pmg_surface_grad": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "pmg_set_reuse": (_I, [_VP, _I, _VP]),
    "pmg_surface_w": (_I, [_VP, _VP, _VP, _VP]),
    "pmg_fnpf_rhs": (_I, [_VP, _VP, _VP, _D, _VP, C.c_int32, _D, _D, C.c_int32, _VP, _VP, C.POINTER(Stats), _VP]),
    "pmg_fnpf_erk4": (_I, [_VP, _VP, _VP, _D, _D, _VP, C.c_int32, _D, _D, C.c_int32, C.POINTER(FnpfStats), _VP]),
    "pmg_schwarz_nodes": (_I, [_VP, _I, _VP, _VP]),
    "pmg_time_kernel": (_I, [_VP, _I, _I, _I, _I, C.POINTER(C.c_double), _VP]),
    "pmg_features": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pmg_net_level": (_I, [_VP]),
    "pmg_net_create": (_I, [_VP, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_VP)]),
    "pmg_net_destroy": (None, [_VP]),
    "pmg_net_size": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "pmg_net_get_params": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "pmg_net_set_params": (_I, [_VP, _VP, _VP, _VP, _D]),
    "pmg_net_forward": (_I, [_VP, _VP, C.c_int64, _VP, _VP]),
    "pmg_net_forward_noalloc": (_I, [_VP, _VP, C.c_int64, _VP, _VP]),
    "pmg_net_loss_grad": (_I, [_VP, _VP, _VP, C.c_int32, _VP, _VP, _VP]),
    "pmg_net_adam_step": (_I, [_VP, _D, _VP]),
    "pmg_net_train": (_I, [_VP, _VP, _VP, C.c_int64, C.c_int32, C.c_int32, _D, C.c_uint64, _VP, _VP]),
    "pmg_net_save": (_I, [_VP, C.c_char_p]),
    "pmg_net_load": (_I, [_VP, C.c_char_p]),
}
KERNELS = {"element_op": 0, "assemble": 1, "geometry": 2, "restrict": 3, "prolong": 4, "copy": 5, "schwarz": 6,
           "colsum_op": 7, "col_sum_store": 8, "col_sum_cheb": 9}
SMOOTHERS = {"jacobi": 0, "chebyshev": 1, "schwarz": 2}


def lib():
    """Load libpmg.so (built in-tree by ``paper_2009_00705_amd.build``).

    torch is imported first: its bundled HIP runtime then also serves this
    library (same soname), so one process never holds two HIP runtimes.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (HIP runtime shared with the library)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run `python -m paper_2009_00705_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc < 0:
        L = lib()
        msg = (L.pmg_last_error(ctx) if ctx else L.pmg_global_error()) or b""
        raise PmgError(rc, msg.decode())
    return rc


def _dptr(t, dtype=None):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def default_options(**kw) -> Options:
    o = Options()
    lib().pmg_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "omega":
            vals = list(v) + [0.0] * (8 - len(v))
            o.omega = (C.c_double * 8)(*vals)
        elif k == "precision" and isinstance(v, str):
            o.precision = PRECISIONS[v]
        elif k == "krylov" and isinstance(v, str):
            o.krylov = KRYLOV[v]
        elif k == "smoother" and isinstance(v, str):
            o.smoother = SMOOTHERS[v]
        elif k == "coarse" and isinstance(v, str):
            o.coarse = {"exact": PMG_COARSE_EXACT, "chebyshev": PMG_COARSE_CHEBYSHEV}[v]
        elif k == "schwarz_store" and isinstance(v, str):
            o.schwarz_store = sum({"fp64": 1, "fp32": 2, "bf16": 4}[x] for x in v.split(",") if x)
        elif k == "coarsening" and isinstance(v, str):
            o.coarsening = {"both": PMG_COARSEN_BOTH, "xy": PMG_COARSEN_XY_FIRST, "equal": PMG_COARSEN_EQUAL}[v]
        elif k == "geometry" and isinstance(v, str):
            o.geometry = {"stored": 0, "column": 1}[v]
        else:
            setattr(o, k, v)
    return o


class Context:
    """Owner of one ``pmg_ctx`` (a mesh, an order and its level hierarchy)."""

    def __init__(self, mesh: dict, **opts):
        self._keep = []
        xy = np.ascontiguousarray(mesh["xy"], dtype=np.float64)
        tri = np.ascontiguousarray(mesh["tri"], dtype=np.int32)
        tags = np.ascontiguousarray(mesh["edge_tag"], dtype=np.int32)
        ce = np.ascontiguousarray(mesh.get("curved_edge", np.zeros((0, 2))), dtype=np.int32)
        circ = np.ascontiguousarray(mesh.get("circle", np.zeros((0, 3))), dtype=np.float64)
        self._keep += [xy, tri, tags, ce, circ]
        m = Mesh()
        m.nv = xy.shape[0]
        m.xy = xy.ctypes.data_as(C.POINTER(C.c_double))
        m.nt = tri.shape[0]
        self.n_tri = int(tri.shape[0])
        m.tri = tri.ctypes.data_as(C.POINTER(C.c_int32))
        m.edge_tag = tags.ctypes.data_as(C.POINTER(C.c_int32))
        m.ncurved = ce.shape[0]
        m.curved_edge = ce.ctypes.data_as(C.POINTER(C.c_int32)) if ce.shape[0] else None
        m.circle = circ.ctypes.data_as(C.POINTER(C.c_double)) if ce.shape[0] else None
        m.n_layers = int(mesh["n_layers"])
        m.depth = float(mesh["depth"])
        self.options = default_options(**opts)
        h = C.c_void_p()
        _check(lib().pmg_create(C.byref(m), C.byref(self.options), C.byref(h)))
        self.h = h
        self.n_levels = lib().pmg_n_levels(h)
        self.levels = [self.level_info(i) for i in range(self.n_levels)]

    def close(self):
        if getattr(self, "h", None):
            lib().pmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc):
        return _check(rc, self.h)

    # ---- host queries
    def level_info(self, level: int) -> dict:
        li = LevelInfo()
        self._c(lib().pmg_level_info_get(self.h, level, C.byref(li)))
        return {f: getattr(li, f) for f, _ in LevelInfo._fields_}

    def gather_map(self, level: int = 0) -> np.ndarray:
        li = self.levels[level]
        out = np.empty((li["n_elem"], li["np"]), dtype=np.int32)
        self._c(lib().pmg_gather_map(self.h, level, out.ctypes.data_as(C.c_void_p)))
        return out

    def colours(self, level: int = 0) -> np.ndarray:
        out = np.empty(self.levels[level]["n_elem"], dtype=np.int32)
        self._c(lib().pmg_colours(self.h, level, out.ctypes.data_as(C.c_void_p)))
        return out

    def dss_colours(self, level: int = 0) -> np.ndarray:
        """Triangle colours of the coloured direct-stiffness sum (pmg_dss_colours)."""
        out = np.empty(self.n_tri, dtype=np.int32)
        self._c(lib().pmg_dss_colours(self.h, level, out.ctypes.data_as(C.c_void_p)))
        return out

    def surface_xy(self) -> np.ndarray:
        out = np.empty((self.levels[0]["n_surface"], 2))
        self._c(lib().pmg_surface_xy(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def dirichlet_mask(self, level: int = 0) -> np.ndarray:
        out = np.empty(self.levels[level]["n_dof"], dtype=np.uint8)
        self._c(lib().pmg_dirichlet_mask(self.h, level, out.ctypes.data_as(C.c_void_p)))
        return out

    def node_xyz(self, level: int = 0) -> np.ndarray:
        out = np.empty((self.levels[level]["n_dof"], 3))
        self._c(lib().pmg_node_xyz(self.h, level, out.ctypes.data_as(C.c_void_p)))
        return out

    def params(self):
        om = np.zeros(self.n_levels)
        lo, hi = C.c_double(), C.c_double()
        self._c(lib().pmg_get_params(self.h, om.ctypes.data_as(C.c_void_p), C.byref(lo), C.byref(hi)))
        return om, lo.value, hi.value

    def schwarz_info(self, level: int) -> dict:
        si = SchwarzInfo()
        self._c(lib().pmg_schwarz_info_get(self.h, level, C.byref(si)))
        return {f: getattr(si, f) for f, _ in SchwarzInfo._fields_}

    def schwarz_nodes(self, level: int):
        """Free global nodes of every Schwarz subdomain of a level (list of arrays)."""
        info = self.schwarz_info(level)
        ptr = np.empty(info["n_sub"] + 1, dtype=np.int32)
        nodes = np.empty(max(1, info["total"]), dtype=np.int32)
        self._c(lib().pmg_schwarz_nodes(self.h, level, ptr.ctypes.data_as(C.c_void_p),
                                        nodes.ctypes.data_as(C.c_void_p)))
        return [nodes[ptr[k]:ptr[k + 1]] for k in range(info["n_sub"])]

    def coarse_info(self) -> dict:
        mode, deg = C.c_int(), C.c_int()
        lo, hi = C.c_double(), C.c_double()
        nf = C.c_int64()
        self._c(lib().pmg_coarse_info(self.h, C.byref(mode), C.byref(deg), C.byref(lo), C.byref(hi), C.byref(nf)))
        return {"mode": "exact" if mode.value == 0 else "chebyshev", "degree": deg.value, "lmin": lo.value,
                "lmax": hi.value, "n_free": nf.value}

    def set_params(self, omega=None, cheb_lmin=0.0, cheb_lmax=0.0):
        om = None
        if omega is not None:
            om = np.ascontiguousarray(omega, dtype=np.float64)
            self._keep.append(om)
        self._c(lib().pmg_set_params(self.h, om.ctypes.data_as(C.c_void_p) if om is not None else None,
                                     float(cheb_lmin), float(cheb_lmax)))

    # ---- device calls (torch tensors)
    def set_surface(self, eta, stream=None):
        import torch
        self._c(lib().pmg_set_surface(self.h, _dptr(eta, torch.float64), _stream(stream)))

    def apply(self, level, x, y, precision="fp64", masked=True, stream=None):
        p = PRECISIONS[precision]
        self._c(lib().pmg_apply(self.h, level, p, 1 if masked else 0, _dptr(x), _dptr(y), _stream(stream)))

    def diagonal(self, level, d, stream=None):
        self._c(lib().pmg_diagonal(self.h, level, _dptr(d), _stream(stream)))

    def smooth(self, level, f, u, sweeps=1, precision="fp64", stream=None):
        self._c(lib().pmg_smooth(self.h, level, PRECISIONS[precision], sweeps, _dptr(f), _dptr(u), _stream(stream)))

    def prolong(self, level, xc, yf, precision="fp64", stream=None):
        self._c(lib().pmg_prolong(self.h, level, PRECISIONS[precision], _dptr(xc), _dptr(yf), _stream(stream)))

    def restrict(self, level, xf, yc, precision="fp64", stream=None):
        self._c(lib().pmg_restrict(self.h, level, PRECISIONS[precision], _dptr(xf), _dptr(yc), _stream(stream)))

    def coarse_solve(self, f, u, precision="fp64", stream=None):
        self._c(lib().pmg_coarse_solve(self.h, PRECISIONS[precision], _dptr(f), _dptr(u), _stream(stream)))

    def vcycle(self, r, z, precision="fp64", stream=None):
        self._c(lib().pmg_vcycle(self.h, PRECISIONS[precision], _dptr(r), _dptr(z), _stream(stream)))

    def set_reuse(self, mode="none", stream=None):
        """Operator reuse across surfaces: "none" (strategy III), "t0" (I), "lin" (II)."""
        self._c(lib().pmg_set_reuse(self.h, {"none": 0, "t0": 1, "lin": 2}[mode], _stream(stream)))

    def set_solver(self, precision="fp64", krylov="pcg"):
        self._c(lib().pmg_set_solver(self.h, PRECISIONS[precision], KRYLOV[krylov]))

    def time_kernel(self, kernel, level=0, precision="fp64", reps=20, stream=None) -> float:
        """Average ms per launch of one kernel, timed with hipEvents on the stream."""
        ms = C.c_double()
        self._c(lib().pmg_time_kernel(self.h, KERNELS[kernel], level, PRECISIONS[precision], reps,
                                      C.byref(ms), _stream(stream)))
        return ms.value

    @property
    def net_level(self) -> int:
        """Level whose nodes carry the learned correction (features have its n_dof rows)."""
        return self._c(lib().pmg_net_level(self.h))

    def features(self, surf, p1, p2, X, pnow=None, T=None, p3=None, stream=None):
        self._c(lib().pmg_features(self.h, _dptr(surf), _dptr(p1), _dptr(p2), _dptr(p3), _dptr(pnow), _dptr(X),
                                   _dptr(T), _stream(stream)))

    def solve(self, phi, phi_surf=None, phi_bc=None, guess="zero", rtol=1e-8, atol=0.0, imax=500,
              net=None, hist=None, stream=None):
        """Solve in place into ``phi``; returns (status, stats dict)."""
        import torch
        gm = {"given": PMG_GUESS_GIVEN, "zero": PMG_GUESS_ZERO, "learned": PMG_GUESS_LEARNED,
              "extrap": PMG_GUESS_EXTRAP, "extrap3": PMG_GUESS_EXTRAP3, "learned3": PMG_GUESS_LEARNED3}[guess]
        st = Stats()
        hp = None
        if hist is not None:
            arr = (C.c_void_p * len(hist))(*[t.data_ptr() for t in hist])
            self._keep.append(arr)
            hp = C.cast(arr, C.c_void_p)
        rc = lib().pmg_solve(self.h, _dptr(phi_surf, torch.float64), _dptr(phi_bc, torch.float64),
                             _dptr(phi, torch.float64), gm, net.h if net is not None else None, hp,
                             float(rtol), float(atol), int(imax), C.byref(st), _stream(stream))
        self._c(rc)
        return rc, st.as_dict()


    # ---- free-surface time stepping
    def surface_grad(self, f, stream=None):
        """(f_x, f_y) of a surface field (device FP64 tensors)."""
        import torch
        fx = torch.empty_like(f)
        fy = torch.empty_like(f)
        self._c(lib().pmg_surface_grad(self.h, _dptr(f, torch.float64), _dptr(fx), _dptr(fy), _stream(stream)))
        return fx, fy

    def surface_w(self, phi, stream=None):
        """w~ = d phi / dz at the surface nodes under the current surface."""
        import torch
        w = torch.empty(self.levels[0]["n_surface"], dtype=torch.float64, device=phi.device)
        self._c(lib().pmg_surface_w(self.h, _dptr(phi, torch.float64), _dptr(w), _stream(stream)))
        return w

    def fnpf_rhs(self, eta, phis, phi, g=9.81, warm=False, rtol=1e-10, atol=0.0, imax=500, stream=None):
        """(eta_t, phi~_t, status, stats) at the state (eta, phi~); phi receives the Laplace solution."""
        import torch
        deta = torch.empty_like(eta)
        dphis = torch.empty_like(phis)
        st = Stats()
        rc = lib().pmg_fnpf_rhs(self.h, _dptr(eta, torch.float64), _dptr(phis, torch.float64), float(g),
                                _dptr(phi, torch.float64), int(bool(warm)), float(rtol), float(atol), int(imax),
                                _dptr(deta), _dptr(dphis), C.byref(st), _stream(stream))
        self._c(rc)
        return deta, dphis, rc, st.as_dict()

    def fnpf_erk4(self, eta, phis, phi, dt, g=9.81, warm=True, rtol=1e-8, atol=0.0, imax=500, stream=None):
        """One ERK4 step of (eta, phi~) in place; returns (status, stats dict)."""
        import torch
        st = FnpfStats()
        rc = lib().pmg_fnpf_erk4(self.h, _dptr(eta, torch.float64), _dptr(phis, torch.float64), float(dt), float(g),
                                 _dptr(phi, torch.float64), int(bool(warm)), float(rtol), float(atol), int(imax),
                                 C.byref(st), _stream(stream))
        self._c(rc)
        return rc, st.as_dict()


class Net:
    """Owner of one ``pmg_net`` (the warm-start network of a context's GPU)."""

    def __init__(self, ctx: Context, width: int = 160, depth: int = 3, seed: int = 0):
        h = C.c_void_p()
        _check(lib().pmg_net_create(ctx.h, width, depth, seed, C.byref(h)))
        self.h = h
        np_, din = C.c_int64(), C.c_int32()
        lib().pmg_net_size(h, C.byref(np_), C.byref(din), None, None)
        self.n_params, self.d_in, self.width, self.depth = np_.value, din.value, width, depth

    def close(self):
        if getattr(self, "h", None):
            lib().pmg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc):
        return _check(rc)

    def get_params(self):
        th = np.empty(self.n_params, np.float32)
        mean = np.empty(self.d_in, np.float32)
        istd = np.empty(self.d_in, np.float32)
        ts = C.c_double()
        self._c(lib().pmg_net_get_params(self.h, th.ctypes.data_as(C.c_void_p), mean.ctypes.data_as(C.c_void_p),
                                         istd.ctypes.data_as(C.c_void_p), C.byref(ts)))
        return th, mean, istd, ts.value

    def set_params(self, theta=None, mean=None, inv_std=None, tscale=0.0):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (theta, mean, inv_std)]
        ptr = [None if a is None else a.ctypes.data_as(C.c_void_p) for a in arrs]
        self._c(lib().pmg_net_set_params(self.h, *ptr, float(tscale)))

    def forward(self, X, y, stream=None):
        self._c(lib().pmg_net_forward(self.h, _dptr(X), X.shape[0], _dptr(y), _stream(stream)))

    def forward_noalloc(self, X, y, stream=None):
        self._c(lib().pmg_net_forward_noalloc(self.h, _dptr(X), X.shape[0], _dptr(y), _stream(stream)))

    def loss_grad(self, X, T, stream=None):
        g = np.empty(self.n_params, np.float32)
        loss = C.c_double()
        self._c(lib().pmg_net_loss_grad(self.h, _dptr(X), _dptr(T), X.shape[0], C.byref(loss),
                                        g.ctypes.data_as(C.c_void_p), _stream(stream)))
        return loss.value, g

    def adam_step(self, lr, stream=None):
        self._c(lib().pmg_net_adam_step(self.h, float(lr), _stream(stream)))

    def train(self, X, T, steps=2000, batch=4096, lr=1e-3, seed=7, stream=None):
        fl = C.c_double()
        self._c(lib().pmg_net_train(self.h, _dptr(X), _dptr(T), X.shape[0], steps, batch, float(lr), seed,
                                    C.byref(fl), _stream(stream)))
        return fl.value

    def save(self, path):
        self._c(lib().pmg_net_save(self.h, str(path).encode()))

    def load(self, path):
        self._c(lib().pmg_net_load(self.h, str(path).encode()))
