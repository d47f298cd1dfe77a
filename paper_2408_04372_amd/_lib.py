"""ctypes binding of libstmg.so (argument marshalling only; all work runs in the library).

Vectors are torch tensors on the GPU (contiguous float64 or float32, shape
[n_t, N_x] or flat); the handle's stream is the torch stream current at
creation unless one is given.  The library must be built
(``python -m paper_2408_04372_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstmg.so")
ABI_VERSION = 4
MAX_LEVELS = 16

STATUS = {0: "OK", 1: "E_ARG", 2: "E_NOMEM", 3: "E_HIP", 4: "E_NOCONV", 5: "E_NONFINITE",
          6: "E_UNSUPPORTED", 7: "E_STATE"}


class StmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stmg {STATUS.get(code, code)}: {msg}")
        self.code = code


class CConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dim", ctypes.c_int32), ("problem", ctypes.c_int32),
        ("time_method", ctypes.c_int32), ("p", ctypes.c_int32), ("k", ctypes.c_int32),
        ("n_time_cells", ctypes.c_int32), ("n_cells", ctypes.c_int32 * 3),
        ("t0", ctypes.c_double), ("tau", ctypes.c_double),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("n_smooth", ctypes.c_int32), ("min_p", ctypes.c_int32), ("coarse_cells", ctypes.c_int32),
        ("vcycle_dtypes", ctypes.c_int32), ("omega", ctypes.c_double),
        ("precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("gram_schmidt", ctypes.c_int32), ("rtol", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("asm_variant", ctypes.c_int32), ("time_mg", ctypes.c_int32), ("kernel_path", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
        ("t_smoother", ctypes.c_double), ("t_gmg_other", ctypes.c_double),
        ("t_operator", ctypes.c_double), ("t_other", ctypes.c_double),
        ("cnn_used", ctypes.c_int32), ("cnn_fallbacks", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32), ("n_t", ctypes.c_int32), ("nt_cell", ctypes.c_int32),
        ("temporal_nnz", ctypes.c_int32),
        ("n_x", ctypes.c_int64 * MAX_LEVELS), ("p", ctypes.c_int32 * MAX_LEVELS),
        ("cells", (ctypes.c_int32 * 3) * MAX_LEVELS), ("omega", ctypes.c_double * MAX_LEVELS),
        ("coarse_unknowns", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
        ("setup_seconds", ctypes.c_double),
        ("n_t_level", ctypes.c_int32 * MAX_LEVELS), ("nt_cell_level", ctypes.c_int32 * MAX_LEVELS),
        ("eig_resolves", ctypes.c_int32),
    ]


class KernelStats(ctypes.Structure):
    _fields_ = [("n_operator", ctypes.c_int64), ("n_smoother", ctypes.c_int64),
                ("t_operator", ctypes.c_double), ("t_smoother", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None

# exported symbols and their argument types
_SIGS = {
    "stmg_create": ([ctypes.POINTER(CConfig), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "stmg_vmult": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "stmg_vmult_noalloc": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
                           ctypes.c_int),
    "stmg_smooth": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_int], ctypes.c_int),
    "stmg_vcycle": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "stmg_prolongate": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
                        ctypes.c_int),
    "stmg_restrict": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
                      ctypes.c_int),
    "stmg_solve": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SolveInfo)],
                   ctypes.c_int),
    "stmg_set_omega": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double], ctypes.c_int),
    "stmg_set_precision": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "stmg_kernel_stats_get": ([ctypes.c_void_p, ctypes.POINTER(KernelStats), ctypes.c_int], ctypes.c_int),
    "stmg_query": ([ctypes.c_void_p, ctypes.POINTER(Info)], ctypes.c_int),
    "stmg_cnn_create": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "stmg_cnn_param_count": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "stmg_cnn_set_params": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "stmg_cnn_get_params": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "stmg_cnn_forward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "stmg_wave_velocity": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "stmg_slab_rhs": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p], ctypes.c_int),
    "stmg_node_coordinates": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "stmg_point_values": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                           ctypes.c_void_p], ctypes.c_int),
    "stmg_cnn_param_grad": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64],
                            ctypes.c_int),
    "stmg_cnn_train_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "stmg_destroy": ([ctypes.c_void_p], None),
    "stmg_last_error": ([], ctypes.c_char_p),
    "stmg_temporal_matrices": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p], ctypes.c_int),
    "stmg_temporal_cell_factors": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "stmg_transfer_1d": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p],
                         ctypes.c_int),
    "stmg_temporal_dof_times": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p],
                                ctypes.c_int),
    "stmg_mg_step": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                     ctypes.c_int),
    "stmg_temporal_prolongation": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p], ctypes.c_int),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libstmg.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2408_04372_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(code: int):
    if code != 0:
        msg = load().stmg_last_error().decode(errors="replace")
        raise StmgError(code, msg)


def temporal_matrices(problem: int, method: int, k: int, n_time_cells: int, tau: float):
    """(M_T, A_T, N_T) as the library builds them (host only; numpy arrays, n_t x n_t)."""
    import numpy as np
    lib = load()
    n = ctypes.c_int32()
    _check(lib.stmg_temporal_matrices(problem, method, k, n_time_cells, tau, 0, ctypes.byref(n), None, None, None))
    out = [np.empty((n.value, n.value)) for _ in range(3)]
    _check(lib.stmg_temporal_matrices(problem, method, k, n_time_cells, tau, n.value * n.value, ctypes.byref(n),
                                      *[ctypes.c_void_p(a.ctypes.data) for a in out]))
    return tuple(out)


def temporal_cell_factors(problem: int, method: int, k: int, tau: float):
    """(M_tau, N_tilde) of the smoother's local blocks as the library builds them (host only)."""
    import numpy as np
    lib = load()
    n = ctypes.c_int32()
    _check(lib.stmg_temporal_cell_factors(problem, method, k, tau, 0, ctypes.byref(n), None, None))
    out = [np.empty((n.value, n.value)) for _ in range(2)]
    _check(lib.stmg_temporal_cell_factors(problem, method, k, tau, n.value * n.value, ctypes.byref(n),
                                          *[ctypes.c_void_p(a.ctypes.data) for a in out]))
    return tuple(out)


def temporal_dof_times(problem: int, method: int, k: int, n_time_cells: int, tau: float, t0: float = 0.0):
    """Times of a slab's temporal DoFs as the library places them (host only; numpy array)."""
    import numpy as np
    lib = load()
    n = ctypes.c_int32()
    _check(lib.stmg_temporal_dof_times(problem, method, k, n_time_cells, tau, t0, 0, ctypes.byref(n), None))
    out = np.empty(n.value)
    _check(lib.stmg_temporal_dof_times(problem, method, k, n_time_cells, tau, t0, n.value, ctypes.byref(n),
                                       ctypes.c_void_p(out.ctypes.data)))
    return out


def transfer_1d(p_coarse: int, n_coarse: int, p_fine: int, n_fine: int):
    """1D factor of the spatial prolongation (Dirichlet end rows and columns zero; host only)."""
    import numpy as np
    lib = load()
    r, c = ctypes.c_int32(), ctypes.c_int32()
    args = (p_coarse, n_coarse, p_fine, n_fine)
    _check(lib.stmg_transfer_1d(*args, 0, ctypes.byref(r), ctypes.byref(c), None))
    P = np.empty((r.value, c.value))
    _check(lib.stmg_transfer_1d(*args, P.size, ctypes.byref(r), ctypes.byref(c), ctypes.c_void_p(P.ctypes.data)))
    return P


def temporal_prolongation(problem: int, method: int, k_fine: int, c_fine: int, k_coarse: int, c_coarse: int,
                          slab_length: float):
    """Temporal prolongation fine n_t x coarse n_t as the library builds it (host only)."""
    import numpy as np
    lib = load()
    r, c = ctypes.c_int32(), ctypes.c_int32()
    args = (problem, method, k_fine, c_fine, k_coarse, c_coarse, slab_length)
    _check(lib.stmg_temporal_prolongation(*args, 0, ctypes.byref(r), ctypes.byref(c), None))
    P = np.empty((r.value, c.value))
    _check(lib.stmg_temporal_prolongation(*args, P.size, ctypes.byref(r), ctypes.byref(c),
                                          ctypes.c_void_p(P.ctypes.data)))
    return P


def c_config(cfg, **overrides) -> CConfig:
    """stmg_config from an object with the stmg_inputs.Config attributes (plus overrides)."""
    get = lambda k: overrides.get(k, getattr(cfg, k))
    c = CConfig()
    c.abi_version = ABI_VERSION
    for f in ("dim", "problem", "time_method", "p", "k", "n_time_cells", "n_smooth", "min_p",
              "coarse_cells", "precision", "restart", "max_iter"):
        setattr(c, f, int(get(f)))
    nc = list(get("n_cells")) + [1, 1, 1]
    c.n_cells[:] = [int(v) for v in nc[:3]]
    c.t0 = float(get("t0"))
    c.tau = float(get("tau"))
    c.lo[:] = [float(v) for v in (list(get("lo")) + [0, 0, 0])[:3]]
    c.hi[:] = [float(v) for v in (list(get("hi")) + [1, 1, 1])[:3]]
    c.vcycle_dtypes = int(overrides.get("vcycle_dtypes", 0))
    c.gram_schmidt = int(overrides.get("gram_schmidt", 0))
    c.asm_variant = int(overrides.get("asm_variant", getattr(cfg, "asm_variant", 0)))
    c.time_mg = int(overrides.get("time_mg", 0))
    c.kernel_path = int(overrides.get("kernel_path", 0))
    c.omega = float(get("omega"))
    c.rtol = float(get("rtol"))
    c.seed = int(get("seed"))
    return c


def _ptr(t, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError("vectors must be float64 or float32")


class Handle:
    """One stmg_handle: hierarchy + solver for one slab problem."""

    def __init__(self, cfg, vertices: Optional[np.ndarray] = None, coeff: Optional[np.ndarray] = None,
                 stream=None, **overrides):
        import torch
        self.lib = load()
        self.cfg = cfg
        self.ccfg = c_config(cfg, **overrides)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        sp = ctypes.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else ctypes.c_void_p(stream)
        self._v = None if vertices is None else np.ascontiguousarray(vertices, dtype=np.float64)
        self._c = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64)
        vp = None if self._v is None else self._v.ctypes.data_as(ctypes.c_void_p)
        cp = None if self._c is None else self._c.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(self.lib.stmg_create(ctypes.byref(self.ccfg), vp, cp, sp, ctypes.byref(h)))
        self.h = h
        self.info = self.query()

    # -- sizes
    def query(self) -> dict:
        inf = Info()
        _check(self.lib.stmg_query(self.h, ctypes.byref(inf)))
        L = inf.n_levels
        return {"n_levels": L, "n_t": inf.n_t, "nt_cell": inf.nt_cell, "temporal_nnz": inf.temporal_nnz,
                "n_x": [inf.n_x[i] for i in range(L)], "p": [inf.p[i] for i in range(L)],
                "cells": [tuple(inf.cells[i][:]) for i in range(L)],
                "omega": [inf.omega[i] for i in range(L)], "coarse_unknowns": inf.coarse_unknowns,
                "device_bytes": inf.device_bytes, "setup_seconds": inf.setup_seconds,
                "n_t_level": [inf.n_t_level[i] for i in range(L)],
                "nt_cell_level": [inf.nt_cell_level[i] for i in range(L)],
                "eig_resolves": inf.eig_resolves}

    def size(self, level: int = 0) -> int:
        return self.info["n_t_level"][level] * self.info["n_x"][level]

    def _sz(self, t, level):
        if t.numel() != self.size(level):
            raise ValueError(f"vector has {t.numel()} entries, level {level} needs {self.size(level)}")

    # -- operations (asynchronous on the handle's stream)
    def vmult(self, x, y, level: int = 0):
        self._sz(x, level); self._sz(y, level)
        d = _dtype_code(x)
        _check(self.lib.stmg_vmult(self.h, level, d, _ptr(x, x.dtype), _ptr(y, x.dtype)))
        return y

    def vmult_noalloc(self, x, y, level: int = 0):
        self._sz(x, level); self._sz(y, level)
        d = _dtype_code(x)
        _check(self.lib.stmg_vmult_noalloc(self.h, level, d, _ptr(x, x.dtype), _ptr(y, x.dtype)))
        return y

    def smooth(self, b, x, steps: int = 1, level: int = 0):
        self._sz(b, level); self._sz(x, level)
        d = _dtype_code(b)
        _check(self.lib.stmg_smooth(self.h, level, d, _ptr(b, b.dtype), _ptr(x, b.dtype), steps))
        return x

    def vcycle(self, r, z):
        self._sz(r, 0); self._sz(z, 0)
        d = _dtype_code(r)
        _check(self.lib.stmg_vcycle(self.h, d, _ptr(r, r.dtype), _ptr(z, r.dtype)))
        return z

    def mg_step(self, b, x, r, z):
        """x <- x + V(b - S x) on the finest level; r, z receive the residual and the correction."""
        for t in (b, x, r, z):
            self._sz(t, 0)
        d = _dtype_code(x)
        _check(self.lib.stmg_mg_step(self.h, d, _ptr(b, x.dtype), _ptr(x, x.dtype), _ptr(r, x.dtype), _ptr(z, x.dtype)))
        return x

    def prolongate(self, coarse, fine, level: int = 0):
        self._sz(coarse, level + 1); self._sz(fine, level)
        d = _dtype_code(coarse)
        _check(self.lib.stmg_prolongate(self.h, level, d, _ptr(coarse, coarse.dtype), _ptr(fine, coarse.dtype)))
        return fine

    def restrict(self, fine, coarse, level: int = 0):
        self._sz(coarse, level + 1); self._sz(fine, level)
        d = _dtype_code(fine)
        _check(self.lib.stmg_restrict(self.h, level, d, _ptr(fine, fine.dtype), _ptr(coarse, fine.dtype)))
        return coarse

    def solve(self, b, x, raise_on_noconv: bool = True) -> dict:
        import torch
        self._sz(b, 0); self._sz(x, 0)
        inf = SolveInfo()
        code = self.lib.stmg_solve(self.h, _ptr(b, torch.float64), _ptr(x, torch.float64), ctypes.byref(inf))
        out = inf.as_dict()
        out["status"] = STATUS.get(code, code)
        if code != 0 and (raise_on_noconv or code != 4):
            _check(code)
        return out

    def set_precision(self, precision: int):
        _check(self.lib.stmg_set_precision(self.h, int(precision)))

    def kernel_stats(self, reset: bool = False) -> dict:
        ks = KernelStats()
        _check(self.lib.stmg_kernel_stats_get(self.h, ctypes.byref(ks), 1 if reset else 0))
        return ks.as_dict()

    # -- learned stage
    def cnn_create(self, channels):
        arr = (ctypes.c_int32 * len(channels))(*[int(c) for c in channels])
        _check(self.lib.stmg_cnn_create(self.h, len(channels) - 1, arr))
        n = ctypes.c_int64()
        _check(self.lib.stmg_cnn_param_count(self.h, ctypes.byref(n)))
        self.cnn_nparam = n.value
        self.cnn_channels = list(channels)
        return n.value

    def cnn_set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        _check(self.lib.stmg_cnn_set_params(self.h, th.ctypes.data_as(ctypes.c_void_p), th.size))

    def cnn_get_params(self):
        th = np.empty(self.cnn_nparam, dtype=np.float32)
        _check(self.lib.stmg_cnn_get_params(self.h, th.ctypes.data_as(ctypes.c_void_p), th.size))
        return th

    def node_coordinates(self) -> np.ndarray:
        """Finest-level node coordinates, shape (N_x, dim) (Cartesian meshes)."""
        nx = self.info["n_x"][0]
        out = np.empty((nx, self.cfg.dim), dtype=np.float64)
        _check(self.lib.stmg_node_coordinates(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def point_values(self, U, points, n_planes: int = None) -> np.ndarray:
        """Values of the first n_planes temporal planes of U at points (npts, dim): (n_planes, npts)."""
        import torch
        self._sz(U, 0)
        n_planes = self.info["n_t"] if n_planes is None else int(n_planes)
        pts = np.ascontiguousarray(points, dtype=np.float64)
        out = np.empty((n_planes, pts.shape[0]), dtype=np.float64)
        _check(self.lib.stmg_point_values(self.h, _ptr(U, torch.float64), n_planes, pts.shape[0],
                                          pts.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def slab_rhs(self, b, F=None, F0=None, u0=None, v0=None):
        """b = slab right-hand side from loads F [n_t N_x] (and F0 [N_x] for cGP) and the
        initial data u0, v0 [N_x] of the slab (None reads as zero)."""
        import torch
        self._sz(b, 0)
        if F is not None:
            self._sz(F, 0)
        nx = self.info["n_x"][0]
        for t in (F0, u0, v0):
            if t is not None and (t.numel() != nx or t.dtype != torch.float64 or not t.is_contiguous()):
                raise ValueError(f"plane data must be contiguous float64 with {nx} entries")
        ptr = lambda t: _ptr(t, torch.float64) if t is not None else None
        _check(self.lib.stmg_slab_rhs(self.h, ptr(F), ptr(F0), ptr(u0), ptr(v0), _ptr(b, torch.float64)))
        return b

    def wave_velocity(self, U, V, u0=None, v0=None):
        """V = velocity of the wave slab from displacement U (u0, v0: initial data or None)."""
        import torch
        self._sz(U, 0); self._sz(V, 0)
        nx = self.info["n_x"][0]
        for t in (u0, v0):
            if t is not None and (t.numel() != nx or t.dtype != torch.float64 or not t.is_contiguous()):
                raise ValueError(f"initial data must be contiguous float64 with {nx} entries")
        p0 = _ptr(u0, torch.float64) if u0 is not None else None
        p1 = _ptr(v0, torch.float64) if v0 is not None else None
        _check(self.lib.stmg_wave_velocity(self.h, _ptr(U, torch.float64), p0, p1, _ptr(V, torch.float64)))
        return V

    def cnn_forward(self, r, z):
        import torch
        self._sz(r, 0); self._sz(z, 0)
        _check(self.lib.stmg_cnn_forward(self.h, _ptr(r, torch.float64), _ptr(z, torch.float64)))
        return z

    def cnn_param_grad(self, r, dz):
        import torch
        g = np.empty(self.cnn_nparam, dtype=np.float32)
        _check(self.lib.stmg_cnn_param_grad(self.h, _ptr(r, torch.float64), _ptr(dz, torch.float64),
                                            g.ctypes.data_as(ctypes.c_void_p), g.size))
        return g

    def cnn_train_step(self, r, e, lr: float) -> float:
        import torch
        loss = ctypes.c_double()
        _check(self.lib.stmg_cnn_train_step(self.h, _ptr(r, torch.float64), _ptr(e, torch.float64), float(lr),
                                            ctypes.byref(loss)))
        return loss.value

    def set_omega(self, level: int, omega: float):
        _check(self.lib.stmg_set_omega(self.h, level, float(omega)))
        self.info = self.query()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.stmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
