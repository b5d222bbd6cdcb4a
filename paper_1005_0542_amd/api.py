"""Python binding of the C ABI: argument marshalling only.

Every step of the hot path runs in the HIP kernels of ``liblaguerre.so``;
PyTorch supplies device memory (``torch.Tensor.data_ptr()``) and the HIP
stream (``torch.cuda.current_stream()``).  Names follow the C calls.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import check

__all__ = ["Plan", "source_coeffs", "laguerre_weights", "SolveResult"]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def source_coeffs(f0: float, t0: float, alpha: int, h: float, n: int, wavelet: str = "ricker",
                  gamma: float = 4.0) -> np.ndarray:
    """``f_m`` of the source wavelet (host computation in the library)."""
    lib = _lib.load()
    out = np.zeros(n)
    lag = _lib.Laguerre(alpha, h, n)
    wv = _lib.LG_RICKER if wavelet == "ricker" else _lib.LG_GAUSS_SINE
    check(lib.lg_source_coeffs(wv, f0, t0, gamma, ctypes.byref(lag), _dptr(out)), "lg_source_coeffs")
    return out


def laguerre_weights(t: Sequence[float], alpha: int, h: float, n: int) -> np.ndarray:
    """Synthesis weights ``W[q, m]`` (host computation in the library)."""
    lib = _lib.load()
    tt = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    out = np.zeros((len(tt), n))
    lag = _lib.Laguerre(alpha, h, n)
    check(lib.lg_laguerre_weights(ctypes.byref(lag), _dptr(tt), len(tt), _dptr(out)), "lg_laguerre_weights")
    return out


class SolveResult:
    def __init__(self, status: int, infos: List[_lib.SolveInfo]):
        self.status = status
        self.iters = [int(i.iters) for i in infos]
        self.statuses = [int(i.status) for i in infos]
        self.relres = [float(i.relres) for i in infos]

    def __repr__(self):
        return f"SolveResult(status={self.status}, iters={self.iters}, relres={self.relres})"


class Plan:
    """An ``lg_plan``: one medium, ``nshots`` shots, one precision."""

    def __init__(self, kind: str, nx: int, nz: int, dx: float, dz: float, alpha: int, h: float,
                 n: int, medium: np.ndarray, precision: str = "fp64", nshots: int = 1,
                 segments: int = 0, graph_iters: int = 0, op_shots: int = 0, seg_per_wave: int = 0,
                 op_fusion: int = 0, top: str = "dirichlet", geometry: str = "cartesian",
                 order: int = 2, x_ring: int = 0, stream=None):
        import torch
        self.lib = _lib.load()
        self.kind = kind
        self.nx, self.nz, self.nshots = nx, nz, nshots
        self.ncomp = 1 if kind == "acoustic" else 2
        self.precision = precision
        self.wdtype = torch.float64 if precision == "fp64" else torch.float32
        med = np.ascontiguousarray(np.asarray(medium, dtype=np.float64))
        if top not in ("dirichlet", "free"):
            raise ValueError("top must be 'dirichlet' or 'free'")
        self.top = top
        if geometry not in ("cartesian", "cylindrical"):
            raise ValueError("geometry must be 'cartesian' or 'cylindrical'")
        self.geometry = geometry
        self.order = order
        grid = _lib.Grid(nx, nz, dx, dz, _lib.LG_TOP_FREE if top == "free" else _lib.LG_TOP_DIRICHLET,
                         _lib.LG_CYLINDRICAL if geometry == "cylindrical" else _lib.LG_CARTESIAN, order, 0)
        lag = _lib.Laguerre(alpha, h, n)
        tun = _lib.Tuning(segments, graph_iters, op_shots, seg_per_wave, op_fusion, x_ring)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        st = self.lib.lg_plan_create(
            ctypes.byref(handle), _lib.LG_ACOUSTIC if kind == "acoustic" else _lib.LG_ELASTIC,
            ctypes.byref(grid), ctypes.byref(lag),
            _lib.LG_FP64 if precision == "fp64" else _lib.LG_MIXED, nshots, _dptr(med),
            ctypes.byref(tun), ctypes.c_void_p(stream.cuda_stream))
        check(st, "lg_plan_create")
        self.handle = handle
        self._medium = med

    # -- helpers --------------------------------------------------------------
    def vec_shape(self, comps: Optional[int] = None):
        c = self.ncomp if comps is None else comps
        if self.geometry == "cylindrical":          # [Nr-1][Nz], z fastest
            return (self.nshots, c, self.nz - 1, self.nx)
        return (self.nshots, c, self.nz - 1, self.nx - 1)

    def _ptr(self, t, dtype, name, numel=None):
        if t is None:
            return None
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
            raise ValueError(f"{name}: need a contiguous CUDA tensor of dtype {dtype}")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    def _nvec(self, comps=None):
        s = self.vec_shape(comps)
        return s[0] * s[1] * s[2] * s[3]

    def layout(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.lg_plan_layout(self.handle, ctypes.byref(a), ctypes.byref(b)), "lg_plan_layout")
        return a.value, b.value

    def x_ring(self) -> int:
        a = ctypes.c_int32()
        check(self.lib.lg_plan_x_ring(self.handle, ctypes.byref(a)), "lg_plan_x_ring")
        return a.value

    def set_sources(self, src_ij: np.ndarray):
        s = np.ascontiguousarray(np.asarray(src_ij, dtype=np.int32).reshape(self.nshots, 2))
        check(self.lib.lg_plan_set_sources(self.handle, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "lg_plan_set_sources")

    # -- the hot path ---------------------------------------------------------
    def laguerre_rhs(self, m: int, R_prev, Phat, Qhat, fsrc: Sequence[float], rhs):
        import torch
        n = self._nvec()
        f = np.ascontiguousarray(np.asarray(fsrc, dtype=np.float64).reshape(self.nshots))
        check(self.lib.lg_laguerre_rhs(self.handle, m, self._ptr(R_prev, torch.float64, "R_prev", n),
                                       self._ptr(Phat, torch.float64, "Phat", n),
                                       self._ptr(Qhat, torch.float64, "Qhat", n), _dptr(f),
                                       self._ptr(rhs, torch.float64, "rhs", n)), "lg_laguerre_rhs")

    def stencil_apply(self, x, y):
        n = self._nvec()
        check(self.lib.lg_stencil_apply(self.handle, self._ptr(x, self.wdtype, "x", n),
                                        self._ptr(y, self.wdtype, "y", n)), "lg_stencil_apply")

    def precond_dst(self, inverse: bool, x, y):
        n = self._nvec()
        check(self.lib.lg_precond_dst(self.handle, int(bool(inverse)), self._ptr(x, self.wdtype, "in", n),
                                      self._ptr(y, self.wdtype, "out", n)), "lg_precond_dst")

    def precond_dichotomy_tdma(self, block: int, rhs_hat, sol_hat):
        n = self._nvec(1)
        check(self.lib.lg_precond_dichotomy_tdma(self.handle, block,
                                                 self._ptr(rhs_hat, self.wdtype, "rhs_hat", n),
                                                 self._ptr(sol_hat, self.wdtype, "sol_hat", n)),
              "lg_precond_dichotomy_tdma")

    def precond_apply(self, r, z):
        n = self._nvec()
        check(self.lib.lg_precond_apply(self.handle, self._ptr(r, self.wdtype, "r", n),
                                        self._ptr(z, self.wdtype, "z", n)), "lg_precond_apply")

    def _solve(self, fn, name, b, x, tol, max_iter, restart, x0_given=False):
        import torch
        n = self._nvec()
        opts = _lib.SolveOpts(tol, max_iter, restart, 1 if x0_given else 0, 0)
        infos = (_lib.SolveInfo * self.nshots)()
        st = fn(self.handle, self._ptr(b, torch.float64, "b", n), self._ptr(x, torch.float64, "x", n),
                ctypes.byref(opts), infos)
        check(st, name, allowed=(_lib.LG_OK, _lib.LG_ERR_NOT_CONVERGED, _lib.LG_ERR_BREAKDOWN,
                                 _lib.LG_ERR_NONFINITE))
        return SolveResult(st, list(infos))

    def pcg_solve(self, b, x, tol: float = 1e-10, max_iter: int = 10000, x0_given: bool = False) -> SolveResult:
        """x0_given: start from the values in x (otherwise from 0)."""
        return self._solve(self.lib.lg_pcg_solve, "lg_pcg_solve", b, x, tol, max_iter, 1, x0_given)

    def gmres_solve(self, b, x, tol: float = 1e-10, max_iter: int = 10000, restart: int = 10) -> SolveResult:
        return self._solve(self.lib.lg_gmres_solve, "lg_gmres_solve", b, x, tol, max_iter, restart)

    def pcg_profile(self, b, x, iters: int = 10) -> List[float]:
        """Average duration (ms) of the five kernels of one CG iteration."""
        import torch
        n = self._nvec()
        ms = (ctypes.c_float * 5)()
        check(self.lib.lg_pcg_profile(self.handle, self._ptr(b, torch.float64, "b", n),
                                      self._ptr(x, torch.float64, "x", n), iters, ms), "lg_pcg_profile")
        return [float(v) for v in ms]

    def laguerre_synthesize(self, m: int, R, W_snap: Sequence[float], snap, rec_row: int = 1, rec=None):
        import torch
        w = np.ascontiguousarray(np.asarray(W_snap, dtype=np.float64))
        n = self._nvec()
        check(self.lib.lg_laguerre_synthesize(
            self.handle, m, self._ptr(R, torch.float64, "R", n), _dptr(w) if len(w) else None, len(w),
            self._ptr(snap, torch.float64, "snap", len(w) * n) if len(w) else None, rec_row,
            self._ptr(rec, torch.float64, "rec")), "lg_laguerre_synthesize")

    def laguerre_synthesize_batch(self, m0: int, Rs: Sequence, W_snap: np.ndarray, snap, rec_row: int = 1,
                                  rec=None):
        """Harmonics m0 .. m0+len(Rs)-1 in one pass; W_snap: [n_snap][len(Rs)]."""
        import torch
        nb = len(Rs)
        w = np.ascontiguousarray(np.asarray(W_snap, dtype=np.float64).reshape(-1, nb))
        ns = w.shape[0]
        n = self._nvec()
        ptrs = (ctypes.c_void_p * nb)(*[self._ptr(R, torch.float64, "R", n) for R in Rs])
        check(self.lib.lg_laguerre_synthesize_batch(
            self.handle, m0, nb, ptrs, _dptr(w) if ns else None, ns,
            self._ptr(snap, torch.float64, "snap", ns * n) if ns else None, rec_row,
            self._ptr(rec, torch.float64, "rec")), "lg_laguerre_synthesize_batch")

    def trace_synthesize(self, rec, W: np.ndarray, traces):
        import torch
        Wc = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
        check(self.lib.lg_trace_synthesize(self.handle, self._ptr(rec, torch.float64, "rec"), _dptr(Wc),
                                           Wc.shape[0], self._ptr(traces, torch.float64, "traces")),
              "lg_trace_synthesize")

    def destroy(self):
        if getattr(self, "handle", None):
            self.lib.lg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
