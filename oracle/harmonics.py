"""Harmonic recurrence, harmonic loop and synthesis (oracle, test infra only).

Eq. laguerre_h of the paper gives, for every harmonic ``m``, an elliptic
problem with one fixed operator and a right-hand side that depends on all
earlier harmonics.  In the SPD sign convention (both sides times -1) and the
2D Cartesian reading (no ``1/(2 pi r)`` factor, a discrete delta ``1/(dx dz)``
at the source node)::

    A R_m = phi_m,
    phi_m = delta_h f_m e_src - h^2 rho * n_m sum_{k<m} (m-k) R_k / n_k,

with ``n_m = sqrt(m!/(m+alpha)!)`` (so ``sqrt((k+alpha)!/k!) = 1/n_k``).

Two equivalent ways to form the sum are provided:

* :func:`rhs_direct` -- the double sum exactly as printed;
* :class:`RunningSums` -- an exact reassociation with two stored fields,
  ``P_m = (n_m/n_{m-1}) P_{m-1} + R_m`` and
  ``Q_{m+1} = (n_{m+1}/n_m)(Q_m + P_m)``, ``Q_0 = 0``, for which
  ``n_m sum_{k<m}(m-k) R_k/n_k = Q_m``.

Synthesis follows eq. series_lag: ``u(t) = sum_m W_m(t) R_m``.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import laguerre


def source_field(shape: Tuple[int, int], src_ij: Sequence[int], value: float,
                 dx: float, dz: float) -> np.ndarray:
    """``value / (dx dz)`` at node ``(i, j)`` (interior index ``(j-1, i-1)``)."""
    out = np.zeros(shape)
    i, j = int(src_ij[0]), int(src_ij[1])
    out[j - 1, i - 1] = value / (dx * dz)
    return out


def rhs_direct(m: int, R: List[np.ndarray], rho_int: np.ndarray, h: float, alpha: int,
               src: np.ndarray) -> np.ndarray:
    """``phi_m`` by the double sum of eq. laguerre_h.

    ``src`` is ``delta_h f_m e_src``; ``R`` holds ``R_0..R_{m-1}``."""
    if m == 0:
        return src.copy()
    ln = laguerre.log_norm(np.arange(m + 1), alpha)
    acc = np.zeros_like(src)
    for k in range(m):
        acc += (m - k) * math.exp(ln[m] - ln[k]) * R[k]
    return src - h * h * rho_int * acc


class RunningSums:
    """Running form of the recurrence sum (exact reassociation).

    ``step(m, R_prev)`` must be called for m = 0, 1, 2, ... with
    ``R_prev = R_{m-1}`` (ignored for m = 0) and returns ``Q_m``.
    """

    def __init__(self, shape, alpha: int):
        self.alpha = alpha
        self.P = np.zeros(shape)        # P_{m-1} after step(m)
        self.Q = np.zeros(shape)        # Q_m after step(m)

    def step(self, m: int, R_prev: Optional[np.ndarray]) -> np.ndarray:
        if m == 0:
            self.P[...] = 0.0
            self.Q[...] = 0.0
            return self.Q
        a = self.alpha
        # P_{m-1} = (n_{m-1}/n_{m-2}) P_{m-2} + R_{m-1}   (P_{-1} = 0)
        ratio_p = math.sqrt((m - 1) / (m - 1 + a)) if m >= 2 else 0.0
        self.P = ratio_p * self.P + R_prev
        # Q_m = (n_m/n_{m-1}) (Q_{m-1} + P_{m-1})
        self.Q = math.sqrt(m / (m + a)) * (self.Q + self.P)
        return self.Q


def rhs_running(m: int, sums: RunningSums, R_prev: Optional[np.ndarray], rho_int: np.ndarray,
                h: float, src: np.ndarray) -> np.ndarray:
    """``phi_m = src - h^2 rho Q_m`` using :class:`RunningSums`."""
    Q = sums.step(m, R_prev)
    return src - h * h * rho_int * Q


def harmonic_loop(n_harm: int, solve: Callable[[np.ndarray], Tuple[np.ndarray, int, float, int]],
                  rho_int: np.ndarray, h: float, alpha: int, f_m: np.ndarray,
                  src_ij: Sequence[int], dx: float, dz: float,
                  snap_w: Optional[np.ndarray] = None, rec_row: Optional[int] = None,
                  direct: bool = False, m_start: int = 0,
                  state: Optional[Dict] = None, keep_all: bool = True) -> Dict:
    """Run harmonics ``m_start .. n_harm-1`` of the acoustic problem.

    ``solve(phi) -> (R, iters, relres, status)`` inverts A.  ``snap_w`` is
    ``[n_snap, n_harm]`` synthesis weights.  Returns a dict with the list of
    ``R_m``, per-harmonic iteration counts, snapshots ``[n_snap, ...]`` and the
    receiver-row coefficients ``[n_harm, Nx-1]``; ``state`` resumes a run.
    With ``keep_all=False`` only the latest ``R`` is kept (large grids).
    """
    shape = rho_int.shape
    if state is None:
        state = {
            "R": [], "R_prev": None, "iters": [], "relres": [], "status": [],
            "sums": RunningSums(shape, alpha),
            "snap": None if snap_w is None else np.zeros((snap_w.shape[0],) + shape),
            "rec": [] if rec_row is not None else None,
        }
    for m in range(m_start, n_harm):
        src = source_field(shape, src_ij, f_m[m], dx, dz)
        if direct:
            phi = rhs_direct(m, state["R"], rho_int, h, alpha, src)
            state["sums"].step(m, state["R_prev"] if m else None)
        else:
            phi = rhs_running(m, state["sums"], state["R_prev"] if m else None, rho_int, h, src)
        R, it, rr, st = solve(phi)
        state["R_prev"] = R
        if keep_all or direct:
            state["R"].append(R)
        state["iters"].append(it)
        state["relres"].append(rr)
        state["status"].append(st)
        if snap_w is not None:
            state["snap"] += snap_w[:, m][:, None, None] * R[None]
        if rec_row is not None:
            state["rec"].append(R[rec_row - 1].copy())
    return state


def traces(rec: np.ndarray, W: np.ndarray) -> np.ndarray:
    """``u(x_r, t_l) = sum_m W_m(t_l) R_m(x_r)``: ``[nt, n] @ [n, Nx-1]``."""
    return W @ rec
