"""Textbook Krylov solvers (oracle, test infrastructure only).

Sec. 2.3: the acoustic system ``A y = f`` (A = A* > 0) is solved by the
conjugate gradient method and the elastic system ``C y = f`` by restarted
GMRES(k), both as given in Saad, *Iterative Methods for Sparse Linear
Systems* (preconditioned CG, Alg. 9.1; right-preconditioned GMRES with
modified Gram-Schmidt Arnoldi and Givens rotations, Alg. 6.9 / 9.5).

Conventions (readings where the paper is silent): the initial guess is 0,
and the stopping test is on the unpreconditioned residual,
``||r||_2 <= tol ||b||_2``.  A zero right-hand side returns 0 after 0
iterations.
"""
from __future__ import annotations

import math
from typing import Callable, Tuple

import numpy as np

from . import OK, NOT_CONVERGED, BREAKDOWN, NONFINITE

Op = Callable[[np.ndarray], np.ndarray]


def _dot(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.dot(a.ravel(), b.ravel()))


def pcg(apply_A: Op, apply_Minv: Op, b: np.ndarray, tol: float,
        max_iter: int, x0: np.ndarray = None) -> Tuple[np.ndarray, int, float, int]:
    """Preconditioned CG from ``x0`` (default 0).  Returns ``(x, iters, relres, status)``.

    ``iters`` counts operator applications; the residual is updated
    recursively (``r -= alpha A p``) and tested right after each update.  A
    given ``x0`` starts from ``r = b - A x0``, which is tested first (0
    iterations when it already meets the tolerance); ``b = 0`` gives ``x = 0``.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = math.sqrt(_dot(b, b))
    if not math.isfinite(bnorm):
        return x, 0, float("nan"), NONFINITE
    if bnorm == 0.0:
        return x, 0, 0.0, OK
    if x0 is None:
        r = b.copy()
        rnorm = bnorm
    else:
        x = np.array(x0, dtype=np.float64)
        r = b - apply_A(x)
        rnorm = math.sqrt(_dot(r, r))
        if not math.isfinite(rnorm):
            return x, 0, float("nan"), NONFINITE
        if rnorm <= tol * bnorm:
            return x, 0, rnorm / bnorm, OK
    z = apply_Minv(r)
    p = z.copy()
    rz = _dot(r, z)
    for it in range(1, max_iter + 1):
        q = apply_A(p)
        pq = _dot(p, q)
        if not math.isfinite(pq):
            return x, it - 1, rnorm / bnorm, NONFINITE
        if pq <= 0.0:
            return x, it - 1, rnorm / bnorm, BREAKDOWN
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        rnorm = math.sqrt(_dot(r, r))
        if not math.isfinite(rnorm):
            return x, it, float("nan"), NONFINITE
        if rnorm <= tol * bnorm:
            return x, it, rnorm / bnorm, OK
        if it == max_iter:
            break
        z = apply_Minv(r)
        rz_new = _dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, max_iter, rnorm / bnorm, NOT_CONVERGED


def gmres(apply_A: Op, apply_Minv: Op, b: np.ndarray, tol: float, restart: int,
          max_cycles: int = 200, max_iter: int = None) -> Tuple[np.ndarray, int, float, int]:
    """Right-preconditioned restarted GMRES(k) from ``x0 = 0``.

    Inner iterations use the Givens estimate ``|g_{j+1}|`` of the residual
    norm; each restart recomputes the true residual ``b - A x``.  Returns
    ``(x, inner_iterations, relres_estimate, status)``.  ``max_iter``, if
    given, caps the total number of inner iterations: the cycle in progress
    then ends with its update of x and the status is NOT_CONVERGED (with
    ``tol = 0`` this runs exactly ``max_iter`` iterations).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = math.sqrt(_dot(b, b))
    if not math.isfinite(bnorm):
        return x, 0, float("nan"), NONFINITE
    if bnorm == 0.0:
        return x, 0, 0.0, OK
    k = restart
    total = 0
    est = 1.0
    for _cycle in range(max_cycles):
        r = b - apply_A(x) if total else b.copy()
        beta = math.sqrt(_dot(r, r))
        if not math.isfinite(beta):
            return x, total, float("nan"), NONFINITE
        if beta <= tol * bnorm:
            return x, total, beta / bnorm, OK
        V = [r / beta]
        H = np.zeros((k + 1, k))
        cs = np.zeros(k)
        sn = np.zeros(k)
        g = np.zeros(k + 1)
        g[0] = beta
        done = False
        capped = False
        j_used = 0
        for j in range(k):
            w = apply_A(apply_Minv(V[j]))
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = _dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = math.sqrt(_dot(w, w))
            for i in range(j):                     # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            if den == 0.0:
                return x, total, est, BREAKDOWN
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            hj1 = H[j + 1, j]
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_used = j + 1
            est = abs(g[j + 1]) / bnorm
            if not math.isfinite(est):
                return x, total, float("nan"), NONFINITE
            if est <= tol or hj1 == 0.0:
                done = True
                break
            if max_iter is not None and total >= max_iter:
                capped = True
                break
            V.append(w / hj1)
        y = np.zeros(j_used)
        for i in range(j_used - 1, -1, -1):        # back substitution
            y[i] = (g[i] - np.dot(H[i, i + 1:j_used], y[i + 1:j_used])) / H[i, i]
        upd = np.zeros_like(b)
        for i in range(j_used):
            upd += y[i] * V[i]
        x += apply_Minv(upd)
        if done:
            return x, total, est, OK
        if capped:
            return x, total, est, NOT_CONVERGED
    return x, total, est, NOT_CONVERGED
