"""Laguerre transform quantities (oracle, test infrastructure only).

Follows Sec. 2.1 of the paper (eqs. series_lag and laguerre_h):

* orthonormal Laguerre functions
  ``l_m(ht) = sqrt(h m!/(m+alpha)!) (ht)^{alpha/2} exp(-ht/2) L_m^alpha(ht)``;
* forward transform ``f_m = int_0^inf f(t) (ht)^{-alpha/2} l_m(ht) dt``;
* inverse transform ``u(t) = (ht)^{alpha/2} sum_m R_m l_m(ht)``.

Writing ``n_m = sqrt(m!/(m+alpha)!)`` and ``psi_m(x) = n_m exp(-x/2) L_m^alpha(x)``
these become ``f_m = sqrt(h) int f(t) psi_m(ht) dt`` and
``u(t) = sum_m W_m(t) R_m`` with ``W_m(t) = sqrt(h) (ht)^alpha psi_m(ht)``.

``psi_m`` is evaluated by the three-term recurrence of the generalised Laguerre
polynomials (Abramowitz & Stegun 22.7.12) with the normalisation folded in,
carrying a separate power-of-two exponent so that ``exp(-x/2)`` never
underflows for large ``x``.
"""
from __future__ import annotations

import math
from typing import Callable, Tuple

import numpy as np

_RESCALE = 2.0 ** 500
_LOG2_RESCALE = 500.0


def log_norm(m: np.ndarray, alpha: int) -> np.ndarray:
    """``log n_m = 0.5 (log m! - log (m+alpha)!)``."""
    m = np.asarray(m, dtype=np.float64)
    lg = np.vectorize(math.lgamma)
    return 0.5 * (lg(m + 1.0) - lg(m + alpha + 1.0))


def norm_ratio(m: int, alpha: int) -> float:
    """``n_m / n_{m-1} = sqrt(m / (m + alpha))`` for ``m >= 1``."""
    return math.sqrt(m / (m + alpha))


def psi_scaled(n: int, x: np.ndarray, alpha: int) -> Tuple[np.ndarray, np.ndarray]:
    """Return ``(mant, e2)`` with ``psi_m(x) = mant[m] * 2**e2[m]`` for m < n.

    Recurrence in ``m`` (derived from ``m L_m = (2m-1+a-x) L_{m-1} - (m-1+a) L_{m-2}``
    and ``n_m/n_{m-1} = sqrt(m/(m+a))``)::

        psi_0 = exp(-x/2) / sqrt(Gamma(a+1))
        psi_1 = (1 + a - x) psi_0 / sqrt(1 + a)
        psi_m = ((2m-1+a-x) psi_{m-1} - sqrt((m-1)(m-1+a)) psi_{m-2}) / sqrt(m (m+a))
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    a = float(alpha)
    mant = np.zeros((n,) + x.shape)
    e2 = np.zeros((n,) + x.shape)
    # psi_0 = 2**e with e = log2(exp(-x/2)/sqrt(Gamma(a+1))); mantissa 1.
    e = (-0.5 * x - 0.5 * math.lgamma(a + 1.0)) / math.log(2.0)
    prev2 = np.zeros_like(x)          # psi_{m-2} mantissa (relative to e)
    prev1 = np.ones_like(x)           # psi_{m-1} mantissa
    mant[0] = prev1
    e2[0] = e
    if n == 1:
        return mant, e2
    cur = (1.0 + a - x) * prev1 / math.sqrt(1.0 + a)
    mant[1] = cur
    e2[1] = e
    prev2, prev1 = prev1, cur
    for m in range(2, n):
        cur = ((2.0 * m - 1.0 + a - x) * prev1
               - math.sqrt((m - 1.0) * (m - 1.0 + a)) * prev2) / math.sqrt(m * (m + a))
        big = np.abs(cur) > _RESCALE
        if np.any(big):
            cur = np.where(big, cur / _RESCALE, cur)
            prev1 = np.where(big, prev1 / _RESCALE, prev1)
            e = np.where(big, e + _LOG2_RESCALE, e)
        mant[m] = cur
        e2[m] = e
        prev2, prev1 = prev1, cur
    return mant, e2


def psi(n: int, x: np.ndarray, alpha: int) -> np.ndarray:
    """``psi_m(x)`` for ``m < n`` as plain doubles (may underflow to 0)."""
    mant, e2 = psi_scaled(n, x, alpha)
    return mant * np.exp2(e2)


def synthesis_weights(t: np.ndarray, h: float, alpha: int, n: int) -> np.ndarray:
    """``W[q, m] = sqrt(h) (h t_q)^alpha psi_m(h t_q)``, shape ``[len(t), n]``.

    The power ``(ht)^alpha`` and the tracked exponent are combined in log2
    before exponentiating, so large ``h t`` does not underflow early.
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    x = h * t
    mant, e2 = psi_scaled(n, x, alpha)
    out = np.zeros((len(t), n))
    pos = x > 0
    if np.any(pos):
        lg = 0.5 * math.log2(h) + alpha * np.log2(x[pos])
        out[pos, :] = (mant[:, pos] * np.exp2(e2[:, pos] + lg[None, :])).T
    return out


# ---------------------------------------------------------------------------
# source wavelets
# ---------------------------------------------------------------------------

def ricker(f0: float, t0: float) -> Callable[[np.ndarray], np.ndarray]:
    """``f(t) = (1 - 2 (pi f0 (t-t0))^2) exp(-(pi f0 (t-t0))^2)``."""
    def f(t):
        a = (math.pi * f0 * (np.asarray(t) - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    return f


def gauss_sine(f0: float, t0: float, gamma: float) -> Callable[[np.ndarray], np.ndarray]:
    """The paper's pulse (eq. functiont):
    ``exp(-(2 pi f0 (t-t0))^2 / gamma^2) sin(2 pi f0 (t-t0))``."""
    def f(t):
        s = 2.0 * math.pi * f0 * (np.asarray(t) - t0)
        return np.exp(-(s * s) / (gamma * gamma)) * np.sin(s)
    return f


def source_coeffs(f: Callable[[np.ndarray], np.ndarray], t_end: float, h: float,
                  alpha: int, n: int, rel_tol: float = 1e-14, n_gl: int = 32,
                  panels0: int = 8, max_panels: int = 4096) -> np.ndarray:
    """``f_m = sqrt(h) int_0^{t_end} f(t) psi_m(ht) dt`` for m < n.

    Composite Gauss-Legendre quadrature (``n_gl`` points per panel) on equal
    panels; the panel count is doubled until the largest change of any
    coefficient is below ``rel_tol`` times the largest coefficient (or
    ``max_panels`` is reached).
    """
    xg, wg = np.polynomial.legendre.leggauss(n_gl)

    def integrate(panels: int) -> np.ndarray:
        edges = np.linspace(0.0, t_end, panels + 1)
        half = 0.5 * (edges[1:] - edges[:-1])
        mid = 0.5 * (edges[1:] + edges[:-1])
        tq = (mid[:, None] + half[:, None] * xg[None, :]).ravel()
        wq = (half[:, None] * wg[None, :]).ravel()
        acc = np.zeros(n)
        chunk = 1 << 14
        for s0 in range(0, len(tq), chunk):
            ps = psi(n, h * tq[s0:s0 + chunk], alpha)      # [n, chunk]
            acc += ps @ (wq[s0:s0 + chunk] * f(tq[s0:s0 + chunk]))
        return math.sqrt(h) * acc

    panels = panels0
    prev = integrate(panels)
    while panels < max_panels:
        panels *= 2
        cur = integrate(panels)
        if np.max(np.abs(cur - prev)) <= rel_tol * max(np.max(np.abs(cur)), 1e-300):
            return cur
        prev = cur
    return prev


def ricker_coeffs(f0: float, t0: float, h: float, alpha: int, n: int) -> np.ndarray:
    """Source coefficients of the Ricker wavelet, integrated to ``t0 + 8/f0``
    (beyond which the wavelet is below 1e-270)."""
    return source_coeffs(ricker(f0, t0), t0 + 8.0 / f0, h, alpha, n)
