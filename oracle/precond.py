"""The Laplace preconditioner B and its inverse (oracle, test infrastructure only).

Sec. 2.4, eq. precond1: ``B = Lambda_r + Lambda_z - d`` with constant
coefficients built from the midrange mean ``f~ = (min f + max f)/2`` of the
medium (footnote to eq. precond1).  In the 2D Cartesian Dirichlet reading,
with the SPD sign convention of :mod:`oracle.operator`::

    B y = -kappa~ (D_xx + D_zz) y + (rho~ h^2/4) y

B is inverted by separation of variables (Sec. 2.4): a sine transform along x
diagonalises ``-D_xx`` with eigenvalues ``mu_k = (4/dx^2) sin^2(pi k/(2 Nx))``,
leaving one tridiagonal system per wavenumber k along z, solved here by the
Thomas algorithm (sequential Gaussian elimination without pivoting).
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def midrange(f: np.ndarray) -> float:
    """``(min f + max f) / 2`` over all nodes of the medium array."""
    return 0.5 * (float(np.min(f)) + float(np.max(f)))


def sine_matrix(nx: int) -> np.ndarray:
    """``S[i-1, k-1] = sin(pi i k / Nx)`` for ``i, k = 1..Nx-1``."""
    i = np.arange(1, nx)
    return np.sin(np.pi * np.outer(i, i) / nx)


def dst1_direct(x: np.ndarray, nx: int) -> np.ndarray:
    """DST-I along the last axis by its definition:
    ``X_k = sum_{i=1}^{Nx-1} x_i sin(pi i k / Nx)`` (a matrix product)."""
    return np.asarray(x, dtype=np.float64) @ sine_matrix(nx)


def dst1_fft(x: np.ndarray, nx: int) -> np.ndarray:
    """Same transform via the library DST-I (scipy's type-1 DST is twice ours)."""
    return 0.5 * scipy.fft.dst(np.asarray(x, dtype=np.float64), type=1, axis=-1)


def dst1(x: np.ndarray, nx: int) -> np.ndarray:
    """DST-I along the last axis; direct sum for small ``Nx``, library FFT above."""
    return dst1_direct(x, nx) if nx <= 128 else dst1_fft(x, nx)


def thomas(lower: np.ndarray, diag: np.ndarray, upper: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve tridiagonal systems along axis 0 by the Thomas algorithm.

    Row ``j``: ``lower[j] x[j-1] + diag[j] x[j] + upper[j] x[j+1] = rhs[j]``
    (``lower[0]`` and ``upper[-1]`` are ignored).  Trailing axes of the
    arrays are independent systems (broadcasting).
    """
    n = rhs.shape[0]
    cp = np.zeros(np.broadcast(diag, rhs).shape)
    dp = np.zeros_like(cp)
    cp[0] = upper[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for j in range(1, n):
        den = diag[j] - lower[j] * cp[j - 1]
        cp[j] = upper[j] / den
        dp[j] = (rhs[j] - lower[j] * dp[j - 1]) / den
    x = np.zeros_like(dp)
    x[n - 1] = dp[n - 1]
    for j in range(n - 2, -1, -1):
        x[j] = dp[j] - cp[j] * x[j + 1]
    return x


class Laplace:
    """Constant-coefficient operator ``-kx (D_xx) - kz (D_zz) + d`` on the
    Dirichlet interior grid, with its separation-of-variables inverse.

    The acoustic preconditioner uses ``kx = kz = kappa~``, ``d = rho~ h^2/4``;
    the elastic blocks use different x and z coefficients (eq. precond2).
    """

    def __init__(self, nx: int, nz: int, dx: float, dz: float, kx: float, kz: float, d: float,
                 free_top: bool = False, surface_node: bool = False):
        self.free_top = bool(free_top)
        # surface on the first unknown row (elastic traction-free reading): the
        # z-second difference of that row is 2 (z_0 - z_1)/dz^2
        self.surface_node = bool(surface_node)
        self.nx, self.nz, self.dx, self.dz = nx, nz, dx, dz
        self.kx, self.kz, self.d = float(kx), float(kz), float(d)
        k = np.arange(1, nx)
        self.mu = (4.0 / dx ** 2) * np.sin(np.pi * k / (2.0 * nx)) ** 2
        self.off = -self.kz / dz ** 2                              # z off-diagonal
        self.diag = 2.0 * self.kz / dz ** 2 + self.kx * self.mu + self.d   # per k

    def tridiag_solve(self, rhat: np.ndarray) -> np.ndarray:
        """Solve, for every wavenumber k (last axis) the z-system
        ``off*z[j-1] + diag_k z[j] + off*z[j+1] = rhat[j]`` (axis -2 = j)."""
        nz1 = self.nz - 1
        lower = np.full(nz1, self.off)[:, None]
        upper = lower
        diag = np.broadcast_to(self.diag[None, :], (nz1, self.nx - 1))
        if self.free_top:                       # no z-flux above the first row
            diag = diag.copy()
            diag[0, :] -= self.kz / self.dz ** 2
        if self.surface_node:                   # surface row: 2 kz (z_0 - z_1)/dz^2
            upper = upper.copy()
            upper[0, :] = 2.0 * self.off
        if rhat.ndim == 2:
            return thomas(lower, diag, upper, rhat)
        return np.stack([thomas(lower, diag, upper, r) for r in rhat])

    def solve(self, r: np.ndarray) -> np.ndarray:
        """``B^{-1} r``: DST along x, Thomas along z, inverse DST (scale 2/Nx)."""
        rhat = dst1(r, self.nx)
        zhat = self.tridiag_solve(rhat)
        return (2.0 / self.nx) * dst1(zhat, self.nx)

    def apply(self, y: np.ndarray) -> np.ndarray:
        """``B y`` by the 5-point formula (for tests)."""
        pad = [(0, 0)] * (y.ndim - 2) + [(1, 1), (1, 1)]
        Y = np.pad(y, pad)
        c = Y[..., 1:-1, 1:-1]
        if self.free_top:                       # mirror row: the top face carries no flux
            Y[..., 0, 1:-1] = Y[..., 1, 1:-1]
        if self.surface_node:                   # mirror about the surface row
            Y[..., 0, 1:-1] = Y[..., 2, 1:-1]
        dxx = (Y[..., 1:-1, 2:] - 2 * c + Y[..., 1:-1, :-2]) / self.dx ** 2
        dzz = (Y[..., 2:, 1:-1] - 2 * c + Y[..., :-2, 1:-1]) / self.dz ** 2
        return -self.kx * dxx - self.kz * dzz + self.d * c


def acoustic_preconditioner(kappa: np.ndarray, rho: np.ndarray, h: float,
                            nx: int, nz: int, dx: float, dz: float, free_top: bool = False) -> Laplace:
    """B of eq. precond1: ``kappa~`` on both axes and ``d = rho~ h^2/4``; with
    a free surface B keeps the operator's flux-free top face."""
    kt, rt = midrange(kappa), midrange(rho)
    return Laplace(nx, nz, dx, dz, kt, kt, rt * h * h / 4.0, free_top=free_top)
