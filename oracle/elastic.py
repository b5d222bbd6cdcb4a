"""2D Cartesian elastic operator C and block preconditioner K (oracle, test infra).

The paper (Sec. 2.2, eq. elastic_problemQn) applies the Laguerre transform to
the Lame equations and approximates them "by the finite-volume method with
second order of accuracy" (Sec. 2.3) without printing the scheme.  The
reading used here, in 2D Cartesian coordinates with Dirichlet boundaries on
all four sides and the SPD sign convention, is the second-order flux form of
``-div sigma + rho h^2/4 u``::

    (C u)_x = -Dx+((l+2m)^f Dx- ux) - Dz+(m^f Dz- ux) - Dxc(l Dzc uz) - Dzc(m Dxc uz) + w ux
    (C u)_z = -Dx+(m^f Dx- uz) - Dz+((l+2m)^f Dz- uz) - Dzc(l Dxc ux) - Dxc(m Dzc ux) + w uz

with face values the arithmetic mean of node values, ``Dc`` the two-cell
central difference and ``w = rho h^2/4``.  Because ``Dc`` is antisymmetric
under zero Dirichlet padding, C is symmetric.  Fidelity of this scheme to the
paper's own finite-volume scheme is parity unpinned (the scheme is not in the
paper); it is pinned against dense assembly, symmetry and positivity.

The preconditioner is eq. precond2 without the cylindrical hoop term:
``K = diag(B1, B2)``, B1 with x-coefficient ``(l+2m)~`` and z-coefficient
``m~``, B2 with ``m~`` and ``(l+2m)~``, both with ``d = rho~ h^2/4``.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from .precond import Laplace, midrange


def _pad(u: np.ndarray) -> np.ndarray:
    return np.pad(u, [(0, 0)] * (u.ndim - 2) + [(1, 1), (1, 1)])


def apply_C(u: np.ndarray, lam: np.ndarray, mu: np.ndarray, w: np.ndarray,
            dx: float, dz: float) -> np.ndarray:
    """``C u`` for ``u`` of shape ``(2, Nz-1, Nx-1)`` (components x, z)."""
    ux, uz = _pad(u[0]), _pad(u[1])          # node arrays, zero boundary
    lp2m = lam + 2.0 * mu

    def div_flux(v, cx, cz):
        # -Dx+(cx^f Dx- v) - Dz+(cz^f Dz- v) on interior nodes
        fx = 0.5 * (cx[1:-1, :-1] + cx[1:-1, 1:])        # x faces, rows 1..Nz-1
        fz = 0.5 * (cz[:-1, 1:-1] + cz[1:, 1:-1])        # z faces, cols 1..Nx-1
        c = v[1:-1, 1:-1]
        tx = (fx[:, 1:] * (c - v[1:-1, 2:]) + fx[:, :-1] * (c - v[1:-1, :-2])) / dx ** 2
        tz = (fz[1:, :] * (c - v[2:, 1:-1]) + fz[:-1, :] * (c - v[:-2, 1:-1])) / dz ** 2
        return tx + tz

    def dxc(v):   # central x-difference on node rows 0..Nz, interior columns
        return (v[:, 2:] - v[:, :-2]) / (2.0 * dx)

    def dzc(v):   # central z-difference on interior rows, node columns 0..Nx
        return (v[2:, :] - v[:-2, :]) / (2.0 * dz)

    # Dxc(c * Dzc v): inner on interior rows x all columns, outer on interior cols
    def mix_xz(c, v):
        inner = c[1:-1, :] * dzc(v)              # rows 1..Nz-1, cols 0..Nx
        return dxc(inner)

    def mix_zx(c, v):
        inner = c[:, 1:-1] * dxc(v)              # rows 0..Nz, cols 1..Nx-1
        return dzc(inner)

    cx = div_flux(ux, lp2m, mu) - mix_xz(lam, uz) - mix_zx(mu, uz) + w * u[0]
    cz = div_flux(uz, mu, lp2m) - mix_zx(lam, ux) - mix_xz(mu, ux) + w * u[1]
    return np.stack([cx, cz])


def assemble_C(lam: np.ndarray, mu: np.ndarray, w: np.ndarray, dx: float, dz: float) -> np.ndarray:
    """Dense C by applying it to unit vectors of the *full* node grid through an
    independent loop formulation (small grids only)."""
    nz1, nx1 = w.shape
    n = nz1 * nx1
    M = np.zeros((2 * n, 2 * n))
    lp2m = lam + 2 * mu

    def idx(comp, j, i):          # node (i, j) interior -> unknown index, else None
        if 1 <= i <= nx1 and 1 <= j <= nz1:
            return comp * n + (j - 1) * nx1 + (i - 1)
        return None

    def add(row, comp, j, i, val):
        col = idx(comp, j, i)
        if col is not None:
            M[row, col] += val

    for J in range(1, nz1 + 1):
        for I in range(1, nx1 + 1):
            for comp in (0, 1):
                row = idx(comp, J, I)
                cxx = lp2m if comp == 0 else mu      # coefficient of d/dx in own comp
                czz = mu if comp == 0 else lp2m
                e = 0.5 * (cxx[J, I] + cxx[J, I + 1]); wv = 0.5 * (cxx[J, I] + cxx[J, I - 1])
                s = 0.5 * (czz[J, I] + czz[J + 1, I]); nn = 0.5 * (czz[J, I] + czz[J - 1, I])
                add(row, comp, J, I, (e + wv) / dx ** 2 + (s + nn) / dz ** 2 + w[J - 1, I - 1])
                add(row, comp, J, I + 1, -e / dx ** 2)
                add(row, comp, J, I - 1, -wv / dx ** 2)
                add(row, comp, J + 1, I, -s / dz ** 2)
                add(row, comp, J - 1, I, -nn / dz ** 2)
                other = 1 - comp
                # x-eq: -Dxc(l Dzc uz) - Dzc(m Dxc uz); z-eq: -Dzc(l Dxc ux) - Dxc(m Dzc ux)
                c_xz = lam if comp == 0 else mu       # coefficient inside Dxc( . Dzc)
                c_zx = mu if comp == 0 else lam       # coefficient inside Dzc( . Dxc)
                f = 1.0 / (4.0 * dx * dz)
                for si in (+1, -1):          # outer Dxc: node I+si, inner Dzc at J+-1
                    for sj in (+1, -1):
                        add(row, other, J + sj, I + si, -si * sj * f * c_xz[J, I + si])
                for sj in (+1, -1):          # outer Dzc: node J+sj, inner Dxc at I+-1
                    for si in (+1, -1):
                        add(row, other, J + sj, I + si, -sj * si * f * c_zx[J + sj, I])
    return M


def block_preconditioner(lam: np.ndarray, mu: np.ndarray, rho: np.ndarray, h: float,
                         nx: int, nz: int, dx: float, dz: float) -> Tuple[Laplace, Laplace]:
    """``(B1, B2)`` of eq. precond2 in the Cartesian reading."""
    p = midrange(lam + 2.0 * mu)
    s = midrange(mu)
    d = midrange(rho) * h * h / 4.0
    return Laplace(nx, nz, dx, dz, p, s, d), Laplace(nx, nz, dx, dz, s, p, d)


def apply_Kinv(u: np.ndarray, B1: Laplace, B2: Laplace) -> np.ndarray:
    return np.stack([B1.solve(u[0]), B2.solve(u[1])])
