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

Traction-free surface (Sec. 2.2, eq. boundary_elastic: tau_xz = sigma_zz = 0
at z = 0).  The paper prints only the continuous conditions.  The reading
used here puts the surface on the first unknown node row and takes the
operator from the discrete strain energy, whose natural boundary condition is
the traction-free one::

    E(u) = 1/2 sum_xfaces c_j [(l+2m)^f (Dx ux)^2 + m^f (Dx uz)^2]
         + 1/2 sum_zfaces       [m^f (Dz ux)^2 + (l+2m)^f (Dz uz)^2]
         +     sum_nodes  c_j [l (Dxc ux)(Dz uz) + m (Dz ux)(Dxc uz)]
         + 1/2 sum_nodes  c_j w |u|^2

with c_j = 1/2 on the surface row (its control strip is half a cell) and 1
below, no z-face above the surface, and the z-derivative of the node terms
central below the surface and one-sided, (u_{j+1} - u_j)/dz, on it.  With all
c_j = 1, the face above the first row present and central differences
everywhere, E's gradient is the Dirichlet C above.  The free operator is the
strong form ``C_free u = D_c^{-1} grad E`` (lumped mass c_j per row), so the
right-hand side of every harmonic keeps its form; ``D_c C_free`` (the Hessian
of E) is symmetric.  The surface row's truncation error is first order (the
traction terms cancel to O(1)), the scheme converges at second order.
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
                         nx: int, nz: int, dx: float, dz: float,
                         surface_node: bool = False) -> Tuple[Laplace, Laplace]:
    """``(B1, B2)`` of eq. precond2 in the Cartesian reading; with
    ``surface_node`` their top row is the traction-free surface row (the
    z-second difference there is 2 (u_1 - u_2)/dz^2: no flux through the
    surface, half a control cell)."""
    p = midrange(lam + 2.0 * mu)
    s = midrange(mu)
    d = midrange(rho) * h * h / 4.0
    return (Laplace(nx, nz, dx, dz, p, s, d, surface_node=surface_node),
            Laplace(nx, nz, dx, dz, s, p, d, surface_node=surface_node))


def apply_Kinv(u: np.ndarray, B1: Laplace, B2: Laplace) -> np.ndarray:
    return np.stack([B1.solve(u[0]), B2.solve(u[1])])


# ---------------------------------------------------------------------------
# traction-free surface on the first unknown row
# ---------------------------------------------------------------------------

def surface_weights(nz1: int) -> np.ndarray:
    """Control-strip weight c_j of the unknown rows: 1/2 on the surface row."""
    c = np.ones(nz1)
    c[0] = 0.5
    return c


def _node(u: np.ndarray) -> np.ndarray:
    """Interior values -> node array (Nz+1, Nx+1) with a zero ring (the top
    ring row is outside the body and never read)."""
    return np.pad(u, [(1, 1), (1, 1)])


def _dz_nodes(V: np.ndarray, dz: float) -> np.ndarray:
    """z-derivative at the unknown rows (node rows 1..Nz-1): one-sided on the
    surface row, central below."""
    d = np.empty_like(V[1:-1, :])
    d[0] = (V[2] - V[1]) / dz
    d[1:] = (V[3:] - V[1:-2]) / (2.0 * dz)
    return d


def energy_free(u: np.ndarray, lam: np.ndarray, mu: np.ndarray, w: np.ndarray,
                dx: float, dz: float) -> float:
    """The discrete energy E(u) of the traction-free problem (per cell area)."""
    Ux, Uz = _node(u[0]), _node(u[1])
    lp2m = lam + 2.0 * mu
    c = surface_weights(w.shape[0])[:, None]
    # x faces (i+1/2, j), rows 1..Nz-1
    fp = 0.5 * (lp2m[1:-1, :-1] + lp2m[1:-1, 1:])
    fm = 0.5 * (mu[1:-1, :-1] + mu[1:-1, 1:])
    ex = 0.5 * np.sum(c * (fp * ((Ux[1:-1, 1:] - Ux[1:-1, :-1]) / dx) ** 2 +
                           fm * ((Uz[1:-1, 1:] - Uz[1:-1, :-1]) / dx) ** 2))
    # z faces (i, j+1/2) below the surface, columns 1..Nx-1
    gp = 0.5 * (lp2m[1:-1, 1:-1] + lp2m[2:, 1:-1])
    gm = 0.5 * (mu[1:-1, 1:-1] + mu[2:, 1:-1])
    ez = 0.5 * np.sum(gm * ((Ux[2:, 1:-1] - Ux[1:-1, 1:-1]) / dz) ** 2 +
                      gp * ((Uz[2:, 1:-1] - Uz[1:-1, 1:-1]) / dz) ** 2)
    # node cross terms, interior columns
    a = (Ux[1:-1, 2:] - Ux[1:-1, :-2]) / (2.0 * dx)        # Dxc ux
    cc = (Uz[1:-1, 2:] - Uz[1:-1, :-2]) / (2.0 * dx)       # Dxc uz
    b = _dz_nodes(Ux, dz)[:, 1:-1]                          # Dz ux
    d = _dz_nodes(Uz, dz)[:, 1:-1]                          # Dz uz
    ec = np.sum(c * (lam[1:-1, 1:-1] * a * d + mu[1:-1, 1:-1] * b * cc))
    ew = 0.5 * np.sum(c * w * (u[0] ** 2 + u[1] ** 2))
    return float(ex + ez + ec + ew)


def apply_C_free(u: np.ndarray, lam: np.ndarray, mu: np.ndarray, w: np.ndarray,
                 dx: float, dz: float) -> np.ndarray:
    """``C_free u = D_c^{-1} grad E(u)``: every term of E contributes the
    transpose of its difference applied to its weighted flux."""
    Ux, Uz = _node(u[0]), _node(u[1])
    Gx, Gz = np.zeros_like(Ux), np.zeros_like(Uz)
    lp2m = lam + 2.0 * mu
    c = surface_weights(w.shape[0])[:, None]
    # x faces: flux F on face (i+1/2, j) adds +F/dx at i+1 and -F/dx at i
    for G, V, k in ((Gx, Ux, lp2m), (Gz, Uz, mu)):
        F = c * 0.5 * (k[1:-1, :-1] + k[1:-1, 1:]) * (V[1:-1, 1:] - V[1:-1, :-1]) / dx
        G[1:-1, 1:] += F / dx
        G[1:-1, :-1] -= F / dx
    # z faces below the surface: flux on (i, j+1/2) adds +/dz at j+1, -/dz at j
    for G, V, k in ((Gx, Ux, mu), (Gz, Uz, lp2m)):
        F = 0.5 * (k[1:-1, 1:-1] + k[2:, 1:-1]) * (V[2:, 1:-1] - V[1:-1, 1:-1]) / dz
        G[2:, 1:-1] += F / dz
        G[1:-1, 1:-1] -= F / dz

    def add_dx(G, coef):
        # the term coef * Dxc(V) at interior nodes: d/dV(i+1) = +1/2dx, d/dV(i-1) = -1/2dx
        G[1:-1, 2:] += coef / (2.0 * dx)
        G[1:-1, :-2] -= coef / (2.0 * dx)

    def add_dz(G, coef):
        # the term coef * Dz(V) at interior nodes, one-sided on the surface row
        G[2, 1:-1] += coef[0] / dz
        G[1, 1:-1] -= coef[0] / dz
        G[3:, 1:-1] += coef[1:] / (2.0 * dz)
        G[1:-2, 1:-1] -= coef[1:] / (2.0 * dz)

    a = (Ux[1:-1, 2:] - Ux[1:-1, :-2]) / (2.0 * dx)
    cc = (Uz[1:-1, 2:] - Uz[1:-1, :-2]) / (2.0 * dx)
    b = _dz_nodes(Ux, dz)[:, 1:-1]
    d = _dz_nodes(Uz, dz)[:, 1:-1]
    lm, mm = lam[1:-1, 1:-1], mu[1:-1, 1:-1]
    add_dx(Gx, c * lm * d)          # l a d, through a = Dxc ux
    add_dz(Gz, c * lm * a)          # l a d, through d = Dz uz
    add_dz(Gx, c * mm * cc)         # m b cc, through b = Dz ux
    add_dx(Gz, c * mm * b)          # m b cc, through cc = Dxc uz
    gx = Gx[1:-1, 1:-1] + c * w * u[0]
    gz = Gz[1:-1, 1:-1] + c * w * u[1]
    return np.stack([gx / c, gz / c])


def source_field_free(shape, src_ij, value: float, dx: float, dz: float) -> np.ndarray:
    """Vertical point force of strength ``value`` at node ``(i, j)`` of the
    traction-free problem: ``value / (c_j dx dz)`` on the z component, c_j the
    row's control-strip weight (a force on the surface row acts on half a
    cell).  Shape ``(2, Nz-1, Nx-1)``."""
    out = np.zeros((2,) + tuple(shape))
    i, j = int(src_ij[0]), int(src_ij[1])
    out[1, j - 1, i - 1] = value / (surface_weights(shape[0])[j - 1] * dx * dz)
    return out
