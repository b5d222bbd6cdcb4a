"""The 5-point Laguerre-shifted operator A (oracle, test infrastructure only).

Sec. 2.3 (eqs. poisson_diff_2, scheme_op_r_z, diff_approx1) writes the
discrete problem as ``(Lambda_r + Lambda_z) y - w y = -phi`` with
``Lambda y = (a y_xbar)_x`` (flux form, coefficients on the cell faces) and
``w = rho h^2/4``.  In the 2D Cartesian Dirichlet reading used here the radial
weights ``r_i`` drop out, and the operator is taken with the opposite sign so
that it is symmetric positive definite (the paper's ``A = A* > 0``)::

    (A y)_{j,i} = [kx_{i+1/2} (y_{i} - y_{i+1}) + kx_{i-1/2} (y_{i} - y_{i-1})] / dx^2
                + [kz_{j+1/2} (y_{j} - y_{j+1}) + kz_{j-1/2} (y_{j} - y_{j-1})] / dz^2
                + w_{j,i} y_{j,i}

Face coefficients are the arithmetic mean of the two node values of kappa,
``y`` is zero on every boundary node, unknowns are the interior nodes.

Free surface (``free_top=True``): the paper's condition du/dz = 0 at z = 0
(Sec. 2.1, eq. boundary_cond), in the form its staggered mesh gives it
(Sec. 2.3: the first unknown lies half a cell below the surface): no flux
crosses the face above the first unknown row, i.e. that face coefficient is
zero.  The other three sides stay Dirichlet.
"""
from __future__ import annotations

import numpy as np


def shift_coeff(rho: np.ndarray, h: float) -> np.ndarray:
    """``w = rho h^2 / 4`` on the interior nodes (rho given on all nodes)."""
    return rho[1:-1, 1:-1] * (h * h / 4.0)


def apply_A(y: np.ndarray, kappa: np.ndarray, w: np.ndarray, dx: float, dz: float,
            free_top: bool = False) -> np.ndarray:
    """``A y`` for interior values ``y`` of shape ``(Nz-1, Nx-1)`` (or a leading
    batch axis).  ``kappa`` is the node array ``(Nz+1, Nx+1)``, ``w`` interior."""
    y = np.asarray(y, dtype=np.float64)
    pad = [(0, 0)] * (y.ndim - 2) + [(1, 1), (1, 1)]
    Y = np.pad(y, pad)                       # zero Dirichlet ring
    kx = 0.5 * (kappa[1:-1, :-1] + kappa[1:-1, 1:])   # faces i+1/2, rows 1..Nz-1
    kz = 0.5 * (kappa[:-1, 1:-1] + kappa[1:, 1:-1])   # faces j+1/2, cols 1..Nx-1
    if free_top:
        kz = kz.copy()
        kz[0, :] = 0.0                                # no flux through the surface face
    c = Y[..., 1:-1, 1:-1]
    ax = (kx[:, 1:] * (c - Y[..., 1:-1, 2:]) + kx[:, :-1] * (c - Y[..., 1:-1, :-2])) / (dx * dx)
    az = (kz[1:, :] * (c - Y[..., 2:, 1:-1]) + kz[:-1, :] * (c - Y[..., :-2, 1:-1])) / (dz * dz)
    return ax + az + w * c


def assemble_A(kappa: np.ndarray, w: np.ndarray, dx: float, dz: float, free_top: bool = False) -> np.ndarray:
    """Dense matrix of A by explicit loops over the stencil (small grids only).

    Written independently of :func:`apply_A` so that the two can check each
    other; unknown ``(j, i)`` (interior, 0-based) has index ``j*(Nx-1) + i``.
    """
    nz1, nx1 = w.shape
    n = nz1 * nx1
    M = np.zeros((n, n))
    for j in range(nz1):
        for i in range(nx1):
            row = j * nx1 + i
            J, I = j + 1, i + 1                      # node indices
            kE = 0.5 * (kappa[J, I] + kappa[J, I + 1])
            kW = 0.5 * (kappa[J, I] + kappa[J, I - 1])
            kS = 0.5 * (kappa[J, I] + kappa[J + 1, I])
            kN = 0.5 * (kappa[J, I] + kappa[J - 1, I])
            if free_top and j == 0:
                kN = 0.0
            M[row, row] = (kE + kW) / dx ** 2 + (kS + kN) / dz ** 2 + w[j, i]
            if i + 1 < nx1:
                M[row, row + 1] = -kE / dx ** 2
            if i - 1 >= 0:
                M[row, row - 1] = -kW / dx ** 2
            if j + 1 < nz1:
                M[row, row + nx1] = -kS / dz ** 2
            if j - 1 >= 0:
                M[row, row - nx1] = -kN / dz ** 2
    return M
