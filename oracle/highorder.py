"""Fourth-order acoustic operator (oracle, test infrastructure only).

The paper remarks (Sec. 3.2, after the accuracy study) that higher-order
schemes fit the method, preconditioned by the same second-order Laplace
operator B, at the price of somewhat more CG iterations.  It names no scheme;
the one used here keeps the flux form of Sec. 2.3 and its symmetry:

    A4 = Dx^T Kx Dx + Dz^T Kz Dz + w,

with D the fourth-order staggered difference from nodes to faces,

    (D u)_{m+1/2} = [27 (u_{m+1} - u_m) - (u_{m+2} - u_{m-1})] / (24 h),

and the Dirichlet sides taken by odd reflection (u_{-1} = -u_1 and
u_{N+1} = -u_{N-1}, with u_0 = u_N = 0) folded into D, so that A4 is
symmetric, and positive definite for K > 0.  A sine mode of the grid is then
an eigenvector of Dx^T Dx with eigenvalue [(27 sin(t/2) - sin(3t/2))/(12 h)]^2,
t = pi k / N (against [2 sin(t/2)/h]^2 for the second-order difference), so
B^{-1} A4 stays within a factor (7/6)^2 of B^{-1} A for a constant medium.

Face coefficients: the fourth-order interpolant of the node values,
(-k_{m-1} + 9 k_m + 9 k_{m+1} - k_{m+2}) / 16, with the one-sided
(5 k_0 + 15 k_1 - 5 k_2 + k_3) / 16 at the two end faces.  Next to a strong
jump the interpolant can undershoot (to zero or below for contrasts beyond
about 9); wherever it falls under half the smaller of the face's two node
values the face takes the two-point mean instead, so every K is positive.

Layout as in :mod:`oracle.operator`: interior fields (Nz-1, Nx-1), x fastest;
``kx`` (Nz-1, Nx) holds the x-faces m+1/2 (m = 0..Nx-1) of the interior rows,
``kz`` (Nz, Nx-1) the z-faces n+1/2 (n = 0..Nz-1) of the interior columns.
"""
from __future__ import annotations

import numpy as np


def interp_faces4(k: np.ndarray) -> np.ndarray:
    """Face values along the last axis: nodes 0..N -> faces 1/2..N-1/2."""
    k = np.asarray(k, dtype=np.float64)
    n = k.shape[-1] - 1
    lo = np.minimum(k[..., :-1], k[..., 1:])
    mean = 0.5 * (k[..., :-1] + k[..., 1:])
    f = mean.copy()
    if n >= 3:
        f[..., 1:-1] = (-k[..., :-3] + 9.0 * k[..., 1:-2] + 9.0 * k[..., 2:-1] - k[..., 3:]) / 16.0
        f[..., 0] = (5.0 * k[..., 0] + 15.0 * k[..., 1] - 5.0 * k[..., 2] + k[..., 3]) / 16.0
        f[..., -1] = (5.0 * k[..., -1] + 15.0 * k[..., -2] - 5.0 * k[..., -3] + k[..., -4]) / 16.0
    bad = f < 0.5 * lo
    f[bad] = mean[bad]
    return f


def face_coeffs4(kappa: np.ndarray):
    """``(kx, kz)`` from the node array ``kappa`` (Nz+1, Nx+1)."""
    kx = interp_faces4(kappa[1:-1, :])                  # (Nz-1, Nx)
    kz = interp_faces4(kappa[:, 1:-1].T).T              # (Nz, Nx-1)
    return kx, kz


def _odd_extend(Y: np.ndarray, axis: int) -> np.ndarray:
    """Nodes 0..N (zero at both ends) -> nodes -1..N+1 by odd reflection."""
    first = -np.take(Y, [1], axis=axis)
    last = -np.take(Y, [Y.shape[axis] - 2], axis=axis)
    return np.concatenate([first, Y, last], axis=axis)


def _d4(E: np.ndarray, axis: int) -> np.ndarray:
    """Staggered differences on nodes -1..N+1 -> faces 1/2..N-1/2 (times 24 h)."""
    n = E.shape[axis] - 3                                # N
    s = lambda a, b: np.take(E, np.arange(a, a + n), axis=axis) - np.take(E, np.arange(b, b + n), axis=axis)
    return 27.0 * s(2, 1) - s(3, 0)


def _d4t(g: np.ndarray, axis: int) -> np.ndarray:
    """Transpose: faces 1/2..N-1/2 -> interior nodes 1..N-1 (times 24 h); the
    faces -1/2 and N+1/2 are the mirrors of 1/2 and N-1/2."""
    G = np.concatenate([np.take(g, [0], axis=axis), g, np.take(g, [g.shape[axis] - 1], axis=axis)], axis=axis)
    n1 = g.shape[axis] - 1                               # N-1 interior nodes
    t = lambda a: np.take(G, np.arange(a, a + n1), axis=axis)
    # node i (1..N-1): faces i-3/2, i-1/2, i+1/2, i+3/2 are G[i-1], G[i], G[i+1], G[i+2]
    return 27.0 * t(1) - 27.0 * t(2) - t(0) + t(3)


def apply_A4(y: np.ndarray, kx: np.ndarray, kz: np.ndarray, w: np.ndarray, dx: float, dz: float) -> np.ndarray:
    """``A4 y`` for interior values ``y`` (.., Nz-1, Nx-1)."""
    y = np.asarray(y, dtype=np.float64)
    pad = [(0, 0)] * (y.ndim - 2) + [(1, 1), (1, 1)]
    Y = np.pad(y, pad)                                   # zero Dirichlet ring, nodes 0..N
    ax = y.ndim - 1
    az = y.ndim - 2
    Ex = _odd_extend(Y[..., 1:-1, :], ax)                # interior rows, nodes -1..Nx+1
    gx = kx * _d4(Ex, ax) / (24.0 * dx)
    Ez = _odd_extend(Y[..., :, 1:-1], az)                # interior columns, nodes -1..Nz+1
    gz = kz * _d4(Ez, az) / (24.0 * dz)
    return _d4t(gx, ax) / (24.0 * dx) + _d4t(gz, az) / (24.0 * dz) + w * y


def difference_matrix4(n: int, h: float) -> np.ndarray:
    """D as an (N faces) x (N-1 interior nodes) matrix, the reflections folded
    in, by explicit loops (independent of :func:`apply_A4`)."""
    D = np.zeros((n, n - 1))
    for m in range(n):                                   # face m+1/2
        for node, c in ((m - 1, 1.0), (m, -27.0), (m + 1, 27.0), (m + 2, -1.0)):
            sign = 1.0
            if node == -1:
                node, sign = 1, -1.0
            elif node == n + 1:
                node, sign = n - 1, -1.0
            if 1 <= node <= n - 1:
                D[m, node - 1] += sign * c / (24.0 * h)
    return D


def assemble_A4(kx: np.ndarray, kz: np.ndarray, w: np.ndarray, dx: float, dz: float) -> np.ndarray:
    """Dense A4 = Dx^T Kx Dx + Dz^T Kz Dz + diag(w) (small grids); unknown
    (j, i) has index j*(Nx-1) + i."""
    nz1, nx1 = w.shape
    Dx = difference_matrix4(nx1 + 1, dx)
    Dz = difference_matrix4(nz1 + 1, dz)
    A = np.diag(w.ravel()).astype(np.float64)
    for j in range(nz1):                                 # x-faces of row j
        blk = Dx.T @ np.diag(kx[j]) @ Dx
        A[j * nx1:(j + 1) * nx1, j * nx1:(j + 1) * nx1] += blk
    for i in range(nx1):                                 # z-faces of column i
        blk = Dz.T @ np.diag(kz[:, i]) @ Dz
        idx = np.arange(nz1) * nx1 + i
        A[np.ix_(idx, idx)] += blk
    return A


def sine_eigenvalue4(k, n: int, h: float):
    """Eigenvalue of Dx^T Dx on the k-th grid sine mode of N cells."""
    t = np.pi * np.asarray(k, dtype=np.float64) / n
    return ((27.0 * np.sin(t / 2) - np.sin(1.5 * t)) / (12.0 * h)) ** 2
