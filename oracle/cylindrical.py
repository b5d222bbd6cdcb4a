"""The paper's 2.5D axisymmetric acoustic problem (oracle, test infrastructure
only): operator, cosine transform along z, and the Laplace preconditioner with
its non-Toeplitz r-systems.

Mesh (Sec. 2.3): r_i = (i - 1/2) h_r, i = 1..Nr, and z_k = (k - 1/2) h_z,
k = 1..Nz.  Unknowns are i = 1..Nr-1 (row i-1 of a field) and k = 1..Nz
(column k-1); y = 0 on the row i = Nr (the side r = l1).  A field is
``[Nr-1][Nz]`` with z fastest; the medium is given at all nodes, ``[Nr][Nz]``.

Operator (eqs. poisson_diff_2, scheme_op_r_z, diff_approx1; SPD sign,
``A = -(Lambda_r + Lambda_z) + w``)::

    (A y)_{i,k} = [a1_{i}(y_i - y_{i+1}) + a1_{i-1}(y_i - y_{i-1})] / h_r^2
                + [a2_{k}(y_k - y_{k+1}) + a2_{k-1}(y_k - y_{k-1})] / h_z^2
                + w_{i,k} y_{i,k}

with a1 on the r-faces rbar_i = r_i + h_r/2 (a1 = rbar kappa), a2 on the
z-faces (a2 = r_i kappa), w = r_i rho h^2/4.  The face at r = 0 has rbar = 0
(the symmetry condition of the first row), the two z-ends carry no flux (du/dz
= 0 at z = 0 and z = l2: the first and last rows of scheme_op_r_z), and the
side r = l1 is Dirichlet.  Face values of kappa are the mean of the two
adjacent node values.

Right-hand side of harmonic m, with the whole equation multiplied by r_i (the
weighting of w): phi = delta_h f_m / (2 pi) at the source node, delta_h =
1/(h_r h_z), minus h^2 r_i rho Q_m (the running history sum).
"""
from __future__ import annotations

import numpy as np


def radii(nr: int, hr: float) -> np.ndarray:
    """r_i of the unknown rows i = 1..Nr-1."""
    return (np.arange(1, nr) - 0.5) * hr


def coefficients(kappa: np.ndarray, rho: np.ndarray, h: float, hr: float):
    """Face coefficients and shift from node arrays ``[Nr][Nz]``:
    ``a1 [Nr-1][Nz]`` on the faces rbar_i (i = 1..Nr-1), ``a2 [Nr-1][Nz-1]``
    on the z-faces of the unknown rows, ``w [Nr-1][Nz]``."""
    nr = kappa.shape[0]
    r = radii(nr, hr)[:, None]
    rbar = r + 0.5 * hr
    a1 = rbar * 0.5 * (kappa[:-1, :] + kappa[1:, :])
    a2 = r * 0.5 * (kappa[:-1, :-1] + kappa[:-1, 1:])
    w = r * rho[:-1, :] * (h * h / 4.0)
    return a1, a2, w


def apply_A(y: np.ndarray, a1: np.ndarray, a2: np.ndarray, w: np.ndarray, hr: float, hz: float) -> np.ndarray:
    """``A y`` for ``y [.., Nr-1, Nz]``."""
    y = np.asarray(y, dtype=np.float64)
    out = w * y
    # r-direction: faces between rows i and i+1 (the last one to the Dirichlet row)
    yn = np.zeros_like(y)
    yn[..., :-1, :] = y[..., 1:, :]
    flux = a1 * (y - yn)                                 # face rbar_i, outward
    out = out + flux / (hr * hr)
    out[..., 1:, :] -= flux[..., :-1, :] / (hr * hr)     # the same face seen from row i+1
    # z-direction: interior faces only (both ends carry no flux)
    fz = a2 * (y[..., :, :-1] - y[..., :, 1:])
    out[..., :, :-1] += fz / (hz * hz)
    out[..., :, 1:] -= fz / (hz * hz)
    return out


def assemble_A(a1: np.ndarray, a2: np.ndarray, w: np.ndarray, hr: float, hz: float) -> np.ndarray:
    """Dense A by explicit loops (small meshes); unknown (i, k) has index
    i*Nz + k.  Written independently of :func:`apply_A`."""
    n_r, n_z = w.shape
    M = np.zeros((n_r * n_z, n_r * n_z))
    for i in range(n_r):
        for k in range(n_z):
            row = i * n_z + k
            out_r = a1[i, k] / hr ** 2                       # face to row i+1 (or the boundary)
            in_r = a1[i - 1, k] / hr ** 2 if i > 0 else 0.0  # face to row i-1 (none at r = 0)
            up_z = a2[i, k - 1] / hz ** 2 if k > 0 else 0.0
            dn_z = a2[i, k] / hz ** 2 if k < n_z - 1 else 0.0
            M[row, row] = out_r + in_r + up_z + dn_z + w[i, k]
            if i + 1 < n_r:
                M[row, row + n_z] = -out_r
            if i > 0:
                M[row, row - n_z] = -in_r
            if k > 0:
                M[row, row - 1] = -up_z
            if k < n_z - 1:
                M[row, row + 1] = -dn_z
    return M


# ---------------------------------------------------------------------------
# Cosine transform along z (the Neumann-Neumann axis)
# ---------------------------------------------------------------------------

def dct2_direct(x: np.ndarray) -> np.ndarray:
    """``C_k = sum_n x_n cos(pi k (2n+1) / (2N))`` along the last axis."""
    n = x.shape[-1]
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    C = np.cos(np.pi * k * (2 * j + 1) / (2 * n))
    return x @ C.T


def dct2(x: np.ndarray) -> np.ndarray:
    """Same as :func:`dct2_direct` through the library FFT of the half-sample
    symmetric extension (length 2N)."""
    n = x.shape[-1]
    ext = np.concatenate([x, x[..., ::-1]], axis=-1)
    Y = np.fft.fft(ext, axis=-1)[..., :n]
    return 0.5 * np.real(np.exp(-1j * np.pi * np.arange(n) / (2 * n)) * Y)


def idct2(c: np.ndarray) -> np.ndarray:
    """Inverse of :func:`dct2`: ``x_n = C_0/N + (2/N) sum_{k>0} C_k cos(pi k (2n+1)/(2N))``."""
    n = c.shape[-1]
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    wts = np.full(n, 2.0 / n)
    wts[0] = 1.0 / n
    Cm = np.cos(np.pi * k * (2 * j + 1) / (2 * n)) * wts[:, None]
    return c @ Cm


def neumann_eigenvalues(nz: int, hz: float) -> np.ndarray:
    """Eigenvalues of -(second difference) with no-flux ends, on the DCT-II
    basis: (4/hz^2) sin^2(pi k / (2 Nz)), k = 0..Nz-1."""
    return (4.0 / hz ** 2) * np.sin(np.pi * np.arange(nz) / (2 * nz)) ** 2


class CylindricalPreconditioner:
    """B of eq. precond1 in the cylindrical form: a1 = rbar kappa~, a2 = r
    kappa~, d = r rho~ h^2/4, inverted by separation of variables: cosine
    transform along z, then for every z-wavenumber one symmetric tridiagonal
    system along r, whose coefficients vary with r (non-Toeplitz), by Thomas."""

    def __init__(self, nr: int, nz: int, hr: float, hz: float, kappa_t: float, rho_t: float, h: float):
        self.nr, self.nz, self.hr, self.hz = nr, nz, hr, hz
        r = radii(nr, hr)
        self.r = r
        self.A1 = (r + 0.5 * hr) * kappa_t / hr ** 2          # face rbar_i coupling
        self.lam = neumann_eigenvalues(nz, hz)
        self.kt = kappa_t
        self.d = r * rho_t * h * h / 4.0
        A1m = np.concatenate([[0.0], self.A1[:-1]])           # face rbar_{i-1} (0 at r = 0)
        # diag[i, k]
        self.diag = (self.A1 + A1m + self.d)[:, None] + (r[:, None] * kappa_t) * self.lam[None, :]
        self.off = -self.A1[:-1]                              # couples rows i and i+1

    def tridiag_solve(self, rhat: np.ndarray) -> np.ndarray:
        """Solve every wavenumber's r-system (axis -2 = i, last axis = k)."""
        from .precond import thomas
        n = self.nr - 1
        lower = np.concatenate([[0.0], self.off])[:, None]
        upper = np.concatenate([self.off, [0.0]])[:, None]
        lower = np.broadcast_to(lower, (n, self.nz))
        upper = np.broadcast_to(upper, (n, self.nz))
        if rhat.ndim == 2:
            return thomas(lower, self.diag, upper, rhat)
        return np.stack([thomas(lower, self.diag, upper, q) for q in rhat])

    def solve(self, r: np.ndarray) -> np.ndarray:
        return idct2(self.tridiag_solve(dct2(r)))

    def apply(self, y: np.ndarray) -> np.ndarray:
        """``B y`` from the same five-point form as A with constant kappa, rho."""
        nr = self.nr
        ones = np.ones((nr, self.nz))
        a1, a2, _ = coefficients(self.kt * ones, ones, 0.0, self.hr)
        return apply_A(y, a1, a2, self.d[:, None] * np.ones((1, self.nz)), self.hr, self.hz)


def preconditioner(kappa: np.ndarray, rho: np.ndarray, h: float, hr: float, hz: float) -> CylindricalPreconditioner:
    """Midrange coefficients (the footnote to eq. precond1) over all nodes."""
    from .precond import midrange
    nr, nz = kappa.shape
    return CylindricalPreconditioner(nr, nz, hr, hz, midrange(kappa), midrange(rho), h)


def source_field(shape, src_ki, value: float, hr: float, hz: float) -> np.ndarray:
    """(1/2 pi) delta_h f_m at the source node (k, i) (1-based paper indices)."""
    f = np.zeros(shape)
    k, i = src_ki
    f[i - 1, k - 1] = value / (2.0 * np.pi * hr * hz)
    return f
