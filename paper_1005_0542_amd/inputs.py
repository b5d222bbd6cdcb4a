"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module only *generates data*: grids, media, source positions and the
workload parameters.  It holds none of the method's arithmetic (no operator,
no transform, no solver, no Laguerre quantity), so both sides of every parity
check can draw their inputs from here without sharing any of the computation.

Array conventions
-----------------
* A grid of ``N`` cells per axis has nodes ``i, j = 0..N``; node arrays have
  shape ``(N+1, N+1)`` indexed ``[j, i]`` (``j`` = depth index, ``i`` = x index,
  x fastest in memory).
* The unknowns of the Dirichlet problem are the ``(N-1)**2`` interior nodes.

Media (the paper's Marmousi model is not available; these layered and
perturbed media stand in for it, with the paper's velocity and density ranges)
* acoustic: a velocity ``v``; the constant-density reading of the acoustic
  equation ``rho u_tt = div(kappa grad u) + delta f`` is ``kappa = 1``,
  ``rho = 1 / v**2``.  A variable-density test medium uses
  ``kappa = 1/rho_phys``, ``rho = 1/(rho_phys v**2)`` with Gardner's density.
* elastic: ``Vp``, ``Vs = Vp/1.73`` and the physical density give the Lame
  parameters ``lambda = rho (Vp^2 - 2 Vs^2)``, ``mu = rho Vs^2``.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "layered_velocity", "correlated_noise",
    "perturbed_layered_velocity", "two_layer_velocity", "acoustic_coeffs",
    "variable_density_coeffs", "elastic_coeffs", "shot_positions",
    "acoustic_medium_for", "elastic_medium_for", "random_field",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named synthetic workload (grid, medium recipe, source, expansion)."""
    name: str
    kind: str            # "acoustic" | "elastic"
    n_cells: int         # N cells per axis (nodes 0..N)
    d: float             # dx = dz in metres
    medium: str          # "two_layer" | "layered_perturbed" | "elastic_layered"
    f0: float            # Ricker peak frequency (Hz)
    alpha: int           # Laguerre order
    h: float             # Laguerre scale parameter (1/s)
    n_harm: int          # number of harmonics
    T: float             # final time (s)
    precision: str       # "fp64" | "mixed"
    tol: float
    shots: int
    src: Optional[Tuple[int, int]] = None   # (i, j) for single-shot workloads
    src_row: int = 8
    rec_row: int = 8
    noise_seed: int = 1
    rho_seed: int = 2
    shot_seed: int = 3

    @property
    def t0(self) -> float:
        # Ricker delay: 1.5 periods, so f(0) is ~1e-8 of the peak.
        return 1.5 / self.f0

    @property
    def unknowns(self) -> int:
        return (self.n_cells - 1) ** 2


WORKLOADS: Dict[str, Workload] = {
    "acoustic64": Workload(
        name="acoustic64", kind="acoustic", n_cells=64, d=10.0, medium="two_layer",
        f0=15.0, alpha=9, h=200.0, n_harm=64, T=0.4, precision="fp64", tol=1e-10,
        shots=1, src=(32, 8)),
    "acoustic1024": Workload(
        name="acoustic1024", kind="acoustic", n_cells=1024, d=5.0, medium="layered_perturbed",
        f0=25.0, alpha=9, h=400.0, n_harm=512, T=1.0, precision="fp64", tol=1e-10,
        shots=1, src=(512, 8)),
    "elastic1024": Workload(
        name="elastic1024", kind="elastic", n_cells=1024, d=5.0, medium="elastic_layered",
        f0=20.0, alpha=8, h=300.0, n_harm=256, T=0.6, precision="fp64", tol=1e-10,
        shots=1, src=(512, 8)),
    "acoustic4096_mixed": Workload(
        name="acoustic4096_mixed", kind="acoustic", n_cells=4096, d=2.5,
        medium="layered_perturbed", f0=30.0, alpha=9, h=600.0, n_harm=1024, T=2.0,
        precision="mixed", tol=1e-9, shots=1, src=(2048, 8)),
    "acoustic2048x64_mixed": Workload(
        name="acoustic2048x64_mixed", kind="acoustic", n_cells=2048, d=5.0,
        medium="layered_perturbed", f0=25.0, alpha=9, h=400.0, n_harm=512, T=1.0,
        precision="mixed", tol=1e-9, shots=64),
}


def layered_velocity(n_cells: int, v_top: float, v_bottom: float, n_layers: int = 5) -> np.ndarray:
    """Node array of ``n_layers`` equal-thickness horizontal layers whose
    velocities rise linearly from ``v_top`` to ``v_bottom``."""
    j = np.arange(n_cells + 1)
    layer = np.minimum((j * n_layers) // n_cells, n_layers - 1)
    vel = np.linspace(v_top, v_bottom, n_layers)[layer]
    return np.repeat(vel[:, None], n_cells + 1, axis=1).astype(np.float64)


def correlated_noise(n_cells: int, d: float, seed: int, corr_len: float = 50.0) -> np.ndarray:
    """Standardised Gaussian-correlated noise, clipped to +-3.

    White N(0,1) noise from ``numpy.random.default_rng(seed)`` smoothed by a
    separable Gaussian of standard deviation ``corr_len/2`` (so the field's
    autocorrelation is ``exp(-r^2/corr_len^2)``), truncated at 4 sigma with
    reflect padding, then standardised and clipped.
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal((n_cells + 1, n_cells + 1))
    sigma_cells = 0.5 * corr_len / d
    eps = gaussian_filter(eps, sigma=sigma_cells, mode="reflect", truncate=4.0)
    eps = (eps - eps.mean()) / eps.std()
    return np.clip(eps, -3.0, 3.0)


def perturbed_layered_velocity(n_cells: int, d: float, v_top: float, v_bottom: float,
                               seed: int, rel_std: float = 0.10) -> np.ndarray:
    """Five layers plus a 10 % Gaussian-correlated perturbation (50 m)."""
    v = layered_velocity(n_cells, v_top, v_bottom)
    return v * (1.0 + rel_std * correlated_noise(n_cells, d, seed))


def two_layer_velocity(n_cells: int, j_interface: int, v_top: float, v_bottom: float) -> np.ndarray:
    """Velocity ``v_top`` for node rows ``j < j_interface``, ``v_bottom`` below."""
    v = np.full((n_cells + 1, n_cells + 1), v_bottom, dtype=np.float64)
    v[:j_interface, :] = v_top
    return v


def acoustic_coeffs(v: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Constant-density acoustic coefficients: ``kappa = 1``, ``rho = 1/v^2``."""
    return np.ones_like(v), 1.0 / (v * v)


def variable_density_coeffs(v: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Variable-density acoustic coefficients with Gardner's density
    ``rho_phys = 310 v^0.25``: ``kappa = 1/rho_phys``, ``rho = 1/(rho_phys v^2)``."""
    rho_phys = 310.0 * v ** 0.25
    return 1.0 / rho_phys, 1.0 / (rho_phys * v * v)


def elastic_coeffs(vp: np.ndarray, rho_phys: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Lame parameters with ``Vs = Vp/1.73``: returns ``(lambda, mu, rho)``."""
    vs = vp / 1.73
    mu = rho_phys * vs * vs
    lam = rho_phys * (vp * vp - 2.0 * vs * vs)
    return lam, mu, rho_phys.copy()


def shot_positions(n_cells: int, shots: int, seed: int = 3, row: int = 8) -> np.ndarray:
    """``shots`` distinct surface source columns drawn without replacement
    from ``[N/16, 15N/16]``; returns an int32 array ``[shots, 2]`` of ``(i, j)``."""
    rng = np.random.default_rng(seed)
    lo, hi = n_cells // 16, (15 * n_cells) // 16
    cols = rng.choice(np.arange(lo, hi + 1), size=shots, replace=False)
    out = np.empty((shots, 2), dtype=np.int32)
    out[:, 0] = cols
    out[:, 1] = row
    return out


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random FP64 test vector (for operator/transform parity cases)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def acoustic_medium_for(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """``(kappa, rho)`` node arrays of shape ``(N+1, N+1)`` for an acoustic workload."""
    n = w.n_cells
    if w.medium == "two_layer":
        v = two_layer_velocity(n, 32 * n // 64, 2000.0, 3000.0)
    elif w.medium == "layered_perturbed":
        v = perturbed_layered_velocity(n, w.d, 1500.0, 4000.0, w.noise_seed)
    else:
        raise ValueError(w.medium)
    return acoustic_coeffs(v)


def elastic_medium_for(w: Workload) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """``(lambda, mu, rho)`` node arrays for an elastic workload."""
    n = w.n_cells
    vp = perturbed_layered_velocity(n, w.d, 2000.0, 4500.0, w.noise_seed)
    rho = perturbed_layered_velocity(n, w.d, 2000.0, 2600.0, w.rho_seed)
    return elastic_coeffs(vp, rho)


def sources_for(w: Workload) -> np.ndarray:
    """int32 ``[shots, 2]`` source nodes ``(i, j)``."""
    if w.shots == 1 and w.src is not None:
        return np.array([w.src], dtype=np.int32)
    return shot_positions(w.n_cells, w.shots, w.shot_seed, w.src_row)


def snapshot_times(w: Workload) -> List[float]:
    return [w.T * q / 4.0 for q in (1, 2, 3, 4)]


def trace_times(w: Workload, dt: float = 1e-3) -> np.ndarray:
    nt = int(round(w.T / dt)) + 1
    return np.arange(nt) * dt
