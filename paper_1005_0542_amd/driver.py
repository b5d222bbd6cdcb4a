"""Harmonic loop of the Laguerre method on the HIP library (product path).

For harmonics m = 0, 1, ... (strictly in order, eq. laguerre_h):
  1. ``lg_laguerre_rhs``        right-hand side from the running history sums;
  2. ``lg_pcg_solve``           A R_m = rhs by preconditioned CG (all shots);
  3. ``lg_laguerre_synthesize`` snapshots += W_m(t_s) R_m, receiver-row store.
Traces are formed at the end with ``lg_trace_synthesize``.  Everything runs in
the library's kernels; this module only allocates the buffers and sequences
the calls.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import api, inputs


class AcousticRun:
    """One workload on one GPU: medium, sources, buffers, plan.

    ``geometry="cylindrical"`` runs the 2.5D axisymmetric problem on an
    N_r x N_z = N x N mesh (Sec. 2.3): the workload's layered medium with its
    depth axis along z, fields [shots][1][N-1][N] with z fastest, and every
    source on the axis (row i = 1) at the depth index the Cartesian recipe
    gives as its x position."""

    def __init__(self, w: inputs.Workload, precision: Optional[str] = None, shots: Optional[int] = None,
                 n_harm: Optional[int] = None, segments: int = 0, graph_iters: int = 0,
                 snapshots: bool = True, rec: bool = True, tol: Optional[float] = None,
                 max_iter: int = 10000, medium=None, op_shots: int = 0, seg_per_wave: int = 0,
                 op_fusion: int = 0, top: str = "dirichlet", warm_start: bool = False,
                 geometry: str = "cartesian", order: int = 2, x_ring: int = 0, synth_batch: int = 4):
        import torch
        self.torch = torch
        self.w = w
        self.precision = precision or w.precision
        self.shots = shots or w.shots
        self.n_harm = n_harm or w.n_harm
        self.tol = w.tol if tol is None else tol
        if self.precision == "fp64" and tol is None:
            self.tol = min(self.tol, 1e-10)
        self.max_iter = max_iter
        self.warm_start = warm_start      # start each solve from the previous harmonic
        N = w.n_cells
        cyl = geometry == "cylindrical"
        self.geometry = geometry
        if medium is not None:
            kappa, rho = medium
        else:
            kappa, rho = inputs.acoustic_medium_for(w)
            if cyl:   # node arrays [N_r][N_z], depth along z
                kappa = np.ascontiguousarray(kappa[:N, :N].T)
                rho = np.ascontiguousarray(rho[:N, :N].T)
        self.kappa, self.rho = kappa, rho
        self.plan = api.Plan("acoustic", N, N, w.d, w.d, w.alpha, w.h, self.n_harm,
                             np.stack([kappa, rho]), precision=self.precision, nshots=self.shots,
                             segments=segments, graph_iters=graph_iters, op_shots=op_shots,
                             seg_per_wave=seg_per_wave, op_fusion=op_fusion, top=top, geometry=geometry,
                             order=order, x_ring=x_ring)
        if self.shots == w.shots:
            src = inputs.sources_for(w)
        else:
            src = inputs.shot_positions(N, self.shots, w.shot_seed, w.src_row) if self.shots > 1 \
                else np.array([w.src or (N // 2, w.src_row)], dtype=np.int32)
        if cyl:       # (depth index k, axis row 1)
            src = np.ascontiguousarray(np.stack([src[:, 0], np.ones(len(src), dtype=np.int32)], axis=1),
                                       dtype=np.int32)
        self.src = src
        self.plan.set_sources(src)
        self.f_m = api.source_coeffs(w.f0, w.t0, w.alpha, w.h, self.n_harm)
        self.t_snap = inputs.snapshot_times(w)
        self.W_snap = api.laguerre_weights(self.t_snap, w.alpha, w.h, self.n_harm)   # [4, n]
        dev = "cuda"
        ncol = N if cyl else N - 1          # row length
        self.ncol = ncol
        shape = (self.shots, 1, N - 1, ncol)
        f64 = torch.float64
        # The synthesis of `synth_batch` consecutive harmonics runs as one pass
        # (lg_laguerre_synthesize_batch: the snapshots are read and written
        # once per batch, bitwise the same sums), so the solutions R_m of a
        # batch are kept in a ring; `snap`, `rec`, `traces` and checkpoints
        # first synthesize the harmonics still pending.
        self.synth_batch = max(1, min(int(synth_batch), 8)) if (snapshots or rec) else 1
        self._Rs = [torch.zeros(shape, dtype=f64, device=dev) for _ in range(self.synth_batch)]
        self._pending: List[int] = []
        self.Ph = torch.zeros(shape, dtype=f64, device=dev)
        self.Qh = torch.zeros(shape, dtype=f64, device=dev)
        self.rhs = torch.zeros(shape, dtype=f64, device=dev)
        self._snap = torch.zeros((len(self.t_snap),) + shape, dtype=f64, device=dev) if snapshots else None
        self._rec = torch.zeros((self.shots, 1, self.n_harm, ncol), dtype=f64, device=dev) if rec else None
        self.iters: List[List[int]] = []
        self.status: List[int] = []
        self.m = 0

    @property
    def R(self):
        """The latest solution R_{m-1} (before the first step: a zero vector)."""
        return self._Rs[(self.m - 1) % self.synth_batch] if self.m > 0 else self._Rs[0]

    @property
    def snap(self):
        self.finish()
        return self._snap

    @property
    def rec(self):
        self.finish()
        return self._rec

    def finish(self) -> None:
        """Synthesize the harmonics still pending (the rest of a batch)."""
        if not self._pending or (self._snap is None and self._rec is None):
            self._pending = []
            return
        m0, nb = self._pending[0], len(self._pending)
        Rs = [self._Rs[m % self.synth_batch] for m in self._pending]
        W = self.W_snap[:, m0:m0 + nb] if self._snap is not None else np.zeros((0, nb))
        self.plan.laguerre_synthesize_batch(m0, Rs, W, self._snap, self.w.rec_row, self._rec)
        self._pending = []

    def step(self) -> api.SolveResult:
        """Advance one harmonic (rhs, solve; the synthesis once per batch)."""
        m = self.m
        fs = np.full(self.shots, self.f_m[m])
        R_prev = self._Rs[(m - 1) % self.synth_batch] if m else None
        R = self._Rs[m % self.synth_batch]
        self.plan.laguerre_rhs(m, R_prev, self.Ph, self.Qh, fs, self.rhs)
        warm = self.warm_start and m > 0
        if warm and R is not R_prev:
            R.copy_(R_prev)
        res = self.plan.pcg_solve(self.rhs, R, tol=self.tol, max_iter=self.max_iter, x0_given=warm)
        self._pending.append(m)
        if len(self._pending) == self.synth_batch:
            self.finish()
        self.iters.append(res.iters)
        self.status.append(res.status)
        self.m += 1
        return res

    # -- checkpoint / resume ----------------------------------------------------
    def state_dict(self) -> dict:
        """Complete harmonic-loop state: the next harmonic m, the last solution
        R_{m-1}, the running history sums, the snapshot accumulators and the
        receiver coefficients (device tensors are copied to the host)."""
        self.finish()
        out = {"m": self.m, "iters": [list(i) for i in self.iters], "status": list(self.status),
               "R": self.R.cpu(), "Ph": self.Ph.cpu(), "Qh": self.Qh.cpu()}
        if self._snap is not None:
            out["snap"] = self._snap.cpu()
        if self._rec is not None:
            out["rec"] = self._rec.cpu()
        return out

    def load_state_dict(self, st: dict) -> None:
        self.m = int(st["m"])
        self.iters = [list(i) for i in st["iters"]]
        self.status = list(st["status"])
        self._pending = []
        for name, t in (("R", self.R), ("Ph", self.Ph), ("Qh", self.Qh), ("snap", self._snap), ("rec", self._rec)):
            if t is not None and name in st:
                t.copy_(st[name].to(t.device))

    def traces(self, t: np.ndarray):
        W = api.laguerre_weights(t, self.w.alpha, self.w.h, self.n_harm)
        out = self.torch.zeros((self.shots, 1, len(t), self.ncol), dtype=self.torch.float64, device="cuda")
        self.plan.trace_synthesize(self.rec, W, out)
        return out


class ElasticRun:
    """The elastic harmonic loop on one GPU (eq. elastic_problemQn): for each
    harmonic the right-hand side from the running sums of both displacement
    components, right-preconditioned GMRES(k) with K = diag(B1, B2), and the
    synthesis.  Vectors are [shots][2][nz-1][nx-1] (u_x, u_z).  ``top="free"``:
    the traction-free surface on the first unknown row (Sec. 2.2)."""

    def __init__(self, w: inputs.Workload, shots: Optional[int] = None, n_harm: Optional[int] = None,
                 restart: int = 10, tol: Optional[float] = None, max_iter: int = 10000, snapshots: bool = True,
                 rec: bool = True, segments: int = 0, top: str = "dirichlet"):
        import torch
        self.torch = torch
        self.w = w
        self.shots = shots or w.shots
        self.n_harm = n_harm or w.n_harm
        self.restart = restart
        self.tol = w.tol if tol is None else tol
        self.max_iter = max_iter
        N = w.n_cells
        lam, mu, rho = inputs.elastic_medium_for(w)
        self.lam, self.mu, self.rho = lam, mu, rho
        self.plan = api.Plan("elastic", N, N, w.d, w.d, w.alpha, w.h, self.n_harm, np.stack([lam, mu, rho]),
                             precision="fp64", nshots=self.shots, segments=segments, top=top)
        src = inputs.sources_for(w) if self.shots == w.shots else \
            inputs.shot_positions(N, self.shots, w.shot_seed, w.src_row)
        self.src = src
        self.plan.set_sources(src)
        self.f_m = api.source_coeffs(w.f0, w.t0, w.alpha, w.h, self.n_harm)
        self.t_snap = inputs.snapshot_times(w)
        self.W_snap = api.laguerre_weights(self.t_snap, w.alpha, w.h, self.n_harm)
        shape = (self.shots, 2, N - 1, N - 1)
        f64 = torch.float64
        self.R, self.Ph, self.Qh, self.rhs = (torch.zeros(shape, dtype=f64, device="cuda") for _ in range(4))
        self.snap = torch.zeros((len(self.t_snap),) + shape, dtype=f64, device="cuda") if snapshots else None
        self.rec = torch.zeros((self.shots, 2, self.n_harm, N - 1), dtype=f64, device="cuda") if rec else None
        self.iters: List[List[int]] = []
        self.status: List[int] = []
        self.m = 0

    def step(self) -> api.SolveResult:
        m = self.m
        fs = np.full(self.shots, self.f_m[m])
        self.plan.laguerre_rhs(m, self.R if m else None, self.Ph, self.Qh, fs, self.rhs)
        res = self.plan.gmres_solve(self.rhs, self.R, tol=self.tol, max_iter=self.max_iter, restart=self.restart)
        if self.snap is not None or self.rec is not None:
            ws = self.W_snap[:, m] if self.snap is not None else []
            self.plan.laguerre_synthesize(m, self.R, ws, self.snap, self.w.rec_row, self.rec)
        self.iters.append(res.iters)
        self.status.append(res.status)
        self.m += 1
        return res
