"""FP64 oracle harmonic chains of a workload's shots, for the full-size GPU
tests (CPU only: imports the oracle and the neutral input generators, never
torch, so it can run in worker processes beside the GPU process)."""
import numpy as np

from oracle import harmonics, krylov, laguerre, operator, precond
from paper_1005_0542_amd import inputs


def oracle_chain(name, shot, n_harm, tol):
    """The oracle's own chain for one shot of workload `name`: every R_m, the
    CG iteration counts and the partial snapshots after n_harm harmonics."""
    w = inputs.WORKLOADS[name]
    kappa, rho = inputs.acoustic_medium_for(w)
    N, d = w.n_cells, w.d
    src = inputs.sources_for(w)[shot]
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    solve = lambda phi: krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, phi, tol, 10000)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n_harm)
    t_snap = np.array(inputs.snapshot_times(w))
    W = laguerre.synthesis_weights(t_snap, w.h, w.alpha, n_harm)            # [n_snap, n]
    st = harmonics.harmonic_loop(n_harm, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, src, d, d, snap_w=W,
                                 keep_all=True)
    return {"R": st["R"], "iters": st["iters"], "status": st["status"], "snap": st["snap"]}


def oracle_elastic_chain(name, n_harm, tol):
    """The oracle's own elastic chain (GMRES(10), K = diag(B1, B2)) for the
    workload's shot: every R_m and its inner iteration count."""
    from oracle import elastic
    w = inputs.WORKLOADS[name]
    lam, mu, rho = inputs.elastic_medium_for(w)
    N, d = w.n_cells, w.d
    src = inputs.sources_for(w)[0]
    wv = rho[1:-1, 1:-1] * w.h * w.h / 4
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, w.h, N, N, d, d)
    C = lambda u: elastic.apply_C(u, lam, mu, wv, d, d)
    K = lambda u: elastic.apply_Kinv(u, B1, B2)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n_harm)
    shape = (2, N - 1, N - 1)
    sums = harmonics.RunningSums(shape, w.alpha)
    Rs, its, Rp = [], [], None
    for m in range(n_harm):
        src_f = np.zeros(shape)
        src_f[1] = harmonics.source_field(shape[1:], src, f_m[m], d, d)
        phi = src_f - w.h * w.h * rho[1:-1, 1:-1][None] * sums.step(m, Rp)
        R, it, _, st = krylov.gmres(C, K, phi, tol, 10)
        assert st == 0
        Rs.append(R)
        its.append(it)
        Rp = R
    return {"R": Rs, "iters": its}
