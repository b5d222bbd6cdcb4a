"""End-to-end harmonic loop on the GPU against the FP64 oracle: every harmonic
of the 64x64 two-layer workload, the synthesized snapshots and traces, the
mixed-precision wavefield error, batching and checkpoint/resume."""
import numpy as np
import pytest

from oracle import operator, precond, krylov, harmonics, laguerre
from paper_1005_0542_amd import inputs
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import log, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_run(run, n, tol=1e-10, keep_all=True):
    w = run.w
    kappa, rho = run.kappa, run.rho
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    solve = lambda phi: krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, phi, tol, 10000)
    W = laguerre.synthesis_weights(inputs.snapshot_times(w), w.h, w.alpha, n)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n)      # the oracle's own coefficients
    return harmonics.harmonic_loop(n, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, run.src[0], d, d,
                                   snap_w=W, rec_row=w.rec_row, keep_all=keep_all)


def _errors(run, st, n):
    torch = torch_cuda()
    snap = run.snap.cpu().numpy()[:, 0, 0]
    t = inputs.trace_times(run.w)
    tr = run.traces(t).cpu().numpy()[0, 0]
    Wt = laguerre.synthesis_weights(t, run.w.h, run.w.alpha, n)
    tr_ref = harmonics.traces(np.array(st["rec"]), Wt)
    return (np.linalg.norm(snap - st["snap"]) / np.linalg.norm(st["snap"]),
            np.linalg.norm(tr - tr_ref) / np.linalg.norm(tr_ref))


def test_acoustic64_all_harmonics_fp64():
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic64"]
    run = AcousticRun(w)
    st = _oracle_run(run, w.n_harm)
    worst = 0.0
    for m in range(w.n_harm):
        log(f"acoustic64 fp64 harmonic {m}")
        res = run.step()
        R = run.R.cpu().numpy()[0, 0]
        Ro = st["R"][m]
        den = max(np.linalg.norm(Ro), 1e-30 * max(np.linalg.norm(r) for r in st["R"]))
        e_m = np.linalg.norm(R - Ro) / den
        worst = max(worst, e_m)
        assert res.iters[0] == st["iters"][m], (m, res.iters, st["iters"][m])
        assert e_m <= 1e-12, (m, e_m)
    es, et = _errors(run, st, w.n_harm)
    print(f"fp64: worst per-harmonic error {worst:.2e}, snapshots {es:.2e}, traces {et:.2e}")
    assert es <= 1e-12 and et <= 1e-12


@pytest.mark.parametrize("name,n,crop", [("acoustic64", 64, None), ("acoustic1024", 96, 256)])
def test_mixed_precision_wavefield_error(name, n, crop):
    """Mixed precision (FP32 operator, transform and tridiagonal solves; FP64
    Krylov scalars, residual refinement, recurrence and synthesis) against the
    FP64 oracle (tol 1e-10): the synthesized wavefield must agree to 1e-6.
    The solve tolerance, not the FP32 arithmetic, sets this error (FP64 and
    mixed runs at the same tolerance agree), so the mixed workloads use 1e-9."""
    torch = torch_cuda()
    w0 = inputs.WORKLOADS[name]
    w = w0 if crop is None else inputs.Workload(**{**w0.__dict__, "name": name + "_crop",
                                                   "n_cells": crop, "src": (crop // 2, 8)})
    run = AcousticRun(w, precision="mixed", n_harm=n, tol=1e-9, max_iter=1000)
    st = _oracle_run(run, n, keep_all=False)
    for m in range(n):
        run.step()
    es, et = _errors(run, st, n)
    print(f"{name} mixed ({w.n_cells}^2, {n} harmonics): snapshot error {es:.2e}, trace error {et:.2e}")
    assert es <= 1e-6 and et <= 1e-6


def test_batched_shots_equal_single_shots_over_harmonics():
    torch = torch_cuda()
    w = inputs.Workload(**{**inputs.WORKLOADS["acoustic2048x64_mixed"].__dict__, "n_cells": 128, "d": 20.0,
                           "precision": "fp64", "tol": 1e-10, "shots": 4})
    batch = AcousticRun(w, n_harm=6)
    for _ in range(6):
        batch.step()
    for s in range(4):
        single = AcousticRun(w, shots=1, n_harm=6)
        single.plan.set_sources(batch.src[s:s + 1])
        for _ in range(6):
            single.step()
        assert [i[0] for i in single.iters] == [i[s] for i in batch.iters]
        assert np.array_equal(single.R.cpu().numpy()[0], batch.R.cpu().numpy()[s])
        assert np.array_equal(single.snap.cpu().numpy()[:, 0], batch.snap.cpu().numpy()[:, s])


def test_checkpoint_resume_bitwise():
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic64"]
    full = AcousticRun(w, n_harm=20)
    for _ in range(20):
        full.step()
    part = AcousticRun(w, n_harm=20)
    for _ in range(9):
        part.step()
    ck = part.state_dict()
    del part
    resumed = AcousticRun(w, n_harm=20)
    resumed.load_state_dict(ck)
    for _ in range(11):
        resumed.step()
    assert resumed.iters == full.iters
    for name in ("R", "Ph", "Qh", "snap", "rec"):
        assert torch.equal(getattr(resumed, name), getattr(full, name)), name
