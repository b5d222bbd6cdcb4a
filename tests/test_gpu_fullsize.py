"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (the autotuner's cached tiles).

Where the FP64 oracle can afford the whole problem it is compared output for
output; at 64 shots it checks sampled shots and, for every shot, a property
that holds at any size (the FP64 true residual of the returned solution);
at 4096^2 it compares a fixed number of CG iterations.
"""
import numpy as np
import pytest

from oracle import OK, NOT_CONVERGED
from oracle import elastic, harmonics, krylov, laguerre, operator, precond
from paper_1005_0542_amd import api, inputs, tune
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import log, rel, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def _l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _tuned(w, precision, shots):
    return tune.lookup(w.n_cells, w.n_cells, precision, shots)


def _tiles(t, graph=True):
    keys = ("segments", "graph_iters", "op_shots", "seg_per_wave", "op_fusion") if graph else \
        ("segments", "op_shots", "seg_per_wave", "op_fusion")
    return {k: t.get(k, 0) for k in keys}


def _acoustic_run(name, precision=None, n_harm=2, **kw):
    w = inputs.WORKLOADS[name]
    prec = precision or w.precision
    t = _tuned(w, prec, w.shots)
    log(f"{name} {prec} full size, tiles {t}")
    return AcousticRun(w, precision=prec, n_harm=n_harm, snapshots=False, rec=False, **_tiles(t), **kw)


def _oracle_harmonics(w, kappa, rho, src, n, tol):
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    solve = lambda phi: krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, phi, tol, 10000)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n)
    return harmonics.harmonic_loop(n, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, src, d, d, keep_all=True)


def test_full_acoustic1024_fp64_harmonics():
    """1023^2 unknowns, FP64: the first three harmonics match the oracle to
    1e-12 (relative L2) with identical iteration counts."""
    torch_cuda()
    run = _acoustic_run("acoustic1024", n_harm=3)
    st = _oracle_harmonics(run.w, run.kappa, run.rho, run.src[0], 3, run.tol)
    for m in range(3):
        log(f"acoustic1024 harmonic {m}")
        res = run.step()
        assert res.statuses == [OK]
        assert res.iters[0] == st["iters"][m], (m, res.iters, st["iters"][m])
        e = _l2(run.R.cpu().numpy()[0, 0], st["R"][m])
        print(f"acoustic1024 harmonic {m}: {res.iters[0]} iterations, rel L2 {e:.2e}")
        assert e <= 1e-12


def test_full_acoustic2048x64_mixed_sampled_shots():
    """64 shots on 2047^2 unknowns in mixed precision: two harmonics; shots 0
    and 63 against the FP64 oracle (1e-6 relative L2), every shot's FP64 true
    residual within the tolerance."""
    torch = torch_cuda()
    run = _acoustic_run("acoustic2048x64_mixed", n_harm=2)
    w = run.w
    for m in range(2):
        log(f"acoustic2048x64 harmonic {m}")
        res = run.step()
        assert res.statuses == [OK] * w.shots
    R = run.R.cpu().numpy()[:, 0]
    oracle = {}
    for s in (0, 63):
        oracle[s] = _oracle_harmonics(w, run.kappa, run.rho, run.src[s], 2, 1e-12)
        e = _l2(R[s], oracle[s]["R"][1])
        print(f"acoustic2048x64 shot {s}: rel L2 {e:.2e} (oracle {oracle[s]['iters']} iterations)")
        assert e <= 1e-6
    # every shot: || phi_1 - A R_1 || <= tol || phi_1 || in FP64, with phi_1 the
    # library's right-hand side (itself checked against the oracle on shot 0)
    wv = operator.shift_coeff(run.rho, w.h)
    phi = run.rhs.cpu().numpy()[:, 0]
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, 2)
    sums = harmonics.RunningSums(phi.shape[1:], w.alpha)
    sums.step(0, None)
    src = harmonics.source_field(phi.shape[1:], run.src[0], f_m[1], w.d, w.d)
    phi0 = harmonics.rhs_running(1, sums, oracle[0]["R"][0], run.rho[1:-1, 1:-1], w.h, src)
    assert _l2(phi[0], phi0) <= 1e-6
    worst = 0.0
    for s in range(w.shots):
        r = phi[s] - operator.apply_A(R[s], run.kappa, wv, w.d, w.d)
        worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(phi[s])))
    print(f"acoustic2048x64: worst FP64 true residual over 64 shots {worst:.2e} (tol {w.tol:.0e})")
    assert worst <= 1.5 * w.tol
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_acoustic4096_fixed_iterations(precision):
    """4095^2 unknowns: four CG iterations from x = 0 (tolerance 0) match the
    oracle's four iterations (FP64: 1e-12; mixed: 1e-5, the FP32 level)."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic4096_mixed"]
    kappa, rho = inputs.acoustic_medium_for(w)
    N, d = w.n_cells, w.d
    t = _tuned(w, precision, 1)
    plan = api.Plan("acoustic", N, N, d, d, w.alpha, w.h, 2, np.stack([kappa, rho]), precision=precision,
                    nshots=1, **_tiles(t))
    b = inputs.random_field((N - 1, N - 1), seed=17)
    log(f"acoustic4096 {precision}: 4 iterations, tiles {t}")
    bd = to_dev(b[None, None], torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=0.0, max_iter=4)
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    xo, ito, rro, sto = krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, b, 0.0, 4)
    # tolerance 0 stops every run at the iteration cap; a mixed run is not
    # restarted by its FP64 refinement once the cap has been reached
    assert sto == NOT_CONVERGED and ito == 4
    assert res.statuses == [NOT_CONVERGED] and res.iters == [4]
    e = _l2(to_np(xd)[0, 0], xo)
    print(f"acoustic4096 {precision}: 4 iterations, rel L2 {e:.2e}")
    assert e <= (1e-12 if precision == "fp64" else 1e-5)
    plan.destroy()


def test_full_acoustic4096_mixed_true_residual():
    """4095^2 unknowns, mixed precision to the workload tolerance: the FP64
    true residual of the returned solution meets it."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic4096_mixed"]
    run = _acoustic_run("acoustic4096_mixed", n_harm=1)
    log("acoustic4096 mixed harmonic 0")
    res = run.step()
    assert res.statuses == [OK]
    phi = harmonics.source_field((w.n_cells - 1,) * 2, run.src[0],
                                 laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, 1)[0], w.d, w.d)
    R = run.R.cpu().numpy()[0, 0]
    r = phi - operator.apply_A(R, run.kappa, operator.shift_coeff(run.rho, w.h), w.d, w.d)
    rr = float(np.linalg.norm(r) / np.linalg.norm(phi))
    print(f"acoustic4096 mixed: {res.iters[0]} iterations, FP64 true residual {rr:.2e}")
    assert rr <= 1.5 * w.tol
    torch.cuda.synchronize()


def test_full_kernels_acoustic2048x64_sampled():
    """The three preconditioner/operator calls on all 64 shots at 2047^2,
    sampled shots checked against the oracle (FP32 working type)."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic2048x64_mixed"]
    kappa, rho = inputs.acoustic_medium_for(w)
    N, d, S = w.n_cells, w.d, w.shots
    t = _tuned(w, "mixed", S)
    plan = api.Plan("acoustic", N, N, d, d, w.alpha, w.h, 2, np.stack([kappa, rho]), precision="mixed",
                    nshots=S, **_tiles(t, graph=False))
    xd = torch.from_numpy(inputs.random_field((S, 1, N - 1, N - 1), seed=5).astype(np.float32)).cuda()
    yd = torch.empty_like(xd)
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    samples = (0, 41, 63)
    log("2048x64 stencil")
    plan.stencil_apply(xd, yd)
    for s in samples:
        x = xd[s, 0].double().cpu().numpy()
        assert rel(yd[s, 0].double().cpu().numpy(), operator.apply_A(x, kappa, wv, d, d)) < 2e-5
    log("2048x64 forward DST")
    plan.precond_dst(0, xd, yd)
    for s in samples:
        x = xd[s, 0].double().cpu().numpy()
        assert rel(yd[s, 0].double().cpu().numpy(), precond.dst1(x, N)) < 5e-5
    log("2048x64 Dichotomy")
    plan.precond_dichotomy_tdma(0, xd, yd)
    for s in samples:
        x = xd[s, 0].double().cpu().numpy()
        assert rel(yd[s, 0].double().cpu().numpy(), B.tridiag_solve(x)) < 5e-5
    plan.destroy()


def test_full_elastic1024_gmres():
    """Elastic 1023^2 x 2 unknowns, FP64 GMRES(10): the first harmonic matches
    the oracle's GMRES(10) (iterations within one, solution to 1e-8) and its
    FP64 true residual meets the tolerance; run for exactly the oracle's
    iteration count it matches to 1e-12."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["elastic1024"]
    lam, mu, rho = inputs.elastic_medium_for(w)
    N, d = w.n_cells, w.d
    plan = api.Plan("elastic", N, N, d, d, w.alpha, w.h, 2, np.stack([lam, mu, rho]), precision="fp64", nshots=1)
    src = inputs.sources_for(w)
    plan.set_sources(src)
    f = api.source_coeffs(w.f0, w.t0, w.alpha, w.h, 1)
    shape = (1, 2, N - 1, N - 1)
    R, Ph, Qh, rhs = (torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(4))
    log("elastic1024 harmonic 0")
    plan.laguerre_rhs(0, None, Ph, Qh, [f[0]], rhs)
    res = plan.gmres_solve(rhs, R, tol=w.tol, max_iter=5000, restart=10)
    assert res.statuses == [OK]
    fo = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, 1)
    phi = np.zeros((2, N - 1, N - 1))
    phi[1] = harmonics.source_field((N - 1, N - 1), src[0], fo[0], d, d)
    assert rel(to_np(rhs)[0], phi) < 1e-12
    wv = rho[1:-1, 1:-1] * w.h * w.h / 4
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, w.h, N, N, d, d)
    C = lambda u: elastic.apply_C(u, lam, mu, wv, d, d)
    xo, ito, rro, sto = krylov.gmres(C, lambda u: elastic.apply_Kinv(u, B1, B2), phi, w.tol, 10)
    x = to_np(R)[0]
    e = _l2(x, xo)
    rr = float(np.linalg.norm(phi - C(x)) / np.linalg.norm(phi))
    print(f"elastic1024: {res.iters[0]} iterations (oracle {ito}), rel L2 {e:.2e}, true residual {rr:.2e}")
    assert sto == OK and abs(res.iters[0] - ito) <= 1
    assert e <= 1e-8 and rr <= 10 * w.tol
    # the same harmonic run for exactly the oracle's iteration count (tol = 0):
    # the same Krylov minimiser, equal to rounding
    log(f"elastic1024 harmonic 0, fixed {ito} iterations")
    resf = plan.gmres_solve(rhs, R, tol=0.0, max_iter=ito, restart=10)
    ef = _l2(to_np(R)[0], xo)
    print(f"elastic1024 fixed {ito} iterations: rel L2 {ef:.2e}")
    assert resf.iters == [ito] and ef <= 1e-12
    plan.destroy()
