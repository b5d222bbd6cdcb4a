"""GPU parity of the free-surface top boundary (Sec. 2.1, eq. boundary_cond:
du/dz = 0 at z = 0, flux-free face above the first row) against the FP64
oracle: operator, the rank-one corrected Dichotomy solve, the preconditioner,
PCG and a whole harmonic chain."""
import numpy as np
import pytest

from oracle import OK, operator, precond, krylov, harmonics, laguerre
from paper_1005_0542_amd import api, inputs
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import heterogeneous, log, rel, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(nx, nz, kappa, rho, h=200.0, precision="fp64", shots=1, segments=0, dx=10.0, dz=10.0, **kw):
    return api.Plan("acoustic", nx, nz, dx, dz, 9, h, 8, np.stack([kappa, rho]), precision=precision,
                    nshots=shots, segments=segments, top="free", **kw)


def _wdt(prec):
    torch = torch_cuda()
    return torch.float64 if prec == "fp64" else torch.float32


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,nz,shots", [(16, 16, 1), (64, 32, 3), (2, 4, 1), (128, 256, 2)])
def test_free_surface_stencil_parity(prec, nx, nz, shots):
    kappa, rho = heterogeneous(nx, nz)
    h = 300.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision=prec, shots=shots, dx=7.0, dz=5.0)
    x = np.random.default_rng(nx + 3 * nz).standard_normal((shots, nz - 1, nx - 1))
    log(f"free-surface stencil {prec} {nx}x{nz} shots={shots}")
    xd = to_dev(x, _wdt(prec))
    yd = torch_cuda().empty_like(xd)
    plan.stencil_apply(xd, yd)
    ref = operator.apply_A(to_np(xd), kappa, operator.shift_coeff(rho, h), 7.0, 5.0, free_top=True)
    assert rel(to_np(yd), ref) < (1e-13 if prec == "fp64" else 2e-5)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,nz,P", [(16, 16, 1), (16, 16, 4), (8, 64, 2), (8, 64, 32), (64, 1024, 16),
                                     (64, 1024, 64), (4, 2, 1)])
def test_free_surface_tdma_parity(prec, nx, nz, P):
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision=prec, shots=2, segments=P)
    B = precond.acoustic_preconditioner(kappa, rho, h, nx, nz, 10.0, 10.0, free_top=True)
    rhs = np.random.default_rng(P + nz).standard_normal((2, nz - 1, nx - 1))
    log(f"free-surface tdma {prec} nx={nx} nz={nz} P={P}")
    rd = to_dev(rhs, _wdt(prec))
    sd = torch_cuda().empty_like(rd)
    plan.precond_dichotomy_tdma(0, rd, sd)
    ref = B.tridiag_solve(to_np(rd))
    assert rel(to_np(sd), ref) < (1e-12 if prec == "fp64" else 5e-5)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,nz,P", [(16, 16, 1), (64, 64, 4), (256, 256, 16)])
def test_free_surface_precond_apply_parity(prec, nx, nz, P):
    kappa, rho = heterogeneous(nx, nz)
    h = 300.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision=prec, segments=P, dx=5.0, dz=5.0)
    B = precond.acoustic_preconditioner(kappa, rho, h, nx, nz, 5.0, 5.0, free_top=True)
    r = np.random.default_rng(nx).standard_normal((1, nz - 1, nx - 1))
    log(f"free-surface precond_apply {prec} {nx}x{nz} P={P}")
    rd = to_dev(r, _wdt(prec))
    zd = torch_cuda().empty_like(rd)
    plan.precond_apply(rd, zd)
    assert rel(to_np(zd)[0], B.solve(to_np(rd)[0])) < (1e-12 if prec == "fp64" else 5e-5)


def _oracle_pcg(kappa, rho, h, nx, nz, b, tol, max_iter=500, dx=10.0, dz=10.0):
    w = operator.shift_coeff(rho, h)
    B = precond.acoustic_preconditioner(kappa, rho, h, nx, nz, dx, dz, free_top=True)
    return krylov.pcg(lambda y: operator.apply_A(y, kappa, w, dx, dz, free_top=True), B.solve, b, tol, max_iter)


@pytest.mark.parametrize("nx,nz,P,fus", [(64, 64, 4, 1), (64, 64, 1, 2), (128, 256, 8, 1), (1024, 256, 16, 1),
                                         (32, 128, 32, 2)])
def test_free_surface_pcg_parity_fp64(nx, nz, P, fus):
    torch = torch_cuda()
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = _plan(nx, nz, kappa, rho, h=h, segments=P, op_fusion=fus)
    b = np.random.default_rng(6).standard_normal((nz - 1, nx - 1))
    xo, ito, rro, sto = _oracle_pcg(kappa, rho, h, nx, nz, b, 1e-10)
    log(f"free-surface pcg fp64 {nx}x{nz} P={P} op_fusion={fus}")
    bd = to_dev(b[None], torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=1e-10, max_iter=500)
    assert res.statuses == [OK] and sto == OK
    assert res.iters[0] == ito
    assert rel(to_np(xd)[0], xo) < 1e-12


@pytest.mark.parametrize("nx,nz", [(64, 64), (512, 256)])
def test_free_surface_pcg_mixed_true_residual(nx, nz):
    torch = torch_cuda()
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision="mixed", shots=2)
    b = np.random.default_rng(7).standard_normal((2, nz - 1, nx - 1))
    log(f"free-surface pcg mixed {nx}x{nz}")
    bd = to_dev(b, torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=1e-9, max_iter=500)
    assert res.statuses == [OK, OK]
    w = operator.shift_coeff(rho, h)
    for s in range(2):
        r = b[s] - operator.apply_A(to_np(xd)[s], kappa, w, 10.0, 10.0, free_top=True)
        assert np.linalg.norm(r) <= 1.5e-9 * np.linalg.norm(b[s])
        xo = _oracle_pcg(kappa, rho, h, nx, nz, b[s], 1e-12)[0]
        assert rel(to_np(xd)[s], xo) < 1e-6


def test_free_surface_harmonic_chain_fp64():
    """All 64 harmonics of the 64^2 two-layer workload with a free surface:
    per-harmonic 1e-12, identical iteration counts, snapshots 1e-12."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic64"]
    run = AcousticRun(w, top="free")
    kappa, rho = run.kappa, run.rho
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d, free_top=True)
    solve = lambda phi: krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d, free_top=True), B.solve,
                                   phi, 1e-10, 10000)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, w.n_harm)
    Ws = laguerre.synthesis_weights(np.array(inputs.snapshot_times(w)), w.h, w.alpha, w.n_harm)
    st = harmonics.harmonic_loop(w.n_harm, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, run.src[0], d, d,
                                 snap_w=Ws, keep_all=True)
    worst = 0.0
    for m in range(w.n_harm):
        log(f"free-surface acoustic64 harmonic {m}")
        res = run.step()
        assert res.iters[0] == st["iters"][m], (m, res.iters, st["iters"][m])
        Ro = st["R"][m]
        e = np.linalg.norm(run.R.cpu().numpy()[0, 0] - Ro) / max(np.linalg.norm(Ro), 1e-300)
        worst = max(worst, e)
        assert e <= 1e-12, (m, e)
    snap = run.snap.cpu().numpy()[:, 0, 0]
    es = np.linalg.norm(snap - st["snap"]) / np.linalg.norm(st["snap"])
    print(f"free surface: worst per-harmonic error {worst:.2e}, snapshots {es:.2e}")
    assert es <= 1e-12
    # the surface changes the field: it differs from the Dirichlet run
    dir_run = AcousticRun(w, n_harm=w.n_harm)
    for _ in range(w.n_harm):
        dir_run.step()
    dsnap = dir_run.snap.cpu().numpy()[:, 0, 0]
    assert np.linalg.norm(dsnap - snap) > 1e-3 * np.linalg.norm(snap)


def test_free_surface_batched_equals_single():
    torch = torch_cuda()
    nx = nz = 64
    kappa, rho = heterogeneous(nx, nz)
    b = np.random.default_rng(12).standard_normal((3, 1, nz - 1, nx - 1))
    plan = _plan(nx, nz, kappa, rho, shots=3, segments=4)
    bd = to_dev(b, torch.float64)
    xd = torch.empty_like(bd)
    log("free-surface batched")
    res = plan.pcg_solve(bd, xd, tol=1e-10, max_iter=500)
    plan1 = _plan(nx, nz, kappa, rho, shots=1, segments=4)
    for s in range(3):
        x1 = torch.empty_like(bd[s:s + 1])
        r1 = plan1.pcg_solve(bd[s:s + 1].contiguous(), x1, tol=1e-10, max_iter=500)
        assert r1.iters[0] == res.iters[s]
        assert np.array_equal(to_np(x1)[0], to_np(xd)[s])
