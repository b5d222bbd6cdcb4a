"""PCG from a given initial guess (x0_given), e.g. the previous harmonic,
against the oracle's PCG from the same x0."""
import numpy as np
import pytest

from oracle import OK, operator, precond, krylov, harmonics, laguerre
from paper_1005_0542_amd import api, inputs
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import acoustic_plan, heterogeneous, log, rel, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle(kappa, rho, h, nx, nz, b, tol, x0=None, dx=10.0, dz=10.0):
    w = operator.shift_coeff(rho, h)
    B = precond.acoustic_preconditioner(kappa, rho, h, nx, nz, dx, dz)
    return krylov.pcg(lambda y: operator.apply_A(y, kappa, w, dx, dz), B.solve, b, tol, 500, x0=x0)


@pytest.mark.parametrize("nx,nz,P", [(64, 64, 4), (256, 128, 8), (1024, 256, 16)])
def test_warm_start_parity_fp64(nx, nz, P):
    torch = torch_cuda()
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho, h=h, shots=2, segments=P)
    rng = np.random.default_rng(nx + P)
    b = rng.standard_normal((2, 1, nz - 1, nx - 1))
    x0 = rng.standard_normal((2, 1, nz - 1, nx - 1))
    log(f"warm start fp64 {nx}x{nz} P={P}")
    xd = to_dev(x0, torch.float64)
    res = plan.pcg_solve(to_dev(b, torch.float64), xd, tol=1e-10, max_iter=500, x0_given=True)
    assert res.statuses == [OK, OK]
    for s in range(2):
        xo, ito, rro, sto = _oracle(kappa, rho, h, nx, nz, b[s, 0], 1e-10, x0=x0[s, 0])
        assert sto == OK and res.iters[s] == ito
        assert rel(to_np(xd)[s, 0], xo) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_warm_start_special_cases(prec):
    """x0 = 0 given equals the default start bit for bit; a converged x0 needs
    no iteration; b = 0 gives x = 0 whatever x0."""
    torch = torch_cuda()
    nx = nz = 64
    kappa, rho = heterogeneous(nx, nz)
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho, h=200.0, precision=prec, shots=3, segments=4)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((3, 1, nz - 1, nx - 1))
    b[2] = 0.0
    bd = to_dev(b, torch.float64)
    log(f"warm start special cases {prec}")
    xa = torch.empty_like(bd)
    ra = plan.pcg_solve(bd, xa, tol=1e-9, max_iter=500)
    xb = torch.zeros_like(bd)
    rb = plan.pcg_solve(bd, xb, tol=1e-9, max_iter=500, x0_given=True)
    assert ra.iters == rb.iters and torch.equal(xa, xb)
    xc = xa.clone()
    xc[2] = 1.0                                     # b = 0 with a nonzero start
    rc = plan.pcg_solve(bd, xc, tol=1e-6, max_iter=500, x0_given=True)
    assert rc.statuses == [OK] * 3 and rc.iters == [0, 0, 0]
    assert torch.equal(xc[:2], xa[:2]) and not xc[2].any()


def test_warm_start_mixed_true_residual():
    torch = torch_cuda()
    nx, nz = 256, 128
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho, h=h, precision="mixed", shots=1, segments=8)
    rng = np.random.default_rng(9)
    b = rng.standard_normal((1, 1, nz - 1, nx - 1))
    x0 = rng.standard_normal((1, 1, nz - 1, nx - 1))
    log("warm start mixed")
    xd = to_dev(x0, torch.float64)
    res = plan.pcg_solve(to_dev(b, torch.float64), xd, tol=1e-9, max_iter=500, x0_given=True)
    assert res.statuses == [OK]
    r = b[0, 0] - operator.apply_A(to_np(xd)[0, 0], kappa, operator.shift_coeff(rho, h), 10.0, 10.0)
    assert np.linalg.norm(r) <= 1.5e-9 * np.linalg.norm(b)


def test_warm_started_harmonic_chain_fp64():
    """Each harmonic starts from the previous one: per-harmonic 1e-12 against
    the oracle doing the same, identical iteration counts."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic64"]
    n = 24
    run = AcousticRun(w, n_harm=n, warm_start=True)
    kappa, rho = run.kappa, run.rho
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n)
    sums = harmonics.RunningSums((N - 1, N - 1), w.alpha)
    Rp = None
    for m in range(n):
        log(f"warm-started harmonic {m}")
        res = run.step()
        src = harmonics.source_field((N - 1, N - 1), run.src[0], f_m[m], d, d)
        phi = harmonics.rhs_running(m, sums, Rp, rho[1:-1, 1:-1], w.h, src)
        xo, ito, _, sto = krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, phi, 1e-10, 10000,
                                     x0=Rp if m > 0 else None)
        assert sto == OK and res.iters[0] == ito, (m, res.iters, ito)
        assert rel(run.R.cpu().numpy()[0, 0], xo) < 1e-12
        Rp = xo


def test_initial_guess_option_errors():
    import ctypes
    from paper_1005_0542_amd import _lib
    torch = torch_cuda()
    nx = nz = 16
    kappa, rho = heterogeneous(nx, nz)
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho)
    b = torch.ones((1, 1, nz - 1, nx - 1), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    lib = _lib.load()
    opts = _lib.SolveOpts(1e-8, 100, 1, 2, 0)
    log("x0_given = 2 rejected")
    assert lib.lg_pcg_solve(plan.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                            ctypes.byref(opts), None) == _lib.LG_ERR_INVALID_ARG
    lam = np.full((nz + 1, nx + 1), 2e9)
    el = api.Plan("elastic", nx, nz, 5.0, 5.0, 8, 300.0, 4, np.stack([lam, lam / 2, np.full_like(lam, 2000.0)]))
    b2 = torch.ones((1, 2, nz - 1, nx - 1), dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(b2)
    opts = _lib.SolveOpts(1e-8, 100, 10, 1, 0)
    log("GMRES with a given x0 rejected")
    assert lib.lg_gmres_solve(el.handle, ctypes.c_void_p(b2.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
                              ctypes.byref(opts), None) == _lib.LG_ERR_UNSUPPORTED
