"""GPU parity of the fourth-order acoustic operator (Sec. 3.2: a higher-order
scheme preconditioned by the same second-order B) against the FP64 oracle:
the 13-point operator, PCG with the second-order preconditioner (FP64 and
mixed with FP64 refinement) and a whole harmonic chain."""
import numpy as np
import pytest

from oracle import OK, harmonics, highorder as ho, krylov, laguerre, operator, precond
from paper_1005_0542_amd import _lib, api, inputs
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import heterogeneous, log, rel, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(nx, nz, kappa, rho, h=200.0, precision="fp64", shots=1, segments=0, dx=10.0, dz=10.0, **kw):
    return api.Plan("acoustic", nx, nz, dx, dz, 9, h, 8, np.stack([kappa, rho]), precision=precision,
                    nshots=shots, segments=segments, order=4, **kw)


def _wdt(prec):
    torch = torch_cuda()
    return torch.float64 if prec == "fp64" else torch.float32


def _oracle_op(kappa, rho, h, dx, dz):
    kx, kz = ho.face_coeffs4(kappa)
    w = operator.shift_coeff(rho, h)
    return lambda y: ho.apply_A4(y, kx, kz, w, dx, dz)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,nz,shots,osh", [(16, 16, 1, 0), (64, 32, 3, 0), (2, 4, 1, 0), (4, 2, 2, 0),
                                             (8, 8, 2, 0), (128, 256, 5, 2), (1024, 64, 1, 0), (64, 1024, 3, 3)])
def test_order4_stencil_parity(prec, nx, nz, shots, osh):
    kappa, rho = heterogeneous(nx, nz)
    h = 300.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision=prec, shots=shots, dx=7.0, dz=5.0, op_shots=osh)
    x = np.random.default_rng(nx + 5 * nz).standard_normal((shots, nz - 1, nx - 1))
    log(f"order4 stencil {prec} {nx}x{nz} shots={shots} op_shots={osh}")
    xd = to_dev(x, _wdt(prec))
    yd = torch_cuda().empty_like(xd)
    plan.stencil_apply(xd, yd)
    ref = _oracle_op(kappa, rho, h, 7.0, 5.0)(to_np(xd))
    assert rel(to_np(yd), ref) < (1e-13 if prec == "fp64" else 1e-5)


def _oracle_pcg(kappa, rho, h, nx, nz, b, tol, max_iter=1000, dx=10.0, dz=10.0):
    B = precond.acoustic_preconditioner(kappa, rho, h, nx, nz, dx, dz)
    return krylov.pcg(_oracle_op(kappa, rho, h, dx, dz), B.solve, b, tol, max_iter)


@pytest.mark.parametrize("nx,nz,P,gi", [(64, 64, 4, 0), (128, 256, 8, 4), (1024, 256, 16, 8), (32, 128, 32, 0)])
def test_order4_pcg_parity_fp64(nx, nz, P, gi):
    torch = torch_cuda()
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = _plan(nx, nz, kappa, rho, h=h, segments=P, shots=2, graph_iters=gi)
    b = np.random.default_rng(6).standard_normal((2, nz - 1, nx - 1))
    log(f"order4 pcg fp64 {nx}x{nz} P={P} graph_iters={gi}")
    bd = to_dev(b, torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=1e-10, max_iter=1000)
    it2 = None
    for s in range(2):
        xo, ito, rro, sto = _oracle_pcg(kappa, rho, h, nx, nz, b[s], 1e-10)
        assert res.statuses[s] == OK and sto == OK
        assert res.iters[s] == ito, (s, res.iters, ito)
        assert rel(to_np(xd)[s], xo) < 1e-12
    # the second-order B still preconditions A4: a few more iterations than A
    plan2 = api.Plan("acoustic", nx, nz, 10.0, 10.0, 9, h, 8, np.stack([kappa, rho]), nshots=2, segments=P)
    x2 = torch.empty_like(bd)
    it2 = plan2.pcg_solve(bd, x2, tol=1e-10, max_iter=1000).iters
    for a4, a2 in zip(res.iters, it2):
        assert a2 <= a4 <= 7 * a2 / 6 + 3, (res.iters, it2)


@pytest.mark.parametrize("nx,nz,shots", [(64, 64, 2), (512, 256, 3)])
def test_order4_pcg_mixed_true_residual(nx, nz, shots):
    torch = torch_cuda()
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    plan = _plan(nx, nz, kappa, rho, h=h, precision="mixed", shots=shots, graph_iters=8)
    b = np.random.default_rng(7).standard_normal((shots, nz - 1, nx - 1))
    log(f"order4 pcg mixed {nx}x{nz} shots={shots}")
    bd = to_dev(b, torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=1e-9, max_iter=1000)
    assert res.statuses == [OK] * shots
    A4 = _oracle_op(kappa, rho, h, 10.0, 10.0)
    for s in range(shots):
        r = b[s] - A4(to_np(xd)[s])
        assert np.linalg.norm(r) <= 1.5e-9 * np.linalg.norm(b[s])
        xo = _oracle_pcg(kappa, rho, h, nx, nz, b[s], 1e-12)[0]
        assert rel(to_np(xd)[s], xo) < 1e-6


def test_order4_options_and_profile():
    """x0_given is rejected; the profile helper runs the fourth-order
    iteration (stored q) and leaves x equal to 6 oracle iterations (5 timed,
    one untimed first one)."""
    torch = torch_cuda()
    nx = nz = 64
    kappa, rho = heterogeneous(nx, nz)
    plan = _plan(nx, nz, kappa, rho, shots=2, segments=4)
    b = np.random.default_rng(3).standard_normal((2, nz - 1, nx - 1))
    bd = to_dev(b, torch.float64)
    xd = torch.zeros_like(bd)
    log("order4 options + profile")
    with pytest.raises(_lib.LgError) as ei:
        plan.pcg_solve(bd, xd, x0_given=True)
    assert ei.value.status == _lib.LG_ERR_UNSUPPORTED
    ms = plan.pcg_profile(bd, xd, iters=5)
    assert all(m > 0.0 for m in ms)
    for s in range(2):
        xo = _oracle_pcg(kappa, rho, 200.0, nx, nz, b[s], 0.0, max_iter=6)[0]
        assert rel(to_np(xd)[s], xo) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_order4_harmonic_chain(prec):
    """32 harmonics of the 64^2 two-layer workload with the fourth-order
    operator: FP64 identical iteration counts and 1e-12 per harmonic against
    the oracle's own chain; mixed (tol 1e-9, FP64 refinement) within 1e-6."""
    w = inputs.WORKLOADS["acoustic64"]
    n_harm = 32
    run = AcousticRun(w, precision=prec, n_harm=n_harm, order=4, tol=1e-9 if prec == "mixed" else None)
    kappa, rho = run.kappa, run.rho
    N, d = w.n_cells, w.d
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    A4 = _oracle_op(kappa, rho, w.h, d, d)
    solve = lambda phi: krylov.pcg(A4, B.solve, phi, 1e-10, 10000)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n_harm)
    Ws = laguerre.synthesis_weights(np.array(inputs.snapshot_times(w)), w.h, w.alpha, n_harm)
    st = harmonics.harmonic_loop(n_harm, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, run.src[0], d, d,
                                 snap_w=Ws, keep_all=True)
    mixed = prec == "mixed"
    worst = 0.0
    for m in range(n_harm):
        log(f"order4 acoustic64 {prec} harmonic {m}")
        res = run.step()
        assert res.statuses == [OK]
        if not mixed:
            assert res.iters[0] == st["iters"][m], (m, res.iters, st["iters"][m])
        Ro = st["R"][m]
        e = np.linalg.norm(run.R.cpu().numpy()[0, 0] - Ro) / max(np.linalg.norm(Ro), 1e-300)
        worst = max(worst, e)
        assert e <= (1e-6 if mixed else 1e-12), (m, e)
    snap = run.snap.cpu().numpy()[:, 0, 0]
    es = np.linalg.norm(snap - st["snap"]) / np.linalg.norm(st["snap"])
    print(f"order 4 {prec}: worst per-harmonic error {worst:.2e}, snapshots {es:.2e}")
    assert es <= (1e-6 if mixed else 1e-12)
