"""GPU parity of the elastic traction-free surface (Sec. 2.2, eq.
boundary_elastic) against the FP64 oracle: the operator with the surface on
the first unknown row, the block preconditioner whose z-systems carry the
surface row, GMRES(k) at a fixed iteration count, and a harmonic chain."""
import numpy as np
import pytest

from oracle import NOT_CONVERGED, OK, elastic, harmonics, krylov, laguerre
from paper_1005_0542_amd import api, inputs

from _gpu import log, rel, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


def _medium(nx, nz, d, seed=1):
    n = max(nx, nz)
    vp = inputs.perturbed_layered_velocity(n, d, 2000.0, 4500.0, seed)[: nz + 1, : nx + 1]
    rho = inputs.perturbed_layered_velocity(n, d, 2000.0, 2600.0, seed + 1)[: nz + 1, : nx + 1]
    return inputs.elastic_coeffs(vp, rho)


def _plan(nx, nz, d, lam, mu, rho, h=300.0, shots=1, precision="fp64", segments=0, n=8, alpha=8):
    return api.Plan("elastic", nx, nz, d, d, alpha, h, n, np.stack([lam, mu, rho]), precision=precision,
                    nshots=shots, segments=segments, top="free")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,nz,shots", [(16, 16, 1), (64, 32, 2), (8, 128, 1), (16, 2, 3), (256, 8, 2)])
def test_free_elastic_operator_parity(prec, nx, nz, shots):
    torch = torch_cuda()
    d, h = 5.0, 300.0
    lam, mu, rho = _medium(nx, nz, d)
    plan = _plan(nx, nz, d, lam, mu, rho, h=h, shots=shots, precision=prec)
    u = np.random.default_rng(nx + 3 * nz).standard_normal((shots, 2, nz - 1, nx - 1))
    log(f"free elastic operator {prec} {nx}x{nz} shots={shots}")
    dt = torch.float64 if prec == "fp64" else torch.float32
    ud = to_dev(u, dt)
    yd = torch.empty_like(ud)
    plan.stencil_apply(ud, yd)
    w = rho[1:-1, 1:-1] * h * h / 4
    ur = to_np(ud)
    for s in range(shots):
        ref = elastic.apply_C_free(ur[s], lam, mu, w, d, d)
        assert rel(to_np(yd)[s], ref) < (1e-13 if prec == "fp64" else 2e-5), s
    plan.destroy()


@pytest.mark.parametrize("nx,nz,P", [(16, 16, 1), (16, 16, 2), (64, 64, 4), (32, 256, 16), (8, 4, 2)])
def test_free_elastic_preconditioner_parity(nx, nz, P):
    torch = torch_cuda()
    d, h = 5.0, 300.0
    lam, mu, rho = _medium(nx, nz, d)
    plan = _plan(nx, nz, d, lam, mu, rho, h=h, shots=2, segments=P)
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, h, nx, nz, d, d, surface_node=True)
    r = np.random.default_rng(P + nz).standard_normal((2, 2, nz - 1, nx - 1))
    log(f"free elastic K^-1 {nx}x{nz} P={P}")
    rd = to_dev(r, torch.float64)
    zd = torch.empty_like(rd)
    plan.precond_apply(rd, zd)
    for s in range(2):
        assert rel(to_np(zd)[s], elastic.apply_Kinv(r[s], B1, B2)) < 1e-12
    for blk, B in ((1, B1), (2, B2)):
        rh = to_dev(r[:, 0], torch.float64)
        sh = torch.empty_like(rh)
        plan.precond_dichotomy_tdma(blk, rh, sh)
        for s in range(2):
            assert rel(to_np(sh)[s], B.tridiag_solve(r[s, 0])) < 1e-12
    plan.destroy()


@pytest.mark.parametrize("nx,nz,k", [(32, 32, 10), (64, 64, 10), (64, 32, 4)])
def test_free_elastic_gmres_parity(nx, nz, k):
    """GMRES(k) on the free operator with the surface preconditioner: run to
    the oracle's iteration count (tol = 0) it matches to 1e-12; to tolerance
    the counts agree within one and the FP64 true residual meets it."""
    torch = torch_cuda()
    d, h = 5.0, 300.0
    lam, mu, rho = _medium(nx, nz, d)
    plan = _plan(nx, nz, d, lam, mu, rho, h=h)
    w = rho[1:-1, 1:-1] * h * h / 4
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, h, nx, nz, d, d, surface_node=True)
    C = lambda u: elastic.apply_C_free(u, lam, mu, w, d, d)
    K = lambda u: elastic.apply_Kinv(u, B1, B2)
    b = np.random.default_rng(nx * k + 1).standard_normal((2, nz - 1, nx - 1))
    xo, ito, _, sto = krylov.gmres(C, K, b, 1e-10, k)
    assert sto == OK
    bd = to_dev(b[None], torch.float64)
    xd = torch.empty_like(bd)
    log(f"free gmres {nx}x{nz} k={k}: fixed {ito} iterations")
    res = plan.gmres_solve(bd, xd, tol=0.0, max_iter=ito, restart=k)
    assert res.statuses == [NOT_CONVERGED] and res.iters == [ito]
    assert rel(to_np(xd)[0], xo) < 1e-12, rel(to_np(xd)[0], xo)
    log(f"free gmres {nx}x{nz} k={k}: to tolerance")
    res = plan.gmres_solve(bd, xd, tol=1e-10, max_iter=5000, restart=k)
    assert res.statuses == [OK] and abs(res.iters[0] - ito) <= 1
    r = b - C(to_np(xd)[0])
    assert np.linalg.norm(r) <= 10 * 1e-10 * np.linalg.norm(b)
    plan.destroy()


def test_free_elastic_harmonic_chain_and_surface_source():
    """Six harmonics of a vertical point force below the surface, each run for
    the oracle's GMRES(10) iteration count: right-hand sides and solutions
    match the oracle's own chain to 1e-12; and a force on the surface row
    enters the right-hand side as 2 f_m/(dx dz) (half a control cell)."""
    torch = torch_cuda()
    nx = nz = 32
    d, h, alpha, nh = 5.0, 300.0, 8, 6
    lam, mu, rho = _medium(nx, nz, d)
    plan = _plan(nx, nz, d, lam, mu, rho, h=h, shots=2, n=nh, alpha=alpha)
    src = np.array([[16, 6], [9, 1]], dtype=np.int32)        # shot 1: on the surface row
    plan.set_sources(src)
    f = api.source_coeffs(20.0, 1.5 / 20.0, alpha, h, nh)
    fo = laguerre.ricker_coeffs(20.0, 1.5 / 20.0, h, alpha, nh)
    shape = (2, 2, nz - 1, nx - 1)
    R, Ph, Qh, rhs = (torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(4))
    w = rho[1:-1, 1:-1] * h * h / 4
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, h, nx, nz, d, d, surface_node=True)
    C = lambda u: elastic.apply_C_free(u, lam, mu, w, d, d)
    K = lambda u: elastic.apply_Kinv(u, B1, B2)
    sums = [harmonics.RunningSums((2, nz - 1, nx - 1), alpha) for _ in range(2)]
    Rprev = [None, None]
    for m in range(nh):
        plan.laguerre_rhs(m, R if m else None, Ph, Qh, [f[m], f[m]], rhs)
        xos, its, phis = [], [], []
        for s in range(2):
            phi = elastic.source_field_free((nz - 1, nx - 1), src[s], fo[m], d, d) - \
                h * h * rho[1:-1, 1:-1][None] * sums[s].step(m, Rprev[s])
            assert rel(to_np(rhs)[s], phi) < 1e-12, (m, s)
            xo, ito, _, sto = krylov.gmres(C, K, phi, 1e-11, 10)
            assert sto == OK
            xos.append(xo)
            its.append(ito)
            phis.append(phi)
        # both shots run for the larger count: the other shot's oracle run repeats with it
        cap = max(its)
        for s in range(2):
            if its[s] != cap:
                xos[s], itc, _, _ = krylov.gmres(C, K, phis[s], 0.0, 10, max_iter=cap)
                assert itc == cap
        log(f"free elastic harmonic {m}: fixed {cap} iterations")
        res = plan.gmres_solve(rhs, R, tol=0.0, max_iter=cap, restart=10)
        assert res.iters == [cap, cap]
        for s in range(2):
            assert rel(to_np(R)[s], xos[s]) < 1e-12, (m, s, rel(to_np(R)[s], xos[s]))
            Rprev[s] = xos[s]
    plan.destroy()


def test_full_elastic1024_free_surface_fixed_iterations():
    """The 1023^2 x 2 elastic workload with the traction-free surface: its
    first harmonic, two full GMRES(10) cycles from x = 0, against the oracle
    (1e-12)."""
    torch = torch_cuda()
    w = inputs.WORKLOADS["elastic1024"]
    lam, mu, rho = inputs.elastic_medium_for(w)
    N, d = w.n_cells, w.d
    plan = api.Plan("elastic", N, N, d, d, w.alpha, w.h, 2, np.stack([lam, mu, rho]), precision="fp64",
                    nshots=1, top="free")
    src = inputs.sources_for(w)
    plan.set_sources(src)
    f = api.source_coeffs(w.f0, w.t0, w.alpha, w.h, 1)
    shape = (1, 2, N - 1, N - 1)
    R, Ph, Qh, rhs = (torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(4))
    log("free elastic1024 harmonic 0: 20 iterations")
    plan.laguerre_rhs(0, None, Ph, Qh, [f[0]], rhs)
    res = plan.gmres_solve(rhs, R, tol=0.0, max_iter=20, restart=10)
    assert res.iters == [20]
    fo = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, 1)
    phi = elastic.source_field_free((N - 1, N - 1), src[0], fo[0], d, d)
    assert rel(to_np(rhs)[0], phi) < 1e-12
    wv = rho[1:-1, 1:-1] * w.h * w.h / 4
    B1, B2 = elastic.block_preconditioner(lam, mu, rho, w.h, N, N, d, d, surface_node=True)
    xo, ito, _, _ = krylov.gmres(lambda u: elastic.apply_C_free(u, lam, mu, wv, d, d),
                                 lambda u: elastic.apply_Kinv(u, B1, B2), phi, 0.0, 10, max_iter=20)
    x = to_np(R)[0]
    e = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
    print(f"free elastic1024: 20 iterations, rel L2 {e:.2e}")
    assert ito == 20 and e <= 1e-12
    plan.destroy()
