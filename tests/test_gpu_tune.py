"""The plan's tile parameters (operator shots per block, Dichotomy segments per
wave, iterations per graph) change only the launch shape, never the
arithmetic: every setting gives the oracle's solution, and the autotuner
returns a setting from its candidate set."""
import numpy as np
import pytest

from oracle import OK
from paper_1005_0542_amd import api, tune

from _gpu import heterogeneous, log, rel, to_dev, to_np, torch_cuda
from test_gpu_parity import _oracle_pcg

pytestmark = pytest.mark.gpu


def _solve(nx, nz, kappa, rho, h, b, shots, **kw):
    torch = torch_cuda()
    plan = api.Plan("acoustic", nx, nz, 10.0, 10.0, 9, h, 8, np.stack([kappa, rho]), precision="fp64",
                    nshots=shots, **kw)
    bd = to_dev(b, torch.float64)
    xd = torch.empty_like(bd)
    res = plan.pcg_solve(bd, xd, tol=1e-10, max_iter=500)
    plan.destroy()
    return to_np(xd), res


@pytest.mark.parametrize("op_shots,spw", [(1, 1), (3, 2), (8, 4), (5, 0)])
def test_tile_parameters_keep_the_solution(op_shots, spw):
    nx, nz, shots, P = 128, 256, 5, 16
    kappa, rho = heterogeneous(nx, nz)
    h = 200.0
    b = np.random.default_rng(21).standard_normal((shots, 1, nz - 1, nx - 1))
    log(f"tile parameters op_shots={op_shots} seg_per_wave={spw}")
    x_ref, r_ref = _solve(nx, nz, kappa, rho, h, b, shots, segments=P)
    x, r = _solve(nx, nz, kappa, rho, h, b, shots, segments=P, op_shots=op_shots, seg_per_wave=spw)
    assert r.statuses == [OK] * shots and r.iters == r_ref.iters
    assert rel(x, x_ref) < 1e-13
    xo, ito, _, _ = _oracle_pcg(kappa, rho, h, nx, nz, 10.0, 10.0, b[0, 0], 1e-10, 500)
    assert r.iters[0] == ito and rel(x[0, 0], xo) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_op_fusion_bitwise(precision):
    """A p recomputed inside the update kernel (op_fusion 1) and A p stored by
    the operator kernel (op_fusion 2) give bitwise the same iterates."""
    torch = torch_cuda()
    nx, nz, shots = 256, 128, 3
    kappa, rho = heterogeneous(nx, nz)
    b = np.random.default_rng(8).standard_normal((shots, 1, nz - 1, nx - 1))
    out = {}
    for fus in (1, 2):
        log(f"op_fusion={fus} {precision}")
        plan = api.Plan("acoustic", nx, nz, 10.0, 10.0, 9, 200.0, 8, np.stack([kappa, rho]), precision=precision,
                        nshots=shots, segments=8, op_fusion=fus)
        bd = to_dev(b, torch.float64)
        xd = torch.empty_like(bd)
        res = plan.pcg_solve(bd, xd, tol=1e-9, max_iter=500)
        out[fus] = (to_np(xd), res.iters, res.statuses)
        plan.destroy()
    assert out[1][2] == [OK] * shots and out[1][1] == out[2][1]
    assert np.array_equal(out[1][0], out[2][0])


def test_autotuner_picks_a_candidate_and_caches_it(tmp_path):
    torch = torch_cuda()
    nx, nz, shots = 64, 128, 4
    kappa, rho = heterogeneous(nx, nz)
    cache = str(tmp_path / "tune.json")
    log("autotuner 64x128 x4")
    best = tune.tune_acoustic(nx, nz, 10.0, 10.0, 9, 200.0, np.stack([kappa, rho]), "fp64", shots,
                              cache=cache, profile_iters=2)
    assert best["segments"] in tune.segment_candidates(nz)
    assert best["op_shots"] in (1, 4) and best["seg_per_wave"] in (1, 2, 4) and best["op_fusion"] in (1, 2)
    assert best["graph_iters"] in tune.GRAPH_ITERS_CANDIDATES
    again = tune.tune_acoustic(nx, nz, 10.0, 10.0, 9, 200.0, np.stack([kappa, rho]), "fp64", shots,
                               cache=cache)
    assert again == best
    b = np.random.default_rng(4).standard_normal((shots, 1, nz - 1, nx - 1))
    x, r = _solve(nx, nz, kappa, rho, 200.0, b, shots, **best)
    xo, ito, _, _ = _oracle_pcg(kappa, rho, 200.0, nx, nz, 10.0, 10.0, b[2, 0], 1e-10, 500)
    assert r.statuses == [OK] * shots and r.iters[2] == ito and rel(x[2, 0], xo) < 1e-12
    torch.cuda.synchronize()
