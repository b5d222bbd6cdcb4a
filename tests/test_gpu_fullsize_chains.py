"""Mixed-precision harmonic chains at the full benchmark sizes against the
FP64 oracle's own chains (the error of every reported result, per harmonic
and on the synthesized snapshots).

* 4095^2 unknowns, one shot, the first 8 harmonics with the 4 snapshots;
* 64 shots on 2047^2 unknowns, the first 8 harmonics, shots 0, 31 and 63.

Both run in the benchmark's launch configuration (the autotuner's tiles) with
the workloads' mixed tolerance 1e-9 (FP32 operator, transforms and
Dichotomy; FP64 Krylov scalars, residual refinement, recurrence and
synthesis).  The oracle chains (tolerance 1e-10, the FP64 workloads' own) run in worker processes on
the host while the GPU works.  Bar: relative L2 <= 1e-6 for every R_m and
for the partial snapshots.
"""
import concurrent.futures
import multiprocessing
import time

import numpy as np
import pytest

from oracle import OK
from paper_1005_0542_amd import tune
from paper_1005_0542_amd.driver import AcousticRun
from paper_1005_0542_amd import inputs

from _gpu import log, torch_cuda
import _oracle_chains

pytestmark = pytest.mark.gpu

N_HARM = 8
SAMPLES = (0, 31, 63)


def _l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(name, shots):
    w = inputs.WORKLOADS[name]
    t = tune.lookup(w.n_cells, w.n_cells, "mixed", shots)
    tiles = {k: t.get(k, 0) for k in ("segments", "graph_iters", "op_shots", "seg_per_wave", "op_fusion")}
    log(f"{name} mixed x{shots}: {N_HARM} harmonics, tiles {tiles}")
    return AcousticRun(w, precision="mixed", n_harm=N_HARM, snapshots=True, rec=False, **tiles)


@pytest.mark.timeout(1500)
def test_full_mixed_chains_against_fp64_oracle():
    torch = torch_cuda()
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=4, mp_context=ctx) as pool:
        futs = {("acoustic4096_mixed", 0): pool.submit(_oracle_chains.oracle_chain, "acoustic4096_mixed", 0,
                                                       N_HARM, 1e-10)}
        for s in SAMPLES:
            futs[("acoustic2048x64_mixed", s)] = pool.submit(_oracle_chains.oracle_chain, "acoustic2048x64_mixed",
                                                             s, N_HARM, 1e-10)
        gpu = {}
        for name, shots, samples in (("acoustic4096_mixed", 1, (0,)), ("acoustic2048x64_mixed", 64, SAMPLES)):
            run = _run(name, shots)
            Rs = {s: [] for s in samples}
            for m in range(N_HARM):
                log(f"{name} harmonic {m}")
                res = run.step()
                assert res.statuses == [OK] * shots, (name, m, res.statuses)
                for s in samples:
                    Rs[s].append(run.R[s, 0].cpu().numpy())
            snap = run.snap.cpu().numpy()
            gpu[name] = (Rs, {s: snap[:, s, 0] for s in samples}, run.iters)
            run.plan.destroy()
            del run
            torch.cuda.empty_cache()
        # the oracle chains take minutes: report progress every 20 s
        t0 = time.monotonic()
        while True:
            done, pending = concurrent.futures.wait(list(futs.values()), timeout=20.0)
            log(f"oracle chains: {len(done)} of {len(futs)} done after {time.monotonic() - t0:.0f} s")
            if not pending:
                break
        orc = {k: f.result() for k, f in futs.items()}
    worst = {}
    for (name, s), o in orc.items():
        Rs, snaps, iters = gpu[name]
        errs = [_l2(Rs[s][m], o["R"][m]) for m in range(N_HARM)]
        es = _l2(snaps[s], o["snap"])
        its = [int(i[s]) for i in iters]
        print(f"{name} shot {s}: per-harmonic rel L2 {[f'{e:.1e}' for e in errs]}, snapshots {es:.1e}, "
              f"GPU iterations {its}, oracle (tol 1e-10) {o['iters']}")
        worst[(name, s)] = (max(errs), es)
        assert all(st == OK for st in o["status"])
    for k, (er, es) in worst.items():
        assert er <= 1e-6 and es <= 1e-6, (k, er, es)


@pytest.mark.timeout(900)
def test_full_fp64_chains_at_the_oracle_iteration_counts():
    """The FP64 workloads over more harmonics, each harmonic run for exactly the
    oracle's own iteration count (tol = 0): the library's chain and the
    oracle's are then the same computation up to rounding.
    * 1023^2 acoustic FP64: 64 harmonics and the snapshots;
    * 1023^2 x 2 elastic GMRES(10): 6 harmonics.
    Bar: 1e-12 relative L2 per harmonic and on the snapshots."""
    import torch
    from paper_1005_0542_amd import api
    torch_cuda()
    NA, NE = 64, 6
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=2, mp_context=ctx) as pool:
        fa = pool.submit(_oracle_chains.oracle_chain, "acoustic1024", 0, NA, 1e-10)
        fe = pool.submit(_oracle_chains.oracle_elastic_chain, "elastic1024", NE, 1e-10)
        t0 = time.monotonic()
        while True:
            done, pending = concurrent.futures.wait([fa, fe], timeout=20.0)
            log(f"oracle chains: {len(done)} of 2 done after {time.monotonic() - t0:.0f} s")
            if not pending:
                break
        oa, oe = fa.result(), fe.result()
    # acoustic: the driver's buffers and synthesis, the solve at the oracle's counts
    w = inputs.WORKLOADS["acoustic1024"]
    t = tune.lookup(w.n_cells, w.n_cells, "fp64", 1)
    run = AcousticRun(w, precision="fp64", n_harm=NA, snapshots=True, rec=False,
                      **{k: t.get(k, 0) for k in ("segments", "graph_iters", "op_shots", "seg_per_wave", "op_fusion")})
    # the oracle's synthesis weights feed both sides' snapshots (the library's
    # host helper is checked against them separately)
    from oracle import laguerre
    Ws = laguerre.synthesis_weights(np.array(inputs.snapshot_times(w)), w.h, w.alpha, NA)
    errs = []
    for m in range(NA):
        fs = np.full(1, run.f_m[m])
        run.plan.laguerre_rhs(m, run.R if m else None, run.Ph, run.Qh, fs, run.rhs)
        log(f"acoustic1024 harmonic {m}: {oa['iters'][m]} iterations")
        res = run.plan.pcg_solve(run.rhs, run.R, tol=0.0, max_iter=oa["iters"][m])
        assert res.iters == [oa["iters"][m]]
        run.plan.laguerre_synthesize(m, run.R, Ws[:, m], run.snap)
        errs.append(_l2(run.R[0, 0].cpu().numpy(), oa["R"][m]))
    es = _l2(run.snap[:, 0, 0].cpu().numpy(), oa["snap"])
    print(f"acoustic1024 {NA} harmonics at the oracle's counts: per-harmonic rel L2 max {max(errs):.1e}, "
          f"snapshots {es:.1e}")
    assert max(errs) <= 1e-12 and es <= 1e-12, (errs, es)
    run.plan.destroy()
    del run
    # elastic
    we = inputs.WORKLOADS["elastic1024"]
    lam, mu, rho = inputs.elastic_medium_for(we)
    N, d = we.n_cells, we.d
    plan = api.Plan("elastic", N, N, d, d, we.alpha, we.h, NE, np.stack([lam, mu, rho]), precision="fp64", nshots=1)
    plan.set_sources(inputs.sources_for(we))
    f = api.source_coeffs(we.f0, we.t0, we.alpha, we.h, NE)
    shape = (1, 2, N - 1, N - 1)
    R, Ph, Qh, rhs = (torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(4))
    eerrs = []
    for m in range(NE):
        plan.laguerre_rhs(m, R if m else None, Ph, Qh, [f[m]], rhs)
        log(f"elastic1024 harmonic {m}: {oe['iters'][m]} iterations")
        res = plan.gmres_solve(rhs, R, tol=0.0, max_iter=oe["iters"][m], restart=10)
        assert res.iters == [oe["iters"][m]]
        eerrs.append(_l2(R[0].cpu().numpy(), oe["R"][m]))
    print(f"elastic1024 {NE} harmonics at the oracle's counts: per-harmonic rel L2 {[f'{e:.1e}' for e in eerrs]}")
    assert max(eerrs) <= 1e-12
    plan.destroy()
