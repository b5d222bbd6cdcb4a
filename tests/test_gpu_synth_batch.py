"""Synthesis of several harmonics in one pass (lg_laguerre_synthesize_batch,
eq. series_lag): the snapshot sums and the receiver rows must be bitwise
those of one lg_laguerre_synthesize call per harmonic, through the C ABI and
through the harmonic-loop driver (batches of 4 with a partial last batch, and
a checkpoint taken in the middle of a batch)."""
import numpy as np
import pytest

from paper_1005_0542_amd import inputs
from paper_1005_0542_amd.driver import AcousticRun

from _gpu import acoustic_plan, heterogeneous, log, to_dev, to_np, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nb,nsnap,with_rec", [(1, 4, True), (3, 4, True), (5, 2, False), (8, 8, True),
                                               (4, 0, True)])
def test_batch_synthesis_bitwise_equals_single_harmonic_calls(nb, nsnap, with_rec):
    torch = torch_cuda()
    nx, nz, S = 64, 32, 3
    kappa, rho = heterogeneous(nx, nz)
    n = 12
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho, n=n, shots=S)
    rng = np.random.default_rng(nb * 10 + nsnap)
    m0 = n - nb - 1
    Rs = [to_dev(rng.standard_normal((S, 1, nz - 1, nx - 1)), torch.float64) for _ in range(nb)]
    W = rng.standard_normal((nsnap, nb))
    snap0 = rng.standard_normal((nsnap, S, 1, nz - 1, nx - 1))
    rec0 = rng.standard_normal((S, 1, n, nx - 1))
    rec_row = 5
    a_snap, b_snap = to_dev(snap0, torch.float64), to_dev(snap0, torch.float64)
    a_rec = to_dev(rec0, torch.float64) if with_rec else None
    b_rec = to_dev(rec0, torch.float64) if with_rec else None
    log(f"synthesis batch nb={nb} nsnap={nsnap} rec={with_rec}")
    for b in range(nb):
        plan.laguerre_synthesize(m0 + b, Rs[b], W[:, b], a_snap if nsnap else None, rec_row, a_rec)
    plan.laguerre_synthesize_batch(m0, Rs, W, b_snap if nsnap else None, rec_row, b_rec)
    torch.cuda.synchronize()
    if nsnap:
        assert np.array_equal(to_np(a_snap), to_np(b_snap))
        assert not np.array_equal(to_np(b_snap), snap0)
    if with_rec:
        got = to_np(b_rec)
        assert np.array_equal(to_np(a_rec), got)
        for b in range(nb):
            assert np.array_equal(got[:, :, m0 + b], to_np(Rs[b])[:, :, rec_row - 1])


def test_batch_synthesis_rejects_bad_ranges():
    torch = torch_cuda()
    nx = nz = 16
    kappa, rho = heterogeneous(nx, nz)
    plan = acoustic_plan(nx, nz, 10.0, 10.0, kappa, rho, n=6, shots=1)
    R = to_dev(np.ones((1, 1, nz - 1, nx - 1)), torch.float64)
    snap = to_dev(np.zeros((1, 1, 1, nz - 1, nx - 1)), torch.float64)
    for m0, nb in ((4, 3), (-1, 2), (0, 9)):
        with pytest.raises(RuntimeError):
            plan.laguerre_synthesize_batch(m0, [R] * nb, np.ones((1, nb)), snap, 1, None)
    assert not to_np(snap).any()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_driver_batched_synthesis_bitwise_equals_per_harmonic(precision):
    torch = torch_cuda()
    w = inputs.WORKLOADS["acoustic64"]
    n = 11                                            # two batches of 4 and a partial one of 3
    runs = {}
    for sb in (1, 4):
        log(f"driver synthesis batch {sb} ({precision})")
        run = AcousticRun(w, precision=precision, n_harm=n, synth_batch=sb)
        for _ in range(n):
            run.step()
        runs[sb] = (to_np(run.snap), to_np(run.rec), to_np(run.traces(inputs.trace_times(w))), run.iters)
    a, b = runs[1], runs[4]
    assert a[3] == b[3]
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    # a checkpoint in the middle of a batch, resumed in a fresh run
    log(f"driver synthesis batch: checkpoint after 6 harmonics ({precision})")
    run = AcousticRun(w, precision=precision, n_harm=n, synth_batch=4)
    for _ in range(6):
        run.step()
    st = run.state_dict()
    run2 = AcousticRun(w, precision=precision, n_harm=n, synth_batch=4)
    run2.load_state_dict(st)
    for _ in range(n - 6):
        run2.step()
    assert np.array_equal(to_np(run2.snap), a[0])
    assert np.array_equal(to_np(run2.rec), a[1])
