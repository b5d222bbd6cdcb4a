"""Benchmark of the Laguerre-harmonic PCG solve on one MI355X.

One *step* is one harmonic of the Laguerre method over the whole shot batch:
right-hand side (``lg_laguerre_rhs``), preconditioned CG to tolerance
(``lg_pcg_solve``: operator, DST-I, Dichotomy solve, inverse DST per
iteration) and synthesis (``lg_laguerre_synthesize``).  Harmonics are run in
order from m = 0; the first ``--warmup`` are untimed (they also build the
plan's HIP graph), the next ``--steps`` are timed between device
synchronisations.

Metric: PCG Mpoint-iters/s = sum over timed harmonics and shots of
(interior points x CG iterations) / wall time / 1e6.  The headline workload is
the mixed-precision 64-shot batch on a 2048^2 grid; the other precision/shot
combinations of the metric are reported under "variants".

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG Mpoint-iters/s & HBM GB/s: FP64 plain vs mixed precision, 1 vs 64 shots"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(ws: int, shots: int, seg_len: int, fused: bool = True, medium: int = 2,
                 held: bool = False):
    """Algorithmic HBM bytes per shot-point for each kernel of one CG iteration
    (every array touched once per launch; medium arrays shared by all shots).
    fused: the update recomputes A p, so the operator kernel stores no q.
    medium: operator tables per point (kappa, w; the fourth-order operator
    reads its x- and z-face tables and w).  held: the update leaves x alone
    (held search directions; the flush pass is counted by flush_bytes)."""
    xb = 0 if held else 16                                    # x in/out (f64)
    if fused:
        op = ws + 2 * ws / shots                              # p in; kappa, w once per batch
        upd = xb + 16 + 2 * ws + 2 * ws / shots               # r in/out (f64); p in; rhat out; medium
    else:
        op = 2 * ws + medium * ws / shots                     # p in, q out; medium once per batch
        upd = xb + 16 + 3 * ws                                # r in/out (f64); p, q in; rhat out
    return {
        "operator": op,
        "update_fdst": upd,
        "dichotomy_segments": 2 * ws + 24.0 / seg_len,        # rhat in, y out; 3 f64 per segment
        "interfaces": (2 * ws + 24.0) / seg_len,              # separator rows, segment data
        "correct_idst": 3 * ws,                               # y in, p in/out
    }


def flush_bytes(ws: int, mean_iters: float, phases: int) -> float:
    """Held search directions: the flush passes' bytes per shot-point per CG
    iteration: every direction read once; x written once after the cold
    start's phase and read and written once after each later phase."""
    return ws + (8.0 + 16.0 * (phases - 1)) / max(mean_iters, 1.0)


def cyl_kernel_bytes(ws: int, shots: int, fused: bool = True, dichotomy: bool = True, held: bool = False):
    """The same for the axisymmetric iteration (Sec. 2.3): fused, the update
    recomputes A p (stored-q form: the operator writes q, the update reads it);
    the r-systems read rhat and write zhat once (the Thomas sweep's
    intermediate, or the Dichotomy's three values per segment, are not
    counted); the face tables, shift and r-system factors are shared by all
    shots; with the Dichotomy the inverse transform also reads the two
    separator responses of every row (shared by all shots).  held: the update
    leaves x alone (the flush pass is counted by flush_bytes)."""
    xb = 0 if held else 16                                    # x in/out (f64)
    if fused:
        op = ws + 3 * ws / shots                              # p in; a1, a2, w once per batch
        upd = xb + 16 + 2 * ws + 3 * ws / shots               # r in/out (f64); p in; rhat out; medium
    else:
        op = 2 * ws + 3 * ws / shots                          # p in, q out; a1, a2, w once per batch
        upd = xb + 16 + 3 * ws                                # r in/out (f64); p, q in; rhat out
    return {
        "operator": op,
        "update_fdct": upd,
        "r_systems": 2 * ws + 2 * ws / shots,                 # rhat in, zhat out; factors once per batch
        "correct_idct": 3 * ws + (2 * ws / shots if dichotomy else 0),   # zhat in, p in/out
    }


def copy_probe(mib: int = 2048, reps: int = 10):
    """Device-to-device copy bandwidth on this GPU (read + write bytes per
    second), the practical streaming ceiling the kernels are compared with."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def library_source_sha256() -> str:
    """Hash of the library sources (kernels, host code, C header)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1005_0542_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "laguerre.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE / WRITE_SIZE scaled by a plain-copy
    calibration), or None when there is none or the library has changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pcg_kernels_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("library_source_sha256") != library_source_sha256():
        return None
    v = fields.get(f"traffic_bytes_per_launch[{kernel}]")
    return float(v) if v is not None else None


def tuned_params(name, precision, shots, enabled=True):
    """Tile/segment parameters from the autotuner (its JSON cache, or a fresh
    search on this device when the cache has no entry for the problem)."""
    if not enabled:
        return {}
    from paper_1005_0542_amd import inputs, tune
    w = inputs.WORKLOADS[name]
    kappa, rho = inputs.acoustic_medium_for(w)
    t0 = time.perf_counter()
    best = tune.tune_acoustic(w.n_cells, w.n_cells, w.d, w.d, w.alpha, w.h, np.stack([kappa, rho]),
                              precision, shots)
    log(f"{name} {precision} x{shots}: tuned {best} ({time.perf_counter() - t0:.1f} s)")
    return best


def run_variant(name, precision, shots, steps, warmup, segments=0, graph_iters=0, profile=True,
                tuned=None, profile_iters=20, top="dirichlet", geometry="cartesian", order=2):
    import torch
    from paper_1005_0542_amd import inputs
    from paper_1005_0542_amd.driver import AcousticRun

    w = inputs.WORKLOADS[name]
    n_harm = warmup + steps
    tuned = dict(tuned or {})
    if segments:
        tuned["segments"] = segments
    if graph_iters:
        tuned["graph_iters"] = graph_iters
    log(f"{name}: precision={precision} shots={shots} harmonics={n_harm} params={tuned}")
    t0 = time.perf_counter()
    run = AcousticRun(w, precision=precision, shots=shots, n_harm=max(n_harm, 2),
                      segments=tuned.get("segments", 0), graph_iters=tuned.get("graph_iters", 0),
                      op_shots=tuned.get("op_shots", 0), seg_per_wave=tuned.get("seg_per_wave", 0),
                      op_fusion=tuned.get("op_fusion", 0), top=top, geometry=geometry, order=order,
                      x_ring=tuned.get("x_ring", 0))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    cyl = geometry == "cylindrical"
    npts = (w.n_cells - 1) * (w.n_cells if cyl else w.n_cells - 1)
    for _ in range(warmup):
        run.step()
    run.finish()                          # the warm-up harmonics' synthesis, untimed
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters = []
    for _ in range(steps):
        res = run.step()
        iters.append(res.iters)
    run.finish()                          # the timed harmonics still pending synthesis
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    pt_iters = float(npts) * float(np.sum(iters))
    out = {
        "workload": name, "precision": precision, "shots": shots, "top": top, "geometry": geometry,
        "order": order,
        "value": pt_iters / el / 1e6, "ms_per_step": 1e3 * el / steps,
        "iters_per_harmonic": [int(max(i)) for i in iters],
        "mean_iters": float(np.mean(iters)),
        "setup_s": setup_s,
        "status": [int(s) for s in run.status],
    }
    seg, seg_len = run.plan.layout()
    out["segments"] = seg
    ws = 8 if precision == "fp64" else 4
    x_ring = run.plan.x_ring()
    held = x_ring > 1
    # the library's default op_fusion: stored q for FP64 axisymmetric plans
    # and the fourth-order operator, else recomputed in the update
    fusion = tuned.get("op_fusion", 0) or (2 if (cyl and precision == "fp64") or order == 4 else 1)
    if cyl:
        kb = cyl_kernel_bytes(ws, shots, fusion != 2, seg > 1, held=held)
    elif order == 4:
        kb = kernel_bytes(ws, shots, seg_len, fused=False, medium=3, held=held)
    else:
        kb = kernel_bytes(ws, shots, seg_len, fusion != 2, held=held)
    slots = [0, 1, 2, 4] if cyl else [0, 1, 2, 3, 4]          # the profile helper's kernel slots
    mean_it = max(out["mean_iters"], 1e-9)
    fb = flush_bytes(ws, mean_it, 2 if precision == "mixed" else 1) if held else 0.0
    per_iter_bytes = (sum(kb.values()) + fb) * npts * shots
    t_iter = el / (steps * mean_it)
    out["x_ring"] = x_ring
    out["alg_bytes_per_point_iter"] = sum(kb.values()) + fb
    out["whole_iteration_GBps"] = per_iter_bytes / t_iter / 1e9   # includes per-harmonic overheads
    if profile:
        # per-kernel durations on the same plan and stream, with the last timed
        # harmonic's right-hand side and every shot active
        b = run.rhs.clone()
        x = torch.empty_like(b)
        ms = run.plan.pcg_profile(b, x, iters=profile_iters)
        names = list(kb.keys())
        kern = {}
        for k, nm in zip(slots, names):
            byts = kb[nm] * npts * shots
            kern[nm] = {"avg_ms": ms[k], "alg_bytes": byts, "GBps": byts / (ms[k] * 1e-3) / 1e9}
        out["kernels"] = kern
        out["iteration_ms_profiled"] = float(sum(ms[k] for k in slots))
        dom = max(names, key=lambda nm: kern[nm]["avg_ms"])
        out["dominant"] = dom
    out["_run"] = run
    return out


def run_elastic(name="elastic1024", steps=2, warmup=1, restart=10, shots=None, top="dirichlet", segments=0):
    """Elastic harmonics (GMRES(k) per harmonic) timed like the acoustic ones;
    reported with the time of one GMRES(k) cycle (k inner iterations), the
    unit of the paper's Table 2."""
    import torch
    from paper_1005_0542_amd import inputs
    from paper_1005_0542_amd.driver import ElasticRun

    w = inputs.WORKLOADS[name]
    S = shots or w.shots
    log(f"{name}: GMRES({restart}) harmonics={warmup + steps} shots={S} top={top}")
    run = ElasticRun(w, n_harm=warmup + steps, restart=restart, shots=S, top=top, segments=segments)
    for _ in range(warmup):
        run.step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = []
    for _ in range(steps):
        its.append(run.step().iters[0])
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    npts = 2 * (w.n_cells - 1) ** 2
    out = {"workload": name, "precision": "fp64", "shots": S, "top": top, "restart": restart,
           "segments": run.plan.layout()[0],
           "value": npts * S * sum(its) / el / 1e6,
           "unit": "Mpoint-iters/s (GMRES inner iterations, 2 components)",
           "ms_per_step": 1e3 * el / steps, "inner_iters_per_harmonic": its,
           "ms_per_gmres_cycle": 1e3 * el / (sum(its) / restart)}
    run.plan.destroy()
    del run
    torch.cuda.empty_cache()
    return out


def cpu_baseline(name, k_lo=2, k_hi=12):
    """The FP64 oracle's PCG (numpy/scipy) on one shot of the same workload:
    per-iteration time from two fixed-iteration runs (tol = 0)."""
    from paper_1005_0542_amd import inputs
    from oracle import operator, precond, krylov

    w = inputs.WORKLOADS[name]
    kappa, rho = inputs.acoustic_medium_for(w)
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    b = np.zeros((N - 1, N - 1))
    i, j = inputs.sources_for(w)[0]
    b[j - 1, i - 1] = 1.0 / (d * d)
    A = lambda y: operator.apply_A(y, kappa, wv, d, d)
    times, cpus = [], []
    for k in (k_lo, k_hi):
        t = time.perf_counter()
        c = time.process_time()
        krylov.pcg(A, B.solve, b, 0.0, k)
        times.append(time.perf_counter() - t)
        cpus.append(time.process_time() - c)
    dt = max(times[1] - times[0], 1e-9)
    its = k_hi - k_lo
    npts = (N - 1) ** 2
    cores = max(1, int(round((cpus[1] - cpus[0]) / dt)))
    return {
        "value": npts * its / dt / 1e6, "unit": "Mpoint-iters/s", "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 numpy oracle PCG, 1 shot of {name} ({N - 1}^2 points), "
                  f"{its} iterations (difference of {k_hi}- and {k_lo}-iteration runs), "
                  f"{os.cpu_count()} host cores visible",
    }


def parity_leg(name, tuned, samples=(0, 63), n_harm=3):
    """Error of the benchmarked path against the FP64 oracle, outside every
    timed region: the workload's first harmonics in its own precision and
    launch configuration, sampled shots against the oracle's own chains
    (tolerance 1e-10), per harmonic and on the partial snapshots."""
    import torch
    from paper_1005_0542_amd import inputs
    from paper_1005_0542_amd.driver import AcousticRun
    from oracle import harmonics, krylov, laguerre, operator, precond

    w = inputs.WORKLOADS[name]
    samples = tuple(s for s in samples if s < w.shots)
    run = AcousticRun(w, n_harm=n_harm, snapshots=True, rec=False,
                      **{k: tuned.get(k, 0) for k in ("segments", "graph_iters", "op_shots", "seg_per_wave",
                                                      "op_fusion")})
    got = {s: [] for s in samples}
    for _ in range(n_harm):
        run.step()
        for s in samples:
            got[s].append(run.R[s, 0].cpu().numpy())
    snap = run.snap.cpu().numpy()
    kappa, rho = run.kappa, run.rho
    run.plan.destroy()
    del run
    torch.cuda.empty_cache()
    N, d = w.n_cells, w.d
    wv = operator.shift_coeff(rho, w.h)
    B = precond.acoustic_preconditioner(kappa, rho, w.h, N, N, d, d)
    solve = lambda phi: krylov.pcg(lambda y: operator.apply_A(y, kappa, wv, d, d), B.solve, phi, 1e-10, 10000)
    f_m = laguerre.ricker_coeffs(w.f0, w.t0, w.h, w.alpha, n_harm)
    Wsn = laguerre.synthesis_weights(np.array(inputs.snapshot_times(w)), w.h, w.alpha, n_harm)
    l2 = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    per_shot = {}
    for s in samples:
        st = harmonics.harmonic_loop(n_harm, solve, rho[1:-1, 1:-1], w.h, w.alpha, f_m, inputs.sources_for(w)[s],
                                     d, d, snap_w=Wsn, keep_all=True)
        per_shot[str(s)] = {"R_rel_l2": [float("%.3g" % l2(got[s][m], st["R"][m])) for m in range(n_harm)],
                            "snapshots_rel_l2": float("%.3g" % l2(snap[:, s, 0], st["snap"]))}
    worst = max(max(v["R_rel_l2"] + [v["snapshots_rel_l2"]]) for v in per_shot.values())
    return {"vs": "FP64 oracle chain (tol 1e-10)", "workload": name, "precision": w.precision,
            "harmonics": n_harm, "shots": list(samples), "per_shot": per_shot, "worst_rel_l2": worst,
            "bar": 1e-6 if w.precision == "mixed" else 1e-12}


def time_to_solution(name, tuned):
    """One whole run of a workload: all its harmonics (right-hand side, PCG,
    synthesis of the 4 snapshots and the receiver row), then the receiver
    traces at 1 ms, timed end to end after the plan is set up."""
    import torch
    from paper_1005_0542_amd import inputs
    from paper_1005_0542_amd.driver import AcousticRun

    w = inputs.WORKLOADS[name]
    t0 = time.perf_counter()
    run = AcousticRun(w, **{k: tuned.get(k, 0) for k in ("segments", "graph_iters", "op_shots", "seg_per_wave",
                                                         "op_fusion")})
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    log(f"{name}: time to solution over {w.n_harm} harmonics")
    t1 = time.perf_counter()
    its = []
    for _ in range(w.n_harm):
        its.append(run.step().iters)
    tr = run.traces(inputs.trace_times(w))
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    npts = (w.n_cells - 1) ** 2
    total = int(np.sum(its))
    out = {"harmonics": w.n_harm, "shots": w.shots, "seconds": round(el, 3), "setup_s": round(setup, 3),
           "ms_per_harmonic": round(1e3 * el / w.n_harm, 3), "cg_iterations_summed_over_shots": total,
           "mean_iters": round(total / (w.n_harm * w.shots), 2),
           "Mpoint_iters_per_s": round(npts * total / el / 1e6, 1),
           "statuses_ok": bool(all(s == 0 for s in run.status)), "traces": list(tr.shape)}
    run.plan.destroy()
    del run, tr
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="acoustic2048x64_mixed")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the error-vs-oracle leg")
    ap.add_argument("--no-tts", action="store_true", help="skip the whole-run time-to-solution leg")
    ap.add_argument("--segments", type=int, default=0)
    ap.add_argument("--graph-iters", type=int, default=0)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the per-kernel profile of the workload (for hardware-counter runs)")
    ap.add_argument("--profile-iters", type=int, default=20,
                    help="CG iterations timed per kernel by --profile-only")
    ap.add_argument("--precision", default=None, help="override the workload precision")
    ap.add_argument("--shots", type=int, default=None, help="override the workload shot count")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="time a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of autotuned tiles")
    ap.add_argument("--elastic-only", action="store_true",
                    help="only the elastic GMRES(10) harmonics (for kernel traces of the elastic path)")
    ap.add_argument("--op-shots", type=int, default=0, help="override the tuned value")
    ap.add_argument("--seg-per-wave", type=int, default=0, help="override the tuned value")
    ap.add_argument("--op-fusion", type=int, default=0, help="override the tuned value: 1 fused, 2 stored q")
    ap.add_argument("--x-ring", type=int, default=0,
                    help="held CG search directions (1: x updated in every iteration; 0: library default)")
    ap.add_argument("--geometry", default="cartesian", choices=("cartesian", "cylindrical"),
                    help="profile-only: the 2D Cartesian or the 2.5D axisymmetric problem")
    ap.add_argument("--order", type=int, default=2, choices=(2, 4),
                    help="profile-only: the second- or fourth-order operator (Cartesian)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library drives one GPU per process "
              "(a batch of shots would shard across GPUs with no exchange during the solve).", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1005_0542_amd import inputs

    w = inputs.WORKLOADS[args.workload]
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))
        return
    prec = args.precision or w.precision
    shots = args.shots or w.shots
    if args.elastic_only:
        print(json.dumps(run_elastic(steps=args.steps, warmup=args.warmup, shots=args.shots, segments=args.segments)))
        return
    if args.profile_only:
        # the benchmark's own path on two harmonics (one untimed), then the
        # per-kernel profile: a kernel trace of this mode ends with exactly
        # --profile-iters launches of each iteration kernel with all shots active
        geo = args.geometry
        tp = tuned_params(args.workload, prec, shots, not args.no_tune and geo == "cartesian")
        tp.update({k: getattr(args, k) for k in ("op_shots", "seg_per_wave", "op_fusion", "x_ring")
                   if getattr(args, k)})
        if args.order == 4:
            tp["op_fusion"] = 2
        v = run_variant(args.workload, prec, shots, args.steps, args.warmup, segments=args.segments,
                        graph_iters=args.graph_iters, tuned=tp, profile_iters=args.profile_iters, geometry=geo,
                        order=args.order)
        v.pop("_run")
        print(json.dumps({k: v[k] for k in ("workload", "precision", "shots", "geometry", "order", "segments", "kernels",
                                            "iteration_ms_profiled")} | {"tuned": tp,
                                                                         "profile_iterations": args.profile_iters}))
        return
    head_tuned = tuned_params(args.workload, prec, shots, not args.no_tune)
    head_tuned.update({k: getattr(args, k) for k in ("op_shots", "seg_per_wave", "op_fusion", "x_ring")
                       if getattr(args, k)})
    head = run_variant(args.workload, prec, shots, args.steps, args.warmup,
                       segments=args.segments, graph_iters=args.graph_iters, tuned=head_tuned,
                       profile_iters=args.profile_iters)
    head.pop("_run")
    torch.cuda.empty_cache()
    variants = {}
    if not args.no_variants:
        plan = [
            ("acoustic1024", "fp64", 1, "fp64_1shot_1024", "dirichlet"),
            ("acoustic4096_mixed", "fp64", 1, "fp64_1shot_4096", "dirichlet"),
            ("acoustic4096_mixed", "mixed", 1, "mixed_1shot_4096", "dirichlet"),
            ("acoustic2048x64_mixed", "fp64", 64, "fp64_64shot_2048", "dirichlet"),
            # the same batch with the free-surface top boundary (rank-one corrected Dichotomy)
            ("acoustic2048x64_mixed", "mixed", 64, "mixed_64shot_2048_free_surface", "free"),
            # the paper's 2.5D axisymmetric problem, N_r x N_z = 2048 x 2048, sources on the axis
            ("acoustic2048x64_mixed", "fp64", 64, "fp64_64shot_2048_axisymmetric", "cylindrical"),
            ("acoustic2048x64_mixed", "mixed", 64, "mixed_64shot_2048_axisymmetric", "cylindrical"),
            # the fourth-order operator preconditioned by the same second-order B
            ("acoustic2048x64_mixed", "mixed", 64, "mixed_64shot_2048_order4", "order4"),
        ]
        for name, prec, shots, key, top in plan:
            geo = "cylindrical" if top == "cylindrical" else "cartesian"
            order = 4 if top == "order4" else 2
            tp = tuned_params(name, prec, shots, not args.no_tune and geo == "cartesian")
            if order == 4:
                tp["op_fusion"] = 2                            # the update reads a stored q
            v = run_variant(name, prec, shots, max(2, args.steps // 2), 1, tuned=tp,
                            profile_iters=args.profile_iters, top=top if top in ("dirichlet", "free") else "dirichlet",
                            geometry=geo, order=order)
            v.pop("_run")
            variants[key] = {k: v[k] for k in ("workload", "precision", "shots", "top", "geometry", "order", "value",
                                               "ms_per_step", "mean_iters", "whole_iteration_GBps", "dominant")}
            variants[key]["kernels_GBps"] = {k: round(x["GBps"], 1) for k, x in v["kernels"].items()}
            torch.cuda.empty_cache()
        variants["elastic_gmres10_1024"] = run_elastic()
        variants["elastic_gmres10_1024_free_surface"] = run_elastic(top="free")
        variants["elastic_gmres10_1024_x8"] = run_elastic(shots=8)
        torch.cuda.empty_cache()
        fp64_1 = variants["fp64_1shot_4096"]["value"]
        variants["speedup_mixed64_vs_fp64_1shot_per_iteration"] = head["value"] / fp64_1
        # time per harmonic for the same work (every shot-point solved to its
        # tolerance, restart iterations included): mixed 64-shot batch against
        # the FP64 64-shot batch, and per shot-point against FP64 single-shot
        f64b = variants["fp64_64shot_2048"]
        variants["speedup_mixed64_vs_fp64_64shot_time_per_harmonic"] = f64b["ms_per_step"] / head["ms_per_step"]
        pts_head = shots * (w.n_cells - 1) ** 2
        pts_4096 = (inputs.WORKLOADS["acoustic4096_mixed"].n_cells - 1) ** 2
        variants["speedup_mixed64_vs_fp64_1shot_time_per_shot_point_harmonic"] = \
            (variants["fp64_1shot_4096"]["ms_per_step"] / pts_4096) / (head["ms_per_step"] / pts_head)

    dom = head["dominant"]
    kd = head["kernels"][dom]
    achieved = kd["GBps"]
    traffic = counter_traffic(dom, args.workload)
    copy_gbps = copy_probe()
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "alg_bytes_per_launch": round(kd["alg_bytes"]),
            "per_kernel_GBps": {k: round(x["GBps"], 1) for k, x in head["kernels"].items()},
            "per_kernel_ms": {k: round(x["avg_ms"], 4) for k, x in head["kernels"].items()},
            "whole_iteration_GBps": round(head["whole_iteration_GBps"], 1),
            # solver level: one whole iteration's algorithmic bytes over the
            # timed harmonic (per-harmonic work and masked replays included)
            "whole_iteration_frac": round(head["whole_iteration_GBps"] / HBM_PEAK_GBS, 4),
            "profiled_iteration_frac": round(sum(x["alg_bytes"] for x in head["kernels"].values()) /
                                             (head["iteration_ms_profiled"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "copy_probe_GBps": round(copy_gbps, 1),
            "frac_of_copy_probe": round(achieved / copy_gbps, 4),
            "alg_bytes_per_point_iter": round(head["alg_bytes_per_point_iter"], 2)}
    tts = {}
    if not args.no_tts:
        for name in (args.workload, "acoustic4096_mixed"):
            if name in tts:
                continue
            wn = inputs.WORKLOADS[name]
            tp = head_tuned if name == args.workload else tuned_params(name, wn.precision, wn.shots, not args.no_tune)
            tts[name] = time_to_solution(name, tp)
    parity = None
    if not args.no_parity:
        log("parity leg (oracle chains of sampled shots)")
        parity = parity_leg(args.workload, head_tuned)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(args.workload)
    line = {
        "metric": METRIC, "value": round(head["value"], 1), "unit": "Mpoint-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if w.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{w.n_cells}x{w.n_cells}", "dx_m": w.d,
                   "shots": w.shots, "precision": w.precision, "tol": w.tol, "alpha": w.alpha,
                   "h": w.h, "harmonics_timed": f"{args.warmup}..{args.warmup + args.steps - 1}",
                   "segments": head["segments"], "tuned": head_tuned,
                   "parallelism": "single GPU, shot batch"},
        "iters_per_harmonic": head["iters_per_harmonic"],
        "setup_s": round(head["setup_s"], 3),
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "time_to_solution": tts,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
