// Preconditioned CG driver (Sec. 2.3): all shots of the plan iterate together,
// every scalar (alpha, beta, norms, convergence) stays on the device, and
// converged shots drop out by masking.  Batches of iterations are captured in
// a HIP graph once per plan and replayed; the host only reads the per-shot
// "active" flags between batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lg_internal.h"

namespace lg {

namespace {

hipError_t enqueue_iteration(lg_plan* p) {
    const int nf = p->S * p->C;
    if (p->cyl) {   // axisymmetric: transforms along z, Thomas per wavenumber
        hipError_t e = launch_stencil(p, p->p, p->fuse_op ? nullptr : p->qv, true);   // (p, Ap), alpha
        if (e == hipSuccess) e = cyl_launch_update(p, 0, nullptr, nullptr, 0.0, 0);  // x, r, rhat
        if (e == hipSuccess) e = cyl_launch_rsys(p, p->rhat, p->y, nf, 2);         // zhat, beta
        if (e == hipSuccess) e = cyl_launch_correct(p, 0);                         // z, p = z + beta p
        return e;
    }
    // (p, A p) and alpha; q = A p is stored only when the update does not
    // recompute it
    hipError_t e = launch_stencil(p, p->p, p->fuse_op ? nullptr : p->qv, true);
    if (e == hipSuccess) e = launch_update_fdst(p, 0, nullptr, nullptr, 0.0, 0);  // x, r, rhat
    if (e == hipSuccess) e = launch_td(p, 0, p->rhat, p->y, nf, 1);        // segments
    if (e == hipSuccess) e = launch_rs(p, 0, p->rhat, p->y, nf, 2);        // interfaces, beta
    if (e == hipSuccess) e = launch_correct_idst(p, 0);                    // z, p = z + beta p
    return e;
}

lg_status build_graph(lg_plan* p) {
    if (p->cg_graph != nullptr) return LG_OK;
    if (p->cap_stream == nullptr) LG_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = p->stream;
    p->stream = p->cap_stream;
    hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        p->stream = saved;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hipError_t le = hipSuccess;
    for (int i = 0; i < p->graph_iters && le == hipSuccess; ++i) le = enqueue_iteration(p);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    p->stream = saved;
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "kernel launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->cg_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        p->cg_graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return LG_OK;
}

int severity(int s) {
    switch (s) {
        case LG_OK: return 0;
        case LG_ERR_NOT_CONVERGED: return 1;
        case LG_ERR_BREAKDOWN: return 2;
        case LG_ERR_NONFINITE: return 3;
        default: return 4;
    }
}

}  // namespace

double phase_tol(const lg_plan* p, double tol, bool restart) {
    if (p->prec != LG_MIXED || tol <= 0.0) return tol;
    return restart ? LG_MIXED_REFINE_FAC * tol : std::max(tol, LG_MIXED_PHASE1_TOL);
}

void pcg_release(lg_plan* p) {
    if (p->cg_graph) (void)hipGraphExecDestroy(p->cg_graph);
    p->cg_graph = nullptr;
}

lg_status pcg_solve(lg_plan* p, const double* b, double* x, const lg_solve_opts* o, lg_solve_info* info) {
    const int nf = p->S * p->C;
    const bool use_graph = p->graph_iters > 0;
    const int chunk = use_graph ? p->graph_iters : 8;
    if (use_graph) {
        lg_status st = build_graph(p);
        if (st != LG_OK) return st;
    }
    // start: x = 0, r = b (or, from a given x, r = b - A x in FP64), rhat = DST(r),
    // z = B^{-1} r, p = z, rz = (r, z)
    if (p->cyl) {
        LG_HIP(cyl_launch_update(p, 1, b, x, o->tol, o->max_iter));
        LG_HIP(cyl_launch_rsys(p, p->rhat, p->y, nf, 1));
        LG_HIP(cyl_launch_correct(p, 1));
    } else {
        LG_HIP(launch_update_fdst(p, o->x0_given ? 4 : 1, b, x, o->tol, o->max_iter));
        LG_HIP(launch_td(p, 0, p->rhat, p->y, nf, 1));
        LG_HIP(launch_rs(p, 0, p->rhat, p->y, nf, 1));
        LG_HIP(launch_correct_idst(p, 1));
    }

    // Held search directions: x is brought up to date by a flush pass before
    // anything reads it (the FP64 check and restart, the end of the solve) and
    // before a batch could overwrite a direction not yet added (at most
    // pring - 1 iterations between flushes; a batch is shorter).
    const bool held = p->pring > 1;
    int since = 0;                    // iterations queued since the last flush
    auto flush = [&]() -> lg_status {
        if (held) LG_HIP(launch_flush_x(p, x));
        since = 0;
        return LG_OK;
    };

    // Replay batches of captured iterations until every shot has stopped.
    // Consecutive harmonics take similar iteration counts, so as many batches
    // as the previous solve needed in the same phase (up to the first stop,
    // or after the first restart) are queued before the first check; batches
    // past a shot's stop run masked, which still costs every launch.
    auto iterate = [&](long& launched, int expect) -> lg_status {
        long ahead = std::max(1L, (long)((expect + chunk - 1) / chunk));
        const long cap = (long)o->max_iter + chunk;
        while (true) {
            for (long bt = 0; bt < ahead && launched < cap; ++bt) {
                if (held && since + chunk > p->pring - 1) {
                    const lg_status fs = flush();
                    if (fs != LG_OK) return fs;
                }
                since += chunk;
                if (use_graph) {
                    LG_HIP(hipGraphLaunch(p->cg_graph, p->stream));
                } else {
                    for (int i = 0; i < chunk; ++i) LG_HIP(enqueue_iteration(p));
                }
                launched += chunk;
            }
            LG_HIP(hipMemcpyAsync(p->ctl_host, p->ctl, (size_t)nf * sizeof(ShotCtl), hipMemcpyDeviceToHost,
                                  p->stream));
            LG_HIP(hipStreamSynchronize(p->stream));
            bool any = false;
            for (int s = 0; s < nf; ++s) any = any || (p->ctl_host[s].active != 0);
            if (!any || launched >= cap) break;
            ahead = 1;
        }
        return LG_OK;
    };
    auto max_iters = [&]() {
        int m = 0;
        for (int s = 0; s < nf; ++s) m = std::max(m, (int)p->ctl_host[s].iters);
        return m;
    };
    long launched = 0;
    lg_status st = iterate(launched, p->last_iters);
    if (st != LG_OK) return st;
    const int first_stop = max_iters();      // ctl_host is current after iterate
    int after_restart = -1;
    // Mixed precision: the recursive residual converges on the FP32 operator;
    // check the FP64 true residual b - A x and, where it misses the tolerance,
    // restart CG from it (iterative refinement with an FP64 residual).  The
    // check alone reads x and b; the restart also stores r and transforms it.
    // Nearly every shot resumes after the first check and almost none after
    // a later one, so the first restart of the Cartesian second-order path is
    // the fused pass (residual and transform at once) and every other one is
    // preceded by the check.  After the last allowed restart the check still
    // runs: a shot that misses the tolerance there ends NOT_CONVERGED with its
    // true residual reported.
    constexpr int MAX_RESTARTS = 4;
    auto any_active = [&](bool& any) -> lg_status {
        LG_HIP(hipMemcpyAsync(p->ctl_host, p->ctl, (size_t)nf * sizeof(ShotCtl), hipMemcpyDeviceToHost,
                              p->stream));
        LG_HIP(hipStreamSynchronize(p->stream));
        any = false;
        for (int s = 0; s < nf; ++s) any = any || (p->ctl_host[s].active != 0);
        return LG_OK;
    };
    if (p->prec == LG_MIXED) {
        for (int rep = 0; rep <= MAX_RESTARTS; ++rep) {
            bool any = false;
            const bool fused = !p->cyl && p->order == 2 && rep == 0;
            if ((st = flush()) != LG_OK) return st;       // the check and the restart read x
            if (!fused) {
                LG_HIP(launch_residual_check(p, b, x));       // axisymmetric, fourth order: stores r too
                if ((st = any_active(any)) != LG_OK) return st;
                if (!any || rep == MAX_RESTARTS) break;
            }
            if (p->cyl) {                                                  // transform of the stored r
                LG_HIP(cyl_launch_restart(p, b, x, o->tol, o->max_iter));
                LG_HIP(cyl_launch_rsys(p, p->rhat, p->y, nf, 1));
                LG_HIP(cyl_launch_correct(p, 1));
            } else {
                // second order: r = b - A x and its transform in one pass (init 3);
                // fourth order: the transform of the r stored by the check (init 2)
                LG_HIP(launch_update_fdst(p, p->order == 4 ? 2 : 3, b, x, o->tol, o->max_iter));
                LG_HIP(launch_td(p, 0, p->rhat, p->y, nf, 1));
                LG_HIP(launch_rs(p, 0, p->rhat, p->y, nf, 1));
                LG_HIP(launch_correct_idst(p, 1));
            }
            if ((st = any_active(any)) != LG_OK) return st;
            if (!any) break;
            launched = 0;
            st = iterate(launched, rep == 0 ? p->last_iters_restart : 1);
            if (st != LG_OK) return st;
            if (rep == 0) after_restart = max_iters() - first_stop;
        }
    }
    if (held) {                           // the remaining directions; x = 0 for a cold-start
        if ((st = flush()) != LG_OK) return st;   // shot that never iterated
    } else if (!o->x0_given) {            // a cold start stores no x: a shot that never
        for (int s = 0; s < nf; ++s)      // iterated (b = 0, or not finite) gets x = 0
            if (p->ctl_host[s].iters == 0)
                LG_HIP(hipMemsetAsync(x + (size_t)s * p->npts, 0, p->npts * sizeof(double), p->stream));
    }
    if (o->x0_given) {                    // b = 0 from a given x: the solution is 0
        for (int s = 0; s < nf; ++s)
            if (p->ctl_host[s].bb == 0.0 && p->ctl_host[s].status == LG_OK)
                LG_HIP(hipMemsetAsync(x + (size_t)s * p->npts, 0, p->npts * sizeof(double), p->stream));
    }
    int worst = LG_OK;
    for (int s = 0; s < nf; ++s) {
        const ShotCtl& c = p->ctl_host[s];
        int st = c.status;
        if (c.active) st = LG_ERR_NOT_CONVERGED;   // only if the safety cap was hit
        if (severity(st) > severity(worst)) worst = st;
        if (info) {
            info[s].iters = c.iters;
            info[s].status = st;
            info[s].relres = (c.bb > 0.0) ? std::sqrt(c.rr / c.bb) : 0.0;
        }
    }
    p->last_iters = first_stop;
    if (after_restart >= 0) p->last_iters_restart = after_restart;
    return (lg_status)worst;
}

lg_status pcg_profile(lg_plan* p, const double* b, double* x, int iters, float* ms) {
    const int nf = p->S * p->C;
    const bool cy = p->cyl;
    if (cy) {
        LG_HIP(cyl_launch_update(p, 1, b, x, 0.0, iters + 2));
        LG_HIP(cyl_launch_rsys(p, p->rhat, p->y, nf, 1));
        LG_HIP(cyl_launch_correct(p, 1));
    } else {
        LG_HIP(launch_update_fdst(p, 1, b, x, 0.0, iters + 2));
        LG_HIP(launch_td(p, 0, p->rhat, p->y, nf, 1));
        LG_HIP(launch_rs(p, 0, p->rhat, p->y, nf, 1));
        LG_HIP(launch_correct_idst(p, 1));
    }
    hipEvent_t ev[6] = {};
    for (int i = 0; i < 6; ++i) LG_HIP(hipEventCreate(&ev[i]));
    double acc[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipSuccess;
    // iteration 0 is not timed: after a cold start the first update reads b
    // for r and no x (fewer bytes than every later one).  Held directions are
    // flushed into x between timed iterations where needed, and at the end.
    int since = 0;
    for (int it = 0; it <= iters && e == hipSuccess; ++it) {
        if (p->pring > 1 && since + 1 > p->pring - 1) {
            e = launch_flush_x(p, x);
            since = 0;
            if (e != hipSuccess) break;
        }
        ++since;
        e = hipEventRecord(ev[0], p->stream);
        if (e == hipSuccess) e = launch_stencil(p, p->p, p->fuse_op ? nullptr : p->qv, true);
        if (e == hipSuccess) e = hipEventRecord(ev[1], p->stream);
        if (e == hipSuccess)
            e = cy ? cyl_launch_update(p, 0, nullptr, nullptr, 0.0, 0)
                   : launch_update_fdst(p, 0, nullptr, nullptr, 0.0, 0);
        if (e == hipSuccess) e = hipEventRecord(ev[2], p->stream);
        if (e == hipSuccess)
            e = cy ? cyl_launch_rsys(p, p->rhat, p->y, nf, 2) : launch_td(p, 0, p->rhat, p->y, nf, 1);
        if (e == hipSuccess) e = hipEventRecord(ev[3], p->stream);
        if (e == hipSuccess && !cy) e = launch_rs(p, 0, p->rhat, p->y, nf, 2);
        if (e == hipSuccess) e = hipEventRecord(ev[4], p->stream);
        if (e == hipSuccess) e = cy ? cyl_launch_correct(p, 0) : launch_correct_idst(p, 0);
        if (e == hipSuccess) e = hipEventRecord(ev[5], p->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
        for (int k = 0; k < 5 && e == hipSuccess && it > 0; ++k) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
    }
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    if (e == hipSuccess) e = launch_flush_x(p, x);
    if (e != hipSuccess) return hip_fail(e, "lg_pcg_profile");
    for (int k = 0; k < 5; ++k) ms[k] = (float)(acc[k] / iters);
    return LG_OK;
}

}  // namespace lg
