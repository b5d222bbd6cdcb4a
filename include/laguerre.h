/*
 * laguerre.h -- C ABI of the MI355X (gfx950) library for the Laguerre-harmonic
 * Krylov solve of Fatyanov & Terekhov, "High-performance modeling acoustic and
 * elastic waves using the Parallel Dichotomy Algorithm" (arXiv 1005.0542).
 *
 * The method (Sec. 2): an integral Laguerre transform in time turns the wave
 * equation into a sequence of elliptic problems with ONE fixed operator and a
 * right-hand side that depends on the earlier harmonics (eq. laguerre_h).
 * Each problem is solved by a Krylov method (CG for acoustics, GMRES(k) for
 * elasticity, Sec. 2.3) preconditioned by a constant-coefficient Laplace
 * operator (Sec. 2.4, eqs. precond1/precond2), inverted by separation of
 * variables: a sine transform along x, then one tridiagonal system per
 * wavenumber along z, solved by a segmented Dichotomy-style solver.
 *
 * Geometry: 2D Cartesian, nx x nz cells, nodes i = 0..nx, j = 0..nz, zero
 * Dirichlet values on all boundary nodes (the top one optionally flux-free).
 * The unknowns are the (nx-1)(nz-1) interior nodes.  The paper's 2.5D
 * axisymmetric problem is selected by lg_grid.geometry (layout below).
 *
 * ---------------------------------------------------------------------------
 * Conventions for every call below
 * ---------------------------------------------------------------------------
 * Layout.   A "field" is (nz-1) rows of (nx-1) values, row-major, x fastest:
 *           element (i, j) (1-based interior node) is at [(j-1)(nx-1) + (i-1)].
 *           A "vector" is S shots x C components x field, contiguous
 *           ([S][C][nz-1][nx-1]); C = 1 (acoustic) or 2 (elastic: x then z).
 *           Axisymmetric plans: a field is nz-1 rows of nx values, so every
 *           row length nx-1 below reads nx for them.
 * Memory.   Vector and field pointers are DEVICE pointers owned by the caller
 *           (contiguous, no padding, naturally aligned).  Pointers suffixed
 *           _host are host pointers.  The plan owns only its tables and
 *           workspace.
 * Dtypes.   Arguments typed double* are FP64.  Arguments typed void* are the
 *           plan's working type: FP64 for LG_FP64 plans, FP32 for LG_MIXED.
 * Streams.  All device work is enqueued on the plan's stream (a hipStream_t
 *           given at creation, or set later); calls return without waiting,
 *           except those that fill a *_host output (they synchronise it).
 * Errors.   Every argument is checked on the host before any device work; an
 *           invalid call returns LG_ERR_INVALID_ARG (or LG_ERR_UNSUPPORTED for
 *           a valid but unimplemented shape) and leaves outputs untouched.
 *           HIP failures return LG_ERR_HIP; lg_last_error() describes the
 *           last failure of the calling thread.
 * Threads.  A plan must not be used by two threads at once; distinct plans
 *           are independent.
 */
#ifndef LAGUERRE_H
#define LAGUERRE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LG_OK = 0,
    LG_ERR_INVALID_ARG = 1,
    LG_ERR_NOT_CONVERGED = 2,   /* max_iter reached; x holds the last iterate   */
    LG_ERR_BREAKDOWN = 3,       /* (p, Ap) <= 0 in CG, or an exact GMRES stall  */
    LG_ERR_NONFINITE = 4,       /* NaN/Inf met in a residual or inner product   */
    LG_ERR_HIP = 5,
    LG_ERR_OOM = 6,
    LG_ERR_UNSUPPORTED = 7
} lg_status;

typedef enum { LG_FP64 = 0, LG_MIXED = 1 } lg_precision;
typedef enum { LG_ACOUSTIC = 0, LG_ELASTIC = 1 } lg_kind;
typedef enum { LG_RICKER = 0, LG_GAUSS_SINE = 1 } lg_wavelet;

/* Boundary at z = 0 (the top).  LG_TOP_DIRICHLET: zero values on the top
 * node row, like the other three sides.  LG_TOP_FREE: the free surface
 * du/dz = 0 at z = 0 of Sec. 2.1 (eq. boundary_cond), in the form of the
 * paper's staggered mesh (Sec. 2.3), where the first unknown lies half a cell
 * below the surface: no flux crosses the face above the first unknown row
 * (acoustic plans).  The preconditioner keeps the same face.  Elastic plans
 * (Cartesian, second order): the traction-free surface tau_xz = sigma_zz = 0
 * of Sec. 2.2 (eq. boundary_elastic) on the first unknown row (node row 1):
 * the operator's surface row is the gradient of the discrete strain energy
 * with a half control strip there (no face above it, a one-sided
 * z-difference in the mixed terms) divided by that half weight, and the
 * block preconditioner's z-systems get the surface row
 * 2 kz (s_0 - s_1)/dz^2 + ... (solved as the Dirichlet Dichotomy result plus
 * a rank-one term).  A source on the surface row acts on half a control
 * cell (twice delta_h). */
typedef enum { LG_TOP_DIRICHLET = 0, LG_TOP_FREE = 1 } lg_top_bc;

/* Geometry.  LG_CARTESIAN: the 2D Cartesian problem, Dirichlet sides (top:
 * lg_top_bc); fields [nz-1][nx-1].  LG_CYLINDRICAL: the paper's 2.5D
 * axisymmetric acoustic problem (Sec. 2.1, 2.3, eqs. poisson_diff_2,
 * scheme_op_r_z, diff_approx1, precond1) on its mesh r_i = (i-1/2) dz, i =
 * 1..nz, z_k = (k-1/2) dx, k = 1..nx: the unknowns are i = 1..nz-1 (y = 0 on
 * the side r = l1, row i = nz), with the symmetry condition at r = 0 and no
 * flux through the two z-ends; fields [nz-1][nx] (z fastest), medium node
 * arrays [F][nz][nx]; acoustic plans, FP64 or mixed (top_bc is not used).
 * The r-systems vary with r (non-Toeplitz); with tuning.segments = P > 1 they
 * are solved by the Dichotomy with factors of every segment prepared once
 * per plan, with P = 1 by Thomas (default: segments of 64 rows from 128 rows
 * on, Thomas below).  The source term carries 1/(2 pi dx dz) (the 2.5D
 * point source). */
typedef enum { LG_CARTESIAN = 0, LG_CYLINDRICAL = 1 } lg_geometry;

/* Spatial order of the acoustic operator (Sec. 3.2: higher-order schemes are
 * preconditioned by the same second-order B).  2 (or 0): the five-point
 * operator above.  4: A4 = Dx^T Kx Dx + Dz^T Kz Dz + w with the fourth-order
 * staggered difference (D u)_{m+1/2} = [27 (u_{m+1} - u_m) - (u_{m+2} -
 * u_{m-1})] / (24 h), the Dirichlet sides taken by odd reflection (u_{-1} =
 * -u_1, u_{N+1} = -u_{N-1}, folded into D so that A4 stays symmetric), and
 * face coefficients from the fourth-order interpolant of the node values
 * (one-sided cubic at the end faces; the two-point mean where the interpolant
 * falls under half the smaller of the face's two nodes).  A 13-point operator
 * (radius 3 along each axis).  Cartesian acoustic plans with Dirichlet sides
 * only; the CG update reads a stored q = A p (op_fusion is taken as 2) and a
 * solve starts from x0 = 0. */
/* Grid: nx, nz cells (powers of two, 2..4096), spacings dx, dz > 0 (metres),
 * top boundary (lg_top_bc), geometry (lg_geometry), operator order (2 or 4;
 * 0 means 2); reserved must be 0. */
typedef struct {
    int32_t nx, nz;
    double dx, dz;
    int32_t top_bc;
    int32_t geometry;
    int32_t order;
    int32_t reserved;
} lg_grid;

/* Laguerre transform (Sec. 2.1): order alpha >= 2, scale h > 0 (1/s), n >= 1
 * harmonics. */
typedef struct { int32_t alpha; double h; int32_t n; } lg_laguerre;

/* Krylov options: stop when ||r||_2 <= tol ||b||_2 (tol >= 0); max_iter >= 1
 * (CG iterations, or GMRES inner iterations); restart = GMRES k, 1 <= k <= 32
 * (a larger k is LG_ERR_UNSUPPORTED).
 * x0_given (PCG only): 0 = start from x0 = 0; 1 = x holds the initial guess
 * on entry (the previous harmonic, say). */
typedef struct { double tol; int32_t max_iter; int32_t restart; int32_t x0_given; int32_t reserved; } lg_solve_opts;

/* Per-shot solver report. */
typedef struct { int32_t iters; int32_t status; double relres; } lg_solve_info;

/* Optional tuning (zero fields = library default).
 *  segments      number P of Dichotomy segments per z-system (axisymmetric
 *                plans: per r-system) (power of two, 1..64, with nz/P in
 *                {2,4,...,64}; axisymmetric plans also take P = 1 at any nz).
 *  graph_iters   Krylov iterations captured per HIP graph (0: default 8,
 *                -1: no graph, plain stream launches).
 *  op_shots      shots per block of the operator kernel, which reuses the
 *                medium held in registers across them (1..64; default 8).
 *  seg_per_wave  Dichotomy segments solved by one wave (1, 2 or 4; default:
 *                chosen from the grid size).
 *  op_fusion     where the update x += alpha p, r -= alpha A p takes A p from
 *                (acoustic CG): 1 = recomputed inside the update kernel
 *                from p and the medium, so the operator kernel only forms
 *                (p, A p); 2 = stored by the operator kernel and read back.
 *                Both give bitwise the same iterates.  0 = default: 1, except
 *                2 for FP64 axisymmetric plans (faster there) and for the
 *                fourth-order operator (which has only the stored form).
 *  x_ring        search directions held before they are added into x
 *                (acoustic CG, every geometry and order): iteration k keeps
 *                p_k and alpha_k, and x += alpha_j p_j is applied in order,
 *                in FP64, by one pass at the end of each CG phase (or before
 *                a held direction would be overwritten), so the update does
 *                not read and write x in every iteration; the iterates are
 *                bitwise those of the in-place update.  1 = x updated in
 *                every iteration (the only form of the other plans); else
 *                more than graph_iters (8 without a graph) and at most 64
 *                directions (memory: x_ring copies of p); 0 = default:
 *                max(16, graph_iters + 1) (32 for axisymmetric plans),
 *                halved (not below graph_iters + 1) while the copies would
 *                pass 64 GiB, 1 if they still do.
 *  reserved      must be 0. */
typedef struct {
    int32_t segments;
    int32_t graph_iters;
    int32_t op_shots;
    int32_t seg_per_wave;
    int32_t op_fusion;
    int32_t x_ring;
    int32_t reserved[2];
} lg_tuning;

typedef struct lg_plan lg_plan;

/* ---------------------------------------------------------------------------
 * Plan (setup, not on the hot path)
 * ------------------------------------------------------------------------ */

/* Create a plan for S = nshots shots over one medium.
 * medium_host: FP64 host array of node values, shape [F][nz+1][nx+1]:
 *   acoustic F = 2: kappa, rho of  rho u_tt = div(kappa grad u) + f  (eq.
 *            acoustic_problem); the operator A has face coefficients the mean
 *            of the two node kappas and the shift w = rho h^2/4 (eq.
 *            diff_approx1);
 *   elastic  F = 3: lambda, mu, rho (Lame parameters and density).
 * The preconditioner uses the midrange values (min+max)/2 of these arrays
 * (footnote to eq. precond1).  hip_stream may be NULL (null stream).
 * tuning may be NULL.  On success *out owns device tables and workspace.
 * Returns LG_ERR_UNSUPPORTED, before any device call, when nshots times the
 * components (1 acoustic, 2 elastic) times the interior points reaches 2^32
 * (element-wise kernels launch one work-item per vector element). */
lg_status lg_plan_create(lg_plan** out, lg_kind kind, const lg_grid* grid,
                         const lg_laguerre* lag, lg_precision prec, int32_t nshots,
                         const double* medium_host, const lg_tuning* tuning,
                         void* hip_stream);
lg_status lg_plan_destroy(lg_plan* plan);
lg_status lg_plan_set_stream(lg_plan* plan, void* hip_stream);

/* Source nodes, one (i, j) pair per shot, 1 <= i <= nx-1, 1 <= j <= nz-1. */
lg_status lg_plan_set_sources(lg_plan* plan, const int32_t* src_ij_host /*[S][2]*/);

/* Segments P and segment length nz/P actually used by the plan. */
lg_status lg_plan_layout(const lg_plan* plan, int32_t* segments, int32_t* seg_len);

/* Search directions the plan's CG holds before adding them into x (lg_tuning
 * x_ring as resolved at plan creation; 1 = x updated in every iteration). */
lg_status lg_plan_x_ring(const lg_plan* plan, int32_t* x_ring);

/* ---------------------------------------------------------------------------
 * Host helpers for the Laguerre transform (Sec. 2.1, eq. series_lag)
 * ------------------------------------------------------------------------ */

/* f_m = int_0^inf f(t) (ht)^{-alpha/2} l_m(ht) dt for m < n, where l_m are the
 * orthonormal Laguerre functions; RICKER: f = (1-2a) e^{-a}, a = (pi f0 (t-t0))^2;
 * GAUSS_SINE (eq. functiont): exp(-(2 pi f0 (t-t0))^2/gamma^2) sin(2 pi f0 (t-t0)).
 * Composite Gauss-Legendre quadrature.  f_m_host: [n]. */
lg_status lg_source_coeffs(lg_wavelet wavelet, double f0, double t0, double gamma,
                           const lg_laguerre* lag, double* f_m_host);

/* Synthesis weights W[q][m] with u(t_q) = sum_m W[q][m] R_m, i.e.
 * W_m(t) = (ht)^{alpha/2} l_m(ht) (eq. series_lag).  W_host: [nt][n]. */
lg_status lg_laguerre_weights(const lg_laguerre* lag, const double* t_host, int32_t nt,
                              double* W_host);

const char* lg_status_string(lg_status s);
const char* lg_last_error(void);

/* ---------------------------------------------------------------------------
 * The hot path
 * ------------------------------------------------------------------------ */

/* Right-hand side of harmonic m (eq. laguerre_h, SPD sign convention):
 *   rhs = delta_h f_m e_src - h^2 rho * n_m sum_{k<m} (m-k) R_k / n_k,
 * n_m = sqrt(m!/(m+alpha)!), delta_h = 1/(dx dz) at the shot's source node (the
 * z component for elastic plans: a vertical force).  The history sum is kept
 * in two caller-owned running fields Phat, Qhat (FP64 vectors) updated in
 * place: P_{m-1} = sqrt((m-1)/(m-1+alpha)) P_{m-2} + R_{m-1},
 * Q_m = sqrt(m/(m+alpha)) (Q_{m-1} + P_{m-1}); the call with m = 0 zeroes them.
 * Calls must be made for m = 0, 1, 2, ... in order.  R_prev = R_{m-1} (FP64
 * vector; ignored, may be NULL, when m = 0).  fsrc_host: [S] values f_m.
 * rhs: FP64 vector (output). */
lg_status lg_laguerre_rhs(lg_plan* plan, int32_t m, const double* R_prev, double* Phat,
                          double* Qhat, const double* fsrc_host, double* rhs);

/* y = A x (acoustic, 5-point flux form of eq. poisson_diff_2 with the sign
 * flipped so A is SPD) or y = C x (elastic, coupled 9-point second-order
 * scheme) for every shot.  x, y: working-type vectors, x != y. */
lg_status lg_stencil_apply(lg_plan* plan, const void* x, void* y);

/* Row-wise DST-I along x of every field row (Sec. 2.4, variable separation):
 *   forward:  out_k = sum_{i=1}^{nx-1} in_i sin(pi i k / nx),   k = 1..nx-1
 *   inverse:  the same sum times 2/nx (exact inverse).
 * in, out: working-type vectors (all shots and components), in != out. */
lg_status lg_precond_dst(lg_plan* plan, int32_t inverse, const void* in, void* out);

/* For every wavenumber k (column of the transformed field) solve the
 * z-tridiagonal system of the preconditioner block
 *   -(kz/dz^2) s_{j-1} + (2 kz/dz^2 + kx mu_k + d) s_j - (kz/dz^2) s_{j+1} = rhs_j,
 *   mu_k = (4/dx^2) sin^2(pi k/(2 nx)),  s_0 = s_nz = 0,
 * by the segmented Dichotomy solver (Thomas factors prepared once per plan).
 * block 0: acoustic B (kx = kz = kappa~, d = rho~ h^2/4; eq. precond1);
 * block 1: elastic B1 (kx = (lambda+2mu)~, kz = mu~) for the x component;
 * block 2: elastic B2 (kx = mu~, kz = (lambda+2mu)~) for the z component.
 * For acoustic plans rhs/sol are full vectors; for elastic plans they are
 * vectors of ONE component per shot ([S][nz-1][nx-1]).  rhs != sol. */
lg_status lg_precond_dichotomy_tdma(lg_plan* plan, int32_t block, const void* rhs_hat,
                                    void* sol_hat);

/* Composite preconditioner inverse z = B^{-1} r (forward DST, Dichotomy
 * solve, inverse DST) for every shot (and both blocks of elastic plans). */
lg_status lg_precond_apply(lg_plan* plan, const void* r, void* z);

/* Preconditioned CG (Sec. 2.3) for A x = b, every shot independently, from
 * x0 = 0 (or from x on entry when opts->x0_given: r0 = b - A x0 in FP64, and
 * 0 iterations when it already meets the tolerance), stopping per shot when
 * ||r||_2 <= tol ||b||_2 on the recursively updated residual.  Mixed plans
 * stop that first phase at max(tol, 1e-7) (below it the FP32 recursion no
 * longer tracks the true residual), then check the FP64 true residual
 * b - A x and restart CG from it where it misses tol (at most 4 restarts,
 * each phase run to tol/2 on its recursive residual so the next check passes
 * with margin; a shot still missing tol after the last one reports
 * LG_ERR_NOT_CONVERGED with relres of its true residual); tol = 0 runs
 * max_iter iterations.  iters counts every CG iteration of the solve.  A zero b gives
 * x = 0, iters = 0.  Converged shots drop out by masking.  b, x: FP64
 * vectors, b != x (b is read until the solve returns).  info_host: [S] (may
 * be NULL).  Returns the worst per-shot status. */
lg_status lg_pcg_solve(lg_plan* plan, const double* b, double* x, const lg_solve_opts* opts,
                       lg_solve_info* info_host);

/* Right-preconditioned restarted GMRES(k) (Sec. 2.3) for the elastic C x = b,
 * K = diag(B1, B2) (eq. precond2), from x0 = 0 (x0_given must be 0); stops when the Givens
 * estimate of ||b - Cx|| <= tol ||b||.  b, x: FP64 vectors ([S][2][..]).  The
 * Arnoldi basis is orthogonalised by classical Gram-Schmidt twice, each
 * vector's second pass taken in the next Arnoldi step. */
lg_status lg_gmres_solve(lg_plan* plan, const double* b, double* x, const lg_solve_opts* opts,
                         lg_solve_info* info_host);

/* Inverse-transform accumulation for harmonic m (eq. series_lag):
 *   snap_accum[s] += W_snap_host[s] * R_m    for s < n_snap (<= 8),
 *   rec_coeff[shot][c][m][:] = R_m[shot][c][row rec_row][:]  (1 <= rec_row <= nz-1),
 * R_m: FP64 vector; snap_accum: FP64 [n_snap][S][C][nz-1][nx-1] (may be NULL
 * when n_snap = 0); rec_coeff: FP64 [S][C][n][nx-1] (may be NULL). */
lg_status lg_laguerre_synthesize(lg_plan* plan, int32_t m, const double* R_m,
                                 const double* W_snap_host, int32_t n_snap, double* snap_accum,
                                 int32_t rec_row, double* rec_coeff);

/* Largest number of harmonics lg_laguerre_synthesize_batch takes per call. */
#define LG_SYNTH_BATCH_MAX 8

/* lg_laguerre_synthesize for the nb consecutive harmonics m0 .. m0+nb-1 in
 * one pass over the accumulators (eq. series_lag):
 *   snap_accum[s] += W[s][0] R_{m0} + ... + W[s][nb-1] R_{m0+nb-1},
 * the terms added one harmonic at a time in that order, so the result is
 * bitwise that of nb calls of lg_laguerre_synthesize; each harmonic's
 * receiver row is stored as there.  The snapshots are read and written once
 * instead of nb times.  R_host: host array of nb FP64 device vectors
 * (R_host[b] = R_{m0+b}); W_snap_host: [n_snap][nb] (host).  1 <= nb <=
 * LG_SYNTH_BATCH_MAX, 0 <= m0, m0 + nb <= n; other arguments as
 * lg_laguerre_synthesize. */
lg_status lg_laguerre_synthesize_batch(lg_plan* plan, int32_t m0, int32_t nb, const double* const* R_host,
                                       const double* W_snap_host, int32_t n_snap, double* snap_accum,
                                       int32_t rec_row, double* rec_coeff);

/* Receiver traces from the stored coefficients:
 *   traces[shot][c][q][i] = sum_m W_host[q][m] rec_coeff[shot][c][m][i].
 * W_host: [nt][n] (host); rec_coeff: FP64 [S][C][n][nx-1]; traces: FP64
 * [S][C][nt][nx-1] (device). */
lg_status lg_trace_synthesize(lg_plan* plan, const double* rec_coeff, const double* W_host,
                              int32_t nt, double* traces);

/* Largest nt * n accepted by lg_trace_synthesize_noalloc (2^21 doubles, 16 MiB). */
#define LG_TRACE_SCRATCH_MAX (1 << 21)

/* lg_trace_synthesize for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same traces, bit for bit, with the [nt][n] weight table
 * staged in a static device array of LG_TRACE_SCRATCH_MAX doubles that the
 * library holds on each GPU until the process ends, instead of a per-call
 * allocation.  Arguments as lg_trace_synthesize.  Calls no hipMalloc or
 * hipFree.  nt * n > LG_TRACE_SCRATCH_MAX returns LG_ERR_UNSUPPORTED with the
 * traces untouched.  Every call on one GPU shares the staging array: calls
 * that overlap on one GPU (other host threads, other plans) race and must be
 * serialised by the caller.  Synchronises the plan stream before returning. */
lg_status lg_trace_synthesize_noalloc(lg_plan* plan, const double* rec_coeff, const double* W_host,
                                      int32_t nt, double* traces);

/* Measurement helper (not part of the method): starts CG on b with tol = 0
 * (so no shot converges) and runs iters + 1 (iters in 1..1000) eager
 * iterations, the last `iters` with HIP events on the plan stream around each
 * of the five kernels (the first update after the start reads b for r and no
 * x, so it is not timed).  ms_host[0..4] receives the average duration in
 * milliseconds of
 *   0 operator q = A p (+ (p,q), alpha),
 *   1 x/r update + forward DST of r (+ ||r||^2, convergence test),
 *   2 Dichotomy segment solves,
 *   3 interface systems (+ (r,z), beta),
 *   4 segment correction + inverse DST + p update.
 * Axisymmetric plans (LG_CYLINDRICAL) report 0 operator, 1 update + forward
 * cosine transform, 2 the r-systems (+ (r,z), beta), 3 zero (no interface
 * stage), 4 inverse cosine transform + p update.
 * With held search directions the flush pass (x += alpha_j p_j) runs between
 * timed iterations where the ring is full and at the end, outside the timed
 * intervals.  x is overwritten with the iterate after iters + 1 iterations.  Acoustic
 * plans only. */
lg_status lg_pcg_profile(lg_plan* plan, const double* b, double* x, int32_t iters, float* ms_host);

#ifdef __cplusplus
}
#endif

#endif /* LAGUERRE_H */
