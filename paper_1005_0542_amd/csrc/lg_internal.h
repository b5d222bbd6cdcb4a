// Internal declarations of the gfx950 Laguerre-harmonic solver library.
// Not part of the public ABI (see include/laguerre.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "laguerre.h"

namespace lg {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
lg_status fail(lg_status s, const std::string& msg);
lg_status hip_fail(hipError_t e, const char* what);

#define LG_HIP(call)                                                    \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::lg::hip_fail(_e, #call);         \
    } while (0)

// ---------------------------------------------------------------------------
// per-shot Krylov control block, resident in device memory
// ---------------------------------------------------------------------------
struct ShotCtl {
    double rz;        // (r, z) of the current iterate
    double pq;        // (p, A p)
    double alpha;     // CG step
    double beta;      // CG direction update
    double rr;        // ||r||^2
    double bb;        // ||b||^2
    double tol2;      // stopping threshold of the recursive ||r||^2 in the current phase
    double tol2f;     // tol^2 ||b||^2: the requested tolerance (FP64 true-residual check)
    double tol2r;     // stopping threshold of the recursive ||r||^2 in a restart phase
    int32_t iters;    // completed iterations
    int32_t active;   // 1 while the shot still iterates
    int32_t status;   // lg_status of the shot
    int32_t max_iter;
    int32_t fresh;    // 1 from a cold start until the first update: x = 0 and r = b
                      // are implied, not stored (the update reads b, takes x as 0)
    int32_t xzero;    // held-direction plans: 1 while x is implied 0 (cold start, no flush yet)
};

// ---------------------------------------------------------------------------
// preconditioner block: z-tridiagonal systems per wavenumber
// ---------------------------------------------------------------------------
struct PrecBlock {
    double kx = 0, kz = 0, d = 0;  // -kx Dxx - kz Dzz + d
    double b = 0;                  // kz / dz^2 (off-diagonal magnitude)
    int Ls = 0;                    // segment length (interior rows Ls-1 + 1 separator)
    int P = 0;                     // number of segments (power of two)
    int q = 0;                     // log2 P
    int RW = 0;                    // row width of the reduced-system table
    void* etab = nullptr;          // [Ls][nx-1] working type: Thomas factors e_i (row i)
    void* utab = nullptr;          // [Ls][nx-1] working type: end response u_i (row i)
    double* red = nullptr;         // [nx-1][RW]: Ar, Br, beta_l (q), half weights
};

struct lg_plan_impl;

}  // namespace lg

// ---------------------------------------------------------------------------
// the opaque plan
// ---------------------------------------------------------------------------
struct lg_plan {
    lg_kind kind;
    lg_grid g;
    lg_laguerre lag;
    lg_precision prec;
    int S = 1;                 // shots
    int C = 1;                 // components
    int nx1 = 0, nz1 = 0;      // interior extents
    size_t npts = 0;           // nx1 * nz1
    size_t nvec = 0;           // S * C * npts
    int graph_iters = 8;
    int op_shots = 8;          // operator kernel: shots per block
    int td_spw = 0;            // Dichotomy segments per wave (0: automatic)
    bool fuse_op = true;       // CG update recomputes A p (no stored q)
    // Free surface (top face flux-free): the z-systems become T - e1 e1^T,
    // solved as the Dirichlet Dichotomy result plus a rank-one
    // (Sherman-Morrison) term coef_k g_k with g_k = T_k^{-1} e1.
    bool free_top = false;
    void* sm_g = nullptr;      // [nz-1][nx-1] working type: g_k(j)
    double* sm_t = nullptr;    // [2][nx-1]: 1 / (1 - g_k(0)), u_{Ls-1}(k)
    double* sm_c = nullptr;    // [fields][nx-1]: coef_k of the current solve
    // Elastic traction-free surface on the first unknown row: the operator's
    // surface row comes from the discrete strain energy (half control strip),
    // and each block's z-systems have the surface row 2 kz (s_0 - s_1)/dz^2,
    // i.e. T - b e1 e2^T, solved as the Dirichlet result plus the rank-one
    // term g_k s_1 / (1 - g_k(1)) with g_k = T_k^{-1} e1 (normalised).
    bool el_free = false;
    void* es_g[2] = {nullptr, nullptr};     // per block: [nz-1][nx-1] working type, g_k(j)
    double* es_t[2] = {nullptr, nullptr};   // per block: [nx-1], 1 / (1 - g_k(1))
    // 2.5D axisymmetric plans (geometry LG_CYLINDRICAL): fields are
    // [Nr-1][Nz] with z fastest (nx1 = Nz, nz1 = Nr - 1); cosine transform
    // along z, non-Toeplitz r-systems solved by Thomas per wavenumber.
    bool cyl = false;
    void* cy_a1 = nullptr;     // [nz1][nx1] working type: a1 / h_r^2 on the face below row j
    void* cy_a2 = nullptr;     // [nz1][nx1+1]: a2 / h_z^2 on the face left of column k (0 at both ends)
    void* cy_ctw = nullptr;    // [nx1] complex working type: exp(-i pi k / (2 Nz))
    // r-systems by the Dichotomy (blk[0].P segments of blk[0].Ls - 1 rows and
    // P - 1 separator rows c_s = s Ls + Ls - 1): per wavenumber k and row j
    void* cy_cp = nullptr;     // [nz1][nx1]: segment-local Thomas upper factors
    void* cy_invden = nullptr; // [nz1][nx1]: segment-local inverse pivots
    void* cy_UV = nullptr;     // [nz1][nx1] pairs (U, V): responses to the left / right separator
                               // value 1 (0 on separator rows); allocated for more than one segment
    void* cy_lowr = nullptr;   // [nz1]: coupling of row j to row j-1 (0 for the first)
    double* cy_cpl64 = nullptr;   // [2][nz1] FP64: couplings to rows j-1 and j+1
    double* cy_red = nullptr;     // [nx1][P-1][3] FP64: reduced system (sub-diagonal, upper factor, inverse pivot)
    double* cy_a1_64 = nullptr;   // mixed plans: FP64 copies of cy_a1, cy_a2 (true residual)
    double* cy_a2_64 = nullptr;
    double src_scale = 0.0;    // discrete delta: 1/(dx dz), or 1/(2 pi h_r h_z)
    // Fourth-order operator (order 4): face tables with the 1/(576 h^2)
    // scale folded in; the x-faces m+1/2 (m = 0..nx-1) of the interior rows
    // and the z-faces n+1/2 (n = 0..nz-1) of the interior columns.
    int order = 2;
    void* ho_kx = nullptr;     // [nz-1][nx] working type
    void* ho_kz = nullptr;     // [nz][nx-1] working type
    double* ho_kx64 = nullptr; // mixed plans: FP64 copies (true residual)
    double* ho_kz64 = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only for graph capture

    // medium (device)
    void* kap = nullptr;       // acoustic kappa nodes [(nz+1)(nx+1)], working type
    void* lam = nullptr;       // elastic lambda nodes, working type
    void* mu = nullptr;        // elastic mu nodes, working type
    void* w = nullptr;         // interior rho h^2/4, working type
    double* kap64 = nullptr;   // FP64 copies for the true residual of mixed plans
    double* w64 = nullptr;
    double* rho64 = nullptr;   // interior rho, FP64 (right-hand side recurrence)
    double kappa_t = 0, rho_t = 0, lp2m_t = 0, mu_t = 0;   // midrange values

    lg::PrecBlock blk[2];      // acoustic uses blk[0]; elastic blk[0]=B1, blk[1]=B2
    void* tw = nullptr;        // FFT twiddles exp(-2 pi i j / (2 nx)), complex working type

    // sources
    int32_t* src_dev = nullptr;         // [S][2]
    std::vector<int32_t> src_host;

    // Krylov workspace
    double* r = nullptr;       // FP64 residual
    void* p = nullptr;         // working type: pring slots of nvec values
    // Held search directions (acoustic PCG): iteration
    // k reads p_k from slot k % pring and keeps alpha_k; x += alpha_j p_j is
    // applied in order by a flush pass (phase ends, or before a slot would be
    // reused) instead of in every update.  pring = 1: x updated in place.
    int pring = 1;
    double* ahist = nullptr;   // [S*C][pring] alpha_j of the held directions (0 where the shot was masked)
    int* giter = nullptr;      // [0] CG iterations of the solve so far (one count for all shots: the
                               // slot index), [1] iterations already added into x
    void* qv = nullptr;        // A p
    void* rhat = nullptr;      // DST(r)
    void* y = nullptr;         // Dichotomy output / spectral solution
    double* E = nullptr;       // per-segment endpoint data [S*C][P][3][nx-1]
    double* partial = nullptr; // per-block partial sums
    double* partial_pq = nullptr;  // the operator's (p, A p) partials where the update sums them itself
    size_t partial_stride = 0; // per shot
    lg::ShotCtl* ctl = nullptr;    // [S*C]
    lg::ShotCtl* ctl_host = nullptr;  // pinned mirror
    double** xslot = nullptr;  // device slots holding the caller's x and b pointers

    // HIP graph of graph_iters CG iterations
    hipGraphExec_t cg_graph = nullptr;
    int last_iters = 0;        // the previous solve: most CG iterations of a shot before the first
    int last_iters_restart = 0;  // stop, and after the first restart (mixed plans)

    // elastic GMRES workspace
    double* gm_V = nullptr;    // (k+1) basis vectors, FP64
    double* gm_w = nullptr;
    double* gm_z = nullptr;
    double* gm_x = nullptr;
    double* gm_dots = nullptr;
    double* gm_hb = nullptr;   // pinned host: the inner iterations' inner products, two sets
    hipEvent_t gm_ev[2] = {nullptr, nullptr};
    int gm_k = 0;

    size_t bytes_allocated = 0;
};

namespace lg {

// element size of the working type
inline size_t wsize(const lg_plan* p) { return p->prec == LG_FP64 ? 8 : 4; }
// blocks per field of the row-transform kernels (one or more row pairs each)
int dst_blocks_per_field(int nx, int nz1, int ws);

// The row DST-I of nx-cell rows runs as one complex FFT of length nx per row
// pair (with a pre- and post-pass) where the 2 nx-point odd extension would
// take more than 32 KB of LDS per row pair, else as the 2 nx-point transform.
constexpr bool dst_half_form(int nx, int ws) { return 2 * nx * 2 * ws > 32768; }

// launchers (implemented in lg_acoustic.hip); all enqueue on plan->stream
hipError_t launch_stencil(lg_plan* p, const void* x, void* y, bool reduce_pq);
hipError_t launch_dst(lg_plan* p, int inverse, const void* in, void* out, int nfields);
// Dichotomy kernels over `nfields` fields; field f of the launch is buffer
// field f * fstride + foff (acoustic: 1, 0; one elastic component: 2, c).
hipError_t launch_td(lg_plan* p, int blk, const void* rhat, void* y, int nfields, int masked,
                     int fstride = 1, int foff = 0);
hipError_t launch_rs(lg_plan* p, int blk, const void* rhat, void* y, int nfields, int mode,
                     int fstride = 1, int foff = 0);
hipError_t launch_correct(lg_plan* p, int blk, void* y, int nfields, int fstride = 1, int foff = 0);
// CG update + forward DST.  init 0: iteration (x += alpha p, r -= alpha A p);
// 1: start (x = 0, r = b); 2: restart from the stored r; 3 (mixed): restart
// from the FP64 true residual r = b - A x formed in the same pass.
hipError_t launch_update_fdst(lg_plan* p, int init, const double* b, double* x, double tol,
                              int max_iter);
hipError_t launch_correct_idst(lg_plan* p, int init);
hipError_t launch_correct_inv(lg_plan* p, void* z, int nfields, bool surface);
hipError_t launch_surface_coef_fused(lg_plan* p, const void* y, int nfields);
// Held-direction plans: x += alpha_j p_j for the iterations j = giter[1] ..
// giter[0]-1, in order, skipping those where the shot was masked (alpha_j =
// 0; x taken as 0 while xzero), then giter[1] = giter[0], xzero = 0.  No-op
// for pring = 1.
hipError_t launch_flush_x(lg_plan* p, double* x);
// FP64 ||b - A x||^2 per shot and the finalize kernel's restart check: shots
// that had met the tolerance on the recursive residual stop if the true one
// meets it too, else resume (active); the axisymmetric and fourth-order
// variants also store r = b - A x for the restart
hipError_t launch_residual_check(lg_plan* p, const double* b, const double* x);
// finalize kernel over nparts per-block partials per shot: kind 0 (p, Ap)
// -> alpha; 1 ||r||^2 -> convergence; 2 (r, z) * scale -> beta
// (init 1, 4 of kind 1 also take tol2f, the squared requested tolerance, and
// tol2r, the squared recursive tolerance of restart phases; both default to tol2)
hipError_t launch_finalize(lg_plan* p, int kind, int nparts, int init, double tol2, int max_iter, double scale,
                           double tol2f = -1.0, double tol2r = -1.0);
// Recursive-residual tolerance at which a CG phase stops.  Mixed plans run
// iterative refinement: the first phase (start) stops at max(tol,
// LG_MIXED_PHASE1_TOL), about where the FP32 recursion stops tracking the true
// residual; each restart from the FP64 true residual then aims at
// LG_MIXED_REFINE_FAC * tol, so that the true residual checked against tol
// afterwards lands below it with margin.  FP64 plans use tol.
// tol = 0 (a fixed iteration count) stays 0.
double phase_tol(const lg_plan* p, double tol, bool restart);
constexpr double LG_MIXED_PHASE1_TOL = 1e-7;
constexpr double LG_MIXED_REFINE_FAC = 0.5;
// 2.5D axisymmetric plans
hipError_t cyl_launch_stencil(lg_plan* p, const void* x, void* y, bool reduce);
// corr (inverse only): apply the r-system Dichotomy correction to the input rows
hipError_t cyl_launch_dct(lg_plan* p, int inverse, const void* in, void* out, int nfields, int corr = 0);
// r-systems: segments + reduced systems (mode 0 plain, 1 CG start, 2 CG
// iteration with the (r, z) finalize); the correction follows separately
hipError_t cyl_launch_rsys(lg_plan* p, const void* rhat, void* y, int nfields, int mode);
hipError_t cyl_launch_corr(lg_plan* p, void* z, int nfields);
// init 0 iteration, 1 start (x = 0, r = b), 2 restart from the stored r
hipError_t cyl_launch_update(lg_plan* p, int init, const double* b, double* x, double tol, int max_iter);
// FP64 true residual r = b - A x, stored, ||r||^2 and the restart check
hipError_t cyl_launch_residual_check(lg_plan* p, const double* b, const double* x);
// the update pass with init 2 from the r stored by the check
hipError_t cyl_launch_restart(lg_plan* p, const double* b, double* x, double tol, int max_iter);
hipError_t cyl_launch_correct(lg_plan* p, int init);
// fourth-order operator (lg_ho.hip)
hipError_t ho_launch_stencil(lg_plan* p, const void* x, void* y, bool reduce);
// p->r = b - A4 x (FP64), ||r||^2 per shot and the restart check
hipError_t ho_launch_residual(lg_plan* p, const double* b, const double* x);
hipError_t launch_rhs(lg_plan* p, int m, const double* Rprev, double* Ph, double* Qh,
                      const double* fsrc_host, double* rhs);
// synthesis of harmonics m0 .. m0+nb-1 (nb <= 8) in one pass: R[b] their
// solutions, Wsnap [nsnap][nb] (host)
hipError_t launch_synth(lg_plan* p, int m0, int nb, const double* const* R, const double* Wsnap, int nsnap,
                        double* snap, int rec_row, double* rec);
hipError_t launch_traces(lg_plan* p, const double* rec, const double* Wdev, int nt,
                         double* traces);

// PCG driver (lg_pcg.hip)
lg_status pcg_solve(lg_plan* p, const double* b, double* x, const lg_solve_opts* o,
                    lg_solve_info* info);
void pcg_release(lg_plan* p);
lg_status pcg_profile(lg_plan* p, const double* b, double* x, int iters, float* ms);

// GMRES driver (lg_elastic.hip)
lg_status gmres_solve(lg_plan* p, const double* b, double* x, const lg_solve_opts* o,
                      lg_solve_info* info);
hipError_t launch_elastic_stencil(lg_plan* p, const void* x, void* y);
hipError_t launch_elastic_precond(lg_plan* p, const void* r, void* z);
// elastic traction-free surface: the rank-one surface-row term on the
// Dirichlet Dichotomy solution of block blk (fields f * fstride + foff)
hipError_t launch_surface_rows(lg_plan* p, int blk, void* y, int nfields, int fstride, int foff);

}  // namespace lg
