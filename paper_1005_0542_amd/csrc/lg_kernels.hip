// gfx950 kernels of the Laguerre-harmonic preconditioned Krylov solve.
//
// Data layout: a field is (nz-1) rows of (nx-1) values, x fastest; fields of
// all shots (and components) are stacked.  Spectral fields (after the DST
// along x) keep the same layout with the wavenumber k in place of x, so the
// z-systems of consecutive wavenumbers sit in consecutive addresses and every
// sweep over z loads one coalesced row segment per step.
//
// Kernels (one pass of the preconditioned CG iteration is K1..K5; each
// reduction is per-block partials, summed in a fixed order by finalize_kernel):
//   K1 stencil_kernel      partials of (p, A p); finalize: alpha
//   K2 dst_kernel UPDATE   A p recomputed, r -= alpha A p (x += alpha p, or the
//                          direction held for the flush pass), ||r||^2,
//                          rhat = DST(r); finalize: convergence test
//   K3 td_kernel           Dichotomy segments: local Thomas solves
//   K4 rs_kernel           interface (reduced) systems by recursive halving
//                          across the lanes of a wave; (r, z); finalize: beta
//   K5 dst_kernel CORRECT  segment correction, z = (2/nx) DST(zhat), p = z + beta p
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lg_device.h"
#include "lg_internal.h"

namespace lg {

// ===========================================================================
// K1: 5-point operator (Sec. 2.3, eqs. poisson_diff_2 / scheme_op_r_z /
// diff_approx1 in 2D Cartesian form, SPD sign):
//   (A p)_{j,i} = [kE (p - pE) + kW (p - pW)] / dx^2 + [kS (p - pS) + kN (p - pN)] / dz^2
//                 + w p,   face kappa = mean of the two node values.
// Each thread marches down ST_RPT rows of one column, keeping the column's
// p and kappa values in registers; x-neighbours come from the L1/L2.
// ===========================================================================
constexpr int ST_RPT = 8;
constexpr int ST_MAXSH = 64;     // fields per block (op_shots) at most

template <typename T>
struct StArgs {
    const T* p;
    T* q;                // nullptr: no store (dot only)
    const double* b;     // residual-norm mode: right-hand side
    const T* kap;        // node kappa, (nz+1) x (nx+1)
    const T* w;          // interior shift
    int nx1, nz1;
    T idx2, idz2;
    int nfields, nsh;    // fields, fields per block (shot chunks)
    int gx, gy;          // column tiles, row strips (1D grid of gx*gy*chunks blocks)
    int free_top;        // free surface: no flux through the face above row 0
    // CG reduction (ctl == nullptr: plain operator application)
    ShotCtl* ctl;
    double* partial;
    size_t pstride;
    int pring;           // > 1 (with ctl): p at slot giter[0] % pring
    size_t pslot;        // elements per slot
    const int* giter;    // held directions: the solve's iteration count
};

// The medium (kappa at the nodes the column touches, w) is loaded once into
// registers and reused for a chunk of `nsh` shots.  For each shot all p loads
// of the strip are buffer loads issued together (out-of-grid neighbours read
// as the Dirichlet zero through the range check), q is written by buffer
// stores (rows past the grid are dropped), and the (p, A p) partial is
// reduced per wave without barriers; one block barrier at the end combines
// the waves of every shot.  RESN (FP64 only): p is x and the partial is
// ||b - A x||^2 over every shot, nothing is stored (the check of the true
// residual that precedes a restart).
template <typename T, bool RESN>
__global__ __launch_bounds__(256) void stencil_kernel(StArgs<T> a) {
    static_assert(!RESN || sizeof(T) == 8, "the residual norm is formed in FP64");
    __shared__ double red[ST_MAXSH][4];
    const int nx1 = a.nx1, nz1 = a.nz1, NXN = nx1 + 2;
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 1D block of 256 = 64 x 4
    // tiles in x-fastest order, contiguous per XCD: the column neighbours of a
    // tile (sharing its boundary cache lines) run next to it in the same L2
    const int L = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = L % a.gx, by = (L / a.gx) % a.gy, bz = L / (a.gx * a.gy);
    // the chunk's active flags first: a block whose shots have all stopped
    // leaves before loading the medium (the masked iterations of a replay)
    const int s0 = bz * a.nsh;
    const int ns = min(a.nsh, a.nfields - s0);
    __shared__ int act[ST_MAXSH];
    int mine = 0;
    if (threadIdx.x < ns) {
        act[threadIdx.x] = (a.ctl != nullptr && !RESN) ? a.ctl[s0 + threadIdx.x].active : 1;
        mine = act[threadIdx.x];
    }
    if (__syncthreads_or(mine != 0) == 0) return;   // (also the barrier for act) uniform per block
    const int i = bx * 64 + lane;
    const int j0 = (by * 4 + ty) * ST_RPT;
    const bool live = i < nx1;
    const int ic = min(i, nx1 - 1);                 // clamped column (dead lanes)
    const int I = ic + 1;
    const T half = (T)0.5;
    // medium of this column strip: node kappa rows j0 .. j0+RPT+1 and the
    // face coefficients / shift of rows j0 .. j0+RPT-1 (clamped indices)
    T kc[ST_RPT + 2], fE[ST_RPT], fW[ST_RPT], wv[ST_RPT];
#pragma unroll
    for (int r = 0; r < ST_RPT + 2; ++r) {
        const int J = min(j0 + r, nz1 + 1);         // node row (interior row j0+r-1)
        kc[r] = a.kap[(size_t)J * NXN + I];
    }
#pragma unroll
    for (int r = 0; r < ST_RPT; ++r) {
        const int j = min(j0 + r, nz1 - 1), J = j + 1;
        fE[r] = half * (kc[r + 1] + a.kap[(size_t)J * NXN + I + 1]);
        fW[r] = half * (kc[r + 1] + a.kap[(size_t)J * NXN + I - 1]);
        wv[r] = a.w[(size_t)j * nx1 + ic];
    }
    // byte offsets within one field: rows j0-1 .. j0+RPT at column i, and the
    // x-neighbours of rows j0 .. j0+RPT-1; outside the grid: BUF_OOB
    constexpr uint32_t SZ = sizeof(T);
    uint32_t oc[ST_RPT + 2], oe[ST_RPT], ow[ST_RPT];
#pragma unroll
    for (int r = 0; r < ST_RPT + 2; ++r) {
        const int j = j0 - 1 + r;
        oc[r] = (live && j >= 0 && j < nz1) ? (uint32_t)(j * nx1 + i) * SZ : BUF_OOB;
    }
#pragma unroll
    for (int r = 0; r < ST_RPT; ++r) {
        const uint32_t c = oc[r + 1];
        oe[r] = (c != BUF_OOB && i + 1 < nx1) ? c + SZ : BUF_OOB;
        ow[r] = (c != BUF_OOB && i > 0) ? c - SZ : BUF_OOB;
    }
    const uint32_t fbytes = (uint32_t)nx1 * (uint32_t)nz1 * SZ;
    // held directions: this iteration's p slot (one count for every shot)
    const size_t ps = (!RESN && a.pring > 1) ? (size_t)(*a.giter % a.pring) * a.pslot : 0;
    for (int k = 0; k < ns; ++k) {
        const int field = s0 + k;
        if (act[k] == 0) continue;              // uniform per block
        const size_t fb = (size_t)field * nx1 * nz1;
        const rsrc_t rp = buf_rsrc(a.p + ps + fb, fbytes);
        T pv[ST_RPT + 2], pe[ST_RPT], pw[ST_RPT];
#pragma unroll
        for (int r = 0; r < ST_RPT + 2; ++r) pv[r] = bload<T>(rp, oc[r]);
#pragma unroll
        for (int r = 0; r < ST_RPT; ++r) {
            pe[r] = bload<T>(rp, oe[r]);
            pw[r] = bload<T>(rp, ow[r]);
        }
        T bv[RESN ? ST_RPT : 1];
        if constexpr (RESN) {
            const rsrc_t rb = buf_rsrc(a.b + fb, fbytes);
#pragma unroll
            for (int r = 0; r < ST_RPT; ++r) bv[r] = bload<double>(rb, oc[r + 1]);
        }
        double pq = 0.0;
        T v[ST_RPT];
#pragma unroll
        for (int r = 0; r < ST_RPT; ++r) {
            const T fS = half * (kc[r + 1] + kc[r + 2]);
            const T fN = (a.free_top && j0 + r == 0) ? (T)0 : half * (kc[r + 1] + kc[r]);
            const T c = pv[r + 1];                  // 0 outside the grid, so no dot term
            v[r] = stencil_point(c, pe[r], pw[r], pv[r + 2], pv[r], fE[r], fW[r], fS, fN, wv[r],
                                 a.idx2, a.idz2);
            if constexpr (RESN) {
                const double rv = (oc[r + 1] != BUF_OOB) ? bv[r] - v[r] : 0.0;   // rows past the grid: none
                pq += rv * rv;
            } else {
                pq += (double)c * (double)v[r];
            }
        }
        if (a.q != nullptr) {
            const rsrc_t rq = buf_rsrc(a.q + fb, fbytes);
#pragma unroll
            for (int r = 0; r < ST_RPT; ++r)
                bstore<T>(v[r], rq, oc[r + 1]);
        }
        if (a.ctl == nullptr) continue;
        pq = wave_sum(pq);
        if (lane == 0) red[k][ty] = pq;
    }
    if (a.ctl == nullptr) return;
    __syncthreads();
    if (threadIdx.x < ns && act[threadIdx.x] != 0) {
        const int k = threadIdx.x;
        const double s = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
        a.partial[(size_t)(s0 + k) * a.pstride + by * a.gx + bx] = s;
    }
}

// ===========================================================================
// K2 / K5 and the plain transform: row-wise DST-I along x (Sec. 2.4,
// variable separation), F_k = sum_{j=1}^{N-1} f_j sin(pi j k / N), N = nx, by
// one complex FFT of length N per pair of rows.  The two rows (j0, j1) of a
// field are packed as the real and imaginary parts of f (f_0 = 0).  A
// pre-pass forms y_j = sin(pi j/N)(f_j + f_{N-j}) + (f_j - f_{N-j})/2
// (y_0 = 0), whose DFT Y (of each real row) gives the even outputs
// F_{2k} = -Im Y_k and the odd ones by a prefix sum, F_{2k+1} =
// F_{2k-1} + Re Y_k with F_1 = Re Y_0 / 2 (the real-odd symmetry that a
// 2N-point transform of the odd extension would carry twice; the method is
// the classical one of Numerical Recipes' sinft).  With Z = DFT(y) of the
// packed rows, row j0 takes Y_k = (Z_k + conj Z_{N-k})/2 and row j1
// Y_k = (Z_k - conj Z_{N-k})/(2i).  The prefix sum runs over the thread's
// own k, then over the transform's threads (wave shuffles, and the waves'
// totals through LDS).
// The other form (HALF = false) odd-extends the packed rows to length
// M = 2N (w_0 = w_N = 0, w_{M-i} = -w_i), whose DFT is V_k = -2i F_k(j0) +
// 2 F_k(j1): no pre- or post-pass, twice the butterflies and the LDS.  The
// N-point form is used where a 2N-point row pair would take more than 32 KB
// of LDS (FP64 from nx = 2048, FP32 from nx = 4096), which otherwise caps the
// blocks per CU; below that the 2N-point form measured faster (fewer passes
// over LDS and barriers in the CG update, the same correction time).
// ===========================================================================
// DST_UPDATE_OP is DST_UPDATE with A p recomputed from p and the medium
// instead of read from a stored q.  DST_RESTART (mixed precision) forms the
// FP64 true residual r = b - A x from x, b and the FP64 medium, stores it and
// transforms it: the restart of CG from the true residual in one pass.
// DST_UPDATE_PQ is DST_UPDATE that also forms (p, A p) and alpha from the
// operator's per-block partials in every block (the finalize kernel's sum,
// in its order), for fields with few such partials: one launch less per
// iteration where launches, not bytes, set the time.
enum DstMode { DST_FWD = 0, DST_INV = 1, DST_UPDATE = 2, DST_CORRECT = 3, DST_UPDATE_OP = 4, DST_RESTART = 5,
               DST_UPDATE_PQ = 6 };

template <typename T>
struct DstArgs {
    const T* in;           // DST_FWD / DST_INV input
    T* out;                // FWD/INV output; UPDATE: rhat; CORRECT: p (in/out)
    const cpx<T>* tw;      // exp(-2 pi i j / M), j < M
    int nz1;               // rows per field
    int bpf;               // blocks per field
    // CG (UPDATE / CORRECT)
    ShotCtl* ctl;
    double* x;             // UPDATE init: caller x (stored into xslot[0], b into xslot[1])
    double** xslot;
    double* r;
    const double* b;       // UPDATE init: right-hand side
    const T* p;            // UPDATE: search direction (slot 0)
    int pring;             // > 1: held directions, p of iteration g at slot g % pring; x not touched
    size_t pslot;          // elements per slot
    const int* giter;      // held directions: [0] the solve's iteration count g
    const T* q;            // UPDATE: A p
    const T* kap;          // UPDATE_OP: node kappa, (nz+1) x (nx+1)
    const T* wsh;          // UPDATE_OP: interior shift
    T idx2, idz2;          // UPDATE_OP: 1/dx^2, 1/dz^2
    const double* kap64;   // RESTART: FP64 node kappa and shift
    const double* w64;
    double idx2d, idz2d;
    int free_top;          // free surface (operator face; CORRECT: rank-one term)
    const T* smg;          // CORRECT (free surface): g_k rows
    const T* smg2;         // non-null: odd fields take these g_k rows (elastic K, second block)
    const double* smc;     // CORRECT (free surface): coef_k per field
    double* partial;
    size_t pstride;
    const double* pqpart;  // UPDATE_PQ: the operator's (p, A p) partials [field][pstride]
    int pq_nparts;         // UPDATE_PQ: their count per field
    double* ahist;         // UPDATE_PQ with held directions: alpha_g at [field][g % pring]
    double tol2;           // tol^2 (init)
    int max_iter;          // (init)
    int init;
    // CORRECT: Dichotomy segment correction
    const T* y;
    const T* utab;
    const T* utab2;        // non-null: odd fields take this second block's table (elastic K)
    int Ls, P;
};

// Each thread of the one block per field loads FIN_UNROLL partials (strided
// by the block size) before adding them, so a pass costs one memory latency.
// The block size follows the partial count (a large block only where there
// are many partials: launching one costs more), so the order of the
// additions depends on the partial count alone.
constexpr int FIN_UNROLL = 8;
constexpr int FIN_SMALL = 256, FIN_LARGE = 1024;
constexpr int FIN_SMALL_MAX = FIN_UNROLL * FIN_SMALL;     // partials one pass of the small block covers

template <int NT>
__device__ __forceinline__ double fin_sum(const double* __restrict__ part, int n, double* red) {
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += FIN_UNROLL * NT) {
        double v[FIN_UNROLL];
#pragma unroll
        for (int u = 0; u < FIN_UNROLL; ++u) {
            const int i = i0 + u * NT;
            v[u] = i < n ? part[i] : 0.0;
        }
#pragma unroll
        for (int w = FIN_UNROLL / 2; w > 0; w /= 2)
#pragma unroll
            for (int u = 0; u < w; ++u) v[u] += v[u + w];
        s += v[0];
    }
    return block_sum(s, red);
}

// A p on the rows j0 and j0 + 1 of a row pair at column i, with the operator
// kernel's face coefficients and stencil_point, so the values are bitwise
// those of the operator kernel.  rP covers the field's p; c0, c1: p at
// (j0, i) and (j0 + 1, i).  ok0 / ok1: the element / its second row exist
// (otherwise every p read is 0 and the result is 0).
template <typename T>
__device__ __forceinline__ void apply_pair(rsrc_t rP, const T* __restrict__ kap, const T* __restrict__ wsh,
                                           int nx1, int nz1, int i, int j0, bool ok0, bool ok1, T c0, T c1,
                                           T idx2, T idz2, bool free_top, T& q0, T& q1) {
    constexpr uint32_t SZ = sizeof(T);
    const int NXN = nx1 + 2, I = i + 1, J0 = j0 + 1;
    const uint32_t e = (uint32_t)(j0 * nx1 + i);
    const T half = (T)0.5;
    const T pN0 = bload<T>(rP, (ok0 && j0 > 0) ? (e - nx1) * SZ : BUF_OOB);
    const T p0E = bload<T>(rP, (ok0 && i + 1 < nx1) ? (e + 1) * SZ : BUF_OOB);
    const T p0W = bload<T>(rP, (ok0 && i > 0) ? (e - 1) * SZ : BUF_OOB);
    const T pS1 = bload<T>(rP, (ok1 && j0 + 2 < nz1) ? (e + 2 * nx1) * SZ : BUF_OOB);
    const T p1E = bload<T>(rP, (ok1 && i + 1 < nx1) ? (e + nx1 + 1) * SZ : BUF_OOB);
    const T p1W = bload<T>(rP, (ok1 && i > 0) ? (e + nx1 - 1) * SZ : BUF_OOB);
    const T* k0 = kap + (size_t)J0 * NXN + I;
    const T k00 = k0[0], k0E = k0[1], k0W = k0[-1], k0N = k0[-NXN];
    const T k10 = k0[NXN];                                    // node row J0 + 1 <= nz1 + 1
    const T* k1 = kap + (size_t)min(J0 + 1, nz1) * NXN + I;   // second row (clamped)
    const T k1E = k1[1], k1W = k1[-1], k1S = k1[NXN];
    const int j1c = min(j0 + 1, nz1 - 1);
    const T fN0 = (free_top && j0 == 0) ? (T)0 : half * (k00 + k0N);   // free surface: no flux above row 0
    q0 = stencil_point(c0, p0E, p0W, c1, pN0, half * (k00 + k0E), half * (k00 + k0W), half * (k00 + k10),
                       fN0, wsh[(size_t)j0 * nx1 + i], idx2, idz2);
    const T v1 = stencil_point(c1, p1E, p1W, pS1, c0, half * (k10 + k1E), half * (k10 + k1W),
                               half * (k10 + k1S), half * (k10 + k00), wsh[(size_t)j1c * nx1 + i], idx2, idz2);
    q1 = ok1 ? v1 : (T)0;
}

// Phase A: each row element x_i (i = t + it TPF) is loaded once by its
// thread, which writes it to LDS at position 1+i.  The pre-pass pairs j with
// N-j in LDS; the Stockham passes run LDS -> LDS, except the last pass,
// which leaves its outputs in registers; they go back to LDS for the
// post-pass (pairs k, N-k and the prefix sum), whose results are stored to
// global memory from LDS in coalesced order (column t + u TPF).
// The update modes get a waves-per-EU bound of 3: the register room keeps
// more of their loads in flight (measured 1.8 % faster at 64 shots 2048^2).
template <typename T, int M, int R, int FPB, int MODE, bool HALF>
__global__ __launch_bounds__(FPB*(M / R)) __attribute__((amdgpu_waves_per_eu(
    1, (MODE == DST_UPDATE || MODE == DST_UPDATE_OP || MODE == DST_RESTART || MODE == DST_UPDATE_PQ) ? 3 : 8))) void
dst_kernel(DstArgs<T> a) {
    using FP = FftPlan<M, R>;
    constexpr int TPF = M / R;
    constexpr int NX = HALF ? M : M / 2;       // nx: the FFT length is nx (HALF) or 2 nx
    constexpr int NX1 = NX - 1;
    constexpr int NH = NX / 2;                 // post-pass: k = 0 .. NH-1
    constexpr int CK = HALF ? NH / TPF : 1;    // consecutive k per thread (R / 2)
    constexpr int RL = FP::R_LAST, NBL = FP::NB_LAST, NSL = FP::NS_LAST;
    constexpr int LL = LdsLen<M>::value;
    constexpr int NWAVE = (FPB * TPF + 63) / 64;
    constexpr int NIT = (NX1 + TPF - 1) / TPF;
    // outputs per thread: columns t + u TPF (HALF), or the first-half spectrum
    // entries K = t + qb M/R + u NS_LAST of the last pass (2N form)
    constexpr int NOUT = HALF ? NIT : NBL * (RL / 2);
    // loads per chunk of phase A (all in flight together): the FP32 correction
    // takes every element of the row pair at once
    constexpr int CHMAX = (MODE == DST_UPDATE_OP && sizeof(T) == 8) ? 2 : (MODE == DST_CORRECT && sizeof(T) == 4) ? 8 : 4;
    constexpr int CH = NIT < CHMAX ? NIT : CHMAX;
    constexpr bool UPD = MODE == DST_UPDATE || MODE == DST_UPDATE_OP || MODE == DST_RESTART || MODE == DST_UPDATE_PQ;
    static_assert(MODE != DST_UPDATE_PQ || FPB * (M / R) == FIN_SMALL, "the finalize kernel's summation order");
    __shared__ cpx<T> lds[FPB * LL];
    __shared__ double red[NWAVE];
    __shared__ cpx<T> wtot[NWAVE];             // per-wave totals of the prefix sum

    const int fid = threadIdx.x / TPF;
    const int t = threadIdx.x - fid * TPF;
    // Field-major order: the blocks in flight at any time cover a few
    // consecutive row pairs of one or two fields, which keeps the pages they
    // touch few (measured faster than orders that spread the blocks in flight
    // over many fields for medium or halo reuse in one L2).
    const int field = blockIdx.x / a.bpf;
    const int bif = blockIdx.x - field * a.bpf;
    const int pair = bif * FPB + fid;
    const int npairs = (a.nz1 + 1) >> 1;
    const bool live = pair < npairs;
    const int j0 = 2 * pair, j1 = j0 + 1;
    const bool has1 = live && (j1 < a.nz1);

    if constexpr (MODE == DST_UPDATE_PQ) {   // held directions: alpha_g stays 0 unless the update runs
        if (a.pring > 1 && bif == 0 && threadIdx.x == 0)
            a.ahist[(size_t)field * a.pring + *a.giter % a.pring] = 0.0;
    }
    if constexpr (UPD || MODE == DST_CORRECT) {
        bool skip = a.ctl != nullptr && a.ctl[field].active == 0;   // CORRECT without ctl: no mask
        if (UPD && a.init) skip = false;
        if (skip) return;   // uniform per block: blocks never span fields
    }
    double alpha_pq = 0.0;
    if constexpr (MODE == DST_UPDATE_PQ) {
        // (p, A p) and alpha as the finalize kernel forms them; block 0 of the
        // field records them (a breakdown stops the shot in every block alike)
        const double tot = fin_sum<FIN_SMALL>(a.pqpart + (size_t)field * a.pstride, a.pq_nparts, red);
        ShotCtl& c = a.ctl[field];
        if (bif == 0 && threadIdx.x == 0) {
            c.pq = tot;
            if (!isfinite(tot)) {
                c.status = LG_ERR_NONFINITE;
                c.active = 0;
            } else if (tot <= 0.0) {
                c.status = LG_ERR_BREAKDOWN;
                c.active = 0;
            } else {
                c.alpha = c.rz / tot;
                if (a.pring > 1) a.ahist[(size_t)field * a.pring + *a.giter % a.pring] = c.alpha;
            }
        }
        if (!isfinite(tot) || tot <= 0.0) return;
        alpha_pq = c.rz / tot;
    }
    // held directions: the solve's iteration count (the update of iteration
    // g reads p_g; the correction after it, with g + 1 counted, reads p_g and
    // writes p_{g+1}; a start or restart writes the first direction at g)
    const int kit = ((UPD || MODE == DST_CORRECT) && a.pring > 1) ? *a.giter : 0;

    cpx<T>* buf = lds + fid * LL;
    const size_t fbase = (size_t)field * a.nz1 * NX1;
    // CORRECT with held directions: p_{k+1} (or the first direction of a
    // phase) goes to slot iters % pring
    T* const outp = a.out + ((MODE == DST_CORRECT && a.pring > 1) ? (size_t)(kit % a.pring) * a.pslot : 0);
    const size_t o0 = fbase + (size_t)j0 * NX1;
    const size_t o1 = fbase + (size_t)j1 * NX1;
    double rr = 0.0, bb = 0.0;
    T pold0[MODE == DST_CORRECT ? NOUT : 1], pold1[MODE == DST_CORRECT ? NOUT : 1];

    // ---- phase A: gather the two rows into the odd extension (LDS) ---------
    // All loads are buffer loads at per-element byte offsets (BUF_OOB for the
    // missing second row of an odd row count and for i >= nx-1, which read 0);
    // a resource of size 0 turns a whole array off (loads 0, stores dropped),
    // so the start and restart variants of the update run the same code.
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nfe = (uint32_t)a.nz1 * (uint32_t)NX1;     // elements per field
    if (live) {
        if constexpr (MODE == DST_RESTART) {
            // r = b - A x in FP64 with the operator kernel's arithmetic (bitwise
            // the separate true-residual pass), stored, then transformed in FP32
            // init 4 (start from a given x) also forms ||b||^2
            const rsrc_t rX = buf_rsrc(a.x + fbase, nfe * 8u);
            const rsrc_t rB = buf_rsrc(a.b + fbase, nfe * 8u);
            const rsrc_t rRs = buf_rsrc(a.r + fbase, nfe * 8u);
            if (a.init == 4 && blockIdx.x == 0 && threadIdx.x == 0) *a.xslot = a.x;
            constexpr int CR = NIT < 2 ? NIT : 2;
#pragma unroll
            for (int cb = 0; cb < NIT; cb += CR) {
                double x0[CR], x1[CR], b0[CR], b1[CR], q0[CR], q1[CR];
                uint32_t e0[CR], e1[CR];
#pragma unroll
                for (int u = 0; u < CR; ++u) {
                    const int i = t + (cb + u) * TPF;
                    const bool in = (cb + u < NIT) && i < NX1;
                    e0[u] = in ? (uint32_t)(j0 * NX1 + i) : BUF_OOB / 8u;
                    e1[u] = (in && has1) ? (uint32_t)(j1 * NX1 + i) : BUF_OOB / 8u;
                    x0[u] = bload<double>(rX, e0[u] * 8u);
                    x1[u] = bload<double>(rX, e1[u] * 8u);
                    b0[u] = bload<double>(rB, e0[u] * 8u);
                    b1[u] = bload<double>(rB, e1[u] * 8u);
                    apply_pair<double>(rX, a.kap64, a.w64, NX1, a.nz1, min(i, NX1 - 1), j0, in, in && has1,
                                       x0[u], x1[u], a.idx2d, a.idz2d, a.free_top != 0, q0[u], q1[u]);
                }
#pragma unroll
                for (int u = 0; u < CR; ++u) {
                    const int i = t + (cb + u) * TPF;
                    const double ra = b0[u] - q0[u];
                    const double rb = b1[u] - q1[u];
                    bstore<double>(ra, rRs, e0[u] * 8u);
                    bstore<double>(rb, rRs, e1[u] * 8u);
                    rr += ra * ra + rb * rb;
                    bb += b0[u] * b0[u] + b1[u] * b1[u];
                    if (cb + u < NIT && i < NX1) {
                        buf[lpad(1 + i)] = {(T)ra, (T)rb};
                        if constexpr (!HALF) buf[lpad(M - 1 - i)] = {(T)-ra, (T)-rb};
                    }
                }
            }
        } else if constexpr (UPD) {
            // init 1 (cold start): only rhat = DST b and ||b||^2; x = 0 and
            // r = b are not stored: the shot's first update (ShotCtl.fresh)
            // reads b for r and takes x as 0, and writes both.  init 2
            // (restart from the stored r): x is not touched.
            const int init = a.init;
            double* X = nullptr;
            const double* B0 = nullptr;
            double alpha = 0.0;
            bool fresh = false;
            if (init == 1) {
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    a.xslot[0] = a.x;
                    a.xslot[1] = const_cast<double*>(a.b);
                }
            } else if (init == 0) {
                X = wave_uniform(a.xslot[0]);
                alpha = MODE == DST_UPDATE_PQ ? alpha_pq : a.ctl[field].alpha;
                fresh = a.ctl[field].fresh != 0;                     // uniform per block
                if (fresh) B0 = wave_uniform(a.xslot[1]);
            }
            // (the bases join paths around the lane-0 slot stores above, which
            // the compiler otherwise takes as divergent)
            double* const Xb = wave_uniform(X != nullptr ? X + fbase : a.r);
            const double* const Rb =
                wave_uniform(init == 1 ? a.b + fbase : (B0 != nullptr ? B0 + fbase : a.r + fbase));
            // held directions: x is neither read nor written here (the flush
            // pass adds alpha_k p_k later); p_k sits at slot k % pring
            const bool xin = a.pring == 1;
            const rsrc_t rX = buf_rsrc(Xb, (init == 0 && !fresh && xin) ? nfe * 8u : 0u);
            const rsrc_t rXs = buf_rsrc(Xb, (init == 0 && xin) ? nfe * 8u : 0u);
            const rsrc_t rR = buf_rsrc(Rb, nfe * 8u);
            const rsrc_t rRs = buf_rsrc(a.r + fbase, init == 0 ? nfe * 8u : 0u);
            const size_t pofs = (init == 0 && a.pring > 1) ? (size_t)(kit % a.pring) * a.pslot : 0;
            const rsrc_t rP = buf_rsrc(a.p + pofs + fbase, init == 0 ? nfe * SZ : 0u);
            const rsrc_t rQ =
                buf_rsrc(a.q + fbase, (init == 0 && (MODE == DST_UPDATE || MODE == DST_UPDATE_PQ)) ? nfe * SZ : 0u);
#pragma unroll
            for (int cb = 0; cb < NIT; cb += CH) {
                // loads of a chunk first (memory-level parallelism), then update
                // and store; chunks keep the register footprint moderate
                double x0[CH], x1[CH], r0[CH], r1[CH];
                T p0[CH], p1[CH], q0[CH], q1[CH];
                uint32_t e0[CH], e1[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int i = t + (cb + u) * TPF;
                    const bool in = (cb + u < NIT) && i < NX1;
                    e0[u] = in ? (uint32_t)(j0 * NX1 + i) : BUF_OOB / 8u;
                    e1[u] = (in && has1) ? (uint32_t)(j1 * NX1 + i) : BUF_OOB / 8u;
                    x0[u] = bload<double>(rX, e0[u] * 8u);
                    r0[u] = bload<double>(rR, e0[u] * 8u);
                    p0[u] = bload<T>(rP, e0[u] * SZ);
                    x1[u] = bload<double>(rX, e1[u] * 8u);
                    r1[u] = bload<double>(rR, e1[u] * 8u);
                    p1[u] = bload<T>(rP, e1[u] * SZ);
                    if constexpr (MODE == DST_UPDATE_OP) {
                        apply_pair<T>(rP, a.kap, a.wsh, NX1, a.nz1, min(i, NX1 - 1), j0, in, in && has1, p0[u],
                                      p1[u], a.idx2, a.idz2, a.free_top != 0, q0[u], q1[u]);
                    } else {
                        q0[u] = bload<T>(rQ, e0[u] * SZ);
                        q1[u] = bload<T>(rQ, e1[u] * SZ);
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int i = t + (cb + u) * TPF;
                    const double ra = r0[u] - alpha * (double)q0[u];
                    const double rb = r1[u] - alpha * (double)q1[u];
                    bstore<double>(x0[u] + alpha * (double)p0[u], rXs, e0[u] * 8u);
                    bstore<double>(ra, rRs, e0[u] * 8u);
                    bstore<double>(x1[u] + alpha * (double)p1[u], rXs, e1[u] * 8u);
                    bstore<double>(rb, rRs, e1[u] * 8u);
                    rr += ra * ra + rb * rb;
                    if (cb + u < NIT && i < NX1) {
                        buf[lpad(1 + i)] = {(T)ra, (T)rb};
                        if constexpr (!HALF) buf[lpad(M - 1 - i)] = {(T)-ra, (T)-rb};
                    }
                }
            }
        } else if constexpr (MODE == DST_CORRECT) {
            // zhat = y + xl u_rs + xr u_{Ls-rs} on segment rows (separator rows as
            // is); the segment geometry depends on the row only.  Absent terms
            // (separator rows, the first / last segment) read 0.
            const int Ls = a.Ls, P = a.P;
            const rsrc_t rY = buf_rsrc(a.y + fbase, nfe * SZ);
            const rsrc_t rU = buf_rsrc((a.utab2 != nullptr && (field & 1)) ? a.utab2 : a.utab,
                                       (uint32_t)Ls * (uint32_t)NX1 * SZ);
            const int rs0 = (j0 + 1) & (Ls - 1), sg0 = (j0 + 1) / Ls;
            const int rs1 = (j1 + 1) & (Ls - 1);
            const bool c0 = rs0 != 0, c1 = has1 && rs1 != 0;
            // row indices (-1: absent) of the y rows and u-table rows.  Separator
            // rows s Ls - 1 are odd (Ls is a power of two >= 2) and j0 is even,
            // so j0 is never a separator and, whenever row j1 needs the
            // correction, it lies in j0's segment: one pair of separator values
            // serves both rows.
            const int l0 = (c0 && sg0 > 0) ? sg0 * Ls - 1 : -1;
            const int r0 = (c0 && sg0 < P - 1) ? (sg0 + 1) * Ls - 1 : -1;
            const int ua0r = c0 ? rs0 : -1, ub0r = c0 ? Ls - rs0 : -1;
            const int ua1r = c1 ? rs1 : -1, ub1r = c1 ? Ls - rs1 : -1;
            const int y1r = has1 ? j1 : -1;
#pragma unroll
            for (int cb = 0; cb < NIT; cb += CH) {
                T yv0[CH], yv1[CH], xl0[CH], xr0[CH];
                T ua0[CH], ub0[CH], ua1[CH], ub1[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int i = t + (cb + u) * TPF;
                    const bool in = (cb + u < NIT) && i < NX1;
                    auto off = [&](int row) -> uint32_t {
                        return (in && row >= 0) ? (uint32_t)(row * NX1 + i) * SZ : BUF_OOB;
                    };
                    yv0[u] = bload<T>(rY, off(j0));
                    yv1[u] = bload<T>(rY, off(y1r));
                    xl0[u] = bload<T>(rY, off(l0));
                    xr0[u] = bload<T>(rY, off(r0));
                    ua0[u] = bload<T>(rU, off(ua0r));
                    ub0[u] = bload<T>(rU, off(ub0r));
                    ua1[u] = bload<T>(rU, off(ua1r));
                    ub1[u] = bload<T>(rU, off(ub1r));
                }
                T v0[CH], v1[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    v0[u] = c0 ? yv0[u] + xl0[u] * ua0[u] + xr0[u] * ub0[u] : yv0[u];
                    v1[u] = c1 ? yv1[u] + xl0[u] * ua1[u] + xr0[u] * ub1[u] : yv1[u];
                }
                if (a.free_top) {                  // + coef_k g_k(j): the free-surface rank-one term
                    const rsrc_t rG = buf_rsrc((a.smg2 != nullptr && (field & 1)) ? a.smg2 : a.smg, nfe * SZ);
                    const rsrc_t rC = buf_rsrc(a.smc + (size_t)field * NX1, (uint32_t)NX1 * 8u);
                    T cf[CH], g0[CH], g1[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int i = t + (cb + u) * TPF;
                        const bool in = (cb + u < NIT) && i < NX1;
                        cf[u] = (T)bload<double>(rC, in ? (uint32_t)i * 8u : BUF_OOB);
                        g0[u] = bload<T>(rG, in ? (uint32_t)(j0 * NX1 + i) * SZ : BUF_OOB);
                        g1[u] = bload<T>(rG, (in && has1) ? (uint32_t)(j1 * NX1 + i) * SZ : BUF_OOB);
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        v0[u] += cf[u] * g0[u];
                        v1[u] += cf[u] * g1[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int i = t + (cb + u) * TPF;
                    if (cb + u < NIT && i < NX1) {
                        buf[lpad(1 + i)] = {v0[u], v1[u]};
                        if constexpr (!HALF) buf[lpad(M - 1 - i)] = {-v0[u], -v1[u]};
                    }
                }
            }
            // p of the outputs this thread will write (read now, used after the
            // FFT): p_k, at slot k % pring with k = iters - 1 (held directions)
            const size_t rofs = (!a.init && a.pring > 1) ? (size_t)((kit + a.pring - 1) % a.pring) * a.pslot : 0;
            const rsrc_t rPo = buf_rsrc(a.out + rofs + fbase, a.init ? 0u : nfe * SZ);
#pragma unroll
            for (int u = 0; u < NOUT; ++u) {
                const int col = HALF ? t + u * TPF : t + (u / (RL / 2)) * TPF + (u % (RL / 2)) * NSL - 1;
                const bool ok = col >= 0 && col < NX1;
                pold0[u] = bload<T>(rPo, ok ? (uint32_t)(j0 * NX1 + col) * SZ : BUF_OOB);
                pold1[u] = bload<T>(rPo, (ok && has1) ? (uint32_t)(j1 * NX1 + col) * SZ : BUF_OOB);
            }
        } else {
            const rsrc_t rI = buf_rsrc(a.in + fbase, nfe * SZ);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int i = t + it * TPF;
                const bool in = i < NX1;
                const T v0 = bload<T>(rI, in ? (uint32_t)(j0 * NX1 + i) * SZ : BUF_OOB);
                const T v1 = bload<T>(rI, (in && has1) ? (uint32_t)(j1 * NX1 + i) * SZ : BUF_OOB);
                if (in) {
                    buf[lpad(1 + i)] = {v0, v1};
                    if constexpr (!HALF) buf[lpad(M - 1 - i)] = {-v0, -v1};
                }
            }
        }
        if (t == 0) {
            buf[lpad(0)] = {(T)0, (T)0};
            if constexpr (!HALF) buf[lpad(NX)] = {(T)0, (T)0};
        }
    } else {
        for (int i = t; i < M; i += TPF) buf[lpad(i)] = {(T)0, (T)0};
    }
    __syncthreads();

    if constexpr (HALF) {
        // ---- pre-pass: y_j, y_{N-j} from f_j, f_{N-j} (j = 1 .. N/2) -------------
        // tw[j] = exp(-i pi j / N), so sin(pi j / N) = -Im tw[j]; j = N/2 writes
        // the same value twice (f_j - f_{N-j} = 0 there)
#pragma unroll
        for (int c = 0; c < CK; ++c) {
            const int j = 1 + t + c * TPF;
            const cpx<T> fj = buf[lpad(j)];
            const cpx<T> fm = buf[lpad(NX - j)];
            const T sj = -a.tw[j].y;
            const T sx = sj * (fj.x + fm.x), sy = sj * (fj.y + fm.y);
            const T dx = (T)0.5 * (fj.x - fm.x), dy = (T)0.5 * (fj.y - fm.y);
            buf[lpad(j)] = {sx + dx, sy + dy};
            buf[lpad(NX - j)] = {sx - dx, sy - dy};
        }
        __syncthreads();

        // ---- transform (length N; the 2N-entry twiddle table with stride 2) -------
        cpx<T> v[R];
        fft_mid<T, M, R, 1, 2>(buf, a.tw, t);
        fft_last<T, M, R, 2>(buf, a.tw, t, v);
        __syncthreads();                           // every thread has read its last-pass inputs
#pragma unroll
        for (int qb = 0; qb < NBL; ++qb)
#pragma unroll
            for (int u = 0; u < RL; ++u) buf[lpad(t + qb * TPF + u * NSL)] = v[qb * RL + u];
        __syncthreads();

        // ---- post-pass: k = t CK + c; two-for-one split and the prefix sum --------
        // row j0 (real part): F_{2k} = -(Im Z_k - Im Z_{N-k})/2, Re Y_k = (Re Z_k + Re Z_{N-k})/2
        // row j1 (imag part): F_{2k} =  (Re Z_k - Re Z_{N-k})/2, Re Y_k = (Im Z_k + Im Z_{N-k})/2
        T ev0[CK], ev1[CK], s0[CK], s1[CK];
        T run0 = (T)0, run1 = (T)0;
#pragma unroll
        for (int c = 0; c < CK; ++c) {
            const int k = t * CK + c;
            const cpx<T> zk = buf[lpad(k)];
            const cpx<T> zm = buf[lpad(k == 0 ? 0 : NX - k)];
            ev0[c] = (T)-0.5 * (zk.y - zm.y);
            ev1[c] = (T)0.5 * (zk.x - zm.x);
            run0 += (T)0.5 * (zk.x + zm.x);
            run1 += (T)0.5 * (zk.y + zm.y);
            s0[c] = run0;
            s1[c] = run1;
        }
        const cpx<T> z0 = buf[lpad(0)];            // Re Y_0 of both rows: (Re Z_0, Im Z_0)
        // exclusive prefix of the thread totals over the transform's TPF threads
        constexpr int W = TPF < 64 ? TPF : 64;     // lanes of one transform within a wave
        const int lane = threadIdx.x & 63;
        T inc0 = run0, inc1 = run1;
#pragma unroll
        for (int d = 1; d < W; d <<= 1) {
            const T u0 = __shfl_up(inc0, d, W), u1 = __shfl_up(inc1, d, W);
            if ((lane & (W - 1)) >= d) {
                inc0 += u0;
                inc1 += u1;
            }
        }
        T off0 = inc0 - run0, off1 = inc1 - run1;
        if constexpr (TPF > 64) {                  // whole waves per transform: add the earlier waves'
            if (lane == 63) wtot[threadIdx.x >> 6] = {inc0, inc1};   // totals of the same transform
            __syncthreads();
            const int w0 = (fid * TPF) >> 6, wme = threadIdx.x >> 6;
            for (int wv = w0; wv < wme; ++wv) {
                off0 += wtot[wv].x;
                off1 += wtot[wv].y;
            }
        }
        __syncthreads();                           // every thread has read Z: reuse the LDS
#pragma unroll
        for (int c = 0; c < CK; ++c) {
            const int k = t * CK + c;
            buf[lpad(2 * k)] = {off0 + s0[c] - (T)0.5 * z0.x, off1 + s1[c] - (T)0.5 * z0.y};   // F_{2k+1}
            if (k > 0) buf[lpad(2 * k - 1)] = {ev0[c], ev1[c]};                                   // F_{2k}
        }
        __syncthreads();

        // ---- outputs: LDS -> global, column t + u TPF ----------------------------
        if (live) {
            T beta = (T)0;
            if constexpr (MODE == DST_CORRECT) beta = a.init ? (T)0 : (T)a.ctl[field].beta;
#pragma unroll
            for (int u = 0; u < NOUT; ++u) {
                const int col = t + u * TPF;
                if (col >= NX1) continue;
                const cpx<T> F = buf[lpad(col)];
                T x0 = F.x, x1 = F.y;
                if constexpr (MODE == DST_FWD || UPD) {
                    outp[o0 + col] = x0;
                    if (has1) outp[o1 + col] = x1;
                } else if constexpr (MODE == DST_INV) {
                    const T sc = (T)(2.0 / NX);
                    outp[o0 + col] = x0 * sc;
                    if (has1) outp[o1 + col] = x1 * sc;
                } else {   // CORRECT: p = z + beta p  (init: p = z)
                    const T sc = (T)(2.0 / NX);
                    x0 *= sc;
                    x1 *= sc;
                    if (a.init) {
                        outp[o0 + col] = x0;
                        if (has1) outp[o1 + col] = x1;
                    } else {
                        outp[o0 + col] = x0 + beta * pold0[u];
                        if (has1) outp[o1 + col] = x1 + beta * pold1[u];
                    }
                }
            }
        }

    } else {
        // ---- transform (2N form) ----------------------------------------------------
        cpx<T> v[R];
        fft_mid<T, M, R, 1>(buf, a.tw, t);
        fft_last<T, M, R>(buf, a.tw, t, v);

        // ---- outputs: registers -> global (first half of the spectrum) ---------
        if (live) {
            T beta = (T)0;
            if constexpr (MODE == DST_CORRECT) beta = a.init ? (T)0 : (T)a.ctl[field].beta;
#pragma unroll
            for (int qb = 0; qb < NBL; ++qb)
#pragma unroll
                for (int u = 0; u < RL / 2; ++u) {
                    const int K = t + qb * TPF + u * NSL;
                    if (K < 1 || K > NX1) continue;
                    const int col = K - 1;
                    const cpx<T> V = v[qb * RL + u];
                    T x0 = -V.y * (T)0.5, x1 = V.x * (T)0.5;
                    if constexpr (MODE == DST_FWD || UPD) {
                        outp[o0 + col] = x0;
                        if (has1) outp[o1 + col] = x1;
                    } else if constexpr (MODE == DST_INV) {
                        const T sc = (T)(2.0 / NX);
                        outp[o0 + col] = x0 * sc;
                        if (has1) outp[o1 + col] = x1 * sc;
                    } else {   // CORRECT: p = z + beta p  (init: p = z)
                        const T sc = (T)(2.0 / NX);
                        const int oi = qb * (RL / 2) + u;
                        x0 *= sc;
                        x1 *= sc;
                        if (a.init) {
                            outp[o0 + col] = x0;
                            if (has1) outp[o1 + col] = x1;
                        } else {
                            outp[o0 + col] = x0 + beta * pold0[oi];
                            if (has1) outp[o1 + col] = x1 + beta * pold1[oi];
                        }
                    }
                }
        }

    }

    if constexpr (UPD) {
        const double s = block_sum(rr, red);
        if (threadIdx.x == 0) a.partial[(size_t)field * a.pstride + bif] = s;
        if (MODE == DST_RESTART && a.init == 4) {
            const double sb = block_sum(bb, red);
            if (threadIdx.x == 0) a.partial[(size_t)field * a.pstride + a.bpf + bif] = sb;
        }
    }
}

// ===========================================================================
// K3: Dichotomy segments.  Each z-system (one wavenumber k) of length nz-1 is
// split into P segments of Ls rows: Ls-1 interior rows and one separator row
// (the last segment has none).  In the normalised system
//   -s_{j-1} + theta_k s_j - s_{j+1} = rhat_j / b
// every interior block is the same (Ls-1)x(Ls-1) Toeplitz matrix, so its
// Thomas factors e_i = 1/(theta - e_{i-1}) are prepared once per plan and
// shared by all segments, shots and iterations.  A lane owns one (k, segment):
// forward sweep, back substitution with zero end values, store y.  It also
// stores the two end values of y and g^T T^{-1} g = sum h_i d_i (h = L^{-1} g,
// from the LDL^T form of the sweep), which the interface step needs.
// ===========================================================================
template <typename T>
struct TdArgs {
    const T* rhat;
    T* y;
    const T* etab;
    double* E;       // [field][P][3][nx1]
    int nx1, nz1, P;
    int spw;         // segments per wave
    int ktiles, sgroups;   // 1D grid of ktiles * sgroups * fields blocks
    int fstride, foff;   // field = grid index * fstride + foff (component selection)
    T inv_b;
    const T* etab2;  // non-null: odd fields (elastic z component) take this block's factors
    T inv_b2;
    ShotCtl* ctl;    // nullptr: no masking
};

// Block = 4 waves over 64 consecutive wavenumbers (lane = k); each wave
// solves `spw` consecutive segments.  The block's slice of the shared Thomas
// factors (LS x 64) is staged once in LDS, so the sweeps read it from LDS
// instead of streaming it from L2 for every segment.
template <typename T, int LS>
__global__ __launch_bounds__(256) void td_kernel(TdArgs<T> a) {
    __shared__ T es[LS * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wavenumber tiles fastest, contiguous per XCD: neighbouring tiles share
    // the cache lines at their edges (rows are not line aligned)
    const int lb = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = lb % a.ktiles, by = (lb / a.ktiles) % a.sgroups, bz = lb / (a.ktiles * a.sgroups);
    const int k = bx * 64 + lane;
    const int field = bz * a.fstride + a.foff;
    if (a.ctl != nullptr && a.ctl[field].active == 0) return;   // uniform per block
    const int nx1 = a.nx1;
    const bool second = a.etab2 != nullptr && (field & 1);       // uniform per block
    const T* __restrict__ etab = second ? a.etab2 : a.etab;
    const T inv_b = second ? a.inv_b2 : a.inv_b;
    {
        const int kk = bx * 64 + (threadIdx.x & 63);
        for (int i = threadIdx.x >> 6; i < LS; i += 4)
            es[i * 64 + (threadIdx.x & 63)] = (kk < nx1) ? etab[(size_t)i * nx1 + kk] : (T)0;
    }
    __syncthreads();
    if (k >= nx1) return;
    constexpr int L = LS - 1;
    const size_t fb = (size_t)field * a.nz1 * nx1;
    const int s_begin = (by * 4 + wave) * a.spw;
    const int s_end = min(s_begin + a.spw, a.P);
    for (int s = s_begin; s < s_end; ++s) {
        const T* __restrict__ g = a.rhat + fb + (size_t)(s * LS) * nx1 + k;   // row s*LS (+i-1)
        T* __restrict__ yo = a.y + fb + (size_t)(s * LS) * nx1 + k;
        T d[LS];
#pragma unroll
        for (int i = 1; i <= L; ++i) d[i] = g[(size_t)(i - 1) * nx1];
        T prev = (T)0;
        double d0 = 0.0;
#pragma unroll
        for (int i = 1; i <= L; ++i) {
            const T h = d[i] * inv_b + prev;
            prev = h * es[i * 64 + lane];
            d[i] = prev;
            d0 += (double)h * (double)prev;
        }
        T yv = d[L];
        yo[(size_t)(L - 1) * nx1] = yv;
        const T ylast = yv;
#pragma unroll
        for (int i = L - 1; i >= 1; --i) {
            yv = d[i] + es[i * 64 + lane] * yv;
            yo[(size_t)(i - 1) * nx1] = yv;
        }
        double* E = a.E + ((size_t)field * a.P + s) * 3 * nx1 + k;
        E[0] = (double)yv;          // y_1
        E[nx1] = (double)ylast;     // y_{Ls-1}
        E[2 * (size_t)nx1] = d0;    // g^T T^{-1} g on the segment
    }
}

// ===========================================================================
// K4: interface systems.  With the segment solutions y^s and the end
// responses u (T u = e_1, v = reversed u), the separator values x_s satisfy
// a Toeplitz tridiagonal system of size P-1:
//   Ar x_s - Br (x_{s-1} + x_{s+1}) = G_s = g_sep(s) + y^s_last + y^{s+1}_first,
//   Ar = theta - 2 u_1, Br = u_{Ls-1}.
// It is solved by the Dichotomy principle: at level l the unknowns split into
// subdomains of 2^(q-l)-1 bounded by already-known separators; the middle
// unknown of each is a weighted sum of the G in its subdomain (a row of the
// subdomain's inverse, prepared once) plus the response to the two known
// boundary values; the sums are segmented reductions across the lanes of the
// wave (one lane per separator).  The wave also forms this system's share of
// (rhat, zhat) = b (sum_s g^T T^{-1} g + sum_s x_s G_s), one partial per
// block; the finalize kernel turns their sum into (r, z) = (2/nx) (rhat, zhat)
// and beta.
// mode 0: interface only; 1: CG start (rz); 2: CG iteration (beta, rz).
// ===========================================================================
template <typename T>
struct RsArgs {
    const T* rhat;
    T* y;
    const double* E;
    const double* red;   // [nx1][RW]
    int nx1, nz1, P, q, Ls, RW;
    int fstride, foff;   // field = grid index * fstride + foff
    double inv_b;
    const double* red2;  // non-null: odd fields (elastic z component) take this block's tables
    double inv_b2;
    int mode;
    ShotCtl* ctl;
    double* partial;
    size_t pstride;
    int free_top;          // free surface: form coef_k of the rank-one term
    const double* smt;     // 1 / (1 - g_k(0))
    double* smc;           // out: coef_k per field
};

// One block per (KT consecutive wavenumbers, field).  Phase 1 loads, with
// every load issued up front, the interface right-hand sides G[s][k] (row
// reads of the separator rows and of the segment data E) and the block's
// slice of the interface weight table into LDS; phase 2 solves the KT
// systems, each by one wave with one lane per separator, and overwrites G by
// the separator values; phase 3 writes them back row by row and forms this
// block's share of (rhat, zhat) / b.  PM >= P bounds the phase-1 unroll.
constexpr int RS_ILP = 4;       // wavenumbers per wave in flight in phase 2
template <typename T, int KT, int PM>
__global__ __launch_bounds__(256) void rs_kernel(RsArgs<T> a) {
    constexpr int KS = KT + 1;             // padded LDS row
    constexpr int NG = 256 / KT;           // thread groups over separators
    constexpr int NIT1 = (PM + NG - 1) / NG;
    extern __shared__ double rs_lds[];
    __shared__ double red[4];
    const int P = a.P, q = a.q, Ls = a.Ls, nx1 = a.nx1, RW = a.RW;
    double* Gs = rs_lds;                   // [P-1][KS]
    double* Ws = rs_lds + (P - 1) * KS;    // [KT][RW]
    const int nkt = (nx1 + KT - 1) / KT;
    const int lb = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = lb % nkt, bf = lb / nkt;
    const int field = bf * a.fstride + a.foff;
    if (a.mode != 0 && a.ctl[field].active == 0) return;   // uniform per block
    const int tid = threadIdx.x, kl = tid % KT, grp = tid / KT;
    const int k0 = bx * KT;
    const int k = k0 + kl;
    const bool valid = k < nx1;
    constexpr uint32_t SZ = sizeof(T);
    const size_t fb = (size_t)field * a.nz1 * nx1;
    const rsrc_t rR = buf_rsrc(a.rhat + fb, (uint32_t)a.nz1 * (uint32_t)nx1 * SZ);
    const rsrc_t rE = buf_rsrc(a.E + (size_t)field * P * 3 * nx1, (uint32_t)P * 3u * (uint32_t)nx1 * 8u);
    const bool second = a.red2 != nullptr && (field & 1);        // uniform per block
    const double inv_b = second ? a.inv_b2 : a.inv_b;
    const rsrc_t rW = buf_rsrc(second ? a.red2 : a.red, (uint32_t)nx1 * (uint32_t)RW * 8u);
    // weight table rows k0 .. k0+KT-1 are contiguous
    for (int e = tid; e < KT * RW; e += 256)
        Ws[e] = bload<double>(rW, (uint32_t)(k0 * RW + e) * 8u);
    double d0 = 0.0;
    double gv[NIT1];
#pragma unroll
    for (int it = 0; it < NIT1; ++it) {
        const int sg = grp + it * NG;
        const bool okd = valid && sg < P, okg = valid && sg < P - 1;
        d0 += bload<double>(rE, okd ? (uint32_t)((sg * 3 + 2) * nx1 + k) * 8u : BUF_OOB);
        gv[it] = (double)bload<T>(rR, okg ? (uint32_t)(((sg + 1) * Ls - 1) * nx1 + k) * SZ : BUF_OOB) * inv_b +
                 bload<double>(rE, okg ? (uint32_t)((sg * 3 + 1) * nx1 + k) * 8u : BUF_OOB) +
                 bload<double>(rE, okg ? (uint32_t)(((sg + 1) * 3 + 0) * nx1 + k) * 8u : BUF_OOB);
    }
#pragma unroll
    for (int it = 0; it < NIT1; ++it) {
        const int sg = grp + it * NG;
        if (sg < P - 1) Gs[sg * KS + kl] = gv[it];
    }
    __syncthreads();

    // phase 2: Dichotomy on the interface system, lanes = separators
    const int lane = tid & 63, wave = tid >> 6;
    const int sig = lane;
    const bool sepl = sig < P - 1;
    double c = d0;
    // RS_ILP wavenumbers of a wave at a time: independent shuffle chains
    // (each level waits on the previous one's broadcast) interleave; c is
    // accumulated in wavenumber order as with one at a time
    for (int kb = wave; kb < KT; kb += 4 * RS_ILP) {
        if (k0 + kb >= nx1) break;                          // uniform per wave
        double G[RS_ILP], x[RS_ILP];
        const double* tab[RS_ILP];
        bool okk[RS_ILP];
#pragma unroll
        for (int j = 0; j < RS_ILP; ++j) {
            const int kk = kb + 4 * j;
            okk[j] = kk < KT && k0 + kk < nx1;              // uniform per wave
            const int kc = okk[j] ? kk : kb;
            tab[j] = Ws + kc * RW;
            G[j] = sepl ? Gs[sig * KS + kc] : 0.0;
            x[j] = 0.0;
        }
        int woff = 2 + q;
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            if (l >= q) break;
            const int size = P >> l;
            const int pos = sig & (size - 1);
            const bool member = sepl && (pos != size - 1);
            const int widx = min(pos, size - 2 - pos);
            const int base = sig - pos;
            const int ll = base - 1, rl = base + size - 1;
            double tv[RS_ILP];
#pragma unroll
            for (int j = 0; j < RS_ILP; ++j) tv[j] = member ? tab[j][woff + (widx < 0 ? 0 : widx)] * G[j] : 0.0;
            for (int off = 1; off < size; off <<= 1)
#pragma unroll
                for (int j = 0; j < RS_ILP; ++j) tv[j] += __shfl_xor(tv[j], off, 64);
#pragma unroll
            for (int j = 0; j < RS_ILP; ++j) {
                const double xl_ = __shfl(x[j], ll < 0 ? 0 : ll, 64);
                const double xr_ = __shfl(x[j], rl > 63 ? 63 : rl, 64);
                const double xl = (ll < 0) ? 0.0 : xl_;
                const double xr = (rl >= P - 1) ? 0.0 : xr_;
                if (member && pos == (size >> 1) - 1) x[j] = tv[j] + tab[j][2 + l] * (xl + xr);
            }
            woff += size >> 1;
        }
#pragma unroll
        for (int j = 0; j < RS_ILP; ++j) {
            if (!okk[j]) continue;                          // uniform per wave
            const int kk = kb + 4 * j;
            if (sepl) {
                c += x[j] * G[j];
                Gs[sig * KS + kk] = x[j];
            }
            if (a.free_top && sig == 0) {
                // first row of the Dirichlet solution: zhat_0 = y_0 + x_0 u_{Ls-1}
                // (u_{Ls-1} = Br; x = 0 when there is no separator); the rank-one
                // term adds coef g with coef = zhat_0 / (1 - g_0), and
                // (rhat, g) = b zhat_0 adds coef zhat_0 to (rhat, zhat) / b
                const int kg = k0 + kk;
                const double zh0 = bload<double>(rE, (uint32_t)kg * 8u) + x[j] * tab[j][1];
                const double cf = zh0 * a.smt[kg];
                a.smc[(size_t)field * nx1 + kg] = cf;
                c += cf * zh0;
            }
        }
    }
    __syncthreads();

    // phase 3: store the separator values
    const rsrc_t rY = buf_rsrc(a.y + fb, (uint32_t)a.nz1 * (uint32_t)nx1 * SZ);
    for (int sg = grp; sg < P - 1; sg += NG)
        bstore<T>((T)Gs[sg * KS + kl], rY, valid ? (uint32_t)(((sg + 1) * Ls - 1) * nx1 + k) * SZ : BUF_OOB);
    if (a.mode == 0) return;
    const double s = block_sum(c, red);
    if (tid == 0) a.partial[(size_t)field * a.pstride + bx] = s;
}

// ===========================================================================
// Grid-wide reductions of the CG scalars: one block per field sums the
// per-block partials of the preceding kernel in a fixed order (so results
// are bitwise reproducible) and updates the field's control block.
// ===========================================================================
enum FinKind { FIN_PQ = 0, FIN_RR = 1, FIN_RZ = 2 };

struct FinArgs {
    ShotCtl* ctl;
    const double* partial;
    size_t pstride;
    int nparts;
    int kind;
    int init;         // FIN_RR: start of a solve; FIN_RZ: 1 start, 2 iteration
    double tol2;      // (init 1, 4) squared recursive tolerance of the first phase
    double tol2f;     // (init 1, 4) squared requested tolerance
    double tol2r;     // (init 1, 4) squared recursive tolerance of restart phases
    int max_iter;
    double scale;     // FIN_RZ: b * 2/nx
    double* ahist;    // FIN_PQ with pring > 1: alpha_g kept at [field][g % pring] (0: no update)
    int pring;
    int* giter;       // pring > 1: [0] the solve's iteration count g, [1] iterations added into x
};

template <int NT>
__global__ __launch_bounds__(NT) void finalize_kernel(FinArgs a) {
    __shared__ double red[NT / 64];
    const int field = blockIdx.x;
    ShotCtl& c = a.ctl[field];
    const bool start_rr = (a.kind == FIN_RR && a.init);
    if (a.pring > 1 && threadIdx.x == 0) {   // held directions (before the masked shots leave)
        if (a.kind == FIN_PQ)                 // alpha_g stays 0 unless this shot's update runs
            a.ahist[(size_t)field * a.pring + a.giter[0] % a.pring] = 0.0;
        if (a.kind == FIN_RR && blockIdx.x == 0) {
            if (a.init == 1 || a.init == 4) {   // a start: no iteration yet, none added
                a.giter[0] = 0;
                a.giter[1] = 0;
            } else if (a.init == 0) {
                a.giter[0] += 1;               // iteration g done, for every shot
            }
        }
    }
    if (!start_rr && c.active == 0) return;                  // uniform per block
    const double* part = a.partial + (size_t)field * a.pstride;
    const double tot = fin_sum<NT>(part, a.nparts, red);
    double bbt = 0.0;                                        // FIN_RR init 4: ||b||^2 after the rr set
    if (a.kind == FIN_RR && a.init == 4) bbt = fin_sum<NT>(part + a.nparts, a.nparts, red);
    if (threadIdx.x != 0) return;
    if (a.kind == FIN_PQ) {
        c.pq = tot;
        if (!isfinite(tot)) {
            c.status = LG_ERR_NONFINITE;
            c.active = 0;
        } else if (tot <= 0.0) {
            c.status = LG_ERR_BREAKDOWN;
            c.active = 0;
        } else {
            c.alpha = c.rz / tot;
            if (a.pring > 1) a.ahist[(size_t)field * a.pring + *a.giter % a.pring] = c.alpha;
        }
    } else if (a.kind == FIN_RR) {
        c.rr = tot;
        if (a.init == 4) {                   // start from a given x: r = b - A x, ||b||^2 second
            c.bb = bbt;
            c.tol2 = a.tol2 * bbt;
            c.tol2f = a.tol2f * bbt;
            c.tol2r = a.tol2r * bbt;
            c.iters = 0;
            c.fresh = 0;                     // x and r are stored
            c.xzero = 0;
            c.max_iter = a.max_iter;
            c.alpha = 0.0;
            c.beta = 0.0;
            if (!isfinite(tot) || !isfinite(bbt)) {
                c.status = LG_ERR_NONFINITE;
                c.active = 0;
            } else if (bbt == 0.0 || tot <= c.tol2f) {
                c.status = LG_OK;            // b = 0: the host sets x = 0
                c.active = 0;
            } else {
                c.status = LG_ERR_NOT_CONVERGED;
                c.active = 1;
            }
        } else if (a.init == 2) {            // restart from the true residual
            // only shots that met the tolerance are re-checked (b = 0 is final:
            // its solution is 0, set by the host for a given x)
            if (c.status != LG_OK || c.bb == 0.0) return;
            c.alpha = 0.0;
            c.beta = 0.0;
            c.tol2 = c.tol2r;                // the restart phase's recursive target
            if (!isfinite(tot)) {
                c.status = LG_ERR_NONFINITE;
                c.active = 0;
            } else if (tot <= c.tol2f) {
                c.status = LG_OK;
                c.active = 0;
            } else if (c.iters >= c.max_iter) {
                c.status = LG_ERR_NOT_CONVERGED;
                c.active = 0;
            } else {
                c.status = LG_ERR_NOT_CONVERGED;
                c.active = 1;
            }
        } else if (a.init) {
            c.bb = tot;
            c.tol2 = a.tol2 * tot;
            c.tol2f = a.tol2f * tot;
            c.tol2r = a.tol2r * tot;
            c.iters = 0;
            c.max_iter = a.max_iter;
            c.alpha = 0.0;
            c.beta = 0.0;
            c.fresh = 1;                         // cold start: x = 0, r = b implied
            c.xzero = 1;
            if (!isfinite(tot)) {
                c.status = LG_ERR_NONFINITE;
                c.active = 0;
            } else if (tot == 0.0) {
                c.status = LG_OK;
                c.active = 0;
            } else {
                c.status = LG_ERR_NOT_CONVERGED;
                c.active = 1;
            }
        } else {
            const int it = c.iters + 1;
            c.iters = it;
            c.fresh = 0;
            if (!isfinite(tot)) {
                c.status = LG_ERR_NONFINITE;
                c.active = 0;
            } else if (tot <= c.tol2) {
                c.status = LG_OK;
                c.active = 0;
            } else if (it >= c.max_iter) {
                c.status = LG_ERR_NOT_CONVERGED;
                c.active = 0;
            }
        }
    } else {
        const double rz = tot * a.scale;
        if (!isfinite(rz)) {
            c.status = LG_ERR_NONFINITE;
            c.active = 0;
        } else if (a.init == 1) {
            c.rz = rz;
            c.beta = 0.0;
        } else {
            c.beta = rz / c.rz;
            c.rz = rz;
        }
    }
}

// Held search directions: x += alpha_j p_j for the iterations j = giter[1]
// .. giter[0]-1, in order, with the FP64 product and sum of the in-place
// update (so x is bitwise the same); iterations in which the shot was masked
// (alpha_j = 0: no update ran) are skipped.  x is taken as 0 while xzero (a
// cold start not yet flushed), which also writes x = 0 for a shot that never
// iterated.  One pass reads each held direction once and x once, writes x
// once.
constexpr int FLUSH_EPT = 4;   // elements per thread
template <typename T>
__global__ __launch_bounds__(256) void flush_x_kernel(double* __restrict__ x, const T* __restrict__ pr,
                                                      const double* __restrict__ ahist,
                                                      const ShotCtl* __restrict__ ctl, const int* __restrict__ giter,
                                                      int pring, size_t pslot, size_t npts, int bpf) {
    const int field = blockIdx.x / bpf;
    const int bif = blockIdx.x - field * bpf;
    const int j0 = giter[1];
    const int n = giter[0] - j0;
    const bool zero = ctl[field].xzero != 0;
    // nothing to add (no iteration, or the shot was masked in all of them):
    // x stays as it is, unless it is still the implied 0 of a cold start
    bool any = zero;
    for (int j = 0; j < n && !any; ++j) any = ahist[(size_t)field * pring + (j0 + j) % pring] != 0.0;
    if (!any) return;                               // uniform per block
    const size_t fb = (size_t)field * npts;
    const size_t e0 = (size_t)bif * (256 * FLUSH_EPT) + threadIdx.x;
    double v[FLUSH_EPT];
#pragma unroll
    for (int u = 0; u < FLUSH_EPT; ++u) {
        const size_t e = e0 + (size_t)u * 256;
        v[u] = (!zero && e < npts) ? x[fb + e] : 0.0;
    }
    for (int j = 0; j < n; ++j) {
        const int sl = (j0 + j) % pring;
        const double al = ahist[(size_t)field * pring + sl];
        if (al == 0.0) continue;                    // masked in iteration j0 + j (uniform)
        const T* ps = pr + (size_t)sl * pslot + fb;
        T pv[FLUSH_EPT];
#pragma unroll
        for (int u = 0; u < FLUSH_EPT; ++u) {
            const size_t e = e0 + (size_t)u * 256;
            pv[u] = e < npts ? ps[e] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < FLUSH_EPT; ++u) v[u] = v[u] + al * (double)pv[u];
    }
#pragma unroll
    for (int u = 0; u < FLUSH_EPT; ++u) {
        const size_t e = e0 + (size_t)u * 256;
        if (e < npts) x[fb + e] = v[u];
    }
}

// after a flush: every held direction is in x
__global__ __launch_bounds__(256) void flush_done_kernel(ShotCtl* ctl, int* giter, int nf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) giter[1] = giter[0];
    if (f < nf) ctl[f].xzero = 0;
}

// Standalone interface correction (the CG path fuses it into K5):
// zhat = y + xl u_i + xr u_{Ls-i} on segment rows, in place.
template <typename T>
// phase 0: segment rows (the separator rows are read, not written); with a
// free surface (smg != nullptr) also + coef_k g_k(j).  phase 1 (free surface
// only, after phase 0): the separator rows' rank-one term.
__global__ __launch_bounds__(256) void correct_kernel(T* y, const T* utab, const T* utab2, int nx1, int nz1,
                                                      int Ls, int P, size_t total, int fstride,
                                                      int foff, const T* smg, const double* smc, int phase) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const size_t npts = (size_t)nx1 * nz1;
    const size_t f = (e / npts) * fstride + foff;
    const size_t pt = e % npts;
    const int j = (int)(pt / nx1), k = (int)(pt - (size_t)j * nx1);
    const int jj = j + 1;
    const int rs = jj & (Ls - 1);
    T* Y = y + f * npts;
    const T sm = (smg != nullptr) ? (T)smc[f * nx1 + k] * smg[pt] : (T)0;
    if (phase == 1) {
        if (rs == 0) Y[pt] = Y[pt] + sm;
        return;
    }
    if (rs == 0) return;
    const int s = jj / Ls;
    const T xl = (s > 0) ? Y[(size_t)(s * Ls - 1) * nx1 + k] : (T)0;
    const T xr = (s < P - 1) ? Y[(size_t)((s + 1) * Ls - 1) * nx1 + k] : (T)0;
    const T* __restrict__ u = (utab2 != nullptr && (f & 1)) ? utab2 : utab;   // odd fields: the second block
    Y[pt] = Y[pt] + xl * u[(size_t)rs * nx1 + k] + xr * u[(size_t)(Ls - rs) * nx1 + k] + sm;
}

// Elastic traction-free surface, with the correction fused into the inverse
// transform: coef_k = zhat(row 1, k) / (1 - g_k(1)) per field from the
// uncorrected Dichotomy result, zhat(row 1) formed as correct_kernel forms it
// (odd fields: the second block's tables).
template <typename T>
__global__ __launch_bounds__(256) void surface_coef_fused_kernel(const T* __restrict__ y, const T* __restrict__ utab,
                                                                 const T* __restrict__ utab2,
                                                                 const double* __restrict__ t0,
                                                                 const double* __restrict__ t1,
                                                                 double* __restrict__ coef, int nx1, int Ls, int P,
                                                                 size_t npts, int nfields) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)nfields * nx1) return;
    const size_t f = e / nx1;
    const int k = (int)(e - f * nx1);
    const T* Y = y + f * npts;
    const size_t pt = (size_t)nx1 + k;             // row 1
    const int rs = 2 & (Ls - 1);                   // its position in the first segment
    T v = Y[pt];
    if (rs != 0 && P > 1) {                        // no left separator in the first segment
        const T* __restrict__ u = (utab2 != nullptr && (f & 1)) ? utab2 : utab;
        v = v + Y[(size_t)(Ls - 1) * nx1 + k] * u[(size_t)(Ls - rs) * nx1 + k];
    }
    coef[f * nx1 + k] = (double)v * ((f & 1) ? t1 : t0)[k];
}

hipError_t launch_surface_coef_fused(lg_plan* p, const void* y, int nfields) {
    const PrecBlock& B = p->blk[0];
    const dim3 grid((unsigned)(((size_t)nfields * p->nx1 + 255) / 256));
    if (p->prec == LG_FP64)
        hipLaunchKernelGGL(surface_coef_fused_kernel<double>, grid, dim3(256), 0, p->stream, (const double*)y,
                           (const double*)B.utab, (const double*)p->blk[1].utab, p->es_t[0], p->es_t[1], p->sm_c,
                           p->nx1, B.Ls, B.P, p->npts, nfields);
    else
        hipLaunchKernelGGL(surface_coef_fused_kernel<float>, grid, dim3(256), 0, p->stream, (const float*)y,
                           (const float*)B.utab, (const float*)p->blk[1].utab, p->es_t[0], p->es_t[1], p->sm_c,
                           p->nx1, B.Ls, B.P, p->npts, nfields);
    return hipGetLastError();
}

// ===========================================================================
// Right-hand side of harmonic m (eq. laguerre_h, SPD sign):
//   P_{m-1} = sqrt((m-1)/(m-1+a)) P_{m-2} + R_{m-1}
//   Q_m     = sqrt(m/(m+a)) (Q_{m-1} + P_{m-1})
//   rhs     = -h^2 rho Q_m           (the source is added by src_kernel)
// ===========================================================================
__global__ __launch_bounds__(256) void rhs_kernel(int m, const double* __restrict__ Rp,
                                                  double* __restrict__ Ph, double* __restrict__ Qh,
                                                  const double* __restrict__ rho, double hh,
                                                  double rp, double rq, double* __restrict__ rhs,
                                                  size_t npts, size_t total) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    if (m == 0) {
        Ph[e] = 0.0;
        Qh[e] = 0.0;
        rhs[e] = 0.0;
        return;
    }
    const double P = rp * Ph[e] + Rp[e];
    const double Q = rq * (Qh[e] + P);
    Ph[e] = P;
    Qh[e] = Q;
    rhs[e] = 0.0 - (hh * rho[e % npts]) * Q;
}

constexpr int SRC_CHUNK = 64;
struct SrcArgs {
    int n;
    int64_t idx[SRC_CHUNK];     // element offset of the source node, per shot
    double val[SRC_CHUNK];
};

__global__ void src_kernel(SrcArgs s, double* rhs) {
    const int t = threadIdx.x;
    if (t < s.n) rhs[s.idx[t]] += s.val[t];
}

// ===========================================================================
// Synthesis (eq. series_lag): snapshots += W_s R_m; receiver-row coefficients.
// ===========================================================================
constexpr int MAX_SNAP = 8;
constexpr int MAX_SB = 8;      // harmonics per synthesis pass
struct SynArgs {
    const double* R[MAX_SB];      // R_{m0 + b}, b < nb
    double* snap;
    double* rec;
    double W[MAX_SNAP][MAX_SB];   // W[s][b]: snapshot s, harmonic m0 + b
    int nsnap, m0, nb, n, rec_row0, nx1, nz1;
    size_t npts, total;
};

// snap[s] += W[s][0] R_{m0} + W[s][1] R_{m0+1} + ..., added one harmonic at a
// time in order (the same FP64 operations as one pass per harmonic), so nb
// harmonics read and write each snapshot once; receiver rows copied out.
__global__ __launch_bounds__(256) void synth_kernel(SynArgs a) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.total) return;
    double R[MAX_SB];
#pragma unroll
    for (int b = 0; b < MAX_SB; ++b) R[b] = b < a.nb ? a.R[b][e] : 0.0;
#pragma unroll
    for (int s = 0; s < MAX_SNAP; ++s) {
        if (s >= a.nsnap) break;
        double v = a.snap[(size_t)s * a.total + e];
#pragma unroll
        for (int b = 0; b < MAX_SB; ++b)
            if (b < a.nb) v += a.W[s][b] * R[b];
        a.snap[(size_t)s * a.total + e] = v;
    }
    if (a.rec != nullptr) {
        const size_t f = e / a.npts;
        const size_t pt = e - f * a.npts;
        const int j = (int)(pt / a.nx1);
        if (j == a.rec_row0) {
            const int i = (int)(pt - (size_t)j * a.nx1);
#pragma unroll
            for (int b = 0; b < MAX_SB; ++b)
                if (b < a.nb) a.rec[(f * a.n + a.m0 + b) * a.nx1 + i] = R[b];
        }
    }
}

// traces[f][q][i] = sum_m W[q][m] rec[f][m][i]   (FP64; 8 outputs per thread)
constexpr int TR_Q = 8;
__global__ __launch_bounds__(256) void traces_kernel(const double* __restrict__ rec,
                                                     const double* __restrict__ W, int n, int nt,
                                                     int nx1, double* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int q0 = blockIdx.y * TR_Q;
    const int f = blockIdx.z;
    if (i >= nx1) return;
    double acc[TR_Q];
#pragma unroll
    for (int u = 0; u < TR_Q; ++u) acc[u] = 0.0;
    const double* rf = rec + (size_t)f * n * nx1 + i;
    for (int m = 0; m < n; ++m) {
        const double v = rf[(size_t)m * nx1];
#pragma unroll
        for (int u = 0; u < TR_Q; ++u)
            if (q0 + u < nt) acc[u] += W[(size_t)(q0 + u) * n + m] * v;
    }
#pragma unroll
    for (int u = 0; u < TR_Q; ++u)
        if (q0 + u < nt) out[((size_t)f * nt + q0 + u) * nx1 + i] = acc[u];
}

// ===========================================================================
// launchers
// ===========================================================================
// Blocks per field of the row-transform kernels with one row pair per 256
// threads (the FP32 update with A p recomputed takes two pairs per block, so
// fewer): the partial buffer's stride and the stored-q update's grid.
int dst_blocks_per_field(int nx, int nz1, int ws) {
    const int M = dst_half_form(nx, ws) ? nx : 2 * nx;   // FFT length of the row transform
    const int R = M >= 16 ? 16 : M;
    const int TPF = M / R;
    const int FPB = TPF >= 256 ? 1 : 256 / TPF;
    const int npairs = (nz1 + 1) / 2;
    return (npairs + FPB - 1) / FPB;
}

namespace {

hipError_t finalize(lg_plan* p, int kind, int nparts, int init, double tol2, int max_iter, double scale,
                    double tol2f = -1.0, double tol2r = -1.0) {
    FinArgs f;
    f.tol2f = tol2f < 0.0 ? tol2 : tol2f;
    f.tol2r = tol2r < 0.0 ? tol2 : tol2r;
    f.ctl = p->ctl;
    f.partial = p->partial;
    f.pstride = p->partial_stride;
    f.nparts = nparts;
    f.kind = kind;
    f.init = init;
    f.tol2 = tol2;
    f.max_iter = max_iter;
    f.scale = scale;
    f.ahist = p->ahist;
    f.pring = p->pring;
    f.giter = p->giter;
    if (nparts <= FIN_SMALL_MAX)
        hipLaunchKernelGGL(finalize_kernel<FIN_SMALL>, dim3(p->S * p->C), dim3(FIN_SMALL), 0, p->stream, f);
    else
        hipLaunchKernelGGL(finalize_kernel<FIN_LARGE>, dim3(p->S * p->C), dim3(FIN_LARGE), 0, p->stream, f);
    return hipGetLastError();
}

// The stored-q update sums the operator's (p, A p) partials itself
// (DST_UPDATE_PQ) where a field has at most FIN_SMALL_MAX of them and the
// update's blocks re-read at most 32 MB of them in all: a finalize launch
// less per iteration for small batches, where launch latency sets the time.
bool fold_pq(const lg_plan* p) {
    if (p->cyl || p->order != 2 || p->fuse_op) return false;
    const size_t np = (size_t)((p->nx1 + 63) / 64) * ((p->nz1 + 4 * ST_RPT - 1) / (4 * ST_RPT));
    const size_t bpf = (size_t)dst_blocks_per_field(p->g.nx, p->nz1, (int)wsize(p));
    return np <= (size_t)FIN_SMALL_MAX && (size_t)p->S * p->C * bpf * np * 8 <= ((size_t)32 << 20);
}

template <typename T>
hipError_t stencil_T(lg_plan* p, const T* x, T* y, bool reduce) {
    // y == nullptr with reduce: only the (p, A p) partials (the update kernel
    // recomputes A p itself)
    StArgs<T> a;
    a.p = x;
    a.q = y;
    a.b = nullptr;
    a.kap = (const T*)p->kap;
    a.w = (const T*)p->w;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.idx2 = (T)(1.0 / (p->g.dx * p->g.dx));
    a.idz2 = (T)(1.0 / (p->g.dz * p->g.dz));
    a.ctl = reduce ? p->ctl : nullptr;
    a.pring = reduce ? p->pring : 1;
    a.pslot = p->nvec;
    a.giter = p->giter;
    a.free_top = p->free_top ? 1 : 0;
    const bool fold = reduce && fold_pq(p);      // the update sums these partials itself
    a.partial = fold ? p->partial_pq : p->partial;
    a.pstride = p->partial_stride;
    a.nfields = p->S * p->C;
    a.nsh = std::min(a.nfields, p->op_shots);
    a.gx = (p->nx1 + 63) / 64;
    a.gy = (p->nz1 + 4 * ST_RPT - 1) / (4 * ST_RPT);
    const dim3 grid(a.gx * a.gy * ((a.nfields + a.nsh - 1) / a.nsh));
    hipLaunchKernelGGL((stencil_kernel<T, false>), grid, dim3(256), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !reduce || fold) return e;
    return finalize(p, FIN_PQ, a.gx * a.gy, 0, 0.0, 0, 0.0);
}

// ||b - A x||^2 per shot with the FP64 medium, then the restart check of the
// finalize kernel (shots that met the tolerance recursively stop or resume)
hipError_t residual_check_T(lg_plan* p, const double* b, const double* x) {
    StArgs<double> a;
    a.p = x;
    a.q = nullptr;
    a.b = b;
    a.kap = (p->prec == LG_FP64) ? (const double*)p->kap : p->kap64;
    a.w = (p->prec == LG_FP64) ? (const double*)p->w : p->w64;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.idx2 = 1.0 / (p->g.dx * p->g.dx);
    a.idz2 = 1.0 / (p->g.dz * p->g.dz);
    a.ctl = p->ctl;
    a.pring = 1;
    a.pslot = 0;
    a.giter = p->giter;
    a.free_top = p->free_top ? 1 : 0;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.nfields = p->S * p->C;
    a.nsh = std::min(a.nfields, p->op_shots);
    a.gx = (p->nx1 + 63) / 64;
    a.gy = (p->nz1 + 4 * ST_RPT - 1) / (4 * ST_RPT);
    const dim3 grid(a.gx * a.gy * ((a.nfields + a.nsh - 1) / a.nsh));
    hipLaunchKernelGGL((stencil_kernel<double, true>), grid, dim3(256), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(p, FIN_RR, a.gx * a.gy, 2, 0.0, 0, 0.0);
}

template <typename T, int NX, int MODE>
hipError_t dst_launch_M(lg_plan* pl, DstArgs<T>& a, int nfields) {
    constexpr bool H = dst_half_form(NX, (int)sizeof(T));
    constexpr int M = H ? NX : 2 * NX;         // FFT length
    constexpr int R = M >= 16 ? 16 : M;
    constexpr int TPF = M / R;
    // the FP32 update with A p recomputed takes two row pairs of 256 threads
    // per block (their p halo and medium rows overlap: 1.69 -> 1.67 ms at 64
    // shots 2048^2; four pairs, or two in the correction, measured slower);
    // the FP64 N-point transforms of nx = 2048 outside the CG update take one
    // pair of 128 threads (more blocks in flight: GMRES(10) cycle at 1024^2
    // 1.434 -> 1.422 ms, FP64 64 shots 2048^2 78.3 -> 75.6-77.6 ms per harmonic)
    constexpr int FPB = (MODE == DST_UPDATE_OP && TPF == 256 && sizeof(T) == 4) ? 2
                      : ((MODE == DST_FWD || MODE == DST_INV || MODE == DST_CORRECT) && TPF == 128 && sizeof(T) == 8)
                          ? 1
                          : (TPF >= 256 ? 1 : 256 / TPF);
    const int npairs = (a.nz1 + 1) / 2;
    a.bpf = (npairs + FPB - 1) / FPB;
    const dim3 grid(a.bpf * nfields);
    hipLaunchKernelGGL((dst_kernel<T, M, R, FPB, MODE, H>), grid, dim3(FPB * TPF), 0, pl->stream, a);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t dst_dispatch(lg_plan* pl, DstArgs<T>& a, int nfields) {
    switch (pl->g.nx) {
        case 2: return dst_launch_M<T, 2, MODE>(pl, a, nfields);
        case 4: return dst_launch_M<T, 4, MODE>(pl, a, nfields);
        case 8: return dst_launch_M<T, 8, MODE>(pl, a, nfields);
        case 16: return dst_launch_M<T, 16, MODE>(pl, a, nfields);
        case 32: return dst_launch_M<T, 32, MODE>(pl, a, nfields);
        case 64: return dst_launch_M<T, 64, MODE>(pl, a, nfields);
        case 128: return dst_launch_M<T, 128, MODE>(pl, a, nfields);
        case 256: return dst_launch_M<T, 256, MODE>(pl, a, nfields);
        case 512: return dst_launch_M<T, 512, MODE>(pl, a, nfields);
        case 1024: return dst_launch_M<T, 1024, MODE>(pl, a, nfields);
        case 2048: return dst_launch_M<T, 2048, MODE>(pl, a, nfields);
        case 4096: return dst_launch_M<T, 4096, MODE>(pl, a, nfields);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
DstArgs<T> dst_args(lg_plan* p) {
    DstArgs<T> a{};
    a.tw = (const cpx<T>*)p->tw;
    a.nz1 = p->nz1;
    a.ctl = p->ctl;
    a.xslot = p->xslot;
    a.r = p->r;
    a.p = (const T*)p->p;
    a.pring = p->pring;
    a.pslot = p->nvec;
    a.giter = p->giter;
    a.q = (const T*)p->qv;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.pqpart = p->partial_pq;
    a.ahist = p->ahist;
    a.pq_nparts = ((p->nx1 + 63) / 64) * ((p->nz1 + 4 * ST_RPT - 1) / (4 * ST_RPT));   // operator blocks per field
    a.y = (const T*)p->y;
    a.kap = (const T*)p->kap;
    a.wsh = (const T*)p->w;
    a.idx2 = (T)(1.0 / (p->g.dx * p->g.dx));
    a.idz2 = (T)(1.0 / (p->g.dz * p->g.dz));
    a.kap64 = (p->prec == LG_FP64) ? (const double*)p->kap : p->kap64;
    a.w64 = (p->prec == LG_FP64) ? (const double*)p->w : p->w64;
    a.free_top = p->free_top ? 1 : 0;
    a.smg = (const T*)p->sm_g;
    a.smc = p->sm_c;
    a.idx2d = 1.0 / (p->g.dx * p->g.dx);
    a.idz2d = 1.0 / (p->g.dz * p->g.dz);
    a.utab = (const T*)p->blk[0].utab;
    a.Ls = p->blk[0].Ls;
    a.P = p->blk[0].P;
    return a;
}

template <typename T, int LS>
hipError_t td_launch(lg_plan* p, TdArgs<T>& a, int nfields) {
    // segments per wave: up to 4 while the grid keeps >= 2048 blocks
    const int ktiles = (a.nx1 + 63) / 64;
    int spw = 1;
    if (p->td_spw > 0) {
        spw = p->td_spw;
    } else {
        while (spw < 4 && 4 * spw * 2 <= a.P &&
               (long)ktiles * ((a.P + 8 * spw - 1) / (8 * spw)) * nfields >= 2048)
            spw *= 2;
    }
    a.spw = spw;
    a.ktiles = ktiles;
    a.sgroups = (a.P + 4 * spw - 1) / (4 * spw);
    const dim3 grid(ktiles * a.sgroups * nfields);
    hipLaunchKernelGGL((td_kernel<T, LS>), grid, dim3(256), 0, p->stream, a);
    return hipGetLastError();
}

template <typename T>
hipError_t td_T(lg_plan* p, int bi, const T* rhat, T* y, int nfields, bool masked, int fstride,
                int foff) {
    // bi < 0: both elastic blocks in one launch, B1 on even fields, B2 on odd ones
    const PrecBlock& B = p->blk[bi < 0 ? 0 : bi];
    TdArgs<T> a;
    a.etab2 = bi < 0 ? (const T*)p->blk[1].etab : nullptr;
    a.inv_b2 = bi < 0 ? (T)(1.0 / p->blk[1].b) : (T)0;
    a.fstride = fstride;
    a.foff = foff;
    a.rhat = rhat;
    a.y = y;
    a.etab = (const T*)B.etab;
    a.E = p->E;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.P = B.P;
    a.inv_b = (T)(1.0 / B.b);
    a.ctl = masked ? p->ctl : nullptr;
    switch (B.Ls) {
        case 2: return td_launch<T, 2>(p, a, nfields);
        case 4: return td_launch<T, 4>(p, a, nfields);
        case 8: return td_launch<T, 8>(p, a, nfields);
        case 16: return td_launch<T, 16>(p, a, nfields);
        case 32: return td_launch<T, 32>(p, a, nfields);
        case 64: return td_launch<T, 64>(p, a, nfields);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t rs_T(lg_plan* p, int bi, const T* rhat, T* y, int nfields, int mode, int fstride,
                int foff) {
    // bi < 0: both elastic blocks in one launch, B1 on even fields, B2 on odd ones
    const PrecBlock& B = p->blk[bi < 0 ? 0 : bi];
    RsArgs<T> a;
    a.red2 = bi < 0 ? p->blk[1].red : nullptr;
    a.inv_b2 = bi < 0 ? 1.0 / p->blk[1].b : 0.0;
    a.fstride = fstride;
    a.foff = foff;
    a.rhat = rhat;
    a.y = y;
    a.E = p->E;
    a.red = B.red;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.P = B.P;
    a.q = B.q;
    a.Ls = B.Ls;
    a.RW = B.RW;
    a.inv_b = 1.0 / B.b;
    a.mode = mode;
    a.ctl = p->ctl;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.free_top = (p->free_top && bi == 0) ? 1 : 0;
    a.smt = p->sm_t;
    a.smc = p->sm_c;
    // 64 wavenumbers per block when the grid stays large (32 when the LDS
    // tables would pass 48 KB), else 16 (more blocks)
    auto lds_bytes = [&](int kt) {
        return ((size_t)(B.P - 1) * (kt + 1) + (size_t)kt * B.RW) * sizeof(double);
    };
    const bool wide = (long)((p->nx1 + 63) / 64) * nfields >= 1024;
    const int KT = !wide ? 16 : (lds_bytes(64) <= 48 * 1024 ? 64 : 32);
    const int nkt = (p->nx1 + KT - 1) / KT;
    const dim3 grid(nkt * nfields);
    const size_t lds = lds_bytes(KT);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), lds, p->stream, a); };
    if (KT == 64) {
        if (B.P <= 8) go(rs_kernel<T, 64, 8>);
        else if (B.P <= 16) go(rs_kernel<T, 64, 16>);
        else go(rs_kernel<T, 64, 32>);
    } else if (KT == 32) {
        go(rs_kernel<T, 32, 64>);
    } else {
        if (B.P <= 16) go(rs_kernel<T, 16, 16>);
        else go(rs_kernel<T, 16, 64>);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || mode == 0) return e;
    return finalize(p, FIN_RZ, nkt, mode, 0.0, 0, B.b * 2.0 / p->g.nx);
}

}  // namespace

hipError_t launch_finalize(lg_plan* p, int kind, int nparts, int init, double tol2, int max_iter,
                           double scale, double tol2f, double tol2r) {
    return finalize(p, kind, nparts, init, tol2, max_iter, scale, tol2f, tol2r);
}

hipError_t launch_stencil(lg_plan* p, const void* x, void* y, bool reduce_pq) {
    if (p->cyl) return cyl_launch_stencil(p, x, y, reduce_pq);
    if (p->order == 4) return ho_launch_stencil(p, x, y, reduce_pq);
    if (p->prec == LG_FP64) return stencil_T<double>(p, (const double*)x, (double*)y, reduce_pq);
    return stencil_T<float>(p, (const float*)x, (float*)y, reduce_pq);
}

hipError_t launch_dst(lg_plan* p, int inverse, const void* in, void* out, int nfields) {
    if (p->cyl) return cyl_launch_dct(p, inverse, in, out, nfields);
    if (p->prec == LG_FP64) {
        DstArgs<double> a = dst_args<double>(p);
        a.in = (const double*)in;
        a.out = (double*)out;
        return inverse ? dst_dispatch<double, DST_INV>(p, a, nfields)
                       : dst_dispatch<double, DST_FWD>(p, a, nfields);
    }
    DstArgs<float> a = dst_args<float>(p);
    a.in = (const float*)in;
    a.out = (float*)out;
    return inverse ? dst_dispatch<float, DST_INV>(p, a, nfields)
                   : dst_dispatch<float, DST_FWD>(p, a, nfields);
}

hipError_t launch_residual_check(lg_plan* p, const double* b, const double* x) {
    if (p->cyl) return cyl_launch_residual_check(p, b, x);
    if (p->order == 4) return ho_launch_residual(p, b, x);     // stores r = b - A4 x as well
    return residual_check_T(p, b, x);
}

hipError_t launch_update_fdst(lg_plan* p, int init, const double* b, double* x, double tol,
                              int max_iter) {
    hipError_t e;
    int bpf;
    if (init == 3 && p->order == 4) {   // FP64 true residual of A4 (and its check), then the pass from the stored r
        if ((e = ho_launch_residual(p, b, x)) != hipSuccess) return e;
        init = 2;
    }
    if (p->prec == LG_FP64) {
        DstArgs<double> a = dst_args<double>(p);
        a.out = (double*)p->rhat;
        a.init = init;
        a.b = b;
        a.x = x;
        a.tol2 = tol * tol;
        a.max_iter = max_iter;
        if (init >= 3)
            e = dst_dispatch<double, DST_RESTART>(p, a, p->S * p->C);
        else if (p->fuse_op && init == 0)
            e = dst_dispatch<double, DST_UPDATE_OP>(p, a, p->S * p->C);
        else if (init == 0 && fold_pq(p))
            e = dst_dispatch<double, DST_UPDATE_PQ>(p, a, p->S * p->C);
        else
            e = dst_dispatch<double, DST_UPDATE>(p, a, p->S * p->C);
        bpf = a.bpf;
    } else {
        DstArgs<float> a = dst_args<float>(p);
        a.out = (float*)p->rhat;
        a.init = init;
        a.b = b;
        a.x = x;
        a.tol2 = tol * tol;
        a.max_iter = max_iter;
        if (init >= 3)
            e = dst_dispatch<float, DST_RESTART>(p, a, p->S * p->C);
        else if (p->fuse_op && init == 0)
            e = dst_dispatch<float, DST_UPDATE_OP>(p, a, p->S * p->C);
        else if (init == 0 && fold_pq(p))
            e = dst_dispatch<float, DST_UPDATE_PQ>(p, a, p->S * p->C);
        else
            e = dst_dispatch<float, DST_UPDATE>(p, a, p->S * p->C);
        bpf = a.bpf;
    }
    if (e != hipSuccess) return e;
    // init 1: start; 4: start from a given x; 2, 3: restart from the true
    // residual (the thresholds set at the start apply).  Each phase stops at
    // phase_tol; the true residual is checked against tol.
    const double t1 = phase_tol(p, tol, false), tr = phase_tol(p, tol, true);
    return finalize(p, FIN_RR, bpf, init == 3 ? 2 : init, t1 * t1, max_iter, 0.0, tol * tol, tr * tr);
}

hipError_t launch_flush_x(lg_plan* p, double* x) {
    if (p->pring <= 1) return hipSuccess;
    const int nf = p->S * p->C;
    const int bpf = (int)((p->npts + 256 * FLUSH_EPT - 1) / (256 * FLUSH_EPT));
    const dim3 grid((unsigned)bpf * (unsigned)nf);
    if (p->prec == LG_FP64)
        hipLaunchKernelGGL(flush_x_kernel<double>, grid, dim3(256), 0, p->stream, x, (const double*)p->p, p->ahist,
                           p->ctl, p->giter, p->pring, p->nvec, p->npts, bpf);
    else
        hipLaunchKernelGGL(flush_x_kernel<float>, grid, dim3(256), 0, p->stream, x, (const float*)p->p, p->ahist,
                           p->ctl, p->giter, p->pring, p->nvec, p->npts, bpf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(flush_done_kernel, dim3((nf + 255) / 256), dim3(256), 0, p->stream, p->ctl, p->giter, nf);
    return hipGetLastError();
}

hipError_t launch_correct_idst(lg_plan* p, int init) {
    if (p->prec == LG_FP64) {
        DstArgs<double> a = dst_args<double>(p);
        a.out = (double*)p->p;
        a.init = init;
        return dst_dispatch<double, DST_CORRECT>(p, a, p->S * p->C);
    }
    DstArgs<float> a = dst_args<float>(p);
    a.out = (float*)p->p;
    a.init = init;
    return dst_dispatch<float, DST_CORRECT>(p, a, p->S * p->C);
}

// Elastic K^{-1} (P > 1): the segment correction of both blocks (field
// parity) fused into the inverse transform, z = DST^{-1} zhat; no masking and
// no search-direction update.  surface: also + coef_k g_k(j) on every row (the
// traction-free surface's rank-one term, coef_k from surface_coef_fused_kernel).
template <typename T>
hipError_t correct_inv_T(lg_plan* p, T* z, int nfields, bool surface) {
    DstArgs<T> a = dst_args<T>(p);
    a.out = z;
    a.init = 1;
    a.ctl = nullptr;
    a.utab2 = (const T*)p->blk[1].utab;
    a.free_top = surface ? 1 : 0;
    a.smg = surface ? (const T*)p->es_g[0] : nullptr;
    a.smg2 = surface ? (const T*)p->es_g[1] : nullptr;
    a.smc = p->sm_c;
    return dst_dispatch<T, DST_CORRECT>(p, a, nfields);
}

hipError_t launch_correct_inv(lg_plan* p, void* z, int nfields, bool surface) {
    if (p->prec == LG_FP64) return correct_inv_T<double>(p, (double*)z, nfields, surface);
    return correct_inv_T<float>(p, (float*)z, nfields, surface);
}

hipError_t launch_td(lg_plan* p, int blk, const void* rhat, void* y, int nfields, int masked,
                     int fstride, int foff) {
    if (p->prec == LG_FP64)
        return td_T<double>(p, blk, (const double*)rhat, (double*)y, nfields, masked != 0, fstride, foff);
    return td_T<float>(p, blk, (const float*)rhat, (float*)y, nfields, masked != 0, fstride, foff);
}

hipError_t launch_rs(lg_plan* p, int blk, const void* rhat, void* y, int nfields, int mode, int fstride,
                     int foff) {
    if (p->prec == LG_FP64)
        return rs_T<double>(p, blk, (const double*)rhat, (double*)y, nfields, mode, fstride, foff);
    return rs_T<float>(p, blk, (const float*)rhat, (float*)y, nfields, mode, fstride, foff);
}

hipError_t launch_correct(lg_plan* p, int blk, void* y, int nfields, int fstride, int foff) {
    const PrecBlock& B = p->blk[blk < 0 ? 0 : blk];
    const void* u2 = blk < 0 ? p->blk[1].utab : nullptr;     // both elastic blocks by field parity
    const size_t total = (size_t)nfields * p->npts;
    const dim3 grid((unsigned)((total + 255) / 256));
    const bool sm = p->free_top && blk == 0;
    for (int phase = 0; phase < (sm ? 2 : 1); ++phase) {
        if (p->prec == LG_FP64)
            hipLaunchKernelGGL(correct_kernel<double>, grid, dim3(256), 0, p->stream, (double*)y,
                               (const double*)B.utab, (const double*)u2, p->nx1, p->nz1, B.Ls, B.P, total, fstride,
                               foff, sm ? (const double*)p->sm_g : nullptr, p->sm_c, phase);
        else
            hipLaunchKernelGGL(correct_kernel<float>, grid, dim3(256), 0, p->stream, (float*)y,
                               (const float*)B.utab, (const float*)u2, p->nx1, p->nz1, B.Ls, B.P, total, fstride,
                               foff, sm ? (const float*)p->sm_g : nullptr, p->sm_c, phase);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_rhs(lg_plan* p, int m, const double* Rprev, double* Ph, double* Qh,
                      const double* fsrc_host, double* rhs) {
    const size_t total = p->nvec;
    const double a = p->lag.alpha;
    const double rp = (m >= 2) ? std::sqrt((m - 1.0) / (m - 1.0 + a)) : 0.0;
    const double rq = (m >= 1) ? std::sqrt(m / (m + a)) : 0.0;
    const double hh = p->lag.h * p->lag.h;
    hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, p->stream, m,
                       Rprev, Ph, Qh, p->rho64, hh, rp, rq, rhs, p->npts, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double inv = p->src_scale;
    for (int s0 = 0; s0 < p->S; s0 += SRC_CHUNK) {
        SrcArgs sa;
        sa.n = std::min(SRC_CHUNK, p->S - s0);
        for (int t = 0; t < sa.n; ++t) {
            const int s = s0 + t;
            const int i = p->src_host[2 * s], j = p->src_host[2 * s + 1];
            const int comp = p->C - 1;   // acoustic: 0; elastic: z component
            sa.idx[t] = (int64_t)(((size_t)s * p->C + comp) * p->npts + (size_t)(j - 1) * p->nx1 + (i - 1));
            // a point force on the elastic surface row acts on half a control cell
            sa.val[t] = fsrc_host[s] * inv * ((p->el_free && j == 1) ? 2.0 : 1.0);
        }
        hipLaunchKernelGGL(src_kernel, dim3(1), dim3(SRC_CHUNK), 0, p->stream, sa, rhs);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_synth(lg_plan* p, int m0, int nb, const double* const* R, const double* Wsnap, int nsnap,
                        double* snap, int rec_row, double* rec) {
    if (nb < 1 || nb > MAX_SB || nsnap > MAX_SNAP) return hipErrorInvalidValue;
    SynArgs a;
    for (int b = 0; b < MAX_SB; ++b) a.R[b] = b < nb ? R[b] : nullptr;
    a.snap = snap;
    a.rec = rec;
    for (int s = 0; s < MAX_SNAP; ++s)
        for (int b = 0; b < MAX_SB; ++b) a.W[s][b] = (s < nsnap && b < nb) ? Wsnap[(size_t)s * nb + b] : 0.0;
    a.nsnap = nsnap;
    a.m0 = m0;
    a.nb = nb;
    a.n = p->lag.n;
    a.rec_row0 = rec_row - 1;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.npts = p->npts;
    a.total = p->nvec;
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, p->stream, a);
    return hipGetLastError();
}

hipError_t launch_traces(lg_plan* p, const double* rec, const double* Wdev, int nt, double* traces) {
    dim3 grid((p->nx1 + 255) / 256, (nt + TR_Q - 1) / TR_Q, p->S * p->C);
    hipLaunchKernelGGL(traces_kernel, grid, dim3(256), 0, p->stream, rec, Wdev, p->lag.n, nt, p->nx1,
                       traces);
    return hipGetLastError();
}

}  // namespace lg
