// The paper's 2.5D axisymmetric acoustic problem (Sec. 2.1, 2.3, eqs.
// poisson_diff_2, scheme_op_r_z, diff_approx1, precond1) on gfx950.
//
// Mesh r_i = (i - 1/2) h_r, z_k = (k - 1/2) h_z.  A field holds the unknown
// rows i = 1..Nr-1 (row j = i-1) of Nz values each, z fastest; y = 0 on the
// row i = Nr.  The plan's nx1 is Nz (row length) and nz1 is Nr - 1.
//
// Operator (SPD sign): r-faces carry a1 = rbar kappa (0 on the face r = 0:
// the symmetry row), z-faces a2 = r kappa (none at the two z-ends: no flux),
// shift w = r rho h^2/4.  Preconditioner B (eq. precond1, midrange
// coefficients): the cosine transform (DCT-II) along z diagonalises the
// no-flux z-part; each z-wavenumber leaves one symmetric tridiagonal system
// along r whose coefficients vary with r.  These systems are solved by
// Thomas (one lane per system, the default) or by the Dichotomy (segments
// > 1), with the factors of every segment prepared once per plan.
//
// Kernels of one CG iteration:
//   cyl_stencil_kernel        (p, Ap) partials (q = A p stored only in the stored-q form)
//   cyl_dct_kernel<UPDATE_OP> A p recomputed, x += alpha p, r -= alpha A p, ||r||^2, rhat = DCT r
//                             (UPDATE: the stored q is read instead)
//   cyl_thomas_kernel         r-systems by Thomas, (r, z) partials (default), or
//   cyl_seg_kernel +          the Dichotomy: segments of the r-systems, then the
//   cyl_red_kernel            reduced systems over the separators, (r, z) partials
//   cyl_dct_kernel<CORRECT>   (Dichotomy: segment correction,) z = DCT^{-1} zhat, p = z + beta p
// Mixed plans keep p, q, rhat, zhat and the tables in FP32 and x, r in FP64;
// a solve that converges on the FP32 operator is restarted from the FP64
// true residual b - A x (cyl_stencil_kernel<double, true>) until that
// residual meets the tolerance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lg_device.h"
#include "lg_internal.h"

namespace lg {

// ===========================================================================
// operator
// ===========================================================================
constexpr int CY_RPT = 8;   // operator: rows per thread
constexpr int CY_TU = 8;    // r-systems: rows per load chunk

// (A p) at one node from the node value c, its r-neighbours pn (row j-1),
// ps (row j+1), z-neighbours pw, pe, the r-face coefficients fn (face
// j-1|j), fs (face j|j+1), the z-face coefficients fl, fr and the shift w.
// One chain of explicit fused multiply-adds with no free addition left for
// the compiler to contract, so every kernel that forms A p gets the same bits.
template <typename T>
__device__ __forceinline__ T cyl_point(T c, T pn, T ps, T pw, T pe, T fn, T fs, T fl, T fr, T w) {
    return fmad(fs, c - ps, fmad(fn, c - pn, fmad(fr, c - pe, fmad(fl, c - pw, w * c))));
}

template <typename T>
struct CylStArgs {
    const T* p;
    T* q;
    const T* a1;         // [nz1][nx1]: a1 / h_r^2 on the face between rows j and j+1
    const T* a2;         // [nz1][nx1+1]: a2 / h_z^2 on the face left of column k (0 at both ends)
    const T* w;          // [nz1][nx1]
    const double* b;     // residual mode: q = b - A p
    int nx1, nz1;
    int gx, gy;          // column tiles, row strips; 1D grid of gx*gy*ceil(fields/nsh) blocks
    int nfields, nsh;    // fields, fields per block (the medium stays in registers)
    ShotCtl* ctl;        // nullptr: plain application
    double* partial;
    size_t pstride;
    int pring;           // > 1 (CG): p at slot giter[0] % pring (held search directions)
    size_t pslot;        // elements per slot
    const int* giter;
};

// The waves-per-EU bound leaves the register room to keep every load of a
// shot in flight at once (without it the scheduler sinks each load to its use
// behind a full vmcnt(0) wait, which halves the kernel's bandwidth).
template <typename T, bool RES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 4 ? 4 : 2))) void
cyl_stencil_kernel(CylStArgs<T> a) {
    constexpr int MAXSH = 64;                   // fields per block at most (op_shots)
    __shared__ double red[MAXSH][4];
    __shared__ int act[MAXSH];
    const int nx1 = a.nx1, nz1 = a.nz1;
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int L = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = L % a.gx, by = (L / a.gx) % a.gy, grp = L / (a.gx * a.gy);
    // residual mode with a reduction: ||b - A x||^2 of every shot (the check
    // before a restart covers the shots that have stopped); otherwise a block
    // whose shots have all stopped leaves before loading the medium
    const int f0 = grp * a.nsh, ns = min(a.nsh, a.nfields - f0);
    int mine = 0;
    if (threadIdx.x < ns) {
        act[threadIdx.x] = (a.ctl != nullptr && !RES) ? a.ctl[f0 + threadIdx.x].active : 1;
        mine = act[threadIdx.x];
    }
    if (__syncthreads_or(mine != 0) == 0) return;   // (also the barrier for act) uniform per block
    const int k = bx * 64 + lane;
    const int j0 = (by * 4 + ty) * CY_RPT;
    const bool live = k < nx1;
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nf = (uint32_t)nx1 * (uint32_t)nz1;
    const rsrc_t r1 = buf_rsrc(a.a1, nf * SZ);
    const rsrc_t r2 = buf_rsrc(a.a2, (uint32_t)nz1 * (uint32_t)(nx1 + 1) * SZ);
    const rsrc_t rw = buf_rsrc(a.w, nf * SZ);
    // offsets of the strip's rows j0-1 .. j0+RPT (0 outside: the r = 0 face has
    // no coefficient, the row past the last unknown is the Dirichlet side) and
    // of the E/W neighbours (none past the z-ends)
    uint32_t oc[CY_RPT + 2], oe[CY_RPT], ow[CY_RPT];
#pragma unroll
    for (int r = 0; r < CY_RPT + 2; ++r) {
        const int j = j0 - 1 + r;
        oc[r] = (live && j >= 0 && j < nz1) ? (uint32_t)(j * nx1 + k) * SZ : BUF_OOB;
    }
#pragma unroll
    for (int r = 0; r < CY_RPT; ++r) {
        const uint32_t c = oc[r + 1];
        oe[r] = (c != BUF_OOB && k + 1 < nx1) ? c + SZ : BUF_OOB;
        ow[r] = (c != BUF_OOB && k > 0) ? c - SZ : BUF_OOB;
    }
    // medium of the tile, shared by the block's fields
    T f1[CY_RPT + 1], fl[CY_RPT], fr[CY_RPT], wv[CY_RPT];
#pragma unroll
    for (int r = 0; r < CY_RPT + 1; ++r) f1[r] = bload<T>(r1, oc[r]);    // faces j0-1|j0 .. j0+RPT-1|j0+RPT
#pragma unroll
    for (int r = 0; r < CY_RPT; ++r) {
        const int j = j0 + r;
        const bool ok = live && j < nz1;
        const uint32_t e2 = (uint32_t)(j * (nx1 + 1) + k);
        fl[r] = bload<T>(r2, ok ? e2 * SZ : BUF_OOB);
        fr[r] = bload<T>(r2, ok ? (e2 + 1) * SZ : BUF_OOB);
        wv[r] = bload<T>(rw, oc[r + 1]);
    }
    // held directions: this iteration's p slot (one count for every shot)
    const size_t ps = (!RES && a.pring > 1) ? (size_t)(*a.giter % a.pring) * a.pslot : 0;
    // per field: loads, A p, store, per-wave (p, Ap); one barrier at the end
    for (int kf = 0; kf < ns; ++kf) {
        if (act[kf] == 0) continue;                 // uniform per block
        const size_t fo = (size_t)(f0 + kf) * nf;
        const rsrc_t rp = buf_rsrc(a.p + ps + fo, nf * SZ);
        T pv[CY_RPT + 2], pe[CY_RPT], pw[CY_RPT];
#pragma unroll
        for (int r = 0; r < CY_RPT + 2; ++r) pv[r] = bload<T>(rp, oc[r]);
#pragma unroll
        for (int r = 0; r < CY_RPT; ++r) {
            pe[r] = bload<T>(rp, oe[r]);
            pw[r] = bload<T>(rp, ow[r]);
        }
        double pq = 0.0;
        const rsrc_t rq = buf_rsrc((a.q != nullptr ? a.q : const_cast<T*>(a.p)) + fo,
                                   a.q != nullptr ? nf * SZ : 0u);
        const rsrc_t rb = buf_rsrc(a.b + fo, RES ? nf * 8u : 0u);
#pragma unroll
        for (int r = 0; r < CY_RPT; ++r) {
            const T c = pv[r + 1];
            T v = cyl_point<T>(c, pv[r], pv[r + 2], pw[r], pe[r], f1[r], f1[r + 1], fl[r], fr[r], wv[r]);
            if constexpr (RES) {
                v = (T)(bload<double>(rb, oc[r + 1] == BUF_OOB ? BUF_OOB : oc[r + 1] / SZ * 8u) - (double)v);
                if (oc[r + 1] != BUF_OOB) pq += (double)v * (double)v;     // rows past the grid: none
            } else {
                pq += (double)c * (double)v;
            }
            bstore<T>(v, rq, oc[r + 1]);
        }
        if (a.ctl == nullptr) continue;
        pq = wave_sum(pq);
        if (lane == 0) red[kf][ty] = pq;
    }
    if (a.ctl == nullptr) return;
    __syncthreads();
    if (threadIdx.x < ns && act[threadIdx.x] != 0) {
        const int kf = threadIdx.x;
        a.partial[(size_t)(f0 + kf) * a.pstride + by * a.gx + bx] = ((red[kf][0] + red[kf][1]) + red[kf][2]) + red[kf][3];
    }
}

// ===========================================================================
// cosine transform along z (rows).  Two rows (j0, j1) are packed as one
// complex sequence of length Nz, extended half-sample symmetrically to
// M = 2 Nz; with V its DFT, exp(-i pi k / M) V_k / 2 = C_k(j0) + i C_k(j1)
// (C_k = sum_n x_n cos(pi k (2n+1) / M)).  The inverse x_n = C_0/Nz +
// (2/Nz) sum_{k>0} C_k cos(pi k (2n+1) / M) of a packed pair is the
// conjugate of the DFT of conj(U), U_k = D_k e^{i pi k/M}/Nz,
// U_{M-k} = D_k e^{-i pi k/M}/Nz (k > 0), U_0 = D_0/Nz, U_{Nz} = 0.
// ===========================================================================
// CY_UPDATE_OP: the update recomputes q = A p for its two rows from p and the
// face tables (the operator kernel then only forms (p, Ap)).
// CY_INV_D / CY_CORRECT_D: the same with the r-system Dichotomy correction
// applied to the input rows first.
enum CylMode { CY_FWD = 0, CY_INV = 1, CY_UPDATE = 2, CY_CORRECT = 3, CY_UPDATE_OP = 4, CY_INV_D = 5, CY_CORRECT_D = 6 };

template <typename T>
struct CylDctArgs {
    const T* in;
    T* out;
    const cpx<T>* tw;      // exp(-2 pi i j / M)
    const cpx<T>* ctw;     // exp(-i pi k / M), k < Nz
    int nz1;
    int bpf;
    ShotCtl* ctl;
    double* x;
    double** xslot;
    double* r;
    const double* b;
    const T* p;
    const T* q;
    const T* a1;           // CY_UPDATE_OP: face tables and shift
    const T* a2;
    const T* w;
    const cpx<T>* UV;      // CY_*_D: Dichotomy correction of the input rows
    int Ls, P;
    double* partial;
    size_t pstride;
    int init;
    int pring;             // > 1: held directions, p of iteration g at slot g % pring; x not touched
    size_t pslot;          // elements per slot
    const int* giter;      // [0] the solve's iteration count g
};

template <typename T, int M, int R, int FPB, int MODE>
__global__ __launch_bounds__(FPB*(M / R)) void cyl_dct_kernel(CylDctArgs<T> a) {
    using FP = FftPlan<M, R>;
    constexpr int TPF = M / R;
    constexpr int N = M / 2;                   // row length Nz
    constexpr int RL = FP::R_LAST, NBL = FP::NB_LAST, NSL = FP::NS_LAST;
    constexpr int NOUT = NBL * (RL / 2);
    constexpr int LL = LdsLen<M>::value;
    constexpr int NWAVE = (FPB * TPF + 63) / 64;
    constexpr int NIT = (N + TPF - 1) / TPF;
    constexpr bool CORRM = MODE == CY_CORRECT || MODE == CY_CORRECT_D;    // p = z + beta p
    constexpr bool DCH = MODE == CY_INV_D || MODE == CY_CORRECT_D;        // Dichotomy correction
    constexpr bool INVERSE = MODE == CY_INV || MODE == CY_INV_D || CORRM;
    constexpr bool UPD = MODE == CY_UPDATE || MODE == CY_UPDATE_OP;
    __shared__ cpx<T> lds[FPB * LL];
    __shared__ double red[NWAVE];

    const int fid = threadIdx.x / TPF;
    const int t = threadIdx.x - fid * TPF;
    const int field = blockIdx.x / a.bpf;
    const int bif = blockIdx.x - field * a.bpf;
    const int pair = bif * FPB + fid;
    const int npairs = (a.nz1 + 1) >> 1;
    const bool live = pair < npairs;
    const int j0 = 2 * pair, j1 = j0 + 1;
    const bool has1 = live && (j1 < a.nz1);
    if constexpr (UPD || CORRM) {
        if (!a.init && a.ctl[field].active == 0) return;   // uniform per block
    }
    // held directions: the solve's iteration count (the update of iteration g
    // reads p_g; the correction after it reads p_g and writes p_{g+1}; a start
    // or restart writes the first direction at g)
    const int kit = ((UPD || CORRM) && a.pring > 1) ? *a.giter : 0;
    cpx<T>* buf = lds + fid * LL;
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nfe = (uint32_t)a.nz1 * (uint32_t)N;
    const size_t fbase = (size_t)field * nfe;
    double rr = 0.0;
    T pold0[CORRM ? NOUT : 1], pold1[CORRM ? NOUT : 1];

    if (live) {
        if constexpr (!INVERSE) {
            // rows of the input (or, UPDATE, the updated residual) -> symmetric extension
            T v0[NIT], v1[NIT];
            if constexpr (UPD) {
                // init 0: x += alpha p, r -= alpha q; 1 (cold start): only the
                // transform of b and ||b||^2, x = 0 and r = b are not stored: the
                // shot's first update (ShotCtl.fresh) reads b for r, takes x as 0
                // and writes both; 2: r as stored (x untouched)
                const int init = a.init;
                bool fresh = false;
                const double* B0 = nullptr;
                if (init == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
                    a.xslot[0] = a.x;
                    a.xslot[1] = const_cast<double*>(a.b);
                }
                if (init == 0) {
                    fresh = a.ctl[field].fresh != 0;                   // uniform per block
                    if (fresh) B0 = wave_uniform(a.xslot[1]);
                }
                double* const X = wave_uniform(init ? a.x : a.xslot[0]);
                const double alpha = init ? 0.0 : a.ctl[field].alpha;
                // held directions: x is neither read nor written (the flush pass
                // adds alpha_g p_g later)
                const bool xin = a.pring == 1;
                const rsrc_t rX = buf_rsrc(X + fbase, (init == 0 && !fresh && xin) ? nfe * 8u : 0u);
                const rsrc_t rXs = buf_rsrc(X + fbase, (init == 0 && xin) ? nfe * 8u : 0u);
                const rsrc_t rR = buf_rsrc(
                    wave_uniform(init == 1 ? a.b + fbase : (B0 != nullptr ? B0 + fbase : a.r + fbase)), nfe * 8u);
                const rsrc_t rRs = buf_rsrc(a.r + fbase, init == 0 ? nfe * 8u : 0u);
                const size_t pofs = (init == 0 && a.pring > 1) ? (size_t)(kit % a.pring) * a.pslot : 0;
                const rsrc_t rP = buf_rsrc(a.p + pofs + fbase, init ? 0u : nfe * SZ);
                const rsrc_t rQ = buf_rsrc(a.q + fbase, (init || MODE == CY_UPDATE_OP) ? 0u : nfe * SZ);
                const rsrc_t rA1 = buf_rsrc(a.a1, MODE == CY_UPDATE_OP ? nfe * SZ : 0u);
                const rsrc_t rA2 = buf_rsrc(a.a2, MODE == CY_UPDATE_OP ? (uint32_t)a.nz1 * (N + 1) * SZ : 0u);
                const rsrc_t rW = buf_rsrc(a.w, MODE == CY_UPDATE_OP ? nfe * SZ : 0u);
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const int n = t + it * TPF;
                    const bool in = n < N;
                    const uint32_t e0 = in ? (uint32_t)(j0 * N + n) : BUF_OOB / 8u;
                    const uint32_t e1 = (in && has1) ? (uint32_t)(j1 * N + n) : BUF_OOB / 8u;
                    const double x0 = bload<double>(rX, e0 * 8u), x1 = bload<double>(rX, e1 * 8u);
                    const double r0 = bload<double>(rR, e0 * 8u), r1 = bload<double>(rR, e1 * 8u);
                    const T p0 = bload<T>(rP, e0 * SZ), p1 = bload<T>(rP, e1 * SZ);
                    T q0, q1;
                    if constexpr (MODE == CY_UPDATE_OP) {
                        // q = A p for rows j0, j1 from p rows j0-1 .. j1+1 (0 outside: no
                        // face at r = 0, Dirichlet row past the last unknown, no z-end flux)
                        const int jm = j0 - 1, jp = j1 + 1;
                        const bool w0 = in && n > 0, e0ok = in && n + 1 < N;
                        const T pn0 = bload<T>(rP, (in && jm >= 0) ? (uint32_t)(jm * N + n) * SZ : BUF_OOB);
                        const T ps1 = bload<T>(rP, (in && has1 && jp < a.nz1) ? (uint32_t)(jp * N + n) * SZ : BUF_OOB);
                        const T pw0 = bload<T>(rP, w0 ? (e0 - 1) * SZ : BUF_OOB);
                        const T pe0 = bload<T>(rP, e0ok ? (e0 + 1) * SZ : BUF_OOB);
                        const T pw1 = bload<T>(rP, (w0 && has1) ? (e1 - 1) * SZ : BUF_OOB);
                        const T pe1 = bload<T>(rP, (e0ok && has1) ? (e1 + 1) * SZ : BUF_OOB);
                        const T fn0 = bload<T>(rA1, (in && jm >= 0) ? (uint32_t)(jm * N + n) * SZ : BUF_OOB);
                        const T fs0 = bload<T>(rA1, e0 * SZ);
                        const T fs1 = bload<T>(rA1, e1 * SZ);
                        const uint32_t g0 = in ? (uint32_t)(j0 * (N + 1) + n) : BUF_OOB / 8u;
                        const uint32_t g1 = (in && has1) ? (uint32_t)(j1 * (N + 1) + n) : BUF_OOB / 8u;
                        const T fl0 = bload<T>(rA2, g0 * SZ), fr0 = bload<T>(rA2, (g0 + 1) * SZ);
                        const T fl1 = bload<T>(rA2, g1 * SZ), fr1 = bload<T>(rA2, (g1 + 1) * SZ);
                        const T wv0 = bload<T>(rW, e0 * SZ), wv1 = bload<T>(rW, e1 * SZ);
                        q0 = cyl_point<T>(p0, pn0, p1, pw0, pe0, fn0, fs0, fl0, fr0, wv0);
                        // no second row in the last pair (N_r - 1 is odd): q1 must be 0, or
                        // the phantom row's -alpha q1 would enter ||r||^2 and the transform
                        q1 = has1 ? cyl_point<T>(p1, p0, ps1, pw1, pe1, fs0, fs1, fl1, fr1, wv1) : (T)0;
                    } else {
                        q0 = bload<T>(rQ, e0 * SZ);
                        q1 = bload<T>(rQ, e1 * SZ);
                    }
                    const double ra = r0 - alpha * (double)q0, rb = r1 - alpha * (double)q1;
                    bstore<double>(x0 + alpha * (double)p0, rXs, e0 * 8u);
                    bstore<double>(x1 + alpha * (double)p1, rXs, e1 * 8u);
                    bstore<double>(ra, rRs, e0 * 8u);
                    bstore<double>(rb, rRs, e1 * 8u);
                    rr += ra * ra + rb * rb;
                    v0[it] = (T)ra;
                    v1[it] = (T)rb;
                }
            } else {
                const rsrc_t rI = buf_rsrc(a.in + fbase, nfe * SZ);
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const int n = t + it * TPF;
                    const bool in = n < N;
                    v0[it] = bload<T>(rI, in ? (uint32_t)(j0 * N + n) * SZ : BUF_OOB);
                    v1[it] = bload<T>(rI, (in && has1) ? (uint32_t)(j1 * N + n) * SZ : BUF_OOB);
                }
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int n = t + it * TPF;
                if (n < N) {
                    buf[lpad(n)] = {v0[it], v1[it]};
                    buf[lpad(M - 1 - n)] = {v0[it], v1[it]};
                }
            }
        } else {
            // spectral rows D_k -> conj(U) at k and M-k
            const rsrc_t rI = buf_rsrc(a.in + fbase, nfe * SZ);
            const T inv_n = (T)(1.0 / N);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int k = t + it * TPF;
                const bool in = k < N;
                T d0 = bload<T>(rI, in ? (uint32_t)(j0 * N + k) * SZ : BUF_OOB);
                T d1 = bload<T>(rI, (in && has1) ? (uint32_t)(j1 * N + k) * SZ : BUF_OOB);
                if constexpr (DCH) {   // Dichotomy correction: y + x_{c_{s-1}} U + x_{c_s} V
                    // j0 is even and separators are odd, so j1 lies in j0's segment or is
                    // its separator (U = V = 0 there): one pair of separator values serves both
                    const rsrc_t rUV = buf_rsrc(a.UV, nfe * 2 * SZ);
                    const int sg = j0 / a.Ls;
                    const T xl = bload<T>(rI, (in && sg > 0) ? (uint32_t)((sg * a.Ls - 1) * N + k) * SZ : BUF_OOB);
                    const T xr = bload<T>(rI, (in && sg < a.P - 1) ? (uint32_t)((sg * a.Ls + a.Ls - 1) * N + k) * SZ
                                                                  : BUF_OOB);
                    const cpx<T> uv0 = bload2<T>(rUV, in ? (uint32_t)(j0 * N + k) * 2 * SZ : BUF_OOB);
                    const cpx<T> uv1 = bload2<T>(rUV, (in && has1) ? (uint32_t)(j1 * N + k) * 2 * SZ : BUF_OOB);
                    d0 = fmad(xr, uv0.y, fmad(xl, uv0.x, d0));
                    d1 = fmad(xr, uv1.y, fmad(xl, uv1.x, d1));
                }
                if (in) {
                    const cpx<T> cd = {d0 * inv_n, -d1 * inv_n};         // conj(D) / Nz
                    if (k == 0) {
                        buf[lpad(0)] = cd;
                    } else {
                        const cpx<T> e = a.ctw[k];                          // exp(-i pi k / M)
                        buf[lpad(k)] = cmul(cd, e);
                        buf[lpad(M - k)] = cmul(cd, cpx<T>{e.x, -e.y});
                    }
                }
            }
            if (t == 0) buf[lpad(N)] = {(T)0, (T)0};
            if constexpr (CORRM) {
                const size_t rofs = (!a.init && a.pring > 1) ? (size_t)((kit + a.pring - 1) % a.pring) * a.pslot : 0;
                const rsrc_t rPo = buf_rsrc(a.out + rofs + fbase, a.init ? 0u : nfe * SZ);
#pragma unroll
                for (int qb = 0; qb < NBL; ++qb)
#pragma unroll
                    for (int u = 0; u < RL / 2; ++u) {
                        const int K = t + qb * TPF + u * NSL;
                        const int oi = qb * (RL / 2) + u;
                        pold0[oi] = bload<T>(rPo, (uint32_t)(j0 * N + K) * SZ);
                        pold1[oi] = bload<T>(rPo, has1 ? (uint32_t)(j1 * N + K) * SZ : BUF_OOB);
                    }
            }
        }
    } else {
        for (int i = t; i < M; i += TPF) buf[lpad(i)] = {(T)0, (T)0};
    }
    __syncthreads();

    cpx<T> v[R];
    fft_mid<T, M, R, 1>(buf, a.tw, t);
    fft_last<T, M, R>(buf, a.tw, t, v);

    if (live) {
        T beta = (T)0;
        if constexpr (CORRM) beta = (T)a.ctl[field].beta;
        // CORRECT with held directions: the new direction goes to slot g % pring
        T* const outp = a.out + ((CORRM && a.pring > 1) ? (size_t)(kit % a.pring) * a.pslot : 0);
        const size_t o0 = fbase + (size_t)j0 * N, o1 = fbase + (size_t)j1 * N;
#pragma unroll
        for (int qb = 0; qb < NBL; ++qb)
#pragma unroll
            for (int u = 0; u < RL / 2; ++u) {
                const int K = t + qb * TPF + u * NSL;       // 0 <= K < Nz
                const cpx<T> V = v[qb * RL + u];
                T x0, x1;
                if constexpr (!INVERSE) {
                    const cpx<T> c = cmul(a.ctw[K], V);
                    x0 = c.x * (T)0.5;
                    x1 = c.y * (T)0.5;
                } else {
                    x0 = V.x;
                    x1 = -V.y;
                }
                if constexpr (CORRM) {
                    const int oi = qb * (RL / 2) + u;
                    if (!a.init) {
                        x0 += beta * pold0[oi];
                        x1 += beta * pold1[oi];
                    }
                }
                outp[o0 + K] = x0;
                if (has1) outp[o1 + K] = x1;
            }
    }
    if constexpr (UPD) {
        const double s = block_sum(rr, red);
        if (threadIdx.x == 0) a.partial[(size_t)field * a.pstride + bif] = s;
    }
}

// ===========================================================================
// r-systems by Thomas (one segment, the default): one lane per (wavenumber,
// field); the forward sweep stores its intermediate values, back
// substitution overwrites them.  (rhat, zhat) is accumulated in the forward
// sweep from the LDL^T form (sum g_i dp_i) and weighted by the transform's
// inverse weights (1/Nz for k = 0, else 2/Nz).  Rows are taken in chunks of
// CY_TU whose loads are all issued before the chunk's recurrence steps.
// ===========================================================================
template <typename T>
struct CylTdArgs {
    const T* rhat;
    T* z;
    const T* cp;         // [nz1][nx1] upper factors
    const T* invden;     // [nz1][nx1] inverse pivots
    const T* lowr;       // [nz1] coupling to the previous row (0 for the first)
    int nx1, nz1;
    ShotCtl* ctl;        // mode != 0: masked, partials
    double* partial;
    size_t pstride;
    int mode;
};

template <typename T>
__global__ __launch_bounds__(256) void cyl_thomas_kernel(CylTdArgs<T> a) {
    // Rows are taken in chunks of CY_TU: the loads of a chunk do not depend
    // on the recurrence, so they are all issued before its first step.  Rows
    // past either end load as 0 (buffer range check) and leave the recurrence
    // values 0; their stores are dropped.
    constexpr int U = CY_TU;
    __shared__ double red[4];
    const int nx1 = a.nx1, nz1 = a.nz1;
    const int field = blockIdx.y;
    if (a.mode != 0 && a.ctl[field].active == 0) return;    // uniform per block
    const int k = blockIdx.x * 256 + threadIdx.x;
    const bool live = k < nx1;
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nf = (uint32_t)nx1 * (uint32_t)nz1;
    const size_t fo = (size_t)field * nf;
    const rsrc_t rR = buf_rsrc(a.rhat + fo, nf * SZ);
    const rsrc_t rZ = buf_rsrc(a.z + fo, nf * SZ);
    const rsrc_t rC = buf_rsrc(a.cp, nf * SZ);
    const rsrc_t rI = buf_rsrc(a.invden, nf * SZ);
    const rsrc_t rL = buf_rsrc(a.lowr, (uint32_t)nz1 * SZ);
    auto off = [&](int j) -> uint32_t {
        return (live && j >= 0 && j < nz1) ? (uint32_t)(j * nx1 + k) * SZ : BUF_OOB;
    };
    double acc = 0.0;
    T dp = (T)0;
    for (int j0 = 0; j0 < nz1; j0 += U) {
        T rv[U], iv[U], lv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u;
            rv[u] = bload<T>(rR, off(j));
            iv[u] = bload<T>(rI, off(j));
            lv[u] = bload<T>(rL, j < nz1 ? (uint32_t)j * SZ : BUF_OOB);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T g = rv[u] - lv[u] * dp;
            dp = g * iv[u];
            acc += (double)g * (double)dp;
            bstore<T>(dp, rZ, off(j0 + u));
        }
    }
    T xn = (T)0;
    for (int jt = nz1 - 1; jt >= 0; jt -= U) {
        T zv[U], cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            zv[u] = bload<T>(rZ, off(jt - u));
            cv[u] = bload<T>(rC, off(jt - u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xn = zv[u] - cv[u] * xn;
            bstore<T>(xn, rZ, off(jt - u));
        }
    }
    if (a.mode == 0) return;
    acc = live ? acc * ((k == 0) ? 1.0 / nx1 : 2.0 / nx1) : 0.0;
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.partial[(size_t)field * a.pstride + blockIdx.x] = s;
}

// ===========================================================================
// r-systems by the Dichotomy (Sec. 1; eq. precond1 in the axisymmetric form).
// Every wavenumber's system is split into P segments of Ls-1 rows, separated
// by the rows c_s = s Ls + Ls - 1.  The coefficients vary with r, so every
// segment has factors of its own (prepared once per plan, shared by every
// shot and iteration):
//   1. cyl_seg_kernel: each lane solves one (wavenumber, segment) with zero
//      separator values, its rows held in registers; it stores y, the two
//      end values and the local (r, T_s^{-1} r) (LDL^T form, sum g dp);
//   2. cyl_red_kernel: per (shot, wavenumber) the reduced (Schur) tridiagonal
//      system over the separators, serial Thomas with prepared factors; the
//      separator values go into the separator rows of the solution, and
//      (rhat, zhat) = sum of the local terms + G^T x (the reduced LDL^T sum);
//   3. the correction x_j = y_j + x_{c_{s-1}} U_j + x_{c_s} V_j (U, V: the
//      segment's responses to unit separator values, 0 on separator rows),
//      fused into the inverse cosine transform, or cyl_corr_kernel.
// ===========================================================================
template <typename T>
struct CylSegArgs {
    const T* rhat;
    T* y;
    const T* cp;         // [nz1][nx1] segment-local upper factors
    const T* inv;        // [nz1][nx1] segment-local inverse pivots
    const T* lowr;       // [nz1] coupling to the previous row
    double* E;           // [fields][P][3][nx1]: y(first row), y(last row), local (r, T_s^{-1} r)
    int nx1, nz1, P;
    int segtiles;        // ceil(P / 4)
    ShotCtl* ctl;        // masked: skip inactive shots
    int masked;
};

template <typename T, int LS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 4 ? 4 : 2))) void
cyl_seg_kernel(CylSegArgs<T> a) {
    constexpr int L = LS - 1;
    const int field = blockIdx.y;
    if (a.masked && a.ctl[field].active == 0) return;        // uniform per block
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int kt = blockIdx.x / a.segtiles, sg = (blockIdx.x - kt * a.segtiles) * 4 + ty;
    const int k = kt * 64 + lane;
    const bool live = k < a.nx1 && sg < a.P;
    const int nx1 = a.nx1;
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nf = (uint32_t)nx1 * (uint32_t)a.nz1;
    const rsrc_t rR = buf_rsrc(a.rhat + (size_t)field * nf, nf * SZ);
    const rsrc_t rY = buf_rsrc(a.y + (size_t)field * nf, nf * SZ);
    const rsrc_t rC = buf_rsrc(a.cp, nf * SZ);
    const rsrc_t rI = buf_rsrc(a.inv, nf * SZ);
    const rsrc_t rL = buf_rsrc(a.lowr, (uint32_t)a.nz1 * SZ);
    const int row0 = sg * LS;
    auto off = [&](int i) -> uint32_t { return live ? (uint32_t)((row0 + i) * nx1 + k) * SZ : BUF_OOB; };
    T dp[L];
    double acc = 0.0;
    T prev = (T)0;
#pragma unroll
    for (int i0 = 0; i0 < L; i0 += 8) {
        T rv[8], iv[8], lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (i0 + u < L) {
                rv[u] = bload<T>(rR, off(i0 + u));
                iv[u] = bload<T>(rI, off(i0 + u));
                lv[u] = bload<T>(rL, live ? (uint32_t)(row0 + i0 + u) * SZ : BUF_OOB);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (i0 + u < L) {
                const T g = (i0 + u == 0) ? rv[u] : rv[u] - lv[u] * prev;
                prev = g * iv[u];
                dp[i0 + u] = prev;
                acc += (double)g * (double)prev;
            }
        }
    }
    T x = dp[L - 1];
    bstore<T>(x, rY, off(L - 1));
    const T ylast = x;
#pragma unroll
    for (int i0 = L - 2; i0 >= 0; i0 -= 8) {
        T cv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 - u >= 0) cv[u] = bload<T>(rC, off(i0 - u));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (i0 - u >= 0) {
                x = dp[i0 - u] - cv[u] * x;
                bstore<T>(x, rY, off(i0 - u));
            }
        }
    }
    if (!live) return;
    double* e = a.E + ((size_t)field * a.P + sg) * 3 * nx1 + k;
    e[0] = (double)x;
    e[nx1] = (double)ylast;
    e[2 * (size_t)nx1] = acc;
}

template <typename T>
struct CylRedArgs {
    const T* rhat;
    T* y;                // separator rows receive the separator values
    const double* E;
    const double* cpl;   // [2][nz1]: couplings to rows j-1, j+1
    const double* red;   // [nx1][P-1][3]
    int nx1, nz1, Ls;
    ShotCtl* ctl;        // mode != 0: masked, partials
    double* partial;
    size_t pstride;
    int mode;
};

template <typename T, int P>
__global__ __launch_bounds__(256) void cyl_red_kernel(CylRedArgs<T> a) {
    __shared__ double redsum[4];
    const int nx1 = a.nx1, field = blockIdx.y;
    if (a.mode != 0 && a.ctl[field].active == 0) return;      // uniform per block
    const int k = blockIdx.x * 256 + threadIdx.x;
    const bool live = k < nx1;
    const int kc = min(k, nx1 - 1);
    const size_t fo = (size_t)field * nx1 * a.nz1;
    const double* E = a.E + (size_t)field * P * 3 * nx1 + kc;
    double acc = 0.0;
#pragma unroll
    for (int sg = 0; sg < P; ++sg) acc += E[(3 * sg + 2) * (size_t)nx1];
    if constexpr (P > 1) {
        const double* rw = a.red + (size_t)kc * 3 * (P - 1);
        double dpr[P - 1];
        double prev = 0.0;
#pragma unroll
        for (int c = 0; c < P - 1; ++c) {
            const int row = c * a.Ls + a.Ls - 1;
            const double G = (double)a.rhat[fo + (size_t)row * nx1 + kc] - a.cpl[row] * E[(3 * c + 1) * (size_t)nx1] -
                             a.cpl[a.nz1 + row] * E[(3 * (c + 1)) * (size_t)nx1];
            const double g = G - rw[3 * c] * prev;
            prev = g * rw[3 * c + 2];
            dpr[c] = prev;
            acc += g * prev;
        }
        double x = dpr[P - 2];
        if (live) a.y[fo + (size_t)((P - 1) * a.Ls - 1) * nx1 + kc] = (T)x;
#pragma unroll
        for (int c = P - 3; c >= 0; --c) {
            x = dpr[c] - rw[3 * c + 1] * x;
            if (live) a.y[fo + (size_t)(c * a.Ls + a.Ls - 1) * nx1 + kc] = (T)x;
        }
    }
    if (a.mode == 0) return;
    acc = live ? acc * ((k == 0) ? 1.0 / nx1 : 2.0 / nx1) : 0.0;
    const double sblk = block_sum(acc, redsum);
    if (threadIdx.x == 0) a.partial[(size_t)field * a.pstride + blockIdx.x] = sblk;
}

// z = y + x_{c_{s-1}} U + x_{c_s} V in place (the plain r-system call)
template <typename T>
__global__ __launch_bounds__(256) void cyl_corr_kernel(T* z, const cpx<T>* UV, int nx1, int nz1, int Ls, int P) {
    const size_t nf = (size_t)nx1 * nz1;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int field = blockIdx.y;
    if (e >= nf) return;
    const int j = (int)(e / nx1), k = (int)(e - (size_t)j * nx1);
    const int sg = j / Ls;
    if (j - sg * Ls == Ls - 1) return;                 // separator rows already hold their values
    T* zf = z + (size_t)field * nf;
    const T xl = sg > 0 ? zf[(size_t)(sg * Ls - 1) * nx1 + k] : (T)0;
    const T xr = sg < P - 1 ? zf[(size_t)(sg * Ls + Ls - 1) * nx1 + k] : (T)0;
    zf[e] = fmad(xr, UV[e].y, fmad(xl, UV[e].x, zf[e]));
}

// ===========================================================================
// launchers
// ===========================================================================
namespace {

template <typename T, bool RES>
hipError_t cyl_stencil_T(lg_plan* p, const T* x, T* y, bool reduce, int nfields, const T* a1, const T* a2,
                         const T* w, const double* b) {
    CylStArgs<T> a;
    a.p = x;
    a.q = y;
    a.a1 = a1;
    a.a2 = a2;
    a.w = w;
    a.b = b;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.gx = (p->nx1 + 63) / 64;
    a.gy = (p->nz1 + 4 * CY_RPT - 1) / (4 * CY_RPT);
    a.nfields = nfields;
    a.nsh = std::max(1, std::min(nfields, p->op_shots));
    a.ctl = reduce ? p->ctl : nullptr;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.pring = (reduce && !RES) ? p->pring : 1;
    a.pslot = p->nvec;
    a.giter = p->giter;
    const int groups = (nfields + a.nsh - 1) / a.nsh;
    hipLaunchKernelGGL((cyl_stencil_kernel<T, RES>), dim3(a.gx * a.gy * groups), dim3(256), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !reduce) return e;
    // residual mode: the restart check on ||b - A x||^2; else (p, Ap)
    return RES ? launch_finalize(p, 1 /* ||r||^2 */, a.gx * a.gy, 2, 0.0, 0, 0.0)
               : launch_finalize(p, 0 /* (p, Ap) */, a.gx * a.gy, 0, 0.0, 0, 0.0);
}

template <typename T, int M, int MODE>
hipError_t cyl_dct_M(lg_plan* pl, CylDctArgs<T>& a, int nfields) {
    constexpr int R = M >= 16 ? 16 : M;
    constexpr int TPF = M / R;
    constexpr int FPB = TPF >= 256 ? 1 : 256 / TPF;
    const int npairs = (a.nz1 + 1) / 2;
    a.bpf = (npairs + FPB - 1) / FPB;
    hipLaunchKernelGGL((cyl_dct_kernel<T, M, R, FPB, MODE>), dim3(a.bpf * nfields), dim3(FPB * TPF), 0,
                       pl->stream, a);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t cyl_dct_dispatch(lg_plan* pl, CylDctArgs<T>& a, int nfields) {
    switch (2 * pl->nx1) {
        case 4: return cyl_dct_M<T, 4, MODE>(pl, a, nfields);
        case 8: return cyl_dct_M<T, 8, MODE>(pl, a, nfields);
        case 16: return cyl_dct_M<T, 16, MODE>(pl, a, nfields);
        case 32: return cyl_dct_M<T, 32, MODE>(pl, a, nfields);
        case 64: return cyl_dct_M<T, 64, MODE>(pl, a, nfields);
        case 128: return cyl_dct_M<T, 128, MODE>(pl, a, nfields);
        case 256: return cyl_dct_M<T, 256, MODE>(pl, a, nfields);
        case 512: return cyl_dct_M<T, 512, MODE>(pl, a, nfields);
        case 1024: return cyl_dct_M<T, 1024, MODE>(pl, a, nfields);
        case 2048: return cyl_dct_M<T, 2048, MODE>(pl, a, nfields);
        case 4096: return cyl_dct_M<T, 4096, MODE>(pl, a, nfields);
        case 8192: return cyl_dct_M<T, 8192, MODE>(pl, a, nfields);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
CylDctArgs<T> cyl_dct_args(lg_plan* p) {
    CylDctArgs<T> a{};
    a.tw = (const cpx<T>*)p->tw;
    a.ctw = (const cpx<T>*)p->cy_ctw;
    a.nz1 = p->nz1;
    a.ctl = p->ctl;
    a.xslot = p->xslot;
    a.r = p->r;
    a.p = (const T*)p->p;
    a.q = (const T*)p->qv;
    a.a1 = (const T*)p->cy_a1;
    a.a2 = (const T*)p->cy_a2;
    a.w = (const T*)p->w;
    a.UV = (const cpx<T>*)p->cy_UV;
    a.Ls = p->blk[0].Ls;
    a.P = p->blk[0].P;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.pring = p->pring;
    a.pslot = p->nvec;
    a.giter = p->giter;
    return a;
}

template <typename T>
hipError_t cyl_thomas_T(lg_plan* p, const T* rhat, T* z, int nfields, int mode) {
    CylTdArgs<T> a;
    a.rhat = rhat;
    a.z = z;
    a.cp = (const T*)p->cy_cp;
    a.invden = (const T*)p->cy_invden;
    a.lowr = (const T*)p->cy_lowr;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.ctl = p->ctl;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.mode = mode;
    const dim3 grid((p->nx1 + 255) / 256, nfields);
    hipLaunchKernelGGL(cyl_thomas_kernel<T>, grid, dim3(256), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || mode == 0) return e;
    return launch_finalize(p, 2 /* (r, z) */, (int)grid.x, mode, 0.0, 0, 1.0);
}

template <typename T, int LS>
hipError_t cyl_seg_L(lg_plan* p, const T* rhat, T* y, int nfields, int masked) {
    CylSegArgs<T> a;
    a.rhat = rhat;
    a.y = y;
    a.cp = (const T*)p->cy_cp;
    a.inv = (const T*)p->cy_invden;
    a.lowr = (const T*)p->cy_lowr;
    a.E = p->E;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.P = p->blk[0].P;
    a.segtiles = (a.P + 3) / 4;
    a.ctl = p->ctl;
    a.masked = masked;
    const dim3 grid((unsigned)(((p->nx1 + 63) / 64) * a.segtiles), (unsigned)nfields);
    hipLaunchKernelGGL((cyl_seg_kernel<T, LS>), grid, dim3(256), 0, p->stream, a);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t cyl_red_P(lg_plan* p, CylRedArgs<T>& a, int nfields) {
    const dim3 grid((unsigned)((p->nx1 + 255) / 256), (unsigned)nfields);
    hipLaunchKernelGGL((cyl_red_kernel<T, P>), grid, dim3(256), 0, p->stream, a);
    return hipGetLastError();
}

// segments, then the reduced systems (mode 0: plain; 1: CG start; 2: CG
// iteration, masked, with the (r, z) finalize)
template <typename T>
hipError_t cyl_rsys_T(lg_plan* p, const T* rhat, T* y, int nfields, int mode) {
    if (p->blk[0].P == 1) return cyl_thomas_T<T>(p, rhat, y, nfields, mode);
    hipError_t e;
    switch (p->blk[0].Ls) {
        case 2: e = cyl_seg_L<T, 2>(p, rhat, y, nfields, mode != 0); break;
        case 4: e = cyl_seg_L<T, 4>(p, rhat, y, nfields, mode != 0); break;
        case 8: e = cyl_seg_L<T, 8>(p, rhat, y, nfields, mode != 0); break;
        case 16: e = cyl_seg_L<T, 16>(p, rhat, y, nfields, mode != 0); break;
        case 32: e = cyl_seg_L<T, 32>(p, rhat, y, nfields, mode != 0); break;
        case 64: e = cyl_seg_L<T, 64>(p, rhat, y, nfields, mode != 0); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    CylRedArgs<T> a;
    a.rhat = rhat;
    a.y = y;
    a.E = p->E;
    a.cpl = p->cy_cpl64;
    a.red = p->cy_red;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.Ls = p->blk[0].Ls;
    a.ctl = p->ctl;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.mode = mode;
    switch (p->blk[0].P) {
        case 1: e = cyl_red_P<T, 1>(p, a, nfields); break;
        case 2: e = cyl_red_P<T, 2>(p, a, nfields); break;
        case 4: e = cyl_red_P<T, 4>(p, a, nfields); break;
        case 8: e = cyl_red_P<T, 8>(p, a, nfields); break;
        case 16: e = cyl_red_P<T, 16>(p, a, nfields); break;
        case 32: e = cyl_red_P<T, 32>(p, a, nfields); break;
        case 64: e = cyl_red_P<T, 64>(p, a, nfields); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || mode == 0) return e;
    return launch_finalize(p, 2 /* (r, z) */, (p->nx1 + 255) / 256, mode, 0.0, 0, 1.0);
}

template <typename T>
hipError_t cyl_corr_T(lg_plan* p, T* z, int nfields) {
    const size_t nf = (size_t)p->nx1 * p->nz1;
    const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)nfields);
    hipLaunchKernelGGL(cyl_corr_kernel<T>, grid, dim3(256), 0, p->stream, z, (const cpx<T>*)p->cy_UV, p->nx1,
                       p->nz1, p->blk[0].Ls, p->blk[0].P);
    return hipGetLastError();
}

}  // namespace

hipError_t cyl_launch_stencil(lg_plan* p, const void* x, void* y, bool reduce) {
    const int nf = p->S * p->C;
    if (p->prec == LG_FP64)
        return cyl_stencil_T<double, false>(p, (const double*)x, (double*)y, reduce, nf, (const double*)p->cy_a1,
                                            (const double*)p->cy_a2, (const double*)p->w, nullptr);
    return cyl_stencil_T<float, false>(p, (const float*)x, (float*)y, reduce, nf, (const float*)p->cy_a1,
                                       (const float*)p->cy_a2, (const float*)p->w, nullptr);
}

hipError_t cyl_launch_residual_check(lg_plan* p, const double* b, const double* x) {
    // r = b - A x with the FP64 operator (FP64 tables of a mixed plan), stored,
    // and ||r||^2 per shot; the finalize re-checks the shots that had met the
    // tolerance on the recursive residual
    const int nf = p->S * p->C;
    const bool f64 = p->prec == LG_FP64;
    const double* a1 = f64 ? (const double*)p->cy_a1 : p->cy_a1_64;
    const double* a2 = f64 ? (const double*)p->cy_a2 : p->cy_a2_64;
    const double* w = f64 ? (const double*)p->w : p->w64;
    return cyl_stencil_T<double, true>(p, x, p->r, true, nf, a1, a2, w, b);
}

hipError_t cyl_launch_restart(lg_plan* p, const double* b, double* x, double tol, int max_iter) {
    // after the check: the transform pass from the stored r (its finalize
    // re-checks the shots that had met the tolerance, as the check did)
    return cyl_launch_update(p, 2, b, x, tol, max_iter);
}

hipError_t cyl_launch_dct(lg_plan* p, int inverse, const void* in, void* out, int nfields, int corr) {
    if (p->prec == LG_FP64) {
        CylDctArgs<double> a = cyl_dct_args<double>(p);
        a.in = (const double*)in;
        a.out = (double*)out;
        if (inverse && corr) return cyl_dct_dispatch<double, CY_INV_D>(p, a, nfields);
        return inverse ? cyl_dct_dispatch<double, CY_INV>(p, a, nfields)
                       : cyl_dct_dispatch<double, CY_FWD>(p, a, nfields);
    }
    CylDctArgs<float> a = cyl_dct_args<float>(p);
    a.in = (const float*)in;
    a.out = (float*)out;
    if (inverse && corr) return cyl_dct_dispatch<float, CY_INV_D>(p, a, nfields);
    return inverse ? cyl_dct_dispatch<float, CY_INV>(p, a, nfields) : cyl_dct_dispatch<float, CY_FWD>(p, a, nfields);
}

hipError_t cyl_launch_rsys(lg_plan* p, const void* rhat, void* y, int nfields, int mode) {
    if (p->prec == LG_FP64) return cyl_rsys_T<double>(p, (const double*)rhat, (double*)y, nfields, mode);
    return cyl_rsys_T<float>(p, (const float*)rhat, (float*)y, nfields, mode);
}

hipError_t cyl_launch_corr(lg_plan* p, void* z, int nfields) {
    if (p->prec == LG_FP64) return cyl_corr_T<double>(p, (double*)z, nfields);
    return cyl_corr_T<float>(p, (float*)z, nfields);
}

hipError_t cyl_launch_update(lg_plan* p, int init, const double* b, double* x, double tol, int max_iter) {
    const int nf = p->S * p->C;
    hipError_t e;
    int bpf;
    if (p->prec == LG_FP64) {
        CylDctArgs<double> a = cyl_dct_args<double>(p);
        a.out = (double*)p->rhat;
        a.init = init;
        a.b = b;
        a.x = x;
        e = (init == 0 && p->fuse_op) ? cyl_dct_dispatch<double, CY_UPDATE_OP>(p, a, nf)
                                      : cyl_dct_dispatch<double, CY_UPDATE>(p, a, nf);
        bpf = a.bpf;
    } else {
        CylDctArgs<float> a = cyl_dct_args<float>(p);
        a.out = (float*)p->rhat;
        a.init = init;
        a.b = b;
        a.x = x;
        e = (init == 0 && p->fuse_op) ? cyl_dct_dispatch<float, CY_UPDATE_OP>(p, a, nf)
                                      : cyl_dct_dispatch<float, CY_UPDATE>(p, a, nf);
        bpf = a.bpf;
    }
    if (e != hipSuccess) return e;
    // init 1: start; init 2: restart from the true residual (the thresholds
    // set at the start apply)
    const double t1 = phase_tol(p, tol, false), tr = phase_tol(p, tol, true);
    return launch_finalize(p, 1 /* ||r||^2 */, bpf, init, t1 * t1, max_iter, 0.0, tol * tol, tr * tr);
}

hipError_t cyl_launch_correct(lg_plan* p, int init) {
    const int nf = p->S * p->C;
    if (p->prec == LG_FP64) {
        CylDctArgs<double> a = cyl_dct_args<double>(p);
        a.in = (const double*)p->y;
        a.out = (double*)p->p;
        a.init = init;
        return p->blk[0].P > 1 ? cyl_dct_dispatch<double, CY_CORRECT_D>(p, a, nf)
                               : cyl_dct_dispatch<double, CY_CORRECT>(p, a, nf);
    }
    CylDctArgs<float> a = cyl_dct_args<float>(p);
    a.in = (const float*)p->y;
    a.out = (float*)p->p;
    a.init = init;
    return p->blk[0].P > 1 ? cyl_dct_dispatch<float, CY_CORRECT_D>(p, a, nf)
                           : cyl_dct_dispatch<float, CY_CORRECT>(p, a, nf);
}

}  // namespace lg
