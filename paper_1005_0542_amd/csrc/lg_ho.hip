// Fourth-order acoustic operator (Sec. 3.2: a higher-order scheme, still
// preconditioned by the second-order B) on gfx950.
//
//   A4 u = Dx^T Kx Dx u + Dz^T Kz Dz u + w u,
//   (D u)_{m+1/2} = 27 (u_{m+1} - u_m) - (u_{m+2} - u_{m-1})   (times 1/(24 h)),
//
// with the Dirichlet sides by odd reflection (u_0 = u_N = 0, u_{-1} = -u_1,
// u_{N+1} = -u_{N-1}).  The transpose at node i combines the faces
// i-3/2, i-1/2, i+1/2, i+3/2 with weights -1, 27, -27, 1; the faces -1/2 and
// N+1/2 (needed at i = 1 and i = N-1) equal their mirrors 1/2 and N-1/2,
// which is the reflection folded into D.  Kx, Kz carry 1/(24 h)^2.
//
// A block covers 64 columns x 16 rows and stages that tile of the field with
// a 3-node halo in LDS (one coalesced pass, the reflected nodes loaded from
// their mirrors with the sign flipped, nodes outside the grid read as 0
// through the buffer range check); each thread then computes a column strip
// of HO_RPT rows from LDS, while the next shot's tile is already in flight.  The face tables and w of the strip stay in
// registers while the block works through `nsh` shots.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lg_device.h"
#include "lg_internal.h"

namespace lg {

constexpr int HO_RPT = 4;
constexpr int HO_TW = 64 + 6;            // LDS tile width (columns + halo)
constexpr int HO_TH = 4 * HO_RPT + 6;    // LDS tile height (rows + halo)
constexpr int HO_LPT = (HO_TH * HO_TW + 255) / 256;   // tile elements per thread

template <typename T>
struct HoArgs {
    const T* p;
    T* q;
    const T* kx;         // [nz-1][nx]: x-faces of the interior rows
    const T* kz;         // [nz][nx-1]: z-faces of the interior columns
    const T* w;          // [nz-1][nx-1]
    const double* b;     // residual mode: q = b - A4 p
    int nx, nz;          // cells
    int gx, gy;
    int nfields, nsh;
    ShotCtl* ctl;        // nullptr: plain application
    double* partial;
    size_t pstride;
    int pring;           // > 1 (CG): p at slot giter[0] % pring (held search directions)
    size_t pslot;        // elements per slot
    const int* giter;
};

// A4 contribution of one axis at one node from the 7 node values v[0..6]
// (offsets -3..3, reflections applied) and the 4 face coefficients k[0..3]
// (faces -3/2..3/2); lo / hi: the node is the first / last interior one.
template <typename T>
__device__ __forceinline__ T ho_axis(const T* v, const T* k, bool lo, bool hi) {
    T d[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) d[f] = (T)27 * (v[f + 2] - v[f + 1]) - (v[f + 3] - v[f]);
    if (lo) d[0] = d[1];
    if (hi) d[3] = d[2];
    return fmad((T)27, k[1] * d[1] - k[2] * d[2], k[3] * d[3] - k[0] * d[0]);
}

template <typename T, bool RES>
__global__ __launch_bounds__(256) void ho_stencil_kernel(HoArgs<T> a) {
    __shared__ double red[64][4];                  // per-wave (p, Ap) of the block's fields
    const int nx = a.nx, nz = a.nz, nx1 = nx - 1, nz1 = nz - 1;
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int L = xcd_linear(blockIdx.x, gridDim.x);
    const int bx = L % a.gx, by = (L / a.gx) % a.gy, grp = L / (a.gx * a.gy);
    const int ci = bx * 64 + lane;                  // interior column, node i = ci + 1
    const int j0 = (by * 4 + ty) * HO_RPT;          // first interior row of the strip
    const bool live = ci < nx1;
    const int i = ci + 1;
    constexpr uint32_t SZ = sizeof(T);
    const uint32_t nf = (uint32_t)nx1 * (uint32_t)nz1;
    const rsrc_t rkx = buf_rsrc(a.kx, (uint32_t)nz1 * (uint32_t)nx * SZ);
    const rsrc_t rkz = buf_rsrc(a.kz, (uint32_t)nz * (uint32_t)nx1 * SZ);
    const rsrc_t rw = buf_rsrc(a.w, nf * SZ);

    // medium of the strip: x-faces m = i-2..i+1 of each row (mirrored at the
    // ends), z-faces n = j-2..j+1 of the strip's rows (node row j = cj + 1)
    T kx[HO_RPT][4], kz[HO_RPT + 3], wv[HO_RPT];
#pragma unroll
    for (int r = 0; r < HO_RPT; ++r) {
        const int cj = j0 + r;
        const bool ok = live && cj < nz1;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            int m = i - 2 + f;
            m = m < 0 ? 0 : (m > nx - 1 ? nx - 1 : m);
            kx[r][f] = bload<T>(rkx, ok ? (uint32_t)(cj * nx + m) * SZ : BUF_OOB);
        }
        wv[r] = bload<T>(rw, ok ? (uint32_t)(cj * nx1 + ci) * SZ : BUF_OOB);
    }
#pragma unroll
    for (int f = 0; f < HO_RPT + 3; ++f) {
        int n = j0 - 1 + f;                          // faces of node rows j0+1-2 .. j0+HO_RPT+1
        n = n < 0 ? 0 : (n > nz - 1 ? nz - 1 : n);
        kz[f] = bload<T>(rkz, live ? (uint32_t)(n * nx1 + ci) * SZ : BUF_OOB);
    }

    __shared__ T tile[HO_TH * HO_TW];
    const int ni0 = bx * 64 + 1 - 3, nj0 = by * 4 * HO_RPT + 1 - 3;   // node of tile[0]
    const int f0 = grp * a.nsh, f1e = min(a.nfields, f0 + a.nsh);
    // the next field's tile is loaded into registers while the current one is
    // computed from LDS
    auto next_active = [&](int f) {
        while (f < f1e && a.ctl != nullptr && !RES && a.ctl[f].active == 0) ++f;   // uniform per block
        return f;
    };
    // tile element u of this thread: field offset (or out of range) and the
    // sign of the odd reflection, the same for every shot
    uint32_t toff[HO_LPT];
    T tsgn[HO_LPT];
#pragma unroll
    for (int u = 0; u < HO_LPT; ++u) {
        const int t = threadIdx.x + u * 256;
        const int rr = t / HO_TW, cc = t - rr * HO_TW;
        int nj = nj0 + rr, ni = ni0 + cc;
        T sgn = (T)1;
        if (nj == -1) { nj = 1; sgn = -sgn; }
        if (nj == nz + 1) { nj = nz - 1; sgn = -sgn; }
        if (ni == -1) { ni = 1; sgn = -sgn; }
        if (ni == nx + 1) { ni = nx - 1; sgn = -sgn; }
        const bool in = t < HO_TH * HO_TW && nj >= 1 && nj <= nz1 && ni >= 1 && ni <= nx1;
        toff[u] = in ? (uint32_t)((nj - 1) * nx1 + ni - 1) * SZ : BUF_OOB;
        tsgn[u] = sgn;
    }
    // held directions: this iteration's p slot (one count for every shot)
    const size_t ps = (!RES && a.pring > 1) ? (size_t)(*a.giter % a.pring) * a.pslot : 0;
    auto load_tile = [&](int f, T* v) {
        const rsrc_t rp = buf_rsrc(a.p + ps + (size_t)f * nf, nf * SZ);
#pragma unroll
        for (int u = 0; u < HO_LPT; ++u) v[u] = bload<T>(rp, toff[u]);
    };
    T nxt[HO_LPT];
    int field = next_active(f0);
    if (field < f1e) load_tile(field, nxt);
    while (field < f1e) {
        const size_t fo = (size_t)field * nf;
        __syncthreads();                            // the previous field's reads are done
#pragma unroll
        for (int u = 0; u < HO_LPT; ++u) {
            const int t = threadIdx.x + u * 256;
            if (t < HO_TH * HO_TW) tile[t] = tsgn[u] * nxt[u];
        }
        __syncthreads();
        const int fn = next_active(field + 1);
        if (fn < f1e) load_tile(fn, nxt);
        // column: node rows j0-2 .. j0+HO_RPT+3; rows: node columns i-3 .. i+3
        const int lc = lane + 3, lr = ty * HO_RPT;       // tile column of node i; tile row of node row j0-2
        T col[HO_RPT + 6];
#pragma unroll
        for (int r = 0; r < HO_RPT + 6; ++r) col[r] = tile[(lr + r) * HO_TW + lc];
        T row[HO_RPT][7];
#pragma unroll
        for (int r = 0; r < HO_RPT; ++r)
#pragma unroll
            for (int o = 0; o < 7; ++o) row[r][o] = tile[(lr + r + 3) * HO_TW + lc - 3 + o];
        double pq = 0.0;
        const rsrc_t rq = buf_rsrc((a.q != nullptr ? a.q : const_cast<T*>(a.p)) + fo,
                                   a.q != nullptr ? nf * SZ : 0u);
        const rsrc_t rb = buf_rsrc(a.b + fo, RES ? nf * 8u : 0u);
#pragma unroll
        for (int r = 0; r < HO_RPT; ++r) {
            const int cj = j0 + r, nj = cj + 1;
            const uint32_t o = (live && cj < nz1) ? (uint32_t)(cj * nx1 + ci) : BUF_OOB / 8u;
            const T c = col[r + 3];
            T v = ho_axis<T>(row[r], kx[r], i == 1, i == nx1) + ho_axis<T>(&col[r], &kz[r], nj == 1, nj == nz1) +
                  wv[r] * c;
            if constexpr (RES) {
                v = (T)(bload<double>(rb, o * 8u) - (double)v);
                if (o != BUF_OOB / 8u) pq += (double)v * (double)v;     // rows past the grid: none
            } else {
                pq += (double)c * (double)v;
            }
            bstore<T>(v, rq, o * SZ);
        }
        if (a.ctl != nullptr) {
            pq = wave_sum(pq);
            if (lane == 0) red[field - f0][ty] = pq;
        }
        field = fn;
    }
    if (a.ctl == nullptr) return;
    __syncthreads();
    const int kf = threadIdx.x;
    if (kf < f1e - f0 && (RES || a.ctl[f0 + kf].active != 0))
        a.partial[(size_t)(f0 + kf) * a.pstride + by * a.gx + bx] = ((red[kf][0] + red[kf][1]) + red[kf][2]) + red[kf][3];
}

namespace {

template <typename T, bool RES>
hipError_t ho_T(lg_plan* p, const T* x, T* y, bool reduce, const T* kx, const T* kz, const T* w,
                const double* b) {
    HoArgs<T> a;
    a.p = x;
    a.q = y;
    a.kx = kx;
    a.kz = kz;
    a.w = w;
    a.b = b;
    a.nx = p->g.nx;
    a.nz = p->g.nz;
    a.gx = (p->nx1 + 63) / 64;
    a.gy = (p->nz1 + 4 * HO_RPT - 1) / (4 * HO_RPT);
    a.nfields = p->S * p->C;
    a.nsh = std::max(1, std::min(a.nfields, p->op_shots));
    a.ctl = reduce ? p->ctl : nullptr;
    a.partial = p->partial;
    a.pstride = p->partial_stride;
    a.pring = (reduce && !RES) ? p->pring : 1;
    a.pslot = p->nvec;
    a.giter = p->giter;
    const int groups = (a.nfields + a.nsh - 1) / a.nsh;
    hipLaunchKernelGGL((ho_stencil_kernel<T, RES>), dim3(a.gx * a.gy * groups), dim3(256), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !reduce) return e;
    // residual mode: the restart check on ||b - A x||^2; else (p, Ap)
    return RES ? launch_finalize(p, 1 /* ||r||^2 */, a.gx * a.gy, 2, 0.0, 0, 0.0)
               : launch_finalize(p, 0 /* (p, Ap) */, a.gx * a.gy, 0, 0.0, 0, 0.0);
}

}  // namespace

hipError_t ho_launch_stencil(lg_plan* p, const void* x, void* y, bool reduce) {
    if (p->prec == LG_FP64)
        return ho_T<double, false>(p, (const double*)x, (double*)y, reduce, (const double*)p->ho_kx,
                                   (const double*)p->ho_kz, (const double*)p->w, nullptr);
    return ho_T<float, false>(p, (const float*)x, (float*)y, reduce, (const float*)p->ho_kx,
                              (const float*)p->ho_kz, (const float*)p->w, nullptr);
}

hipError_t ho_launch_residual(lg_plan* p, const double* b, const double* x) {
    const bool f64 = p->prec == LG_FP64;
    const double* kx = f64 ? (const double*)p->ho_kx : p->ho_kx64;
    const double* kz = f64 ? (const double*)p->ho_kz : p->ho_kz64;
    const double* w = f64 ? (const double*)p->w : p->w64;
    return ho_T<double, true>(p, x, p->r, true, kx, kz, w, b);
}

}  // namespace lg
