// Elastic (Lame) Laguerre-domain operator, block preconditioner apply, and the
// restarted GMRES(k) driver (Sec. 2.2-2.4, eqs. elastic_problemQn, precond2).
//
// Operator (2D Cartesian reading of the paper's second-order scheme, SPD sign;
// node-sampled lambda, mu; face values are means of node values; Dc is the
// two-cell central difference):
//   (C u)_x = -Dx+((l+2m) Dx- ux) - Dz+(m Dz- ux) - Dxc(l Dzc uz) - Dzc(m Dxc uz) + w ux
//   (C u)_z = -Dx+(m Dx- uz) - Dz+((l+2m) Dz- uz) - Dzc(l Dxc ux) - Dxc(m Dzc ux) + w uz
//
// GMRES(k) is right-preconditioned by K = diag(B1, B2); the Arnoldi basis is
// orthogonalised by classical Gram-Schmidt applied twice (all inner products
// of one pass in a single sweep over the basis), every vector operation and
// inner product runs on the device, and only the (k+1) x k Hessenberg matrix
// with its Givens rotations lives on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lg_device.h"
#include "lg_internal.h"

namespace lg {

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
template <typename T>
struct ElArgs {
    const T* u;     // [S][2][nz1][nx1]
    T* y;
    const T* lam;   // nodes (nz+1)(nx+1)
    const T* mu;
    const T* w;     // interior
    int nx1, nz1, S;
    int free_top;        // traction-free surface on the first unknown row
    T idx2, idz2, ixz;   // 1/dx^2, 1/dz^2, 1/(4 dx dz)
};

// One block computes a tile of EL_TX x EL_TZ points of one shot from LDS
// copies of both components and of the node-sampled lambda and mu over the
// tile and its one-point rim (interior values outside the grid staged as 0).
constexpr int EL_TX = 64, EL_TZ = 4;
constexpr int EL_HX = EL_TX + 2, EL_HZ = EL_TZ + 2;

template <typename T>
__global__ __launch_bounds__(EL_TX * EL_TZ) void elastic_stencil_kernel(ElArgs<T> a) {
    __shared__ T sux[EL_HZ][EL_HX], suz[EL_HZ][EL_HX], slam[EL_HZ][EL_HX], smu[EL_HZ][EL_HX];
    const int nx1 = a.nx1, nz1 = a.nz1, NXN = nx1 + 2;
    const size_t npts = (size_t)nx1 * nz1;
    // blocks in (shot, tile row, tile column) order
    const unsigned xb = (unsigned)(nx1 + EL_TX - 1) / EL_TX;
    const unsigned tiles = xb * (unsigned)((nz1 + EL_TZ - 1) / EL_TZ);
    const unsigned s = blockIdx.x / tiles;
    const unsigned rt = blockIdx.x - s * tiles;
    const unsigned tzb = rt / xb;
    const int i0 = (int)(rt - tzb * xb) * EL_TX, j0 = (int)tzb * EL_TZ;
    const T* gux = a.u + (size_t)s * 2 * npts;
    const T* guz = gux + npts;
    // rim entry (hz, hx) holds interior point (i0 - 1 + hx, j0 - 1 + hz), whose
    // node is (i0 + hx, j0 + hz)
    for (int q = threadIdx.x; q < EL_HZ * EL_HX; q += EL_TX * EL_TZ) {
        const int hz = q / EL_HX, hx = q - hz * EL_HX;
        const int ii = i0 - 1 + hx, jj = j0 - 1 + hz;
        const bool in = ii >= 0 && ii < nx1 && jj >= 0 && jj < nz1;
        const size_t o = in ? (size_t)jj * nx1 + ii : 0;
        sux[hz][hx] = in ? gux[o] : (T)0;
        suz[hz][hx] = in ? guz[o] : (T)0;
        const bool nin = ii <= nx1 && jj <= nz1;            // node index within [0, n + 1]
        const size_t on = nin ? (size_t)(jj + 1) * NXN + (ii + 1) : 0;
        slam[hz][hx] = nin ? a.lam[on] : (T)0;
        smu[hz][hx] = nin ? a.mu[on] : (T)0;
    }
    __syncthreads();
    const int tx = threadIdx.x % EL_TX, tz = threadIdx.x / EL_TX;
    const int i = i0 + tx, j = j0 + tz;
    if (i >= nx1 || j >= nz1) return;
    const size_t pt = (size_t)j * nx1 + i;
    const int I = i + 1, J = j + 1;
    // value of a component (interior, zero on the boundary), lambda and mu at
    // node (Ii, Jj) within one node of (I, J)
    const T(*const ux)[EL_HX] = sux;
    const T(*const uz)[EL_HX] = suz;
    auto U = [&](const T(*f)[EL_HX], int Ii, int Jj) -> T { return f[tz + 1 + (Jj - J)][tx + 1 + (Ii - I)]; };
    auto L = [&](int Ii, int Jj) -> T { return slam[tz + 1 + (Jj - J)][tx + 1 + (Ii - I)]; };
    auto Mu = [&](int Ii, int Jj) -> T { return smu[tz + 1 + (Jj - J)][tx + 1 + (Ii - I)]; };
    const T h = (T)0.5;
    const T l0 = L(I, J), m0 = Mu(I, J);
    const T p0 = l0 + 2 * m0;
    const T pE = h * (p0 + L(I + 1, J) + 2 * Mu(I + 1, J)), pW = h * (p0 + L(I - 1, J) + 2 * Mu(I - 1, J));
    const T pS = h * (p0 + L(I, J + 1) + 2 * Mu(I, J + 1)), pN = h * (p0 + L(I, J - 1) + 2 * Mu(I, J - 1));
    const T mE = h * (m0 + Mu(I + 1, J)), mW = h * (m0 + Mu(I - 1, J));
    const T mS = h * (m0 + Mu(I, J + 1)), mN = h * (m0 + Mu(I, J - 1));
    const T cx = U(ux, I, J), cz = U(uz, I, J);
    const T wv = a.w[pt];
    T* yo = a.y + s * 2 * npts;
    if (a.free_top && J == 1) {
        // Surface row: the gradient of the discrete strain energy divided by
        // the row's half control strip.  x faces as below; no face above the
        // surface, the face below counted twice; the node cross terms use the
        // one-sided z-difference (u(J+1) - u(J))/dz on this row, and the
        // central one on the row below (whose contribution is halved back).
        const T t2 = (T)2 * a.ixz;   // 1/(2 dx dz)
        T fx = (pE * (cx - U(ux, I + 1, J)) + pW * (cx - U(ux, I - 1, J))) * a.idx2 +
               (T)2 * mS * (cx - U(ux, I, J + 1)) * a.idz2;
        T fz = (mE * (cz - U(uz, I + 1, J)) + mW * (cz - U(uz, I - 1, J))) * a.idx2 +
               (T)2 * pS * (cz - U(uz, I, J + 1)) * a.idz2;
        fx -= (L(I + 1, J) * (U(uz, I + 1, J + 1) - U(uz, I + 1, J)) -
               L(I - 1, J) * (U(uz, I - 1, J + 1) - U(uz, I - 1, J))) * t2;
        fx -= (Mu(I, J) * (U(uz, I + 1, J) - U(uz, I - 1, J)) +
               Mu(I, J + 1) * (U(uz, I + 1, J + 1) - U(uz, I - 1, J + 1))) * t2;
        fz -= (L(I, J) * (U(ux, I + 1, J) - U(ux, I - 1, J)) +
               L(I, J + 1) * (U(ux, I + 1, J + 1) - U(ux, I - 1, J + 1))) * t2;
        fz -= (Mu(I + 1, J) * (U(ux, I + 1, J + 1) - U(ux, I + 1, J)) -
               Mu(I - 1, J) * (U(ux, I - 1, J + 1) - U(ux, I - 1, J))) * t2;
        yo[pt] = fx + wv * cx;
        yo[npts + pt] = fz + wv * cz;
        return;
    }
    // diagonal (flux) parts
    T yx = (pE * (cx - U(ux, I + 1, J)) + pW * (cx - U(ux, I - 1, J))) * a.idx2 +
           (mS * (cx - U(ux, I, J + 1)) + mN * (cx - U(ux, I, J - 1))) * a.idz2;
    T yz = (mE * (cz - U(uz, I + 1, J)) + mW * (cz - U(uz, I - 1, J))) * a.idx2 +
           (pS * (cz - U(uz, I, J + 1)) + pN * (cz - U(uz, I, J - 1))) * a.idz2;
    // mixed parts, x-equation: -Dxc(l Dzc uz) - Dzc(m Dxc uz)
    const T dxz_p = U(uz, I + 1, J + 1) - U(uz, I + 1, J - 1);   // Dzc uz at I+1 (x 2dz)
    const T dxz_m = U(uz, I - 1, J + 1) - U(uz, I - 1, J - 1);   // Dzc uz at I-1
    const T dzx_p = U(uz, I + 1, J + 1) - U(uz, I - 1, J + 1);   // Dxc uz at J+1 (x 2dx)
    const T dzx_m = U(uz, I + 1, J - 1) - U(uz, I - 1, J - 1);   // Dxc uz at J-1
    yx -= (L(I + 1, J) * dxz_p - L(I - 1, J) * dxz_m + Mu(I, J + 1) * dzx_p - Mu(I, J - 1) * dzx_m) * a.ixz;
    const T exz_p = U(ux, I + 1, J + 1) - U(ux, I + 1, J - 1);   // Dzc ux at I+1
    const T exz_m = U(ux, I - 1, J + 1) - U(ux, I - 1, J - 1);
    const T ezx_p = U(ux, I + 1, J + 1) - U(ux, I - 1, J + 1);   // Dxc ux at J+1
    const T ezx_m = U(ux, I + 1, J - 1) - U(ux, I - 1, J - 1);
    // z-equation: -Dzc(l Dxc ux) - Dxc(m Dzc ux)
    yz -= (L(I, J + 1) * ezx_p - L(I, J - 1) * ezx_m + Mu(I + 1, J) * exz_p - Mu(I - 1, J) * exz_m) * a.ixz;
    yo[pt] = yx + wv * cx;
    yo[npts + pt] = yz + wv * cz;
}

template <typename T>
hipError_t el_stencil_T(lg_plan* p, const T* x, T* y) {
    ElArgs<T> a;
    a.u = x;
    a.y = y;
    a.lam = (const T*)p->lam;
    a.mu = (const T*)p->mu;
    a.w = (const T*)p->w;
    a.nx1 = p->nx1;
    a.nz1 = p->nz1;
    a.S = p->S;
    a.free_top = p->el_free ? 1 : 0;
    a.idx2 = (T)(1.0 / (p->g.dx * p->g.dx));
    a.idz2 = (T)(1.0 / (p->g.dz * p->g.dz));
    a.ixz = (T)(1.0 / (4.0 * p->g.dx * p->g.dz));
    const size_t tiles = (size_t)((p->nx1 + EL_TX - 1) / EL_TX) * ((p->nz1 + EL_TZ - 1) / EL_TZ);
    hipLaunchKernelGGL(elastic_stencil_kernel<T>, dim3((unsigned)(tiles * p->S)), dim3(EL_TX * EL_TZ), 0,
                       p->stream, a);
    return hipGetLastError();
}

hipError_t launch_elastic_stencil(lg_plan* p, const void* x, void* y) {
    if (p->prec == LG_FP64) return el_stencil_T<double>(p, (const double*)x, (double*)y);
    return el_stencil_T<float>(p, (const float*)x, (float*)y);
}

// Traction-free surface rows of the preconditioner (the rank-one term on the
// Dirichlet solution y of block blk): coef = y(row 1) / (1 - g_k(1)), then
// y += coef g_k on every row.
// (t2, g2 non-null: odd fields take the second block's tables)
template <typename T>
__global__ __launch_bounds__(256) void surface_coef_kernel(const T* __restrict__ y, const double* __restrict__ t,
                                                           const double* __restrict__ t2, double* __restrict__ coef,
                                                           int nx1, size_t npts, int nfields, int fstride, int foff) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)nfields * nx1) return;
    const size_t f = (e / nx1) * fstride + foff;
    const int k = (int)(e % nx1);
    const double* __restrict__ tt = (t2 != nullptr && (f & 1)) ? t2 : t;
    coef[f * nx1 + k] = (double)y[f * npts + nx1 + k] * tt[k];
}

template <typename T>
__global__ __launch_bounds__(256) void surface_apply_kernel(T* __restrict__ y, const T* __restrict__ g,
                                                            const T* __restrict__ g2,
                                                            const double* __restrict__ coef, int nx1, size_t npts,
                                                            size_t total, int fstride, int foff) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const size_t f = (e / npts) * fstride + foff;
    const size_t pt = e % npts;
    const int k = (int)(pt % nx1);
    const T* __restrict__ gg = (g2 != nullptr && (f & 1)) ? g2 : g;
    y[f * npts + pt] += (T)coef[f * nx1 + k] * gg[pt];
}

template <typename T>
hipError_t surface_rows_T(lg_plan* p, int blk, T* y, int nfields, int fstride, int foff) {
    const int b0 = blk < 0 ? 0 : blk;          // blk < 0: both blocks by field parity
    const double* t2 = blk < 0 ? p->es_t[1] : nullptr;
    const T* g2 = blk < 0 ? (const T*)p->es_g[1] : nullptr;
    const unsigned gc = (unsigned)(((size_t)nfields * p->nx1 + 255) / 256);
    hipLaunchKernelGGL(surface_coef_kernel<T>, dim3(gc), dim3(256), 0, p->stream, y, p->es_t[b0], t2, p->sm_c,
                       p->nx1, p->npts, nfields, fstride, foff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)nfields * p->npts;
    hipLaunchKernelGGL(surface_apply_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, p->stream, y,
                       (const T*)p->es_g[b0], g2, p->sm_c, p->nx1, p->npts, total, fstride, foff);
    return hipGetLastError();
}

hipError_t launch_surface_rows(lg_plan* p, int blk, void* y, int nfields, int fstride, int foff) {
    if (!p->el_free || p->nz1 < 2) return hipSuccess;   // one row: the surface row has no neighbour
    if (p->prec == LG_FP64) return surface_rows_T<double>(p, blk, (double*)y, nfields, fstride, foff);
    return surface_rows_T<float>(p, blk, (float*)y, nfields, fstride, foff);
}

// K^{-1} = diag(B1^{-1}, B2^{-1}) on working-type vectors [S][2][..]; uses the
// plan's spectral buffers rhat and y.
hipError_t launch_elastic_precond(lg_plan* p, const void* r, void* z) {
    const int S = p->S;
    // both components' z-systems in one launch of each Dichotomy kernel (block
    // -1: B1 on the x fields, B2 on the z fields; the two share P and Ls)
    hipError_t e = launch_dst(p, 0, r, p->rhat, S * 2);
    if (e == hipSuccess) e = launch_td(p, -1, p->rhat, p->y, S * 2, 0, 1, 0);
    if (e == hipSuccess && p->blk[0].P > 1) e = launch_rs(p, -1, p->rhat, p->y, S * 2, 0, 1, 0);
    // Dirichlet top: the segment correction inside the inverse transform; the
    // traction-free surface needs the corrected surface row first
    if (!p->el_free && p->blk[0].P > 1) return e == hipSuccess ? launch_correct_inv(p, z, S * 2) : e;
    if (e == hipSuccess && p->blk[0].P > 1) e = launch_correct(p, -1, p->y, S * 2, 1, 0);
    if (e == hipSuccess) e = launch_surface_rows(p, -1, p->y, S * 2, 1, 0);
    if (e == hipSuccess) e = launch_dst(p, 1, p->y, z, S * 2);
    return e;
}

// ---------------------------------------------------------------------------
// GMRES vector kernels (FP64), one shot = 2 npts contiguous values
// ---------------------------------------------------------------------------
constexpr int GM_MAXK = 32;            // largest restart length supported
constexpr int GM_BLK = 256;
constexpr int GM_CHUNK = 4096;         // elements per block per shot in reductions

// partial[s][i][b] = sum over block b of the shot's chunk of V_i * w (i < m).
// The basis vectors are taken 8 at a time; within a group every load of an
// element step is an unconditional buffer load (vectors past m have a
// resource of size 0 and read 0), so they are all in flight together.
__global__ __launch_bounds__(GM_BLK) void gm_multidot_kernel(const double* __restrict__ V, size_t vstride,
                                                             int m, const double* __restrict__ w, size_t n_s,
                                                             const int* __restrict__ active,
                                                             double* __restrict__ partial, int nblk) {
    constexpr int G = 8;
    __shared__ double red[GM_BLK / 64];
    const int s = blockIdx.y, b = blockIdx.x;
    if (active[s] == 0) return;
    const size_t base = (size_t)s * n_s;
    const size_t lo = (size_t)b * GM_CHUNK, hi = min(lo + GM_CHUNK, n_s);
    const uint32_t nbytes = (uint32_t)(n_s * 8);
    const rsrc_t rw = buf_rsrc(w + base, nbytes);
    for (int i0 = 0; i0 < m; i0 += G) {           // uniform over the block
        rsrc_t rv[G];
#pragma unroll
        for (int u = 0; u < G; ++u) rv[u] = buf_rsrc(V + (size_t)(i0 + u) * vstride + base, i0 + u < m ? nbytes : 0u);
        double acc[G];
#pragma unroll
        for (int u = 0; u < G; ++u) acc[u] = 0.0;
        for (size_t e = lo + 2 * threadIdx.x; e < hi; e += 2 * GM_BLK) {   // element pairs (n_s, lo, hi even)
            const uint32_t off = (uint32_t)(e * 8);
            const cpx<double> wv = bload2<double>(rw, off);
            cpx<double> vv[G];
#pragma unroll
            for (int u = 0; u < G; ++u) vv[u] = bload2<double>(rv[u], off);
#pragma unroll
            for (int u = 0; u < G; ++u) {
                acc[u] += vv[u].x * wv.x;
                acc[u] += vv[u].y * wv.y;
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (i0 + u < m) {                      // uniform over the block
                const double t = block_sum(acc[u], red);
                if (threadIdx.x == 0) partial[((size_t)s * (GM_MAXK + 1) + i0 + u) * nblk + b] = t;
            }
        }
    }
}

// Sum over the nblk per-block partials of product i of shot s, in the fixed
// order of gm_reduce_kernel (every thread of the block gets the value), so a
// consumer kernel can take a grid-wide result without a reduction launch.
__device__ __forceinline__ double partial_total(const double* __restrict__ partial, int s, int i, int nblk,
                                                double* red) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GM_BLK) v += partial[((size_t)s * (GM_MAXK + 1) + i) * nblk + b];
    return block_sum(v, red);
}

// partial_total for products 0..m-1 at once (m <= MB): one pass over the
// partials and one barrier; per product the same order as partial_total.
template <int MB>
__device__ __forceinline__ void partial_totals(const double* __restrict__ partial, int s, int m, int nblk,
                                               double (*red)[GM_BLK / 64], double* c) {
    double v[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) v[u] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GM_BLK) {
#pragma unroll
        for (int u = 0; u < MB; ++u)
            if (u < m) v[u] += partial[((size_t)s * (GM_MAXK + 1) + u) * nblk + b];
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        v[u] = wave_sum(v[u]);
        if (lane == 0) red[u][wave] = v[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        double t = 0.0;
        for (int i = 0; i < GM_BLK / 64; ++i) t += red[u][i];
        c[u] = u < m ? t : 0.0;
    }
    __syncthreads();   // red may be reused by the caller
}

// Classical Gram-Schmidt twice, with each subtraction fused into the sweep
// that follows it (one read of the basis instead of two):
//   NORM = false: w -= sum_{i<m} coef[s][i] V_i, then the block partials of
//                 (V_i, w) for i < m (the second pass's inner products);
//   NORM = true:  w -= sum_{i<m} coef[s][i] V_i, then the block partial of
//                 (w, w) in slot 0.
// Per element the subtraction is gm_subtract_kernel's and the products and
// per-thread sums are gm_multidot_kernel's, in the same order, so the
// results are those of the separate kernels.  MB >= m bounds the unroll.
// The coefficients are the previous sweep's products: with pin != nullptr
// every block sums them from that sweep's per-block partials (pin) and block
// 0 of the shot also stores them to coef (for the host's Hessenberg column);
// with pin == nullptr they are read from coef.
template <int MB, bool NORM>
__global__ __launch_bounds__(GM_BLK) void gm_subdot_kernel(const double* __restrict__ V, size_t vstride, int m,
                                                           double* __restrict__ coef, int coef_stride,
                                                           const double* __restrict__ pin,
                                                           double* __restrict__ w, size_t n_s,
                                                           const int* __restrict__ active,
                                                           double* __restrict__ partial, int nblk) {
    __shared__ double red[GM_BLK / 64];
    const int s = blockIdx.y, b = blockIdx.x;
    if (active[s] == 0) return;
    const size_t base = (size_t)s * n_s;
    const size_t lo = (size_t)b * GM_CHUNK, hi = min(lo + GM_CHUNK, n_s);
    const uint32_t nbytes = (uint32_t)(n_s * 8);
    const rsrc_t rw = buf_rsrc(w + base, nbytes);
    __shared__ double redm[MB][GM_BLK / 64];
    rsrc_t rv[MB];
    double c[MB];
    if (pin != nullptr) {                          // uniform over the launch
        partial_totals<MB>(pin, s, m, nblk, redm, c);
        if (b == 0 && threadIdx.x == 0)
            for (int u = 0; u < m; ++u) coef[(size_t)s * coef_stride + u] = c[u];
    }
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        rv[u] = buf_rsrc(V + (size_t)u * vstride + base, u < m ? nbytes : 0u);
        if (pin == nullptr) c[u] = u < m ? coef[(size_t)s * coef_stride + u] : 0.0;
    }
    constexpr int NA = NORM ? 1 : MB;
    double acc[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) acc[u] = 0.0;
    for (size_t e = lo + 2 * threadIdx.x; e < hi; e += 2 * GM_BLK) {   // element pairs (n_s, lo, hi even)
        const uint32_t off = (uint32_t)(e * 8);
        cpx<double> vv[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) vv[u] = bload2<double>(rv[u], off);
        cpx<double> wv = bload2<double>(rw, off);
#pragma unroll
        for (int u = 0; u < MB; ++u)
            if (u < m) {
                wv.x -= c[u] * vv[u].x;
                wv.y -= c[u] * vv[u].y;
            }
        bstore2(wv, rw, off);
        if constexpr (NORM) {
            acc[0] += wv.x * wv.x;
            acc[0] += wv.y * wv.y;
        } else {
#pragma unroll
            for (int u = 0; u < MB; ++u) {
                acc[u] += vv[u].x * wv.x;
                acc[u] += vv[u].y * wv.y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        if (u < (NORM ? 1 : m)) {                  // uniform over the block
            const double t = block_sum(acc[u], red);
            if (threadIdx.x == 0) partial[((size_t)s * (GM_MAXK + 1) + u) * nblk + b] = t;
        }
    }
}

// out[s][i] = sum_b partial[s][i][b] (fixed order), i < m; plus add[s][i] if given
__global__ __launch_bounds__(GM_BLK) void gm_reduce_kernel(const double* __restrict__ partial, int m, int nblk,
                                                           const int* __restrict__ active,
                                                           double* __restrict__ out, int out_stride) {
    __shared__ double red[GM_BLK / 64];
    const int s = blockIdx.x;
    if (active[s] == 0) return;
    for (int i = 0; i < m; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += GM_BLK) v += partial[((size_t)s * (GM_MAXK + 1) + i) * nblk + b];
        v = block_sum(v, red);
        if (threadIdx.x == 0) out[(size_t)s * out_stride + i] = v;
    }
}

// w -= sum_{i<m} coef[s][i] V_i   (per-shot coefficients in device memory)
__global__ __launch_bounds__(GM_BLK) void gm_subtract_kernel(const double* __restrict__ V, size_t vstride, int m,
                                                             const double* __restrict__ coef, int coef_stride,
                                                             double* __restrict__ w, size_t n_s, int S,
                                                             const int* __restrict__ active) {
    const size_t e = (size_t)blockIdx.x * GM_BLK + threadIdx.x;
    if (e >= n_s * S) return;
    const int s = (int)(e / n_s);
    if (active[s] == 0) return;
    double acc = w[e];
    for (int i = 0; i < m; ++i) acc -= coef[(size_t)s * coef_stride + i] * V[i * vstride + e];
    w[e] = acc;
}

// out = x * (1/sqrt(nrm2[s])) when nrm2 > 0
__global__ __launch_bounds__(GM_BLK) void gm_normalize_kernel(const double* __restrict__ x,
                                                              const double* __restrict__ nrm2, int nrm_stride,
                                                              double* __restrict__ out, size_t n_s, int S,
                                                              const int* __restrict__ active) {
    const size_t e = (size_t)blockIdx.x * GM_BLK + threadIdx.x;
    if (e >= n_s * S) return;
    const int s = (int)(e / n_s);
    if (active[s] == 0) return;
    const double q = nrm2[(size_t)s * nrm_stride];
    out[e] = q > 0.0 ? x[e] / sqrt(q) : 0.0;
}

// out = x / sqrt(||x||^2) over the shot's chunk, ||x||^2 summed by every block
// from the previous sweep's partials (product 0); block 0 of the shot stores
// it to nrm2 (the host's Hessenberg entry).  The arithmetic is that of
// gm_normalize_kernel after gm_reduce_kernel.
__global__ __launch_bounds__(GM_BLK) void gm_normalize_fused_kernel(const double* __restrict__ x,
                                                                    const double* __restrict__ pin,
                                                                    double* __restrict__ nrm2, int nrm_stride,
                                                                    double* __restrict__ out, size_t n_s,
                                                                    const int* __restrict__ active, int nblk) {
    __shared__ double red[GM_BLK / 64];
    const int s = blockIdx.y, b = blockIdx.x;
    if (active[s] == 0) return;
    const double q = partial_total(pin, s, 0, nblk, red);
    if (b == 0 && threadIdx.x == 0) nrm2[(size_t)s * nrm_stride] = q;
    const size_t base = (size_t)s * n_s;
    const size_t lo = (size_t)b * GM_CHUNK, hi = min(lo + GM_CHUNK, n_s);
    const double* xs = x + base;
    double* os = out + base;
    for (size_t e = lo + 2 * threadIdx.x; e < hi; e += 2 * GM_BLK) {   // element pairs (n_s, lo, hi even)
        const double2 v = *reinterpret_cast<const double2*>(xs + e);
        double2 r;
        r.x = q > 0.0 ? v.x / sqrt(q) : 0.0;
        r.y = q > 0.0 ? v.y / sqrt(q) : 0.0;
        *reinterpret_cast<double2*>(os + e) = r;
    }
}

// out = sum_{i<m} y[s][i] V_i
__global__ __launch_bounds__(GM_BLK) void gm_combine_kernel(const double* __restrict__ V, size_t vstride, int m,
                                                            const double* __restrict__ y, int y_stride,
                                                            double* __restrict__ out, size_t n_s, int S,
                                                            const int* __restrict__ active) {
    const size_t e = (size_t)blockIdx.x * GM_BLK + threadIdx.x;
    if (e >= n_s * S) return;
    const int s = (int)(e / n_s);
    if (active[s] == 0) return;
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc += y[(size_t)s * y_stride + i] * V[i * vstride + e];
    out[e] = acc;
}

// out = a + sa * b   (masked per shot)
__global__ __launch_bounds__(GM_BLK) void gm_axpy_kernel(const double* __restrict__ a, double sa,
                                                         const double* __restrict__ b, double* __restrict__ out,
                                                         size_t n_s, int S, const int* __restrict__ active) {
    const size_t e = (size_t)blockIdx.x * GM_BLK + threadIdx.x;
    if (e >= n_s * S) return;
    const int s = (int)(e / n_s);
    if (active[s] == 0) return;
    out[e] = a[e] + sa * b[e];
}

namespace {

struct GmState {
    double* V = nullptr;       // [k+1][nvec]
    double* w = nullptr;       // [nvec]
    double* z = nullptr;       // [nvec]
    double* partial = nullptr; // [S][MAXK+1][nblk]
    double* partial2 = nullptr;  // a second set
    double* dots = nullptr;    // [S][DS]
    int* active = nullptr;     // [S]
};

constexpr int DS = 2 * (GM_MAXK + 1) + 2;   // h (k+1), h2 (k+1), norm^2, restart beta^2
constexpr int GM_BETA_SLOT = DS - 1;

inline unsigned nblocks(size_t n) { return (unsigned)((n + GM_BLK - 1) / GM_BLK); }

}  // namespace

lg_status gmres_solve(lg_plan* p, const double* b, double* x, const lg_solve_opts* o, lg_solve_info* info) {
    if (p->prec != LG_FP64) return fail(LG_ERR_UNSUPPORTED, "GMRES is built for FP64 plans");
    const int k = o->restart;
    if (k > GM_MAXK) return fail(LG_ERR_UNSUPPORTED, "restart must be <= 32");
    const int S = p->S;
    const size_t n_s = 2 * p->npts, nvec = p->nvec;
    const int nblk = (int)((n_s + GM_CHUNK - 1) / GM_CHUNK);
    // workspace (grown on demand, owned by the plan)
    if (p->gm_k < k) {
        if (p->gm_V) (void)hipFree(p->gm_V);
        p->gm_V = nullptr;
        p->gm_k = 0;
        LG_HIP(hipMalloc((void**)&p->gm_V, (size_t)(k + 1) * nvec * 8));
        p->gm_k = k;
    }
    if (!p->gm_w) LG_HIP(hipMalloc((void**)&p->gm_w, nvec * 8));
    if (!p->gm_z) LG_HIP(hipMalloc((void**)&p->gm_z, nvec * 8));
    if (!p->gm_x)   // two partial sets (a sweep reads one while writing the other), dots, flags
        LG_HIP(hipMalloc((void**)&p->gm_x, (2 * (size_t)S * (GM_MAXK + 1) * nblk + (size_t)S * DS) * 8 + S * 4 + 64));
    if (!p->gm_hb) LG_HIP(hipHostMalloc((void**)&p->gm_hb, (size_t)2 * S * DS * 8, hipHostMallocDefault));
    for (hipEvent_t& e : p->gm_ev)
        if (!e) LG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    GmState g;
    g.V = p->gm_V;
    g.w = p->gm_w;
    g.z = p->gm_z;
    g.partial = p->gm_x;
    g.partial2 = g.partial + (size_t)S * (GM_MAXK + 1) * nblk;
    g.dots = g.partial2 + (size_t)S * (GM_MAXK + 1) * nblk;
    g.active = (int*)(g.dots + (size_t)S * DS);
    hipStream_t st = p->stream;
    const unsigned nb = nblocks(nvec);

    std::vector<int> act(S, 1), status(S, LG_ERR_NOT_CONVERGED), total(S, 0);
    std::vector<double> bnorm(S, 0.0), est(S, 1.0), dots_h((size_t)S * DS);
    auto push_active = [&]() -> hipError_t {
        return hipMemcpyAsync(g.active, act.data(), S * sizeof(int), hipMemcpyHostToDevice, st);
    };
    auto dot_into = [&](const double* Vb, size_t vstride, int m, const double* wv, int slot) -> hipError_t {
        hipLaunchKernelGGL(gm_multidot_kernel, dim3(nblk, S), dim3(GM_BLK), 0, st, Vb, vstride, m, wv, n_s,
                           g.active, g.partial, nblk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gm_reduce_kernel, dim3(S), dim3(GM_BLK), 0, st, g.partial, m, nblk, g.active,
                           g.dots + slot, DS);
        return hipGetLastError();
    };
    // one classical Gram-Schmidt subtraction fused with the sweep after it
    // (the inner products of the second pass, or the norm).  pin: the
    // previous sweep's per-block partials, from which every block sums the
    // coefficients (and stores them to dots at coef_slot), or nullptr (the
    // coefficients are read from dots); pout: this sweep's partials; reduce:
    // sum them into dots at out_slot with a separate kernel.  m > 16 takes
    // the separate kernels (coefficients from dots).
    auto subdot = [&](int m, int coef_slot, bool norm, int out_slot, const double* pin, double* pout,
                      bool reduce) -> hipError_t {
        const dim3 grid(nblk, S);
        double* cf = g.dots + coef_slot;
        if (m <= 8) {
            if (norm) hipLaunchKernelGGL((gm_subdot_kernel<8, true>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                         pin, g.w, n_s, g.active, pout, nblk);
            else hipLaunchKernelGGL((gm_subdot_kernel<8, false>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                    pin, g.w, n_s, g.active, pout, nblk);
        } else if (m <= 12) {
            if (norm) hipLaunchKernelGGL((gm_subdot_kernel<12, true>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                         pin, g.w, n_s, g.active, pout, nblk);
            else hipLaunchKernelGGL((gm_subdot_kernel<12, false>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                    pin, g.w, n_s, g.active, pout, nblk);
        } else if (m <= 16) {
            if (norm) hipLaunchKernelGGL((gm_subdot_kernel<16, true>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                         pin, g.w, n_s, g.active, pout, nblk);
            else hipLaunchKernelGGL((gm_subdot_kernel<16, false>), grid, dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS,
                                    pin, g.w, n_s, g.active, pout, nblk);
        } else {
            hipLaunchKernelGGL(gm_subtract_kernel, dim3(nb), dim3(GM_BLK), 0, st, g.V, nvec, m, cf, DS, g.w, n_s, S,
                               g.active);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return norm ? dot_into(g.w, 0, 1, g.w, out_slot) : dot_into(g.V, nvec, m, g.w, out_slot);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !reduce) return e;
        hipLaunchKernelGGL(gm_reduce_kernel, dim3(S), dim3(GM_BLK), 0, st, pout, norm ? 1 : m, nblk, g.active,
                           g.dots + out_slot, DS);
        return hipGetLastError();
    };
    auto fetch_dots = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(dots_h.data(), g.dots, (size_t)S * DS * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    };
    auto fin = [&](lg_status s) {
        int worst = LG_OK;
        for (int i = 0; i < S; ++i) {
            if (info) {
                info[i].iters = total[i];
                info[i].status = status[i];
                info[i].relres = bnorm[i] > 0 ? est[i] : 0.0;
            }
            auto sev = [](int v) { return v == LG_OK ? 0 : v == LG_ERR_NOT_CONVERGED ? 1 : v == LG_ERR_BREAKDOWN ? 2 : 3; };
            if (sev(status[i]) > sev(worst)) worst = status[i];
        }
        return s != LG_OK ? s : (lg_status)worst;
    };

    // ||b||, x = 0
    LG_HIP(push_active());
    LG_HIP(hipMemsetAsync(x, 0, nvec * 8, st));
    // the sweeps load element pairs (16 bytes): ||b|| from an aligned copy of b
    LG_HIP(hipMemcpyAsync(g.w, b, nvec * 8, hipMemcpyDeviceToDevice, st));
    LG_HIP(dot_into(g.w, 0, 1, g.w, 2 * (GM_MAXK + 1)));
    LG_HIP(fetch_dots());
    for (int s = 0; s < S; ++s) {
        const double bb = dots_h[(size_t)s * DS + 2 * (GM_MAXK + 1)];
        bnorm[s] = std::sqrt(bb);
        if (!std::isfinite(bnorm[s])) {
            status[s] = LG_ERR_NONFINITE;
            act[s] = 0;
            est[s] = NAN;
        } else if (bnorm[s] == 0.0) {
            status[s] = LG_OK;
            act[s] = 0;
            est[s] = 0.0;
        }
    }
    const double tol = o->tol;
    std::vector<double> H((size_t)S * (k + 1) * k), cs((size_t)S * k), sn((size_t)S * k), gv((size_t)S * (k + 1));
    std::vector<double> yv((size_t)S * (GM_MAXK + 1));
    std::vector<int> jused(S), cyc(S);
    bool first = true;
    for (int cycle = 0; cycle < 100000; ++cycle) {
        bool any = false;
        for (int s = 0; s < S; ++s) any = any || act[s];
        if (!any) break;
        LG_HIP(push_active());
        // r = b - C x  (first cycle: r = b), into V_0; beta = ||r||
        double* V0 = g.V;
        if (first) {
            LG_HIP(hipMemcpyAsync(V0, b, nvec * 8, hipMemcpyDeviceToDevice, st));
        } else {
            LG_HIP(launch_elastic_stencil(p, x, g.w));
            hipLaunchKernelGGL(gm_axpy_kernel, dim3(nb), dim3(GM_BLK), 0, st, b, -1.0, g.w, V0, n_s, S, g.active);
            LG_HIP(hipGetLastError());
        }
        first = false;
        // beta^2 goes to its own slot (the steps' sweeps do not touch it): V_0 =
        // r / beta is formed on the device and step 0 is queued at once; the
        // host reads beta with step 0's products and only then drops shots
        // whose residual already meets the tolerance (their step 0 and the
        // step queued after it write only their own unused basis vectors).
        LG_HIP(dot_into(V0, 0, 1, V0, GM_BETA_SLOT));
        hipLaunchKernelGGL(gm_normalize_kernel, dim3(nb), dim3(GM_BLK), 0, st, V0, g.dots + GM_BETA_SLOT, DS,
                           V0, n_s, S, g.active);
        LG_HIP(hipGetLastError());
        for (int s = 0; s < S; ++s) {
            cyc[s] = act[s];
            jused[s] = 0;
        }
        std::vector<int> inner = act;   // shots still in this cycle's Arnoldi
        // Arnoldi step j on the device: w = C K^{-1} v_j, classical Gram-Schmidt
        // twice, v_{j+1} = w / ||w||; its inner products then go to pinned host
        // set j % 2 and an event marks them.  Step j + 1 needs only v_{j+1}, so
        // it is queued before the host waits for step j's numbers (the GPU
        // works through it meanwhile).  A shot that stops at step j still runs
        // through that queued step (with the mask of step j), which writes only
        // v_{j+2} and scratch of that shot, never used for it.
        auto queue_step = [&](int j) -> hipError_t {
            double* Vj = g.V + (size_t)j * nvec;
            double* Vn = g.V + (size_t)(j + 1) * nvec;
            hipError_t e = launch_elastic_precond(p, Vj, g.z);
            if (e == hipSuccess) e = launch_elastic_stencil(p, g.z, g.w);
            const int m = j + 1;
            if (m <= 16) {
                // no reduction launches: pass-1 products (partials A); the pass-1
                // subtraction with the pass-2 products (coefficients summed from A,
                // partials B); the pass-2 subtraction with ||w||^2 (from B, partials
                // A); the normalisation (||w||^2 summed from A).  Each consumer
                // stores the sums it formed into dots for the host.
                if (e == hipSuccess) {
                    hipLaunchKernelGGL(gm_multidot_kernel, dim3(nblk, S), dim3(GM_BLK), 0, st, g.V, nvec, m, g.w, n_s,
                                       g.active, g.partial, nblk);
                    e = hipGetLastError();
                }
                if (e == hipSuccess) e = subdot(m, 0, false, GM_MAXK + 1, g.partial, g.partial2, false);
                if (e == hipSuccess) e = subdot(m, GM_MAXK + 1, true, 2 * (GM_MAXK + 1), g.partial2, g.partial, false);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(gm_normalize_fused_kernel, dim3(nblk, S), dim3(GM_BLK), 0, st, g.w, g.partial,
                                   g.dots + 2 * (GM_MAXK + 1), DS, Vn, n_s, g.active, nblk);
            } else {
                if (e == hipSuccess) e = dot_into(g.V, nvec, m, g.w, 0);                                 // pass 1
                if (e == hipSuccess) e = subdot(m, 0, false, GM_MAXK + 1, nullptr, g.partial, true);     // pass 2
                if (e == hipSuccess) e = subdot(m, GM_MAXK + 1, true, 2 * (GM_MAXK + 1), nullptr, g.partial, true);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(gm_normalize_kernel, dim3(nb), dim3(GM_BLK), 0, st, g.w,
                                   g.dots + 2 * (GM_MAXK + 1), DS, Vn, n_s, S, g.active);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            e = hipMemcpyAsync(p->gm_hb + (size_t)(j & 1) * S * DS, g.dots, (size_t)S * DS * 8,
                               hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipEventRecord(p->gm_ev[j & 1], st);
            return e;
        };
        {
            bool anyin = false;
            for (int s = 0; s < S; ++s) anyin = anyin || inner[s];
            if (anyin) LG_HIP(queue_step(0));
        }
        for (int j = 0; j < k; ++j) {
            bool anyin = false;
            for (int s = 0; s < S; ++s) anyin = anyin || inner[s];
            if (!anyin) break;
            if (j + 1 < k) LG_HIP(queue_step(j + 1));
            LG_HIP(hipEventSynchronize(p->gm_ev[j & 1]));
            const double* dset = p->gm_hb + (size_t)(j & 1) * S * DS;
            bool stopped = false;
            if (j == 0) {                // the restart residual's norm (see above)
                for (int s = 0; s < S; ++s) {
                    if (!inner[s]) continue;
                    const double beta = std::sqrt(dset[(size_t)s * DS + GM_BETA_SLOT]);
                    if (!std::isfinite(beta)) {
                        status[s] = LG_ERR_NONFINITE;
                        act[s] = cyc[s] = inner[s] = 0;
                        est[s] = NAN;
                        stopped = true;
                    } else if (beta <= tol * bnorm[s]) {
                        status[s] = LG_OK;
                        act[s] = cyc[s] = inner[s] = 0;
                        est[s] = beta / bnorm[s];
                        stopped = true;
                    } else {
                        std::fill(gv.begin() + (size_t)s * (k + 1), gv.begin() + (size_t)(s + 1) * (k + 1), 0.0);
                        gv[(size_t)s * (k + 1)] = beta;
                    }
                }
            }
            for (int s = 0; s < S; ++s) {
                if (!inner[s]) continue;
                const double* d = &dset[(size_t)s * DS];
                double* Hs = &H[(size_t)s * (k + 1) * k];
                auto Hc = [&](int r, int c) -> double& { return Hs[(size_t)r * k + c]; };
                for (int i = 0; i <= j; ++i) Hc(i, j) = d[i] + d[GM_MAXK + 1 + i];
                Hc(j + 1, j) = std::sqrt(d[2 * (GM_MAXK + 1)]);
                double* csv = &cs[(size_t)s * k];
                double* snv = &sn[(size_t)s * k];
                double* gs = &gv[(size_t)s * (k + 1)];
                for (int i = 0; i < j; ++i) {
                    const double tmp = csv[i] * Hc(i, j) + snv[i] * Hc(i + 1, j);
                    Hc(i + 1, j) = -snv[i] * Hc(i, j) + csv[i] * Hc(i + 1, j);
                    Hc(i, j) = tmp;
                }
                const double hj1 = Hc(j + 1, j);
                const double den = std::hypot(Hc(j, j), hj1);
                total[s] += 1;
                jused[s] = j + 1;
                if (den == 0.0) {
                    status[s] = LG_ERR_BREAKDOWN;
                    act[s] = inner[s] = cyc[s] = 0;
                    jused[s] = 0;
                    stopped = true;
                    continue;
                }
                csv[j] = Hc(j, j) / den;
                snv[j] = hj1 / den;
                Hc(j, j) = den;
                Hc(j + 1, j) = 0.0;
                gs[j + 1] = -snv[j] * gs[j];
                gs[j] = csv[j] * gs[j];
                est[s] = std::fabs(gs[j + 1]) / bnorm[s];
                if (!std::isfinite(est[s])) {
                    status[s] = LG_ERR_NONFINITE;
                    act[s] = inner[s] = cyc[s] = 0;
                    jused[s] = 0;
                    stopped = true;
                    continue;
                }
                if (est[s] <= tol || hj1 == 0.0) {
                    status[s] = LG_OK;
                    act[s] = 0;          // converged: finish after this cycle's update
                    inner[s] = 0;
                    stopped = true;
                } else if (total[s] >= o->max_iter) {
                    status[s] = LG_ERR_NOT_CONVERGED;
                    act[s] = 0;
                    inner[s] = 0;
                    stopped = true;
                }
            }
            // shots that stopped keep their basis; the kernels skip them from
            // the step after the one already queued
            if (stopped) {
                std::vector<int> mask = inner;
                LG_HIP(hipMemcpyAsync(g.active, mask.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
            }
        }
        // x += K^{-1} (V y) for every shot that ran an Arnoldi cycle
        bool anyupd = false;
        for (int s = 0; s < S; ++s) {
            const int m = cyc[s] ? jused[s] : 0;
            double* ys = &yv[(size_t)s * (GM_MAXK + 1)];
            std::fill(ys, ys + GM_MAXK + 1, 0.0);
            if (m == 0) continue;
            anyupd = true;
            const double* Hs = &H[(size_t)s * (k + 1) * k];
            const double* gs = &gv[(size_t)s * (k + 1)];
            for (int i = m - 1; i >= 0; --i) {
                double acc = gs[i];
                for (int c = i + 1; c < m; ++c) acc -= Hs[(size_t)i * k + c] * ys[c];
                ys[i] = acc / Hs[(size_t)i * k + i];
            }
        }
        if (!anyupd) continue;
        std::vector<int> upd(S);
        int mmax = 0;
        for (int s = 0; s < S; ++s) {
            upd[s] = (cyc[s] && jused[s] > 0) ? 1 : 0;
            mmax = std::max(mmax, upd[s] ? jused[s] : 0);
        }
        LG_HIP(hipMemcpyAsync(g.dots, yv.data(), (size_t)S * (GM_MAXK + 1) * 8, hipMemcpyHostToDevice, st));
        LG_HIP(hipMemcpyAsync(g.active, upd.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(gm_combine_kernel, dim3(nb), dim3(GM_BLK), 0, st, g.V, nvec, mmax, g.dots, GM_MAXK + 1,
                           g.w, n_s, S, g.active);
        LG_HIP(hipGetLastError());
        LG_HIP(launch_elastic_precond(p, g.w, g.z));
        hipLaunchKernelGGL(gm_axpy_kernel, dim3(nb), dim3(GM_BLK), 0, st, x, 1.0, g.z, x, n_s, S, g.active);
        LG_HIP(hipGetLastError());
        // no wait here: the next cycle's work is stream-ordered after this update
    }
    LG_HIP(hipStreamSynchronize(st));
    return fin(LG_OK);
}

}  // namespace lg
