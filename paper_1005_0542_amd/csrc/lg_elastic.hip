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
// orthogonalised by classical Gram-Schmidt applied twice, with the second pass
// of each vector delayed into the next step (two sweeps over the basis per
// step).  Every vector operation and inner product runs on the device, which
// also keeps the Hessenberg columns it needs for the delayed pass; the host
// applies the Givens rotations to its copy and tests convergence.
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
    // P > 1: the segment correction inside the inverse transform; with the
    // traction-free surface also its rank-one term, whose coefficients come
    // from the corrected row 1 (formed from the uncorrected result first)
    if (p->blk[0].P > 1) {
        if (e == hipSuccess && p->el_free) e = launch_surface_coef_fused(p, p->y, S * 2);
        return e == hipSuccess ? launch_correct_inv(p, z, S * 2, p->el_free) : e;
    }
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

// ---------------------------------------------------------------------------
// Arnoldi with delayed reorthogonalisation: classical Gram-Schmidt twice, the
// second pass (and the normalisation) of q_j carried out inside step j + 1's
// two sweeps, so a step reads the basis twice instead of three times.
//
// Step j starts from q_0..q_{j-1} (final, orthonormal) and t = V_j, which is
// A q_{j-1} after one projection pass (t = A q_{j-1} - Q h, h the pass-1
// coefficients of column j-1), neither reprojected nor normalised; at j = 0,
// t = q_0 itself (final).  With u = A t (the operator applied to t):
//   sweep 1:  a_i = (q_i, t) and b_i = (q_i, u) for i < j, (t, t), (t, u);
//   q_j = (t - Q a) / rho with rho^2 = (t, t) - |a|^2 (at j = 0: rho = 1,
//     a = 0), so column j-1 of H is final: H[i][j-1] = h_i + a_i (i < j),
//     H[j][j-1] = rho;
//   A q_j = (u - Q_{j+1} d) / rho with d = H[0..j][0..j-1] a (from the
//     Arnoldi relation of the earlier columns); its pass-1 coefficients
//     g_i = (q_i, A q_j) are (b_i - d_i) / rho for i < j and
//     g_j = ((t, u) - a.b) / rho^2 - d_j / rho;
//   sweep 2:  q_j stored over t, and step j + 1's
//     t' = A q_j - Q_{j+1} g = u / rho - Q_{j+1} c,  c = d / rho + g.
// rho^2 is a difference of a squared norm and the squares of the small
// second-pass coefficients (t is already orthogonal to Q up to rounding), so
// no cancellation occurs.  The end of a cycle runs sweep 1 without u and the
// coefficient step only, to finalise the last column.
// ---------------------------------------------------------------------------
constexpr int GM_NS = 2 * GM_MAXK + 2;           // products per shot: a, b, (t,t), (t,u)
constexpr int GM_HDS = (GM_MAXK + 1) * (GM_MAXK + 1);   // per shot: H (k+1) x k, then h

// Sweep 1: per-block partials of the products of step j (u == nullptr: a and
// (t, t) only).  Basis vectors 8 at a time; t, u and (t, t), (t, u) in the
// first group.  Partials at pd[(s GM_NS + slot) nblk + b]: a_i at slot i,
// b_i at GM_MAXK + i, (t, t) at 2 GM_MAXK, (t, u) at 2 GM_MAXK + 1.
__global__ __launch_bounds__(GM_BLK) void gm_dcgs_dots_kernel(const double* __restrict__ V, size_t vstride, int j,
                                                              const double* __restrict__ u, size_t n_s,
                                                              const int* __restrict__ active,
                                                              double* __restrict__ pd, int nblk) {
    constexpr int G = 8;
    constexpr int NV = 2 * G + 2;                 // products of one group: a, b, (t,t), (t,u)
    __shared__ double red[NV][GM_BLK / 64];
    const int s = blockIdx.y, b = blockIdx.x;
    if (active[s] == 0) return;
    const size_t base = (size_t)s * n_s;
    const size_t lo = (size_t)b * GM_CHUNK, hi = min(lo + GM_CHUNK, n_s);
    const uint32_t nbytes = (uint32_t)(n_s * 8);
    const bool hu = u != nullptr;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const rsrc_t rt = buf_rsrc(V + (size_t)j * vstride + base, nbytes);
    const rsrc_t ru = buf_rsrc(hu ? u + base : V, hu ? nbytes : 0u);
    double* const ps = pd + (size_t)s * GM_NS * nblk + b;
    for (int i0 = 0; i0 == 0 || i0 < j; i0 += G) {   // uniform over the block
        rsrc_t rv[G];
#pragma unroll
        for (int q = 0; q < G; ++q) rv[q] = buf_rsrc(V + (size_t)(i0 + q) * vstride + base, i0 + q < j ? nbytes : 0u);
        double aa[G], ab[G], tt = 0.0, tu = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) aa[q] = ab[q] = 0.0;
        for (size_t e = lo + 2 * threadIdx.x; e < hi; e += 2 * GM_BLK) {   // element pairs (n_s, lo, hi even)
            const uint32_t off = (uint32_t)(e * 8);
            const cpx<double> tv = bload2<double>(rt, off);
            const cpx<double> uv = bload2<double>(ru, off);
            cpx<double> vv[G];
#pragma unroll
            for (int q = 0; q < G; ++q) vv[q] = bload2<double>(rv[q], off);
#pragma unroll
            for (int q = 0; q < G; ++q) {
                aa[q] += vv[q].x * tv.x;
                aa[q] += vv[q].y * tv.y;
                ab[q] += vv[q].x * uv.x;
                ab[q] += vv[q].y * uv.y;
            }
            if (i0 == 0) {
                tt += tv.x * tv.x;
                tt += tv.y * tv.y;
                tu += tv.x * uv.x;
                tu += tv.y * uv.y;
            }
        }
        // block sums (wave trees, then the waves in order): value v of the
        // group is a_{i0+v} (v < G), b_{i0+v-G} (v < 2G), (t,t), (t,u)
#pragma unroll
        for (int q = 0; q < G; ++q) {
            aa[q] = wave_sum(aa[q]);
            ab[q] = wave_sum(ab[q]);
        }
        tt = wave_sum(tt);
        tu = wave_sum(tu);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                red[q][wave] = aa[q];
                red[G + q][wave] = ab[q];
            }
            red[2 * G][wave] = tt;
            red[2 * G + 1][wave] = tu;
        }
        __syncthreads();
        const int v = threadIdx.x;
        if (v < NV) {
            const bool isa = v < G, isb = v >= G && v < 2 * G;
            const int i = isa ? i0 + v : i0 + v - G;
            const bool want = (isa && i < j) || (isb && hu && i < j) || (i0 == 0 && v == 2 * G) ||
                              (i0 == 0 && hu && v == 2 * G + 1);
            if (want) {
                double t = 0.0;
                for (int w = 0; w < GM_BLK / 64; ++w) t += red[v][w];
                const int slot = isa ? i : isb ? GM_MAXK + i : 2 * GM_MAXK + (v - 2 * G);
                ps[(size_t)slot * nblk] = t;
            }
        }
        __syncthreads();                           // red is reused by the next group
    }
}

// Coefficients of step j, one block per shot: the products summed from the
// partials (one wave per product, lanes over the blocks in a fixed order),
// then rho, the final column j-1 of H (into Hd and, for the host, dots[0..j]),
// and (fin == 0) the sweep-2 coefficients coef = [a (GM_MAXK), c (GM_MAXK + 1),
// 1/rho] and g as the next column's h.  rho = 0 (t in the span of Q: an exact
// solution) gives 1/rho = 0 and c = g = 0; the host stops the shot there.
constexpr int GM_COEF_THREADS = 1024;
__global__ __launch_bounds__(GM_COEF_THREADS) void gm_dcgs_coef_kernel(const double* __restrict__ pd, int nblk, int j,
                                                              int fin, const int* __restrict__ active,
                                                              double* __restrict__ Hd, double* __restrict__ coef,
                                                              double* __restrict__ dots, int dstride) {
    __shared__ double sv[GM_NS];
    __shared__ double scol[GM_MAXK + 1];
    __shared__ double sd[GM_MAXK + 1];
    __shared__ double srho, sab;
    const int s = blockIdx.x;
    if (active[s] == 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double* ps = pd + (size_t)s * GM_NS * nblk;
    for (int v = wave; v < GM_NS; v += GM_COEF_THREADS / 64) {   // uniform per wave
        const bool need = (v < GM_MAXK) ? v < j
                        : (v < 2 * GM_MAXK) ? (!fin && v - GM_MAXK < j)
                        : (v == 2 * GM_MAXK || !fin);
        if (!need) continue;
        // lane sums blocks lane, lane + 64, ... in that order, 8 loads in flight
        double acc = 0.0;
        for (int b0 = lane; b0 < nblk; b0 += 64 * 8) {
            double x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = b0 + 64 * q < nblk ? ps[(size_t)v * nblk + b0 + 64 * q] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += x[q];
        }
        acc = wave_sum(acc);
        if (lane == 0) sv[v] = acc;
    }
    __syncthreads();
    double* H = Hd + (size_t)s * GM_HDS;         // H[r][c] at r GM_MAXK + c
    double* h = H + (GM_MAXK + 1) * GM_MAXK;     // pass-1 coefficients of the latest column
    if (threadIdx.x == 0) {
        double rho = 1.0;
        if (j > 0) {
            double aa = 0.0, ab = 0.0;
            for (int i = 0; i < j; ++i) {
                aa += sv[i] * sv[i];
                if (!fin) ab += sv[i] * sv[GM_MAXK + i];
            }
            const double r2 = sv[2 * GM_MAXK] - aa;
            rho = r2 > 0.0 ? sqrt(r2) : (r2 == 0.0 || isfinite(r2) ? 0.0 : r2);   // NaN passes to the host
            for (int i = 0; i < j; ++i) scol[i] = h[i] + sv[i];
            scol[j] = rho;
            for (int i = 0; i <= j; ++i) {
                H[(size_t)i * GM_MAXK + (j - 1)] = scol[i];
                dots[(size_t)s * dstride + i] = scol[i];
            }
            sab = ab;
        } else {
            sab = 0.0;
        }
        srho = rho;
    }
    __syncthreads();
    if (fin) return;
    const double rho = srho;
    const bool ok = rho > 0.0;                    // false also for NaN
    const double ir = ok ? 1.0 / rho : 0.0;
    // d = H[0..j][0..j-1] a (Hessenberg: row r has columns c >= r - 1)
    const int r = threadIdx.x;
    if (r <= j) {
        double d = 0.0;
        for (int c = (r > 0 ? r - 1 : 0); c < j; ++c)
            d += (c == j - 1 ? scol[r] : H[(size_t)r * GM_MAXK + c]) * sv[c];
        sd[r] = d;
    }
    __syncthreads();
    if (r <= j) {
        const double d = sd[r];
        double g = r < j ? (sv[GM_MAXK + r] - d) * ir : ((sv[2 * GM_MAXK + 1] - sab) * ir - d) * ir;
        double c = d * ir + g;
        if (!ok) g = c = 0.0;
        h[r] = g;
        coef[(size_t)s * GM_NS + GM_MAXK + r] = c;
        if (r < j) coef[(size_t)s * GM_NS + r] = sv[r];
    }
    if (r == 0) coef[(size_t)s * GM_NS + 2 * GM_MAXK + 1] = ir;
}

// Sweep 2 of step j: q_j = (t - Q a) / rho over V_j and t' = u / rho - Q c
// - c_j q_j into V_{j+1}, coefficients from gm_dcgs_coef_kernel.
__global__ __launch_bounds__(GM_BLK) void gm_dcgs_update_kernel(double* __restrict__ V, size_t vstride, int j,
                                                                const double* __restrict__ u,
                                                                const double* __restrict__ coef, size_t n_s,
                                                                const int* __restrict__ active) {
    constexpr int G = 8;
    __shared__ double sa[GM_MAXK], sc[GM_MAXK + 1];
    const int s = blockIdx.y, b = blockIdx.x;
    if (active[s] == 0) return;
    const double* cs = coef + (size_t)s * GM_NS;
    if (threadIdx.x < j) sa[threadIdx.x] = cs[threadIdx.x];
    if (threadIdx.x <= j) sc[threadIdx.x] = cs[GM_MAXK + threadIdx.x];
    const double ir = cs[2 * GM_MAXK + 1];
    __syncthreads();
    const size_t base = (size_t)s * n_s;
    const size_t lo = (size_t)b * GM_CHUNK, hi = min(lo + GM_CHUNK, n_s);
    const uint32_t nbytes = (uint32_t)(n_s * 8);
    const rsrc_t rt = buf_rsrc(V + (size_t)j * vstride + base, nbytes);
    const rsrc_t rn = buf_rsrc(V + (size_t)(j + 1) * vstride + base, nbytes);
    const rsrc_t ru = buf_rsrc(u + base, nbytes);
    const double cj = sc[j];
    for (size_t e = lo + 2 * threadIdx.x; e < hi; e += 2 * GM_BLK) {   // element pairs (n_s, lo, hi even)
        const uint32_t off = (uint32_t)(e * 8);
        const cpx<double> tv = bload2<double>(rt, off);
        const cpx<double> uv = bload2<double>(ru, off);
        cpx<double> qa = {0.0, 0.0}, qc = {0.0, 0.0};
        for (int i0 = 0; i0 < j; i0 += G) {
            cpx<double> vv[G];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const rsrc_t rv = buf_rsrc(V + (size_t)(i0 + q) * vstride + base, i0 + q < j ? nbytes : 0u);
                vv[q] = bload2<double>(rv, off);
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (i0 + q < j) {
                    const double ai = sa[i0 + q], ci = sc[i0 + q];
                    qa.x += ai * vv[q].x;
                    qa.y += ai * vv[q].y;
                    qc.x += ci * vv[q].x;
                    qc.y += ci * vv[q].y;
                }
            }
        }
        cpx<double> qj, tn;
        qj.x = (tv.x - qa.x) * ir;
        qj.y = (tv.y - qa.y) * ir;
        tn.x = uv.x * ir - qc.x - cj * qj.x;
        tn.y = uv.y * ir - qc.y - cj * qj.y;
        bstore2(qj, rt, off);
        bstore2(tn, rn, off);
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
    double* partial = nullptr; // [S][MAXK+1][nblk] (single products); [S][GM_NS][nblk] (Arnoldi steps)
    double* dots = nullptr;    // [S][DS]
    double* coef = nullptr;    // [S][GM_NS]: a step's sweep-2 coefficients
    double* Hd = nullptr;      // [S][GM_HDS]: H and the latest pass-1 coefficients
    int* active = nullptr;     // [S]
};

constexpr int DS = 2 * (GM_MAXK + 1) + 2;   // a final Hessenberg column (k+1), ..., restart beta^2
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
    if (!p->gm_x)   // partials, dots, step coefficients, H, flags
        LG_HIP(hipMalloc((void**)&p->gm_x,
                         ((size_t)S * GM_NS * nblk + (size_t)S * (DS + GM_NS + GM_HDS)) * 8 + S * 4 + 64));
    if (!p->gm_hb) LG_HIP(hipHostMalloc((void**)&p->gm_hb, (size_t)2 * S * DS * 8, hipHostMallocDefault));
    for (hipEvent_t& e : p->gm_ev)
        if (!e) LG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    GmState g;
    g.V = p->gm_V;
    g.w = p->gm_w;
    g.z = p->gm_z;
    g.partial = p->gm_x;
    g.dots = g.partial + (size_t)S * GM_NS * nblk;
    g.coef = g.dots + (size_t)S * DS;
    g.Hd = g.coef + (size_t)S * GM_NS;
    g.active = (int*)(g.Hd + (size_t)S * GM_HDS);
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
        // Arnoldi step j on the device (delayed reorthogonalisation, see the
        // kernels): u = C K^{-1} t_j, sweep 1, the coefficients, sweep 2 (q_j
        // final, t_{j+1}); step k (the end of the cycle) only finalises column
        // k-1.  Event j marks the final column j-1 (j >= 1) in pinned host set
        // j % 2.  Step j + 1 needs nothing from the host, so it is queued
        // before the host waits for event j (the GPU works through it
        // meanwhile).  A shot that stops at event j still runs through the
        // steps already queued (with the mask of step j), which write only its
        // basis vectors past the ones in use and scratch, never used for it.
        auto queue_step = [&](int j) -> hipError_t {
            const bool fin = j == k;
            hipError_t e = hipSuccess;
            if (!fin) {
                e = launch_elastic_precond(p, g.V + (size_t)j * nvec, g.z);
                if (e == hipSuccess) e = launch_elastic_stencil(p, g.z, g.w);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(gm_dcgs_dots_kernel, dim3(nblk, S), dim3(GM_BLK), 0, st, g.V, nvec, j,
                               fin ? nullptr : g.w, n_s, g.active, g.partial, nblk);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(gm_dcgs_coef_kernel, dim3(S), dim3(GM_COEF_THREADS), 0, st, g.partial, nblk, j,
                               fin ? 1 : 0,
                               g.active, g.Hd, g.coef, g.dots, DS);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (!fin) {
                hipLaunchKernelGGL(gm_dcgs_update_kernel, dim3(nblk, S), dim3(GM_BLK), 0, st, g.V, nvec, j, g.w,
                                   g.coef, n_s, g.active);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
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
        // event j: the restart norm (j = 0) or the final column j - 1 of H
        for (int j = 0; j <= k; ++j) {
            bool anyin = false;
            for (int s = 0; s < S; ++s) anyin = anyin || inner[s];
            if (!anyin) break;
            if (j + 1 <= k) LG_HIP(queue_step(j + 1));
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
            const int c = j - 1;         // the column this event completes
            for (int s = 0; s < S && c >= 0; ++s) {
                if (!inner[s]) continue;
                const double* d = &dset[(size_t)s * DS];
                double* Hs = &H[(size_t)s * (k + 1) * k];
                auto Hc = [&](int r, int cc) -> double& { return Hs[(size_t)r * k + cc]; };
                for (int i = 0; i <= c + 1; ++i) Hc(i, c) = d[i];
                double* csv = &cs[(size_t)s * k];
                double* snv = &sn[(size_t)s * k];
                double* gs = &gv[(size_t)s * (k + 1)];
                for (int i = 0; i < c; ++i) {
                    const double tmp = csv[i] * Hc(i, c) + snv[i] * Hc(i + 1, c);
                    Hc(i + 1, c) = -snv[i] * Hc(i, c) + csv[i] * Hc(i + 1, c);
                    Hc(i, c) = tmp;
                }
                const double hj1 = Hc(c + 1, c);
                const double den = std::hypot(Hc(c, c), hj1);
                total[s] += 1;
                jused[s] = c + 1;
                if (den == 0.0) {
                    status[s] = LG_ERR_BREAKDOWN;
                    act[s] = inner[s] = cyc[s] = 0;
                    jused[s] = 0;
                    stopped = true;
                    continue;
                }
                csv[c] = Hc(c, c) / den;
                snv[c] = hj1 / den;
                Hc(c, c) = den;
                Hc(c + 1, c) = 0.0;
                gs[c + 1] = -snv[c] * gs[c];
                gs[c] = csv[c] * gs[c];
                est[s] = std::fabs(gs[c + 1]) / bnorm[s];
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
