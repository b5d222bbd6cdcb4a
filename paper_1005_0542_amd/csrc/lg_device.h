// Device-side building blocks shared by the gfx950 kernels: complex helpers,
// small in-register DFTs, the LDS Stockham FFT and wave/block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lg_internal.h"

namespace lg {

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// cos(2 pi j / 16) for j = 0..15 (exact constants; sin via a quarter shift)
__host__ __device__ constexpr double cos16(int j) {
    j &= 15;
    return j == 0 ? 1.0
         : j == 1 ? 0.92387953251128675613
         : j == 2 ? 0.70710678118654752440
         : j == 3 ? 0.38268343236508977173
         : j == 4 ? 0.0
         : j == 5 ? -0.38268343236508977173
         : j == 6 ? -0.70710678118654752440
         : j == 7 ? -0.92387953251128675613
         : j == 8 ? -1.0
         : j == 9 ? -0.92387953251128675613
         : j == 10 ? -0.70710678118654752440
         : j == 11 ? -0.38268343236508977173
         : j == 12 ? 0.0
         : j == 13 ? 0.38268343236508977173
         : j == 14 ? 0.70710678118654752440
         : 0.92387953251128675613;
}
__host__ __device__ constexpr double sin16(int j) { return cos16(j - 4); }

// In-register forward DFT of length r (power of two, r <= 16):
//   V_k = sum_u v_u exp(-2 pi i u k / r),
// by recursive radix-2 decimation in time with compile-time twiddles.
template <typename T, int r>
__device__ __forceinline__ void dft(cpx<T>* v) {
    if constexpr (r == 2) {
        cpx<T> a = v[0], b = v[1];
        v[0] = {a.x + b.x, a.y + b.y};
        v[1] = {a.x - b.x, a.y - b.y};
    } else if constexpr (r > 2) {
        constexpr int h = r / 2;
        cpx<T> e[h], o[h];
#pragma unroll
        for (int u = 0; u < h; ++u) {
            e[u] = v[2 * u];
            o[u] = v[2 * u + 1];
        }
        dft<T, h>(e);
        dft<T, h>(o);
#pragma unroll
        for (int k = 0; k < h; ++k) {
            cpx<T> t;
            const int j = k * (16 / r);
            if (j == 0) {
                t = o[k];
            } else if (j == 4) {            // multiply by -i
                t = {o[k].y, -o[k].x};
            } else {
                const T wr = (T)cos16(j), wi = (T)(-sin16(j));
                t = {o[k].x * wr - o[k].y * wi, o[k].x * wi + o[k].y * wr};
            }
            v[k] = {e[k].x + t.x, e[k].y + t.y};
            v[k + h] = {e[k].x - t.x, e[k].y - t.y};
        }
    }
}

// LDS index with one element of padding every 16 complex elements, which
// breaks the power-of-two strides of the first Stockham passes across banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
template <int M>
struct LdsLen {
    static constexpr int value = M + M / 16;
};

// Pass structure of a length-M Stockham FFT with radix-R passes: every pass
// but the last has radix R; the last pass has radix R_LAST = M / NS_LAST.
template <int M, int R>
struct FftPlan {
    static constexpr int ns_last() {
        int ns = 1;
        while (ns * R < M) ns *= R;
        return ns;
    }
    static constexpr int NS_LAST = ns_last();
    static constexpr int R_LAST = M / NS_LAST;
    static constexpr int NB_LAST = R / R_LAST;   // last-pass butterflies per thread
};

// Twiddles w[u] = tw[u j] (u < r) of one butterfly from at most four table
// loads (u = 1, 2, 4, 8); the others are products of at most three factors.
template <typename T, int r>
__device__ __forceinline__ void make_twiddles(const cpx<T>* __restrict__ tw, int j, cpx<T>* w) {
    w[0] = {(T)1, (T)0};
    if constexpr (r >= 2) w[1] = tw[j];
    if constexpr (r >= 4) {
        w[2] = tw[2 * j];
        w[3] = cmul(w[2], w[1]);
    }
    if constexpr (r >= 8) {
        w[4] = tw[4 * j];
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
    if constexpr (r >= 16) {
        w[8] = tw[8 * j];
#pragma unroll
        for (int u = 9; u < 16; ++u) w[u] = cmul(w[8], w[u - 8]);
    }
}

// Stockham passes (LDS -> LDS) of span Ns .. NS_LAST/R, radix R, one
// butterfly per thread: read -> barrier -> twiddle + DFT -> write -> barrier
// (no twiddles for the span-1 pass).  The last pass is fft_last.  All threads
// of the block must call this.  tw[TS j] = exp(-2 pi i j / M): a table of
// TS M entries serves a transform of length M with stride TS.
template <typename T, int M, int R, int Ns, int TS = 1>
__device__ __forceinline__ void fft_mid(cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ tw, int t) {
    if constexpr (Ns < FftPlan<M, R>::NS_LAST) {
        cpx<T> v[R];
#pragma unroll
        for (int u = 0; u < R; ++u) v[u] = buf[lpad(t + u * (M / R))];
        __syncthreads();
        const int k = t & (Ns - 1);
        if constexpr (Ns > 1) {
            cpx<T> w[R];
            make_twiddles<T, R>(tw, TS * k * (M / (Ns * R)), w);
#pragma unroll
            for (int u = 1; u < R; ++u) v[u] = cmul(v[u], w[u]);
        }
        dft<T, R>(v);
        const int base = (t - k) * R + k;
#pragma unroll
        for (int u = 0; u < R; ++u) buf[lpad(base + u * Ns)] = v[u];
        __syncthreads();
        fft_mid<T, M, R, Ns * R, TS>(buf, tw, t);
    }
}

// Last Stockham pass (span NS_LAST, radix R_LAST): reads LDS, leaves the
// results in registers: v[qb*R_LAST + u] is output K = t + qb*(M/R) + u*NS_LAST.
template <typename T, int M, int R, int TS = 1>
__device__ __forceinline__ void fft_last(const cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ tw,
                                         int t, cpx<T>* v) {
    using FP = FftPlan<M, R>;
    constexpr int r = FP::R_LAST, NB = FP::NB_LAST, Ns = FP::NS_LAST, TPF = M / R;
#pragma unroll
    for (int qb = 0; qb < NB; ++qb)
#pragma unroll
        for (int u = 0; u < r; ++u) v[qb * r + u] = buf[lpad(t + qb * TPF + u * Ns)];
#pragma unroll
    for (int qb = 0; qb < NB; ++qb) {
        const int k = t + qb * TPF;               // < Ns: the twiddle index is k itself
        cpx<T> w[r];
        make_twiddles<T, r>(tw, TS * k, w);
#pragma unroll
        for (int u = 1; u < r; ++u) v[qb * r + u] = cmul(v[qb * r + u], w[u]);
        dft<T, r>(&v[qb * r]);
    }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2: hardware block b runs on XCD b % 8.  xcd_linear maps b to a logical
// index so that every XCD works through one contiguous range of logical
// indices (a bijection of [0, n)); kernels order their tiles so that tiles
// sharing cache lines (halo rows and columns, medium rows) are neighbours in
// that order and therefore meet in the same L2.
constexpr int NUM_XCD = 8;

// A pointer that every lane holds the same value of but that the compiler
// cannot prove uniform (it was loaded from memory): taken through
// readfirstlane, so buffer resources built on it stay in scalar registers
// instead of a per-lane loop around every load and store that uses them.
template <typename P>
__device__ __forceinline__ P* wave_uniform(P* ptr) {
    const uint64_t v = (uint64_t)ptr;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P*)(((uint64_t)hi << 32) | (uint64_t)lo);
}
__device__ __forceinline__ int xcd_linear(int b, int n) {
    const int q = n / NUM_XCD, r = n - q * NUM_XCD;
    const int x = b % NUM_XCD, i = b / NUM_XCD;
    return x * q + min(x, r) + i;
}

// Raw buffer addressing.  A resource covers nbytes from a wave-uniform base;
// a load at a byte offset outside [0, nbytes) returns 0 and a store there is
// dropped (the hardware range check).  Out-of-grid neighbours (the Dirichlet
// zero) and padding lanes therefore need no branch, and every load of a
// strip is issued back to back.
constexpr uint32_t BUF_OOB = 0xFFFFFFF0u;     // an offset beyond any resource
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t buf_rsrc(const void* base, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// a pair of consecutive values (one 8- or 16-byte load)
template <typename T>
__device__ __forceinline__ cpx<T> bload2(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ cpx<float> bload2<float>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cpx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ cpx<double> bload2<double>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(cpx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

// a pair of consecutive doubles (one 16-byte store)
__device__ __forceinline__ void bstore2(cpx<double> v, rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t, v), r,
                                           (int)off, 0, 0);
}

template <typename T>
__device__ __forceinline__ void bstore(T v, rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ void bstore<float>(float v, rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void bstore<double>(double v, rsrc_t r, uint32_t off) {
    using u2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, 0);
}

template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c);
template <>
__device__ __forceinline__ float fmad<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmad<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The 5-point operator at one node (Sec. 2.3, SPD sign):
//   [fE (c - pE) + fW (c - pW)] / dx^2 + [fS (c - pS) + fN (c - pN)] / dz^2 + w c
// with explicit fused multiply-adds, so every kernel that evaluates it (the
// operator, the fused CG update) produces bitwise the same value.
template <typename T>
__device__ __forceinline__ T stencil_point(T c, T pE, T pW, T pS, T pN, T fE, T fW, T fS, T fN, T w,
                                           T idx2, T idz2) {
    const T sx = fmad(fE, c - pE, fW * (c - pW));
    const T sz = fmad(fS, c - pS, fN * (c - pN));
    return fmad(sx, idx2, fmad(sz, idz2, w * c));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum (fixed tree); result valid in every thread.
// `scratch` needs blockDim.x/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    return s;
}

}  // namespace lg
