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

// Stockham autosort FFT (forward, natural order in and out) of length M held
// in LDS, executed by TPF = M/R threads of the block (t = 0..TPF-1), each
// doing R/r radix-r butterflies per pass; r = R except for the last pass.
// Every pass: read inputs -> barrier -> twiddle + DFT -> write -> barrier.
// All threads of the block must call this (it contains __syncthreads).
template <typename T, int M, int R, int Ns>
__device__ __forceinline__ void fft_passes(cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ tw,
                                           int t) {
    if constexpr (Ns < M) {
        constexpr int r = (M / Ns >= R) ? R : (M / Ns);
        constexpr int NB = R / r;
        constexpr int TPF = M / R;
        cpx<T> v[R];
#pragma unroll
        for (int qb = 0; qb < NB; ++qb) {
            const int bi = t + qb * TPF;
#pragma unroll
            for (int u = 0; u < r; ++u) v[qb * r + u] = buf[lpad(bi + u * (M / r))];
        }
        __syncthreads();
#pragma unroll
        for (int qb = 0; qb < NB; ++qb) {
            const int bi = t + qb * TPF;
            const int k = bi & (Ns - 1);
            if constexpr (Ns > 1) {
#pragma unroll
                for (int u = 1; u < r; ++u) {
                    const cpx<T> w = tw[(u * k) * (M / (Ns * r))];
                    v[qb * r + u] = cmul(v[qb * r + u], w);
                }
            }
            dft<T, r>(&v[qb * r]);
            const int base = (bi - k) * r + k;
#pragma unroll
            for (int u = 0; u < r; ++u) buf[lpad(base + u * Ns)] = v[qb * r + u];
        }
        __syncthreads();
        fft_passes<T, M, R, Ns * r>(buf, tw, t);
    }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
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
