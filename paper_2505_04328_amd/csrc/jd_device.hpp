// Device-side building blocks of the hot path for gfx950: the counter-based
// draws, the Euler-Maruyama step, the adjoint step and the deterministic FP64
// block reduction.  Everything a forward sweep and a recomputing adjoint sweep
// share lives here, so that both evaluate bit-identical steps (the library is
// built with -ffp-contract=off and every fused multiply-add is written out).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jd {

constexpr int kThreads = 256;  // threads per block of every sweep kernel

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The counter word c0 is
// the path index (lane-varying); c1..c3 and the key are wave-uniform, so the
// compiler keeps the key schedule on the scalar unit.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t* out) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Uniform in [2^-24, 1 - 2^-24] from the top 24 bits of a word (lowest forced
// to one); exact in both precisions.
template <typename Real>
__device__ __forceinline__ Real unit_uniform(uint32_t w) {
    return (Real)((w >> 8) | 1u) * (Real)(1.0 / 16777216.0);
}

// Box-Muller pair from two words: cosine branch and sine branch.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& zc, float& zs) {
    const float r = sqrtf(-2.0f * logf(unit_uniform<float>(a)));
    float s, c;
    sincospif(2.0f * unit_uniform<float>(b), &s, &c);
    zc = r * c;
    zs = r * s;
}
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& zc, double& zs) {
    const double r = sqrt(-2.0 * log(unit_uniform<double>(a)));
    double s, c;
    sincospi(2.0 * unit_uniform<double>(b), &s, &c);
    zc = r * c;
    zs = r * s;
}

// Inverse-CDF Poisson thresholds, prepared on the host (kernel argument).
struct PoissonThresholds {
    uint64_t t[32];
};

// Word made of the low bytes of the four words of Philox block 0.
__device__ __forceinline__ uint32_t poisson_word(const uint32_t* w) {
    return (w[0] & 0xFFu) | ((w[1] & 0xFFu) << 8) | ((w[2] & 0xFFu) << 16) | (w[3] << 24);
}

// Smallest j with P < thr_j.  The first comparison is the common case; the
// loop runs only in lanes that jump, with a wave-uniform index.
__device__ __forceinline__ int poisson_count(uint32_t P, const PoissonThresholds& thr) {
    const uint64_t p = (uint64_t)P;
    int n = 0;
    if (p >= thr.t[0]) {
        n = 1;
        for (int j = 1; j < 31; ++j) {
            if (p < thr.t[j])
                break;
            n = j + 1;
        }
    }
    return n;
}

// Path-independent coefficients of the Euler step in the path precision.  D is
// the padded dimension (1, 2, 4 or 8); padded components have zero rows and
// columns, zero noise and zero jumps, so they stay exactly zero.
template <typename Real, int D>
struct Coef {
    Real A[D * D];   // row-major
    Real sq[D];      // sqrt(dt) * s
    Real jm[D];      // jump mean
    Real js[D];      // jump std
    Real x0[D];
    Real xT[D];
    Real dt;
    Real c3;
};

// Draws of path-step (m, k) under iteration word `iter`.
template <typename Real, int D>
__device__ __forceinline__ void draws(uint32_t m, uint32_t k, uint32_t iter, uint32_t key0,
                                      uint32_t key1, const PoissonThresholds& thr, Real* zw,
                                      Real* zj, int& n) {
    constexpr int NB = (D + 1) / 2;
    uint32_t w[4 * NB];
#pragma unroll
    for (int s = 0; s < NB; ++s)
        philox4x32_10(m, k, iter, (uint32_t)s, key0, key1, &w[4 * s]);
#pragma unroll
    for (int i = 0; i < D; ++i)
        box_muller(w[2 * i], w[2 * i + 1], zw[i], zj[i]);
    n = poisson_count(poisson_word(w), thr);
}

template <typename Real>
__device__ __forceinline__ Real count_sqrt(int n);
template <>
__device__ __forceinline__ float count_sqrt<float>(int n) {
    return sqrtf((float)n);
}
template <>
__device__ __forceinline__ double count_sqrt<double>(int n) {
    return sqrt((double)n);
}

// One Euler-Maruyama step with additive compound-Poisson jumps:
//   X <- X + dt (A X - c3 X^3 + Bu_k) + sqrt(dt) s Z^W + n m_J + s_J sqrt(n) Z^J
// bu = B u_k (per-step table row).
template <typename Real, int D>
__device__ __forceinline__ void euler_step(const Coef<Real, D>& c, const Real* __restrict__ bu,
                                           Real* X, const Real* zw, const Real* zj, int n) {
    const Real fn = (Real)n;
    const Real sn = count_sqrt<Real>(n);
    Real Y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        Real f = bu[i];
#pragma unroll
        for (int j = 0; j < D; ++j)
            f = fma(c.A[i * D + j], X[j], f);
        const Real x3 = X[i] * X[i] * X[i];
        f = fma(-c.c3, x3, f);
        Real y = fma(c.dt, f, X[i]);
        y = fma(c.sq[i], zw[i], y);
        const Real jump = fma(c.js[i] * sn, zj[i], fn * c.jm[i]);
        Y[i] = y + jump;
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
        X[i] = Y[i];
}

// One backward adjoint step at state X_k:
//   lam <- lam + dt [ (A - 3 c3 diag(X_k^2))^T lam + (X_k - xd_k) ]
template <typename Real, int D>
__device__ __forceinline__ void adjoint_step(const Coef<Real, D>& c, const Real* __restrict__ xd,
                                             const Real* X, Real* lam) {
    Real Y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        Real a = X[i] - xd[i];
#pragma unroll
        for (int j = 0; j < D; ++j)
            a = fma(c.A[j * D + i], lam[j], a);
        const Real q = (Real)3 * c.c3 * X[i] * X[i];
        a = fma(-q, lam[i], a);
        Y[i] = fma(c.dt, a, lam[i]);
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
        lam[i] = Y[i];
}

// Running-cost term |X_k - xd_k|^2 in the path precision.
template <typename Real, int D>
__device__ __forceinline__ Real sq_dist(const Real* X, const Real* __restrict__ xd) {
    Real e = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const Real r = X[i] - xd[i];
        e = fma(r, r, e);
    }
    return e;
}

// Deterministic FP64 sum over a block of kThreads threads (fixed tree).
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s)
            sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Per-step sums over the block's paths of the adjoint (the Monte Carlo
// gradient's summand), written as FP64 block partials part[row * nblk + blk]
// with row = k*D + c.  Each thread deposits its values into an LDS tile of
// kRows rows x kThreads columns; when the tile is full, 16 lanes per row sum
// 16 columns each (column q, q+16, ...) and combine by an xor butterfly, so
// the order of every sum is fixed and the result is bit-reproducible.
template <int D>
struct StepReducer {
    static constexpr int kRows = 16;
    static constexpr int kSteps = kRows / D;  // steps per flush
    double (*tile)[kThreads];
    int filled;   // steps deposited since the last flush
    int k_first;  // step index of the first deposited step (steps go downwards)

    __device__ __forceinline__ void init(double (*t)[kThreads]) {
        tile = t;
        filled = 0;
        k_first = 0;
    }

    template <typename Real>
    __device__ __forceinline__ void push(int k, const Real* v, double* __restrict__ part, int nblk) {
        if (filled == 0)
            k_first = k;
#pragma unroll
        for (int c = 0; c < D; ++c)
            tile[filled * D + c][threadIdx.x] = (double)v[c];
        if (++filled == kSteps)
            flush(part, nblk);
    }

    __device__ __forceinline__ void flush(double* __restrict__ part, int nblk) {
        if (filled == 0)
            return;
        __syncthreads();
        const int t = threadIdx.x;
        const int r = t >> 4;
        const int q = t & 15;
        if (r < filled * D) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < kThreads / 16; ++j)
                s += tile[r][j * 16 + q];
            s += __shfl_xor(s, 8, 16);
            s += __shfl_xor(s, 4, 16);
            s += __shfl_xor(s, 2, 16);
            s += __shfl_xor(s, 1, 16);
            if (q == 0) {
                const int step = r / D, c = r - step * D;
                const int k = k_first - step;
                part[(size_t)(k * D + c) * nblk + blockIdx.x] = s;
            }
        }
        __syncthreads();
        filled = 0;
    }
};

}  // namespace jd
