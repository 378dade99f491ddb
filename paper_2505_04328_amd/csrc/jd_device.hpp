// Device-side building blocks of the hot path for gfx950: the counter-based
// draws, the Euler-Maruyama step, the adjoint step and the deterministic FP64
// block reduction.  Everything a forward sweep and a recomputing adjoint sweep
// share lives here, so that both evaluate bit-identical steps (the library is
// built with -ffp-contract=off and every fused multiply-add is written out).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jd_launch.hpp"

namespace jd {

constexpr int kThreads = 256;  // threads per block of every sweep kernel

// True when a gated launch must not run (its tag is not the header's phase).
// The word is read once per block; it is written only by earlier kernels on
// the stream, so every block of a launch sees the same value.
__device__ __forceinline__ bool gate_closed(const Gate& g) {
    return g.word != nullptr && *g.word != g.tag;
}

// Three-input xor in one VALU instruction (gfx950 v_bitop3_b32, truth table
// 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// 32x32->64-bit product as (lo, hi).  SCALAR writes it as a 32-bit multiply
// and a high multiply, which the compiler keeps on the scalar unit for
// wave-uniform operands; the 64-bit form is matched to the vector
// v_mad_u64_u32 (one instruction for lane-varying operands) even when the
// operands are uniform.  Both give the same value.
template <bool SCALAR>
__device__ __forceinline__ void mul_wide(uint32_t m, uint32_t c, uint32_t& lo, uint32_t& hi) {
    if (SCALAR) {
        lo = m * c;
        hi = __umulhi(m, c);
    } else {
        const uint64_t p = (uint64_t)m * (uint64_t)c;
        lo = (uint32_t)p;
        hi = (uint32_t)(p >> 32);
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Per round: two
// 32x32->64-bit products and two three-input xors.  In a sweep the counter is
// (path m, step k, iteration, block) with c1..c3 and the key wave-uniform, so
// round 1's second product, its xor into c0 and round 2's first product are
// wave-uniform; SWEEP computes those on the scalar unit (v_bitop3 is a vector
// instruction, so the uniform xor is written as two plain xors).
template <bool SWEEP = false>
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t* out) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t p0lo, p0hi, p1lo, p1hi;
        if (SWEEP && r == 1)
            mul_wide<true>(0xD2511F53u, c0, p0lo, p0hi);
        else
            mul_wide<false>(0xD2511F53u, c0, p0lo, p0hi);
        if (SWEEP && r == 0)
            mul_wide<true>(0xCD9E8D57u, c2, p1lo, p1hi);
        else
            mul_wide<false>(0xCD9E8D57u, c2, p1lo, p1hi);
        const uint32_t n0 = (SWEEP && r == 0) ? (p1hi ^ c1) ^ k0 : xor3(p1hi, c1, k0);
        const uint32_t n2 = xor3(p0hi, c3, k1);
        c1 = p1lo;
        c3 = p0lo;
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

// Box-Muller pair from two words (u_a, u_b): radius r = sqrt(-2 ln u_a) and
// angle 2 pi u_b; the cosine branch r cos(2 pi u_b) and the sine branch
// r sin(2 pi u_b) are two independent standard normals.  FP32 uses the
// hardware transcendentals directly: v_log_f32 (log2), v_sqrt_f32 and
// v_sin_f32 / v_cos_f32, whose argument is in revolutions, so cos(2 pi u) is
// one instruction.  The uniforms are never 0, denormal or 1, so no range
// handling is needed; the result matches the FP64 transform to within 1e-6
// absolute, like the correctly-rounded library functions.
__device__ __forceinline__ float bm_radius(uint32_t a, float) {
    const float l2 = __builtin_amdgcn_logf(unit_uniform<float>(a));  // log2(u_a)
    return __builtin_amdgcn_sqrtf(-1.38629436111989061883f * l2);    // sqrt(-2 ln u_a)
}
__device__ __forceinline__ float bm_cos(float r, float ub) { return r * __builtin_amdgcn_cosf(ub); }
__device__ __forceinline__ float bm_sin(float r, float ub) { return r * __builtin_amdgcn_sinf(ub); }
__device__ __forceinline__ double bm_radius(uint32_t a, double) {
    return sqrt(-2.0 * log(unit_uniform<double>(a)));
}
__device__ __forceinline__ double bm_cos(double r, double ub) { return r * cospi(2.0 * ub); }
__device__ __forceinline__ double bm_sin(double r, double ub) { return r * sinpi(2.0 * ub); }

// Word made of the low bytes of the four words of Philox block 0:
// byte j = low byte of word j.  v_perm_b32 selects bytes of the 8-byte value
// {S0 (bytes 4-7), S1 (bytes 0-3)}; selector 0x0c gives a zero byte.
__device__ __forceinline__ uint32_t poisson_word(const uint32_t* w) {
    const uint32_t lo = __builtin_amdgcn_perm(w[1], w[0], 0x0c0c0400u);  // [w0.b0, w1.b0, 0, 0]
    const uint32_t hi = __builtin_amdgcn_perm(w[3], w[2], 0x04000c0cu);  // [0, 0, w2.b0, w3.b0]
    return lo | hi;
}

// Count for word P.  The first comparison (against t0 = tm1[0], which a sweep
// keeps in a register) is the common case; the loop runs only in lanes that
// jump.
__device__ __forceinline__ int poisson_count(uint32_t P, uint32_t t0,
                                             const PoissonTable* __restrict__ tb) {
    int n = P > t0 ? 1 : 0;
    if (n) {
        const int jmax = tb->jmax;
#pragma unroll 1
        for (int j = 1; j < jmax; ++j) {
            if (P <= tb->tm1[j])
                break;
            n = j + 1;
        }
    }
    return n;
}
__device__ __forceinline__ int poisson_count(uint32_t P, const PoissonTable* __restrict__ tb) {
    return poisson_count(P, tb->tm1[0], tb);
}

// Path-independent coefficients of the Euler step in the path precision.  D is
// the padded dimension (1, 2, 4 or 8); padded components have zero rows and
// columns, zero noise and zero jumps, so they stay exactly zero.
template <typename Real, int D>
struct alignas(16) Coef {
    Real A[D * D];   // row-major
    Real AT[D * D];  // A^T, row-major (the adjoint step reads rows of A^T)
    Real sq[D];      // sqrt(dt) * s
    Real jm[D];      // jump mean
    Real js[D];      // jump std
    Real x0[D];
    Real xT[D];
    Real dt;
    Real c3;
};

// Coefficient placement.  Small problems keep every coefficient in scalar
// registers (the kernel argument).  In the forward step of FP32 d = 8 and of
// FP64 d >= 2 the drift matrix, the jump law and the endpoints do not fit the
// scalar register file next to the Philox key schedule and the per-step table
// rows, and the compiler spills them to vector-register lanes (a v_readlane
// per use); there each block stages the coefficients in LDS once and every
// step reads the matrix and the jump law from there.  The adjoint step needs
// no key schedule: it reads A^T from LDS only in FP64 (d >= 2), where the
// matrix alone takes 2 d^2 scalar registers.  The scalars of a step
// (sqrt(dt) s, dt, the cubic coefficient) stay in scalar registers.
template <typename Real, int D>
struct CoefInLds {
    static constexpr bool forward = sizeof(Real) == 8 ? D >= 2 : D >= 8;
    static constexpr bool adjoint = sizeof(Real) == 8 && D >= 2;
    static constexpr bool any = forward || adjoint;
};

// A zero the compiler cannot see through: offsetting the LDS coefficients by
// it in each step keeps their loads inside the step loop instead of hoisting
// the whole matrix into registers for the duration of the sweep.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

// Where the matrix comes from LDS, a scheduling barrier after each row of a
// matrix-vector product keeps at most one row of coefficients in registers
// (the scheduler would otherwise issue every row's loads at once).
template <bool LDS>
__device__ __forceinline__ void row_barrier() {
    if constexpr (LDS)
        __builtin_amdgcn_sched_barrier(0);
}

// The coefficient rows a step reads: the LDS copy (reloaded every step) or
// the kernel argument.
template <bool LDS, typename Real, int D>
__device__ __forceinline__ const Coef<Real, D>& coef_rows(const Coef<Real, D>& arg,
                                                          const Coef<Real, D>* lds) {
    if constexpr (LDS)
        return *(lds + opaque_zero());
    else
        return arg;
}

// The coefficients used once per path (x0, xT): the LDS copy where the
// kernel staged one (lds != nullptr), without the opaque offset.
template <typename Real, int D>
__device__ __forceinline__ const Coef<Real, D>& coef_once(const Coef<Real, D>& arg,
                                                          const Coef<Real, D>* lds) {
    if constexpr (CoefInLds<Real, D>::any)
        return lds != nullptr ? *lds : arg;
    else
        return arg;
}

// Draws of one path-step.  Component i's Gaussian pair comes from one
// Box-Muller transform of words (2i, 2i+1): Z^W_i is its cosine branch, always
// needed; Z^J_i its sine branch, evaluated by jump_normal() only where a jump
// happens.
template <typename Real, int D>
struct StepDraws {
    Real zw[D];
    Real rad[D];  // Box-Muller radius
    Real ang[D];  // angle uniform (revolutions)
    int n;        // Poisson count
};

template <typename Real, int D>
__device__ __forceinline__ Real jump_normal(const StepDraws<Real, D>& s, int i) {
    return bm_sin(s.rad[i], s.ang[i]);
}

// Draws of path-step (m, k) under iteration word `iter`; t0 = thr->tm1[0].
template <typename Real, int D>
__device__ __forceinline__ void draws(uint32_t m, uint32_t k, uint32_t iter, uint32_t key0,
                                      uint32_t key1, const PoissonTable* __restrict__ thr,
                                      uint32_t t0, StepDraws<Real, D>& s) {
    constexpr int NB = (D + 1) / 2;
    uint32_t w[4 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        philox4x32_10<true>(m, k, iter, (uint32_t)b, key0, key1, &w[4 * b]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        s.rad[i] = bm_radius(w[2 * i], (Real)0);
        s.ang[i] = unit_uniform<Real>(w[2 * i + 1]);
        s.zw[i] = bm_cos(s.rad[i], s.ang[i]);
    }
    s.n = poisson_count(poisson_word(w), t0, thr);
}

template <typename Real>
__device__ __forceinline__ Real count_sqrt(int n);
template <>
__device__ __forceinline__ float count_sqrt<float>(int n) {
    return __builtin_amdgcn_sqrtf((float)n);
}
template <>
__device__ __forceinline__ double count_sqrt<double>(int n) {
    return sqrt((double)n);
}

// The deterministic part of one Euler-Maruyama step and the Brownian term:
//   Y = X + dt (A X - c3 X^3 + Bu_k) + sqrt(dt) s Z^W
// bu = B u_k (per-step table row), zw = Z^W.  CUBIC = false compiles the step
// of a drift without the cubic term (the kernels are instantiated for both
// and launched by whether c3 is zero).
template <typename Real, int D, bool LDS, bool CUBIC>
__device__ __forceinline__ void euler_drift(const Coef<Real, D>& c, const Coef<Real, D>& rows,
                                            const Real* __restrict__ bu, const Real* X,
                                            const Real* zw, Real* Y) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
        Real f = bu[i];
#pragma unroll
        for (int j = 0; j < D; ++j)
            f = fma(rows.A[i * D + j], X[j], f);
        row_barrier<LDS>();
        if (CUBIC) {
            const Real x3 = X[i] * X[i] * X[i];
            f = fma(-c.c3, x3, f);
        }
        Real y = fma(c.dt, f, X[i]);
        Y[i] = fma(c.sq[i], zw[i], y);
    }
}

// Jump increment of component i for a path-step with count n > 0:
//   n m_J + s_J sqrt(n) Z^J.
template <typename Real, int D>
__device__ __forceinline__ Real jump_increment(const Coef<Real, D>& rows,
                                               const StepDraws<Real, D>& s, int i) {
    const Real fn = (Real)s.n;
    const Real sn = count_sqrt<Real>(s.n);
    return fma(rows.js[i] * sn, jump_normal(s, i), fn * rows.jm[i]);
}

// One Euler-Maruyama step with additive compound-Poisson jumps:
//   X <- X + dt (A X - c3 X^3 + Bu_k) + sqrt(dt) s Z^W + n m_J + s_J sqrt(n) Z^J
// The jump term (with Z^J) is evaluated only in waves where some lane jumps
// (lambda dt per path-step, so most waves skip it) and applied only in the
// lanes with n > 0.
template <typename Real, int D, bool CUBIC = true>
__device__ __forceinline__ void euler_step(const Coef<Real, D>& c, const Coef<Real, D>* lc,
                                           const Real* __restrict__ bu, Real* X,
                                           const StepDraws<Real, D>& s) {
    constexpr bool LDS = CoefInLds<Real, D>::forward;
    const Coef<Real, D>& rows = coef_rows<LDS>(c, lc);
    Real Y[D];
    euler_drift<Real, D, LDS, CUBIC>(c, rows, bu, X, s.zw, Y);
    if (__builtin_amdgcn_ballot_w64(s.n != 0)) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const Real yj = Y[i] + jump_increment<Real, D>(rows, s, i);
            Y[i] = s.n != 0 ? yj : Y[i];
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
        X[i] = Y[i];
}

// The same step with its noise read from a precomputed table: zw = Z^W and
// jinc = the jump increment of the path-step, or -0.0 where the count is
// zero (y + (-0.0) is y for every y, signed zeros and NaN included), so the
// result equals euler_step's bit for bit.
template <typename Real, int D, bool CUBIC = true>
__device__ __forceinline__ void euler_step_noise(const Coef<Real, D>& c, const Coef<Real, D>* lc,
                                                 const Real* __restrict__ bu, Real* X,
                                                 const Real* zw, const Real* jinc) {
    constexpr bool LDS = CoefInLds<Real, D>::forward;
    const Coef<Real, D>& rows = coef_rows<LDS>(c, lc);
    Real Y[D];
    euler_drift<Real, D, LDS, CUBIC>(c, rows, bu, X, zw, Y);
#pragma unroll
    for (int i = 0; i < D; ++i)
        X[i] = Y[i] + jinc[i];
}

// One backward adjoint step at state X_k:
//   lam <- lam + dt [ (A - 3 c3 diag(X_k^2))^T lam + (X_k - xd_k) ]
// LDS: read the rows of A^T from the block's LDS copy (same values, same
// arithmetic) -- kernels that also run forward steps set it wherever those
// read their matrix from LDS.
template <typename Real, int D, bool LDS = CoefInLds<Real, D>::adjoint,
          bool CUBIC = true>
__device__ __forceinline__ void adjoint_step(const Coef<Real, D>& c, const Coef<Real, D>* lc,
                                             const Real* __restrict__ xd, const Real* X, Real* lam) {
    const Coef<Real, D>& rows = coef_rows<LDS>(c, lc);
    Real Y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        Real a = X[i] - xd[i];
#pragma unroll
        for (int j = 0; j < D; ++j)
            a = fma(rows.AT[i * D + j], lam[j], a);
        row_barrier<LDS>();
        if (CUBIC) {
            const Real q = (Real)3 * c.c3 * X[i] * X[i];
            a = fma(-q, lam[i], a);
        }
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

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// fences global memory, which makes every wave wait for all of its outstanding
// loads (the prefetched trajectory tiles) at each barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Deterministic FP64 sum over a block of NT threads (fixed tree).
template <int NT = kThreads>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
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
// with row = k*D + c.  Each thread deposits its values, in the path precision
// T (exact), into an LDS tile of kRows rows x kThreads columns; when the tile
// is full, 16 lanes per row sum 16 columns each (column q, q+16, ...) in FP64
// and combine by an xor butterfly, so the order of every sum is fixed and the
// result is bit-reproducible.  An FP32 tile is 16 KB, which leaves room for
// eight blocks per CU.
template <int D, typename T>
struct StepReducer {
    static constexpr int kRows = 16;
    static constexpr int kSteps = kRows / D;  // steps per flush
    T (*tile)[kThreads];
    int filled;   // steps deposited since the last flush
    int k_first;  // step index of the first deposited step (steps go downwards)
    int col;      // partial-sum column: the 256-path group this block sums

    __device__ __forceinline__ void init(T (*t)[kThreads], int group) {
        tile = t;
        filled = 0;
        k_first = 0;
        col = group;
    }

    // Deposit the values of the s-th step of the current tile (no flush).
    template <typename Real>
    __device__ __forceinline__ void put(int s, const Real* v) {
#pragma unroll
        for (int c = 0; c < D; ++c)
            tile[s * D + c][threadIdx.x] = (T)v[c];
    }

    // Flush a tile filled by put() with `count` steps, the first being step k0.
    __device__ __forceinline__ void flush_tile(int k0, int count, double* __restrict__ part,
                                               int nblk) {
        k_first = k0;
        filled = count;
        flush(part, nblk);
    }

    __device__ __forceinline__ void flush(double* __restrict__ part, int nblk) {
        if (filled == 0)
            return;
        lds_barrier();
        const int t = threadIdx.x;
        const int r = t >> 4;
        const int q = t & 15;
        if (r < filled * D) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < kThreads / 16; ++j)
                s += (double)tile[r][j * 16 + q];
            s += __shfl_xor(s, 8, 16);
            s += __shfl_xor(s, 4, 16);
            s += __shfl_xor(s, 2, 16);
            s += __shfl_xor(s, 1, 16);
            if (q == 0) {
                const int step = r / D, c = r - step * D;
                const int k = k_first - step;
                part[(size_t)(k * D + c) * nblk + col] = s;
            }
        }
        lds_barrier();
        filled = 0;
    }
};

}  // namespace jd
