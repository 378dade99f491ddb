// Kernels of the hot path on gfx950 and their typed launchers.
//
//  k_table            per-step table: B u_k and x_d(t_k) in the path precision
//  k_forward          forward Euler-Maruyama sweep, one path per lane, draws in
//                     registers (or read from the noise table), FP64 path cost,
//                     trajectory or checkpoint store
//  k_noise            the draws of one iteration as a table, for small grids
//  k_adjoint_stored   backward adjoint sweep over the stored trajectory
//  k_cost_grad_stored forward then backward sweep in one launch, per block
//  k_adjoint_recompute backward adjoint sweep regenerating each checkpoint
//                     segment with the same counters (bit-identical states)
//  k_finalize_grad    fixed-order FP64 sum of the per-block partials -> g
//  k_finalize_cost    fixed-order FP64 sum of the path costs -> J, ||g||^2
//  k_trial, k_armijo  line-search step and sufficient-decrease test
//  k_draws, k_philox  the draws / raw Philox words, for parity checks
//
// The paper's method: forward model (Section 3, eq. model_approximation;
// Section 5, model equation), adjoint (Section 4, eq. AdjointModel; Section 5,
// adjoint equation), gradient (Section 4, eq. definition_Gradient), line search
// (Section 5, eq. Stochastic_Armijo, Algorithm 5.4).
#include "jd_device.hpp"
#include "jd_launch.hpp"

namespace jd {

template <typename Real, int D>
struct SweepArgs {
    Coef<Real, D> c;
    const Coef<Real, D>* lc;  // the block's LDS copy of c (set in the kernel), see CoefInLds
    const PoissonTable* thr;  // staged in the workspace header, then in the block's LDS
    uint32_t thr0;            // thr->tm1[0], read once per block
    Gate gate;        // launch gate (word null: always runs)
    void* traj;       // trajectory or checkpoints
    double* part;     // per-block partial sums
    int64_t M;
    int nblk;  // 256-path groups: ceil(M / 256), the columns of the partial sums
    int N, d, K;
    int nslots;  // trajectory slots per block: N (store) or ceil(N/K) (checkpoints)
    uint32_t key0, key1, iter;
    double dt64;
    // per-path diagnostics
    int64_t dm0, dcount;
    Real* dX;
    Real* dlam;
    double* dcost;
};

// Trajectory layout, blocked by the 256 paths of a sweep block: block b owns
// a contiguous region of nslots * d rows of 256 elements; row (slot*d + c)
// holds component c of X_k (slot k-1) or of checkpoint j (slot j-1) for the
// block's paths.  A block therefore streams through one contiguous region
// (1 KB per FP32 row), and every lane, including lanes past the last path,
// owns an in-bounds column.  Padded components re-read component d-1 and
// return 0.
struct Cols {
    int64_t stride;  // d * 256: elements between consecutive slots
};

// Raw buffer descriptor word 3 for gfx9-family buffer loads of plain dwords,
// and the non-temporal cache policy bit of buffer/global loads.
constexpr int kBufferConfig = 0x00020000;
constexpr int kNontemporal = 2;

__device__ __forceinline__ Cols make_cols(int d) {
    Cols c;
    c.stride = (int64_t)d * kThreads;
    return c;
}

// Start of slot `slot` of path group g's region (uniform).
template <typename Real>
__device__ __forceinline__ const Real* slot_row(const void* base, const Cols& cl, int nslots,
                                                int64_t g, int slot) {
    return (const Real*)base + (g * nslots + slot) * cl.stride;
}

template <typename Real, int D>
__device__ __forceinline__ void load_row(const Real* __restrict__ row, int d, Real* X) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const int ce = c < d ? c : d - 1;
        const Real v = __builtin_nontemporal_load(row + ce * kThreads + threadIdx.x);
        X[c] = c < d ? v : (Real)0;
    }
}

typedef unsigned int U32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

// One state row (d components of 256 lanes) by raw buffer stores: one
// descriptor per row, the lane's byte offset in a vector register and each
// component's offset in a scalar one, so no 64-bit address is formed per
// component (global stores reach only 4 KB past a base).  With every
// component present (d = D) the stores need no per-component branch.
// AUX: cache policy.
template <typename Real, int D, int AUX>
__device__ __forceinline__ void buffer_store_row(Real* row, int d, const Real* X) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)row, (short)0, (int)(d * kThreads * (int)sizeof(Real)), kBufferConfig);
    const uint32_t voff = threadIdx.x * (uint32_t)sizeof(Real);
    auto put = [&](int c) {
        // the byte offset split into a multiple of 4 KB (the scalar operand)
        // and the rest, added to the lane's offset (loop-invariant values)
        const uint32_t off = (uint32_t)(c * kThreads * (int)sizeof(Real));
        const uint32_t soff = off & ~4095u;
        const uint32_t vo = voff + (off & 4095u);
        if constexpr (sizeof(Real) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)X[c]), r,
                                                  vo, soff, AUX);
        else
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, (double)X[c]), r,
                                                  vo, soff, AUX);
    };
    if (D == 1 || d == D) {  // a one-component sweep always has d = 1
#pragma unroll
        for (int c = 0; c < D; ++c)
            put(c);
    } else {
#pragma unroll
        for (int c = 0; c < D; ++c)
            if (c < d)
                put(c);
    }
}

// Trajectory and checkpoint rows are read once, by the adjoint: non-temporal.
template <typename Real, int D>
__device__ __forceinline__ void store_row(Real* __restrict__ row, int d, const Real* X) {
    buffer_store_row<Real, D, kNontemporal>(row, d, X);
}

template <typename Real, int D>
__device__ __forceinline__ void dump_state(const SweepArgs<Real, D>& a, Real* dst, int k, int64_t m,
                                           const Real* v) {
    const int64_t p = m - a.dm0;
    if (dst != nullptr && p >= 0 && p < a.dcount) {
#pragma unroll
        for (int c = 0; c < D; ++c)
            if (c < a.d)
                dst[((size_t)(k - 1) * a.d + c) * a.dcount + p] = v[c];
    }
}

// Stages the coefficients in LDS when the kernel's steps read them from there
// (USE; one lane copies the argument struct) and points a.lc at the copy;
// otherwise does nothing and a.lc stays null.
template <bool USE, typename Real, int D>
__device__ __forceinline__ void stage_coef(SweepArgs<Real, D>& a, Coef<Real, D>* sc) {
    if constexpr (USE) {
        if (threadIdx.x == 0)
            *sc = a.c;
        __syncthreads();
        a.lc = sc;
    }
}

// Stages the Poisson thresholds in LDS and points a.thr at the copy.  Sweeps
// that store to global memory inside their step loop need it: the compiler
// cannot tell those stores from the thresholds in the workspace header, so it
// would reload the first threshold with a vector load in every step and wait
// for all of the wave's outstanding stores before the comparison (the
// vector-memory counter covers stores too).  LDS cannot alias global memory,
// so the copy's loads stay off that counter.
template <typename Real, int D>
__device__ __forceinline__ void stage_thresholds(SweepArgs<Real, D>& a, PoissonTable* st) {
    if (threadIdx.x < 32)
        st->tm1[threadIdx.x] = a.thr->tm1[threadIdx.x];
    if (threadIdx.x == 0)
        st->jmax = a.thr->jmax;
    __syncthreads();
    a.thr = st;
    a.thr0 = st->tm1[0];
}

// ---------------------------------------------------------------------------
// B u_k and x_d rows.  B is passed by value (d*d <= 64 doubles).
struct BMat {
    double b[64];
};

// Entry idx = k D + i of the per-step table (B u_k and x_d(t_k), row k), and
// at idx < 32 the header's thresholds and flags.  g != nullptr: a line-search
// trial.  The table is built for ut = u - zeta g, which the lanes of
// components i < d also write out (each lane evaluates the trial entries of
// its row with k_trial's expression, so the table and ut are bitwise those of
// k_trial followed by the plain table).
template <typename Real, int D>
__device__ __forceinline__ void table_entry(int idx, const double* __restrict__ u,
                                            const double* __restrict__ xd, Real* __restrict__ tab,
                                            int N, int d, const BMat& B, WsHeader* hdr,
                                            int clear_flag, const PoissonTable& pt,
                                            const double* __restrict__ g, double zeta,
                                            double* __restrict__ ut) {
    if (idx == 0 && clear_flag)
        hdr->nonfinite = 0;  // every entry point starts here: the flag describes this call
    if (idx < 32)
        hdr->poisson.tm1[idx] = pt.tm1[idx];
    if (idx == 0)
        hdr->poisson.jmax = pt.jmax;
    if (idx >= N * D)
        return;
    const int k = idx / D, i = idx - k * D;
    auto uk = [&](int j) {
        const size_t q = (size_t)k * d + j;
        return g != nullptr ? u[q] - zeta * g[q] : u[q];
    };
    double bu = 0.0, x = 0.0;
    if (i < d) {
        for (int j = 0; j < d; ++j)
            bu += B.b[i * d + j] * uk(j);
        x = xd[(size_t)k * d + i];
        if (g != nullptr)
            ut[(size_t)k * d + i] = uk(i);
    }
    tab[(size_t)k * 2 * D + i] = (Real)bu;
    tab[(size_t)k * 2 * D + D + i] = (Real)x;
}

template <typename Real, int D>
__global__ void __launch_bounds__(kThreads)
k_table(const double* __restrict__ u, const double* __restrict__ xd, Real* __restrict__ tab, int N,
        int d, BMat B, WsHeader* hdr, int clear_flag, PoissonTable pt, Gate gate,
        const double* __restrict__ g, double zeta, double* __restrict__ ut) {
    if (gate_closed(gate))
        return;
    table_entry<Real, D>(blockIdx.x * kThreads + threadIdx.x, u, xd, tab, N, d, B, hdr,
                         clear_flag, pt, g, zeta, ut);
}

// Blocks of the per-step table for N steps (at least one: the header's
// thresholds and flags).
inline int64_t table_blocks(int N, int D) {
    const int64_t n = (int64_t)N * D > 32 ? (int64_t)N * D : 32;
    return (n + kThreads - 1) / kThreads;
}

// ---------------------------------------------------------------------------
// The per-step table is a separate __restrict__ argument so that its rows are
// read with scalar loads (they are wave-uniform), which do not join the
// in-order vector-memory counter the trajectory loads and stores use.
// Forward sweep of one 256-path group g, one step at a time: begin(), step(k)
// for k = 0..N-1, finish().  The path of this lane is m = 256 g + lane.
template <typename Real, int D, int MODE, bool CB>
struct ForwardSweep {
    Real X[D];
    double acc;
    Real* row;  // next trajectory slot to write
    int64_t m;
    bool act;

    __device__ __forceinline__ void begin(const SweepArgs<Real, D>& a, int64_t g) {
        m = g * kThreads + threadIdx.x;
        act = m < a.M;
#pragma unroll
        for (int i = 0; i < D; ++i)
            X[i] = coef_once<Real, D>(a.c, a.lc).x0[i];
        acc = 0.0;
        row = (Real*)slot_row<Real>(a.traj, make_cols(a.d), a.nslots, g, 0);
    }

    __device__ __forceinline__ void step(const SweepArgs<Real, D>& a, const Real* __restrict__ tab,
                                         int k) {
        const Real* trow = tab + (size_t)k * 2 * D;
        acc += (double)sq_dist<Real, D>(X, trow + D);
        StepDraws<Real, D> z;
        draws<Real, D>((uint32_t)m, (uint32_t)k, a.iter, a.key0, a.key1, a.thr, a.thr0, z);
        euler_step<Real, D, CB>(a.c, a.lc, trow, X, z);
        put(a, k);
    }

    // Step k with its noise from the iteration's noise table; trow: the
    // step's row of the per-step table.
    __device__ __forceinline__ void step_noise(const SweepArgs<Real, D>& a, const Real* trow, int k,
                                               const Real* zw, const Real* jinc) {
        acc += (double)sq_dist<Real, D>(X, trow + D);
        euler_step_noise<Real, D, CB>(a.c, a.lc, trow, X, zw, jinc);
        put(a, k);
    }

    // Stores X_{k+1} where the mode keeps it.
    __device__ __forceinline__ void put(const SweepArgs<Real, D>& a, int k) {
        if (MODE == FWD_STORE) {
            store_row<Real, D>(row, a.d, X);
            row += (int64_t)a.d * kThreads;
        } else if (MODE == FWD_CKPT) {
            if ((k + 1) % a.K == 0 || k + 1 == a.N) {
                store_row<Real, D>(row, a.d, X);
                row += (int64_t)a.d * kThreads;
            }
        }
    }

    // Path cost (left-point running cost plus terminal term) and the group's
    // fixed-order sum into cpart[g].  All threads of the block call it.
    __device__ __forceinline__ void finish(const SweepArgs<Real, D>& a, double* __restrict__ cpart,
                                           double* sh, int64_t g) {
        double C = 0.5 * a.dt64 * acc + 0.5 * (double)sq_dist<Real, D>(X, coef_once<Real, D>(a.c, a.lc).xT);
        if (!act)
            C = 0.0;
        if (a.dcost != nullptr) {
            const int64_t p = m - a.dm0;
            if (act && p >= 0 && p < a.dcount)
                a.dcost[p] = C;
        }
        const double s = block_sum(C, sh);
        if (threadIdx.x == 0)
            cpart[g] = s;
    }
};

// ---------------------------------------------------------------------------
// Noise table of one gradient iteration, for grids that leave most of the
// chip idle.  The draws of a path-step depend only on (path, step, iteration
// word, seed); a sweep of a few blocks spends its time on the latency of the
// per-step draw chain, which nothing else hides.  There one launch over all
// path-steps computes the draws, and every forward sweep of the iteration (the
// gradient's and its line-search trials', which reuse the iteration's draws)
// reads them.  Layout, blocked by the 256 paths of a sweep block like the
// trajectory: group g owns N steps of 2d rows of 256 elements; row (k*2d + c)
// holds Z^W_c of step k and row (k*2d + d + c) the jump increment of component
// c (-0.0 where the count is zero).  Lanes past the last path get their
// draws like in a sweep.
//
// The same launch builds the evaluation's per-step table (k_table's work, in
// its first tb blocks): the thresholds come from the argument, since the
// table's blocks are only now writing them into the header.
template <typename Real, int D>
__global__ void __launch_bounds__(kThreads)
k_noise(SweepArgs<Real, D> a, Real* __restrict__ noise, PoissonTable pt, int tb,
        const double* __restrict__ u, const double* __restrict__ xd, Real* __restrict__ tab,
        BMat B, WsHeader* hdr, int clear_flag) {
    if (gate_closed(a.gate))
        return;
    if ((int)blockIdx.x < tb) {
        table_entry<Real, D>(blockIdx.x * kThreads + threadIdx.x, u, xd, tab, a.N, a.d, B, hdr,
                             clear_flag, pt, nullptr, 0.0, nullptr);
        return;
    }
    __shared__ PoissonTable thr;
    if (threadIdx.x < 32)
        thr.tm1[threadIdx.x] = pt.tm1[threadIdx.x];
    if (threadIdx.x == 0)
        thr.jmax = pt.jmax;
    __syncthreads();
    a.thr = &thr;
    a.thr0 = thr.tm1[0];
    const int64_t nb = (int64_t)a.nblk * a.N;
    const int64_t rows = 2 * (int64_t)a.d * kThreads;
    for (int64_t b = blockIdx.x - tb; b < nb; b += gridDim.x - tb) {
        const int64_t g = b / a.N;
        const int k = (int)(b - g * a.N);
        const int64_t m = g * kThreads + threadIdx.x;
        StepDraws<Real, D> z;
        draws<Real, D>((uint32_t)m, (uint32_t)k, a.iter, a.key0, a.key1, a.thr, a.thr0, z);
        Real* out = noise + b * rows + threadIdx.x;  // b = g N + k: step k of group g
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (i < a.d) {
                out[i * kThreads] = z.zw[i];
                out[(a.d + i) * kThreads] =
                    z.n != 0 ? jump_increment<Real, D>(a.c, z, i) : (Real)-0.0;
            }
        }
    }
}

// P consecutive steps of the noise table in registers (P D = 16 values of
// each kind).  Padded components read component d-1 and take Z^W = 0 and
// increment -0.0, which leave them zero as the drawn values do (their noise
// scales are zero).
template <typename Real, int D>
struct NoiseTile {
    static constexpr int P = 16 / D;
    Real zw[P][D];
    Real ji[P][D];

    // Steps k0 .. k0+P-1 (clamped to N-1) of the block's region.  Components
    // past d hold component d-1's values: they are masked where a step uses
    // them, so that no select waits for a load here.
    __device__ __forceinline__ void load(const Real* __restrict__ region, int d, int N, int k0) {
        const int64_t rows = 2 * (int64_t)d * kThreads;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const int kk = k0 + s < N ? k0 + s : N - 1;
            const Real* r = region + kk * rows + threadIdx.x;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const int ce = c < d ? c : d - 1;
                zw[s][c] = r[ce * kThreads];
                ji[s][c] = r[(d + ce) * kThreads];
            }
        }
    }
    // The noise of step s: none past component d (Z^W 0, jump increment -0.0);
    // d >= 1, so component 0 is never masked.
    __device__ __forceinline__ void get(int s, int d, Real (&z)[D], Real (&j)[D]) const {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            z[c] = c == 0 || c < d ? zw[s][c] : (Real)0;
            j[c] = c == 0 || c < d ? ji[s][c] : (Real)-0.0;
        }
    }
};

// Steps of the per-step table a block copies into LDS at a time (16 KB).
// Without the copy every step waits for a scalar load of its row: with the
// draws precomputed nothing else covers that latency.
constexpr int kTabChunkBytes = 16384;
template <typename Real, int D>
constexpr int tab_chunk_steps() { return kTabChunkBytes / (int)(2 * D * sizeof(Real)); }

// All N steps of a forward sweep from the noise table: the next tile's loads
// are issued before the current tile is swept, and the per-step table is read
// from the block's LDS copy, a chunk of steps at a time.  Every thread of the
// block calls it (the chunk copy has barriers).
template <typename Real, int D, int MODE, bool CB>
__device__ __forceinline__ void sweep_noise(ForwardSweep<Real, D, MODE, CB>& f,
                                            const SweepArgs<Real, D>& a,
                                            const Real* __restrict__ tab,
                                            const Real* __restrict__ noise) {
    constexpr int P = NoiseTile<Real, D>::P;
    constexpr int CS = tab_chunk_steps<Real, D>();
    static_assert(CS % P == 0, "a table chunk holds whole noise tiles");
    __shared__ Real ltab[CS * 2 * D];
    const Real* region = noise + (int64_t)blockIdx.x * a.N * 2 * a.d * kThreads;
    NoiseTile<Real, D> cur, nxt;
    cur.load(region, a.d, a.N, 0);
    // The first tile waits here, once: the compiler's wait counts at a step
    // merge the loop's entry with its back edge, and a first tile still in
    // flight at the entry would make every tile's first step wait for the
    // next tile's loads just issued.
    __builtin_amdgcn_s_waitcnt(0);
    for (int k0 = 0;; k0 += P) {
        if (k0 % CS == 0) {
            const int n = (a.N - k0 < CS ? a.N - k0 : CS) * 2 * D;
            if (k0 != 0)
                lds_barrier();  // the previous chunk's readers are done
            for (int e = threadIdx.x; e < n; e += kThreads)
                ltab[e] = tab[(size_t)k0 * 2 * D + e];
            lds_barrier();
        }
        const bool more = k0 + P < a.N;
        if (more)
            nxt.load(region, a.d, a.N, k0 + P);
        const Real* lrow = ltab + (k0 % CS) * 2 * D;
        if (more) {
            // a full tile: no per-step condition, so its table reads issue together
#pragma unroll
            for (int s = 0; s < P; ++s) {
                Real z[D], j[D];
                cur.get(s, a.d, z, j);
                f.step_noise(a, lrow + s * 2 * D, k0 + s, z, j);
            }
        } else {
#pragma unroll
            for (int s = 0; s < P; ++s)
                if (k0 + s < a.N) {
                    Real z[D], j[D];
                    cur.get(s, a.d, z, j);
                    f.step_noise(a, lrow + s * 2 * D, k0 + s, z, j);
                }
        }
        if (!more)
            break;
        cur = nxt;
    }
}

// NOISE: the draws come from the iteration's noise table.
template <typename Real, int D, int MODE, bool CB, bool NOISE>
__global__ void __launch_bounds__(kThreads)
k_forward(SweepArgs<Real, D> a, const Real* __restrict__ tab, double* __restrict__ cpart,
          const Real* __restrict__ noise) {
    if (gate_closed(a.gate))
        return;
    __shared__ double sh[kThreads];
    __shared__ Coef<Real, D> sc;
    stage_coef<CoefInLds<Real, D>::forward>(a, &sc);
    __shared__ PoissonTable thr;
    stage_thresholds(a, &thr);
    ForwardSweep<Real, D, MODE, CB> f;
    f.begin(a, blockIdx.x);
    if constexpr (NOISE) {
        sweep_noise<Real, D, MODE, CB>(f, a, tab, noise);
    } else {
        for (int k = 0; k < a.N; ++k)
            f.step(a, tab, k);
    }
    f.finish(a, cpart, sh, blockIdx.x);
}

// ---------------------------------------------------------------------------

// The stored trajectory is read in tiles of kSteps steps (the reducer's flush
// granularity): the loads of the next tile are issued before the current tile
// is swept, so every wave keeps kSteps*D loads in flight.  A full tile (all of
// its steps >= 1) is one contiguous piece of the block's region and is read with
// raw buffer loads: one scalar descriptor per tile and per-lane byte offsets
// computed once, so the loads need no address arithmetic.  The last (partial)
// tile uses ordinary loads with clamped slots.
template <typename Real, int D>
__device__ __forceinline__ void load_tile(const SweepArgs<Real, D>& a, const Real* region,
                                          const Cols& cl, int k, Real (*X)[D]) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    // X_kk lives in slot kk-1; steps below 1 re-read slot 0 (never used)
    const Real* row = region + (int64_t)(k >= 1 ? k - 1 : 0) * cl.stride;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        load_row<Real, D>(row, a.d, X[s]);
        if (k - s > 1)
            row -= cl.stride;
    }
}

// voff: per-lane byte offset; soff: wave-uniform byte offset (a scalar
// register); AUX: cache policy (kNontemporal for data read once).
template <typename Real, int AUX = kNontemporal>
__device__ __forceinline__ Real buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(Real) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

// Full tile with top step k: slots k-1 (s = 0) down to k-S (s = S-1).
// Components past d hold component d-1's values (voff points there); the
// sweep masks them where a step uses them, so that no select waits for the
// prefetched loads as they are issued.
template <typename Real, int D>
__device__ __forceinline__ void load_tile_buffer(const Real* region, int64_t stride, int k,
                                                 const uint32_t* voff, Real (*X)[D]) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    const Real* base = region + (int64_t)(k - S) * stride;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)base, (short)0, (int)(S * stride * (int64_t)sizeof(Real)), kBufferConfig);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            X[s][c] = buffer_load<Real>(
                r, voff[c], (uint32_t)((S - 1 - s) * stride * (int64_t)sizeof(Real)));
        }
}

// One tile of the backward sweep: steps k, k-1, ..., k-count+1.  FULL tiles
// have every step >= 1; the last tile may end at step 0, which contributes to
// the gradient (lam_1) but needs no adjoint step.
template <typename Real, int D, bool DUMP, bool FULL, bool CB>
__device__ __forceinline__ void sweep_tile(const SweepArgs<Real, D>& a, const Real* __restrict__ tab,
                                           int k, Real (*X)[D], Real* lam, bool act, int64_t m,
                                           StepReducer<D, Real>& red) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    // a full tile's table rows are contiguous: one base, constant offsets
    const Real* trow = FULL ? tab + (size_t)(k - S + 1) * 2 * D : tab;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int kk = k - s;
        if (!FULL && kk < 0)
            break;
        Real v[D];
#pragma unroll
        for (int c = 0; c < D; ++c)
            v[c] = act ? lam[c] : (Real)0;
        red.put(s, v);
        if (FULL || kk >= 1) {
            const Real* xd = FULL ? trow + (S - 1 - s) * 2 * D + D : tab + (size_t)kk * 2 * D + D;
            Real xs[D];  // components past d are zero (d >= 1: component 0 never is)
#pragma unroll
            for (int c = 0; c < D; ++c)
                xs[c] = c == 0 || c < a.d ? X[s][c] : (Real)0;
            adjoint_step<Real, D, CoefInLds<Real, D>::adjoint, CB>(a.c, a.lc, xd, xs, lam);
            if (DUMP) {
                dump_state(a, a.dX, kk, m, X[s]);
                dump_state(a, a.dlam, kk, m, lam);
            }
        }
    }
}

// Backward sweep of one 256-path group g over its stored trajectory, a tile at
// a time: begin() sets lam_N and loads the first tile, full_tile() sweeps one
// full tile while the next one loads, tail() sweeps what is left (down to step
// 0).  Steps are reduced into partial column g.
template <typename Real, int D, bool DUMP, bool CB>
struct StoredAdjoint {
    static constexpr int S = StepReducer<D, Real>::kSteps;
    StepReducer<D, Real> red;
    const Real* region;
    uint32_t voff[D];  // lane's byte offset of component c within a slot
    Real lam[D];
    Real cur[S][D], nxt[S][D];
    Cols cl;
    int64_t m;
    bool act;
    int k;  // top step of the current tile

    // lam_N and the reducer; no tile is loaded yet.
    __device__ __forceinline__ void start(const SweepArgs<Real, D>& a, Real (*tile)[kThreads],
                                          int64_t g) {
        red.init(tile, (int)g);
        m = g * kThreads + threadIdx.x;
        act = m < a.M;
        cl = make_cols(a.d);
        region = slot_row<Real>(a.traj, cl, a.nslots, g, 0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int ce = c < a.d ? c : a.d - 1;
            voff[c] = (uint32_t)((ce * kThreads + threadIdx.x) * sizeof(Real));
        }
        Real XN[D];
        load_row<Real, D>(region + (int64_t)(a.N - 1) * cl.stride, a.d, XN);
#pragma unroll
        for (int i = 0; i < D; ++i)
            lam[i] = XN[i] - coef_once<Real, D>(a.c, a.lc).xT[i];
        if (DUMP) {
            dump_state(a, a.dX, a.N, m, XN);
            dump_state(a, a.dlam, a.N, m, lam);
        }
        k = a.N - 1;
    }

    // Loads the tile with top step k into cur.
    __device__ __forceinline__ void load(const SweepArgs<Real, D>& a) {
        if (full())
            load_tile_buffer<Real, D>(region, cl.stride, k, voff, cur);
        else
            load_tile<Real, D>(a, region, cl, k, cur);
    }

    // Sweeps the full tile in cur and moves to the next one.
    __device__ __forceinline__ void sweep(const SweepArgs<Real, D>& a, const Real* __restrict__ tab) {
        sweep_tile<Real, D, DUMP, true, CB>(a, tab, k, cur, lam, act, m, red);
        red.flush_tile(k, S, a.part, a.nblk);
        k -= S;
    }

    __device__ __forceinline__ bool full() const { return k - S + 1 >= 1; }

    // Issues the next tile's loads; run() then sweeps the current tile.  Work
    // placed between the two hides the loads.
    __device__ __forceinline__ void prefetch(const SweepArgs<Real, D>& a) {
        const int kn = k - S;
        if (kn - S + 1 >= 1)
            load_tile_buffer<Real, D>(region, cl.stride, kn, voff, nxt);
        else if (kn >= 1)
            load_tile<Real, D>(a, region, cl, kn, nxt);
    }

    __device__ __forceinline__ void run(const SweepArgs<Real, D>& a, const Real* __restrict__ tab) {
        sweep(a, tab);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c)
                cur[s][c] = nxt[s][c];
    }

    __device__ __forceinline__ void tail(const SweepArgs<Real, D>& a, const Real* __restrict__ tab) {
        if (k >= 0) {
            sweep_tile<Real, D, DUMP, false, CB>(a, tab, k, cur, lam, act, m, red);
            red.flush_tile(k, k + 1, a.part, a.nblk);
        }
    }
};

template <typename Real, int D, bool DUMP, bool CB>
__global__ void __launch_bounds__(kThreads)
k_adjoint_stored(SweepArgs<Real, D> a, const Real* __restrict__ tab) {
    if (gate_closed(a.gate))
        return;
    __shared__ Real tile[StepReducer<D, Real>::kRows][kThreads];
    __shared__ Coef<Real, D> sc;
    stage_coef<CoefInLds<Real, D>::adjoint>(a, &sc);
    StoredAdjoint<Real, D, DUMP, CB> b;
    b.start(a, tile, blockIdx.x);
    b.load(a);
    while (b.full()) {
        b.prefetch(a);
        b.run(a, tab);
    }
    b.tail(a, tab);
}

// Forward sweep with the stored trajectory, then, in the same block, the
// backward sweep over that block's own paths.  Paths are independent and each
// thread reads back only what it wrote itself (after a fence), so no grid-wide
// ordering is needed: while some blocks are in their VALU-bound forward phase,
// others are in their HBM-bound backward phase, and the two overlap on the
// device.  Every value is computed exactly as by k_forward followed by
// k_adjoint_stored.
template <typename Real, int D, bool CB, bool NOISE>
__global__ void __launch_bounds__(kThreads)
k_cost_grad_stored(SweepArgs<Real, D> a, const Real* __restrict__ tab, double* __restrict__ cpart,
                   const Real* __restrict__ noise) {
    if (gate_closed(a.gate))
        return;
    __shared__ double sh[kThreads];
    __shared__ Real tile[StepReducer<D, Real>::kRows][kThreads];
    __shared__ Coef<Real, D> sc;
    stage_coef<CoefInLds<Real, D>::any>(a, &sc);
    __shared__ PoissonTable thr;
    stage_thresholds(a, &thr);
    {
        ForwardSweep<Real, D, FWD_STORE, CB> f;
        f.begin(a, blockIdx.x);
        if constexpr (NOISE) {
            sweep_noise<Real, D, FWD_STORE, CB>(f, a, tab, noise);
        } else {
            for (int k = 0; k < a.N; ++k)
                f.step(a, tab, k);
        }
        f.finish(a, cpart, sh, blockIdx.x);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    StoredAdjoint<Real, D, false, CB> b;
    b.start(a, tile, blockIdx.x);
    b.load(a);
    while (b.full()) {
        b.prefetch(a);
        b.run(a, tab);
    }
    b.tail(a, tab);
}

// ---------------------------------------------------------------------------
// Segment j covers steps [jK, min((j+1)K, N)).  Its states are rebuilt from
// checkpoint j (x0 for j = 0) in sub-segments of R steps: a first pass keeps
// the sub-segment starts (at most SMAX of them) in registers, then each
// sub-segment, last first, is regenerated into an R-entry register buffer and
// swept backwards.
template <typename Real, int D, int R, int SMAX, bool CB>
__global__ void __launch_bounds__(kThreads)
k_adjoint_recompute(SweepArgs<Real, D> a, const Real* __restrict__ tab) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    static_assert(R % S == 0, "register buffer length must be a multiple of the reducer tile");
    if (gate_closed(a.gate))
        return;
    __shared__ Real tile[StepReducer<D, Real>::kRows][kThreads];
    __shared__ Coef<Real, D> sc;
    stage_coef<CoefInLds<Real, D>::any>(a, &sc);
    __shared__ PoissonTable thr;
    stage_thresholds(a, &thr);
    StepReducer<D, Real> red;
    red.init(tile, blockIdx.x);
    const int64_t m = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool act = m < a.M;
    const int N = a.N, K = a.K, nblk = a.nblk;
    const int nseg = (N + K - 1) / K;
    const Cols cl = make_cols(a.d);
    Real lam[D];
    {
        Real XN[D];
        load_row<Real, D>(slot_row<Real>(a.traj, cl, a.nslots, blockIdx.x, nseg - 1), a.d, XN);
#pragma unroll
        for (int i = 0; i < D; ++i)
            lam[i] = XN[i] - coef_once<Real, D>(a.c, a.lc).xT[i];
        dump_state(a, a.dX, N, m, XN);
        dump_state(a, a.dlam, N, m, lam);
    }
    for (int j = nseg - 1; j >= 0; --j) {
        const int s0 = j * K;
        const int s1 = min(s0 + K, N);
        const int ns = (s1 - s0 + R - 1) / R;
        Real sub[SMAX][D];
        Real X[D];
        if (j == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i)
                X[i] = coef_once<Real, D>(a.c, a.lc).x0[i];
        } else {
            load_row<Real, D>(slot_row<Real>(a.traj, cl, a.nslots, blockIdx.x, j - 1), a.d, X);
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
            sub[0][i] = X[i];
        for (int s = 1; s < ns; ++s) {
            for (int k = s0 + (s - 1) * R; k < s0 + s * R; ++k) {
                StepDraws<Real, D> z;
                draws<Real, D>((uint32_t)m, (uint32_t)k, a.iter, a.key0, a.key1, a.thr, a.thr0, z);
                euler_step<Real, D, CB>(a.c, a.lc, tab + (size_t)k * 2 * D, X, z);
            }
#pragma unroll
            for (int t = 1; t < SMAX; ++t)
                if (t == s) {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        sub[t][i] = X[i];
                }
        }
        for (int s = ns - 1; s >= 0; --s) {
            const int a0 = s0 + s * R;
            const int a1 = min(a0 + R, s1);
            Real buf[R][D];
#pragma unroll
            for (int t = 0; t < SMAX; ++t)
                if (t == s) {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        buf[0][i] = sub[t][i];
                }
#pragma unroll
            for (int r = 1; r < R; ++r) {
                if (a0 + r < a1) {
                    const int k = a0 + r - 1;
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        buf[r][i] = buf[r - 1][i];
                    StepDraws<Real, D> z;
                    draws<Real, D>((uint32_t)m, (uint32_t)k, a.iter, a.key0, a.key1, a.thr, a.thr0, z);
                    euler_step<Real, D, CB>(a.c, a.lc, tab + (size_t)k * 2 * D, buf[r], z);
                }
            }
            // Backward over the sub-segment in chunks of one reducer tile
            // (R is a multiple of the tile height), with one flush per chunk.
            // A step's partial sum does not depend on the tile it is flushed
            // in, so the chunking only fixes where the flush code sits.
#pragma unroll
            for (int c0 = R - S; c0 >= 0; c0 -= S) {
                const int top = min(a0 + c0 + S, a1) - 1;  // highest step of the chunk
                if (top < a0 + c0)
                    continue;
#pragma unroll
                for (int i = S - 1; i >= 0; --i) {
                    const int r = c0 + i;
                    const int k = a0 + r;
                    if (k <= top) {
                        Real v[D];
#pragma unroll
                        for (int c = 0; c < D; ++c)
                            v[c] = act ? lam[c] : (Real)0;
                        red.put(top - k, v);
                        if (k >= 1) {
                            adjoint_step<Real, D, CoefInLds<Real, D>::adjoint, CB>(
                                a.c, a.lc, tab + (size_t)k * 2 * D + D, buf[r], lam);
                            dump_state(a, a.dX, k, m, buf[r]);
                            dump_state(a, a.dlam, k, m, lam);
                        }
                    }
                }
                red.flush_tile(top, top - (a0 + c0) + 1, a.part, nblk);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Checkpoint-recompute adjoint that regenerates each segment once.  The states
// of a segment [s0, s1) (K steps) do not fit the registers when d K is large
// (d = 8, K = 64: 512 values per lane), and the register kernel above then
// regenerates every step twice.  Here each block owns a scratch region of K
// slots (slot q = X_{s0+q}, rows of 256 lanes as in the trajectory layout):
// for each segment, last first, it reloads the checkpoint into slot 0,
// regenerates X_{s0+1} .. X_{s1-1} into slots 1 .. K-1 (X_{s1} is the next
// checkpoint and is not needed), and sweeps the segment backwards reading the
// slots a reducer tile at a time, the next tile's loads issued before the
// current tile is swept.  Each lane reads back only what it wrote (after a
// fence).  The grid is persistent: gridDim.x blocks (at most kSegBlocks) take
// the 256-path groups g = blockIdx.x, blockIdx.x + gridDim.x, ..., so the
// scratch is gridDim.x regions whatever M is.  The steps, the draws and the
// reduction are those of the other sweeps: the result is bitwise the stored
// variant's.

// Slots q, q-1, ..., q-S+1 of a segment region into X[0..S-1] (q >= S-1), by
// raw buffer loads with the default cache policy (the slots were just written
// and are read once, soon).
template <typename Real, int D>
__device__ __forceinline__ void seg_load_full(const Real* region, int64_t stride, int q,
                                              const uint32_t* voff, int d, Real (*X)[D]) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    const Real* base = region + (int64_t)(q - S + 1) * stride;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)base, (short)0, (int)(S * stride * (int64_t)sizeof(Real)), kBufferConfig);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            // non-temporal: each regenerated state is read back once (c3/c4
            // segment adjoint 9.95 -> 9.67 ms against cached loads)
            const Real v = buffer_load<Real, kNontemporal>(
                r, voff[c], (uint32_t)((S - 1 - s) * stride * (int64_t)sizeof(Real)));
            X[s][c] = c < d ? v : (Real)0;
        }
}

// The last tile of a segment (q < S-1): slots q .. 0, then slot 0 again (unused).
template <typename Real, int D>
__device__ __forceinline__ void seg_load_tail(const Real* region, int64_t stride, int q, int d,
                                              Real (*X)[D]) {
    constexpr int S = StepReducer<D, Real>::kSteps;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const Real* row = region + (int64_t)(q - s > 0 ? q - s : 0) * stride;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int ce = c < d ? c : d - 1;
            const Real v = row[ce * kThreads + threadIdx.x];
            X[s][c] = c < d ? v : (Real)0;
        }
    }
}

template <typename Real, int D>
__device__ __forceinline__ void seg_load(const Real* region, int64_t stride, int q,
                                         const uint32_t* voff, int d, Real (*X)[D]) {
    if (q >= StepReducer<D, Real>::kSteps - 1)
        seg_load_full<Real, D>(region, stride, q, voff, d, X);
    else
        seg_load_tail<Real, D>(region, stride, q, d, X);
}

template <typename Real, int D>
__device__ __forceinline__ void seg_store(Real* __restrict__ row, int d, const Real* X) {
    buffer_store_row<Real, D, 0>(row, d, X);
}

template <typename Real, int D, bool DUMP, bool CB>
__global__ void __launch_bounds__(kThreads, sizeof(Real) == 4 ? 4 : 1)
k_adjoint_segments(SweepArgs<Real, D> a, const Real* __restrict__ tab, Real* __restrict__ scratch) {
    constexpr int S = StepReducer<D, Real>::kSteps;
    if (gate_closed(a.gate))
        return;
    __shared__ Real tile[StepReducer<D, Real>::kRows][kThreads];
    __shared__ Coef<Real, D> sc;
    stage_coef<CoefInLds<Real, D>::any>(a, &sc);
    __shared__ PoissonTable thr;
    stage_thresholds(a, &thr);
    const int N = a.N, K = a.K;
    const int nseg = (N + K - 1) / K;
    const Cols cl = make_cols(a.d);
    Real* region = scratch + (int64_t)blockIdx.x * K * cl.stride;
    uint32_t voff[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const int ce = c < a.d ? c : a.d - 1;
        voff[c] = (uint32_t)((ce * kThreads + threadIdx.x) * sizeof(Real));
    }
    for (int64_t g = blockIdx.x; g < a.nblk; g += gridDim.x) {
        StepReducer<D, Real> red;
        red.init(tile, (int)g);
        const int64_t m = g * kThreads + threadIdx.x;
        const bool act = m < a.M;
        Real lam[D];
        {
            Real XN[D];
            load_row<Real, D>(slot_row<Real>(a.traj, cl, a.nslots, g, nseg - 1), a.d, XN);
#pragma unroll
            for (int i = 0; i < D; ++i)
                lam[i] = XN[i] - coef_once<Real, D>(a.c, a.lc).xT[i];
            if (DUMP) {
                dump_state(a, a.dX, N, m, XN);
                dump_state(a, a.dlam, N, m, lam);
            }
        }
        for (int j = nseg - 1; j >= 0; --j) {
            const int s0 = j * K;
            const int s1 = min(s0 + K, N);
            {
                Real X[D];
                if (j == 0) {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        X[i] = coef_once<Real, D>(a.c, a.lc).x0[i];
                } else {
                    load_row<Real, D>(slot_row<Real>(a.traj, cl, a.nslots, g, j - 1), a.d, X);
                }
                seg_store<Real, D>(region, a.d, X);
                Real* row = region + cl.stride;
                for (int k = s0; k < s1 - 1; ++k) {
                    StepDraws<Real, D> z;
                    draws<Real, D>((uint32_t)m, (uint32_t)k, a.iter, a.key0, a.key1, a.thr, a.thr0, z);
                    euler_step<Real, D, CB>(a.c, a.lc, tab + (size_t)k * 2 * D, X, z);
                    seg_store<Real, D>(row, a.d, X);
                    row += cl.stride;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            // backwards over the segment, a reducer tile at a time: two tile
            // buffers in turn (the loop is unrolled by two, so no tile is
            // copied), the next tile's loads issued before the current tile
            // is swept; a group with every path active skips the masking
            Real ta[S][D], tb[S][D];
            const bool full = (g + 1) * kThreads <= a.M;
            auto sweep = [&](Real (*X)[D], int k) {
                const int cnt = k - s0 + 1 < S ? k - s0 + 1 : S;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int kk = k - s;
                    if (s < cnt) {
                        if (full) {
                            red.put(s, lam);
                        } else {
                            Real v[D];
#pragma unroll
                            for (int c = 0; c < D; ++c)
                                v[c] = act ? lam[c] : (Real)0;
                            red.put(s, v);
                        }
                        if (kk >= 1) {
                            adjoint_step<Real, D, CoefInLds<Real, D>::any, CB>(
                                a.c, a.lc, tab + (size_t)kk * 2 * D + D, X[s], lam);
                            if (DUMP) {
                                dump_state(a, a.dX, kk, m, X[s]);
                                dump_state(a, a.dlam, kk, m, lam);
                            }
                        }
                    }
                }
                red.flush_tile(k, cnt, a.part, a.nblk);
            };
            int k = s1 - 1;
            seg_load<Real, D>(region, cl.stride, k - s0, voff, a.d, ta);
            for (;;) {
                int kn = k - S;
                if (kn >= s0)
                    seg_load<Real, D>(region, cl.stride, kn - s0, voff, a.d, tb);
                sweep(ta, k);
                if (kn < s0)
                    break;
                k = kn;
                kn = k - S;
                if (kn >= s0)
                    seg_load<Real, D>(region, cl.stride, kn - s0, voff, a.d, ta);
                sweep(tb, k);
                if (kn < s0)
                    break;
                k = kn;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Step k's gradient (one block): sums the d rows (k, c) of block partials in
// a fixed order, then g_k = nu u_k + B^T (sum / M); a non-finite entry raises
// the flag.  sh: kThreads doubles of LDS, G: 8.
__device__ __forceinline__ void finalize_grad_step(const double* __restrict__ part, int nblk,
                                                   int D, int d, int64_t M, double nu,
                                                   const double* __restrict__ u, const BMat& B,
                                                   double* g, WsHeader* hdr, int k, double* sh,
                                                   double* G) {
    for (int c = 0; c < d; ++c) {
        const double* row = part + (size_t)(k * D + c) * nblk;
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kThreads)
            s += row[b];
        s = block_sum(s, sh);
        if (threadIdx.x == 0)
            G[c] = s / (double)M;
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < d) {
        double v = 0.0;
        for (int j = 0; j < d; ++j)
            v += B.b[j * d + i] * G[j];
        const double gi = nu * u[(size_t)k * d + i] + v;
        g[(size_t)k * d + i] = gi;
        if (!isfinite(gi))
            hdr->nonfinite = 1;
    }
}

// One block per step k.
__global__ void __launch_bounds__(kThreads)
k_finalize_grad(const double* __restrict__ part, int nblk, int D, int d, int64_t M, double nu,
                const double* __restrict__ u, BMat B, double* __restrict__ g, WsHeader* hdr,
                Gate gate) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    __shared__ double G[8];
    finalize_grad_step(part, nblk, D, d, M, nu, u, B, g, hdr, blockIdx.x, sh, G);
}

// Sufficient decrease J(u - zeta g) <= J(u) - c zeta ||g||^2_L2 on the same
// draws (a non-finite trial cost is rejected); on acceptance records
// ||u' - u||^2_L2, moves u to u', writes the iteration's log entry and opens
// the next phase of the device-driven iteration (see LsArmijo).  All threads
// of one block; sh: kThreads doubles of LDS.
__device__ __forceinline__ void armijo_step(WsHeader* hdr, LsLog* __restrict__ ring,
                                            double* __restrict__ u, const double* __restrict__ ut,
                                            int nd, const LsArmijo& ls, double* sh) {
    __shared__ int acc;
    if (threadIdx.x == 0) {
        const double J = hdr->J, Jt = hdr->J_trial;
        acc = (isfinite(Jt) && Jt <= J - ls.c_armijo * ls.zeta * hdr->gnorm2) ? 1 : 0;
        hdr->accept = acc;
    }
    __syncthreads();
    if (!acc) {
        if (threadIdx.x == 0) {
            if (ls.j + 1 >= ls.max_backtracks) {
                hdr->ls_status = JD_ELINESEARCH;
                hdr->ls_phase = kLsStop;
            } else {
                hdr->ls_phase = ls_phase(ls.n, ls.j + 1);
            }
        }
        return;
    }
    double e = 0.0;
    for (int q = threadIdx.x; q < nd; q += kThreads) {
        const double r = ut[q] - u[q];
        e += r * r;
    }
    e = block_sum(e, sh);
    for (int q = threadIdx.x; q < nd; q += kThreads)
        u[q] = ut[q];
    if (threadIdx.x == 0) {
        const double E2 = ls.dt * e;
        hdr->E2 = E2;
        LsLog& L = ring[ls.n % kLsLogCap];
        L.J = hdr->J;
        L.gnorm2 = hdr->gnorm2;
        L.zeta = ls.zeta;
        L.J_new = hdr->J_trial;
        L.E2 = E2;
        L.iter = ls.iter;
        L.backtracks = ls.j;
        L.n = ls.n;
        hdr->ls_done = ls.n + 1;
        if (ls.n + 1 >= ls.n_max || sqrt(E2) <= ls.tol) {
            hdr->ls_status = kLsDone;
            hdr->ls_phase = kLsStop;
        } else {
            hdr->ls_phase = ls_phase(ls.n + 1, -1);
        }
    }
}

// Gated by the phase of trial (ls.n, ls.j).
__global__ void __launch_bounds__(kThreads)
k_armijo(WsHeader* hdr, LsLog* __restrict__ ring, double* __restrict__ u,
         const double* __restrict__ ut, int nd, LsArmijo ls) {
    if (hdr->ls_phase != ls_phase(ls.n, ls.j))
        return;
    __shared__ double sh[kThreads];
    armijo_step(hdr, ring, u, ut, nd, ls, sh);
}

// After the gradient of iteration n (one thread): on to trial (n, 0), or stop
// with JD_ENONFINITE.
__device__ __forceinline__ void ls_after_grad_step(WsHeader* hdr, int n) {
    if (hdr->ls_phase == ls_phase(n, -1)) {
        if (hdr->nonfinite) {
            hdr->ls_status = JD_ENONFINITE;
            hdr->ls_phase = kLsStop;
        } else {
            hdr->ls_phase = ls_phase(n, 0);
        }
    }
}

// J = (1/M) sum C + nu dt/2 sum |u|^2, and if g is given also dt sum |g|^2
// (one block); flags non-finite results, then runs the line-search tail.
__device__ __forceinline__ void finalize_cost_block(const double* __restrict__ cpart, int nblk,
                                                    int64_t M, double nu, double dt,
                                                    const double* __restrict__ u, const double* g,
                                                    int nd, double* J_out, WsHeader* hdr, int slot,
                                                    const LsTail& tail, double* sh) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
        s += cpart[b];
    const double csum = block_sum(s, sh);
    double uu = 0.0;
    for (int q = threadIdx.x; q < nd; q += kThreads)
        uu += u[q] * u[q];
    uu = block_sum(uu, sh);
    double gg = 0.0;
    int bad = 0;
    if (g != nullptr) {
        for (int q = threadIdx.x; q < nd; q += kThreads) {
            gg += g[q] * g[q];
            bad |= !isfinite(g[q]);
        }
        gg = block_sum(gg, sh);
        bad = (int)block_sum((double)bad, sh);
    }
    if (threadIdx.x == 0) {
        const double J = csum / (double)M + 0.5 * nu * dt * uu;
        if (slot == 0) {
            hdr->J = J;
            if (g != nullptr)
                hdr->gnorm2 = dt * gg;
        } else {
            hdr->J_trial = J;
        }
        if (J_out != nullptr)
            *J_out = J;
        // a trial's cost (slot 1) may overflow: the Armijo test rejects it
        if (slot == 0 && (!isfinite(J) || bad))
            hdr->nonfinite = 1;
        if (tail.mode == kLsTailAfterGrad)
            ls_after_grad_step(hdr, tail.n);
    }
    if (tail.mode == kLsTailArmijo) {
        __syncthreads();
        armijo_step(hdr, tail.ring, tail.u, tail.ut, tail.nd, tail.ls, sh);
    }
}

__global__ void __launch_bounds__(kThreads)
k_finalize_cost(const double* __restrict__ cpart, int nblk, int64_t M, double nu, double dt,
                const double* __restrict__ u, const double* __restrict__ g, int nd,
                double* __restrict__ J_out, WsHeader* hdr, int slot, Gate gate, LsTail tail) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    finalize_cost_block(cpart, nblk, M, nu, dt, u, g, nd, J_out, hdr, slot, tail, sh);
}

__global__ void __launch_bounds__(kThreads)
k_trial(const double* __restrict__ u, const double* __restrict__ g, double zeta,
        double* __restrict__ ut, int nd, Gate gate) {
    if (gate_closed(gate))
        return;
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q < nd)
        ut[q] = u[q] - zeta * g[q];
}

__global__ void k_ls_start(WsHeader* hdr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        hdr->nonfinite = 0;
        hdr->accept = 0;
        hdr->ls_status = kLsRunning;
        hdr->ls_phase = ls_phase(0, -1);
        hdr->ls_done = 0;
    }
}

// After the evaluation of J(u^n), g^n: stop on a non-finite result, else
// open the first trial.
__global__ void k_ls_after_grad(WsHeader* hdr, int n) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        ls_after_grad_step(hdr, n);
}

__global__ void k_clear_flag(WsHeader* hdr) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        hdr->nonfinite = 0;
}

// ---------------------------------------------------------------------------
template <typename Real, int D>
__global__ void __launch_bounds__(kThreads)
k_draws(SweepArgs<Real, D> a, PoissonTable pt, int64_t m0, int64_t mc, int k0, int kc,
        Real* __restrict__ zw, Real* __restrict__ zj, int32_t* __restrict__ counts) {
    __shared__ PoissonTable tb;
    if (threadIdx.x < 32)
        tb.tm1[threadIdx.x] = pt.tm1[threadIdx.x];
    if (threadIdx.x == 0)
        tb.jmax = pt.jmax;
    __syncthreads();
    a.thr = &tb;
    a.thr0 = tb.tm1[0];
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= mc * kc)
        return;
    const int64_t p = idx / kc;
    const int q = (int)(idx - p * kc);
    StepDraws<Real, D> z;
    draws<Real, D>((uint32_t)(m0 + p), (uint32_t)(k0 + q), a.iter, a.key0, a.key1, a.thr, a.thr0, z);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (i < a.d) {
            if (zw)
                zw[idx * a.d + i] = z.zw[i];
            if (zj)
                zj[idx * a.d + i] = jump_normal(z, i);
        }
    }
    if (counts)
        counts[idx] = z.n;
}

__global__ void __launch_bounds__(kThreads)
k_philox(uint32_t key0, uint32_t key1, const uint32_t* __restrict__ ctr, int64_t n,
         uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n)
        return;
    uint32_t w[4];
    philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key0, key1, w);
    for (int q = 0; q < 4; ++q)
        out[4 * i + q] = w[q];
}

// ===========================================================================
// Launchers.

template <typename Real, int D>
static SweepArgs<Real, D> make_args(const HostProblem& p, const HostRun& r) {
    SweepArgs<Real, D> a;
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            a.c.A[i * D + j] = (Real)p.A[i * D + j];
            a.c.AT[j * D + i] = (Real)p.A[i * D + j];
        }
    const double sq = sqrt(p.dt);
    for (int i = 0; i < D; ++i) {
        a.c.sq[i] = (Real)(sq * p.s[i]);
        a.c.jm[i] = (Real)p.jm[i];
        a.c.js[i] = (Real)p.js[i];
        a.c.x0[i] = (Real)p.x0[i];
        a.c.xT[i] = (Real)p.xT[i];
    }
    a.c.dt = (Real)p.dt;
    a.c.c3 = (Real)p.cubic;
    a.thr = nullptr;
    a.thr0 = 0;
    a.lc = nullptr;
    a.gate = kNoGate;
    a.traj = nullptr;
    a.part = nullptr;
    a.M = r.M;
    a.nblk = r.nblk;
    a.nslots = r.mode == JD_RECOMPUTE ? (p.N + r.K - 1) / r.K : p.N;
    a.N = p.N;
    a.d = p.d;
    a.K = r.K;
    a.key0 = (uint32_t)(r.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(r.seed >> 32);
    a.iter = r.iter;
    a.dt64 = p.dt;
    a.dm0 = 0;
    a.dcount = 0;
    a.dX = nullptr;
    a.dlam = nullptr;
    a.dcost = nullptr;
    if (r.dump != nullptr) {
        a.dm0 = r.dump->m0;
        a.dcount = r.dump->count;
        a.dX = (Real*)r.dump->X;
        a.dlam = (Real*)r.dump->lam;
        a.dcost = r.dump->cost;
    }
    return a;
}

static BMat make_B(const HostProblem& p) {
    BMat B;
    for (int i = 0; i < 64; ++i)
        B.b[i] = i < p.d * p.d ? p.B[i] : 0.0;
    return B;
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Dispatch on (precision, padded dimension).
#define JD_DISPATCH(prec, D, FN)                                 \
    do {                                                         \
        if ((prec) == JD_FP64) {                                 \
            switch (D) {                                         \
            case 1: FN(double, 1); break;                        \
            case 2: FN(double, 2); break;                        \
            case 4: FN(double, 4); break;                        \
            default: FN(double, 8); break;                       \
            }                                                    \
        } else {                                                 \
            switch (D) {                                         \
            case 1: FN(float, 1); break;                         \
            case 2: FN(float, 2); break;                         \
            case 4: FN(float, 4); break;                         \
            default: FN(float, 8); break;                        \
            }                                                    \
        }                                                        \
    } while (0)

hipError_t launch_setup(const HostProblem& p, const HostRun& r, const double* u, void* tab,
                        WsHeader* hdr, int clear_flag, hipStream_t st, Gate gate) {
    const BMat B = make_B(p);
    const unsigned nb = (unsigned)table_blocks(p.N, p.D);
#define JD_SETUP(T, DD)                                                                           \
    hipLaunchKernelGGL((k_table<T, DD>), dim3(nb), dim3(kThreads), 0, st, u, p.xd, (T*)tab, p.N,    \
                       p.d, B, hdr, clear_flag, p.poisson, gate, nullptr, 0.0, nullptr)
    JD_DISPATCH(r.prec, p.D, JD_SETUP);
#undef JD_SETUP
    return hipGetLastError();
}

hipError_t launch_setup_trial(const HostProblem& p, const HostRun& r, const double* u,
                              const double* g, double zeta, double* ut, void* tab, WsHeader* hdr,
                              hipStream_t st, Gate gate) {
    const BMat B = make_B(p);
    const unsigned nb = (unsigned)table_blocks(p.N, p.D);
#define JD_SETUP(T, DD)                                                                           \
    hipLaunchKernelGGL((k_table<T, DD>), dim3(nb), dim3(kThreads), 0, st, u, p.xd, (T*)tab, p.N,    \
                       p.d, B, hdr, 0, p.poisson, gate, g, zeta, ut)
    JD_DISPATCH(r.prec, p.D, JD_SETUP);
#undef JD_SETUP
    return hipGetLastError();
}

hipError_t launch_forward(const HostProblem& p, const HostRun& r, const void* tab, void* traj,
                          int fwd_mode, double* cpart, const WsHeader* hdr, hipStream_t st,
                          Gate gate, const void* noise) {
    const unsigned nb = (unsigned)r.nblk;
#define JD_FWD_NZ(T, DD, CB, NZ)                                                                    \
    do {                                                                                            \
        SweepArgs<T, DD> a = make_args<T, DD>(p, r);                                                \
        a.gate = gate;                                                                              \
        a.traj = traj;                                                                              \
        a.thr = &hdr->poisson;                                                                      \
        if (fwd_mode == FWD_STORE)                                                                  \
            hipLaunchKernelGGL((k_forward<T, DD, FWD_STORE, CB, NZ>), dim3(nb), dim3(kThreads), 0,  \
                               st, a, (const T*)tab, cpart, (const T*)noise);                       \
        else if (fwd_mode == FWD_CKPT)                                                              \
            hipLaunchKernelGGL((k_forward<T, DD, FWD_CKPT, CB, NZ>), dim3(nb), dim3(kThreads), 0,   \
                               st, a, (const T*)tab, cpart, (const T*)noise);                       \
        else                                                                                        \
            hipLaunchKernelGGL((k_forward<T, DD, FWD_COST, CB, NZ>), dim3(nb), dim3(kThreads), 0,   \
                               st, a, (const T*)tab, cpart, (const T*)noise);                       \
    } while (0)
#define JD_FWD_CB(T, DD, CB)                                                                        \
    do {                                                                                            \
        if (noise != nullptr)                                                                       \
            JD_FWD_NZ(T, DD, CB, true);                                                             \
        else                                                                                        \
            JD_FWD_NZ(T, DD, CB, false);                                                            \
    } while (0)
#define JD_FWD(T, DD)                                                                               \
    do {                                                                                            \
        if (p.cubic != 0.0)                                                                         \
            JD_FWD_CB(T, DD, true);                                                                 \
        else                                                                                        \
            JD_FWD_CB(T, DD, false);                                                                \
    } while (0)
    JD_DISPATCH(r.prec, p.D, JD_FWD);
#undef JD_FWD
#undef JD_FWD_CB
#undef JD_FWD_NZ
    return hipGetLastError();
}

hipError_t launch_setup_noise(const HostProblem& p, const HostRun& r, const double* u, void* tab,
                              void* noise, WsHeader* hdr, int clear_flag, hipStream_t st,
                              Gate gate) {
    const int64_t tb = table_blocks(p.N, p.D);
    const int64_t nb = (int64_t)r.nblk * p.N;
    const unsigned grid = (unsigned)(tb + (nb < kNoiseGrid ? nb : kNoiseGrid));
    const BMat B = make_B(p);
#define JD_NOISE(T, DD)                                                                           \
    do {                                                                                          \
        SweepArgs<T, DD> a = make_args<T, DD>(p, r);                                              \
        a.gate = gate;                                                                            \
        hipLaunchKernelGGL((k_noise<T, DD>), dim3(grid), dim3(kThreads), 0, st, a, (T*)noise,     \
                           p.poisson, (int)tb, u, p.xd, (T*)tab, B, hdr, clear_flag);             \
    } while (0)
    JD_DISPATCH(r.prec, p.D, JD_NOISE);
#undef JD_NOISE
    return hipGetLastError();
}

// Blocks of the persistent segment kernel: as many as are resident at once on
// the current device (its compute units times the kernel's blocks per unit),
// at most the scratch regions of the workspace.
template <typename Real, int D, bool DUMP, bool CB>
static unsigned seg_grid_for(const HostRun& r) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adjoint_segments<Real, D, DUMP, CB>,
                                                         kThreads, 0) != hipSuccess || n < 1)
            n = 1;
        return n;
    }();
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 1;
    const int64_t g = (int64_t)cus * per_cu;
    return (unsigned)(g < seg_blocks(r) ? g : seg_blocks(r));
}

hipError_t launch_adjoint(const HostProblem& p, const HostRun& r, const void* tab, const void* traj,
                          double* apart, void* seg, const WsHeader* hdr, hipStream_t st,
                          Gate gate) {
    const unsigned nb = (unsigned)r.nblk;
    const bool segments = r.mode == JD_RECOMPUTE && recompute_uses_segments(r.prec, p.D, r.K);
#define JD_ADJ_CB(T, DD, CB)                                                                      \
    do {                                                                                          \
        const unsigned seg_grid = !segments ? 0u                                                  \
                                  : r.dump != nullptr ? seg_grid_for<T, DD, true, CB>(r)          \
                                                      : seg_grid_for<T, DD, false, CB>(r);        \
        SweepArgs<T, DD> a = make_args<T, DD>(p, r);                                              \
        a.gate = gate;                                                                            \
        a.traj = const_cast<void*>(traj);                                                         \
        a.part = apart;                                                                           \
        a.thr = &hdr->poisson;                                                                    \
        if (segments && r.dump != nullptr)                                                        \
            hipLaunchKernelGGL((k_adjoint_segments<T, DD, true, CB>), dim3(seg_grid),             \
                               dim3(kThreads), 0, st, a, (const T*)tab, (T*)seg);                 \
        else if (segments)                                                                        \
            hipLaunchKernelGGL((k_adjoint_segments<T, DD, false, CB>), dim3(seg_grid),            \
                               dim3(kThreads), 0, st, a, (const T*)tab, (T*)seg);                 \
        else if (r.mode == JD_RECOMPUTE)                                                          \
            hipLaunchKernelGGL((k_adjoint_recompute<T, DD, RecomputeShape<T, DD>::R,              \
                                                    RecomputeShape<T, DD>::S, CB>),               \
                               dim3(nb), dim3(kThreads), 0, st, a, (const T*)tab);                \
        else if (r.dump != nullptr)                                                               \
            hipLaunchKernelGGL((k_adjoint_stored<T, DD, true, CB>), dim3(nb), dim3(kThreads), 0,  \
                               st, a, (const T*)tab);                                             \
        else                                                                                      \
            hipLaunchKernelGGL((k_adjoint_stored<T, DD, false, CB>), dim3(nb), dim3(kThreads), 0, \
                               st, a, (const T*)tab);                                             \
    } while (0)
#define JD_ADJ(T, DD)                                                                             \
    do {                                                                                          \
        if (p.cubic != 0.0)                                                                       \
            JD_ADJ_CB(T, DD, true);                                                               \
        else                                                                                      \
            JD_ADJ_CB(T, DD, false);                                                              \
    } while (0)
    JD_DISPATCH(r.prec, p.D, JD_ADJ);
#undef JD_ADJ
#undef JD_ADJ_CB
    return hipGetLastError();
}

hipError_t launch_cost_grad_stored(const HostProblem& p, const HostRun& r, const void* tab,
                                  void* traj, double* cpart, double* apart, const WsHeader* hdr,
                                  hipStream_t st, Gate gate, const void* noise) {
    const unsigned nb = (unsigned)r.nblk;
#define JD_CG_NZ(T, DD, CB, NZ)                                                                   \
    hipLaunchKernelGGL((k_cost_grad_stored<T, DD, CB, NZ>), dim3(nb), dim3(kThreads), 0, st, a,   \
                       (const T*)tab, cpart, (const T*)noise)
#define JD_CG(T, DD)                                                                              \
    do {                                                                                          \
        SweepArgs<T, DD> a = make_args<T, DD>(p, r);                                              \
        a.gate = gate;                                                                            \
        a.traj = traj;                                                                            \
        a.part = apart;                                                                           \
        a.thr = &hdr->poisson;                                                                    \
        if (p.cubic != 0.0) {                                                                     \
            if (noise != nullptr)                                                                 \
                JD_CG_NZ(T, DD, true, true);                                                      \
            else                                                                                  \
                JD_CG_NZ(T, DD, true, false);                                                     \
        } else {                                                                                  \
            if (noise != nullptr)                                                                 \
                JD_CG_NZ(T, DD, false, true);                                                     \
            else                                                                                  \
                JD_CG_NZ(T, DD, false, false);                                                    \
        }                                                                                         \
    } while (0)
    JD_DISPATCH(r.prec, p.D, JD_CG);
#undef JD_CG
#undef JD_CG_NZ
    return hipGetLastError();
}

hipError_t launch_finalize_grad(const HostProblem& p, const HostRun& r, const double* apart,
                                const double* u, double* g, WsHeader* hdr, hipStream_t st,
                                Gate gate) {
    hipLaunchKernelGGL(k_finalize_grad, dim3(p.N), dim3(kThreads), 0, st, apart, r.nblk, p.D, p.d,
                       r.M, p.nu, u, make_B(p), g, hdr, gate);
    return hipGetLastError();
}

hipError_t launch_finalize_cost(const HostProblem& p, const HostRun& r, const double* cpart,
                                const double* u, const double* g, double* J_out, WsHeader* hdr,
                                int slot, hipStream_t st, Gate gate, const LsTail* tail) {
    LsTail t{};
    t.mode = kLsTailNone;
    if (tail != nullptr)
        t = *tail;
    hipLaunchKernelGGL(k_finalize_cost, dim3(1), dim3(kThreads), 0, st, cpart, r.nblk, r.M, p.nu,
                       p.dt, u, g, p.N * p.d, J_out, hdr, slot, gate, t);
    return hipGetLastError();
}

hipError_t launch_trial(const double* u, const double* g, double zeta, double* ut, int nd,
                        hipStream_t st, Gate gate) {
    hipLaunchKernelGGL(k_trial, dim3(blocks_for(nd)), dim3(kThreads), 0, st, u, g, zeta, ut, nd,
                       gate);
    return hipGetLastError();
}

hipError_t launch_armijo(WsHeader* hdr, LsLog* ring, double* u, const double* ut, int nd,
                         const LsArmijo& ls, hipStream_t st) {
    hipLaunchKernelGGL(k_armijo, dim3(1), dim3(kThreads), 0, st, hdr, ring, u, ut, nd, ls);
    return hipGetLastError();
}

hipError_t launch_ls_start(WsHeader* hdr, hipStream_t st) {
    hipLaunchKernelGGL(k_ls_start, dim3(1), dim3(64), 0, st, hdr);
    return hipGetLastError();
}

hipError_t launch_ls_after_grad(WsHeader* hdr, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_ls_after_grad, dim3(1), dim3(64), 0, st, hdr, n);
    return hipGetLastError();
}

hipError_t launch_clear_flag(WsHeader* hdr, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, hdr);
    return hipGetLastError();
}

hipError_t launch_draws(const HostProblem& p, const HostRun& r, int64_t m0, int64_t mc, int k0,
                        int kc, void* zw, void* zj, int32_t* counts, hipStream_t st) {
    const unsigned nb = blocks_for(mc * kc);
#define JD_DRAWS(T, DD)                                                                           \
    do {                                                                                          \
        SweepArgs<T, DD> a = make_args<T, DD>(p, r);                                              \
        hipLaunchKernelGGL((k_draws<T, DD>), dim3(nb), dim3(kThreads), 0, st, a, p.poisson, m0, mc, k0, kc,  \
                           (T*)zw, (T*)zj, counts);                                               \
    } while (0)
    JD_DISPATCH(r.prec, p.D, JD_DRAWS);
#undef JD_DRAWS
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out,
                         hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), ctr, n, out);
    return hipGetLastError();
}

}  // namespace jd
