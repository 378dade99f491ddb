// Kernels of the paper's model problem (include/jd_feedback.h) on gfx950:
//
//  k_fb_table          mu (FP64) -> path-precision rows padded to nvp, targets,
//                      Keilson-Storer factors; stages the Poisson table
//  k_fb_forward        forward sweep, one particle per lane (G per lane for
//                      rings): shape functions, feedback control, ring
//                      coupling, draws, Euler step, jumps, FP64 cost; stores
//                      the trajectory and each step's jump count
//  k_fb_adjoint        backward sweep over the stored trajectory (or, for the
//                      surrogate gradient, over counter-drawn surrogate
//                      states); the per-step gradient sum over particles runs
//                      on the matrix cores of the path precision
//  k_fb_forward_grad   the surrogate gradient's forward: forward sweep plus
//                      the control term of the gradient, nothing stored
//  k_fb_forward_adapted, k_fb_adjoint_adapted
//                      the same on the jump-adapted grid (sub-steps between
//                      each particle's jump times, a stack of post-jump states)
//  k_fb_finalize_grad  fixed-order FP64 sum of the per-block gradient partials
//  k_fb_finalize_cost  fixed-order FP64 sum of the path costs, ||g||^2
//  k_fb_draws          initial states, normals and jump counts (parity checks)
//
// The paper's method: model equation and jump law (Section 5, eq.
// SDE_splitted_drift_Euler, eq. jump_law, eq. collision_frequency), control
// and shape functions (eq. control_structure, eq. Gaussian_RBF), cost (eq.
// discrete_functional, eq. tracking_cost), adjoint (eq.
// adjoint_eq_approximation), gradient (eq. definition_Gradient); the
// jump-adapted grid (Section 3, Algorithms 5.1-5.2); the surrogate adjoint
// (Section 6.5); coupled particles, the start on the ellipse and the ellipse
// cost of Section 6.4 (eq. interacting_model, eq. coupled_ellipse, eq.
// phonon_functional_tracking).
#include "fb_launch.hpp"
#include "jd_device.hpp"

namespace jd {

constexpr uint32_t kFbInitStep = 0xFFFFFFFFu;  // counter word 1 of the initial-state draws
constexpr uint32_t kFbSurrWord = 0xFFFFFFFEu;  // counter word 1 of the surrogate samples

// gamma^n and sqrt(V_n), n = 0..31, passed by value to the table kernel.
struct FbKs {
    double v[64];
};

template <typename Real>
struct FbArgs {
    int64_t M;     // particles
    int64_t nsys;  // rings (np > 1)
    int np, sb;    // particles per ring, rings per workgroup
    int cost_kind;
    Real omega, iax2, iav2, ax, av;  // coupling, 1/ax^2, 1/av^2, half-axes
    int nblk, N, nx, nv;
    Real dt, sqb1, sqb2, eta, eps, alpha, hadt, inv2s2, invs2;
    Real b1, b2, gamma, sbeta;  // jump-adapted grid: noise scales, gamma, 1/sqrt(2 beta)
    Real xc0, dxc, vc0, dvc;  // centres x^i = xc0 + i dxc, v^l = vc0 + l dvc
    Real z0x, z0v, s0x, s0v;
    const Real* sd;  // surrogate states' standard deviations per step ((N+1) x 2)
    double* mom;     // surrogate forward: per-step moment partials, or null
    int init_kind;
    uint32_t key0, key1, iter;
    const PoissonTable* thr;  // in the workspace header, then in the block's LDS
    uint32_t thr0;            // thr->tm1[0], read once per block
    Gate gate;  // launch gate (word null: always runs)
    double dt64;
    int64_t dm0, dcount;  // per-path dumps
    Real* dX;
    Real* dlam;
    double* dcost;
};

// The bump of the shape functions at the scaled distance q = eps r:
// b = exp(-1/(1 - q^2)) inside the support, 0 outside; bump_dq also returns
// d = b q / (1 - q^2)^2, so that b'(r) = -2 eps d (callers apply -2 eps once
// to their sums of d).  Callers form q as eps (x - c0) - i eps dc for the
// centre c0 + i dc.  s = 1 - q^2 is clamped below at 1e-3: there the exact
// value exp(-1/s) <= e^-1000 is 0 in FP32 and FP64 alike, and so is the
// clamped one, so the clamp is exact and needs no branch.
__device__ __forceinline__ float bump_q(float q) {
    const float s = fmaxf(fmaf(-q, q, 1.0f), 1e-3f);
    return __builtin_amdgcn_exp2f(-1.44269504088896340736f * __builtin_amdgcn_rcpf(s));
}
// 1/s for s in [1e-3, 1]: the hardware estimate refined by two steps of
// Newton's iteration r <- r + r (1 - s r), each of which squares the relative
// error, so the estimate's ~2^-26 ends within an ulp or two of the quotient
// (an IEEE division costs about twice the instructions: f4 FP64 step 42.4 ->
// 41.0 ms, ring2 FP64 45.7 -> 43.2 ms).
__device__ __forceinline__ double fb_rcp(double s) {
    double r = __builtin_amdgcn_rcp(s);
    r = fma(fma(-s, r, 1.0), r, r);
    return fma(fma(-s, r, 1.0), r, r);
}
// exp(-y) for y in [1, 1000]: -y = k ln2 + r with k = rint(-y / ln2) and r
// reduced against a two-part ln 2 (Cody and Waite's method: the high part
// has 41 significant bits, so k times it is exact for |k| < 2^12), exp(r) by
// its Taylor series to degree 13 (|r| <= ln2 / 2: truncation error below
// 5e-18), and 2^k applied exactly by ldexp (0 or subnormal far below 2^-1022,
// as exp gives).  Skips the library exp's range checks: f4 FP64 step 40.7 ->
// 38.2 ms, ring2 FP64 43.4 -> 41.3 ms.
__device__ __forceinline__ double fb_exp_neg(double y) {
    const double k = rint(y * -1.4426950408889634);
    double r = fma(k, -0.6931471805601177, -y);
    r = fma(k, 1.7239444525614835e-13, r);
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}
__device__ __forceinline__ double bump_q(double q) {
    const double s = fmax(fma(-q, q, 1.0), 1e-3);
    return fb_exp_neg(fb_rcp(s));
}
__device__ __forceinline__ float bump_dq(float q, float& d) {
    const float s = fmaxf(fmaf(-q, q, 1.0f), 1e-3f);
    const float rs = __builtin_amdgcn_rcpf(s);
    const float b = __builtin_amdgcn_exp2f(-1.44269504088896340736f * rs);
    d = b * q * rs * rs;
    return b;
}
__device__ __forceinline__ double bump_dq(double q, double& d) {
    const double s = fmax(fma(-q, q, 1.0), 1e-3);
    const double rs = fb_rcp(s);
    const double b = fb_exp_neg(rs);
    d = b * q * rs * rs;
    return b;
}

template <typename Real>
__device__ __forceinline__ Real fb_exp(Real x);
template <>
__device__ __forceinline__ float fb_exp<float>(float x) {
    return __builtin_amdgcn_exp2f(1.44269504088896340736f * x);
}
template <>
__device__ __forceinline__ double fb_exp<double>(double x) {
    return exp(x);
}

// Initial state of particle m (counter (m, 0xFFFFFFFF, iter, 0)).
template <typename Real>
__device__ __forceinline__ void fb_initial(const FbArgs<Real>& a, uint32_t m, Real& x, Real& v) {
    uint32_t w[4];
    philox4x32_10<true>(m, kFbInitStep, a.iter, 0u, a.key0, a.key1, w);
    if (a.init_kind == 0) {
        const Real R = bm_radius(w[0], (Real)0);
        const Real ub = unit_uniform<Real>(w[1]);
        x = fma(a.s0x, bm_cos(R, ub), a.z0x);
        v = fma(a.s0v, bm_sin(R, ub), a.z0v);
    } else if (a.init_kind == 2) {
        // particle j = m mod np of its ring at angle 2 pi j / np on the ellipse
        double sn, cs;
        sincospi(2.0 * (double)(m % (uint32_t)a.np) / (double)a.np, &sn, &cs);
        const Real R = bm_radius(w[0], (Real)0);
        const Real ub = unit_uniform<Real>(w[1]);
        x = fma(a.s0x, bm_cos(R, ub), (Real)((double)a.ax * cs));
        v = fma(a.s0v, bm_sin(R, ub), (Real)((double)a.av * sn));
    } else {
        x = fma(a.s0x, fma((Real)2, unit_uniform<Real>(w[0]), (Real)-1), a.z0x);
        v = fma(a.s0v, fma((Real)2, unit_uniform<Real>(w[1]), (Real)-1), a.z0v);
    }
}

// The Keilson-Storer jumps of a step: gamma^n and sqrt(V_n) from the table.
template <typename Real>
__device__ __forceinline__ void ks_factors(const Real* __restrict__ ks, int n, Real& gn, Real& sv) {
    gn = ks[2 * n];
    sv = ks[2 * n + 1];
}

// Shape functions of the velocity, b(v - v^l) for l < NVP (entries l >= nv
// meet zero control coefficients).
template <typename Real, int NVP>
__device__ __forceinline__ void shapes_v(const FbArgs<Real>& a, Real v, Real* pv) {
#pragma unroll
    for (int l = 0; l < NVP; ++l)
        pv[l] = bump_q(fma(-(Real)l, a.eps * a.dvc, a.eps * (v - a.vc0)));
}

// Receives the shape-function values a step computes, and the control u
// (the wave transposes of the gradient reduction); NoSink drops them.
struct NoSink {
    template <typename Real>
    __device__ __forceinline__ void put_x(int, Real) const {}
    template <typename Real, int NVP>
    __device__ __forceinline__ void put_v(const Real*, Real) const {}
};

// s + e = a + b exactly (Knuth's TwoSum; needs the build's -ffp-contract=off).
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// One forward step of one particle: control, draws, Euler step, jumps; cpl is
// the ring force omega (2 x_j - x_{j-1} - x_{j+1}) (a literal 0 without rings).
// FP32 paths carry the rounding error of the state updates in (cx, cv) and add
// it to the next increment (compensated summation): the state then drifts from
// the exact one by the rounding of the increments, which are small beside the
// state, instead of by that of the state itself at every step.  FP64 paths
// update plainly.  Returns the control u_k; the bump values go to the sink.
// The feedback control u = sum_i b(x - x^i) sum_l mu_il b(v - v^l); the bump
// values go to the sink.
template <typename Real, int NVP, typename Sink = NoSink, int RU = 2>
__device__ __forceinline__ Real fb_control(const FbArgs<Real>& a, const Real* __restrict__ mk,
                                           Real x, Real v, const Sink& sink = Sink()) {
    Real pv[NVP];
    shapes_v<Real, NVP>(a, v, pv);
    Real u = 0;
    // RU rows per iteration: the next row's scalar loads overlap this row's
    // work (two: f4 forward 5.03 -> 4.95 ms, adjoint 9.85 -> 9.61 ms; five
    // ran out of scalar registers; the ring forward, held to 64 vector
    // registers, keeps one: 5.7 against 5.9 ms)
#pragma unroll RU
    for (int i = 0; i < a.nx; ++i) {
        const Real bx = bump_q(fma(-(Real)i, a.eps * a.dxc, a.eps * (x - a.xc0)));
        const Real* rw = mk + i * NVP;
        Real t = 0;
#pragma unroll
        for (int l = 0; l < NVP; ++l)
            t = fma(rw[l], pv[l], t);
        u = fma(bx, t, u);
        sink.put_x(i, bx);
    }
    sink.template put_v<Real, NVP>(pv, u);
    return u;
}

// fb_control with the row of one of two steps, chosen per lane (sel: mk1).
template <typename Real, int NVP>
__device__ __forceinline__ Real fb_control_of(const FbArgs<Real>& a, const Real* __restrict__ mk0,
                                              const Real* __restrict__ mk1, bool sel, Real x,
                                              Real v) {
    Real pv[NVP];
    shapes_v<Real, NVP>(a, v, pv);
    Real u = 0;
#pragma unroll 2
    for (int i = 0; i < a.nx; ++i) {
        const Real bx = bump_q(fma(-(Real)i, a.eps * a.dxc, a.eps * (x - a.xc0)));
        const Real* r0 = mk0 + i * NVP;
        const Real* r1 = mk1 + i * NVP;
        Real t = 0;
#pragma unroll
        for (int l = 0; l < NVP; ++l)
            t = fma(sel ? r1[l] : r0[l], pv[l], t);
        u = fma(bx, t, u);
    }
    return u;
}

// The Poisson thresholds in the block's LDS, the first one in a register:
// the sweeps store trajectory rows inside their step loops, and with the
// thresholds in global memory the compiler reloads the first one every step
// and waits for the wave's outstanding stores before the comparison.
template <typename Real>
__device__ __forceinline__ void fb_stage_thresholds(FbArgs<Real>& a, PoissonTable* st) {
    if (threadIdx.x < 32)
        st->tm1[threadIdx.x] = a.thr->tm1[threadIdx.x];
    if (threadIdx.x == 0)
        st->jmax = a.thr->jmax;
    __syncthreads();
    a.thr = st;
    a.thr0 = st->tm1[0];
}

// The jump factor table (64 values) in the block's LDS: its per-lane reads
// (indexed by each lane's jump count) would otherwise wait, through the
// in-order vector-memory counter, for every trajectory load or store the wave
// has in flight.  Returns the LDS copy.
template <typename Real>
__device__ __forceinline__ const Real* fb_stage_ks(const Real* __restrict__ ks, Real* st) {
    if (threadIdx.x < 64)
        st[threadIdx.x] = ks[threadIdx.x];
    __syncthreads();
    return st;
}

template <typename Real, int NVP, typename Sink = NoSink, int RU = 2>
__device__ __forceinline__ Real fb_step(const FbArgs<Real>& a, const Real* __restrict__ mk,
                                        const Real* __restrict__ ks, uint32_t m, int k, Real& x,
                                        Real& v, Real& cx, Real& cv, Real cpl,
                                        const Sink& sink = Sink(), int* n_out = nullptr) {
    const Real u = fb_control<Real, NVP, Sink, RU>(a, mk, x, v, sink);
    uint32_t w[4];
    philox4x32_10<true>(m, (uint32_t)k, a.iter, 0u, a.key0, a.key1, w);
    const Real R = bm_radius(w[0], (Real)0);
    const Real ub = unit_uniform<Real>(w[1]);
    const int n = poisson_count(poisson_word(w), a.thr0, a.thr);
    if (n_out != nullptr)
        *n_out = n;
    Real xn, vs, ex = 0, ev = 0;
    if constexpr (sizeof(Real) == 4) {
        xn = two_sum(x, fma(a.dt, v, fma(a.sqb1, bm_cos(R, ub), cx)), ex);
        vs = two_sum(v, fma(a.dt, fma(-a.eta, x, u) - cpl, fma(a.sqb2, bm_sin(R, ub), cv)), ev);
    } else {
        xn = fma(a.sqb1, bm_cos(R, ub), fma(a.dt, v, x));
        vs = fma(a.sqb2, bm_sin(R, ub), fma(a.dt, fma(-a.eta, x, u) - cpl, v));
    }
    if (__builtin_amdgcn_ballot_w64(n != 0)) {
        Real gn, sv;
        ks_factors(ks, n, gn, sv);
        const Real zj = bm_cos(bm_radius(w[2], (Real)0), unit_uniform<Real>(w[3]));
        const Real vj = fma(sv, zj, gn * vs);
        vs = n != 0 ? vj : vs;
        ev = n != 0 ? gn * ev : ev;
    }
    x = xn;
    v = vs;
    cx = ex;
    cv = ev;
    return u;
}

// The surrogate states of Section 6.5 take one position and velocity sample
// per particle and realization: the Box-Muller pair (cx, cv) of words 0, 1 of
// Philox block (m, 0xFFFFFFFE, iter, 1), and at step k the state
// zd_k + sqrt(var(t_k)) (cx, cv).
template <typename Real>
__device__ __forceinline__ void fb_surrogate_sample(const FbArgs<Real>& a, uint32_t m, Real& cx,
                                                    Real& cv) {
    uint32_t w[4];
    philox4x32_10<true>(m, kFbSurrWord, a.iter, 1u, a.key0, a.key1, w);
    const Real R = bm_radius(w[0], (Real)0);
    const Real ub = unit_uniform<Real>(w[1]);
    cx = bm_cos(R, ub);
    cv = bm_sin(R, ub);
}
template <typename Real>
__device__ __forceinline__ void fb_surrogate(const FbArgs<Real>& a, const Real* __restrict__ zd,
                                             int k, Real cx, Real cv, Real& x, Real& v) {
    x = fma(a.sd[2 * k], cx, zd[2 * k]);
    v = fma(a.sd[2 * k + 1], cv, zd[2 * k + 1]);
}

template <typename Real>
__device__ __forceinline__ void fb_dump(const FbArgs<Real>& a, Real* dst, int k, int64_t m, Real x,
                                        Real v) {
    const int64_t p = m - a.dm0;
    if (dst != nullptr && p >= 0 && p < a.dcount) {
        dst[(size_t)(k * 2) * a.dcount + p] = x;
        dst[(size_t)(k * 2 + 1) * a.dcount + p] = v;
    }
}

// Running cost and its gradient: the tracking cost -exp(-|z - zd|^2/(2 sigJ^2))
// or the ellipse cost -exp(-q^2/(2 sigJ^2)), q = x^2/ax^2 + v^2/av^2 - 1.
template <typename Real>
__device__ __forceinline__ Real track(const FbArgs<Real>& a, Real x, Real v, const Real* zd) {
    if (a.cost_kind == 1) {
        const Real q = fma(x * x, a.iax2, fma(v * v, a.iav2, (Real)-1));
        return -fb_exp<Real>(-(q * q) * a.inv2s2);
    }
    const Real rx = x - zd[0], rv = v - zd[1];
    return -fb_exp<Real>(-fma(rx, rx, rv * rv) * a.inv2s2);
}
template <typename Real>
__device__ __forceinline__ void track_grad(const FbArgs<Real>& a, Real x, Real v, const Real* zd,
                                           Real& gx, Real& gv) {
    if (a.cost_kind == 1) {
        const Real q = fma(x * x, a.iax2, fma(v * v, a.iav2, (Real)-1));
        const Real e = (Real)2 * q * a.invs2 * fb_exp<Real>(-(q * q) * a.inv2s2);
        gx = e * x * a.iax2;
        gv = e * v * a.iav2;
        return;
    }
    const Real rx = x - zd[0], rv = v - zd[1];
    const Real e = fb_exp<Real>(-fma(rx, rx, rv * rv) * a.inv2s2) * a.invs2;
    gx = rx * e;
    gv = rv * e;
}

// Slot q = g TPB + threadIdx.x of a workgroup of TPB threads holding G
// particles per lane (G TPB slots): its particle p, whether it holds one, and
// the workgroup slots of its ring neighbours.  np = 1: particle
// blockIdx.x TPB G + q.  np > 1: ring blockIdx.x sb + q / np, position
// q mod np; slots past the sb rings, and rings past the last, hold none (p = M
// then lies outside every dump range).
struct FbSlot {
    uint32_t p;
    bool act;
    int lft, rgt;
};
template <int G, typename Real, int TPB = kThreads>
__device__ __forceinline__ FbSlot fb_slot(const FbArgs<Real>& a, int g) {
    FbSlot s;
    const int q = g * TPB + (int)threadIdx.x;
    s.lft = s.rgt = q;
    if (a.np == 1) {
        const int64_t m = (int64_t)blockIdx.x * (G * TPB) + q;
        s.act = m < a.M;
        s.p = (uint32_t)m;
        return s;
    }
    const int si = q / a.np, j = q - si * a.np;
    const int64_t r = (int64_t)blockIdx.x * a.sb + si;
    s.act = si < a.sb && r < a.nsys;
    s.p = s.act ? (uint32_t)(r * a.np + j) : (uint32_t)a.M;
    if (s.act) {
        s.lft = si * a.np + (j == 0 ? a.np - 1 : j - 1);
        s.rgt = si * a.np + (j + 1 == a.np ? 0 : j + 1);
    }
    return s;
}

// Trajectory: block b owns (N+1) slots x 2 rows x 256 elements.
template <typename Real>
__device__ __forceinline__ Real* fb_row(void* traj, int N, int64_t blk) {
    return (Real*)traj + (size_t)blk * (N + 1) * 2 * kThreads + threadIdx.x;
}
// The trajectory row of workgroup slot g TPB + threadIdx.x (G particles per
// lane): slots map onto consecutive 256-wide trajectory blocks, the same
// layout whatever the workgroup size; blocks past the last (empty slots of the
// last workgroup) read the last one.
template <typename Real, int G, int TPB>
__device__ __forceinline__ Real* fb_slot_row(const void* traj, int N, int64_t nblk, int g) {
    const int q = g * TPB + (int)threadIdx.x;
    int64_t blk = (int64_t)blockIdx.x * (G * TPB / kThreads) + q / kThreads;
    blk = blk < nblk ? blk : nblk - 1;
    return (Real*)const_cast<void*>(traj) + (size_t)blk * (N + 1) * 2 * kThreads + (q % kThreads);
}
// The fixed grid's jump counts follow the states of all nblk trajectory
// blocks: one byte per particle and step, step k of block b's lane l at byte
// (b N + k) 256 + l.  The adjoint reads them instead of regenerating the
// draws.  Same slot mapping as fb_slot_row.
template <typename Real, int G, int TPB>
__device__ __forceinline__ uint8_t* fb_slot_counts(const void* traj, int N, int64_t nblk, int g) {
    const int q = g * TPB + (int)threadIdx.x;
    int64_t blk = (int64_t)blockIdx.x * (G * TPB / kThreads) + q / kThreads;
    blk = blk < nblk ? blk : nblk - 1;
    uint8_t* base = (uint8_t*)((Real*)const_cast<void*>(traj) + (size_t)nblk * (N + 1) * 2 * kThreads);
    return base + (size_t)blk * N * kThreads + (q % kThreads);
}

// ---------------------------------------------------------------------------
template <typename Real>
__global__ void __launch_bounds__(kThreads)
k_fb_table(const double* __restrict__ mu, const double* __restrict__ zd, Real* __restrict__ tab,
           int N, int nx, int nv, int nvp, size_t off_zd, size_t off_ks, FbKs ks, WsHeader* hdr,
           int clear_flag, PoissonTable pt, Gate gate) {
    if (gate_closed(gate))
        return;
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nmu = (int64_t)N * nx * nvp;
    if (idx < nmu) {
        const int64_t k = idx / (nx * nvp);
        const int rem = (int)(idx - k * nx * nvp);
        const int i = rem / nvp, l = rem - i * nvp;
        tab[idx] = l < nv ? (Real)mu[(k * nx + i) * nv + l] : (Real)0;
    }
    if (idx < 2 * (int64_t)(N + 1))
        tab[off_zd + idx] = zd != nullptr ? (Real)zd[idx] : (Real)0;
    if (idx < 64)
        tab[off_ks + idx] = (Real)ks.v[idx];
    if (idx == 0) {
        if (clear_flag)
            hdr->nonfinite = 0;
        hdr->poisson = pt;
    }
}

// Forward sweep.  Without rings (RING = false, G = 1) one particle per lane and
// no synchronisation.  With rings a workgroup of TPB threads carries G
// particles per lane (slots g TPB + threadIdx.x) and every step first
// publishes x_k in LDS (double buffered by step parity, one barrier per step)
// for the ring force.
template <typename Real, int NVP, bool STORE, int G, bool RING, int TPB = kThreads>
__global__ void __launch_bounds__(TPB, TPB == 1024 && sizeof(Real) == 4 ? 8 : 1)
k_fb_forward(FbArgs<Real> a, const Real* __restrict__ mu, const Real* __restrict__ zd,
             const Real* __restrict__ ks, void* traj, double* __restrict__ cpart) {
    if (gate_closed(a.gate))
        return;
    __shared__ PoissonTable thr;
    fb_stage_thresholds(a, &thr);
    __shared__ Real ks_lds[64];
    ks = fb_stage_ks(ks, ks_lds);
    static_assert(RING || (G == 1 && TPB == kThreads), "independent particles run one per lane");
    __shared__ double sh[TPB];
    __shared__ Real xs[RING ? 2 : 1][RING ? G * TPB : 1];
    Real x[G], v[G], cx[G], cv[G];
    double acc[G];
    FbSlot sl[G];
    Real* row[G];
    uint8_t* cnt[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        sl[j] = fb_slot<G, Real, TPB>(a, j);
        fb_initial(a, sl[j].p, x[j], v[j]);
        row[j] = STORE ? fb_slot_row<Real, G, TPB>(traj, a.N, a.nblk, j) : nullptr;
        cnt[j] = STORE ? fb_slot_counts<Real, G, TPB>(traj, a.N, a.nblk, j) : nullptr;
        if (STORE) {
            __builtin_nontemporal_store(x[j], row[j]);
            __builtin_nontemporal_store(v[j], row[j] + kThreads);
        }
        fb_dump(a, a.dX, 0, sl[j].p, x[j], v[j]);
        acc[j] = 0.0;
        cx[j] = cv[j] = 0;
    }
    for (int k = 0; k < a.N; ++k) {
        Real cpl[G];
        if (RING) {
            Real* xb = xs[k & 1];
#pragma unroll
            for (int j = 0; j < G; ++j)
                xb[j * TPB + threadIdx.x] = x[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < G; ++j)
                cpl[j] = a.omega * ((Real)2 * x[j] - xb[sl[j].lft] - xb[sl[j].rgt]);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            constexpr int RU = TPB == 1024 ? 1 : 2;
            int n;
            const Real u = fb_step<Real, NVP, NoSink, RU>(a, mu + (size_t)k * a.nx * NVP, ks, sl[j].p,
                                                          k, x[j], v[j], cx[j], cv[j],
                                                          RING ? cpl[j] : (Real)0, NoSink(), &n);
            acc[j] += (double)(a.hadt * u * u);
            acc[j] += (double)(a.dt * track(a, x[j], v[j], zd + 2 * (k + 1)));
            if (STORE) {
                Real* r = row[j] + (size_t)(k + 1) * 2 * kThreads;
                __builtin_nontemporal_store(x[j], r);
                __builtin_nontemporal_store(v[j], r + kThreads);
                __builtin_nontemporal_store((uint8_t)n, cnt[j] + (size_t)k * kThreads);
            }
            fb_dump(a, a.dX, k + 1, sl[j].p, x[j], v[j]);
        }
    }
    double C = 0.0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const double c = sl[j].act ? acc[j] : 0.0;
        if (a.dcost != nullptr) {
            const int64_t p = (int64_t)sl[j].p - a.dm0;
            if (sl[j].act && p >= 0 && p < a.dcount)
                a.dcost[p] = c;
        }
        C += c;
    }
    const double s = block_sum<TPB>(C, sh);
    if (threadIdx.x == 0)
        cpart[blockIdx.x] = s;
}

// Orders LDS accesses of one wavefront (its own writes, read back by other
// lanes of the same wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}


typedef double fb_d4 __attribute__((ext_vector_type(4)));
typedef float fb_f4 __attribute__((ext_vector_type(4)));

constexpr int kFbWaves = kThreads / 64;  // waves per block

// The matrix-core product of the path precision.  FP64 paths use
// v_mfma_f64_16x16x4f64; FP32 paths v_mfma_f32_16x16x4f32 (twice the rate):
// its FP32 products and sums cover one chain of a wave's 64 G particles per
// step (G particles per lane), whose rounding averages out over the
// 2^20-particle sum far below the gradient's 1e-6 bound; the waves and the
// blocks are summed in FP64.  Both take A[i][kk] and B[kk][j] in lane i + 16 kk; row()
// gives the row of D held in register r of lane ln (the column is ln mod 16).
// The layouts were measured on the device with one-hot operands.
template <typename Real>
struct FbMma;
template <>
struct FbMma<double> {
    typedef fb_d4 acc_t;
    static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int ln, int r) { return 4 * r + (ln >> 4); }
};
template <>
struct FbMma<float> {
    typedef fb_f4 acc_t;
    static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int ln, int r) { return 4 * (ln >> 4) + r; }
};

// Row stride (elements) of the transposes: 64 particles plus padding, so that
// a row offset is 4 dwords mod 32 (FP32: 68 floats; FP64: 66 doubles = 132
// dwords) and the 16-byte operand reads of the 16 rows of one pass fall in
// distinct banks.
template <typename Real>
constexpr int fb_xs() { return sizeof(Real) == 4 ? 68 : 66; }

// One wave's share of the per-step gradient sum over particles,
// G_k[i][j] += sum_p b(x_p - x^i) b(v_p - v^j) w_p: the particles' bump values
// go through LDS transposes (row = shape function, column = particle; lane p
// writes column p) into sixteen 16 x 16 x 4 matrix-core products per 64
// particles, accumulated in one chain.  The sum over particles
// may take them in any order: product q takes particles 16 kk + q for K index
// kk, so lane i + 16 kk reads A[i][kk] (row i of phx) and B[kk][i] (row i of
// phv) for q = 0..15 as 16 consecutive elements, in 16-byte loads.  The weight
// goes into the velocity values as they are written.  Rows of A past nx and
// columns of B past the row count VR (read from row 0) hold finite leftovers;
// they only reach entries of the product that no flush reads (i >= nx,
// j >= nv).
// Most products q that FbWave::add_live issues one by one (scalar operand
// reads) before it takes the sixteen of add() (ja2 adjoint: 17.8 ms with add()
// only, 16.9 ms at 4 or 8, 17.8 ms when it never takes add()).
constexpr int kFbLiveMax = 8;

template <typename Real, int VR>
struct FbWave {
    typedef typename FbMma<Real>::acc_t acc_t;
    static constexpr int XS = fb_xs<Real>();
    Real (*phx)[XS];
    Real (*phv)[XS];
    int ln, ii, kb, rv;
    // one chain: dependent products issue back to back on the matrix core,
    // and the tile then needs no sum of chains (four independent chains summed
    // in FP64 per step: f4 FP32 adjoint 9.64 against 9.41 ms, ja2 20.7
    // against 18.7 ms)
    acc_t acc;

    __device__ __forceinline__ void clear() { acc = acc_t{0, 0, 0, 0}; }
    template <typename R>
    __device__ __forceinline__ void put_x(int i, R b) const { phx[i][ln] = b; }
    // The velocity values times the particle's weight w.
    template <typename R, int NVP>
    __device__ __forceinline__ void put_vw(const R* pv, R w) const {
        static_assert(NVP <= VR, "velocity rows hold NVP values");
#pragma unroll
        for (int l = 0; l < NVP; ++l)
            phv[l][ln] = pv[l] * w;
    }
    // Adds the wave's 64 particles as put since the last add.
    __device__ __forceinline__ void add() {
        typedef Real v16 __attribute__((ext_vector_type(16 / sizeof(Real))));
        constexpr int E = 16 / sizeof(Real);  // elements per 16-byte load
        wave_lds_sync();
        const v16* pa = (const v16*)&phx[ii][kb];
        const v16* pb = (const v16*)&phv[rv][kb];
#pragma unroll
        for (int c = 0; c < 16 / E; ++c) {
            const v16 av = pa[c], bv = pb[c];
#pragma unroll
            for (int e = 0; e < E; ++e)
                acc = FbMma<Real>::mfma(av[e], bv[e], acc);
        }
        wave_lds_sync();
    }
    // add() when only the particles set in the wave-uniform mask `live` carry
    // a weight (the others put zero): products q that hold no live particle
    // add exact zeros and are skipped, the rest run in the same order, so the
    // sum is bitwise that of add().  Pays when few particles are live (a
    // jump-adapted sub-step run for the wave's jumping lanes).
    __device__ __forceinline__ void add_live(uint64_t live) {
        uint32_t qm = (uint32_t)(live | live >> 16 | live >> 32 | live >> 48) & 0xFFFFu;
        if (__builtin_popcount(qm) > kFbLiveMax) {
            add();
            return;
        }
        wave_lds_sync();
        while (qm != 0) {
            const int q = __builtin_ctz(qm);
            qm &= qm - 1;
            acc = FbMma<Real>::mfma(phx[ii][kb + q], phv[rv][kb + q], acc);
        }
        wave_lds_sync();
    }
};

// Sink of the surrogate's forward step: the wave's transposes, the velocity
// values weighted by alpha u (scale = alpha, or 0 for an empty slot).
template <typename Real, int VR>
struct FbControlSink {
    const FbWave<Real, VR>& w;
    Real scale;
    template <typename R>
    __device__ __forceinline__ void put_x(int i, R b) const { w.put_x(i, b); }
    template <typename R, int NVP>
    __device__ __forceinline__ void put_v(const R* pv, R u) const {
        w.template put_vw<R, NVP>(pv, scale * u);
    }
};

// Rows of the velocity transpose for a compiled width NVP.
template <int NVP>
constexpr int fb_vrows() { return NVP; }

// The block's LDS for the reduction: per wave (W of them), the two transposes
// (16 position rows, VR velocity rows); between steps they hold the waves'
// FP64 tiles.
template <typename Real, int VR, int W = kFbWaves>
struct FbShared {
    static constexpr int waves = W;
    alignas(16) Real phx[W][kFbMaxGrid][fb_xs<Real>()];
    alignas(16) Real phv[W][VR][fb_xs<Real>()];
};

template <typename Real, int VR, int W>
__device__ __forceinline__ FbWave<Real, VR> fb_wave(FbShared<Real, VR, W>& sh) {
    static_assert(sizeof(Real) * kFbMaxGrid * fb_xs<Real>() >= sizeof(double) * kFbMaxGrid * kFbMaxGrid,
                  "a wave's transpose buffer must hold its 16 x 16 FP64 tile");
    FbWave<Real, VR> w;
    const int wv = threadIdx.x >> 6;
    w.phx = sh.phx[wv];
    w.phv = sh.phv[wv];
    w.ln = threadIdx.x & 63;
    w.ii = w.ln & 15;
    w.kb = 16 * (w.ln >> 4);
    w.rv = w.ii < VR ? w.ii : 0;
    w.clear();
    return w;
}

// The wave's FP64 16 x 16 tiles of its last H steps (t[0] the latest), in the
// D layout of the path precision's matrix-core product.  The waves of a block
// combine their tiles once per H steps: H = 2 for independent particles on
// the fixed grid (kFbAdjHold), 1 for rings (whose neighbour exchange needs the
// flush's barriers every step) and the surrogate's forward, 4 for the
// jump-adapted adjoint (54.9 -> 51.1 ms on ja2).
template <int H>
struct FbHist {
    fb_d4 t[H];
    int cnt;
    __device__ __forceinline__ void push(const fb_d4& x) {
#pragma unroll
        for (int s = H - 1; s > 0; --s)
            t[s] = t[s - 1];
        t[0] = x;
        ++cnt;
    }
};

// The wave's sums, in FP64.
template <typename Real, int VR>
__device__ __forceinline__ fb_d4 fb_tile(const FbWave<Real, VR>& w) {
    fb_d4 t;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        t[r] = (double)w.acc[r];
    return t;
}

// Number of 16 x 16 FP64 tiles a wave's transposes hold: in phx, in phv.
constexpr int kFbTile = kFbMaxGrid * kFbMaxGrid;
template <typename Real>
constexpr int fb_tiles_x() {
    return (int)(sizeof(Real) * kFbMaxGrid * fb_xs<Real>() / (sizeof(double) * kFbTile));
}
template <typename Real, int VR>
constexpr int fb_tiles_v() { return (int)(sizeof(Real) * VR * fb_xs<Real>() / (sizeof(double) * kFbTile)); }

// LDS home of tile s of wave wv during a flush (the wave's transpose buffers,
// free between steps).
template <typename Real, int VR, int W>
__device__ __forceinline__ double* fb_tile_lds(FbShared<Real, VR, W>& sh, int wv, int s) {
    constexpr int TX = fb_tiles_x<Real>();
    return s < TX ? (double*)&sh.phx[wv][0][0] + s * kFbTile
                  : (double*)&sh.phv[wv][0][0] + (s - TX) * kFbTile;
}

struct FbNoMid {
    __device__ __forceinline__ void operator()() const {}
};

// Sums the W waves' held tiles in a fixed order into the block's partials:
// tile s is step k0 + s dir (ADD: added to what the partial holds).  mid runs
// between the flush's two barriers (with every wave's LDS writes before the
// flush visible, and none of the next step's yet).
template <bool ADD, int H, typename Real, int VR, int W, typename Mid = FbNoMid>
__device__ __forceinline__ void fb_hist_flush(FbShared<Real, VR, W>& sh, const FbWave<Real, VR>& w,
                                              FbHist<H>& h, int k0, int dir, int N, int nx, int nv,
                                              double* __restrict__ apart, const Mid& mid = Mid()) {
    static_assert(H <= fb_tiles_x<Real>() + fb_tiles_v<Real, VR>(),
                  "a wave's transposes must hold its H tiles");
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < H; ++s) {
        if (s < h.cnt) {
            double* cb = fb_tile_lds(sh, wv, s);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                cb[FbMma<Real>::row(w.ln, r) * kFbMaxGrid + w.ii] = h.t[s][r];
        }
    }
    __syncthreads();
    const int t = threadIdx.x, i = t >> 4, j = t & 15;
    if (i < nx && j < nv) {
#pragma unroll
        for (int s = 0; s < H; ++s) {
            if (s < h.cnt) {
                double sum = fb_tile_lds(sh, 0, s)[t];
#pragma unroll
                for (int q = 1; q < W; ++q)
                    sum += fb_tile_lds(sh, q, s)[t];
                double* dst = apart + ((size_t)blockIdx.x * N + (k0 + s * dir)) * (nx * nv) + i * nv + j;
                *dst = ADD ? *dst + sum : sum;
            }
        }
    }
    mid();
    __syncthreads();
    h.cnt = 0;
}

// Per-step moments of the block's particles for the fitted surrogate
// variance: with y = z_k - zd_k, the sums of y_x, y_x^2, y_v, y_v^2 (q = 0..3)
// in FP64.  Each lane puts its particles' values into its wave's transpose
// buffer after the flush tile (free until the next step's shape functions);
// after a barrier wave q adds component q over the W waves, lane by lane, and
// over the 64 lanes by a butterfly, in a fixed order, and lane 0 writes
// mom[(k nb + block) 4 + q].
template <typename Real, int VR, int W>
__device__ __forceinline__ double* fb_mom_lds(FbShared<Real, VR, W>& sh, int wv) {
    static_assert(sizeof(Real) * kFbMaxGrid * fb_xs<Real>() >= sizeof(double) * (kFbTile + 4 * 64),
                  "a wave's position transpose must hold its flush tile and its moments");
    return (double*)&sh.phx[wv][0][0] + kFbTile;
}
template <typename Real, int VR, int W, int G>
__device__ __forceinline__ void fb_mom_put(FbShared<Real, VR, W>& sh, const Real (&x)[G],
                                           const Real (&v)[G], const bool (&act)[G],
                                           const Real* __restrict__ zk) {
    const double zx = (double)zk[0], zv = (double)zk[1];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < G; ++j) {
        if (act[j]) {
            const double yx = (double)x[j] - zx, yv = (double)v[j] - zv;
            s[0] += yx;
            s[1] += yx * yx;
            s[2] += yv;
            s[3] += yv * yv;
        }
    }
    double* m = fb_mom_lds(sh, threadIdx.x >> 6);
    const int ln = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        m[q * 64 + ln] = s[q];
}
template <typename Real, int VR, int W>
__device__ __forceinline__ void fb_mom_sum(FbShared<Real, VR, W>& sh, double* __restrict__ mom,
                                           int k) {
    static_assert(W == 4, "one wave per moment");
    const int q = threadIdx.x >> 6, ln = threadIdx.x & 63;
    double s = fb_mom_lds(sh, 0)[q * 64 + ln];
#pragma unroll
    for (int wv = 1; wv < W; ++wv)
        s += fb_mom_lds(sh, wv)[q * 64 + ln];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if (ln == 0)
        mom[((size_t)k * gridDim.x + blockIdx.x) * 4 + q] = s;
}
template <typename Real, int VR, int W>
struct FbMomMid {
    FbShared<Real, VR, W>& sh;
    double* mom;
    int k;
    __device__ __forceinline__ void operator()() const {
        if (mom != nullptr)
            fb_mom_sum(sh, mom, k);
    }
};

// Storage-free forward of the surrogate gradient (Section 6.5): G particles
// per lane step together; each step adds alpha u_k phi(z_k) to the block's
// partial and each particle's cost to the block's cost.
template <typename Real, int NVP, int G>
__global__ void __launch_bounds__(kThreads)
k_fb_forward_grad(FbArgs<Real> a, const Real* __restrict__ mu, const Real* __restrict__ zd,
                  const Real* __restrict__ ks, double* __restrict__ cpart,
                  double* __restrict__ apart) {
    if (gate_closed(a.gate))
        return;
    __shared__ PoissonTable thr;
    fb_stage_thresholds(a, &thr);
    __shared__ Real ks_lds[64];
    ks = fb_stage_ks(ks, ks_lds);
    __shared__ FbShared<Real, fb_vrows<NVP>()> sh;
    __shared__ double red[kThreads];
    auto wave = fb_wave(sh);
    FbHist<1> hist;
    hist.cnt = 0;
    const int N = a.N;
    Real x[G], v[G], cx[G], cv[G];
    double acc[G];
    int64_t m[G];
    bool act[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int64_t g = (int64_t)blockIdx.x * G + j;
        m[j] = g * kThreads + threadIdx.x;
        act[j] = m[j] < a.M && g < a.nblk;
        fb_initial(a, (uint32_t)m[j], x[j], v[j]);
        fb_dump(a, a.dX, 0, m[j], x[j], v[j]);
        acc[j] = 0.0;
        cx[j] = cv[j] = 0;
    }
    typedef FbShared<Real, fb_vrows<NVP>()> Sh;
    if (a.mom != nullptr) {
        fb_mom_put(sh, x, v, act, zd);
        __syncthreads();
        fb_mom_sum(sh, a.mom, 0);
        __syncthreads();
    }
    for (int k = 0; k < N; ++k) {
        const Real* mk = mu + (size_t)k * a.nx * NVP;
        wave.clear();
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const FbControlSink<Real, fb_vrows<NVP>()> sink{wave, act[j] ? a.alpha : (Real)0};
            const Real u = fb_step<Real, NVP>(a, mk, ks, (uint32_t)m[j], k, x[j], v[j], cx[j], cv[j],
                                              (Real)0, sink);
            wave.add();
            acc[j] += (double)(a.hadt * u * u);
            acc[j] += (double)(a.dt * track(a, x[j], v[j], zd + 2 * (k + 1)));
            fb_dump(a, a.dX, k + 1, m[j], x[j], v[j]);
        }
        hist.push(fb_tile(wave));
        if (a.mom != nullptr)
            fb_mom_put(sh, x, v, act, zd + 2 * (k + 1));
        fb_hist_flush<false>(sh, wave, hist, k, -1, N, a.nx, a.nv, apart,
                             FbMomMid<Real, fb_vrows<NVP>(), Sh::waves>{sh, a.mom, k + 1});
    }
    double C = 0.0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const double c = act[j] ? acc[j] : 0.0;
        if (a.dcost != nullptr) {
            const int64_t p = m[j] - a.dm0;
            if (act[j] && p >= 0 && p < a.dcount)
                a.dcost[p] = c;
        }
        C += c;
    }
    const double s = block_sum(C, red);
    if (threadIdx.x == 0)
        cpart[blockIdx.x] = s;
}

// The adjoint state of one particle between steps.
template <typename Real>
struct FbAdj {
    Real x, v;    // z_k (current step)
    Real xn, vn;  // z_{k-1}, loaded one step ahead (stored trajectory)
    int nn;       // jump count of step k, loaded one step ahead (stored)
    Real sx, sv;  // the particle's surrogate sample (surrogate gradient)
    Real lx, lv;  // lam_{k+1} on entry to step k
};

// Backward sweep.  Each lane of a workgroup of TPB threads carries G particles
// (slots j TPB + threadIdx.x, j < G) through the steps together; at step k
// each particle in turn adds its shape functions times its weight to the
// wave's matrix-core sums, and the waves' sums form one FP64 partial per
// workgroup and step.
//   SURR = false: the states are the stored trajectory and the weight is
//                 alpha u + gamma^n lam^v (the exact gradient);
//   SURR = true:  the states are the surrogate states of Section 6.5 and the
//                 weight gamma^n lam^v is added to the partials of
//                 k_fb_forward_grad (which hold alpha u phi(z)).
//   RING = true:  rings (slots as in k_fb_forward); each particle's
//                 w = gamma^n lam^v_{k+1} goes to LDS (double buffered by step
//                 parity) and, after the block barriers of the step's
//                 gradient flush, its neighbours add dt omega w to their lam^x_k.
// Steps whose tiles a wave holds before the block flush (independent
// particles), and the FP32 kernels held to five waves per SIMD (the matrix-core
// accumulators then stay in vector registers).  On 2^20 x 500: FP32 10.8 ->
// 10.7 ms, surrogate gradient 22.0 -> 21.0 ms, FP64 29.3 -> 28.9 ms; two held
// steps without the five-wave bound fell to four waves (11.6 ms).
constexpr int kFbAdjHold = 2;
template <typename Real, int NVP, bool RING>
constexpr int fb_adj_waves() {
    constexpr int lds = (int)sizeof(FbShared<Real, fb_vrows<NVP>()>);
    return !RING && sizeof(Real) == 4 ? (160 * 1024 / lds < 5 ? 160 * 1024 / lds : 5) : 1;
}

template <typename Real, int NVP, int G, bool SURR, bool RING, int TPB = kThreads>
__global__ void __launch_bounds__(TPB, (fb_adj_waves<Real, NVP, RING>()))
k_fb_adjoint(FbArgs<Real> a, const Real* __restrict__ mu, const Real* __restrict__ zd,
             const Real* __restrict__ ks, const void* traj, double* __restrict__ apart) {
    if (gate_closed(a.gate))
        return;
    __shared__ PoissonTable thr;
    if constexpr (SURR)
        fb_stage_thresholds(a, &thr);
    __shared__ Real ks_lds[64];
    ks = fb_stage_ks(ks, ks_lds);
    static_assert(!(SURR && RING), "the surrogate gradient takes independent particles");
    static_assert(RING || TPB == kThreads, "independent particles run in blocks of 256");
    __shared__ FbShared<Real, fb_vrows<NVP>(), TPB / 64> sh;
    __shared__ Real cw[RING ? 2 : 1][RING ? G * TPB : 1];
    auto wave = fb_wave(sh);
    // rings flush every step: the flush's barriers order the neighbour exchange
    constexpr int H = RING ? 1 : kFbAdjHold;
    FbHist<H> hist;
    hist.cnt = 0;
    const int N = a.N;
    FbAdj<Real> s[G];
    const Real* row[G];
    const uint8_t* cnt[G];
    bool act[G];
    int64_t m[G];
    FbSlot sl[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        sl[j] = fb_slot<G, Real, TPB>(a, j);
        m[j] = sl[j].p;
        act[j] = sl[j].act;
        if (SURR) {
            row[j] = nullptr;
            cnt[j] = nullptr;
            fb_surrogate_sample(a, (uint32_t)m[j], s[j].sx, s[j].sv);
            fb_surrogate(a, zd, N, s[j].sx, s[j].sv, s[j].x, s[j].v);
        } else {
            row[j] = fb_slot_row<Real, G, TPB>(traj, N, a.nblk, j);
            cnt[j] = fb_slot_counts<Real, G, TPB>(traj, N, a.nblk, j);
            s[j].nn = __builtin_nontemporal_load(cnt[j] + (size_t)(N - 1) * kThreads);
            s[j].x = __builtin_nontemporal_load(row[j] + (size_t)N * 2 * kThreads);
            s[j].v = __builtin_nontemporal_load(row[j] + (size_t)N * 2 * kThreads + kThreads);
            s[j].xn = __builtin_nontemporal_load(row[j] + (size_t)(N - 1) * 2 * kThreads);
            s[j].vn = __builtin_nontemporal_load(row[j] + (size_t)(N - 1) * 2 * kThreads + kThreads);
        }
        Real gx, gv;
        track_grad(a, s[j].x, s[j].v, zd + 2 * N, gx, gv);
        s[j].lx = a.dt * gx;
        s[j].lv = a.dt * gv;
        if (act[j])
            fb_dump(a, a.dlam, N, m[j], s[j].lx, s[j].lv);
    }
    for (int k = N - 1; k >= 0; --k) {
        const Real* mk = mu + (size_t)k * a.nx * NVP;
        wave.clear();
#pragma unroll
        for (int j = 0; j < G; ++j) {
            FbAdj<Real>& st = s[j];
            if (SURR) {
                fb_surrogate(a, zd, k, st.sx, st.sv, st.x, st.v);
            } else {
                st.x = st.xn;
                st.v = st.vn;
                if (k >= 1) {
                    st.xn = __builtin_nontemporal_load(row[j] + (size_t)(k - 1) * 2 * kThreads);
                    st.vn = __builtin_nontemporal_load(row[j] + (size_t)(k - 1) * 2 * kThreads + kThreads);
                }
            }
            Real gn = 1;
            {
                int n;
                if (SURR) {
                    uint32_t w[4];
                    philox4x32_10<true>((uint32_t)m[j], (uint32_t)k, a.iter, 0u, a.key0, a.key1, w);
                    n = poisson_count(poisson_word(w), a.thr0, a.thr);
                } else {
                    n = st.nn;
                    if (k >= 1)
                        st.nn = __builtin_nontemporal_load(cnt[j] + (size_t)(k - 1) * kThreads);
                }
                if (n != 0) {
                    Real svn;
                    ks_factors(ks, n, gn, svn);
                }
            }
            Real pv[NVP], dpv[NVP];
#pragma unroll
            for (int l = 0; l < NVP; ++l)
                pv[l] = bump_dq(fma(-(Real)l, a.eps * a.dvc, a.eps * (st.v - a.vc0)), dpv[l]);
            Real u = 0, ux = 0, uv = 0;
#pragma unroll 2
            for (int i = 0; i < a.nx; ++i) {
                Real dbx;
                const Real bx = bump_dq(fma(-(Real)i, a.eps * a.dxc, a.eps * (st.x - a.xc0)), dbx);
                const Real* rw = mk + i * NVP;
                Real t = 0, sv = 0;
#pragma unroll
                for (int l = 0; l < NVP; ++l) {
                    t = fma(rw[l], pv[l], t);
                    sv = fma(rw[l], dpv[l], sv);
                }
                u = fma(bx, t, u);
                ux = fma(dbx, t, ux);
                uv = fma(bx, sv, uv);
                wave.put_x(i, bx);
            }
            ux *= (Real)-2 * a.eps;  // d carries b'(r) / (-2 eps)
            uv *= (Real)-2 * a.eps;
            const Real wk = SURR ? gn * st.lv : fma(a.alpha, u, gn * st.lv);
            wave.template put_vw<Real, NVP>(pv, act[j] ? wk : (Real)0);
            wave.add();
            if (RING)
                cw[k & 1][j * TPB + threadIdx.x] = gn * st.lv;
            if (k >= 1) {
                Real gx, gv;
                track_grad(a, st.x, st.v, zd + 2 * k, gx, gv);
                const Real au = a.alpha * u;
                // ring: the particle's own share -2 omega of its force
                const Real sx = RING ? ux - a.eta - (Real)2 * a.omega : ux - a.eta;
                const Real nlx = fma(a.dt, fma(au, ux, gx), fma(gn * a.dt * sx, st.lv, st.lx));
                const Real nlv = fma(a.dt, fma(au, uv, gv),
                                     fma(gn, fma(a.dt, uv, (Real)1) * st.lv, a.dt * st.lx));
                st.lx = nlx;
                st.lv = nlv;
                if (!RING && act[j])
                    fb_dump(a, a.dlam, k, m[j], st.lx, st.lv);
            }
        }
        hist.push(fb_tile(wave));
        if (hist.cnt == H || k == 0)
            fb_hist_flush<SURR>(sh, wave, hist, k, 1, N, a.nx, a.nv, apart);
        if (RING && k >= 1) {
            const Real* wb = cw[k & 1];
            const Real dto = a.dt * a.omega;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                s[j].lx = fma(dto, wb[sl[j].lft] + wb[sl[j].rgt], s[j].lx);
                if (act[j])
                    fb_dump(a, a.dlam, k, m[j], s[j].lx, s[j].lv);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Jump-adapted grid (Section 3; Algorithms 5.1-5.2): each particle's grid is
// the uniform points plus its jump times.  Uniform interval k holds the n jumps
// counted by Philox block (m, k, iter, 0), at offsets a_1 < ... < a_n (units of
// dt) that are successive minima of uniforms; sub-step r spans [a_r, a_{r+1}]
// with the normals of block (m, k, iter, r) (block 0 for r = 0) and, for r < n,
// ends with the jump v <- gamma v + S sqrt(1/(2 beta)), S the cosine normal of
// words 2, 3 of block (m, k, iter, r + 1).

// V^(1/c) for V in (0, 1).
__device__ __forceinline__ float fb_root(float V, int c) {
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(V) / (float)c);
}
__device__ __forceinline__ double fb_root(double V, int c) { return pow(V, 1.0 / (double)c); }

// a_{r+1} from a_r: the smallest of the n - r uniforms left on (a_r, 1), with
// V_{r+1} = word r mod 4 of block (m, k, iter, 64 + r / 4).
template <typename Real>
__device__ __forceinline__ Real fb_next_offset(const FbArgs<Real>& a, uint32_t m, int k, int r,
                                               int n, Real ar) {
    uint32_t w[4];
    philox4x32_10<false>(m, (uint32_t)k, a.iter, 64u + (uint32_t)(r >> 2), a.key0, a.key1, w);
    const uint32_t wr = (r & 2) ? ((r & 1) ? w[3] : w[2]) : ((r & 1) ? w[1] : w[0]);
    return fma((Real)1 - ar, (Real)1 - fb_root(unit_uniform<Real>(wr), n - r), ar);
}

// One Euler sub-step of length d (noise scales sq1 = b1 sqrt(d), sq2 =
// b2 sqrt(d)) with control u and normals (zx, zv); FP32 compensated as fb_step.
template <typename Real>
__device__ __forceinline__ void fb_euler(const FbArgs<Real>& a, Real d, Real sq1, Real sq2, Real u,
                                         Real zx, Real zv, Real& x, Real& v, Real& cx, Real& cv) {
    if constexpr (sizeof(Real) == 4) {
        Real ex, ev;
        const Real xn = two_sum(x, fma(d, v, fma(sq1, zx, cx)), ex);
        const Real vn = two_sum(v, fma(d, fma(-a.eta, x, u), fma(sq2, zv, cv)), ev);
        x = xn;
        v = vn;
        cx = ex;
        cv = ev;
    } else {
        const Real xn = fma(sq1, zx, fma(d, v, x));
        const Real vn = fma(sq2, zv, fma(d, fma(-a.eta, x, u), v));
        x = xn;
        v = vn;
    }
}

// The target at fraction f in (0, 1] of interval k (zk = zd + 2k): linear
// between the uniform targets, zd_{k+1} itself at f = 1.
template <typename Real>
__device__ __forceinline__ void fb_target(const Real* __restrict__ zk, Real f, Real* t) {
    if (f == (Real)1) {
        t[0] = zk[2];
        t[1] = zk[3];
    } else {
        t[0] = fma(f, zk[2], ((Real)1 - f) * zk[0]);
        t[1] = fma(f, zk[3], ((Real)1 - f) * zk[1]);
    }
}

// The per-particle stack of post-jump states on the jump-adapted grid: entry
// e holds the state after the particle's e-th jump (the start of the sub-step
// that follows it) and the jump's time in its interval (the offset a, in
// units of dt), kFbJumpCap entries per slot in the trajectory buffer after the
// uniform points, then one int32 count per slot.  A particle with more jumps
// than entries has the rest recomputed by the adjoint.
constexpr int kFbJumpCap = kFbJumpStates;
constexpr int kFbJumpComp = 3;  // x, v, a

// After the counts: one byte per slot and interval, the interval's jump count
// (interval k of block b's lane l at byte (b N + k) 256 + l), so that the
// adjoint need not regenerate it.
template <typename Real>
struct FbJumps {
    Real* st;        // slot's entry 0, x (entry e component c at st[(3 e + c) 256])
    int32_t* count;  // slot's jump count
    uint8_t* per;    // slot's count of interval 0 (interval k at per[k 256])
};

template <typename Real>
__device__ __forceinline__ FbJumps<Real> fb_jumps(void* traj, int N, int64_t nblk) {
    FbJumps<Real> j;
    Real* base = (Real*)traj + (size_t)nblk * (N + 1) * 2 * kThreads;
    j.st = base + (size_t)blockIdx.x * kFbJumpCap * kFbJumpComp * kThreads + threadIdx.x;
    int32_t* counts = (int32_t*)(base + (size_t)nblk * kFbJumpCap * kFbJumpComp * kThreads);
    j.count = counts + (size_t)blockIdx.x * kThreads + threadIdx.x;
    j.per = (uint8_t*)(counts + (size_t)nblk * kThreads) + (size_t)blockIdx.x * N * kThreads +
            threadIdx.x;
    return j;
}

// Sub-steps r0 .. r1 - 1 (at most up to n) of interval k of one particle,
// from the state at the start of sub-step r0 with its offsets (a0, a1) and
// normals (zx, zv); the running cost is added to acc when acc is given, and
// each post-jump state pushed as jump entry *nj when jumps is given.  On
// return the same variables describe the start of sub-step r1 (post-jump).
template <typename Real, int NVP>
__device__ __forceinline__ void fb_advance(const FbArgs<Real>& a, const Real* __restrict__ mk,
                                           const Real* __restrict__ zk, uint32_t m, int k, int n,
                                           int r0, int r1, Real& x, Real& v, Real& cx, Real& cv,
                                           Real& a0, Real& a1, Real& zx, Real& zv, double* acc,
                                           const FbJumps<Real>* jumps = nullptr, int* nj = nullptr) {
    for (int r = r0; r < r1 && r <= n; ++r) {
        const bool whole = n == 0;
        const Real d = whole ? a.dt : (a1 - a0) * a.dt;
        const Real u = fb_control<Real, NVP>(a, mk, x, v);
        if (acc != nullptr)
            *acc += (double)((whole ? a.hadt : (Real)0.5 * a.alpha * d) * u * u);
        fb_euler(a, d, whole ? a.sqb1 : a.b1 * sqrt(d), whole ? a.sqb2 : a.b2 * sqrt(d), u, zx, zv,
                 x, v, cx, cv);
        if (r < n) {
            uint32_t w[4];
            philox4x32_10<false>(m, (uint32_t)k, a.iter, (uint32_t)(r + 1), a.key0, a.key1, w);
            const Real S = bm_cos(bm_radius(w[2], (Real)0), unit_uniform<Real>(w[3]));
            v = fma(S, a.sbeta, a.gamma * v);
            cv = a.gamma * cv;
            const Real R = bm_radius(w[0], (Real)0);
            const Real ub = unit_uniform<Real>(w[1]);
            zx = bm_cos(R, ub);
            zv = bm_sin(R, ub);
            if (jumps != nullptr) {
                if (*nj < kFbJumpCap) {
                    jumps->st[(size_t)(kFbJumpComp * *nj) * kThreads] = x;
                    jumps->st[(size_t)(kFbJumpComp * *nj + 1) * kThreads] = v;
                    jumps->st[(size_t)(kFbJumpComp * *nj + 2) * kThreads] = a1;
                }
                ++*nj;
            }
        }
        if (acc != nullptr) {
            Real tg[2];
            fb_target(zk, a1, tg);
            *acc += (double)(d * track(a, x, v, tg));
        }
        a0 = a1;
        a1 = r + 1 < n ? fb_next_offset(a, m, k, r + 1, n, a1) : (Real)1;
    }
}

// The sub-step-0 normals of interval k (words 0, 1 of its block 0).
template <typename Real>
__device__ __forceinline__ void fb_interval_normals(const FbArgs<Real>& a, uint32_t m, int k,
                                                    Real& zx, Real& zv) {
    uint32_t w[4];
    philox4x32_10<true>(m, (uint32_t)k, a.iter, 0u, a.key0, a.key1, w);
    const Real R = bm_radius(w[0], (Real)0);
    const Real ub = unit_uniform<Real>(w[1]);
    zx = bm_cos(R, ub);
    zv = bm_sin(R, ub);
}

// The count and sub-step-0 normals of interval k, and a_1.
template <typename Real>
__device__ __forceinline__ int fb_interval(const FbArgs<Real>& a, uint32_t m, int k, Real& zx,
                                           Real& zv, Real& a1) {
    uint32_t w[4];
    philox4x32_10<true>(m, (uint32_t)k, a.iter, 0u, a.key0, a.key1, w);
    const int n = poisson_count(poisson_word(w), a.thr0, a.thr);
    const Real R = bm_radius(w[0], (Real)0);
    const Real ub = unit_uniform<Real>(w[1]);
    zx = bm_cos(R, ub);
    zv = bm_sin(R, ub);
    a1 = n > 0 ? fb_next_offset(a, m, k, 0, n, (Real)0) : (Real)1;
    return n;
}

// Forward sweep on the jump-adapted grid, one particle per lane: every
// interval's sub-steps and jumps (lanes without jumps take one step), the
// running cost of each sub-step; the trajectory holds the uniform points.
// FP64 held to three waves per SIMD (two without the bound: ja2 38.5 against
// 36.4 ms).
template <typename Real, int NVP, bool STORE>
__global__ void __launch_bounds__(kThreads, (sizeof(Real) == 8 ? 3 : 1))
k_fb_forward_adapted(FbArgs<Real> a, const Real* __restrict__ mu, const Real* __restrict__ zd,
                     void* traj, double* __restrict__ cpart) {
    if (gate_closed(a.gate))
        return;
    __shared__ PoissonTable thr;
    fb_stage_thresholds(a, &thr);
    __shared__ double sh[kThreads];
    const FbSlot sl = fb_slot<1>(a, 0);
    Real x, v, cx = 0, cv = 0;
    fb_initial(a, sl.p, x, v);
    Real* row = STORE ? fb_row<Real>(traj, a.N, blockIdx.x) : nullptr;
    if (STORE) {
        __builtin_nontemporal_store(x, row);
        __builtin_nontemporal_store(v, row + kThreads);
    }
    fb_dump(a, a.dX, 0, sl.p, x, v);
    FbJumps<Real> jumps;
    int nj = 0;
    if (STORE)
        jumps = fb_jumps<Real>(traj, a.N, a.nblk);
    double acc = 0.0;
    // A lane may run one interval ahead of the wave's slowest lane: each
    // iteration every lane in interval kb (the wave's lowest) or kb + 1 takes
    // its next sub-step, so a lane's extra sub-steps after a jump overlap the
    // other lanes' next interval instead of idling them.  The two intervals'
    // control rows and targets are wave-uniform (scalar loads) and each lane
    // picks its own.
    int k = 0, r = 0;
    Real zx, zv, a0 = 0, a1;
    int n = fb_interval(a, sl.p, 0, zx, zv, a1);
    if (STORE)
        __builtin_nontemporal_store((uint8_t)n, jumps.per);
    for (int kb = 0; kb < a.N;) {
        const Real* mk0 = mu + (size_t)kb * a.nx * NVP;
        const Real* mk1 = kb + 1 < a.N ? mk0 + a.nx * NVP : mk0;
        const Real* zk0 = zd + 2 * kb;
        const Real* zk1 = kb + 1 < a.N ? zk0 + 2 : zk0;
        if (k == kb || (k == kb + 1 && k < a.N)) {
            const bool sel = k != kb;
            const bool whole = n == 0;
            const Real d = whole ? a.dt : (a1 - a0) * a.dt;
            const Real u = fb_control_of<Real, NVP>(a, mk0, mk1, sel, x, v);
            acc += (double)((whole ? a.hadt : (Real)0.5 * a.alpha * d) * u * u);
            fb_euler(a, d, whole ? a.sqb1 : a.b1 * sqrt(d), whole ? a.sqb2 : a.b2 * sqrt(d), u,
                     zx, zv, x, v, cx, cv);
            if (r < n) {
                uint32_t w[4];
                philox4x32_10<false>(sl.p, (uint32_t)k, a.iter, (uint32_t)(r + 1), a.key0, a.key1,
                                     w);
                const Real S = bm_cos(bm_radius(w[2], (Real)0), unit_uniform<Real>(w[3]));
                v = fma(S, a.sbeta, a.gamma * v);
                cv = a.gamma * cv;
                const Real R = bm_radius(w[0], (Real)0);
                const Real ub = unit_uniform<Real>(w[1]);
                zx = bm_cos(R, ub);
                zv = bm_sin(R, ub);
                if (STORE) {
                    if (nj < kFbJumpCap) {
                        jumps.st[(size_t)(kFbJumpComp * nj) * kThreads] = x;
                        jumps.st[(size_t)(kFbJumpComp * nj + 1) * kThreads] = v;
                        jumps.st[(size_t)(kFbJumpComp * nj + 2) * kThreads] = a1;
                    }
                }
                ++nj;
            }
            {
                const Real z[4] = {sel ? zk1[0] : zk0[0], sel ? zk1[1] : zk0[1],
                                   sel ? zk1[2] : zk0[2], sel ? zk1[3] : zk0[3]};
                Real tg[2];
                fb_target(z, a1, tg);
                acc += (double)(d * track(a, x, v, tg));
            }
            a0 = a1;
            a1 = r + 1 < n ? fb_next_offset(a, sl.p, k, r + 1, n, a1) : (Real)1;
            if (r < n) {
                ++r;
            } else {
                // the interval is done: its end state is z_{k+1}
                if (STORE) {
                    Real* rw = row + (size_t)(k + 1) * 2 * kThreads;
                    __builtin_nontemporal_store(x, rw);
                    __builtin_nontemporal_store(v, rw + kThreads);
                }
                fb_dump(a, a.dX, k + 1, sl.p, x, v);
                ++k;
                r = 0;
                if (k < a.N) {
                    a0 = 0;
                    n = fb_interval(a, sl.p, k, zx, zv, a1);
                    if (STORE)
                        __builtin_nontemporal_store((uint8_t)n, jumps.per + (size_t)k * kThreads);
                }
            }
        }
        if (!__builtin_amdgcn_ballot_w64(k == kb))
            ++kb;
    }
    if (STORE)
        *jumps.count = nj;
    const double C = sl.act ? acc : 0.0;
    if (a.dcost != nullptr) {
        const int64_t p = (int64_t)sl.p - a.dm0;
        if (sl.act && p >= 0 && p < a.dcount)
            a.dcost[p] = C;
    }
    const double s = block_sum(C, sh);
    if (threadIdx.x == 0)
        cpart[blockIdx.x] = s;
}

// Stack entry e of the slot (x, v and the jump's offset), if want and the
// stack holds it.
template <typename Real>
__device__ __forceinline__ void fb_stack_entry(const FbJumps<Real>& j, int e, bool want, Real& x,
                                               Real& v, Real& o) {
    if (want && e >= 0 && e < kFbJumpCap) {
        x = j.st[(size_t)(kFbJumpComp * e) * kThreads];
        v = j.st[(size_t)(kFbJumpComp * e + 1) * kThreads];
        o = j.st[(size_t)(kFbJumpComp * e + 2) * kThreads];
    }
}

// Backward sweep on the jump-adapted grid, one particle per lane.  The lane
// carries lam~, the adjoint of the interval's end state without the running
// cost charged there, and the unweighted cost gradient at that state; the
// length of the interval's last sub-step completes it (and the dump).  The
// sub-steps then run backwards in a wave-uniform loop over the wave's largest
// count (each lane takes the start of its sub-step r, and the state after
// the jump that ends it, from its stack of post-jump states, recomputing from
// the interval's start only past the stack's capacity), each adding d_r/dt
// phi(z_r) (alpha u_r + lam^v_-) to the matrix-core sums; lam^v_- carries the
// jump factor gamma.
// Held to four waves per SIMD in FP32 (three without the bound: ja2 19.9
// against 18.3 ms) and two in FP64 (one without: 80.0 against 54.8 ms).
template <typename Real, int NVP>
__global__ void __launch_bounds__(kThreads, (sizeof(Real) == 4 ? 4 : 2))
k_fb_adjoint_adapted(FbArgs<Real> a, const Real* __restrict__ mu, const Real* __restrict__ zd,
                     const void* traj, double* __restrict__ apart) {
    if (gate_closed(a.gate))
        return;
    // four held tiles: FP32 needs all 16 velocity rows for them
    __shared__ FbShared<Real, sizeof(Real) == 4 ? kFbMaxGrid : fb_vrows<NVP>()> sh;
    auto wave = fb_wave(sh);
    FbHist<4> hist;
    hist.cnt = 0;
    const int N = a.N;
    const FbSlot sl = fb_slot<1>(a, 0);
    const Real* row = fb_row<Real>(const_cast<void*>(traj), N, blockIdx.x);
    const FbJumps<Real> jumps = fb_jumps<Real>(const_cast<void*>(traj), N, a.nblk);
    int jend = *jumps.count;  // jumps in the intervals up to the current one
    int nk = __builtin_nontemporal_load(jumps.per + (size_t)(N - 1) * kThreads);
    // The stack entry of each interval's first jump (all an interval with one
    // jump reads) is loaded during the interval before, the jump counts two
    // intervals ahead, so that no sub-step waits on the stack's memory.
    // (FP32 paths; the FP64 kernel has no registers to spare for it)
    constexpr bool PF = sizeof(Real) == 4;
    int nk2 = PF && N >= 2 ? __builtin_nontemporal_load(jumps.per + (size_t)(N - 2) * kThreads) : 0;
    Real pfx = 0, pfv = 0, pfa = 0;
    if (PF)
        fb_stack_entry(jumps, jend - nk, nk > 0, pfx, pfv, pfa);
    const Real xN = __builtin_nontemporal_load(row + (size_t)N * 2 * kThreads);
    const Real vN = __builtin_nontemporal_load(row + (size_t)N * 2 * kThreads + kThreads);
    Real gxe, gve;  // unweighted running-cost gradient at the interval's end state
    track_grad(a, xN, vN, zd + 2 * N, gxe, gve);
    Real lx = 0, lv = 0;
    Real xk = __builtin_nontemporal_load(row + (size_t)(N - 1) * 2 * kThreads);
    Real vk = __builtin_nontemporal_load(row + (size_t)(N - 1) * 2 * kThreads + kThreads);
    for (int k = N - 1; k >= 0; --k) {
        const Real* mk = mu + (size_t)k * a.nx * NVP;
        const Real* zk = zd + 2 * k;
        Real xp = 0, vp = 0;
        if (k >= 1) {
            xp = __builtin_nontemporal_load(row + (size_t)(k - 1) * 2 * kThreads);
            vp = __builtin_nontemporal_load(row + (size_t)(k - 1) * 2 * kThreads + kThreads);
        }
        // the count the forward stored
        const int n = nk;
        if (PF) {
            nk = nk2;
            if (k >= 2)
                nk2 = __builtin_nontemporal_load(jumps.per + (size_t)(k - 2) * kThreads);
        } else if (k >= 1) {
            nk = __builtin_nontemporal_load(jumps.per + (size_t)(k - 1) * kThreads);
        }
        const int jb = jend - n;  // stack entry of this interval's first jump
        // entry jb (valid when n > 0 and jb < kFbJumpCap); then the next
        // interval's first entry
        const Real e0x = pfx, e0v = pfv, e0a = pfa;
        if (PF && k >= 1)
            fb_stack_entry(jumps, jb - nk, nk > 0, pfx, pfv, pfa);
        // the jump times a_q (q = 1..n) from the stack when it holds them all,
        // else regenerated
        const bool stk = n > 0 && jb + n - 1 < kFbJumpCap;
        const Real a1_0 = n == 0 ? (Real)1
                          : stk  ? (PF ? e0a : jumps.st[(size_t)(kFbJumpComp * jb + 2) * kThreads])
                                 : fb_next_offset(a, sl.p, k, 0, n, (Real)0);
        // the last sub-step starts at a_n
        Real an = 0;
        if (n > 0) {
            if (stk) {
                an = PF && n == 1 ? e0a
                                  : jumps.st[(size_t)(kFbJumpComp * (jb + n - 1) + 2) * kThreads];
            } else {
                an = a1_0;
                for (int r = 1; r < n; ++r)
                    an = fb_next_offset(a, sl.p, k, r, n, an);
            }
        }
        const Real dlast = n == 0 ? a.dt : ((Real)1 - an) * a.dt;
        lx = fma(dlast, gxe, lx);
        lv = fma(dlast, gve, lv);
        if (sl.act)
            fb_dump(a, a.dlam, k + 1, sl.p, lx, lv);
        int nmax = n;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1)
            nmax = max(nmax, __shfl_xor(nmax, o));
        wave.clear();
        for (int r = nmax; r >= 0; --r) {
            const bool mine = r <= n;
            Real x = xk, v = vk, a0 = 0, a1 = a1_0;
            if (mine && r > 0) {
                if (stk) {
                    a0 = PF && r == 1 ? e0a
                                      : jumps.st[(size_t)(kFbJumpComp * (jb + r - 1) + 2) * kThreads];
                    a1 = r < n ? jumps.st[(size_t)(kFbJumpComp * (jb + r) + 2) * kThreads] : (Real)1;
                } else {
                    for (int q = 1; q <= r; ++q) {
                        a0 = a1;
                        a1 = q < n ? fb_next_offset(a, sl.p, k, q, n, a1) : (Real)1;
                    }
                }
                if (PF && r == 1 && jb < kFbJumpCap) {
                    x = e0x;
                    v = e0v;
                } else if (jb + r - 1 < kFbJumpCap) {
                    x = jumps.st[(size_t)(kFbJumpComp * (jb + r - 1)) * kThreads];
                    v = jumps.st[(size_t)(kFbJumpComp * (jb + r - 1) + 1) * kThreads];
                } else {
                    Real cx = 0, cv = 0, b0 = 0, b1 = a1_0, zx, zv;
                    fb_interval_normals(a, sl.p, k, zx, zv);
                    fb_advance<Real, NVP>(a, mk, zk, sl.p, k, n, 0, r, x, v, cx, cv, b0, b1, zx,
                                          zv, nullptr);
                }
            }
            const Real d = n == 0 ? a.dt : (a1 - a0) * a.dt;
            if (mine && r < n) {
                // the running cost at the jump ending sub-step r, charged to lam~_{r+1}
                Real xe, ve;
                if (PF && r == 0 && jb < kFbJumpCap) {
                    xe = e0x;
                    ve = e0v;
                } else if (jb + r < kFbJumpCap) {
                    xe = jumps.st[(size_t)(kFbJumpComp * (jb + r)) * kThreads];
                    ve = jumps.st[(size_t)(kFbJumpComp * (jb + r) + 1) * kThreads];
                } else {
                    Real cx = 0, cv = 0, b0 = 0, b1 = a1_0, zx, zv;
                    fb_interval_normals(a, sl.p, k, zx, zv);
                    xe = xk;
                    ve = vk;
                    fb_advance<Real, NVP>(a, mk, zk, sl.p, k, n, 0, r + 1, xe, ve, cx, cv, b0, b1,
                                          zx, zv, nullptr);
                }
                Real tg[2], gx, gv;
                fb_target(zk, a1, tg);
                track_grad(a, xe, ve, tg, gx, gv);
                lx = fma(d, gx, lx);
                lv = fma(d, gv, lv);
            }
            const Real lxm = lx, lvm = r < n ? a.gamma * lv : lv;
            Real pv[NVP], dpv[NVP];
#pragma unroll
            for (int l = 0; l < NVP; ++l)
                pv[l] = bump_dq(fma(-(Real)l, a.eps * a.dvc, a.eps * (v - a.vc0)), dpv[l]);
            Real u = 0, ux = 0, uv = 0;
#pragma unroll 2
            for (int i = 0; i < a.nx; ++i) {
                Real dbx;
                const Real bx = bump_dq(fma(-(Real)i, a.eps * a.dxc, a.eps * (x - a.xc0)), dbx);
                const Real* rw = mk + i * NVP;
                Real t = 0, sv = 0;
#pragma unroll
                for (int l = 0; l < NVP; ++l) {
                    t = fma(rw[l], pv[l], t);
                    sv = fma(rw[l], dpv[l], sv);
                }
                u = fma(bx, t, u);
                ux = fma(dbx, t, ux);
                uv = fma(bx, sv, uv);
                wave.put_x(i, bx);
            }
            ux *= (Real)-2 * a.eps;  // d carries b'(r) / (-2 eps)
            uv *= (Real)-2 * a.eps;
            // the sub-step's share d / dt of the step is a1 - a0
            const Real wk = n == 0 ? fma(a.alpha, u, lvm) : (a1 - a0) * fma(a.alpha, u, lvm);
            wave.template put_vw<Real, NVP>(pv, mine && sl.act ? wk : (Real)0);
            wave.add_live(__builtin_amdgcn_ballot_w64(mine && sl.act));
            if (mine) {
                const Real au = a.alpha * u;
                lx = fma(d, fma(au, ux, (ux - a.eta) * lvm), lxm);
                lv = fma(d, fma(au, uv, fma(uv, lvm, lxm)), lvm);
            }
        }
        jend = jb;
        track_grad(a, xk, vk, zk, gxe, gve);
        hist.push(fb_tile(wave));
        if (hist.cnt == 4 || k == 0)
            fb_hist_flush<false>(sh, wave, hist, k, 1, N, a.nx, a.nv, apart);
        xk = xp;
        vk = vp;
    }
}

// Gradient entries q = (k, e): the sum over the per-block partials in a fixed
// order.  A workgroup takes 32 consecutive entries (a block's 256 contiguous
// bytes of them per load); its thread (e, c) sums the partials b = c, c + 8,
// ... of entry e in order, and a fixed LDS tree adds the 8 chunk sums (one
// serial chain of 2048 loads per entry was latency-bound; 8 entries per
// workgroup read 64-byte pieces: f4 step 13.92 against 13.77 ms).
constexpr int kFbFinEntries = 32;
constexpr int kFbFinChunks = kThreads / kFbFinEntries;

__global__ void __launch_bounds__(kThreads)
k_fb_finalize_grad(const double* __restrict__ apart, int nblk, int64_t NL, int64_t M,
                   double* __restrict__ g, WsHeader* hdr, Gate gate) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    const int e = threadIdx.x % kFbFinEntries, c = threadIdx.x / kFbFinEntries;
    const int64_t q = (int64_t)blockIdx.x * kFbFinEntries + e;
    double s = 0.0;
    if (q < NL)
        for (int b = c; b < nblk; b += kFbFinChunks)
            s += apart[(size_t)b * NL + q];
    sh[threadIdx.x] = s;
    __syncthreads();
#pragma unroll
    for (int w = kFbFinChunks / 2; w >= 1; w >>= 1) {
        if (c < w)
            sh[threadIdx.x] += sh[threadIdx.x + kFbFinEntries * w];
        __syncthreads();
    }
    if (c == 0 && q < NL) {
        const double gq = sh[e] / (double)M;
        g[q] = gq;
        if (!isfinite(gq))
            hdr->nonfinite = 1;
    }
}

// One block: J = (1/M) sum of the block costs and, with g, dt sum g^2.
__global__ void __launch_bounds__(kThreads)
k_fb_finalize_cost(const double* __restrict__ cpart, int nblk, int64_t M, double dt,
                   const double* __restrict__ g, int64_t NL, double* __restrict__ J_out,
                   WsHeader* hdr, int slot, Gate gate) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
        s += cpart[b];
    const double csum = block_sum(s, sh);
    double gg = 0.0;
    if (g != nullptr) {
        for (int64_t q = threadIdx.x; q < NL; q += kThreads)
            gg += g[q] * g[q];
        gg = block_sum(gg, sh);
    }
    if (threadIdx.x == 0) {
        const double J = csum / (double)M;
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
        if (slot == 0 && (!isfinite(J) || !isfinite(gg)))
            hdr->nonfinite = 1;
    }
}

template <typename Real>
__global__ void __launch_bounds__(kThreads)
k_fb_draws(FbArgs<Real> a, PoissonTable pt, int64_t m0, int64_t mc, int k0, int kc,
           Real* __restrict__ zi, Real* __restrict__ Z, int32_t* __restrict__ counts) {
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
    const uint32_t m = (uint32_t)(m0 + p);
    if (q == 0 && zi != nullptr) {
        Real x, v;
        fb_initial(a, m, x, v);
        zi[2 * p] = x;
        zi[2 * p + 1] = v;
    }
    uint32_t w[4];
    philox4x32_10<false>(m, (uint32_t)(k0 + q), a.iter, 0u, a.key0, a.key1, w);
    const Real R = bm_radius(w[0], (Real)0);
    const Real ub = unit_uniform<Real>(w[1]);
    if (Z != nullptr) {
        Z[3 * idx] = bm_cos(R, ub);
        Z[3 * idx + 1] = bm_sin(R, ub);
        Z[3 * idx + 2] = bm_cos(bm_radius(w[2], (Real)0), unit_uniform<Real>(w[3]));
    }
    if (counts != nullptr)
        counts[idx] = poisson_count(poisson_word(w), a.thr0, a.thr);
}

// Per-step variance of the surrogate gradient's forward ensemble (block k =
// step k): each thread adds the moment partials of blocks t, t + 256, ... in
// block order, a fixed tree sums the threads, and with y = z_k - zd_k
// V_c = max(0, sum y_c^2 / M - (sum y_c / M)^2) goes to var[2 k + c].
__global__ void __launch_bounds__(kThreads)
k_fb_step_var(const double* __restrict__ mom, int nb, int64_t M, double* __restrict__ var, Gate gate) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    const int k = blockIdx.x;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kThreads) {
        const double* pm = mom + ((size_t)k * nb + b) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            s[q] += pm[q];
    }
    double tot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        tot[q] = block_sum(s[q], sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double mean = tot[2 * c] / (double)M;
            const double v = tot[2 * c + 1] / (double)M - mean * mean;
            var[2 * k + c] = v > 0.0 ? v : 0.0;
        }
    }
}

// The surrogate variance line per component (Section 6.5: a variance growing
// linearly in time): given (a = svar0, b = svar1), or (fit) the ordinary
// least-squares line through (t_k, V_k), k = 0..N, from svar[0 .. 2N+1]:
// b = sum (t_k - tbar)(V_k - Vbar) / sum (t_k - tbar)^2, a = Vbar - b tbar,
// every sum a fixed tree.  Writes the line to svar[2N+2 ..] (a_x, a_v, b_x,
// b_v) and sd[2k + c] = sqrt(max(0, a_c + b_c t_k)) in the path precision.
template <typename Real>
__global__ void __launch_bounds__(kThreads)
k_fb_surr_sd(double* __restrict__ svar, int N, double dt, int fit, double a0x, double a0v,
             double b0x, double b0v, Real* __restrict__ sd, Gate gate) {
    if (gate_closed(gate))
        return;
    __shared__ double sh[kThreads];
    double a[2] = {a0x, a0v}, b[2] = {b0x, b0v};
    if (fit) {
        const double n1 = (double)(N + 1);
        double st = 0.0, sv[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k <= N; k += kThreads) {
            st += (double)k * dt;
            sv[0] += svar[2 * k];
            sv[1] += svar[2 * k + 1];
        }
        const double tbar = block_sum(st, sh) / n1;
        double vbar[2];
        vbar[0] = block_sum(sv[0], sh) / n1;
        vbar[1] = block_sum(sv[1], sh) / n1;
        double sxx = 0.0, sxy[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k <= N; k += kThreads) {
            const double d = (double)k * dt - tbar;
            sxx += d * d;
            sxy[0] += d * (svar[2 * k] - vbar[0]);
            sxy[1] += d * (svar[2 * k + 1] - vbar[1]);
        }
        sxx = block_sum(sxx, sh);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            b[c] = block_sum(sxy[c], sh) / sxx;
            a[c] = vbar[c] - b[c] * tbar;
        }
    }
    for (int k = threadIdx.x; k <= N; k += kThreads) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double v = a[c] + b[c] * ((double)k * dt);
            sd[2 * k + c] = (Real)sqrt(v > 0.0 ? v : 0.0);
        }
    }
    if (threadIdx.x == 0) {
        svar[2 * (N + 1)] = a[0];
        svar[2 * (N + 1) + 1] = a[1];
        svar[2 * (N + 1) + 2] = b[0];
        svar[2 * (N + 1) + 3] = b[1];
    }
}

// ===========================================================================
// Launchers.

template <typename Real>
static FbArgs<Real> fb_args(const FbHost& p, const HostRun& r) {
    FbArgs<Real> a;
    a.M = r.M;
    a.nsys = p.nsys;
    a.np = p.np;
    a.sb = p.rings_per_block;
    a.cost_kind = p.cost_kind;
    a.omega = (Real)p.omega;
    a.iax2 = (Real)(1.0 / (p.ax * p.ax));
    a.iav2 = (Real)(1.0 / (p.av * p.av));
    a.ax = (Real)p.ax;
    a.av = (Real)p.av;
    a.nblk = r.nblk;
    a.N = p.N;
    a.nx = p.nx;
    a.nv = p.nv;
    a.dt = (Real)p.dt;
    a.sqb1 = (Real)(p.b1 * sqrt(p.dt));
    a.sqb2 = (Real)(p.b2 * sqrt(p.dt));
    a.b1 = (Real)p.b1;
    a.b2 = (Real)p.b2;
    a.gamma = (Real)p.gamma;
    a.sbeta = (Real)(1.0 / sqrt(2.0 * p.beta));
    a.eta = (Real)p.eta;
    a.eps = (Real)p.eps;
    a.alpha = (Real)p.alpha;
    a.hadt = (Real)(0.5 * p.alpha * p.dt);
    a.inv2s2 = (Real)(1.0 / (2.0 * p.sigJ * p.sigJ));
    a.invs2 = (Real)(1.0 / (p.sigJ * p.sigJ));
    const double dx = 2.0 * p.xmax / p.nx, dv = 2.0 * p.vmax / p.nv;
    a.xc0 = (Real)(0.5 * dx - p.xmax);
    a.dxc = (Real)dx;
    a.vc0 = (Real)(0.5 * dv - p.vmax);
    a.dvc = (Real)dv;
    a.z0x = (Real)p.z0[0];
    a.z0v = (Real)p.z0[1];
    a.s0x = (Real)p.s0[0];
    a.s0v = (Real)p.s0[1];
    a.sd = nullptr;
    a.mom = nullptr;
    a.init_kind = p.init_kind;
    a.key0 = (uint32_t)(r.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(r.seed >> 32);
    a.iter = r.iter;
    a.thr = nullptr;
    a.thr0 = 0;
    a.gate = kNoGate;
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

static inline unsigned fb_blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

hipError_t fb_launch_table(const FbHost& p, const HostRun& r, const double* mu, void* tab,
                           WsHeader* hdr, int clear_flag, hipStream_t st, Gate gate) {
    const FbTable t = fb_table_layout(p);
    FbKs ks;
    for (int i = 0; i < 64; ++i)
        ks.v[i] = p.ks[i];
    int64_t n = (int64_t)p.N * p.nx * p.nvp;
    if (n < 2 * (int64_t)(p.N + 1))
        n = 2 * (int64_t)(p.N + 1);
    if (n < 64)
        n = 64;
    if (r.prec == JD_FP64)
        hipLaunchKernelGGL(k_fb_table<double>, dim3(fb_blocks(n)), dim3(kThreads), 0, st, mu, p.zd,
                           (double*)tab, p.N, p.nx, p.nv, p.nvp, t.zd, t.ks, ks, hdr, clear_flag,
                           p.poisson, gate);
    else
        hipLaunchKernelGGL(k_fb_table<float>, dim3(fb_blocks(n)), dim3(kThreads), 0, st, mu, p.zd,
                           (float*)tab, p.N, p.nx, p.nv, p.nvp, t.zd, t.ks, ks, hdr, clear_flag,
                           p.poisson, gate);
    return hipGetLastError();
}

#define FB_DISPATCH_NVP(nvp, FN)           \
    do {                                   \
        switch (nvp) {                     \
        case 4: FN(4); break;              \
        case 8: FN(8); break;              \
        case 10: FN(10); break;            \
        case 12: FN(12); break;            \
        default: FN(16); break;            \
        }                                  \
    } while (0)


// Rings of more than 256 particles take workgroups of 2048 slots (eight
// 256-wide trajectory blocks) and are coupled through LDS every step, so one
// ring's workgroup cannot be split.  With 256 threads (eight particles per
// lane) ring2 (512 rings of 2000, 500 steps) ran at two waves per SIMD: FP32
// forward 7.4 ms, adjoint 15.4 ms, against 5.3 / 11.0 ms for rings of 256 at
// one particle per lane.  The FP32 forward runs 1024 threads (two particles per
// lane, held to 64 registers for eight waves per SIMD: 5.75 ms, 6.2 ms
// without), the FP64 forward 512 (four per lane: 23.6 ms against 25.5 ms at
// 1024, which spills, and 28.1 ms at 256).  The adjoint runs the most threads
// of 1024 / 512 / 256 whose per-wave transposes and neighbour buffer fit the
// 160 KB of LDS of a workgroup (FP32: 1024, 12.1 ms; FP64: 512, 30.3 ms against
// 41.7 ms at 256; 256 for 16-wide FP64 rows).
constexpr int kFbRingSlots = 8 * kThreads;
template <typename Real>
constexpr int fb_ring_fwd_threads() { return sizeof(Real) == 4 ? 1024 : 512; }
template <typename Real, int NVP>
constexpr int fb_ring_adj_lds(int tpb) {
    return (int)sizeof(FbShared<Real, fb_vrows<NVP>(), 16>) / 16 * (tpb / 64) + 2 * kFbRingSlots * (int)sizeof(Real);
}
template <typename Real, int NVP>
constexpr int fb_ring_adj_threads() {
    return fb_ring_adj_lds<Real, NVP>(1024) <= 160 * 1024   ? 1024
           : fb_ring_adj_lds<Real, NVP>(512) <= 160 * 1024 ? 512
                                                            : 256;
}


template <typename Real>
static hipError_t fb_forward_t(const FbHost& p, const HostRun& r, const void* tab, void* traj,
                               double* cpart, const WsHeader* hdr, hipStream_t st, Gate gate) {
    const FbTable t = fb_table_layout(p);
    FbArgs<Real> a = fb_args<Real>(p, r);
    a.thr = &hdr->poisson;
    a.gate = gate;
    const Real* tb = (const Real*)tab;
    const unsigned nb = (unsigned)fb_forward_blocks(p, r);
#define FB_FWD_K(NVP, S, GG, RG, TPB)                                                             \
    hipLaunchKernelGGL((k_fb_forward<Real, NVP, S, GG, RG, TPB>), dim3(nb), dim3(TPB), 0, st, a,  \
                       tb + t.mu, tb + t.zd, tb + t.ks, traj, cpart)
#define FB_FWD_S(NVP, S)                                                                          \
    do {                                                                                          \
        if (p.np == 1) FB_FWD_K(NVP, S, 1, false, kThreads);                                      \
        else if (p.G == 1) FB_FWD_K(NVP, S, 1, true, kThreads);                                   \
        else FB_FWD_K(NVP, S, kFbRingSlots / fb_ring_fwd_threads<Real>(), true,                    \
                      fb_ring_fwd_threads<Real>());                                               \
    } while (0)
#define FB_FWD_A(NVP, S)                                                                          \
    hipLaunchKernelGGL((k_fb_forward_adapted<Real, NVP, S>), dim3(nb), dim3(kThreads), 0, st, a,  \
                       tb + t.mu, tb + t.zd, traj, cpart)
#define FB_FWD(NVP)                                                                               \
    do {                                                                                          \
        if (p.grid == 1) {                                                                        \
            if (traj != nullptr) FB_FWD_A(NVP, true);                                             \
            else FB_FWD_A(NVP, false);                                                            \
        } else if (traj != nullptr) FB_FWD_S(NVP, true);                                          \
        else FB_FWD_S(NVP, false);                                                                \
    } while (0)
    FB_DISPATCH_NVP(p.nvp, FB_FWD);
#undef FB_FWD
#undef FB_FWD_A
#undef FB_FWD_S
#undef FB_FWD_K
    return hipGetLastError();
}

hipError_t fb_launch_forward(const FbHost& p, const HostRun& r, const void* tab, void* traj,
                             double* cpart, const WsHeader* hdr, hipStream_t st, Gate gate) {
    return r.prec == JD_FP64 ? fb_forward_t<double>(p, r, tab, traj, cpart, hdr, st, gate)
                             : fb_forward_t<float>(p, r, tab, traj, cpart, hdr, st, gate);
}

template <typename Real>
static hipError_t fb_adjoint_t(const FbHost& p, const HostRun& r, const void* tab, const void* traj,
                               double* apart, const WsHeader* hdr, bool surr, hipStream_t st,
                               Gate gate) {
    const FbTable t = fb_table_layout(p);
    FbArgs<Real> a = fb_args<Real>(p, r);
    a.thr = &hdr->poisson;
    a.gate = gate;
    const Real* tb = (const Real*)tab;
    a.sd = tb + t.sd;
    const int G = fb_adjoint_groups(p, r);
    const unsigned nb = (unsigned)fb_partial_blocks(p, r);
#define FB_ADJ_G(NVP, GG, S, RG)                                                                  \
    hipLaunchKernelGGL((k_fb_adjoint<Real, NVP, GG, S, RG>), dim3(nb), dim3(kThreads), 0, st, a,  \
                       tb + t.mu, tb + t.zd, tb + t.ks, traj, apart)

#define FB_ADJ(NVP)                                                                               \
    do {                                                                                          \
        if (p.grid == 1) {                                                                        \
            hipLaunchKernelGGL((k_fb_adjoint_adapted<Real, NVP>), dim3(nb), dim3(kThreads), 0,    \
                               st, a, tb + t.mu, tb + t.zd, traj, apart);                         \
        } else if (p.np > 1) {                                                                    \
            if (G == 8) {                                                                         \
                constexpr int RT = fb_ring_adj_threads<Real, NVP>();                              \
                hipLaunchKernelGGL((k_fb_adjoint<Real, NVP, kFbRingSlots / RT, false, true, RT>), \
                                   dim3(nb), dim3(RT), 0, st, a, tb + t.mu, tb + t.zd, tb + t.ks, \
                                   traj, apart);                                                  \
            } else {                                                                              \
                FB_ADJ_G(NVP, 1, false, true);                                                    \
            }                                                                                     \
        } else if (G == 2) {                                                                      \
            if constexpr (sizeof(Real) == 8) {                                                    \
                if (surr) FB_ADJ_G(NVP, 2, true, false);                                          \
                else FB_ADJ_G(NVP, 2, false, false);                                              \
            }                                                                                     \
        } else {                                                                                  \
            if (surr) FB_ADJ_G(NVP, 1, true, false);                                              \
            else FB_ADJ_G(NVP, 1, false, false);                                                  \
        }                                                                                         \
    } while (0)
    FB_DISPATCH_NVP(p.nvp, FB_ADJ);
#undef FB_ADJ
#undef FB_ADJ_G
    return hipGetLastError();
}

hipError_t fb_launch_adjoint(const FbHost& p, const HostRun& r, const void* tab, const void* traj,
                             double* apart, const WsHeader* hdr, bool surrogate, hipStream_t st,
                             Gate gate) {
    return r.prec == JD_FP64
               ? fb_adjoint_t<double>(p, r, tab, traj, apart, hdr, surrogate, st, gate)
               : fb_adjoint_t<float>(p, r, tab, traj, apart, hdr, surrogate, st, gate);
}

template <typename Real>
static hipError_t fb_forward_grad_t(const FbHost& p, const HostRun& r, const void* tab,
                                    double* cpart, double* apart, double* mom, const WsHeader* hdr,
                                    hipStream_t st, Gate gate) {
    const FbTable t = fb_table_layout(p);
    FbArgs<Real> a = fb_args<Real>(p, r);
    a.thr = &hdr->poisson;
    a.gate = gate;
    a.mom = mom;
    const Real* tb = (const Real*)tab;
    const int G = fb_adjoint_groups(p, r);
    const unsigned nb = (unsigned)fb_partial_blocks(p, r);
#define FB_FG(NVP)                                                                                \
    do {                                                                                          \
        if constexpr (sizeof(Real) == 8) {                                                        \
            if (G == 2) {                                                                         \
                hipLaunchKernelGGL((k_fb_forward_grad<Real, NVP, 2>), dim3(nb), dim3(kThreads), 0, \
                                   st, a, tb + t.mu, tb + t.zd, tb + t.ks, cpart, apart);         \
                break;                                                                            \
            }                                                                                     \
        }                                                                                         \
        hipLaunchKernelGGL((k_fb_forward_grad<Real, NVP, 1>), dim3(nb), dim3(kThreads), 0, st, a, \
                           tb + t.mu, tb + t.zd, tb + t.ks, cpart, apart);                        \
    } while (0)
    FB_DISPATCH_NVP(p.nvp, FB_FG);
#undef FB_FG
    return hipGetLastError();
}

hipError_t fb_launch_forward_grad(const FbHost& p, const HostRun& r, const void* tab, double* cpart,
                                  double* apart, double* mom, const WsHeader* hdr, hipStream_t st,
                                  Gate gate) {
    return r.prec == JD_FP64
               ? fb_forward_grad_t<double>(p, r, tab, cpart, apart, mom, hdr, st, gate)
               : fb_forward_grad_t<float>(p, r, tab, cpart, apart, mom, hdr, st, gate);
}

hipError_t fb_launch_surrogate_sd(const FbHost& p, const HostRun& r, const double* mom,
                                  double* svar, void* tab, hipStream_t st, Gate gate) {
    const FbTable t = fb_table_layout(p);
    if (mom != nullptr)
        hipLaunchKernelGGL(k_fb_step_var, dim3((unsigned)(p.N + 1)), dim3(kThreads), 0, st, mom,
                           fb_partial_blocks(p, r), r.M, svar, gate);
    if (r.prec == JD_FP64)
        hipLaunchKernelGGL(k_fb_surr_sd<double>, dim3(1), dim3(kThreads), 0, st, svar, p.N, p.dt,
                           (int)(mom != nullptr), p.svar0[0], p.svar0[1], p.svar1[0], p.svar1[1],
                           (double*)tab + t.sd, gate);
    else
        hipLaunchKernelGGL(k_fb_surr_sd<float>, dim3(1), dim3(kThreads), 0, st, svar, p.N, p.dt,
                           (int)(mom != nullptr), p.svar0[0], p.svar0[1], p.svar1[0], p.svar1[1],
                           (float*)tab + t.sd, gate);
    return hipGetLastError();
}


hipError_t fb_launch_finalize_grad(const FbHost& p, const HostRun& r, const double* apart,
                                   double* g, WsHeader* hdr, hipStream_t st, Gate gate) {
    const int64_t NL = (int64_t)p.N * p.L;
    hipLaunchKernelGGL(k_fb_finalize_grad,
                       dim3((unsigned)((NL + kFbFinEntries - 1) / kFbFinEntries)), dim3(kThreads), 0,
                       st, apart, fb_partial_blocks(p, r), NL, r.M, g, hdr, gate);
    return hipGetLastError();
}

hipError_t fb_launch_finalize_cost(const FbHost& p, const HostRun& r, const double* cpart,
                                   int ncpart, const double* g, double* J_out, WsHeader* hdr,
                                   int slot, hipStream_t st, Gate gate) {
    hipLaunchKernelGGL(k_fb_finalize_cost, dim3(1), dim3(kThreads), 0, st, cpart, ncpart, r.M,
                       p.dt, g, (int64_t)p.N * p.L, J_out, hdr, slot, gate);
    return hipGetLastError();
}

hipError_t fb_launch_draws(const FbHost& p, const HostRun& r, int64_t m0, int64_t mc, int k0,
                           int kc, void* z_init, void* Z, int32_t* counts, hipStream_t st) {
    const unsigned nb = fb_blocks(mc * kc);
    if (r.prec == JD_FP64)
        hipLaunchKernelGGL(k_fb_draws<double>, dim3(nb), dim3(kThreads), 0, st,
                           fb_args<double>(p, r), p.poisson, m0, mc, k0, kc, (double*)z_init,
                           (double*)Z, counts);
    else
        hipLaunchKernelGGL(k_fb_draws<float>, dim3(nb), dim3(kThreads), 0, st,
                           fb_args<float>(p, r), p.poisson, m0, mc, k0, kc, (float*)z_init,
                           (float*)Z, counts);
    return hipGetLastError();
}

}  // namespace jd
