// C-ABI layer of libjd: argument validation, problem preparation (padding,
// Poisson thresholds), workspace layout, the order of kernel launches per entry
// point, and the host loop of the line-search gradient iteration.  No device
// memory is allocated here; every buffer comes from the caller.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "jd_host.hpp"

using namespace jd;
using namespace jd::host;

namespace jd {
namespace host {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int padded_dim(int d) { return d <= 1 ? 1 : d <= 2 ? 2 : d <= 4 ? 4 : 8; }

bool finite_array(const double* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i]))
            return false;
    return true;
}

// Poisson(mu) inverse-CDF thresholds against a 32-bit word, accumulated in
// FP64: p_0 = exp(-mu), p_j = (p_{j-1} mu) / j, F_j = F_{j-1} + p_j,
// thr_j = min(2^32, floor(2^32 F_j)), thr_31 = 2^32.
void poisson_thresholds(double mu, uint64_t* thr) {
    const double two32 = 4294967296.0;
    double p = exp(-mu);
    double F = p;
    for (int j = 0; j < 31; ++j) {
        if (j > 0) {
            p = p * mu / (double)j;
            F = F + p;
        }
        const double t = floor(ldexp(F, 32));
        thr[j] = t >= two32 ? (uint64_t)1 << 32 : (uint64_t)t;
    }
    thr[31] = (uint64_t)1 << 32;
}

PoissonTable poisson_table(const uint64_t* thr) {
    PoissonTable t;
    t.jmax = 31;
    for (int j = 0; j < 32; ++j) {
        t.tm1[j] = (uint32_t)(thr[j] - 1);  // thr_j >= thr_0 >= 1 since rate*dt <= 2
        if (thr[j] == ((uint64_t)1 << 32) && t.jmax == 31)
            t.jmax = j;
    }
    return t;
}

int prepare(const jd_problem* prob, const jd_run* run, HostProblem& p, HostRun& r) {
    if (!prob || !run)
        return JD_EINVAL;
    const int d = prob->d, N = prob->N;
    if (d < 1 || d > 8 || N < 1)
        return JD_EINVAL;
    if (!(prob->T > 0.0) || !isfinite(prob->T) || !(prob->lambda >= 0.0) ||
        !isfinite(prob->lambda) || !isfinite(prob->cubic) || !(prob->nu >= 0.0) ||
        !isfinite(prob->nu))
        return JD_EINVAL;
    const double dt = prob->T / (double)N;
    if (prob->lambda * dt > 2.0)
        return JD_EINVAL;
    if (!prob->x0 || !prob->A || !prob->B || !prob->s || !prob->jump_mean || !prob->jump_std ||
        !prob->xT || !prob->xd)
        return JD_EINVAL;
    if (!finite_array(prob->x0, d) || !finite_array(prob->A, d * d) ||
        !finite_array(prob->B, d * d) || !finite_array(prob->s, d) ||
        !finite_array(prob->jump_mean, d) || !finite_array(prob->jump_std, d) ||
        !finite_array(prob->xT, d))
        return JD_EINVAL;
    if (run->M < 1 || run->M > kMaxPaths)
        return JD_EINVAL;
    if (run->precision != JD_FP32 && run->precision != JD_FP64)
        return JD_EINVAL;
    if (run->mode != JD_STORE && run->mode != JD_RECOMPUTE)
        return JD_EINVAL;
    const int D = padded_dim(d);
    if (run->mode == JD_RECOMPUTE && (run->K < 1 || run->K > N))
        return JD_EINVAL;
    if (run->dump) {
        const jd_dump* dp = run->dump;
        if (dp->m0 < 0 || dp->count < 0 || dp->m0 + dp->count > run->M)
            return JD_EINVAL;
    }
    if (run->noise != JD_NOISE_AUTO && run->noise != JD_NOISE_INLINE &&
        run->noise != JD_NOISE_TABLE)
        return JD_EINVAL;

    memset(&p, 0, sizeof(p));
    p.d = d;
    p.D = D;
    p.N = N;
    p.T = prob->T;
    p.dt = dt;
    p.lambda = prob->lambda;
    p.cubic = prob->cubic;
    p.nu = prob->nu;
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j)
            p.A[i * D + j] = prob->A[i * d + j];
        p.x0[i] = prob->x0[i];
        p.s[i] = prob->s[i];
        p.jm[i] = prob->jump_mean[i];
        p.js[i] = prob->jump_std[i];
        p.xT[i] = prob->xT[i];
    }
    for (int q = 0; q < d * d; ++q)
        p.B[q] = prob->B[q];
    p.xd = prob->xd;
    poisson_thresholds(prob->lambda * dt, p.thr);
    p.poisson = poisson_table(p.thr);

    r.M = run->M;
    r.ldm = (int64_t)round_up((size_t)run->M, kBlock);
    r.seed = run->seed;
    r.iter = run->iter;
    r.prec = run->precision;
    r.mode = run->mode;
    r.K = run->mode == JD_RECOMPUTE ? run->K : 0;
    r.nblk = (int)((run->M + kBlock - 1) / kBlock);
    r.dump = run->dump;
    r.noise = false;
    if (run->noise == JD_NOISE_TABLE)
        r.noise = true;
    else if (run->noise == JD_NOISE_AUTO)
        r.noise = r.nblk <= noise_max_blocks(r.prec) && noise_bytes(p, r) <= kNoiseMaxBytes;
    if (r.mode == JD_RECOMPUTE && !recompute_supported(p, r))
        return JD_EUNSUPPORTED;
    return JD_OK;
}

size_t noise_bytes(const HostProblem& p, const HostRun& r) {
    return (size_t)r.ldm * (size_t)p.N * 2 * (size_t)p.d * real_size(r.prec);
}

Layout layout(const HostProblem& p, const HostRun& r) {
    Layout L;
    size_t off = 0;
    L.hdr = off;
    off += round_up(sizeof(WsHeader), kAlign);
    L.ring = off;
    off += round_up(kLsLogCap * sizeof(LsLog), kAlign);
    L.tab = off;
    off += round_up((size_t)p.N * 2 * p.D * real_size(r.prec), kAlign);
    L.cpart = off;
    off += round_up((size_t)r.nblk * sizeof(double), kAlign);
    L.apart = off;
    off += round_up((size_t)p.N * p.D * r.nblk * sizeof(double), kAlign);
    L.gbuf = off;
    off += round_up((size_t)p.N * p.d * sizeof(double), kAlign);
    L.ut = off;
    off += round_up((size_t)p.N * p.d * sizeof(double), kAlign);
    L.seg = off;
    off += round_up(seg_scratch_bytes(p, r), kAlign);
    L.noise = off;
    off += r.noise ? round_up(noise_bytes(p, r), kAlign) : 0;
    L.total = off + kAlign;  // slack for aligning the caller's pointer
    return L;
}

size_t traj_bytes(const HostProblem& p, const HostRun& r) {
    const size_t rows = r.mode == JD_RECOMPUTE ? (size_t)((p.N + r.K - 1) / r.K) : (size_t)p.N;
    return rows * p.d * (size_t)r.ldm * real_size(r.prec);
}

int bind_ws(const HostProblem& p, const HostRun& r, void* ws, size_t ws_bytes, Ws& w) {
    if (!ws)
        return JD_EINVAL;
    const Layout L = layout(p, r);
    if (ws_bytes < L.total)
        return JD_EWORKSPACE;
    char* base = (char*)round_up((size_t)(uintptr_t)ws, kAlign);
    w.hdr = (WsHeader*)(base + L.hdr);
    w.ring = (LsLog*)(base + L.ring);
    w.tab = base + L.tab;
    w.cpart = (double*)(base + L.cpart);
    w.apart = (double*)(base + L.apart);
    w.gbuf = (double*)(base + L.gbuf);
    w.ut = (double*)(base + L.ut);
    w.seg = base + L.seg;
    w.noise = r.noise ? base + L.noise : nullptr;
    return JD_OK;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

int enqueue_forward(const HostProblem& p, const HostRun& r, const double* u, void* traj, double* J,
                    const Ws& w, hipStream_t st) {
    const int fm = traj == nullptr ? FWD_COST : (r.mode == JD_RECOMPUTE ? FWD_CKPT : FWD_STORE);
    if (w.noise)
        JD_TRY(launch_setup_noise(p, r, u, w.tab, w.noise, w.hdr, 1, st));
    else
        JD_TRY(launch_setup(p, r, u, w.tab, w.hdr, 1, st));
    JD_TRY(launch_forward(p, r, w.tab, traj, fm, w.cpart, w.hdr, st, kNoGate, w.noise));
    JD_TRY(launch_finalize_cost(p, r, w.cpart, u, nullptr, J, w.hdr, 0, st));
    return JD_OK;
}

int enqueue_cost_grad(const HostProblem& p, const HostRun& r, const double* u, double* J,
                      double* g, void* traj, const Ws& w, hipStream_t st, Gate gate,
                      const LsTail* tail) {
    if (w.noise)
        JD_TRY(launch_setup_noise(p, r, u, w.tab, w.noise, w.hdr, 1, st, gate));
    else
        JD_TRY(launch_setup(p, r, u, w.tab, w.hdr, 1, st, gate));
    // One kernel (each block's forward, then its backward sweep) up to d = 4;
    // at d = 8 the separate kernels are faster (FP32 c3: 9.4 against 10.2 ms,
    // c4: 9.8 against 11.6 ms); the results are bitwise the same.
    if (r.mode == JD_STORE && r.dump == nullptr && p.D <= 4) {
        JD_TRY(launch_cost_grad_stored(p, r, w.tab, traj, w.cpart, w.apart, w.hdr, st, gate,
                                       w.noise));
    } else {
        const int fm = r.mode == JD_RECOMPUTE ? FWD_CKPT : FWD_STORE;
        JD_TRY(launch_forward(p, r, w.tab, traj, fm, w.cpart, w.hdr, st, gate, w.noise));
        JD_TRY(launch_adjoint(p, r, w.tab, traj, w.apart, w.seg, w.hdr, st, gate));
    }
    JD_TRY(launch_finalize_grad(p, r, w.apart, u, g, w.hdr, st, gate));
    JD_TRY(launch_finalize_cost(p, r, w.cpart, u, g, J, w.hdr, 0, st, gate, tail));
    return JD_OK;
}

int enqueue_trial(const HostProblem& p, const HostRun& r, const double* u, double zeta,
                  const Ws& w, hipStream_t st, Gate gate, const LsTail* tail) {
    JD_TRY(launch_setup_trial(p, r, u, w.gbuf, zeta, w.ut, w.tab, w.hdr, st, gate));
    JD_TRY(launch_forward(p, r, w.tab, nullptr, FWD_COST, w.cpart, w.hdr, st, gate, w.noise));
    JD_TRY(launch_finalize_cost(p, r, w.cpart, w.ut, nullptr, nullptr, w.hdr, 1, st, gate, tail));
    return JD_OK;
}

// ---------------------------------------------------------------------------
int LsDriver::start(hipStream_t st) {
    JD_TRY(launch_ls_start(hdr, st));
    return JD_OK;
}

int LsDriver::enqueue(LsOps& ops, int iters, hipStream_t st) {
    const int end = opt.n_max - n_next < iters ? opt.n_max : n_next + iters;
    int j0 = j_next;
    for (int n = n_next; n < end; ++n) {
        int rc;
        if (j0 < 0) {
            LsTail tg{};
            tg.mode = kLsTailAfterGrad;
            tg.n = n;
            if ((rc = ops.grad(n, tg, gate_of(hdr, ls_phase(n, -1)), st)))
                return rc;
            if (!ops.fused())
                JD_TRY(launch_ls_after_grad(hdr, n, st));
            j0 = 0;
        }
        // zeta_j = zeta0 rho^j by repeated multiplication, as one trial at a time
        double zeta = opt.zeta0;
        for (int j = 0; j < j0; ++j)
            zeta *= opt.rho;
        const int jend = opt.max_backtracks - j0 < ahead ? opt.max_backtracks : j0 + ahead;
        for (int j = j0; j < jend; ++j) {
            LsArmijo a;
            a.c_armijo = opt.c_armijo;
            a.zeta = zeta;
            a.dt = dt;
            a.tol = opt.tol;
            a.n = n;
            a.j = j;
            a.n_max = opt.n_max;
            a.max_backtracks = opt.max_backtracks;
            a.iter = iter0 + (uint32_t)n;
            LsTail ta{};
            ta.mode = kLsTailArmijo;
            ta.n = n;
            ta.ls = a;
            ta.ring = ring;
            ta.u = u;
            ta.ut = ut;
            ta.nd = nd;
            if ((rc = ops.trial(n, zeta, ta, gate_of(hdr, ls_phase(n, j)), st)))
                return rc;
            if (!ops.fused())
                JD_TRY(launch_armijo(hdr, ring, u, ut, nd, a, st));
            zeta *= opt.rho;
        }
        j0 = -1;
    }
    return JD_OK;
}

bool LsDriver::collect(const void* mirror, jd_iter_log* log) {
    const WsHeader& h = *(const WsHeader*)mirror;
    const LsLog* rl = (const LsLog*)((const char*)mirror + sizeof(WsHeader));
    int most = 0;
    for (int i = copied; i < h.ls_done; ++i) {
        const LsLog& L = rl[i % kLsLogCap];
        if (log) {
            log[i].iter = L.iter;
            log[i].backtracks = L.backtracks;
            log[i].J = L.J;
            log[i].gnorm = sqrt(L.gnorm2);
            log[i].zeta = L.zeta;
            log[i].J_new = L.J_new;
            log[i].E = sqrt(L.E2);
        }
        most = L.backtracks > most ? L.backtracks : most;
    }
    copied = h.ls_done;
    if (h.ls_status != kLsRunning) {
        status = h.ls_status == kLsDone ? JD_OK : h.ls_status;
        return true;
    }
    n_next = (int)(h.ls_phase >> 32);
    j_next = (int)(uint32_t)(h.ls_phase & 0xFFFFFFFF) - 1;
    // enqueue as many trials as the batch's iterations needed (twice as many
    // after an iteration that ran out of them)
    int want = j_next >= 0 ? 2 * ahead : most + 1;
    ahead = want < 1 ? 1 : want > opt.max_backtracks ? opt.max_backtracks : want;
    return false;
}

namespace {

struct JdOps : LsOps {
    const HostProblem& p;
    const HostRun& r;
    const double* u;
    void* traj;
    const Ws& w;
    JdOps(const HostProblem& p_, const HostRun& r_, const double* u_, void* traj_, const Ws& w_)
        : p(p_), r(r_), u(u_), traj(traj_), w(w_) {}
    int grad(int n, const LsTail& tail, Gate gate, hipStream_t st) override {
        HostRun rn = r;
        rn.iter = r.iter + (uint32_t)n;
        return enqueue_cost_grad(p, rn, u, nullptr, w.gbuf, traj, w, st, gate, &tail);
    }
    int trial(int n, double zeta, const LsTail& tail, Gate gate, hipStream_t st) override {
        HostRun rn = r;
        rn.iter = r.iter + (uint32_t)n;
        return enqueue_trial(p, rn, u, zeta, w, st, gate, &tail);
    }
    bool fused() const override { return true; }
};

}  // namespace

int validate_opt(const jd_opt* opt) {
    if (!opt || opt->n_max < 0 || opt->max_backtracks < 1 || !(opt->zeta0 > 0.0) ||
        !(opt->rho > 0.0) || !(opt->rho < 1.0) || !(opt->c_armijo > 0.0) || !(opt->tol >= 0.0))
        return JD_EINVAL;
    return JD_OK;
}

}  // namespace host
}  // namespace jd

extern "C" {

int jd_version(void) { return JD_VERSION; }

const char* jd_strerror(int code) {
    switch (code) {
    case JD_OK: return "ok";
    case JD_EINVAL: return "invalid argument";
    case JD_EWORKSPACE: return "workspace too small";
    case JD_EHIP: return "HIP launch or runtime error";
    case JD_ENONFINITE: return "non-finite cost or gradient";
    case JD_ELINESEARCH: return "no Armijo step within max_backtracks";
    case JD_EUNSUPPORTED: return "unsupported configuration (checkpoint interval too long)";
    case JD_EAGAIN: return "not ready";
    default: return "unknown error";
    }
}

int jd_poisson_thresholds(double mu, uint64_t* thr) {
    if (!thr || !(mu >= 0.0) || mu > 2.0)
        return JD_EINVAL;
    poisson_thresholds(mu, thr);
    return JD_OK;
}

size_t jd_workspace_bytes(const jd_problem* prob, const jd_run* run) {
    HostProblem p;
    HostRun r;
    if (prepare(prob, run, p, r) != JD_OK)
        return 0;
    return layout(p, r).total;
}

size_t jd_traj_bytes(const jd_problem* prob, const jd_run* run) {
    HostProblem p;
    HostRun r;
    if (prepare(prob, run, p, r) != JD_OK)
        return 0;
    return traj_bytes(p, r);
}

int jd_forward(const jd_problem* prob, const jd_run* run, const double* u, void* traj, double* J,
               void* ws, size_t ws_bytes, hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!u || !J || (traj && !aligned(traj, real_size(r.prec))))
        return JD_EINVAL;
    Ws w;
    if ((rc = bind_ws(p, r, ws, ws_bytes, w)))
        return rc;
    return enqueue_forward(p, r, u, traj, J, w, stream);
}

int jd_adjoint(const jd_problem* prob, const jd_run* run, const double* u, const void* traj,
               double* grad, void* ws, size_t ws_bytes, hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!u || !traj || !grad || !aligned(traj, real_size(r.prec)))
        return JD_EINVAL;
    Ws w;
    if ((rc = bind_ws(p, r, ws, ws_bytes, w)))
        return rc;
    JD_TRY(launch_setup(p, r, u, w.tab, w.hdr, 1, stream));
    JD_TRY(launch_adjoint(p, r, w.tab, traj, w.apart, w.seg, w.hdr, stream));
    JD_TRY(launch_finalize_grad(p, r, w.apart, u, grad, w.hdr, stream));
    return JD_OK;
}

int jd_cost_grad(const jd_problem* prob, const jd_run* run, const double* u, double* J,
                 double* grad, void* traj, void* ws, size_t ws_bytes, hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!u || !J || !grad || !traj || !aligned(traj, real_size(r.prec)))
        return JD_EINVAL;
    Ws w;
    if ((rc = bind_ws(p, r, ws, ws_bytes, w)))
        return rc;
    return enqueue_cost_grad(p, r, u, J, grad, traj, w, stream);
}

int jd_optimize(const jd_problem* prob, const jd_run* run, const jd_opt* opt, double* u,
                jd_iter_log* log, int32_t* iters_done, void* traj, void* ws, size_t ws_bytes,
                hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!u || !traj || !aligned(traj, real_size(r.prec)) || validate_opt(opt))
        return JD_EINVAL;
    Ws w;
    if ((rc = bind_ws(p, r, ws, ws_bytes, w)))
        return rc;
    if (iters_done)
        *iters_done = 0;
    if (opt->n_max == 0)
        return JD_OK;
    LsDriver drv;
    drv.opt = *opt;
    drv.hdr = w.hdr;
    drv.ring = w.ring;
    drv.u = u;
    drv.ut = w.ut;
    drv.nd = p.N * p.d;
    drv.dt = p.dt;
    drv.iter0 = r.iter;
    JdOps ops(p, r, u, traj, w);
    alignas(16) char mirror[kLsMirrorBytes];
    if ((rc = drv.start(stream)))
        return rc;
    for (;;) {
        if ((rc = drv.enqueue(ops, kLsLogCap, stream)))
            return rc;
        JD_TRY(hipMemcpyAsync(mirror, w.hdr, kLsMirrorBytes, hipMemcpyDeviceToHost, stream));
        JD_TRY(hipStreamSynchronize(stream));
        const bool end = drv.collect(mirror, log);
        if (iters_done)
            *iters_done = drv.copied;
        if (end)
            break;
    }
    return drv.status;
}

int jd_check_finite(void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!ws || ws_bytes < sizeof(WsHeader) + kAlign)
        return JD_EINVAL;
    WsHeader* hdr = (WsHeader*)round_up((size_t)(uintptr_t)ws, kAlign);
    int32_t flag = 0;
    JD_TRY(hipMemcpyAsync(&flag, &hdr->nonfinite, sizeof(flag), hipMemcpyDeviceToHost, stream));
    JD_TRY(hipStreamSynchronize(stream));
    JD_TRY(launch_clear_flag(hdr, stream));
    return flag ? JD_ENONFINITE : JD_OK;
}

int jd_draws(const jd_problem* prob, const jd_run* run, int64_t m0, int64_t mc, int32_t k0,
             int32_t kc, void* zw, void* zj, int32_t* counts, hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (m0 < 0 || mc < 0 || k0 < 0 || kc < 0 || m0 + mc > ((int64_t)1 << 32) ||
        (int64_t)k0 + kc > ((int64_t)1 << 31) || mc * (int64_t)kc > ((int64_t)1 << 40))
        return JD_EINVAL;
    if (mc == 0 || kc == 0)
        return JD_OK;
    JD_TRY(launch_draws(p, r, m0, mc, k0, kc, zw, zj, counts, stream));
    return JD_OK;
}

int jd_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!ctr || !out)))
        return JD_EINVAL;
    JD_TRY(launch_philox(seed, ctr, n, out, stream));
    return JD_OK;
}

}  // extern "C"
