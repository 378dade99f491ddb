// C-ABI layer of libjd for the paper's model problem (include/jd_feedback.h):
// validation, the host-side problem form (cell-centre grid, Keilson-Storer
// factors, Poisson thresholds), workspace layout, launch order per entry point
// and the host loop of the gradient iteration.  No device memory is
// allocated; every buffer comes from the caller.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/jd_feedback.h"
#include "fb_launch.hpp"
#include "jd_host.hpp"

using namespace jd;
using namespace jd::host;

namespace {

bool finite(double x) { return isfinite(x) != 0; }

int fb_prepare(const jd_fb_problem* prob, const jd_run* run, FbHost& p, HostRun& r) {
    if (!prob || !run)
        return JD_EINVAL;
    const jd_fb_problem& q = *prob;
    if (q.N < 1 || q.nx < 1 || q.nv < 1 || q.nx > kFbMaxGrid || q.nv > kFbMaxGrid)
        return JD_EINVAL;
    if (!(q.T > 0.0) || !finite(q.T) || !(q.beta > 0.0) || !finite(q.beta) || !(q.eps > 0.0) ||
        !finite(q.eps) || !(q.sigJ > 0.0) || !finite(q.sigJ) || !(q.xmax > 0.0) ||
        !finite(q.xmax) || !(q.vmax > 0.0) || !finite(q.vmax))
        return JD_EINVAL;
    if (!finite(q.eta) || !(q.b1 >= 0.0) || !finite(q.b1) || !(q.b2 >= 0.0) || !finite(q.b2) ||
        !(q.alpha >= 0.0) || !finite(q.alpha) || !(q.gamma >= -1.0) || !(q.gamma <= 1.0))
        return JD_EINVAL;
    if (q.init_kind != JD_FB_INIT_GAUSS && q.init_kind != JD_FB_INIT_UNIFORM &&
        q.init_kind != JD_FB_INIT_ELLIPSE)
        return JD_EINVAL;
    if (q.cost_kind != JD_FB_COST_TRACK && q.cost_kind != JD_FB_COST_ELLIPSE)
        return JD_EINVAL;
    if (q.np < 1 || q.np > JD_FB_MAX_RING || !finite(q.omega))
        return JD_EINVAL;
    if (q.grid != JD_FB_GRID_FIXED && q.grid != JD_FB_GRID_ADAPTED)
        return JD_EINVAL;
    if ((q.cost_kind == JD_FB_COST_ELLIPSE || q.init_kind == JD_FB_INIT_ELLIPSE) &&
        !(q.ax > 0.0 && finite(q.ax) && q.av > 0.0 && finite(q.av)))
        return JD_EINVAL;
    if (q.svar_kind != JD_FB_SVAR_GIVEN && q.svar_kind != JD_FB_SVAR_FIT)
        return JD_EINVAL;
    for (int c = 0; c < 2; ++c) {
        if (!finite(q.z0[c]) || !(q.s0[c] >= 0.0) || !finite(q.s0[c]))
            return JD_EINVAL;
        if (q.svar_kind == JD_FB_SVAR_GIVEN &&
            (!(q.svar0[c] >= 0.0) || !finite(q.svar0[c]) || !(q.svar1[c] >= 0.0) ||
             !finite(q.svar1[c])))
            return JD_EINVAL;
    }
    if (!q.zd && (q.cost_kind == JD_FB_COST_TRACK || run->mode == JD_SURROGATE))
        return JD_EINVAL;
    const double dt = q.T / (double)q.N;
    const double rate = sqrt(q.beta / 3.141592653589793238462643383280);
    if (rate * dt > 2.0)
        return JD_EINVAL;
    if (run->M < 1 || run->M > kMaxPaths / q.np)
        return JD_EINVAL;
    const int64_t particles = run->M * (int64_t)q.np;
    if (run->precision != JD_FP32 && run->precision != JD_FP64)
        return JD_EINVAL;
    if (run->mode == JD_RECOMPUTE)
        return JD_EUNSUPPORTED;
    if (run->mode != JD_STORE && run->mode != JD_SURROGATE)
        return JD_EINVAL;
    if (run->mode == JD_SURROGATE && (q.np > 1 || q.grid == JD_FB_GRID_ADAPTED))
        return JD_EUNSUPPORTED;
    if (q.grid == JD_FB_GRID_ADAPTED && q.np > 1)
        return JD_EUNSUPPORTED;
    if (run->dump) {
        const jd_dump* dp = run->dump;
        if (dp->m0 < 0 || dp->count < 0 || dp->m0 + dp->count > particles)
            return JD_EINVAL;
    }
    // the particle sweeps always draw inline; the field is only checked
    if (run->noise != JD_NOISE_AUTO && run->noise != JD_NOISE_INLINE &&
        run->noise != JD_NOISE_TABLE)
        return JD_EINVAL;

    memset(&p, 0, sizeof(p));
    p.N = q.N;
    p.nx = q.nx;
    p.nv = q.nv;
    // control rows padded to a compiled width: 4, 8, 10 (the paper's 10 x 10
    // grid without padding), 12 or 16
    p.nvp = q.nv == 9 || q.nv == 10 ? 10 : (q.nv + 3) / 4 * 4;
    p.L = q.nx * q.nv;
    p.T = q.T;
    p.dt = dt;
    p.eta = q.eta;
    p.b1 = q.b1;
    p.b2 = q.b2;
    p.gamma = q.gamma;
    p.beta = q.beta;
    p.rate = rate;
    p.xmax = q.xmax;
    p.vmax = q.vmax;
    p.eps = q.eps;
    p.alpha = q.alpha;
    p.sigJ = q.sigJ;
    p.init_kind = q.init_kind;
    for (int c = 0; c < 2; ++c) {
        p.z0[c] = q.z0[c];
        p.s0[c] = q.s0[c];
        p.svar0[c] = q.svar0[c];
        p.svar1[c] = q.svar1[c];
    }
    p.svar_fit = q.svar_kind == JD_FB_SVAR_FIT;
    p.zd = q.zd;
    p.np = q.np;
    p.omega = q.omega;
    p.cost_kind = q.cost_kind;
    p.ax = q.ax;
    p.av = q.av;
    p.grid = q.grid;
    p.nsys = run->M;
    p.G = 1;
    p.rings_per_block = 0;
    // n jumps v <- gamma v + N(0, 1/(2 beta)) composed: gamma^n v + N(0, V_n),
    // V_n = (1/(2 beta)) sum_{i<n} gamma^{2i}
    double g = 1.0, s = 0.0;
    for (int n = 0; n < 32; ++n) {
        p.ks[2 * n] = g;
        p.ks[2 * n + 1] = sqrt(s / (2.0 * q.beta));
        s += g * g;
        g *= q.gamma;
    }
    poisson_thresholds(rate * dt, p.thr);
    p.poisson = poisson_table(p.thr);

    r.M = particles;
    r.seed = run->seed;
    r.iter = run->iter;
    r.prec = run->precision;
    r.mode = run->mode;
    r.K = 0;
    r.noise = false;
    r.dump = run->dump;
    if (q.np == 1) {
        r.nblk = (int)((particles + kBlock - 1) / kBlock);
    } else {
        // whole rings per workgroup of G 256-slot groups
        p.G = fb_ring_groups(q.np);
        p.rings_per_block = p.G * (int)kBlock / q.np;
        const int64_t nb = (run->M + p.rings_per_block - 1) / p.rings_per_block;
        r.nblk = (int)(nb * p.G);
    }
    r.ldm = (int64_t)r.nblk * kBlock;
    return JD_OK;
}

struct FbLayout {
    size_t hdr, ring, tab, cpart, apart, gbuf, ut, mom, svar, total;
};

FbLayout fb_layout(const FbHost& p, const HostRun& r) {
    FbLayout L;
    size_t off = 0;
    L.hdr = off;
    off += round_up(sizeof(WsHeader), kAlign);
    L.ring = off;
    off += round_up(kLsLogCap * sizeof(LsLog), kAlign);
    L.tab = off;
    off += round_up(fb_table_layout(p).count * real_size(r.prec), kAlign);
    L.cpart = off;
    off += round_up((size_t)r.nblk * sizeof(double), kAlign);
    L.apart = off;
    off += round_up((size_t)r.nblk * p.N * p.L * sizeof(double), kAlign);
    L.gbuf = off;
    off += round_up((size_t)p.N * p.L * sizeof(double), kAlign);
    L.ut = off;
    off += round_up((size_t)p.N * p.L * sizeof(double), kAlign);
    // surrogate gradient: the forward's per-step moment partials (fitted
    // variance only), the per-step variance and the variance line
    L.mom = off;
    if (r.mode == JD_SURROGATE && p.svar_fit)
        off += round_up(fb_mom_count(p, r) * sizeof(double), kAlign);
    L.svar = off;
    if (r.mode == JD_SURROGATE)
        off += round_up(fb_svar_count(p) * sizeof(double), kAlign);
    L.total = off + kAlign;
    return L;
}

size_t fb_traj_bytes(const FbHost& p, const HostRun& r) {
    size_t b = (size_t)(p.N + 1) * 2 * (size_t)r.ldm * real_size(r.prec);
    if (p.grid == JD_FB_GRID_ADAPTED)  // the post-jump state stacks and their counts
        b += (size_t)kFbJumpStates * 3 * (size_t)r.ldm * real_size(r.prec) + (size_t)r.ldm * 4;
    b += (size_t)p.N * (size_t)r.ldm;  // one jump-count byte per particle and step / interval
    return b;
}

struct FbWs {
    WsHeader* hdr;
    LsLog* ring;  // follows the header (one copy of kLsMirrorBytes reads both)
    void* tab;
    double* cpart;
    double* apart;
    double* gbuf;
    double* ut;
    double* mom;   // surrogate, fitted variance: per-step moment partials
    double* svar;  // surrogate: per-step variance and the variance line
};

int fb_bind(const FbHost& p, const HostRun& r, void* ws, size_t ws_bytes, FbWs& w) {
    if (!ws)
        return JD_EINVAL;
    const FbLayout L = fb_layout(p, r);
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
    w.mom = (double*)(base + L.mom);
    w.svar = (double*)(base + L.svar);
    return JD_OK;
}

int fb_enqueue_cost_grad(const FbHost& p, const HostRun& r, const double* mu, double* J, double* g,
                         void* traj, const FbWs& w, hipStream_t st, Gate gate = kNoGate) {
    JD_TRY(fb_launch_table(p, r, mu, w.tab, w.hdr, 1, st, gate));
    if (r.mode == JD_SURROGATE) {
        double* mom = p.svar_fit ? w.mom : nullptr;
        JD_TRY(fb_launch_forward_grad(p, r, w.tab, w.cpart, w.apart, mom, w.hdr, st, gate));
        JD_TRY(fb_launch_surrogate_sd(p, r, mom, w.svar, w.tab, st, gate));
        JD_TRY(fb_launch_adjoint(p, r, w.tab, nullptr, w.apart, w.hdr, true, st, gate));
        JD_TRY(fb_launch_finalize_grad(p, r, w.apart, g, w.hdr, st, gate));
        JD_TRY(fb_launch_finalize_cost(p, r, w.cpart, fb_partial_blocks(p, r), g, J, w.hdr, 0, st,
                                       gate));
        return JD_OK;
    }
    JD_TRY(fb_launch_forward(p, r, w.tab, traj, w.cpart, w.hdr, st, gate));
    JD_TRY(fb_launch_adjoint(p, r, w.tab, traj, w.apart, w.hdr, false, st, gate));
    JD_TRY(fb_launch_finalize_grad(p, r, w.apart, g, w.hdr, st, gate));
    JD_TRY(fb_launch_finalize_cost(p, r, w.cpart, fb_forward_blocks(p, r), g, J, w.hdr, 0, st,
                                   gate));
    return JD_OK;
}

// Trial point mu - zeta g and its cost into the header's J_trial, under gate.
int fb_enqueue_trial(const FbHost& p, const HostRun& r, const double* mu, double zeta,
                     const FbWs& w, hipStream_t st, Gate gate) {
    const int nl = p.N * p.L;
    JD_TRY(launch_trial(mu, w.gbuf, zeta, w.ut, nl, st, gate));
    JD_TRY(fb_launch_table(p, r, w.ut, w.tab, w.hdr, 0, st, gate));
    JD_TRY(fb_launch_forward(p, r, w.tab, nullptr, w.cpart, w.hdr, st, gate));
    JD_TRY(fb_launch_finalize_cost(p, r, w.cpart, fb_forward_blocks(p, r), nullptr, nullptr, w.hdr,
                                   1, st, gate));
    return JD_OK;
}

struct FbOps : LsOps {
    const FbHost& p;
    const HostRun& r;
    const double* mu;
    void* traj;
    const FbWs& w;
    FbOps(const FbHost& p_, const HostRun& r_, const double* mu_, void* traj_, const FbWs& w_)
        : p(p_), r(r_), mu(mu_), traj(traj_), w(w_) {}
    int grad(int n, const LsTail&, Gate gate, hipStream_t st) override {
        HostRun rn = r;
        rn.iter = r.iter + (uint32_t)n;
        return fb_enqueue_cost_grad(p, rn, mu, nullptr, w.gbuf, traj, w, st, gate);
    }
    int trial(int n, double zeta, const LsTail&, Gate gate, hipStream_t st) override {
        HostRun rn = r;
        rn.iter = r.iter + (uint32_t)n;
        return fb_enqueue_trial(p, rn, mu, zeta, w, st, gate);
    }
};

}  // namespace

extern "C" {

size_t jd_fb_workspace_bytes(const jd_fb_problem* prob, const jd_run* run) {
    FbHost p;
    HostRun r;
    if (fb_prepare(prob, run, p, r) != JD_OK)
        return 0;
    return fb_layout(p, r).total;
}

size_t jd_fb_traj_bytes(const jd_fb_problem* prob, const jd_run* run) {
    FbHost p;
    HostRun r;
    if (fb_prepare(prob, run, p, r) != JD_OK)
        return 0;
    return fb_traj_bytes(p, r);
}

int jd_fb_forward(const jd_fb_problem* prob, const jd_run* run, const double* mu, void* traj,
                  double* J, void* ws, size_t ws_bytes, hipStream_t stream) {
    FbHost p;
    HostRun r;
    int rc = fb_prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!mu || !J || (traj && !aligned(traj, real_size(r.prec))))
        return JD_EINVAL;
    FbWs w;
    if ((rc = fb_bind(p, r, ws, ws_bytes, w)))
        return rc;
    JD_TRY(fb_launch_table(p, r, mu, w.tab, w.hdr, 1, stream));
    JD_TRY(fb_launch_forward(p, r, w.tab, traj, w.cpart, w.hdr, stream));
    JD_TRY(fb_launch_finalize_cost(p, r, w.cpart, fb_forward_blocks(p, r), nullptr, J, w.hdr, 0,
                                   stream));
    return JD_OK;
}

int jd_fb_adjoint(const jd_fb_problem* prob, const jd_run* run, const double* mu, const void* traj,
                  double* grad, void* ws, size_t ws_bytes, hipStream_t stream) {
    FbHost p;
    HostRun r;
    int rc = fb_prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (r.mode == JD_SURROGATE)
        return JD_EUNSUPPORTED;
    if (!mu || !traj || !grad || !aligned(traj, real_size(r.prec)))
        return JD_EINVAL;
    FbWs w;
    if ((rc = fb_bind(p, r, ws, ws_bytes, w)))
        return rc;
    JD_TRY(fb_launch_table(p, r, mu, w.tab, w.hdr, 1, stream));
    JD_TRY(fb_launch_adjoint(p, r, w.tab, traj, w.apart, w.hdr, false, stream));
    JD_TRY(fb_launch_finalize_grad(p, r, w.apart, grad, w.hdr, stream));
    return JD_OK;
}

int jd_fb_cost_grad(const jd_fb_problem* prob, const jd_run* run, const double* mu, double* J,
                    double* grad, void* traj, void* ws, size_t ws_bytes, hipStream_t stream) {
    FbHost p;
    HostRun r;
    int rc = fb_prepare(prob, run, p, r);
    if (rc)
        return rc;
    const bool need_traj = r.mode == JD_STORE;
    if (!mu || !J || !grad || (need_traj && !traj) || (traj && !aligned(traj, real_size(r.prec))))
        return JD_EINVAL;
    FbWs w;
    if ((rc = fb_bind(p, r, ws, ws_bytes, w)))
        return rc;
    return fb_enqueue_cost_grad(p, r, mu, J, grad, traj, w, stream);
}

int jd_fb_optimize(const jd_fb_problem* prob, const jd_run* run, const jd_opt* opt, double* mu,
                   jd_iter_log* log, int32_t* iters_done, void* traj, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
    FbHost p;
    HostRun r;
    int rc = fb_prepare(prob, run, p, r);
    if (rc)
        return rc;
    const bool need_traj = r.mode == JD_STORE;
    if (!mu || (need_traj && !traj) || (traj && !aligned(traj, real_size(r.prec))) ||
        validate_opt(opt))
        return JD_EINVAL;
    FbWs w;
    if ((rc = fb_bind(p, r, ws, ws_bytes, w)))
        return rc;
    if (iters_done)
        *iters_done = 0;
    if (opt->n_max == 0)
        return JD_OK;
    LsDriver drv;
    drv.opt = *opt;
    drv.hdr = w.hdr;
    drv.ring = w.ring;
    drv.u = mu;
    drv.ut = w.ut;
    drv.nd = p.N * p.L;
    drv.dt = p.dt;
    drv.iter0 = r.iter;
    FbOps ops(p, r, mu, traj, w);
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

int jd_fb_draws(const jd_fb_problem* prob, const jd_run* run, int64_t m0, int64_t mc, int32_t k0,
                int32_t kc, void* z_init, void* Z, int32_t* counts, hipStream_t stream) {
    FbHost p;
    HostRun r;
    int rc = fb_prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (m0 < 0 || mc < 0 || k0 < 0 || kc < 0 || m0 + mc > ((int64_t)1 << 32) ||
        (int64_t)k0 + kc > ((int64_t)1 << 31) - 1 || mc * (int64_t)kc > ((int64_t)1 << 40))
        return JD_EINVAL;
    if (mc == 0 || kc == 0)
        return JD_OK;
    JD_TRY(fb_launch_draws(p, r, m0, mc, k0, kc, z_init, Z, counts, stream));
    return JD_OK;
}

}  // extern "C"
