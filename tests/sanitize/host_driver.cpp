// Drives the host code of libjd (built with the sanitizers against
// host_stubs.cpp): argument validation of every entry point, workspace and
// trajectory sizing over the shapes the kernels take, the line-search driver,
// and the request server's admission, arena, failure and release paths.
// Exit status 0 when every check holds (and the sanitizers found nothing).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/jd.h"
#include "../../include/jd_feedback.h"
#include "../../include/jd_server.h"

extern int g_fail_event_at;
extern int g_events_created;
extern int g_launches;

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(1);                                                        \
        }                                                                   \
    } while (0)

struct Prob {
    int d, N;
    std::vector<double> x0, A, B, s, jm, js, xT, xd;
    jd_problem st;
    Prob(int d_, int N_, double T, double lam, double cubic) : d(d_), N(N_) {
        x0.assign(d, 0.1);
        A.assign(d * d, 0.0);
        B.assign(d * d, 0.0);
        for (int i = 0; i < d; ++i) {
            A[i * d + i] = -1.0;
            B[i * d + i] = 1.0;
            if (i + 1 < d)
                A[i * d + i + 1] = 0.3;
        }
        s.assign(d, 0.3);
        jm.assign(d, 0.0);
        js.assign(d, 0.2);
        xT.assign(d, 1.0);
        xd.assign((size_t)N * d, 0.5);
        st = {d, N, T, lam, cubic, 1e-3, x0.data(), A.data(), B.data(), s.data(), jm.data(),
              js.data(), xT.data(), xd.data()};
    }
};

static jd_run run_of(int64_t M, int prec, int mode, int K) {
    jd_run r;
    memset(&r, 0, sizeof(r));
    r.M = M;
    r.seed = 1;
    r.precision = prec;
    r.mode = mode;
    r.K = K;
    return r;
}

// Host buffers standing in for device memory, sized by the library.
struct Bufs {
    std::vector<unsigned char> ws, traj;
    std::vector<double> u, g;
    double J;
};

static void validation() {
    Prob p(3, 20, 1.0, 2.0, 0.1);
    jd_run r = run_of(1000, JD_FP32, JD_STORE, 0);
    CHECK(jd_workspace_bytes(&p.st, &r) > 0);
    CHECK(jd_workspace_bytes(nullptr, &r) == 0);
    CHECK(jd_workspace_bytes(&p.st, nullptr) == 0);
    const jd_problem good = p.st;
    auto bad = [&](jd_problem q) { CHECK(jd_workspace_bytes(&q, &r) == 0); };
    jd_problem q = good;
    q.d = 0; bad(q);
    q = good; q.d = 9; bad(q);
    q = good; q.N = 0; bad(q);
    q = good; q.T = 0.0; bad(q);
    q = good; q.T = NAN; bad(q);
    q = good; q.lambda = -1.0; bad(q);
    q = good; q.lambda = 41.0; bad(q);  // lambda dt > 2
    q = good; q.nu = -1.0; bad(q);
    q = good; q.cubic = INFINITY; bad(q);
    q = good; q.xd = nullptr; bad(q);
    q = good; q.A = nullptr; bad(q);
    std::vector<double> Ainf(p.A);
    Ainf[4] = NAN;
    q = good; q.A = Ainf.data(); bad(q);
    auto badrun = [&](jd_run rr) { CHECK(jd_workspace_bytes(&good, &rr) == 0); };
    badrun(run_of(0, JD_FP32, JD_STORE, 0));
    badrun(run_of(((int64_t)1 << 31) + 1, JD_FP32, JD_STORE, 0));
    badrun(run_of(1000, 2, JD_STORE, 0));
    badrun(run_of(1000, JD_FP32, 7, 0));
    badrun(run_of(1000, JD_FP32, JD_RECOMPUTE, 0));
    badrun(run_of(1000, JD_FP32, JD_RECOMPUTE, 21));
    jd_dump dp = {990, 20, nullptr, nullptr, nullptr};
    jd_run rd = r;
    rd.dump = &dp;
    badrun(rd);
    // a segment scratch beyond 8 GiB is refused, one within it is not
    Prob p8(8, 2000, 2.0, 3.0, 0.1);
    jd_run big = run_of((int64_t)1 << 20, JD_FP32, JD_RECOMPUTE, 1100);
    double fake = 0.0;
    CHECK(jd_forward(&p8.st, &big, &fake, nullptr, &fake, &fake, 1 << 20, nullptr) == JD_EUNSUPPORTED);
    big.K = 1000;
    CHECK(jd_workspace_bytes(&p8.st, &big) > ((size_t)1000 * 8 * 256 * 4 * 1024));
    // Poisson thresholds
    uint64_t thr[32];
    CHECK(jd_poisson_thresholds(2.1, thr) == JD_EINVAL);
    CHECK(jd_poisson_thresholds(-0.1, thr) == JD_EINVAL);
    for (double mu : {0.0, 0.005, 0.5, 2.0}) {
        CHECK(jd_poisson_thresholds(mu, thr) == JD_OK);
        for (int j = 1; j < 32; ++j)
            CHECK(thr[j] >= thr[j - 1]);
        CHECK(thr[31] == ((uint64_t)1 << 32));
    }
    CHECK(jd_poisson_thresholds(0.0, thr) == JD_OK && thr[0] == ((uint64_t)1 << 32));
    for (int c = -8; c <= 1; ++c)
        CHECK(jd_strerror(c) != nullptr);
}

// Every entry point with buffers of exactly the sizes the library asks for.
static void entry_points() {
    for (int d = 1; d <= 8; ++d)
        for (int prec : {JD_FP32, JD_FP64})
            for (int K : {0, 1, 7, 16, 64, 65}) {
                Prob p(d, 70, 1.0, 3.0, 0.05);
                const int64_t M = d * 131 + 5;
                jd_run r = run_of(M, prec, K ? JD_RECOMPUTE : JD_STORE, K > 70 ? 70 : K);
                const size_t wb = jd_workspace_bytes(&p.st, &r), tb = jd_traj_bytes(&p.st, &r);
                CHECK(wb > 0 && tb > 0);
                Bufs b;
                b.ws.assign(wb, 0);
                b.traj.assign(tb, 0);
                b.u.assign((size_t)p.N * d, 0.0);
                b.g.assign((size_t)p.N * d, 0.0);
                void* ws = b.ws.data();
                void* tj = b.traj.data();
                CHECK(jd_forward(&p.st, &r, b.u.data(), tj, &b.J, ws, wb, nullptr) == JD_OK);
                CHECK(jd_forward(&p.st, &r, b.u.data(), nullptr, &b.J, ws, wb, nullptr) == JD_OK);
                CHECK(jd_adjoint(&p.st, &r, b.u.data(), tj, b.g.data(), ws, wb, nullptr) == JD_OK);
                CHECK(jd_cost_grad(&p.st, &r, b.u.data(), &b.J, b.g.data(), tj, ws, wb, nullptr) == JD_OK);
                CHECK(jd_cost_grad(&p.st, &r, b.u.data(), &b.J, b.g.data(), tj, ws, wb - 1, nullptr) ==
                      JD_EWORKSPACE);
                CHECK(jd_cost_grad(&p.st, &r, b.u.data(), &b.J, b.g.data(), (char*)tj + 1, ws, wb,
                                   nullptr) == JD_EINVAL);
                CHECK(jd_cost_grad(&p.st, &r, nullptr, &b.J, b.g.data(), tj, ws, wb, nullptr) == JD_EINVAL);
                jd_opt o = {5, 30, 0.0, 1.0, 0.5, 1e-4};
                jd_iter_log log[5];
                int32_t done = -1;
                // the stand-in launches leave the header zero: the iteration
                // reads "done" after the first batch
                CHECK(jd_optimize(&p.st, &r, &o, b.u.data(), log, &done, tj, ws, wb, nullptr) == JD_OK);
                CHECK(done == 0);
                jd_opt bado = o;
                bado.rho = 1.0;
                CHECK(jd_optimize(&p.st, &r, &bado, b.u.data(), log, &done, tj, ws, wb, nullptr) ==
                      JD_EINVAL);
                CHECK(jd_check_finite(ws, wb, nullptr) == JD_OK);
                std::vector<float> zw((size_t)4 * 3 * d);
                std::vector<int32_t> cnt(12);
                CHECK(jd_draws(&p.st, &r, 2, 4, 3, 3, zw.data(), nullptr, cnt.data(), nullptr) == JD_OK);
                CHECK(jd_draws(&p.st, &r, -1, 4, 3, 3, zw.data(), nullptr, cnt.data(), nullptr) == JD_EINVAL);
            }
}

static void feedback() {
    std::vector<double> zd(2 * 51, 0.0);
    for (int grid : {JD_FB_GRID_FIXED, JD_FB_GRID_ADAPTED})
        for (int np : {1, 3, 300}) {
            if (grid == JD_FB_GRID_ADAPTED && np > 1)
                continue;
            jd_fb_problem q;
            memset(&q, 0, sizeof(q));
            q.N = 50; q.nx = 6; q.nv = 5; q.T = 5.0; q.eta = 1.0; q.b1 = 0.1; q.b2 = 0.2;
            q.gamma = 0.9; q.beta = 10.0; q.xmax = 3.0; q.vmax = 3.0; q.eps = 0.7; q.alpha = 0.1;
            q.sigJ = 0.5; q.init_kind = JD_FB_INIT_GAUSS; q.z0[0] = 0.5; q.s0[0] = 0.1;
            q.s0[1] = 0.1; q.zd = zd.data(); q.np = np; q.omega = 0.5;
            q.cost_kind = JD_FB_COST_TRACK; q.ax = 1.0; q.av = 1.0; q.grid = grid;
            for (int mode : {JD_STORE, JD_SURROGATE}) {
                jd_run r = run_of(700, JD_FP32, mode, 0);
                const size_t wb = jd_fb_workspace_bytes(&q, &r), tb = jd_fb_traj_bytes(&q, &r);
                if (mode == JD_SURROGATE && (np > 1 || grid == JD_FB_GRID_ADAPTED)) {
                    CHECK(wb == 0);
                    continue;
                }
                CHECK(wb > 0 && tb > 0);
                std::vector<unsigned char> ws(wb), tj(tb);
                std::vector<double> mu((size_t)q.N * q.nx * q.nv, 0.0), g(mu.size());
                double J;
                CHECK(jd_fb_cost_grad(&q, &r, mu.data(), &J, g.data(), tj.data(), ws.data(), wb,
                                      nullptr) == JD_OK);
                jd_opt o = {3, 30, 0.0, 1.0, 0.5, 1e-4};
                int32_t done = -1;
                CHECK(jd_fb_optimize(&q, &r, &o, mu.data(), nullptr, &done, tj.data(), ws.data(), wb,
                                     nullptr) == JD_OK);
            }
            jd_fb_problem b = q;
            b.nx = 17;
            jd_run r = run_of(700, JD_FP32, JD_STORE, 0);
            CHECK(jd_fb_workspace_bytes(&b, &r) == 0);
        }
}

// The request server over a host arena: requests of different sizes, too
// many to fit at once, one whose admission fails; every request ends, the
// arena is returned whole (the sanitizers see any leak or overrun).
static void server() {
    unsigned lcg = 12345;
    auto rnd = [&](int n) {
        lcg = lcg * 1103515245u + 12345u;
        return (int)((lcg >> 8) % (unsigned)n);
    };
    struct Req {
        Prob* p;
        jd_run r;
        size_t bytes;
    };
    std::vector<Req> reqs;
    for (int i = 0; i < 24; ++i) {
        Req q;
        q.p = new Prob(1 << rnd(4), 20 + rnd(100), 1.0, 3.0, 0.0);
        q.r = run_of(500 + rnd(1500), JD_FP32, rnd(3) ? JD_STORE : JD_RECOMPUTE, 16);
        q.bytes = jd_server_request_bytes(&q.p->st, &q.r);
        CHECK(q.bytes > 0);
        reqs.push_back(q);
    }
    // the three largest first; the arena holds the two largest and half of
    // the third, so the first scheduling step admits two and the third waits
    // for memory while slots are free
    for (int a = 0; a < 3; ++a)
        for (size_t b = a + 1; b < reqs.size(); ++b)
            if (reqs[b].bytes > reqs[a].bytes)
                std::swap(reqs[a], reqs[b]);
    const size_t arena_bytes = reqs[0].bytes + reqs[1].bytes + reqs[2].bytes / 2 + 256;
    std::vector<unsigned char> arena(arena_bytes);
    jd_server* S = nullptr;
    CHECK(jd_server_create(arena.data(), arena_bytes, 32, 3, &S) == JD_OK);
    g_events_created = 0;
    g_fail_event_at = 4;  // the fifth admission fails
    std::vector<int64_t> tickets;
    for (Req& q : reqs) {
        jd_opt o = {3, 30, 0.0, 1.0, 0.5, 1e-4};
        int64_t t = 0;
        CHECK(jd_server_submit(S, &q.p->st, q.p->xd.data(), &q.r, &o, nullptr, &t) == JD_OK);
        tickets.push_back(t);
    }
    {
        Prob big(8, 2000, 1.0, 3.0, 0.0);
        jd_run r = run_of((int64_t)1 << 20, JD_FP32, JD_STORE, 0);
        jd_opt o = {3, 30, 0.0, 1.0, 0.5, 1e-4};
        int64_t t = 0;
        CHECK(jd_server_submit(S, &big.st, big.xd.data(), &r, &o, nullptr, &t) == JD_EWORKSPACE);
    }
    int32_t act = 0, que = 0, most_active = 0, queued_with_slot = 0;
    int64_t done = 0;
    for (int it = 0; it < 10000 && done < (int64_t)tickets.size(); ++it) {
        jd_server_progress(S, &act, &que, &done);
        most_active = act > most_active ? act : most_active;
        if (que > 0 && act < 32)
            ++queued_with_slot;
    }
    printf("server: at most %d admitted at once, %d scheduling steps with a request waiting for memory\n",
           most_active, queued_with_slot);
    CHECK(done == (int64_t)tickets.size());
    CHECK(most_active > 1 && queued_with_slot > 0);
    int failed = 0;
    for (size_t i = 0; i < tickets.size(); ++i) {
        std::vector<double> u((size_t)reqs[i].p->N * reqs[i].p->d, -1.0);
        jd_iter_log log[3];
        int32_t iters = -1, status = 1;
        double queued = -1.0, service = -1.0;
        CHECK(jd_server_times(S, tickets[i], &queued, &service) == JD_OK);
        CHECK(queued >= 0.0 && service >= 0.0);
        CHECK(jd_server_result(S, tickets[i], u.data(), log, &iters, &status) == JD_OK);
        CHECK(jd_server_times(S, tickets[i], &queued, &service) == JD_EINVAL);
        if (status == JD_EHIP)
            ++failed;
        else
            CHECK(status == JD_OK && iters == 0);
        CHECK(jd_server_result(S, tickets[i], u.data(), log, &iters, &status) == JD_EINVAL);
    }
    CHECK(failed == 1);
    CHECK(jd_server_destroy(S) == JD_OK);
    for (Req& q : reqs)
        delete q.p;
    g_fail_event_at = -1;
}

int main() {
    validation();
    entry_points();
    feedback();
    server();
    printf("host checks passed (%d launches)\n", g_launches);
    return 0;
}
