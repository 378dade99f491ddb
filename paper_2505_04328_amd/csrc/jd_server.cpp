// Request server: continuous batching of gradient-iteration requests (the
// paper's Algorithm 5.4, one per request) on one GPU.
//
//  * Admission by device-memory footprint: every request's buffers (control,
//    target, trajectory, workspace) are carved out of one caller-provided
//    device arena by a first-fit allocator; a queued request is admitted (in
//    arrival order, smaller ones may pass a large one that does not fit yet) as
//    soon as a slot and an extent of the arena are free.
//  * Overlap: admitted requests are spread over a few HIP streams; their
//    sweeps, reductions and line-search kernels run concurrently on the
//    device.  Each request's line search runs on the device (the gated phases
//    of jd_optimize: the device decides every Armijo trial and keeps u and the
//    counter word); the host enqueues a batch of kServeBatch iterations at a
//    time and looks at the request again only when the event after that batch
//    has completed, reading its outcome and log from a pinned copy of the
//    workspace header.  The host never blocks on one request.
//  * Results are identical to jd_optimize for the same request alone: the
//    same kernels run on the same per-request data in the same order.
//  * A request whose admission or enqueueing fails ends with that error as
//    its status; its stream is drained before its memory is reused.
//
// Single-threaded: one host thread drives a server.
#include <math.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "jd_host.hpp"
#include "../../include/jd_server.h"

using namespace jd;
using namespace jd::host;

namespace {

struct Extent {
    size_t off, len;
};

// First-fit sub-allocator over [0, size) in kAlign units, free list sorted by
// offset and coalesced on release.
class Arena {
  public:
    explicit Arena(size_t size) { free_.push_back({0, size}); }
    bool alloc(size_t n, size_t* off) {
        n = round_up(n, kAlign);
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].len >= n) {
                *off = free_[i].off;
                free_[i].off += n;
                free_[i].len -= n;
                if (free_[i].len == 0)
                    free_.erase(free_.begin() + i);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = round_up(n, kAlign);
        size_t i = 0;
        while (i < free_.size() && free_[i].off < off)
            ++i;
        free_.insert(free_.begin() + i, {off, n});
        if (i + 1 < free_.size() && free_[i].off + free_[i].len == free_[i + 1].off) {
            free_[i].len += free_[i + 1].len;
            free_.erase(free_.begin() + i + 1);
        }
        if (i > 0 && free_[i - 1].off + free_[i - 1].len == free_[i].off) {
            free_[i - 1].len += free_[i].len;
            free_.erase(free_.begin() + i);
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (const Extent& e : free_)
            s += e.len;
        return s;
    }

  private:
    std::vector<Extent> free_;
};

enum State { QUEUED, RUNNING, FINISHING, DONE };

// Iterations enqueued per request between two looks at it: small enough that
// requests sharing a stream interleave, large enough that the host is not in
// the loop of every iteration.
constexpr int kServeBatch = 4;

struct Request {
    int64_t ticket;
    // host copies of the problem data
    std::vector<double> x0, A, B, s, jm, js, xT, xd, u0;
    jd_problem prob;
    jd_run run;
    jd_opt opt;
    HostProblem p;
    HostRun r;
    size_t sz_u, sz_xd, sz_traj, sz_ws, bytes, off;
    double* u_dev;
    double* xd_dev;
    void* traj;
    void* ws;
    Ws w;
    int stream;
    int mirror;
    hipEvent_t ev;
    State state;
    int status;
    LsDriver drv;
    std::vector<jd_iter_log> log;
    std::vector<double> u_out;
    // host clock (seconds since the server was created): submission,
    // admission (-1 until admitted) and completion as the server saw them
    double t_submit, t_admit, t_done;
};

struct ReqOps : LsOps {
    Request& q;
    explicit ReqOps(Request& q_) : q(q_) {}
    int grad(int n, const LsTail& tail, Gate gate, hipStream_t st) override {
        HostRun rn = q.r;
        rn.iter = q.run.iter + (uint32_t)n;
        return enqueue_cost_grad(q.p, rn, q.u_dev, nullptr, q.w.gbuf, q.traj, q.w, st, gate,
                                 &tail);
    }
    int trial(int n, double zeta, const LsTail& tail, Gate gate, hipStream_t st) override {
        HostRun rn = q.r;
        rn.iter = q.run.iter + (uint32_t)n;
        return enqueue_trial(q.p, rn, q.u_dev, zeta, q.w, st, gate, &tail);
    }
    bool fused() const override { return true; }
};

}  // namespace

struct jd_server {
    char* arena_base;
    size_t arena_bytes;
    std::unique_ptr<Arena> arena;
    int max_active;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    char* mirrors;  // pinned host memory, one header + log ring per active slot
    std::vector<int> free_mirrors;
    std::deque<int64_t> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    int active;
    int64_t next_ticket;
    int64_t completed;
    std::chrono::steady_clock::time_point t0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

size_t footprint(const HostProblem& p, const HostRun& r, size_t* su, size_t* sxd, size_t* st,
                 size_t* sw) {
    *su = round_up((size_t)p.N * p.d * sizeof(double), kAlign);
    *sxd = *su;
    *st = round_up(traj_bytes(p, r), kAlign);
    *sw = round_up(layout(p, r).total, kAlign);
    return *su + *sxd + *st + *sw;
}

char* mirror_of(jd_server* S, const Request& q) { return S->mirrors + (size_t)q.mirror * kLsMirrorBytes; }

// The next batch of the request's iterations, then a copy of its header and
// log ring and the event the host polls.
int enqueue_batch(jd_server* S, Request& q) {
    hipStream_t st = S->streams[q.stream];
    ReqOps ops(q);
    int rc = q.drv.enqueue(ops, kServeBatch, st);
    if (rc)
        return rc;
    JD_TRY(hipMemcpyAsync(mirror_of(S, q), q.w.hdr, kLsMirrorBytes, hipMemcpyDeviceToHost, st));
    JD_TRY(hipEventRecord(q.ev, st));
    return JD_OK;
}

// Copy the final control back and mark the request as finishing.
int enqueue_finish(jd_server* S, Request& q, int status) {
    hipStream_t st = S->streams[q.stream];
    q.status = status;
    q.u_out.resize((size_t)q.p.N * q.p.d);
    JD_TRY(hipMemcpyAsync(q.u_out.data(), q.u_dev, q.u_out.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    JD_TRY(hipEventRecord(q.ev, st));
    q.state = FINISHING;
    return JD_OK;
}

void release(jd_server* S, Request& q) {
    S->arena->release(q.off, q.bytes);
    S->free_mirrors.push_back(q.mirror);
    S->stream_load[q.stream]--;
    (void)hipEventDestroy(q.ev);
    S->active--;
}

// A request that failed after admission: wait until its stream has no more of
// its work in flight, return its slot, mirror and memory, and end it with the
// error as its status (no control is returned).
void fail(jd_server* S, Request& q, int status) {
    (void)hipStreamSynchronize(S->streams[q.stream]);
    q.u_out.clear();
    q.status = status;
    q.state = DONE;
    q.t_done = S->now();
    release(S, q);
    S->completed++;
}

// 0: admitted; 1: does not fit now; otherwise the request ended with that
// error (it is DONE and holds nothing).
int admit(jd_server* S, Request& q) {
    if (!S->arena->alloc(q.bytes, &q.off))
        return 1;  // does not fit now
    char* base = S->arena_base + q.off;
    q.u_dev = (double*)base;
    q.xd_dev = (double*)(base + q.sz_u);
    q.traj = base + q.sz_u + q.sz_xd;
    q.ws = base + q.sz_u + q.sz_xd + q.sz_traj;
    q.p.xd = q.xd_dev;
    int rc = bind_ws(q.p, q.r, q.ws, q.sz_ws, q.w);
    if (rc == JD_OK && hipEventCreateWithFlags(&q.ev, hipEventDisableTiming) != hipSuccess)
        rc = JD_EHIP;
    if (rc) {
        S->arena->release(q.off, q.bytes);
        q.status = rc;
        q.state = DONE;
        q.t_done = S->now();
        S->completed++;
        return rc;
    }
    int best = 0;
    for (int i = 1; i < (int)S->streams.size(); ++i)
        if (S->stream_load[i] < S->stream_load[best])
            best = i;
    q.stream = best;
    S->stream_load[best]++;
    q.mirror = S->free_mirrors.back();
    S->free_mirrors.pop_back();
    S->active++;
    q.state = RUNNING;
    q.t_admit = S->now();
    hipStream_t st = S->streams[q.stream];
    const size_t nd = (size_t)q.p.N * q.p.d;
    q.log.assign((size_t)q.opt.n_max, jd_iter_log());
    q.drv.opt = q.opt;
    q.drv.hdr = q.w.hdr;
    q.drv.ring = q.w.ring;
    q.drv.u = q.u_dev;
    q.drv.ut = q.w.ut;
    q.drv.nd = (int)nd;
    q.drv.dt = q.p.dt;
    q.drv.iter0 = q.run.iter;
    if (hipMemcpyAsync(q.xd_dev, q.xd.data(), nd * sizeof(double), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(q.u_dev, q.u0.data(), nd * sizeof(double), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rc = JD_EHIP;
    else if (q.opt.n_max == 0)
        rc = enqueue_finish(S, q, JD_OK);
    else if (!(rc = q.drv.start(st)))
        rc = enqueue_batch(S, q);
    if (rc) {
        fail(S, q, rc);
        return rc;
    }
    return 0;
}

// Advance one running request whose last enqueued batch has completed.
int advance(jd_server* S, Request& q) {
    if (q.state == FINISHING) {
        q.state = DONE;
        q.t_done = S->now();
        release(S, q);
        S->completed++;
        return JD_OK;
    }
    int rc;
    if (q.drv.collect(mirror_of(S, q), q.log.data()))
        rc = enqueue_finish(S, q, q.drv.status);
    else
        rc = enqueue_batch(S, q);
    if (rc)
        fail(S, q, rc);
    return rc;
}

}  // namespace

extern "C" {

size_t jd_server_request_bytes(const jd_problem* prob, const jd_run* run) {
    HostProblem p;
    HostRun r;
    if (prepare(prob, run, p, r) != JD_OK)
        return 0;
    size_t a, b, c, d;
    return footprint(p, r, &a, &b, &c, &d);
}

int jd_server_create(void* arena, size_t arena_bytes, int32_t max_active, int32_t n_streams,
                     jd_server** out) {
    if (!out || !arena || arena_bytes < kAlign || max_active < 1 || n_streams < 1 ||
        n_streams > 16)
        return JD_EINVAL;
    *out = nullptr;
    std::unique_ptr<jd_server> S(new jd_server());
    char* base = (char*)round_up((size_t)(uintptr_t)arena, kAlign);
    S->arena_bytes = arena_bytes - (size_t)(base - (char*)arena);
    S->arena_base = base;
    S->arena.reset(new Arena(S->arena_bytes / kAlign * kAlign));
    S->max_active = max_active;
    S->active = 0;
    S->next_ticket = 1;
    S->t0 = std::chrono::steady_clock::now();
    S->completed = 0;
    S->mirrors = nullptr;
    if (hipHostMalloc((void**)&S->mirrors, kLsMirrorBytes * max_active, hipHostMallocDefault) !=
        hipSuccess)
        return JD_EHIP;
    for (int i = max_active - 1; i >= 0; --i)
        S->free_mirrors.push_back(i);
    for (int i = 0; i < n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t s : S->streams)
                (void)hipStreamDestroy(s);
            (void)hipHostFree(S->mirrors);
            return JD_EHIP;
        }
        S->streams.push_back(st);
        S->stream_load.push_back(0);
    }
    *out = S.release();
    return JD_OK;
}

int jd_server_submit(jd_server* S, const jd_problem* prob, const double* xd_host,
                     const jd_run* run, const jd_opt* opt, const double* u0_host, int64_t* ticket) {
    if (!S || !prob || !xd_host || !run || !ticket || validate_opt(opt))
        return JD_EINVAL;
    if (run->dump)
        return JD_EINVAL;
    std::unique_ptr<Request> q(new Request());
    const int d = prob->d, N = prob->N;
    if (d < 1 || d > 8 || N < 1 || !prob->x0 || !prob->A || !prob->B || !prob->s ||
        !prob->jump_mean || !prob->jump_std || !prob->xT)
        return JD_EINVAL;
    q->x0.assign(prob->x0, prob->x0 + d);
    q->A.assign(prob->A, prob->A + d * d);
    q->B.assign(prob->B, prob->B + d * d);
    q->s.assign(prob->s, prob->s + d);
    q->jm.assign(prob->jump_mean, prob->jump_mean + d);
    q->js.assign(prob->jump_std, prob->jump_std + d);
    q->xT.assign(prob->xT, prob->xT + d);
    q->xd.assign(xd_host, xd_host + (size_t)N * d);
    if (u0_host)
        q->u0.assign(u0_host, u0_host + (size_t)N * d);
    else
        q->u0.assign((size_t)N * d, 0.0);
    q->prob = *prob;
    q->prob.x0 = q->x0.data();
    q->prob.A = q->A.data();
    q->prob.B = q->B.data();
    q->prob.s = q->s.data();
    q->prob.jump_mean = q->jm.data();
    q->prob.jump_std = q->js.data();
    q->prob.xT = q->xT.data();
    q->prob.xd = q->xd.data();  // replaced by the device copy at admission
    q->run = *run;
    q->opt = *opt;
    int rc = prepare(&q->prob, &q->run, q->p, q->r);
    if (rc)
        return rc;
    q->bytes = footprint(q->p, q->r, &q->sz_u, &q->sz_xd, &q->sz_traj, &q->sz_ws);
    if (q->bytes > S->arena_bytes)
        return JD_EWORKSPACE;  // can never be admitted
    q->ticket = S->next_ticket++;
    q->state = QUEUED;
    q->status = JD_OK;
    q->t_submit = S->now();
    q->t_admit = -1.0;
    q->t_done = -1.0;
    *ticket = q->ticket;
    S->queue.push_back(q->ticket);
    S->reqs[q->ticket] = std::move(q);
    return JD_OK;
}

int jd_server_progress(jd_server* S, int32_t* n_active, int32_t* n_queued, int64_t* n_completed) {
    if (!S)
        return JD_EINVAL;
    int rc = JD_OK;
    // 1. advance requests whose last enqueued step finished
    for (auto& kv : S->reqs) {
        Request& q = *kv.second;
        if (q.state != RUNNING && q.state != FINISHING)
            continue;
        const hipError_t e = hipEventQuery(q.ev);
        if (e == hipErrorNotReady)
            continue;
        if (e != hipSuccess) {
            fail(S, q, JD_EHIP);
            if (!rc)
                rc = JD_EHIP;
            continue;
        }
        const int r2 = advance(S, q);
        if (r2 && !rc)
            rc = r2;
    }
    // 2. admit queued requests while slots and arena extents are free
    for (auto it = S->queue.begin(); it != S->queue.end() && S->active < S->max_active;) {
        Request& q = *S->reqs[*it];
        const int a = admit(S, q);
        if (a == 1) {
            ++it;  // does not fit yet; a smaller request behind it may
            continue;
        }
        it = S->queue.erase(it);
        if (a && !rc)
            rc = a;
    }
    if (n_active)
        *n_active = S->active;
    if (n_queued)
        *n_queued = (int32_t)S->queue.size();
    if (n_completed)
        *n_completed = S->completed;
    return rc;
}

int jd_server_result(jd_server* S, int64_t ticket, double* u_host, jd_iter_log* log,
                     int32_t* iters, int32_t* status) {
    if (!S)
        return JD_EINVAL;
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return JD_EINVAL;
    Request& q = *it->second;
    if (q.state != DONE)
        return JD_EAGAIN;
    if (u_host && !q.u_out.empty())  // a request that failed returns no control
        memcpy(u_host, q.u_out.data(), q.u_out.size() * sizeof(double));
    if (log && q.drv.copied > 0)
        memcpy(log, q.log.data(), (size_t)q.drv.copied * sizeof(jd_iter_log));
    if (iters)
        *iters = (int32_t)q.drv.copied;
    if (status)
        *status = q.status;
    S->reqs.erase(it);
    return JD_OK;
}

int jd_server_times(jd_server* S, int64_t ticket, double* queued, double* service) {
    if (!S)
        return JD_EINVAL;
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return JD_EINVAL;
    const Request& q = *it->second;
    if (q.state != DONE)
        return JD_EAGAIN;
    const double ta = q.t_admit >= 0.0 ? q.t_admit : q.t_done;  // never ran: all queueing
    if (queued)
        *queued = ta - q.t_submit;
    if (service)
        *service = q.t_done - ta;
    return JD_OK;
}

int jd_server_destroy(jd_server* S) {
    if (!S)
        return JD_EINVAL;
    for (hipStream_t st : S->streams)
        (void)hipStreamSynchronize(st);
    for (auto& kv : S->reqs) {
        Request& q = *kv.second;
        if (q.state == RUNNING || q.state == FINISHING)
            (void)hipEventDestroy(q.ev);
    }
    for (hipStream_t st : S->streams)
        (void)hipStreamDestroy(st);
    (void)hipHostFree(S->mirrors);
    delete S;
    return JD_OK;
}

}  // extern "C"
