// Host-side internals shared by the C-ABI entry points (jd_api.cpp) and the
// request server (jd_server.cpp): validation, workspace layout and the launch
// sequences of one evaluation.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "jd_launch.hpp"

#define JD_TRY(expr)              \
    do {                          \
        if ((expr) != hipSuccess) \
            return JD_EHIP;       \
    } while (0)

namespace jd {
namespace host {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxPaths = (int64_t)1 << 31;

// JD_NOISE_AUTO takes the noise table for grids of at most
// noise_max_blocks(prec) blocks whose table takes at most kNoiseMaxBytes.
// Measured on c1's model (100 steps, 20 iterations, MI355X): FP64 with the
// table 2.13 / 3.37 ms at 10^4 / 65536 paths against 3.42 / 3.53 inline, and
// 9.97 against 8.49 at 2^18; FP32 1.96 against 2.11 ms at 10^4 paths and
// 2.21 against 2.15 at 3 10^4 (the table's HBM traffic, written once and
// read by every sweep, outweighs the draws an FP32 sweep computes sooner).
inline int noise_max_blocks(int prec) { return prec == JD_FP64 ? 256 : 64; }
constexpr size_t kNoiseMaxBytes = (size_t)1 << 30;
size_t noise_bytes(const HostProblem& p, const HostRun& r);

size_t round_up(size_t x, size_t a);

// Poisson(mu) inverse-CDF thresholds against a 32-bit word (32 entries).
void poisson_thresholds(double mu, uint64_t* thr);
// The 32-bit thresholds minus one and the last index below 2^32, for the kernels.
PoissonTable poisson_table(const uint64_t* thr);

// Validates the problem and run and fills the padded host-side form.
int prepare(const jd_problem* prob, const jd_run* run, HostProblem& p, HostRun& r);
int validate_opt(const jd_opt* opt);

struct Layout {
    size_t hdr, ring, tab, cpart, apart, gbuf, ut, seg, noise, total;
};
Layout layout(const HostProblem& p, const HostRun& r);
size_t traj_bytes(const HostProblem& p, const HostRun& r);

// The workspace regions, bound to a caller pointer.  The line-search log
// ring directly follows the header, so one copy of kLsMirrorBytes from the
// workspace start reads both.
constexpr size_t kLsMirrorBytes = sizeof(WsHeader) + kLsLogCap * sizeof(LsLog);
struct Ws {
    WsHeader* hdr;
    LsLog* ring;
    void* tab;
    double* cpart;
    double* apart;
    double* gbuf;
    double* ut;
    void* seg;  // segment scratch of the recompute adjoint (may be empty)
    void* noise;  // the iteration's noise table, or nullptr (draws in the sweeps)
};
int bind_ws(const HostProblem& p, const HostRun& r, void* ws, size_t ws_bytes, Ws& w);
bool aligned(const void* ptr, size_t a);

// J(u) only (traj may be null) / J(u) and g(u) into g / one Armijo trial
// u' = u - zeta g (g in the workspace) with the test that moves u to u' on
// acceptance; the outcome is in the workspace header.
int enqueue_forward(const HostProblem& p, const HostRun& r, const double* u, void* traj, double* J,
                    const Ws& w, hipStream_t st);
// tail (may be null): the line-search step that the final cost reduction
// runs (the after-gradient step).
int enqueue_cost_grad(const HostProblem& p, const HostRun& r, const double* u, double* J,
                      double* g, void* traj, const Ws& w, hipStream_t st, Gate gate = kNoGate,
                      const LsTail* tail = nullptr);
// Trial point u' = u - zeta g (g in the workspace) and its cost-only forward
// into the header's J_trial, all under `gate`; tail (may be null): the Armijo
// test, run by the trial's cost reduction.  With the noise table it reads
// the table that enqueue_cost_grad of the same iteration (r.iter) wrote into
// the workspace.
int enqueue_trial(const HostProblem& p, const HostRun& r, const double* u, double zeta,
                  const Ws& w, hipStream_t st, Gate gate, const LsTail* tail = nullptr);

// ---------------------------------------------------------------------------
// Device-driven gradient iteration (Section 5, Algorithm 5.4 with eq.
// Stochastic_Armijo).  The host enqueues, in the order they can run, the
// phases of up to a batch of iterations: for each iteration the evaluation of
// J(u^n), g^n, then `ahead` Armijo trials; every phase is gated by the
// header's phase word, which the device advances (see LsArmijo), so phases
// the device does not reach return at once.  After the batch the host reads
// the header and the log ring (one synchronization or event per batch), and
// resumes where the device stopped: at the next iteration, or at the next
// trial of an iteration that needed more trials than were enqueued.  The
// arithmetic and its order are those of one trial at a time.
struct LsOps {
    virtual ~LsOps() {}
    // J(u^n), g^n with counter word iter0 + n, under gate; tail: the
    // after-gradient step, which fused() evaluations run themselves
    virtual int grad(int n, const LsTail& tail, Gate gate, hipStream_t st) = 0;
    // trial point and cost of iteration n at step zeta, under gate; tail: the
    // Armijo test, which fused() trials run themselves
    virtual int trial(int n, double zeta, const LsTail& tail, Gate gate, hipStream_t st) = 0;
    // the tails run inside grad() and trial() (no launches of their own)
    virtual bool fused() const { return false; }
};

struct LsDriver {
    jd_opt opt;
    WsHeader* hdr;   // device
    LsLog* ring;     // device
    double* u;       // device, the iterate
    const double* ut;  // device, the trial point
    int nd;
    double dt;
    uint32_t iter0;
    int n_next = 0, j_next = -1;  // where the device stopped
    int ahead = 2;                // trials enqueued per iteration
    int copied = 0;               // log entries read
    int status = JD_OK;

    // Opens the iteration on the device (ls_start).
    int start(hipStream_t st);
    // Enqueues phases from the resume point for up to `iters` iterations.
    int enqueue(LsOps& ops, int iters, hipStream_t st);
    // Reads a completed batch from a host copy of header + ring; appends log
    // records (host, may be null) and returns true when the iteration ended
    // (status in `status`).
    bool collect(const void* mirror, jd_iter_log* log);
};

}  // namespace host
}  // namespace jd
