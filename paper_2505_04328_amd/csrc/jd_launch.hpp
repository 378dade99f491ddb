// Internal interface between the C-ABI layer (jd_api.cpp) and the kernels
// (jd_kernels.hip).  Host-side, validated, FP64 problem data in the padded
// layout the kernels use.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/jd.h"

namespace jd {

constexpr int kBlock = 256;  // threads per block of the sweep kernels

// Inverse-CDF Poisson thresholds in the form the sweeps compare against: the
// count is the smallest j with P < thr_j, i.e. the number of leading j with
// P > thr_j - 1.  tm1[j] = thr_j - 1 fits 32 bits (thr_0 >= 1 for rate*dt <= 2,
// and a saturated thr_j = 2^32 becomes 0xFFFFFFFF, which no word exceeds);
// jmax is the first j whose threshold saturates, beyond which the count cannot
// grow.  Prepared on the host, staged in the workspace header by the table
// kernel, read by the sweeps with wave-uniform indices.
struct PoissonTable {
    uint32_t tm1[32];
    int32_t jmax;
};

struct HostProblem {
    int d;   // caller's dimension
    int D;   // padded dimension: 1, 2, 4 or 8
    int N;
    double T, dt, lambda, cubic, nu;
    double A[64];  // D x D row-major, zero-padded
    double B[64];  // d x d row-major (caller layout)
    double x0[8], s[8], jm[8], js[8], xT[8];  // zero-padded to D
    const double* xd;  // device, N x d
    uint64_t thr[32];  // Poisson thresholds for lambda*dt
    PoissonTable poisson;
};

struct HostRun {
    int64_t M;
    int64_t ldm;  // M rounded up to a multiple of kBlock (trajectory columns)
    uint64_t seed;
    uint32_t iter;
    int prec;  // JD_FP32 / JD_FP64
    int mode;  // JD_STORE / JD_RECOMPUTE
    int K;
    int nblk;  // blocks of the sweeps = ceil(M / kBlock)
    bool noise;  // forward sweeps read the iteration's noise table
    const jd_dump* dump;
};

// Device header at the start of every workspace.
struct WsHeader {
    double J;        // last cost reduction
    double gnorm2;   // dt * sum |g_k|^2 of the last gradient reduction
    double J_trial;  // last cost-only reduction of a line-search trial
    double E2;       // dt * sum |u' - u|^2 of the last accepted trial
    int32_t accept;  // last Armijo test
    int32_t nonfinite;
    PoissonTable poisson;  // staged by the table kernel for the sweeps
    // Line-search state of a device-driven gradient iteration (jd_optimize,
    // the request server): the phase that may run next, ls_phase(n, j) with
    // j = -1 the evaluation of J(u^n), g^n and j >= 0 Armijo trial j of
    // iteration n, or kLsStop; the outcome (kLsRunning, kLsDone or a JD_E*
    // code); the number of accepted iterations.
    int32_t ls_status;
    int64_t ls_phase;
    int32_t ls_done;
    int32_t pad[17];
};
static_assert(sizeof(WsHeader) == 256, "header is one 256-byte line");

constexpr int32_t kLsRunning = 1;
constexpr int32_t kLsDone = 0;
constexpr int64_t kLsStop = -1;
__host__ __device__ inline int64_t ls_phase(int n, int j) {
    return ((int64_t)n << 32) | (int64_t)(uint32_t)(j + 1);
}

// One accepted iteration of a device-driven gradient iteration, written by
// the Armijo kernel into a ring of kLsLogCap entries that follows the header
// in the workspace (entry n % kLsLogCap for iteration n).
struct LsLog {
    double J, gnorm2, zeta, J_new, E2;
    uint32_t iter;
    int32_t backtracks;
    int32_t n;
    int32_t pad[3];
};
static_assert(sizeof(LsLog) == 64, "log entries are 64 bytes");
constexpr int kLsLogCap = 64;

// A launch gate: a kernel launched with a gate runs only when the header's
// phase word equals `tag`, and otherwise returns at once (every block reads
// the same word, which only a previous kernel on the stream writes).  A null
// word means an ungated launch.
struct Gate {
    const int64_t* word;
    int64_t tag;
};
constexpr Gate kNoGate = {nullptr, 0};
inline Gate gate_of(WsHeader* hdr, int64_t tag) { return Gate{&hdr->ls_phase, tag}; }

enum FwdMode { FWD_COST = 0, FWD_STORE = 1, FWD_CKPT = 2 };

size_t real_size(int prec);

// Register-buffer shape of the recomputing adjoint's register kernel: R steps
// of D values plus S sub-segment starts; it takes checkpoint intervals up to
// R S, regenerating every step once for K <= R and twice beyond.
template <typename Real, int D>
struct RecomputeShape;
template <> struct RecomputeShape<float, 1> { static constexpr int R = 32, S = 4; };
template <> struct RecomputeShape<float, 2> { static constexpr int R = 16, S = 4; };
template <> struct RecomputeShape<float, 4> { static constexpr int R = 8, S = 8; };
template <> struct RecomputeShape<float, 8> { static constexpr int R = 8, S = 8; };
template <> struct RecomputeShape<double, 1> { static constexpr int R = 16, S = 4; };
template <> struct RecomputeShape<double, 2> { static constexpr int R = 8, S = 4; };
template <> struct RecomputeShape<double, 4> { static constexpr int R = 4, S = 8; };
template <> struct RecomputeShape<double, 8> { static constexpr int R = 4, S = 4; };

// Checkpoint-recompute adjoint.  Short intervals run a kernel that rebuilds
// each segment in registers; where that would regenerate every step twice
// (d = 8) or the interval exceeds its buffers, a persistent kernel of
// seg_blocks() blocks regenerates each segment once into a scratch region of
// K d 256 elements per block in the workspace (seg_scratch_bytes(), at most
// kSegScratchMax; larger intervals are JD_EUNSUPPORTED).
constexpr int kSegBlocks = 1024;
constexpr size_t kSegScratchMax = (size_t)8 << 30;
inline int seg_blocks(const HostRun& r) { return r.nblk < kSegBlocks ? r.nblk : kSegBlocks; }
bool recompute_uses_segments(int prec, int D, int K);
size_t seg_scratch_bytes(const HostProblem& p, const HostRun& r);
bool recompute_supported(const HostProblem& p, const HostRun& r);

// The table kernel runs first in every entry point and (clear_flag != 0)
// clears the non-finite flag; the reductions raise it.  Every launcher takes
// an optional gate (kNoGate: always runs).
hipError_t launch_setup(const HostProblem& p, const HostRun& r, const double* u, void* tab,
                        WsHeader* hdr, int clear_flag, hipStream_t st, Gate gate = kNoGate);
// noise: the iteration's noise table (launch_setup_noise) or nullptr (draws in the
// sweep); the results are bitwise the same.
hipError_t launch_forward(const HostProblem& p, const HostRun& r, const void* tab, void* traj,
                          int fwd_mode, double* cpart, const WsHeader* hdr, hipStream_t st,
                          Gate gate = kNoGate, const void* noise = nullptr);
// launch_setup and the noise table of iteration r.iter (noise_bytes(): the
// Brownian normals and jump increments of every path-step) in one launch: the
// table's blocks, then min(nblk N, kNoiseGrid) blocks of draws.
constexpr int64_t kNoiseGrid = 65536;
hipError_t launch_setup_noise(const HostProblem& p, const HostRun& r, const double* u, void* tab,
                              void* noise, WsHeader* hdr, int clear_flag, hipStream_t st,
                              Gate gate = kNoGate);
// seg: the workspace's segment scratch (seg_scratch_bytes(); unused otherwise)
hipError_t launch_adjoint(const HostProblem& p, const HostRun& r, const void* tab, const void* traj,
                          double* apart, void* seg, const WsHeader* hdr, hipStream_t st,
                          Gate gate = kNoGate);
// Forward (stored trajectory) and adjoint fused per block (no dump support).
hipError_t launch_cost_grad_stored(const HostProblem& p, const HostRun& r, const void* tab,
                                  void* traj, double* cpart, double* apart, const WsHeader* hdr,
                                  hipStream_t st, Gate gate = kNoGate,
                                  const void* noise = nullptr);
hipError_t launch_finalize_grad(const HostProblem& p, const HostRun& r, const double* apart,
                                const double* u, double* g, WsHeader* hdr, hipStream_t st,
                                Gate gate = kNoGate);
// Device-driven line search (Section 5, Algorithm 5.4 with eq.
// Stochastic_Armijo).  ls_start opens phase (0, -1); ls_after_grad (gated
// by phase (n, -1)) moves to trial (n, 0), or stops with JD_ENONFINITE when
// J or g is not finite; the Armijo test of trial (n, j) (gated by its phase)
// accepts when J_trial is finite and J_trial <= J - c zeta ||g||^2_L2, moves u
// to the trial point, logs the iteration and opens (n + 1, -1) or stops
// (n + 1 == n_max, or ||u' - u||_L2 <= tol); on rejection it opens (n, j + 1)
// or stops with JD_ELINESEARCH after max_backtracks trials.
struct LsArmijo {
    double c_armijo, zeta, dt, tol;
    int n, j, n_max, max_backtracks;
    uint32_t iter;
};

// A line-search step run by the cost reduction that precedes it
// (launch_finalize_cost), in place of its own launch: the after-gradient step
// of iteration n, or the Armijo test of a trial (ring, u, ut, nd as for
// launch_armijo).  The reduction's gate is the step's phase.
constexpr int kLsTailNone = 0;
constexpr int kLsTailAfterGrad = 1;
constexpr int kLsTailArmijo = 2;
struct LsTail {
    int mode;
    int n;
    LsArmijo ls;
    LsLog* ring;
    double* u;
    const double* ut;
    int nd;
};

// slot 0: J -> hdr->J (and J_out), with gnorm2 from g if g != nullptr, and a
// non-finite J or g raises the flag; slot 1 (a line-search trial): ->
// hdr->J_trial, no flag (the Armijo test rejects a non-finite trial cost).
// tail (may be null): the line-search step that follows.
hipError_t launch_finalize_cost(const HostProblem& p, const HostRun& r, const double* cpart,
                                const double* u, const double* g, double* J_out, WsHeader* hdr,
                                int slot, hipStream_t st, Gate gate = kNoGate,
                                const LsTail* tail = nullptr);
hipError_t launch_trial(const double* u, const double* g, double zeta, double* ut, int nd,
                        hipStream_t st, Gate gate = kNoGate);
// launch_trial and launch_setup(ut) in one launch: ut = u - zeta g and the
// per-step table of ut (no flag clearing), bitwise the two launches' results.
hipError_t launch_setup_trial(const HostProblem& p, const HostRun& r, const double* u,
                              const double* g, double zeta, double* ut, void* tab, WsHeader* hdr,
                              hipStream_t st, Gate gate = kNoGate);

hipError_t launch_ls_start(WsHeader* hdr, hipStream_t st);
hipError_t launch_ls_after_grad(WsHeader* hdr, int n, hipStream_t st);
hipError_t launch_armijo(WsHeader* hdr, LsLog* ring, double* u, const double* ut, int nd,
                         const LsArmijo& ls, hipStream_t st);
hipError_t launch_draws(const HostProblem& p, const HostRun& r, int64_t m0, int64_t mc, int k0,
                        int kc, void* zw, void* zj, int32_t* counts, hipStream_t st);
hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out,
                         hipStream_t st);
hipError_t launch_clear_flag(WsHeader* hdr, hipStream_t st);

}  // namespace jd
