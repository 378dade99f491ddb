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
    int32_t pad[21];
};
static_assert(sizeof(WsHeader) == 256, "header is one 256-byte line");

enum FwdMode { FWD_COST = 0, FWD_STORE = 1, FWD_CKPT = 2 };

size_t real_size(int prec);
bool recompute_supported(int prec, int D, int K);

// The table kernel runs first in every entry point and (clear_flag != 0)
// clears the non-finite flag; the reductions raise it.
hipError_t launch_setup(const HostProblem& p, const HostRun& r, const double* u, void* tab,
                        WsHeader* hdr, int clear_flag, hipStream_t st);
hipError_t launch_forward(const HostProblem& p, const HostRun& r, const void* tab, void* traj,
                          int fwd_mode, double* cpart, const WsHeader* hdr, hipStream_t st);
hipError_t launch_adjoint(const HostProblem& p, const HostRun& r, const void* tab, const void* traj,
                          double* apart, const WsHeader* hdr, hipStream_t st);
// Forward (stored trajectory) and adjoint fused per block (no dump support).
hipError_t launch_cost_grad_stored(const HostProblem& p, const HostRun& r, const void* tab,
                                  void* traj, double* cpart, double* apart, const WsHeader* hdr,
                                  hipStream_t st);
hipError_t launch_finalize_grad(const HostProblem& p, const HostRun& r, const double* apart,
                                const double* u, double* g, WsHeader* hdr, hipStream_t st);
// slot 0: J -> hdr->J (and J_out), with gnorm2 from g if g != nullptr; slot 1: -> hdr->J_trial
hipError_t launch_finalize_cost(const HostProblem& p, const HostRun& r, const double* cpart,
                                const double* u, const double* g, double* J_out, WsHeader* hdr,
                                int slot, hipStream_t st);
hipError_t launch_trial(const double* u, const double* g, double zeta, double* ut, int nd,
                        hipStream_t st);
hipError_t launch_armijo(WsHeader* hdr, double* u, const double* ut, int nd, double c_armijo,
                         double zeta, double dt, hipStream_t st);
hipError_t launch_draws(const HostProblem& p, const HostRun& r, int64_t m0, int64_t mc, int k0,
                        int kc, void* zw, void* zj, int32_t* counts, hipStream_t st);
hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out,
                         hipStream_t st);
hipError_t launch_clear_flag(WsHeader* hdr, hipStream_t st);

}  // namespace jd
