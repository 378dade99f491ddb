// Host-side form of the feedback-model problem (include/jd_feedback.h) and
// the typed launchers of its kernels (fb_kernels.hip).
#pragma once

#include <stdint.h>

#include "jd_launch.hpp"

namespace jd {

constexpr int kFbMaxGrid = 16;  // nx, nv <= 16: one 16 x 16 matrix-core tile per step
constexpr int kFbJumpStates = 32;  // post-jump states (x, v, jump time) kept per particle (jump-adapted grid)

struct FbHost {
    int N, nx, nv, nvp, L;  // nvp: the compiled row width >= nv (zero-padded control rows)
    double T, dt, eta, b1, b2, gamma, beta, rate;
    double xmax, vmax, eps, alpha, sigJ;
    int init_kind;
    double z0[2], s0[2];
    double svar0[2], svar1[2];  // surrogate-state variance var(t) = svar0 + svar1 t
    bool svar_fit;              // surrogate variance fitted to the forward ensemble instead
    const double* zd;     // device (N+1) x 2, or null (ellipse cost)
    int np;               // particles per ring (1: independent particles)
    int G;                // ring kernels: 256-slot groups per workgroup
    int rings_per_block;  // ring kernels: rings per workgroup
    int64_t nsys;         // rings (np > 1)
    double omega;         // nearest-neighbour coupling
    int cost_kind;        // JD_FB_COST_TRACK / JD_FB_COST_ELLIPSE
    double ax, av;        // ellipse half-axes
    int grid;             // JD_FB_GRID_FIXED / JD_FB_GRID_ADAPTED
    double ks[64];        // gamma^n and sqrt(V_n) for n = 0..31
    uint64_t thr[32];     // Poisson(rate dt) thresholds
    PoissonTable poisson;
};

// Per-step table in the path precision: mu rows (N x nx x nvp, zero-padded),
// targets ((N+1) x 2), the Keilson-Storer factors (32 x 2) and the surrogate
// states' standard deviations ((N+1) x 2, surrogate gradient only).
struct FbTable {
    size_t mu, zd, ks, sd, count;  // element offsets and total elements
};
FbTable fb_table_layout(const FbHost& p);
// FP64 elements of the surrogate gradient's per-step moment partials
// ((N+1) x forward blocks x 4) and of its variance record ((N+1) x 2 per-step
// variances, then the line a_x, a_v, b_x, b_v).
size_t fb_mom_count(const FbHost& p, const HostRun& r);
size_t fb_svar_count(const FbHost& p);

hipError_t fb_launch_table(const FbHost& p, const HostRun& r, const double* mu, void* tab,
                           WsHeader* hdr, int clear_flag, hipStream_t st, Gate gate = kNoGate);
hipError_t fb_launch_forward(const FbHost& p, const HostRun& r, const void* tab, void* traj,
                             double* cpart, const WsHeader* hdr, hipStream_t st,
                             Gate gate = kNoGate);
// surrogate: the adjoint on the surrogate states, added to the partials of
// fb_launch_forward_grad (Section 6.5); else the exact adjoint over traj.
hipError_t fb_launch_adjoint(const FbHost& p, const HostRun& r, const void* tab, const void* traj,
                             double* apart, const WsHeader* hdr, bool surrogate, hipStream_t st,
                             Gate gate = kNoGate);
// Storage-free forward that also writes the alpha u phi(z) part of the
// gradient partials (surrogate gradient) and the per-block costs.
hipError_t fb_launch_forward_grad(const FbHost& p, const HostRun& r, const void* tab, double* cpart,
                                  double* apart, double* mom, const WsHeader* hdr, hipStream_t st,
                                  Gate gate = kNoGate);
// The surrogate variance line (given, or fitted to the moment partials mom of
// fb_launch_forward_grad when mom is not null) into svar, and the per-step
// standard deviations into the table.
hipError_t fb_launch_surrogate_sd(const FbHost& p, const HostRun& r, const double* mom,
                                  double* svar, void* tab, hipStream_t st, Gate gate = kNoGate);
// 256-particle groups per block of the adjoint (and of the surrogate's
// forward, which shares its partials).
int fb_adjoint_groups(const FbHost& p, const HostRun& r);
// Number of per-block partials of the adjoint / forward_grad kernels, and of
// the per-block costs of the forward kernel.
int fb_partial_blocks(const FbHost& p, const HostRun& r);
int fb_forward_blocks(const FbHost& p, const HostRun& r);
// 256-slot groups per workgroup of the ring kernels for rings of np particles.
int fb_ring_groups(int np);
hipError_t fb_launch_finalize_grad(const FbHost& p, const HostRun& r, const double* apart,
                                   double* g, WsHeader* hdr, hipStream_t st, Gate gate = kNoGate);
hipError_t fb_launch_finalize_cost(const FbHost& p, const HostRun& r, const double* cpart,
                                   int ncpart, const double* g, double* J_out, WsHeader* hdr,
                                   int slot, hipStream_t st, Gate gate = kNoGate);
hipError_t fb_launch_draws(const FbHost& p, const HostRun& r, int64_t m0, int64_t mc, int k0,
                           int kc, void* z_init, void* Z, int32_t* counts, hipStream_t st);

}  // namespace jd
