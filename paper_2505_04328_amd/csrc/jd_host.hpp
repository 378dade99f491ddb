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

size_t round_up(size_t x, size_t a);

// Poisson(mu) inverse-CDF thresholds against a 32-bit word (32 entries).
void poisson_thresholds(double mu, uint64_t* thr);
// The 32-bit thresholds minus one and the last index below 2^32, for the kernels.
PoissonTable poisson_table(const uint64_t* thr);

// Validates the problem and run and fills the padded host-side form.
int prepare(const jd_problem* prob, const jd_run* run, HostProblem& p, HostRun& r);
int validate_opt(const jd_opt* opt);

struct Layout {
    size_t hdr, tab, cpart, apart, gbuf, ut, total;
};
Layout layout(const HostProblem& p, const HostRun& r);
size_t traj_bytes(const HostProblem& p, const HostRun& r);

// The workspace regions, bound to a caller pointer.
struct Ws {
    WsHeader* hdr;
    void* tab;
    double* cpart;
    double* apart;
    double* gbuf;
    double* ut;
};
int bind_ws(const HostProblem& p, const HostRun& r, void* ws, size_t ws_bytes, Ws& w);
bool aligned(const void* ptr, size_t a);

// J(u) only (traj may be null) / J(u) and g(u) into g / one Armijo trial
// u' = u - zeta g (g in the workspace) with the test that moves u to u' on
// acceptance; the outcome is in the workspace header.
int enqueue_forward(const HostProblem& p, const HostRun& r, const double* u, void* traj, double* J,
                    const Ws& w, hipStream_t st);
int enqueue_cost_grad(const HostProblem& p, const HostRun& r, const double* u, double* J,
                      double* g, void* traj, const Ws& w, hipStream_t st);
int enqueue_trial(const HostProblem& p, const HostRun& r, double* u, const jd_opt& opt, double zeta,
                  const Ws& w, hipStream_t st);

}  // namespace host
}  // namespace jd
