// Host-only stand-ins for the HIP runtime calls and the kernel launchers of
// libjd, so that the library's host code (argument validation, workspace
// layout, the line-search driver, the request server and its arena) can be
// built with the address and undefined-behaviour sanitizers and run without a
// GPU.  "Device" memory is host memory here; copies are memcpy; launches do
// nothing.  A failure can be injected into the n-th event creation.
#include <stdlib.h>
#include <string.h>

#include "../../paper_2505_04328_amd/csrc/fb_launch.hpp"
#include "../../paper_2505_04328_amd/csrc/jd_host.hpp"

int g_fail_event_at = -1;  // 0-based index of the event creation that fails
int g_events_created = 0;
int g_launches = 0;

extern "C" {
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
    memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    *s = (hipStream_t)malloc(16);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    free((void*)s);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    if (g_events_created++ == g_fail_event_at)
        return hipErrorOutOfMemory;
    *e = (hipEvent_t)malloc(16);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    free((void*)e);
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = calloc(1, n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
    free(p);
    return hipSuccess;
}
}

namespace jd {
static hipError_t launched() {
    ++g_launches;
    return hipSuccess;
}
hipError_t launch_setup(const HostProblem&, const HostRun&, const double*, void*, WsHeader*, int,
                        hipStream_t, Gate) { return launched(); }
hipError_t launch_forward(const HostProblem&, const HostRun&, const void*, void*, int, double*,
                          const WsHeader*, hipStream_t, Gate, const void*) { return launched(); }
hipError_t launch_setup_noise(const HostProblem&, const HostRun&, const double*, void*, void*,
                              WsHeader*, int, hipStream_t, Gate) { return launched(); }
hipError_t launch_adjoint(const HostProblem&, const HostRun&, const void*, const void*, double*,
                          void*, const WsHeader*, hipStream_t, Gate) { return launched(); }
hipError_t launch_cost_grad_stored(const HostProblem&, const HostRun&, const void*, void*, double*,
                                   double*, const WsHeader*, hipStream_t, Gate, const void*) {
    return launched();
}
hipError_t launch_finalize_grad(const HostProblem&, const HostRun&, const double*, const double*,
                                double*, WsHeader*, hipStream_t, Gate) { return launched(); }
hipError_t launch_finalize_cost(const HostProblem&, const HostRun&, const double*, const double*,
                                const double*, double*, WsHeader*, int, hipStream_t, Gate,
                                const LsTail*) {
    return launched();
}
hipError_t launch_setup_trial(const HostProblem&, const HostRun&, const double*, const double*,
                              double, double*, void*, WsHeader*, hipStream_t, Gate) {
    return launched();
}
hipError_t launch_trial(const double*, const double*, double, double*, int, hipStream_t, Gate) {
    return launched();
}
hipError_t launch_ls_start(WsHeader*, hipStream_t) { return launched(); }
hipError_t launch_ls_after_grad(WsHeader*, int, hipStream_t) { return launched(); }
hipError_t launch_armijo(WsHeader*, LsLog*, double*, const double*, int, const LsArmijo&,
                         hipStream_t) { return launched(); }
hipError_t launch_draws(const HostProblem&, const HostRun&, int64_t, int64_t, int, int, void*, void*,
                        int32_t*, hipStream_t) { return launched(); }
hipError_t launch_philox(uint64_t, const uint32_t*, int64_t, uint32_t*, hipStream_t) {
    return launched();
}
hipError_t launch_clear_flag(WsHeader*, hipStream_t) { return launched(); }
hipError_t fb_launch_table(const FbHost&, const HostRun&, const double*, void*, WsHeader*, int,
                           hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_forward(const FbHost&, const HostRun&, const void*, void*, double*,
                             const WsHeader*, hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_adjoint(const FbHost&, const HostRun&, const void*, const void*, double*,
                             const WsHeader*, bool, hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_forward_grad(const FbHost&, const HostRun&, const void*, double*, double*,
                                  double*, const WsHeader*, hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_surrogate_sd(const FbHost&, const HostRun&, const double*, double*, void*,
                                  hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_finalize_grad(const FbHost&, const HostRun&, const double*, double*, WsHeader*,
                                   hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_finalize_cost(const FbHost&, const HostRun&, const double*, int, const double*,
                                   double*, WsHeader*, int, hipStream_t, Gate) { return launched(); }
hipError_t fb_launch_draws(const FbHost&, const HostRun&, int64_t, int64_t, int, int, void*, void*,
                           int32_t*, hipStream_t) { return launched(); }
}  // namespace jd
