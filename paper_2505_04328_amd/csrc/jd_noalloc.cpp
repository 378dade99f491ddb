// jd_cost_grad without a caller workspace, for callers that cannot allocate
// device memory: the workspace (the per-step table, the per-block partial sums,
// the header) lives in a file-scope device array of kNoAllocBytes that every
// GPU the library runs on holds until the process ends.  The kernels and their
// order are jd_cost_grad's; only the workspace pointer differs.
#include <mutex>

#include "jd_host.hpp"

using namespace jd;
using namespace jd::host;

namespace {

// Largest workspace served from the static array: the 1-D workloads of up to
// 2^20 paths and 1000 steps (33 MB) fit; larger ones are refused.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// The static workspace.  In host code `scratch` names a host-side stand-in,
// not the device array: host code uses only the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// The current device's address of `scratch`, looked up once per device with
// that device current.
int scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return JD_EHIP;
    std::call_once(g_once[dev], [dev] {
        void* ptr = nullptr;
        g_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? ptr : nullptr;
    });
    if (g_err[dev] != hipSuccess || g_ptr[dev] == nullptr)
        return JD_EHIP;
    *out = g_ptr[dev];
    return JD_OK;
}

}  // namespace

extern "C" {

size_t jd_noalloc_capacity(void) { return kNoAllocBytes; }

int jd_cost_grad_noalloc(const jd_problem* prob, const jd_run* run, const double* u, double* J,
                         double* grad, void* traj, hipStream_t stream) {
    HostProblem p;
    HostRun r;
    int rc = prepare(prob, run, p, r);
    if (rc)
        return rc;
    if (!u || !J || !grad || !traj || !aligned(traj, real_size(r.prec)))
        return JD_EINVAL;
    // the array is 256-byte aligned, so the layout needs no alignment slack;
    // a noise table chosen by JD_NOISE_AUTO gives way to inline draws
    if (layout(p, r).total - kAlign > kNoAllocBytes && r.noise && run->noise == JD_NOISE_AUTO)
        r.noise = false;
    if (layout(p, r).total - kAlign > kNoAllocBytes)
        return JD_EWORKSPACE;
    void* ws = nullptr;
    if ((rc = scratch_ptr(&ws)))
        return rc;
    Ws w;
    if ((rc = bind_ws(p, r, ws, kNoAllocBytes + kAlign, w)))
        return rc;
    return enqueue_cost_grad(p, r, u, J, grad, traj, w, stream);
}

}  // extern "C"
