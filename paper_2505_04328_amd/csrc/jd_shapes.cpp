// Host-side sizing of the launches: element sizes, which recompute kernel a
// checkpoint interval takes and its scratch, and the feedback model's table
// layout and block counts.  Plain host code (no kernels), shared by the entry
// points and the launchers.
#include "fb_launch.hpp"
#include "jd_launch.hpp"

namespace jd {

size_t real_size(int prec) { return prec == JD_FP64 ? sizeof(double) : sizeof(float); }

template <typename Real, int D>
static int max_K() { return RecomputeShape<Real, D>::R * RecomputeShape<Real, D>::S; }

template <typename Real, int D>
static int reg_R() { return RecomputeShape<Real, D>::R; }

// Longest checkpoint interval of the register kernel, and the longest it
// sweeps with one regeneration of each step (K <= R: one sub-segment).
static int register_max_K(int prec, int D) {
    if (prec == JD_FP64)
        return D == 1 ? max_K<double, 1>() : D == 2 ? max_K<double, 2>()
             : D == 4 ? max_K<double, 4>() : max_K<double, 8>();
    return D == 1 ? max_K<float, 1>() : D == 2 ? max_K<float, 2>()
         : D == 4 ? max_K<float, 4>() : max_K<float, 8>();
}
static int register_single_K(int prec, int D) {
    if (prec == JD_FP64)
        return D == 1 ? reg_R<double, 1>() : D == 2 ? reg_R<double, 2>()
             : D == 4 ? reg_R<double, 4>() : reg_R<double, 8>();
    return D == 1 ? reg_R<float, 1>() : D == 2 ? reg_R<float, 2>()
         : D == 4 ? reg_R<float, 4>() : reg_R<float, 8>();
}

// The segment kernel (one regeneration, workspace scratch) where the register
// kernel would regenerate every step twice at d = 8, and wherever K exceeds
// the register kernel's buffers.  At d <= 4 a second regeneration costs less
// than writing and reading back the states.
bool recompute_uses_segments(int prec, int D, int K) {
    return K > register_max_K(prec, D) || (D == 8 && K > register_single_K(prec, D));
}

size_t seg_scratch_bytes(const HostProblem& p, const HostRun& r) {
    if (r.mode != JD_RECOMPUTE || !recompute_uses_segments(r.prec, p.D, r.K))
        return 0;
    return (size_t)seg_blocks(r) * (size_t)r.K * (size_t)p.d * kBlock * real_size(r.prec);
}

bool recompute_supported(const HostProblem& p, const HostRun& r) {
    return r.K >= 1 && seg_scratch_bytes(p, r) <= kSegScratchMax;
}

// ---------------------------------------------------------------------------
// The feedback model.

FbTable fb_table_layout(const FbHost& p) {
    FbTable t;
    auto up = [](size_t x) { return (x + 63) / 64 * 64; };
    t.mu = 0;
    t.zd = up((size_t)p.N * p.nx * p.nvp);
    t.ks = t.zd + up((size_t)(p.N + 1) * 2);
    t.sd = t.ks + 64;
    t.count = t.sd + up((size_t)(p.N + 1) * 2);
    return t;
}

size_t fb_mom_count(const FbHost& p, const HostRun& r) {
    return (size_t)(p.N + 1) * (size_t)fb_partial_blocks(p, r) * 4;
}

size_t fb_svar_count(const FbHost& p) { return (size_t)(p.N + 1) * 2 + 4; }

int fb_ring_groups(int np) { return np <= kBlock ? 1 : 8; }

int fb_forward_blocks(const FbHost& p, const HostRun& r) {
    return p.np == 1 ? r.nblk : r.nblk / p.G;
}

// Several groups per block divide the per-step gradient partials but cost
// registers.  Measured on 2^20 x 500: FP64 paths 31.1 / 28.9 ms for 1 / 2
// groups (16.2 / 15.5 / 18.3 ms for 1 / 2 / 4 on FP32 paths while these used
// the FP64 matrix cores); FP32 paths on the FP32 matrix cores with velocity
// transposes of the compiled row width fit five waves per SIMD with one group:
// 10.8 ms against 11.3 ms for two (four waves) and 11.0 ms for two forced to
// five waves (spills).  Rings keep their own G (whole rings per block); the
// jump-adapted adjoint runs one group.
int fb_adjoint_groups(const FbHost& p, const HostRun& r) {
    if (p.np > 1)
        return p.G;
    return p.grid == 0 && r.prec == JD_FP64 && r.nblk >= 2048 ? 2 : 1;
}

int fb_partial_blocks(const FbHost& p, const HostRun& r) {
    const int G = fb_adjoint_groups(p, r);
    return (r.nblk + G - 1) / G;
}

}  // namespace jd
