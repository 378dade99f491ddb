#!/usr/bin/env python3
"""Benchmark of the hot path: forward + adjoint path-steps per second.

One step = one jd_cost_grad call (forward Euler-Maruyama sweep with in-register
Philox draws, backward adjoint sweep, FP64 Monte Carlo reductions of J and g)
over the whole workload, with every input already resident in HBM.

Workload (the configuration the metric is quoted on): the 1-D controlled OU
jump-diffusion with M = 2^20 paths, N = 1000 steps, lambda = 5, jump sizes
N(-0.1, 0.3^2), FP32 path arithmetic with FP64 reductions, stored trajectory.
Also measured: the checkpoint-every-32-steps recompute variant and the pure
FP64 GPU form, p50/p99 per call, per-kernel times (HIP events on the stream the
library launches on), errors against the FP64 oracle on a bounded sample, and
the oracle's own throughput on the host cores.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU peak: MI355X FP32 vector 157.3 TFLOP/s counts a fused multiply-add as
# two flops, i.e. 78.6e12 full-rate 32-bit lane operations per second
# (256 CUs x 4 SIMDs x 32 lanes/clk x 2.4 GHz).  One "slot" is one such
# operation; transcendentals (log2, sqrt, sin, cos) and 32x32->64-bit integer
# products are quarter rate (4 slots), FP64 adds and converts half rate (2).
VALU_PEAK_SLOTS = 256 * 4 * 32 * 2.4e9
# Algorithmic slots per path-step of the forward sweep (d = 1, FP32): the work
# the method needs when counter words 1-3 and the key are wave-uniform.  The
# path index enters Philox only through counter word 0, so the products of the
# first Philox round and the second product of the second are per path (hoisted
# out of the step loop), and the first products of the second and third Philox
# rounds are uniform or per path:
#   Philox4x32-10 block: 15 lane-varying 32x32->64 products (60) + 17 xor3 (17)  = 77
#   Box-Muller cosine half: 2 uniforms (8), log2 (4), scale (1), sqrt (4),
#                           cos (4), product (1)                                 = 22
#   Poisson word (2 byte permutes + or = 3) and the first threshold compare (1)  =  4
#   Euler step: A X + B u, dt and noise terms (c2's drift has no cubic term;
#   one adds X^2, X^3 and its product: 3)                                        =  3
#   running cost: difference, square, FP64 convert (2) and accumulate (2)       =  6
# The jump term (sine half of Box-Muller, sqrt(n), scaling: ~15 slots) is
# needed only in lanes that jump, lambda*dt = 0.005 of them (0.08 slots).
FWD_SLOTS_PER_PATH_STEP = 112
# Backward step per path-step: X - x_d, the drift transpose, dt (1), the masked
# deposit into the reduction tile (1), and the amortised FP64 tile reduction
# (16 converts + adds per 16 steps, 4 slots); a cubic term would add 3 products
# and an FMA (4)
ADJ_SLOTS_PER_PATH_STEP = 8
# The paper's model problem (include/jd_feedback.h, f4: 2^20 particles, 500
# steps, nx = nv = 10 shape functions), algorithmic slots per particle-step:
# forward  20 bumps (scaled distance eps x - i eps dx, 1 - q^2, clamp,
#          reciprocal 4, scale, exp2 4 = 12 each) 240, control
#          sum_i b_x,i sum_l mu_il b_v,l 110, Philox 77 + Poisson 4,
#          Box-Muller both halves 27, Euler 6, FP64 cost (control and
#          tracking terms, one exp) 18                                    = 482
# adjoint  20 bumps with derivatives (3 more products each: 15) 300, control,
#          u_x and u_v (two dot products per row, the derivative's -2 eps
#          once per sum) 232, gradient weight, adjoint update and the
#          tracking gradient (one exp) 24                                 = 556
#          (the jump count is read from the trajectory, one byte the forward
#          stored; regenerating it, as the surrogate adjoint does, adds
#          Philox 77 + Poisson 4                                          = 637)
# plus, on the matrix cores, 2 nx nv = 200 flops per particle-step for the
# gradient's outer products.
# d = 8 (c3, c4; FP32 paths), algorithmic slots per path-step:
# forward  four Philox blocks 308, eight Box-Muller cosine halves 176, the
#          8 x 8 drift product and per-component Euler terms 80 (c4's cubic
#          term adds 3 per component: 104), Poisson 4, running cost 20      = 588 (c4: 612)
# adjoint  per component: X - x_d (1), the A^T lam row (8), the dt update
#          (1) = 10 (c4's cubic term: 3 more), times 8 = 80 (104); the FP64
#          step reduction, per component a convert and an FP64 add (2 + 2) =  32
#                                                                         = 112 (c4: 136)
# The checkpoint-recompute adjoint regenerates each step once more without
# its cost (568, c4: 592).  HBM: the stored trajectory costs 4 d = 32 B per
# path-step written and read back.
def d8_slots(cubic: bool):
    """(forward, adjoint, regenerated step) slots per path-step at d = 8."""
    fwd, adj = (612, 136) if cubic else (588, 112)
    return fwd, adj, fwd - 20


FB_FWD_SLOTS = 482
FB_ADJ_SLOTS = 556
# Coupled rings (Section 6.4, ring2: 512 rings of 2000 particles, 500 steps):
# the forward adds the ring force omega (2x - x_l - x_r) (4 slots) and the
# ellipse cost q = x^2/ax^2 + v^2/av^2 - 1, q^2 (2 more than the tracking
# cost); the adjoint adds -2 omega to u_x - eta (1), the neighbours' dt omega
# (w_l + w_r) (2) and the ellipse gradient (3 more than the tracking one).  The
# neighbour exchange itself is LDS traffic and barriers, not VALU work.
RING_FWD_SLOTS = 488
RING_ADJ_SLOTS = 562
# Jump-adapted grid (ja2 / ja3): the fixed-grid work per particle-step plus,
# per jump (sigma dt of them per particle-step), one more sub-step: forward
# control 350, Euler 6, the sub-step's Philox block and Box-Muller 104, its
# offset (a quarter Philox block and one root, 28), running cost 18 = 506;
# adjoint: the sub-step's adjoint without the count's Philox (556) and its
# offset (28) = 584.  Recomputing the sub-step's start state and the lanes
# that wait on a jumping lane in their wave are not algorithmic work.
ADAPT_FWD_EXTRA = 506
ADAPT_ADJ_EXTRA = 584
HBM_PEAK = 8.0e12  # B/s
METRIC = "forward+adjoint path-steps/s (FP32 vs FP64 GPU) at 1e-6 rel grad err; p50/p99"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-feedback", action="store_true",
                    help="skip the paper's model problem (feedback control) section")
    ap.add_argument("--fb-sample-paths", type=int, default=1 << 15)
    ap.add_argument("--no-ring", action="store_true",
                    help="skip the coupled-rings section (Section 6.4)")
    ap.add_argument("--ring-sample-rings", type=int, default=16)
    ap.add_argument("--no-adapted", action="store_true",
                    help="skip the jump-adapted grid section (Section 3)")
    ap.add_argument("--cpu-sample-paths", type=int, default=1 << 20)
    ap.add_argument("--only", choices=["all", "fp32_store", "kernels", "d8-kernels", "fb-kernels",
                                       "ja-kernels", "fp64-kernels", "c1"],
                    default="all",
                    help="kernels: c2's jd_cost_grad, jd_forward and jd_adjoint only; d8-kernels: "
                         "c3's FP32 stored and K = 64 recompute forward and adjoint only; "
                         "fb-kernels: the f4 FP32 gradient only; ja-kernels: the ja2 and ja3 "
                         "FP32 gradients only; fp64-kernels: the FP64 gradients of c2, c3 (stored), "
                         "f4 and ja2 only; c1: c1's 20 FP64 gradient iterations, noise table "
                         "then inline draws, one run each (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--serving", action="store_true",
                    help="instead: the request-server mix (Poisson arrivals, d in {1,2,4,8})")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration section (c1, c2 iterations, c3, c4)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the request-server mix in the default run")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-m-hi", type=int, default=1 << 20)
    ap.add_argument("--serving-n-hi", type=int, default=2000)
    ap.add_argument("--serving-iters", type=int, default=30)
    ap.add_argument("--serving-moderate-requests", type=int, default=48,
                    help="requests of the second, below-capacity mix (0: skip it)")
    ap.add_argument("--serving-moderate-rate", type=float, default=3.0,
                    help="arrival rate of the below-capacity mix (requests/s)")
    ap.add_argument("--arena-gb", type=float, default=160.0)
    return ap.parse_args()


def serving_main(args):
    """Request mix alone: Poisson arrivals at 50/s, d in {1,2,4,8}, M uniform in
    [2^14, M_hi], N uniform in [100, N_hi], rate in [0, 10], 30 iterations each,
    served by the request server from one device arena (admission by footprint,
    stored trajectory when it takes at most 1/16 of the arena, else checkpoint
    recompute)."""
    sv = serving_section(args)
    line = {
        "metric": "serving: request latency p50/p99 and aggregate forward+adjoint path-steps/s",
        "value": sv["gradient_path_steps_per_s"], "unit": "path-steps/s", "n_gpus": 1,
        "higher_is_better": True, "config": {"workload": sv["workload"]}, "serving": sv,
    }
    print(json.dumps(line), flush=True)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("jd_device.hpp", "jd_kernels.hip", "jd_launch.hpp"):
        with open(os.path.join(ROOT, "paper_2505_04328_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy), if it was
    taken from the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "c2_sweeps_fp32_store.md")
    try:
        with open(path) as fh:
            for ln in fh:
                if ln.strip().startswith("TRAFFIC "):
                    rec = json.loads(ln.strip()[len("TRAFFIC "):])
                    if rec.get("src") == kernel_source_hash():
                        return rec["bytes_per_launch"].get(kernel)
    except OSError:
        pass
    return None


def fb_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("fb_kernels.hip", "fb_launch.hpp", "jd_device.hpp"):
        with open(os.path.join(ROOT, "paper_2505_04328_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


FP64_FLOP_PEAK = 78.6e12  # published FP64 vector peak, FLOP/s


def fp64_counted(kernel: str, units: float, seconds: float):
    """Issue-rate record of an FP64 kernel from the committed counter summary
    (counted slots per unit and FP64 flops per unit), if it was taken from the
    current kernel sources; else None.  frac: counted slots against the slot
    peak; fp64_flop_frac: FP64 flops against the FP64 vector peak."""
    path = os.path.join(ROOT, "profiles", "fp64_kernels_sq_counters.md")
    try:
        with open(path) as fh:
            for ln in fh:
                if ln.strip().startswith("FP64COUNTS "):
                    rec = json.loads(ln.strip()[len("FP64COUNTS "):])
                    src = rec["src_fb"] if "k_fb" in kernel else rec["src_jd"]
                    cur = fb_source_hash() if "k_fb" in kernel else kernel_source_hash()
                    c = rec["per_unit"].get(kernel)
                    if c is None or src != cur:
                        return None
                    return {"kernel": kernel, "bound": "alu", "basis": "counted instructions",
                            "counted_slots_per_unit": c["slots"],
                            "frac": c["slots"] * units / seconds / VALU_PEAK_SLOTS,
                            "fp64_tflops": c["fp64_flops"] * units / seconds / 1e12,
                            "fp64_flop_frac": c["fp64_flops"] * units / seconds / FP64_FLOP_PEAK,
                            "kernel_ms": seconds * 1e3}
    except OSError:
        pass
    return None


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def composite_roofline(phases, units, seconds):
    """The composite roofline of a sequence of kernels: each phase (slots,
    bytes) per unit bounded by the larger of its VALU time and its HBM time,
    summed; frac = that time over the measured one."""
    t_roof = sum(max(sl * units / VALU_PEAK_SLOTS, by * units / HBM_PEAK) for sl, by in phases)
    return {"t_roof_ms": t_roof * 1e3, "t_ms": seconds * 1e3, "frac": t_roof / seconds,
            "phases_slots_bytes_per_unit": [list(ph) for ph in phases]}


def configs_section(args, time_calls, dev):
    """Every benchmark configuration: c1 (20 FP64 gradient iterations), c2 (50
    iterations, stored vs checkpoint-recompute K = 32), c3 (d = 8; stored and
    K = 64, FP32 and FP64), c4 (the K = 64 forward + backward step of the
    autograd function J(u)), each against its composite roofline."""
    import torch
    from paper_2505_04328_amd import binding as B
    from paper_2505_04328_amd import workloads as wl
    from paper_2505_04328_amd.autograd import jd_cost
    out = {}

    def sync_wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    # c1: 10^4 paths x 100 steps, FP64, 20 iterations from u = 0; the draws
    # from the iteration's noise table (the automatic choice at this size) and
    # computed in the sweeps, which give bitwise the same iterates
    w = wl.config("c1")
    p = w.problem
    c1 = {}
    for noise in ("table", "inline"):
        e = B.Engine(p, M=w.M, seed=w.seed, precision="fp64", device=dev, noise=noise)
        e.optimize(torch.zeros((p.N, 1), dtype=torch.float64, device=dev), n_max=2)  # warm
        walls = []
        for _ in range(3):
            u = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
            wall, (_, logs) = sync_wall(lambda: e.optimize(u, n_max=w.iters))
            walls.append(wall)
        c1[noise] = (min(walls), logs, u.cpu().numpy())
        del e
    wall, logs, u_tab = c1["table"]
    trials = sum(1 + l["backtracks"] for l in logs)
    out["c1"] = {"form": "FP64, 20 gradient iterations (jd_optimize, line search on the device), "
                         "draws from the per-iteration noise table",
                 "wall_s_best_of_3": wall, "ms_per_iteration": wall / w.iters * 1e3,
                 "wall_s_inline_draws_best_of_3": c1["inline"][0],
                 "inline_bitwise_equal": bool(logs == c1["inline"][1]
                                              and np.array_equal(u_tab, c1["inline"][2])),
                 "iterations": len(logs), "trials": trials, "J_first": logs[0]["J"],
                 "J_last_new": logs[-1]["J_new"],
                 "note": "10^4 paths = 40 blocks of 256: launch- and latency-bound, no roofline"}
    log(f"c1: {wall * 1e3:.2f} ms for {w.iters} iterations "
        f"({c1['inline'][0] * 1e3:.2f} ms with the draws in the sweeps)")

    # c2: 50 iterations, stored and K = 32 (bitwise the same iterates)
    w = wl.config("c2")
    p = w.problem
    res = {}
    finals = {}
    for mode, K in (("store", 0), ("recompute", w.K)):
        e = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode=mode, K=K, device=dev)
        e.optimize(torch.zeros((p.N, 1), dtype=torch.float64, device=dev), n_max=1)  # warm
        walls = []
        for _ in range(3):  # best of 3, each from u = 0 (the same iterates every time)
            u = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
            wall, (_, logs) = sync_wall(lambda: e.optimize(u, n_max=w.iters))
            walls.append(wall)
        wall = min(walls)
        trials = sum(1 + l["backtracks"] for l in logs)
        finals[mode] = u.cpu().numpy()
        # swept path-steps: each iteration's forward + adjoint and every trial's forward
        res[f"{mode}{'_K' + str(K) if K else ''}"] = {
            "wall_s_best_of_3": wall, "iterations": len(logs), "trials": trials,
            "ms_per_iteration": wall / len(logs) * 1e3,
            "gradient_path_steps_per_s": len(logs) * w.M * p.N / wall,
            "J_first": logs[0]["J"], "J_last_new": logs[-1]["J_new"]}
        log(f"c2 {mode}: 50 iterations in {wall:.3f} s ({trials} trials)")
        del e
        torch.cuda.empty_cache()
    res["final_u_bitwise_equal"] = bool(np.array_equal(finals["store"], finals["recompute"]))
    out["c2_iterations"] = res

    # c3 (and c4's stored/FP64 forms): jd_cost_grad per call
    for name in ("c3", "c4"):
        w = wl.config(name)
        p = w.problem
        MN = w.M * p.N
        u = torch.zeros((p.N, p.d), dtype=torch.float64, device=dev)
        res = {}
        for prec, mode, K in (("fp32", "store", 0), ("fp32", "recompute", 64), ("fp64", "store", 0),
                              ("fp64", "recompute", 64)):
            e = B.Engine(p, M=w.M, seed=w.seed, precision=prec, mode=mode, K=K, device=dev)
            e.cost_grad(u, it=1)
            reps = 10 if prec == "fp32" else 4
            t = time_calls(lambda: e.cost_grad(u, it=1), reps)
            tf = time_calls(lambda: e.forward(u, it=1), reps)
            ta = time_calls(lambda: e.adjoint(u, it=1), reps)
            key = f"{prec}_{mode}{'_K' + str(K) if K else ''}"
            rec = {"p50_ms": percentile(t, 50), "p99_ms": percentile(t, 99),
                   "forward_ms": percentile(tf, 50), "adjoint_ms": percentile(ta, 50),
                   "path_steps_per_s": MN / (percentile(t, 50) * 1e-3)}
            if prec == "fp32":
                f8, a8, r8 = d8_slots(p.cubic != 0.0)
                if mode == "store":
                    ph = [(f8, 32), (a8, 32)]
                else:
                    ph = [(f8, 32.0 / K), (r8 + a8, 32.0 / K)]
                rec["roofline"] = composite_roofline(ph, MN, percentile(t, 50) * 1e-3)
            elif mode == "store":
                if name == "c3":  # counted on c3's linear drift
                    rec["forward_issue"] = fp64_counted("jd::k_forward<double, 8, 1, false, false>", MN,
                                                        percentile(tf, 50) * 1e-3)
                # the stored adjoint reads z_k (8 FP64) per path-step: HBM-bound
                ta_s = percentile(ta, 50) * 1e-3
                rec["adjoint_roofline"] = {"kernel": "k_adjoint_stored<double,8>", "bound": "hbm",
                                           "achieved": 64.0 * MN / ta_s / 1e9, "peak": 8000.0,
                                           "unit": "GB/s", "frac": 64.0 * MN / ta_s / 8e12}
            res[key] = rec
            log(f"{name} {key}: {rec['p50_ms']:.2f} ms")
            del e
            torch.cuda.empty_cache()
        res["speedup_fp32_over_fp64_store"] = res["fp64_store"]["p50_ms"] / res["fp32_store"]["p50_ms"]
        out[name] = res

    # c4: the autograd step J(u).backward() with checkpoints every 64 steps
    w = wl.config("c4")
    p = w.problem
    e = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="recompute", K=w.K, device=dev)
    u0 = torch.tensor(wl.random_control(p, 3, 0.3), dtype=torch.float64, device=dev)

    def step():
        u = u0.clone().requires_grad_(True)
        J = jd_cost(u, e, 0)
        J.backward()
        return u.grad

    step()
    t = time_calls(step, 10)
    MN = w.M * p.N
    out["c4_autograd_step"] = {
        "form": "FP32 paths, checkpoints every 64 steps: jd_forward + jd_adjoint (recompute)",
        "p50_ms": percentile(t, 50), "p99_ms": percentile(t, 99),
        "path_steps_per_s": MN / (percentile(t, 50) * 1e-3),
        "roofline": composite_roofline([(d8_slots(True)[0], 32.0 / w.K),
                                        (d8_slots(True)[2] + d8_slots(True)[1], 32.0 / w.K)], MN,
                                       percentile(t, 50) * 1e-3)}
    log(f"c4 autograd step: {percentile(t, 50):.2f} ms")
    del e
    torch.cuda.empty_cache()
    return out


def serving_run(args, count: int, rate: float):
    """One request mix through a fresh server: Poisson arrivals at `rate`,
    d in {1,2,4,8}, M uniform in [2^14, M_hi], N uniform in [100, N_hi], rate
    in [0, 10], the set number of iterations each (see serving_main)."""
    from paper_2505_04328_amd import serving as S
    from paper_2505_04328_amd import workloads as wl
    reqs = wl.serving_requests(count=count, rate=rate, seed=11, M_hi=args.serving_m_hi,
                               N_hi=args.serving_n_hi, iters=args.serving_iters)
    arena = int(args.arena_gb * (1 << 30))
    srv = S.Server(arena, max_active=32, n_streams=4)
    t_last = [time.perf_counter()]

    def on_done(rec):
        if time.perf_counter() - t_last[0] > 5:
            log(f"  request {rec.rid} done, latency {rec.latency:.2f} s")
            t_last[0] = time.perf_counter()

    log(f"serving {len(reqs)} requests at {rate}/s, arena {args.arena_gb} GB")
    recs, wall = S.run_mix(srv, reqs, precision="fp32", store_limit=arena // 16, on_done=on_done)
    srv.close()
    lat = np.array([r.latency for r in recs])
    ps = sum(r.path_steps for r in recs)
    sw = sum(r.swept for r in recs)
    return {
        "requests": len(recs), "wall_s": wall, "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        # the server's own split of each latency: waiting for a slot and arena
        # memory, then running on the device among the admitted requests
        "queued_p50_s": float(np.percentile([r.queued for r in recs], 50)),
        "queued_p99_s": float(np.percentile([r.queued for r in recs], 99)),
        "service_p50_s": float(np.percentile([r.service for r in recs], 50)),
        "service_p99_s": float(np.percentile([r.service for r in recs], 99)),
        "gradient_path_steps_per_s": ps / wall, "swept_path_steps_per_s": sw / wall,
        "failed": int(sum(r.status != 0 for r in recs)),
        "peak_admitted": srv.stats["max_active"], "peak_queued": srv.stats["max_queued"],
        "workload": f"{len(recs)} requests, Poisson {rate}/s, d in {{1,2,4,8}}, "
                    f"M in [2^14, {args.serving_m_hi}], N in [100, {args.serving_n_hi}], "
                    f"lambda in [0,10], {args.serving_iters} iterations, FP32 paths, arena "
                    f"{args.arena_gb} GB, 32 slots over 4 streams"}


def serving_section(args):
    """The c5 request mix (Poisson 50/s, about 12 times what the device
    serves, so its latency is mostly the admission queue), then a smaller mix
    below capacity, whose latency is the service time of requests sharing
    the device."""
    out = serving_run(args, args.serving_requests, 50.0)
    out["workload"] = "c5 mix: " + out["workload"]
    if args.serving_moderate_requests > 0:
        out["below_capacity"] = serving_run(args, args.serving_moderate_requests,
                                            args.serving_moderate_rate)
    return out


def feedback_section(args, time_calls, dev):
    """The paper's own model problem (RBF feedback control, Keilson-Storer
    jumps) at 2^20 particles x 500 steps: per-call times of jd_fb_cost_grad
    (FP32 and FP64 paths), the forward and adjoint kernels alone, the slot
    roofline, and the oracle on a bounded sample."""
    import torch
    from paper_2505_04328_amd import binding as B
    from paper_2505_04328_amd import workloads as wl
    w = wl.feedback_config("f4")
    p = w.problem
    mu = torch.tensor(wl.random_feedback_control(p, 4, 0.5), device=dev)
    out = {"workload": "f4: paper's model problem (Section 5/6), 2^20 particles, 500 steps, "
                       "10 x 10 bump shape functions, Keilson-Storer jumps beta 10 gamma 0.9",
           "M": w.M, "N": p.N, "L": p.L}
    ps = w.M * p.N
    res = {}
    for prec in ("fp32", "fp64"):
        e = B.FbEngine(p, M=w.M, seed=w.seed, precision=prec, device=dev)
        for it in range(args.warmup):
            e.cost_grad(mu, it=it)
        cg = time_calls(lambda: e.cost_grad(mu, it=5), args.steps)
        fw = time_calls(lambda: e.forward(mu, it=5), max(5, args.steps // 2))
        ad = time_calls(lambda: e.adjoint(mu, it=5), max(5, args.steps // 2))
        J, g = e.cost_grad(mu, it=0)
        res[prec] = (float(J), g.cpu().numpy())
        out[prec] = {"p50_ms": percentile(cg, 50), "p99_ms": percentile(cg, 99),
                     "path_steps_per_s_p50": ps / (percentile(cg, 50) * 1e-3),
                     "forward_ms": float(np.mean(fw)), "adjoint_ms": float(np.mean(ad))}
        if prec == "fp64":
            out[prec]["forward_issue"] = fp64_counted(
                "jd::k_fb_forward<double, 10, true, 1, false, 256>", ps, float(np.mean(fw)) * 1e-3)
            out[prec]["adjoint_issue"] = fp64_counted(
                "jd::k_fb_adjoint<double, 10, 2, false, false, 256>", ps, float(np.mean(ad)) * 1e-3)
        del e
        torch.cuda.empty_cache()
    # the storage-free surrogate gradient (Section 6.5): no trajectory buffer
    es = B.FbEngine(p, M=w.M, seed=w.seed, precision="fp32", device=dev, mode="surrogate")
    for it in range(args.warmup):
        es.cost_grad(mu, it=it)
    sg = time_calls(lambda: es.cost_grad(mu, it=5), args.steps)
    out["fp32_surrogate"] = {"p50_ms": percentile(sg, 50), "p99_ms": percentile(sg, 99),
                             "path_steps_per_s_p50": ps / (percentile(sg, 50) * 1e-3),
                             "trajectory_bytes_saved": (p.N + 1) * 2 * 4 * es.nblk * 256}
    del es
    torch.cuda.empty_cache()
    # the same with the variance fitted to the forward ensemble (per-step
    # moments in the forward, a reduction and the least-squares line between
    # the sweeps)
    pf = dataclasses.replace(p, svar_kind=1)
    es = B.FbEngine(pf, M=w.M, seed=w.seed, precision="fp32", device=dev, mode="surrogate")
    for it in range(args.warmup):
        es.cost_grad(mu, it=it)
    sg = time_calls(lambda: es.cost_grad(mu, it=5), args.steps)
    out["fp32_surrogate_fit"] = {"p50_ms": percentile(sg, 50), "p99_ms": percentile(sg, 99),
                                 "path_steps_per_s_p50": ps / (percentile(sg, 50) * 1e-3)}
    del es
    torch.cuda.empty_cache()
    t_f, t_a = out["fp32"]["forward_ms"] * 1e-3, out["fp32"]["adjoint_ms"] * 1e-3
    t_cg = out["fp32"]["p50_ms"] * 1e-3
    out["roofline"] = {
        "bound": "alu", "kernel": "k_fb_adjoint<float,10,1,false,false,256>",
        "achieved": FB_ADJ_SLOTS * ps / t_a / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
        "unit": "TOP/s (full-rate VALU lane-op slots)",
        "frac": FB_ADJ_SLOTS * ps / t_a / VALU_PEAK_SLOTS, "traffic": None,
        "slots_per_path_step": FB_ADJ_SLOTS, "kernel_ms": t_a * 1e3}
    out["forward_roofline"] = {"kernel": "k_fb_forward<float,10,true,1,false,256>", "bound": "alu",
                               "frac": FB_FWD_SLOTS * ps / t_f / VALU_PEAK_SLOTS,
                               "slots_per_path_step": FB_FWD_SLOTS}
    out["step_frac"] = (FB_FWD_SLOTS + FB_ADJ_SLOTS) * ps / t_cg / VALU_PEAK_SLOTS
    # Section 6.5's comparison at the paper's size and setting (f3: 2000
    # particles, 50 steps, time-dependent target): the gradient iteration from
    # mu = 0 with the exact and with the surrogate gradient (FP64, 40
    # iterations at most, Armijo from zeta0 = 10), both scored on a held-out
    # sample of 2^16 particles with other draws.
    wc = wl.feedback_config("f3")
    pc = wc.problem
    mu0 = torch.zeros((pc.N, pc.L), dtype=torch.float64, device=dev)
    held = B.FbEngine(pc, M=1 << 16, seed=wc.seed + 100, precision="fp64", device=dev)
    J0h, _ = held.cost_grad(mu0, it=0)
    conv = {"workload": "f3 (Section 6.3 / 6.5 setting), FP64", "held_out_J_zero_control": float(J0h)}
    for key, mode, pk in (("exact", "store", pc), ("surrogate", "surrogate", pc),
                          ("surrogate_fitted_variance", "surrogate",
                           dataclasses.replace(pc, svar_kind=1))):
        ec = B.FbEngine(pk, M=wc.M, seed=wc.seed, precision="fp64", device=dev, mode=mode)
        muc, logs = ec.optimize(mu0.clone(), n_max=40, zeta0=10.0, allow_stall=True)
        Jh, _ = held.cost_grad(muc, it=0)
        conv[key] = {"iterations": len(logs), "stalled": len(logs) < 40,
                     "J": [round(l["J"], 6) for l in logs], "held_out_J": float(Jh)}
        del ec
    del held
    out["surrogate_vs_exact_iteration"] = conv
    log(f"surrogate vs exact iteration (f3): exact {conv['exact']['iterations']} it -> held-out "
        f"{conv['exact']['held_out_J']:.4f}, surrogate {conv['surrogate']['iterations']} it -> "
        f"{conv['surrogate']['held_out_J']:.4f}, fitted variance "
        f"{conv['surrogate_fitted_variance']['iterations']} it -> "
        f"{conv['surrogate_fitted_variance']['held_out_J']:.4f}")
    J64, g64 = res["fp64"]
    J32, g32 = res["fp32"]
    out["fp32_vs_fp64_full_size"] = {"J_rel": abs(J32 - J64) / abs(J64),
                                     "g_rel": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
    if not args.no_cpu_baseline:
        from oracle import ref
        Ms = args.fb_sample_paths
        nth = ref.default_threads()
        log(f"feedback oracle: {Ms} particles x {p.N} steps on {nth} threads")
        t0 = time.perf_counter()
        Jo, go = ref.fb_cost_grad(p, Ms, w.seed, 0, mu.cpu().numpy(), nthreads=nth)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": Ms * p.N / tc, "unit": "path-steps/s", "cores": nth,
                               "kind": "oracle",
                               "sample": f"f4 with M={Ms} of {w.M} particles, all {p.N} steps, "
                                         f"forward+adjoint+reductions, FP64, {tc:.1f} s wall"}
        errs = {}
        for prec in ("fp32", "fp64"):
            es = B.FbEngine(p, M=Ms, seed=w.seed, precision=prec, device=dev)
            Js, gs = es.cost_grad(mu, it=0)
            errs[prec] = {"J_rel": abs(float(Js) - Jo) / abs(Jo),
                          "g_rel": float(np.linalg.norm(gs.cpu().numpy() - go) / np.linalg.norm(go))}
            del es
        out["oracle_error_on_sample"] = errs
        log(f"feedback oracle errors: {errs}")
    return out


def adapted_section(args, time_calls, dev):
    """The jump-adapted grid (Section 3, Algorithms 5.1-5.2) at f4's size
    (ja2: 2^20 particles, 500 steps of 0.01) in FP32 and FP64, and at the
    paper's step (ja3: 2^20 particles, 50 steps of 0.1) in FP32: per-call times
    of jd_fb_cost_grad, the forward and adjoint kernels alone, the slot
    roofline, and the oracle on a bounded sample."""
    import torch
    from paper_2505_04328_amd import binding as B
    from paper_2505_04328_amd import workloads as wl
    out = {}
    for name, precs in (("ja2", ("fp32", "fp64")), ("ja3", ("fp32",))):
        w = wl.adapted_config(name)
        p = w.problem
        mu = torch.tensor(wl.random_feedback_control(p, 4, 0.5), device=dev)
        ps = w.M * p.N
        sdt = p.rate * p.dt
        o = {"M": w.M, "N": p.N, "dt": p.dt, "jumps_per_particle_step": sdt}
        res = {}
        for prec in precs:
            e = B.FbEngine(p, M=w.M, seed=w.seed, precision=prec, device=dev)
            for it in range(args.warmup):
                e.cost_grad(mu, it=it)
            cg = time_calls(lambda: e.cost_grad(mu, it=5), args.steps)
            fw = time_calls(lambda: e.forward(mu, it=5), max(5, args.steps // 2))
            ad = time_calls(lambda: e.adjoint(mu, it=5), max(5, args.steps // 2))
            J, g = e.cost_grad(mu, it=0)
            res[prec] = (float(J), g.cpu().numpy())
            o[prec] = {"p50_ms": percentile(cg, 50), "p99_ms": percentile(cg, 99),
                       "particle_steps_per_s_p50": ps / (percentile(cg, 50) * 1e-3),
                       "forward_ms": float(np.mean(fw)), "adjoint_ms": float(np.mean(ad))}
            if prec == "fp64" and name == "ja2":
                o[prec]["forward_issue"] = fp64_counted(
                    "jd::k_fb_forward_adapted<double, 10, true>", ps, float(np.mean(fw)) * 1e-3)
                o[prec]["adjoint_issue"] = fp64_counted(
                    "jd::k_fb_adjoint_adapted<double, 10>", ps, float(np.mean(ad)) * 1e-3)
            del e
            torch.cuda.empty_cache()
        fs = FB_FWD_SLOTS + sdt * ADAPT_FWD_EXTRA
        as_ = FB_ADJ_SLOTS + sdt * ADAPT_ADJ_EXTRA
        t_f, t_a = o["fp32"]["forward_ms"] * 1e-3, o["fp32"]["adjoint_ms"] * 1e-3
        o["roofline"] = {"bound": "alu", "kernel": "k_fb_adjoint_adapted<float,10>",
                         "achieved": as_ * ps / t_a / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                         "unit": "TOP/s (full-rate VALU lane-op slots)",
                         "frac": as_ * ps / t_a / VALU_PEAK_SLOTS, "traffic": None,
                         "slots_per_particle_step": as_, "kernel_ms": t_a * 1e3}
        o["forward_roofline"] = {"kernel": "k_fb_forward_adapted<float,10,true>", "bound": "alu",
                                 "frac": fs * ps / t_f / VALU_PEAK_SLOTS,
                                 "slots_per_particle_step": fs}
        if "fp64" in res:
            J64, g64 = res["fp64"]
            J32, g32 = res["fp32"]
            o["fp32_vs_fp64_full_size"] = {
                "J_rel": abs(J32 - J64) / abs(J64),
                "g_rel": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
        if name == "ja2" and not args.no_cpu_baseline:
            from oracle import ref
            Ms = args.fb_sample_paths
            nth = ref.default_threads()
            log(f"adapted-grid oracle: {Ms} particles x {p.N} steps on {nth} threads")
            t0 = time.perf_counter()
            Jo, go = ref.fb_cost_grad(p, Ms, w.seed, 0, mu.cpu().numpy(), nthreads=nth)
            tc = time.perf_counter() - t0
            o["cpu_baseline"] = {"value": Ms * p.N / tc, "unit": "particle-steps/s",
                                 "cores": min(nth, -(-Ms // 4096)), "kind": "oracle",
                                 "sample": f"ja2 with M={Ms} of {w.M} particles, all {p.N} steps, "
                                           f"forward+adjoint+reductions, FP64, {tc:.1f} s wall"}
            errs = {}
            for prec in ("fp32", "fp64"):
                es = B.FbEngine(p, M=Ms, seed=w.seed, precision=prec, device=dev)
                Js, gs = es.cost_grad(mu, it=0)
                errs[prec] = {"J_rel": abs(float(Js) - Jo) / abs(Jo),
                              "g_rel": float(np.linalg.norm(gs.cpu().numpy() - go) / np.linalg.norm(go))}
                del es
            o["oracle_error_on_sample"] = errs
            log(f"adapted-grid oracle errors: {errs}")
        out[name] = o
    out["workload"] = ("jump-adapted grid (Section 3): ja2 = f4's model and size (2^20 particles, "
                       "500 steps of 0.01) and ja3 = 2^20 particles at the paper's step (50 steps of "
                       "0.1), 10 x 10 bump shape functions, Keilson-Storer jumps beta 10 gamma 0.9")
    return out


def ring_section(args, time_calls, dev):
    """Coupled particles (Section 6.4) at the measured size ring2: 512 rings of
    2000 nearest-neighbour coupled particles, 500 steps, the ellipse cost and
    the start on the ellipse: per-call times of jd_fb_cost_grad (FP32 and FP64
    paths), the forward and adjoint kernels alone, the slot roofline, and the
    oracle on a bounded sample of rings."""
    import torch
    from paper_2505_04328_amd import binding as B
    from paper_2505_04328_amd import workloads as wl
    w = wl.ring_config("ring2")
    p = w.problem
    mu = torch.tensor(wl.random_feedback_control(p, 4, 0.5), device=dev)
    P = w.M * p.np
    out = {"workload": "ring2: coupled particles (Section 6.4), 512 rings of 2000 particles "
                       "(omega 0.5, eta 1), 500 steps, ellipse cost, 10 x 10 bump shape "
                       "functions, Keilson-Storer jumps beta 10 gamma 0.9",
           "rings": w.M, "np": p.np, "particles": P, "N": p.N, "L": p.L}
    ps = P * p.N
    res = {}
    for prec in ("fp32", "fp64"):
        e = B.FbEngine(p, M=w.M, seed=w.seed, precision=prec, device=dev)
        for it in range(args.warmup):
            e.cost_grad(mu, it=it)
        cg = time_calls(lambda: e.cost_grad(mu, it=5), args.steps)
        fw = time_calls(lambda: e.forward(mu, it=5), max(5, args.steps // 2))
        ad = time_calls(lambda: e.adjoint(mu, it=5), max(5, args.steps // 2))
        J, g = e.cost_grad(mu, it=0)
        res[prec] = (float(J), g.cpu().numpy())
        out[prec] = {"p50_ms": percentile(cg, 50), "p99_ms": percentile(cg, 99),
                     "particle_steps_per_s_p50": ps / (percentile(cg, 50) * 1e-3),
                     "forward_ms": float(np.mean(fw)), "adjoint_ms": float(np.mean(ad))}
        del e
        torch.cuda.empty_cache()
    t_f, t_a = out["fp32"]["forward_ms"] * 1e-3, out["fp32"]["adjoint_ms"] * 1e-3
    t_cg = out["fp32"]["p50_ms"] * 1e-3
    out["roofline"] = {
        "bound": "alu", "kernel": "k_fb_adjoint<float,10,2,false,true,1024>",
        "achieved": RING_ADJ_SLOTS * ps / t_a / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
        "unit": "TOP/s (full-rate VALU lane-op slots)",
        "frac": RING_ADJ_SLOTS * ps / t_a / VALU_PEAK_SLOTS, "traffic": None,
        "slots_per_particle_step": RING_ADJ_SLOTS, "kernel_ms": t_a * 1e3}
    out["forward_roofline"] = {"kernel": "k_fb_forward<float,10,true,2,true,1024>", "bound": "alu",
                               "frac": RING_FWD_SLOTS * ps / t_f / VALU_PEAK_SLOTS,
                               "slots_per_particle_step": RING_FWD_SLOTS}
    out["step_frac"] = (RING_FWD_SLOTS + RING_ADJ_SLOTS) * ps / t_cg / VALU_PEAK_SLOTS
    J64, g64 = res["fp64"]
    J32, g32 = res["fp32"]
    out["fp32_vs_fp64_full_size"] = {"J_rel": abs(J32 - J64) / abs(J64),
                                     "g_rel": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
    if not args.no_cpu_baseline:
        from oracle import ref
        Ms = args.ring_sample_rings
        nth = ref.default_threads()
        log(f"ring oracle: {Ms} rings of {p.np} x {p.N} steps on {nth} threads")
        t0 = time.perf_counter()
        Jo, go = ref.fb_cost_grad(p, Ms, w.seed, 0, mu.cpu().numpy(), nthreads=nth)
        tc = time.perf_counter() - t0
        # the oracle splits the rings into chunks of 4096 // np rings, one chunk per thread
        used = min(nth, -(-Ms // max(1, 4096 // p.np)))
        out["cpu_baseline"] = {"value": Ms * p.np * p.N / tc, "unit": "particle-steps/s",
                               "cores": used, "kind": "oracle",
                               "sample": f"ring2 with {Ms} of {w.M} rings ({Ms * p.np} particles), "
                                         f"all {p.N} steps, forward+adjoint+reductions, FP64, "
                                         f"{tc:.1f} s wall"}
        errs = {}
        for prec in ("fp32", "fp64"):
            es = B.FbEngine(p, M=Ms, seed=w.seed, precision=prec, device=dev)
            Js, gs = es.cost_grad(mu, it=0)
            errs[prec] = {"J_rel": abs(float(Js) - Jo) / abs(Jo),
                          "g_rel": float(np.linalg.norm(gs.cpu().numpy() - go) / np.linalg.norm(go))}
            del es
        out["oracle_error_on_sample"] = errs
        log(f"ring oracle errors: {errs}")
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py: runs on one GPU only (the paths shard across GPUs "
                 "by contiguous path ranges, but no multi-GPU path is built); use --gpus 1")
    if args.serving:
        return serving_main(args)
    import torch
    from paper_2505_04328_amd import binding as B
    from paper_2505_04328_amd import workloads as wl

    dev = torch.device("cuda:0")
    if args.only == "fb-kernels":
        # the feedback model's forward and adjoint at f4, FP32, for counter runs
        wf = wl.feedback_config("f4")
        mu = torch.tensor(wl.random_feedback_control(wf.problem, 4, 0.5), device=dev)
        ef = B.FbEngine(wf.problem, M=wf.M, seed=wf.seed, precision="fp32", device=dev)
        for it in range(args.warmup + args.steps):
            ef.cost_grad(mu, it=it)
        torch.cuda.synchronize()
        log("feedback-model kernel loop done")
        print(json.dumps({"fb_kernels_only": True, "calls": args.warmup + args.steps}))
        return
    if args.only == "fp64-kernels":
        # the FP64 sweeps: c2 (fused), c3 stored, f4 and ja2, for counter runs
        for name in ("c2", "c3"):
            wc = wl.config(name)
            uc = torch.zeros((wc.problem.N, wc.problem.d), dtype=torch.float64, device=dev)
            e = B.Engine(wc.problem, M=wc.M, seed=wc.seed, precision="fp64", mode="store",
                         device=dev)
            for it in range(args.warmup + args.steps):
                e.cost_grad(uc, it=it)
            torch.cuda.synchronize()
            del e
            torch.cuda.empty_cache()
        for wf in (wl.feedback_config("f4"), wl.adapted_config("ja2")):
            mu = torch.tensor(wl.random_feedback_control(wf.problem, 4, 0.5), device=dev)
            ef = B.FbEngine(wf.problem, M=wf.M, seed=wf.seed, precision="fp64", device=dev)
            for it in range(args.warmup + args.steps):
                ef.cost_grad(mu, it=it)
            torch.cuda.synchronize()
            del ef
            torch.cuda.empty_cache()
        log("fp64 kernel loop done")
        print(json.dumps({"fp64_kernels_only": True, "calls": args.warmup + args.steps}))
        return
    if args.only == "c1":
        # c1's 20 FP64 gradient iterations from u = 0, once with the noise
        # table and once with the draws in the sweeps, after one warm call each
        w1 = wl.config("c1")
        logs = {}
        for noise in ("table", "inline"):
            e = B.Engine(w1.problem, M=w1.M, seed=w1.seed, precision="fp64", device=dev,
                         noise=noise)
            e.optimize(torch.zeros((w1.problem.N, 1), dtype=torch.float64, device=dev), n_max=2)
            u = torch.zeros((w1.problem.N, 1), dtype=torch.float64, device=dev)
            _, logs[noise] = e.optimize(u, n_max=w1.iters)
            torch.cuda.synchronize()
            del e
            log(f"c1 {noise} done")
        print(json.dumps({"c1_only": True, "iterations": len(logs["table"]),
                          "trials": sum(1 + l["backtracks"] for l in logs["table"]),
                          "inline_same_log": logs["table"] == logs["inline"]}))
        return
    if args.only == "ja-kernels":
        # the jump-adapted forward and adjoint at ja2 and ja3, FP32, for counter runs
        for name in ("ja2", "ja3"):
            wa = wl.adapted_config(name)
            mu = torch.tensor(wl.random_feedback_control(wa.problem, 4, 0.5), device=dev)
            ea = B.FbEngine(wa.problem, M=wa.M, seed=wa.seed, precision="fp32", device=dev)
            for it in range(args.warmup + args.steps):
                ea.cost_grad(mu, it=it)
            torch.cuda.synchronize()
            del ea
            torch.cuda.empty_cache()
            log(f"{name} kernel loop done")
        print(json.dumps({"ja_kernels_only": True, "calls": args.warmup + args.steps}))
        return
    if args.only == "d8-kernels":
        # the d = 8 sweeps at c3, FP32: stored forward and adjoint, then the
        # checkpoint forward and the recompute adjoint (K = 64), for counter runs
        w3 = wl.config("c3")
        u3 = torch.zeros((w3.problem.N, w3.problem.d), dtype=torch.float64, device=dev)
        for mode, K in (("store", 0), ("recompute", 64)):
            e = B.Engine(w3.problem, M=w3.M, seed=w3.seed, precision="fp32", mode=mode, K=K,
                         device=dev)
            for it in range(args.warmup + args.steps):
                e.forward(u3, it=it)
                e.adjoint(u3, it=it)
            torch.cuda.synchronize()
            del e
            torch.cuda.empty_cache()
        log("d = 8 kernel loop done")
        print(json.dumps({"d8_kernels_only": True, "calls": args.warmup + args.steps}))
        return
    w = wl.config("c2")
    p = w.problem
    M, N = w.M, p.N
    u = torch.zeros((N, p.d), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def time_calls(fn, reps):
        """Per-call times (ms) with events on the library's stream."""
        out = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record(st)
            fn()
            b.record(st)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return out

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies done")
        del x, y

    log(f"workload c2: M={M} N={N} d={p.d}; building engines")
    e32 = B.Engine(p, M=M, seed=w.seed, precision="fp32", mode="store", device=dev)

    if args.only == "kernels":
        # the fused step, then forward (store) and adjoint alone, for the profiler
        for it in range(args.warmup + args.steps):
            e32.cost_grad(u, it=it)
            e32.forward(u, it=it)
            e32.adjoint(u, it=it)
        torch.cuda.synchronize()
        log("kernel timing loop done")
        print(json.dumps({"kernels_only": True, "calls": args.warmup + args.steps}))
        return

    # ---- the contract: W warmups, then exactly K timed steps, FP32 stored
    for it in range(args.warmup):
        e32.cost_grad(u, it=it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(args.steps):
        e32.cost_grad(u, it=it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = t1 - t0
    value = M * N * args.steps / total
    log(f"fp32 store: {total / args.steps * 1e3:.3f} ms/step, {value:.4e} path-steps/s")

    res = {}
    res["fp32_store_ms"] = time_calls(lambda: e32.cost_grad(u, it=7), args.steps)
    # per-kernel: jd_forward (table + forward sweep + cost reduction) and
    # jd_adjoint (table + adjoint sweep + gradient reduction)
    fwd_ms = time_calls(lambda: e32.forward(u, it=7), max(5, args.steps // 2))
    adj_ms = time_calls(lambda: e32.adjoint(u, it=7), max(5, args.steps // 2))
    J32, g32 = e32.cost_grad(u, it=0)
    J32, g32 = float(J32), g32.cpu().numpy()
    del e32
    torch.cuda.empty_cache()

    forms = {}
    if args.only == "all":
        er = B.Engine(p, M=M, seed=w.seed, precision="fp32", mode="recompute", K=w.K, device=dev)
        for it in range(args.warmup):
            er.cost_grad(u, it=it)
        res["fp32_recompute_ms"] = time_calls(lambda: er.cost_grad(u, it=7), args.steps)
        Jr, gr = er.cost_grad(u, it=0)
        recompute_bitwise = float(Jr) == J32 and np.array_equal(gr.cpu().numpy(), g32)
        del er
        torch.cuda.empty_cache()
        e64 = B.Engine(p, M=M, seed=w.seed, precision="fp64", mode="store", device=dev)
        for it in range(args.warmup):
            e64.cost_grad(u, it=it)
        res["fp64_store_ms"] = time_calls(lambda: e64.cost_grad(u, it=7), args.steps)
        J64, g64 = e64.cost_grad(u, it=0)
        J64, g64 = float(J64), g64.cpu().numpy()
        del e64
        torch.cuda.empty_cache()
        for k, v in res.items():
            forms[k.replace("_ms", "")] = {
                "p50_ms": percentile(v, 50), "p99_ms": percentile(v, 99),
                "path_steps_per_s_p50": M * N / (percentile(v, 50) * 1e-3)}
        forms["fp32_recompute"]["bitwise_equal_to_store"] = recompute_bitwise
        forms["fp32_vs_fp64_full_size"] = {
            "J_rel": abs(J32 - J64) / abs(J64),
            "g_rel": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
        forms["speedup_fp32_over_fp64_p50"] = (percentile(res["fp64_store_ms"], 50) /
                                               percentile(res["fp32_store_ms"], 50))
        # the fused FP64 kernel is >99% of the call
        forms["fp64_store"]["issue"] = fp64_counted("jd::k_cost_grad_stored<double, 1, false, false>", M * N,
                                                    percentile(res["fp64_store_ms"], 50) * 1e-3)
    # average launch durations over the event-timed calls (the fused kernel is
    # >99% of a jd_cost_grad call; the table and finalize kernels take ~20 us)
    t_fwd = float(np.mean(fwd_ms)) * 1e-3
    t_adj = float(np.mean(adj_ms)) * 1e-3
    t_cg = float(np.mean(res["fp32_store_ms"])) * 1e-3
    # The dominant kernel is the fused per-block forward + adjoint sweep
    # (k_cost_grad_stored): one launch per step, >99% of the step's time (the
    # table and the two finalize kernels take ~20 us).  It is VALU-bound; its
    # HBM traffic (8 B per path-step) overlaps with the forward arithmetic.
    slots = (FWD_SLOTS_PER_PATH_STEP + ADJ_SLOTS_PER_PATH_STEP) * M * N
    roofline = {"bound": "alu", "kernel": "k_cost_grad_stored<float,1>",
                "achieved": slots / t_cg / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                "unit": "TOP/s (full-rate VALU lane-op slots)",
                "frac": slots / t_cg / VALU_PEAK_SLOTS,
                "traffic": profiled_traffic("jd::k_cost_grad_stored<float, 1, false, false>"),
                "slots_per_path_step": FWD_SLOTS_PER_PATH_STEP + ADJ_SLOTS_PER_PATH_STEP,
                "kernel_ms": t_cg * 1e3,
                "hbm_bytes_per_path_step": 8, "hbm_frac": 8.0 * M * N / t_cg / HBM_PEAK}
    fwd_slots = FWD_SLOTS_PER_PATH_STEP * M * N
    separate = {
        "forward": {"kernel": "k_forward<float,1,store>", "bound": "alu", "kernel_ms": t_fwd * 1e3,
                    "achieved": fwd_slots / t_fwd / 1e12, "frac": fwd_slots / t_fwd / VALU_PEAK_SLOTS,
                    "traffic": profiled_traffic("jd::k_forward<float, 1, 1, false, false>")},
        "adjoint": {"kernel": "k_adjoint_stored<float,1>", "bound": "hbm", "kernel_ms": t_adj * 1e3,
                    "achieved": 4.0 * M * N / t_adj / 1e9, "unit": "GB/s",
                    "frac": 4.0 * M * N / t_adj / HBM_PEAK,
                    "traffic": profiled_traffic("jd::k_adjoint_stored<float, 1, false, false>")},
    }

    # ---- oracle on a bounded sample of the same workload, and GPU errors there
    cpu = None
    sample_err = None
    if not args.no_cpu_baseline:
        from oracle import ref
        Ms = args.cpu_sample_paths
        nth = ref.default_threads()
        log(f"oracle: {Ms} paths x {N} steps on {nth} threads, best of 3")
        tcs = []
        for _ in range(3):
            t0 = time.perf_counter()
            Jo, go = ref.cost_grad(p, Ms, w.seed, 0, np.zeros((N, p.d)), nthreads=nth)
            tcs.append(time.perf_counter() - t0)
        tc = min(tcs)
        cpu = {"value": Ms * N / tc, "unit": "path-steps/s", "cores": nth, "kind": "oracle",
               "sample": f"c2 with M={Ms} of {M} paths, all N={N} steps, forward+adjoint+reductions, "
                         f"FP64, best of 3 runs ({', '.join(f'{x:.1f}' for x in tcs)} s wall)"}
        sample_err = {}
        for prec in ("fp32", "fp64"):
            es = B.Engine(p, M=Ms, seed=w.seed, precision=prec, mode="store", device=dev)
            Js, gs = es.cost_grad(u, it=0)
            sample_err[prec] = {"J_rel": abs(float(Js) - Jo) / abs(Jo),
                                "g_rel": float(np.linalg.norm(gs.cpu().numpy() - go) /
                                               np.linalg.norm(go))}
            del es
        log(f"oracle errors: {sample_err}")

    feedback = None
    if not args.no_feedback and args.only == "all":
        log("feedback model (f4)")
        feedback = feedback_section(args, time_calls, dev)
    adapted = None
    if not args.no_adapted and args.only == "all":
        log("jump-adapted grid (ja2, ja3)")
        adapted = adapted_section(args, time_calls, dev)
    rings = None
    if not args.no_ring and args.only == "all":
        log("coupled rings (ring2)")
        rings = ring_section(args, time_calls, dev)
    configs = None
    if not args.no_configs and args.only == "all":
        log("configurations c1, c2 iterations, c3, c4")
        configs = configs_section(args, time_calls, dev)
    serving = None
    if not args.no_serving and args.only == "all":
        serving = serving_section(args)

    fp32s = res["fp32_store_ms"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 paths, f64 reductions",
        "data": "synthetic (seeded Philox draws)",
        "config": {"workload": "c2: 1-D OU jump-diffusion, M=2^20 paths, N=1000 steps, lambda=5, "
                               "jumps N(-0.1,0.3^2), FP32 paths + FP64 reductions, stored trajectory",
                   "M": M, "N": N, "d": p.d},
        "p50_ms": percentile(fp32s, 50),
        "p99_ms": percentile(fp32s, 99),
        "roofline": roofline,
        "separate_kernels": separate,
        "cpu_baseline": cpu,
        "forms": forms,
        "oracle_error_on_sample": sample_err,
        "feedback": feedback,
        "rings": rings,
        "adapted": adapted,
        "configs": configs,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
