"""The request server: a mix of requests of different dimension, path count,
horizon and jump rate arrives while others run; the arena is too small for all
of them at once, so admission has to wait for memory.  Every request's result
(final control and per-iteration log) must be bitwise the one jd_optimize gives
for the same request alone."""
import sys

import numpy as np
import pytest

from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import serving as S
from paper_2505_04328_amd import workloads as wl

from parity_util import gpu_device

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def small_mix():
    reqs = wl.serving_requests(count=12, rate=400.0, seed=21, M_lo=500, M_hi=6000, N_lo=40,
                               N_hi=300, lam_hi=10.0, iters=4)
    return reqs


def test_mix_equals_alone(dev):
    import torch
    reqs = small_mix()
    sizes = [S.request_bytes(r.problem, r.M) for r in reqs]
    # the three largest requests arrive first, together; the arena holds the
    # two largest and half of the third, so the first scheduling step admits
    # two of them and the third waits for memory; the rest arrive while those
    # run
    big = sorted(range(len(reqs)), key=lambda i: -sizes[i])[:3]
    for i in big:
        reqs[i].arrival = 0.0
    s3 = sorted(sizes, reverse=True)
    arena = s3[0] + s3[1] + s3[2] // 2
    say("server mix", len(reqs), "requests, arena", arena, "bytes, largest", max(sizes))
    srv = S.Server(arena, max_active=8, n_streams=4, device=dev)
    recs, wall = S.run_mix(srv, reqs, precision="fp32", store_limit=1 << 40, time_scale=1.0,
                           timeout=300)
    srv.close()
    say("   server stats", srv.stats)
    assert len(recs) == len(reqs)
    # requests overlapped on the device, and some waited for arena memory
    assert srv.stats["max_active"] > 1
    assert srv.stats["waited_for_memory"] > 0
    # the three largest arrive together and one of them waits for the others' memory
    assert max(rec.queued for rec in recs if rec.rid in {reqs[i].rid for i in big}) > 0
    by_rid = {r.rid: r for r in reqs}
    for rec in recs:
        r = by_rid[rec.rid]
        assert rec.status == 0, rec.status
        assert rec.iterations == r.iters
        say(f"   req {rec.rid}: d={r.problem.d} M={r.M} N={r.problem.N} lam={r.problem.lam:.2f} "
            f"latency {rec.latency * 1e3:.1f} ms (queued {rec.queued * 1e3:.1f}, "
            f"service {rec.service * 1e3:.1f})")
        # the server's split of the latency: both parts non-negative and within it
        assert rec.queued >= 0 and rec.service > 0
        assert rec.queued + rec.service <= rec.latency + 0.05
        eng = B.Engine(r.problem, M=r.M, seed=r.seed, precision="fp32", mode="store", device=dev)
        u = torch.zeros((r.problem.N, r.problem.d), dtype=torch.float64, device=dev)
        _, log = eng.optimize(u, n_max=r.iters, it0=0)
        assert np.array_equal(u.cpu().numpy(), rec.u), f"request {rec.rid} differs from alone"
        assert log == rec.log, f"request {rec.rid}: iteration log differs from alone"


def test_oversized_request_rejected(dev):
    p = wl.general_problem(4, 200, seed=1)
    need = S.request_bytes(p, 5000)
    srv = S.Server(need // 2, max_active=2, n_streams=1, device=dev)
    with pytest.raises(B.JdError) as e:
        srv.submit(p, 5000, 1, 2)
    assert e.value.code == B.JD_EWORKSPACE
    srv.close()


def test_recompute_requests_in_mix(dev):
    """Requests served with checkpoint recompute give the same control as the
    stored mode (bit-identical sweeps)."""
    import torch
    reqs = wl.serving_requests(count=4, rate=1000.0, seed=5, M_lo=700, M_hi=3000, N_lo=80,
                               N_hi=200, iters=3)
    srv = S.Server(1 << 30, max_active=4, n_streams=2, device=dev)
    recs, _ = S.run_mix(srv, reqs, precision="fp32", store_limit=0, timeout=300)
    srv.close()
    by_rid = {r.rid: r for r in reqs}
    for rec in recs:
        r = by_rid[rec.rid]
        eng = B.Engine(r.problem, M=r.M, seed=r.seed, precision="fp32", mode="store", device=dev)
        u = torch.zeros((r.problem.N, r.problem.d), dtype=torch.float64, device=dev)
        eng.optimize(u, n_max=r.iters, it0=0)
        assert np.array_equal(u.cpu().numpy(), rec.u)
