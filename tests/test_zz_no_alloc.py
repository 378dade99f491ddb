"""jd_cost_grad_noalloc (the workspace in the library's static device array)
against jd_cost_grad with a caller workspace, through the C ABI: bitwise the
same J and g on two calls in a row, the second with a smaller problem (and
another mode); and the refusal of a problem beyond the array's capacity."""
import ctypes as C
import sys

import pytest

from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import gpu_device

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _noalloc(eng, u, it):
    import torch
    J = torch.full((), float("nan"), dtype=torch.float64, device=eng.device)
    g = torch.full((eng.p.N, eng.p.d), float("nan"), dtype=torch.float64, device=eng.device)
    run = eng.run(it)
    rc = B.lib().jd_cost_grad_noalloc(eng.prob.ref, C.byref(run), u.data_ptr(), J.data_ptr(),
                                      g.data_ptr(), eng.traj.data_ptr(), B._stream_ptr(eng.device))
    B.check(rc, "jd_cost_grad_noalloc")
    return J, g


def test_noalloc_equals_cost_grad():
    import torch
    dev = gpu_device()
    big = wl.config("c2")  # 2^20 paths x 1000 steps: a 33 MB workspace
    small = wl.Workload(wl.general_problem(3, 120, seed=5, cubic=0.1, lam=6.0), M=1300, seed=9)
    for w, mode, K in ((big, "store", 0), (small, "recompute", 16)):
        p = w.problem
        say("noalloc", f"d={p.d} M={w.M} N={p.N}", mode)
        eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode=mode, K=K, device=dev)
        assert eng.ws_bytes - 256 <= B.lib().jd_noalloc_capacity()
        u = torch.tensor(wl.random_control(p, 3, 0.3), dtype=torch.float64, device=dev)
        J1, g1 = eng.cost_grad(u, it=2)
        J2, g2 = _noalloc(eng, u, it=2)
        torch.cuda.synchronize()
        assert float(J1) == float(J2)
        assert torch.equal(g1, g2)
        del eng
        torch.cuda.empty_cache()


def test_noalloc_leaves_out_an_automatic_noise_table_that_does_not_fit():
    """c1's model at 65536 paths in FP64: the automatic choice takes the noise
    table (105 MB, beyond the static array), which the allocation-free entry
    point replaces by draws in the sweeps; J and g are bitwise the same."""
    import torch
    dev = gpu_device()
    w = wl.config("c1")
    p = w.problem
    say("noalloc without the noise table", f"M=65536 N={p.N} FP64")
    eng = B.Engine(p, M=65536, seed=w.seed, precision="fp64", device=dev)
    inline = B.make_run(65536, precision="fp64", noise="inline")
    assert eng.ws_bytes - 256 > B.lib().jd_noalloc_capacity()
    assert B.lib().jd_workspace_bytes(eng.prob.ref, C.byref(inline)) - 256 <= \
        B.lib().jd_noalloc_capacity()
    u = torch.tensor(wl.random_control(p, 3, 0.3), dtype=torch.float64, device=dev)
    for it in (1, 4):
        J1, g1 = eng.cost_grad(u, it=it)
        J2, g2 = _noalloc(eng, u, it=it)
        torch.cuda.synchronize()
        assert float(J1) == float(J2)
        assert torch.equal(g1, g2)


def test_noalloc_refuses_beyond_capacity():
    dev = gpu_device()
    assert B.lib().jd_noalloc_capacity() == 64 << 20
    w = wl.config("c3")  # 131 MB of per-block partial sums
    prob = B.Problem(w.problem, dev)
    run = B.make_run(w.M, precision="fp32")
    assert B.lib().jd_workspace_bytes(prob.ref, C.byref(run)) > (64 << 20) + 256
    x = C.c_void_p(256)  # never dereferenced: the size check comes first
    rc = B.lib().jd_cost_grad_noalloc(prob.ref, C.byref(run), x, x, x, x, None)
    assert rc == B.JD_EWORKSPACE
