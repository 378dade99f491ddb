"""J(u) as torch.autograd.Function: backward (the checkpoint-recompute adjoint
kernel) against central finite differences of J under common random numbers,
against the oracle gradient, and torch.autograd.gradcheck on a tiny FP64 case.

The c4 workload (d = 8, cubic drift, M = 2^18, N = 2000, K = 64): FP32 path
arithmetic in the adjoint, FP64 forward for the differences (FP32 differences
would carry ~1e-7/h of rounding noise).  The sample J is smooth in u because the
jumps do not depend on u, so the central difference with h = 1e-4 is accurate to
O(h^2)."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import gpu_device, norm_err

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def test_c4_backward_vs_central_differences(dev):
    import torch
    from paper_2505_04328_amd.autograd import jd_cost
    w = wl.config("c4")
    p = w.problem
    say("c4 autograd", w.M, p.N, p.d, "K", w.K)
    u0 = wl.random_control(p, 3, 0.3)
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="recompute", K=w.K, device=dev)
    u = torch.tensor(u0, dtype=torch.float64, device=dev, requires_grad=True)
    J = jd_cost(u, eng, 0)
    J.backward()
    grad = u.grad.cpu().numpy()  # = dt * g
    f64 = B.Engine(p, M=w.M, seed=w.seed, precision="fp64", mode="store", device=dev)
    h = 1e-4
    gnorm = np.sqrt(np.sum(grad * grad) / p.dt)  # ||g||_L2 with g = grad / dt
    worst = 0.0
    for i, dl in enumerate(wl.fd_directions(p, 16, seed=2)):
        jp = float(f64.forward(u0 + h * dl, it=0, store=False))
        jm = float(f64.forward(u0 - h * dl, it=0, store=False))
        fd = (jp - jm) / (2 * h)
        ad = float(np.sum(grad * dl))
        err = abs(fd - ad) / gnorm  # directions are L2-normalised
        worst = max(worst, err)
    say(f"   worst |FD - <grad, delta>| / ||g|| = {worst:.2e}")
    assert worst <= 1e-6


def test_backward_matches_oracle_gradient(dev):
    import torch
    from paper_2505_04328_amd.autograd import jd_cost
    w = wl.scaled(wl.config("c4"), M=700, N=300)
    p = w.problem
    u0 = wl.random_control(p, 4, 0.3)
    eng = B.Engine(p, M=w.M, seed=5, precision="fp32", mode="recompute", K=64, device=dev)
    u = torch.tensor(u0, dtype=torch.float64, device=dev, requires_grad=True)
    J = jd_cost(u, eng, 3)
    J_ref, g_ref = ref.cost_grad(p, w.M, 5, 3, u0)
    assert abs(float(J) - J_ref) / J_ref <= 1e-6
    (2.0 * J).backward()
    assert norm_err(u.grad.cpu().numpy(), 2.0 * p.dt * g_ref) <= 1e-6


def test_backward_after_interleaved_forward(dev):
    """A second forward on the same engine before the first backward: the first
    backward still returns its own gradient."""
    import torch
    from paper_2505_04328_amd.autograd import jd_cost
    p = wl.general_problem(3, 50, seed=8, cubic=0.1)
    eng = B.Engine(p, M=900, seed=2, precision="fp64", mode="recompute", K=16, device=dev)
    ua = torch.tensor(wl.random_control(p, 1, 0.3), device=dev, requires_grad=True)
    ub = torch.tensor(wl.random_control(p, 2, 0.3), device=dev, requires_grad=True)
    Ja = jd_cost(ua, eng, 0)
    Jb = jd_cost(ub, eng, 1)
    Ja.backward()
    Jb.backward()
    _, ga = ref.cost_grad(p, 900, 2, 0, ua.detach().cpu().numpy())
    _, gb = ref.cost_grad(p, 900, 2, 1, ub.detach().cpu().numpy())
    assert norm_err(ua.grad.cpu().numpy(), p.dt * ga) <= 1e-12
    assert norm_err(ub.grad.cpu().numpy(), p.dt * gb) <= 1e-12


def test_gradcheck_tiny_fp64(dev):
    import torch
    from paper_2505_04328_amd.autograd import jd_cost
    p = wl.general_problem(2, 6, seed=9, cubic=0.2, lam=3.0)
    eng = B.Engine(p, M=300, seed=4, precision="fp64", mode="store", device=dev)
    u = torch.tensor(wl.random_control(p, 5, 0.4), device=dev, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: jd_cost(x, eng, 7), (u,), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)
