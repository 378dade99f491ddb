"""Parity at the full workload sizes (c2: 2^20 x 1000, c3: 2^20 x 500 x 8,
c4: 2^18 x 2000 x 8 with the cubic drift), in the launch configuration the
benchmark times.

* J, ||g||, 16 L2 projections of g and every entry of g (normwise and entry by
  entry) against FP64 oracle values written by tests/golden/make_full_size.py;
* per-path states, adjoints and costs of the first and last 4096 paths against
  the oracle computed here, path by path;
* the checkpoint-recompute variant bitwise equal to the stored one;
* the FP32 path form within the stated tolerance of the FP64 GPU form."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import (TOL, assert_grad, dump_to_paths, golden, golden_g, gpu_device, norm_err,
                         per_path_error, rel_err)

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def check_against_golden(p, J, g, gd, g_ref, s_ref, tol):
    assert rel_err(J, gd["J"]) <= tol["J"], (J, gd["J"])
    gn = np.sqrt(p.dt * np.sum(g * g))
    assert rel_err(gn, gd["gnorm_L2"]) <= tol["g"]
    dirs = wl.fd_directions(p, 16, seed=2)
    for dl, pr in zip(dirs, gd["projections"]):
        assert abs(p.dt * np.sum(g * dl) - pr) <= tol["g"] * gd["gnorm_L2"]
    flat = g.reshape(-1)
    for i, v in zip(gd["sample_index"], gd["sample_g"]):
        assert flat[i] == pytest.approx(v, rel=0, abs=tol["g"] * gd["gnorm_L2"])
    assert g_ref.shape == (p.N, p.d)
    en, ee = assert_grad(g, g_ref, s_ref, tol["g"])
    say(f"   g vs oracle: normwise {en:.2e}, per entry {ee:.2e}")


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_full_size(dev, name):
    import torch
    w = wl.config(name)
    p = w.problem
    M = w.M
    K = w.K or 64
    gd = golden(name)
    g_ref, s_ref = golden_g(name)
    g_ref, s_ref = g_ref.reshape(p.N, p.d), s_ref.reshape(p.N, p.d)
    assert gd["M"] == M and gd["N"] == p.N
    u = np.zeros((p.N, p.d))
    tol = TOL["fp32"]
    say(name, "fp32 store full size", M, p.N, p.d)
    e = B.Engine(p, M=M, seed=w.seed, precision="fp32", mode="store", device=dev)
    J, g = e.cost_grad(u, it=0)
    J, g = float(J), g.cpu().numpy()
    assert e.check_finite()
    check_against_golden(p, J, g, gd, g_ref, s_ref, tol)
    # per-path parity on the first and last 4096 paths
    for m0 in (0, M - 4096):
        say(name, "per-path dump", m0)
        dp, dumps = e.path_dump(m0, 4096)
        e.forward(u, it=0, dump=dp)
        e.adjoint(u, it=0, dump=dp)
        torch.cuda.synchronize()
        X, lam, C = ref.paths(p, w.seed, 0, m0, 4096, u)
        assert per_path_error(dump_to_paths(dumps["X"], 4096), X[:, 1:, :]) <= tol["path"]
        assert per_path_error(dump_to_paths(dumps["lam"], 4096), lam[:, 1:, :]) <= tol["path"]
        assert np.max(np.abs(dumps["cost"].cpu().numpy() - C) / np.abs(C)) <= tol["path"]
    del e, dumps, dp
    torch.cuda.empty_cache()
    say(name, "fp32 recompute full size, K =", K)
    r = B.Engine(p, M=M, seed=w.seed, precision="fp32", mode="recompute", K=K, device=dev)
    Jr, gr = r.cost_grad(u, it=0)
    assert float(Jr) == J and np.array_equal(gr.cpu().numpy(), g)
    del r
    torch.cuda.empty_cache()
    say(name, "fp64 store full size")
    e64 = B.Engine(p, M=M, seed=w.seed, precision="fp64", mode="store", device=dev)
    J64, g64 = e64.cost_grad(u, it=0)
    J64, g64 = float(J64), g64.cpu().numpy()
    check_against_golden(p, J64, g64, gd, g_ref, s_ref, TOL["fp64"])
    assert rel_err(J, J64) <= tol["J"] and norm_err(g, g64) <= tol["g"]
    say(f"   {name}: J32 {J:.12f} J64 {J64:.12f} oracle {gd['J']:.12f}; "
        f"g32 rel {norm_err(g, g64):.2e}")
    del e64
    torch.cuda.empty_cache()
