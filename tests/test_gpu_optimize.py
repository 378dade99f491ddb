"""The gradient iteration (jd_optimize) against the oracle, by replay: every
iteration n is re-run by the oracle from the GPU's own iterate u^n with the same
counter word, and must give the same J_n, g_n, step and backtrack count.
Running the iterations one call at a time must give bitwise the same final
control as one call with n_max iterations (the state is (u^n, n) only)."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import TOL, gpu_device, norm_err, rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _replay(dev, p, M, seed, precision, iters, mode="store", K=0, zeta0=1.0, c=1e-4):
    import torch
    eng = B.Engine(p, M=M, seed=seed, precision=precision, mode=mode, K=K, device=dev)
    tol = TOL[precision]
    u = torch.zeros((p.N, p.d), dtype=torch.float64, device=dev)
    u_full = u.clone()
    _, logs_full = eng.optimize(u_full, n_max=iters, it0=0, zeta0=zeta0, c_armijo=c)
    assert len(logs_full) == iters
    mismatched_decisions = 0
    for n in range(iters):
        u_before = u.clone()
        _, lg = eng.optimize(u, n_max=1, it0=n, zeta0=zeta0, c_armijo=c)
        lg = lg[0]
        ub = u_before.cpu().numpy()
        J_ref, g_ref = ref.cost_grad(p, M, seed, n, ub)
        Jg, gg = eng.cost_grad(u_before, it=n)
        assert rel_err(lg["J"], J_ref) <= tol["J"]
        assert rel_err(float(Jg), J_ref) <= tol["J"]
        assert norm_err(gg.cpu().numpy(), g_ref) <= tol["g"]
        gn_ref = np.sqrt(p.dt * np.sum(g_ref * g_ref))
        assert rel_err(lg["gnorm"], gn_ref) <= tol["g"]
        # Armijo on the same draws, and the step is -zeta g
        assert lg["J_new"] <= lg["J"] - c * lg["zeta"] * lg["gnorm"] ** 2
        assert lg["E"] == pytest.approx(lg["zeta"] * lg["gnorm"], rel=1e-12)
        # the oracle's own line search from the GPU iterate
        u_o, lo, _ = ref.optimize(p, M, seed, n, u0=ub, n_max=1, zeta0=zeta0, c_armijo=c)
        if lo["backtracks"][0] != lg["backtracks"]:
            mismatched_decisions += 1
        else:
            assert lo["zeta"][0] == lg["zeta"]
            np.testing.assert_allclose(u.cpu().numpy(), u_o, rtol=0, atol=tol["g"] * 10 *
                                       max(1.0, np.abs(u_o).max()))
        say(f"   iter {n}: J {lg['J']:.10f} (oracle {J_ref:.10f}) zeta {lg['zeta']} "
            f"bt {lg['backtracks']} (oracle {lo['backtracks'][0]})")
    assert torch.equal(u, u_full), "one-call and iteration-by-iteration runs differ"
    return mismatched_decisions


def test_c1_twenty_iterations_fp64(dev):
    say("c1 fp64 20 iterations")
    w = wl.config("c1")
    assert _replay(dev, w.problem, w.M, w.seed, "fp64", 20) == 0


def test_c1_backtracking_fp64(dev):
    """A large first step and a strict constant force backtracking every iteration."""
    say("c1 fp64 backtracking")
    w = wl.config("c1")
    assert _replay(dev, w.problem, w.M, w.seed, "fp64", 4, zeta0=64.0, c=0.5) == 0


@pytest.mark.parametrize("mode,K", [("store", 0), ("recompute", 32)])
def test_c2_shape_fp32(dev, mode, K):
    say("c2-shaped fp32", mode)
    w = wl.scaled(wl.config("c2"), M=5000)
    # FP32 sums may flip a near-tie Armijo decision; none is expected here
    assert _replay(dev, w.problem, w.M, w.seed, "fp32", 5, mode=mode, K=K) == 0


def test_cubic_d8_fp32(dev):
    say("c4-shaped fp32 recompute")
    w = wl.scaled(wl.config("c4"), M=600, N=400)
    assert _replay(dev, w.problem, w.M, w.seed, "fp32", 3, mode="recompute", K=64,
                   zeta0=16.0) == 0


def test_linesearch_failure_leaves_u(dev):
    """With max_backtracks = 1 and an absurd first step the trial is rejected:
    JD_ELINESEARCH and u unchanged."""
    import torch
    w = wl.config("c1")
    eng = B.Engine(w.problem, M=2000, seed=1, precision="fp64", device=dev)
    u = torch.zeros((w.problem.N, 1), dtype=torch.float64, device=dev)
    with pytest.raises(B.JdError) as e:
        eng.optimize(u, n_max=3, it0=0, zeta0=1e6, max_backtracks=1)
    assert e.value.code == B.JD_ELINESEARCH
    assert torch.count_nonzero(u).item() == 0
