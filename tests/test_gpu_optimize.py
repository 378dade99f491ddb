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

from parity_util import TOL, assert_grad, gpu_device, rel_err

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
        s_ref = ref.grad_scale(p, M, seed, n, ub)
        Jg, gg = eng.cost_grad(u_before, it=n)
        assert rel_err(lg["J"], J_ref) <= tol["J"]
        assert rel_err(float(Jg), J_ref) <= tol["J"]
        assert_grad(gg.cpu().numpy(), g_ref, s_ref, tol["g"], f"iteration {n}")
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


def test_overflowing_trial_is_rejected_fp64(dev):
    """A first step so large that the trial's cubic drift overflows (J of the
    trial is not finite): the Armijo test rejects the trial and backtracks, as
    the oracle does, instead of ending the iteration with JD_ENONFINITE."""
    say("c4-shaped fp64, overflowing first trials")
    w = wl.scaled(wl.config("c4"), M=300, N=100)
    p = w.problem
    J, _ = ref.cost_grad(p, w.M, w.seed, 0, 1e4 * np.ones((p.N, p.d)), grad=False)
    assert not np.isfinite(J)  # a step to u ~ 1e4 overflows
    assert _replay(dev, p, w.M, w.seed, "fp64", 2, zeta0=1e5) == 0


def test_overflowing_trial_is_rejected_fp32(dev):
    import torch
    w = wl.scaled(wl.config("c4"), M=300, N=100)
    p = w.problem
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="recompute", K=64, device=dev)
    u = torch.zeros((p.N, p.d), dtype=torch.float64, device=dev)
    _, logs = eng.optimize(u, n_max=2, zeta0=1e5)
    assert len(logs) == 2 and logs[0]["backtracks"] > 0
    assert all(np.isfinite(l["J_new"]) for l in logs)


def test_more_iterations_than_one_batch(dev):
    """70 iterations in one call: more than one batch of the device-driven
    iteration (64) and its log ring; the logs and the control equal those of
    70 calls of one iteration each, bit for bit."""
    import torch
    w = wl.scaled(wl.config("c1"), M=2000)
    p = w.problem
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp64", device=dev)
    u1 = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
    _, logs1 = eng.optimize(u1, n_max=70, zeta0=4.0)
    assert len(logs1) == 70
    u2 = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
    logs2 = []
    for n in range(70):
        _, lg = eng.optimize(u2, n_max=1, it0=n, zeta0=4.0)
        logs2 += lg
    assert torch.equal(u1, u2)
    assert logs1 == logs2
    assert [l["iter"] for l in logs1] == list(range(70))
    assert any(l["backtracks"] > 0 for l in logs1)


@pytest.mark.parametrize("precision,mode,K,zeta0", [("fp64", "store", 0, 4.0),
                                                     ("fp32", "recompute", 25, 64.0)])
def test_noise_table_iterates_bitwise_inline(dev, precision, mode, K, zeta0):
    """The line-search trials of an iteration read the noise table its
    gradient evaluation wrote, also across the device-driven batches (70
    iterations, backtracking): logs and control equal the inline draws', bit
    for bit."""
    import torch
    say("noise table iterates", precision, mode)
    w = wl.scaled(wl.config("c1"), M=3000)
    p = w.problem
    res = []
    for noise in ("table", "inline"):
        eng = B.Engine(p, M=w.M, seed=w.seed, precision=precision, mode=mode, K=K, device=dev,
                       noise=noise)
        u = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
        _, logs = eng.optimize(u, n_max=70, zeta0=zeta0)
        res.append((u.cpu().numpy(), logs))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]
    assert len(res[0][1]) == 70 and any(l["backtracks"] > 0 for l in res[0][1])


def test_tolerance_stops_on_the_device(dev):
    """tol > 0: the device stops the iteration at the first accepted step with
    ||u' - u||_L2 <= tol; the call reports the iterations done."""
    import torch
    w = wl.scaled(wl.config("c1"), M=2000)
    p = w.problem
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp64", device=dev)
    u = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
    _, full = eng.optimize(u.clone(), n_max=20)
    Es = [l["E"] for l in full]
    tol = sorted(Es)[len(Es) // 2]
    stop = next(i for i, E in enumerate(Es) if E <= tol)
    _, logs = eng.optimize(u, n_max=20, tol=tol)
    assert len(logs) == stop + 1
    assert logs == full[:stop + 1]


@pytest.mark.timeout(900)
def test_c2_fifty_iterations_full_size(dev):
    """c2 at full size (2^20 paths x 1000 steps, FP32 paths): 50 gradient
    iterations stored and with checkpoints every 32 steps give bitwise the same
    iterates and logs; iterations 0, 1, 25 and 49 are replayed through the
    oracle from the GPU's own iterate on the same counter word: J, g (normwise
    and entry by entry), the accepted step and the backtrack count, and the
    next iterate."""
    import torch
    from parity_util import per_entry_error
    w = wl.config("c2")
    p = w.problem
    assert w.M == 1 << 20 and p.N == 1000 and w.iters == 50
    tol = TOL["fp32"]
    say("c2 full size, 50 iterations stored")
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="store", device=dev)
    replay = (0, 1, 25, 49)
    u = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
    snaps, logs = {}, []
    for n in range(w.iters):
        if n in replay or n - 1 in replay:
            snaps[n] = u.cpu().numpy().copy()
        _, lg = eng.optimize(u, n_max=1, it0=n)
        logs += lg
    snaps[w.iters] = u.cpu().numpy().copy()
    say("c2 full size, 50 iterations with checkpoints every 32 steps, one call")
    er = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="recompute", K=w.K, device=dev)
    ur = torch.zeros((p.N, 1), dtype=torch.float64, device=dev)
    _, logs_r = er.optimize(ur, n_max=w.iters)
    assert torch.equal(u, ur), "stored and recomputed iterations differ"
    assert logs_r == logs
    del er
    torch.cuda.empty_cache()
    for n in replay:
        ub = snaps[n]
        say(f"   replay iteration {n} through the oracle")
        J_ref, g_ref = ref.cost_grad(p, w.M, w.seed, n, ub)
        s_ref = ref.grad_scale(p, w.M, w.seed, n, ub)
        Jg, gg = eng.cost_grad(torch.tensor(ub, device=dev), it=n)
        assert rel_err(logs[n]["J"], J_ref) <= tol["J"]
        assert rel_err(float(Jg), J_ref) <= tol["J"]
        en, ee = assert_grad(gg.cpu().numpy(), g_ref, s_ref, tol["g"], f"iteration {n}")
        _, lo, _ = ref.optimize(p, w.M, w.seed, n, u0=ub, n_max=1)
        assert lo["backtracks"][0] == logs[n]["backtracks"]
        assert lo["zeta"][0] == logs[n]["zeta"]
        # the GPU's next iterate against u_n - zeta g_ref, entry by entry
        zeta = logs[n]["zeta"]
        step_err = per_entry_error((ub - snaps[n + 1]) / zeta, g_ref, s_ref)
        assert step_err <= tol["g"], step_err
        say(f"   iteration {n}: J {logs[n]['J']:.10f} (oracle {J_ref:.10f}), g {en:.1e} / {ee:.1e}, "
            f"zeta {zeta}, backtracks {logs[n]['backtracks']}")
