"""GPU parity of the jump-adapted grid (Section 3, Algorithms 5.1-5.2: each
particle's grid is the uniform points plus its jump times) against the FP64
oracle on the same counter-based draws.

Per-particle states and adjoints at the uniform points, particle costs, J and
the gradient, in both path precisions: the paper's step (dt = 0.1, a jump in
one interval of six, up to several per interval), a fine step (dt = 0.01),
a moving target (interpolated at the jump times), the ellipse cost, padded
shape-function rows and the full 16 x 16 grid; edge shapes; the no-jump limit
against the fixed grid; the gradient iteration against the oracle's."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import (TOL, assert_grad, golden, golden_g, gpu_device, grad_errors, norm_err,
                         per_path_error, rel_err)

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _track(N, T):
    t = np.arange(N + 1) * (T / N)
    return np.stack([0.4 * np.cos(2 * t), -0.3 * np.sin(t)], axis=1)


CASES = {
    # name: (problem kwargs, M, seed)
    "paper_step": (dict(N=50, T=5.0), 2000, 1),
    "fine_step": (dict(N=200, T=2.0, nx=6, nv=6, alpha=0.1), 700, 3),
    "moving_target": (dict(N=40, T=4.0, zd="track", b1=0.2, b2=0.3, gamma=0.8), 900, 5),
    "ellipse": (dict(N=30, T=3.0, cost="ellipse", init="ellipse", s0=(0.1, 0.1), nv=5), 600, 7),
    "grid_16x16": (dict(N=12, T=1.2, nx=16, nv=16, eps=0.8, beta=40.0), 500, 9),
    # about 40 jumps per particle: most particles overflow the adjoint's stack
    # of 32 post-jump states and have the rest recomputed
    "beyond_the_jump_stack": (dict(N=50, T=5.0, beta=200.0, gamma=0.95, b1=0.05, b2=0.05), 300, 11),
}


def _problem(name):
    kw, M, seed = CASES[name]
    kw = dict(kw)
    if kw.get("zd") == "track":
        kw["zd"] = _track(kw["N"], kw["T"])
    else:
        kw.setdefault("zd", _track(kw.get("N", 50), kw.get("T", 5.0)))
    return wl.feedback_problem(grid="adapted", **kw), M, seed


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_adapted_cost_grad_and_paths(dev, name, precision):
    p, M, seed = _problem(name)
    say(name, precision, f"M={M} N={p.N} nx={p.nx} nv={p.nv} sigma dt={p.rate * p.dt:.3f}")
    mu = wl.random_feedback_control(p, 4, 0.5)
    it = 2
    z, lam, _, n, C = ref.fb_paths(p, seed, it, 0, M, mu)
    J_ref, g_ref = ref.fb_cost_grad(p, M, seed, it, mu)
    s_ref = ref.fb_grad_scale(p, M, seed, it, mu)
    assert n.sum() > 0
    if name == "beyond_the_jump_stack":
        assert (n.sum(axis=1) > 32).mean() > 0.5
    eng = B.FbEngine(p, M=M, seed=seed, precision=precision, device=dev)
    dp, d = eng.path_dump(0, M)
    J = eng.forward(mu, it=it, dump=dp)
    eng.adjoint(mu, it=it, dump=dp)
    Jc, gc = eng.cost_grad(mu, it=it)
    import torch
    torch.cuda.synchronize()
    assert eng.check_finite()
    tol = TOL[precision]
    zg = np.transpose(d["X"].double().cpu().numpy(), (2, 0, 1))
    lg = np.transpose(d["lam"].double().cpu().numpy(), (2, 0, 1))
    e_z = per_path_error(zg, z)
    e_l = per_path_error(lg[:, 1:], lam[:, 1:])
    e_c = float(np.max(np.abs(d["cost"].cpu().numpy() - C) / (np.abs(C) + np.sqrt(np.mean(C * C)))))
    e_J, e_J2 = rel_err(float(J), J_ref), rel_err(float(Jc), J_ref)
    e_g, e_ge = grad_errors(gc.cpu().numpy(), g_ref, s_ref)
    say(f"   jumps {int(n.sum())} (max {int(n.max())} per interval); errors: z {e_z:.2e} "
        f"lam {e_l:.2e} C {e_c:.2e} J {e_J:.2e} g {e_g:.2e} (per entry {e_ge:.2e})")
    assert e_z <= tol["path"]
    assert e_l <= tol["path"]
    assert e_c <= tol["path"]
    assert e_J <= tol["J"] and e_J2 <= tol["J"]
    assert e_g <= tol["g"] and e_ge <= tol["g"]


EDGE = [
    # (label, N, M)
    ("one particle", 10, 1),
    ("one block plus one", 8, 257),
    ("one step", 1, 300),
]


@pytest.mark.parametrize("label,N,M", EDGE)
def test_adapted_edge_shapes(dev, label, N, M):
    say("adapted edge", label)
    p = wl.feedback_problem(N=N, T=0.5 * N, zd=_track(N, 0.5 * N), alpha=0.2, grid="adapted")
    mu = wl.random_feedback_control(p, 6, 1.0)
    for prec in ("fp32", "fp64"):
        eng = B.FbEngine(p, M=M, seed=13, precision=prec, device=dev)
        J, g = eng.cost_grad(mu, it=1)
        J_ref, g_ref = ref.fb_cost_grad(p, M, 13, 1, mu)
        s_ref = ref.fb_grad_scale(p, M, 13, 1, mu)
        assert rel_err(float(J), J_ref) <= TOL[prec]["J"]
        # one particle: each entry is that particle's own summand, held to the
        # per-path bound (no mean over paths averages its rounding)
        assert_grad(g.cpu().numpy(), g_ref, s_ref, TOL[prec]["g"], f"{label} {prec}",
                    tol_entry=TOL[prec]["path"] if M == 1 else None)


def test_adapted_without_jumps_is_the_fixed_grid(dev):
    kw = dict(N=20, T=2.0, beta=1e-12, alpha=0.2, zd=_track(20, 2.0))
    fixed = wl.feedback_problem(**kw)
    adapted = wl.feedback_problem(grid="adapted", **kw)
    mu = wl.random_feedback_control(fixed, 3, 0.5)
    ef = B.FbEngine(fixed, M=1000, seed=4, precision="fp64", device=dev)
    ea = B.FbEngine(adapted, M=1000, seed=4, precision="fp64", device=dev)
    Jf, gf = ef.cost_grad(mu)
    Ja, ga = ea.cost_grad(mu)
    assert float(Ja) == float(Jf)
    assert norm_err(ga.cpu().numpy(), gf.cpu().numpy()) <= 1e-14


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_adapted_optimize_matches_oracle(dev, precision):
    p, M, seed = _problem("moving_target")
    say("adapted optimize", precision)
    mu0 = np.zeros((p.N, p.L))
    mu_ref, logs_ref, n_ref = ref.fb_optimize(p, M, seed, 0, mu0, n_max=3, zeta0=5.0)
    assert n_ref == 3
    eng = B.FbEngine(p, M=M, seed=seed, precision=precision, device=dev)
    mu, logs = eng.optimize(mu0, n_max=3, zeta0=5.0)
    assert len(logs) == 3
    tol = TOL[precision]
    for a, b in zip(logs, logs_ref):
        assert a["backtracks"] == b["backtracks"]
        assert rel_err(a["J"], b["J"]) <= tol["J"]
    assert norm_err(mu.cpu().numpy(), mu_ref) <= 10 * tol["g"]


def test_adapted_full_size_ja2(dev):
    """The measured size on the jump-adapted grid (2^20 particles x 500 steps,
    FP32 paths) in the launch configuration the benchmark times: J, ||g||, 16
    projections, 64 sampled entries and every entry of g against the oracle
    values of tests/golden/full_ja2_it0.json and full_ja2_it0_g.npz (written by
    tests/golden/make_full_size.py);
    per-particle states, adjoints and costs of the first and last 4096
    particles against the oracle here."""
    import torch
    gd = golden("ja2")
    w = wl.adapted_config("ja2")
    p = w.problem
    say("adapted full size ja2", w.M, p.N)
    mu = wl.random_feedback_control(p, 4, 0.5)
    eng = B.FbEngine(p, M=w.M, seed=w.seed, precision="fp32", device=dev)
    J, g = eng.cost_grad(mu, it=0)
    J, g = float(J), g.cpu().numpy()
    tol = TOL["fp32"]
    say(f"   J {J:.12g} vs {gd['J']:.12g}")
    assert rel_err(J, gd["J"]) <= tol["J"]
    gn = np.sqrt(p.dt * np.sum(g * g))
    assert rel_err(gn, gd["gnorm_L2"]) <= tol["g"]
    rng = np.random.default_rng(2)
    for pr in gd["projections"]:
        d = rng.normal(size=(p.N, p.L))
        d = d / np.sqrt(p.dt * np.sum(d * d))
        assert abs(p.dt * np.sum(g * d) - pr) <= tol["g"] * gd["gnorm_L2"]
    flat = g.reshape(-1)
    for i, v in zip(gd["sample_index"], gd["sample_g"]):
        assert abs(flat[i] - v) <= tol["g"] * gd["gnorm_L2"]
    en, ee = assert_grad(g, *golden_g("ja2"), tol["g"])
    say(f"   g vs oracle: normwise {en:.2e}, per entry {ee:.2e}")
    for m0 in (0, w.M - 4096):
        dp, dd = eng.path_dump(m0, 4096)
        eng.forward(mu, it=0, dump=dp)
        eng.adjoint(mu, it=0, dump=dp)
        torch.cuda.synchronize()
        z, lam, _, _, C = ref.fb_paths(p, w.seed, 0, m0, 4096, mu)
        zg = np.transpose(dd["X"].double().cpu().numpy(), (2, 0, 1))
        lg = np.transpose(dd["lam"].double().cpu().numpy(), (2, 0, 1))
        e_z, e_l = per_path_error(zg, z), per_path_error(lg[:, 1:], lam[:, 1:])
        say(f"   paths {m0}+4096: z {e_z:.2e} lam {e_l:.2e}")
        assert e_z <= tol["path"] and e_l <= tol["path"]
        e_c = float(np.max(np.abs(dd["cost"].cpu().numpy() - C) / (np.abs(C) + np.sqrt(np.mean(C * C)))))
        assert e_c <= tol["path"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_adapted_stored_jump_counts(dev, precision):
    """The jump-adapted forward's per-slot jump totals (int32) and per-interval
    counts (one byte per slot and interval), laid out as the header states,
    equal the oracle's counts."""
    import torch
    p, M, seed = _problem("paper_step")
    mu = wl.random_feedback_control(p, 4, 0.5)
    eng = B.FbEngine(p, M=M, seed=seed, precision=precision, device=dev)
    eng.forward(mu, it=2)
    torch.cuda.synchronize()
    _, _, _, n_ref, _ = ref.fb_paths(p, seed, 2, 0, M, mu)
    esz = eng.traj.element_size()
    slots = eng.nblk * 256
    T = slots * (p.N + 1) * 2 + slots * 32 * 3  # states, then the jump stacks
    raw = eng.traj.view(torch.uint8)[T * esz:].cpu().numpy()
    totals = raw[:slots * 4].view(np.int32)[:M]
    np.testing.assert_array_equal(totals, n_ref.sum(axis=1))
    per = raw[slots * 4:]
    assert per.size == eng.nblk * p.N * 256
    s = np.arange(M)
    k = np.arange(p.N)
    got = per[((s[:, None] // 256) * p.N + k[None, :]) * 256 + (s[:, None] % 256)]
    np.testing.assert_array_equal(got, n_ref)
