"""GPU parity of coupled particles (Section 6.4: rings of np nearest-neighbour
coupled oscillators, the ellipse cost and the start on the ellipse) against the
FP64 oracle on the same counter-based draws.

Per-particle states z_0..z_N, adjoints lam_1..lam_N and particle costs to the
per-path tolerance, J and the gradient to the J / g tolerances, in both path
precisions, over ring sizes that cover: several rings per workgroup with a
partial last workgroup (np = 3, 7), two-particle rings whose two neighbours
coincide (np = 2), a workgroup exactly full (np = 256), rings across the
eight 256-slot groups of a workgroup with several rings per workgroup
(np = 300), the paper's ring of 2000 and the largest ring (2048); also the
tracking cost on rings, the ellipse cost without a target, and the gradient
iteration replayed against the oracle's."""
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


RINGS = {
    # name: (problem kwargs, M rings, seed)
    "ring3": (dict(N=20, T=2.0, np_=3, alpha=0.3, s0=(0.05, 0.05), sigJ=0.4), 100, 3),
    "ring2": (dict(N=15, T=1.5, np_=2, omega=1.1, alpha=0.2), 300, 5),
    "ring7_track": (dict(N=20, T=2.0, np_=7, omega=0.8, cost="track", init="gauss",
                         s0=(0.3, 0.3), zd="track"), 80, 7),
    "ring256": (dict(N=10, T=1.0, np_=256, alpha=0.1, s0=(0.02, 0.02)), 5, 9),
    "ring300": (dict(N=10, T=1.0, np_=300, nx=6, nv=7, gamma=-0.5), 9, 11),
    "ring2000": (dict(N=12, T=1.2, np_=2000, alpha=0.1), 3, 1),
    "ring2048": (dict(N=6, T=0.6, np_=2048, nx=16, nv=16, eps=0.8), 2, 2),
}


def _ring(name):
    kw, M, seed = RINGS[name]
    kw = dict(kw)
    if kw.get("zd") == "track":
        kw["zd"] = _track(kw["N"], kw["T"])
    cost = kw.pop("cost", "ellipse")
    init = kw.pop("init", "ellipse")
    p = wl.feedback_problem(cost=cost, init=init, omega=kw.pop("omega", 0.5), **kw)
    return p, M, seed


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(RINGS))
def test_ring_cost_grad_and_paths(dev, name, precision):
    p, M, seed = _ring(name)
    P = M * p.np
    say(name, precision, f"rings={M} np={p.np} N={p.N} nx={p.nx} nv={p.nv}")
    mu = wl.random_feedback_control(p, 4, 0.5)
    it = 2
    z, lam, _, n, C = ref.fb_paths(p, seed, it, 0, M, mu)
    J_ref, g_ref = ref.fb_cost_grad(p, M, seed, it, mu)
    s_ref = ref.fb_grad_scale(p, M, seed, it, mu)
    assert n.sum() > 0
    eng = B.FbEngine(p, M=M, seed=seed, precision=precision, device=dev)
    dp, d = eng.path_dump(0, P)
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
    say(f"   per-entry g error {e_ge:.2e}")
    say(f"   errors: z {e_z:.2e} lam {e_l:.2e} C {e_c:.2e} J {e_J:.2e} g {e_g:.2e}")
    assert e_z <= tol["path"]
    assert e_l <= tol["path"]
    assert e_c <= tol["path"]
    assert e_J <= tol["J"] and e_J2 <= tol["J"]
    assert e_g <= tol["g"] and e_ge <= tol["g"]
    traj = np.transpose(eng.trajectory().double().cpu().numpy(), (2, 0, 1))
    assert per_path_error(traj, z) <= tol["path"]


def test_ring_partial_dump_window(dev):
    """A dump window that starts and ends inside rings."""
    p, M, seed = _ring("ring7_track")
    mu = wl.random_feedback_control(p, 5, 0.5)
    z, lam, _, _, C = ref.fb_paths(p, seed, 0, 0, M, mu)
    eng = B.FbEngine(p, M=M, seed=seed, precision="fp64", device=dev)
    m0, cnt = 23, 101
    dp, d = eng.path_dump(m0, cnt)
    eng.forward(mu, dump=dp)
    eng.adjoint(mu, dump=dp)
    zg = np.transpose(d["X"].double().cpu().numpy(), (2, 0, 1))
    lg = np.transpose(d["lam"].double().cpu().numpy(), (2, 0, 1))
    assert per_path_error(zg, z[m0:m0 + cnt]) <= TOL["fp64"]["path"]
    assert per_path_error(lg[:, 1:], lam[m0:m0 + cnt, 1:]) <= TOL["fp64"]["path"]
    np.testing.assert_allclose(d["cost"].cpu().numpy(), C[m0:m0 + cnt], rtol=1e-12, atol=1e-14)


def test_ring_ellipse_cost_needs_no_target(dev):
    p, M, seed = _ring("ring3")
    mu = wl.random_feedback_control(p, 6, 0.5)
    eng = B.FbEngine(p, M=M, seed=seed, precision="fp64", device=dev)
    J1, g1 = eng.cost_grad(mu, it=1)
    J1, g1 = float(J1), g1.cpu().numpy()
    eng.prob.st.zd = None
    J2, g2 = eng.cost_grad(mu, it=1)
    assert float(J2) == J1
    np.testing.assert_array_equal(g2.cpu().numpy(), g1)


def test_ring_uncoupled_equals_independent_particles(dev):
    """omega = 0: rings of 4 give the particles of the one-particle model."""
    kw = dict(N=12, T=1.2, alpha=0.2, zd=_track(12, 1.2), init="gauss", s0=(0.2, 0.3))
    ring = wl.feedback_problem(np_=4, omega=0.0, **kw)
    single = wl.feedback_problem(**kw)
    mu = wl.random_feedback_control(ring, 3, 0.5)
    er = B.FbEngine(ring, M=90, seed=9, precision="fp64", device=dev)
    es = B.FbEngine(single, M=360, seed=9, precision="fp64", device=dev)
    dr, d1 = er.path_dump(0, 360)
    ds, d2 = es.path_dump(0, 360)
    er.forward(mu, dump=dr)
    es.forward(mu, dump=ds)
    np.testing.assert_array_equal(d1["X"].cpu().numpy(), d2["X"].cpu().numpy())
    Jr, gr = er.cost_grad(mu)
    Js, gs = es.cost_grad(mu)
    assert rel_err(float(Jr), float(Js)) <= 1e-13
    assert norm_err(gr.cpu().numpy(), gs.cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ring_optimize_matches_oracle(dev, precision):
    p, M, seed = _ring("ring3")
    say("ring optimize", precision)
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
    assert logs[-1]["J"] < logs[0]["J"]


def test_ring_full_size_ring2(dev):
    """The measured size (512 rings of 2000 particles, 500 steps, FP32 paths)
    in the launch configuration the benchmark times: J, ||g||, 16 projections
    64 sampled entries and every entry of g against the oracle values of
    tests/golden/full_ring2_it0.json and full_ring2_it0_g.npz (written by
    tests/golden/make_full_size.py);
    per-particle states, adjoints and costs of the first and the last two rings
    against the oracle here."""
    import torch
    gd = golden("ring2")
    w = wl.ring_config("ring2")
    p = w.problem
    say("ring full size ring2", w.M, p.np, p.N)
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
    en, ee = assert_grad(g, *golden_g("ring2"), tol["g"])
    say(f"   g vs oracle: normwise {en:.2e}, per entry {ee:.2e}")
    for r0 in (0, w.M - 2):
        cnt = 2 * p.np
        dp, dd = eng.path_dump(r0 * p.np, cnt)
        eng.forward(mu, it=0, dump=dp)
        eng.adjoint(mu, it=0, dump=dp)
        torch.cuda.synchronize()
        z, lam, _, _, C = ref.fb_paths(p, w.seed, 0, r0, 2, mu)
        zg = np.transpose(dd["X"].double().cpu().numpy(), (2, 0, 1))
        lg = np.transpose(dd["lam"].double().cpu().numpy(), (2, 0, 1))
        e_z, e_l = per_path_error(zg, z), per_path_error(lg[:, 1:], lam[:, 1:])
        say(f"   rings {r0}+2: z {e_z:.2e} lam {e_l:.2e}")
        assert e_z <= tol["path"] and e_l <= tol["path"]
        e_c = float(np.max(np.abs(dd["cost"].cpu().numpy() - C) / (np.abs(C) + np.sqrt(np.mean(C * C)))))
        assert e_c <= tol["path"]


def test_ring_stored_jump_counts(dev):
    """Rings of 300 across a workgroup's 256-slot groups: the stored jump
    counts, addressed by slot as the header states, equal the oracle's."""
    p, M, seed = _ring("ring300")
    mu = wl.random_feedback_control(p, 4, 0.5)
    eng = B.FbEngine(p, M=M, seed=seed, precision="fp32", device=dev)
    eng.forward(mu, it=1)
    import torch
    torch.cuda.synchronize()
    _, _, _, n_ref, _ = ref.fb_paths(p, seed, 1, 0, M, mu)
    assert n_ref.sum() > 0
    T = eng.nblk * (p.N + 1) * 2 * 256
    cb = eng.traj.view(torch.uint8)[T * 4:].cpu().numpy()
    s = eng.slots()
    k = np.arange(p.N)
    got = cb[((s[:, None] // 256) * p.N + k[None, :]) * 256 + (s[:, None] % 256)]
    np.testing.assert_array_equal(got, n_ref)
