"""Parity of the HIP path with the FP64 oracle, element by element, on the same
seeded inputs and the same counter-based draws (all calls go through the C ABI).

Sizes are such that the oracle finishes in seconds while the GPU grid still
spans several blocks and a ragged last block.  Every case is printed (and
flushed) before its GPU work starts."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

from parity_util import (TOL, assert_grad, dump_to_paths, gpu_device, grad_errors, per_path_error,
                         rel_err)

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


# ---------------------------------------------------------------- draws
def test_philox_words_bitwise(dev):
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    for seed in (0, 1, 0xA4093822299F31D0, 2**64 - 1):
        say("philox", hex(seed))
        gpu = B.philox(seed, ctr, device=dev)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        mine = ref.philox(ctr[:256], key)
        np.testing.assert_array_equal(gpu[:256], mine)
    # the published known answers through the GPU path
    kat = np.array([[0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344]], np.uint32)
    out = B.philox(0x299f31d0a4093822, kat, device=dev)
    assert [hex(x) for x in out[0]] == ["0xd16cfe09", "0x94fdcceb", "0x5001e420", "0x24126ea1"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("d,lam", [(1, 2.0), (2, 10.0), (3, 5.0), (8, 3.0), (1, 0.0)])
def test_draws_match_oracle(dev, precision, d, lam):
    say("draws", precision, d, lam)
    p = wl.general_problem(d, 200, seed=d, lam=lam, T=1.0)
    eng = B.Engine(p, M=1000, seed=12345, precision=precision, device=dev)
    zw, zj, n = eng.draws(m0=100, mc=300, k0=5, kc=150, it=7)
    rzw, rzj, rn = ref.draws(12345, 7, d, lam * p.dt, 100, 300, 5, 150)
    np.testing.assert_array_equal(n.cpu().numpy(), rn)
    if lam > 0:
        assert rn.sum() > 0
    for g, r in ((zw, rzw), (zj, rzj)):
        g = g.double().cpu().numpy()
        err = np.abs(g - r) / np.maximum(1.0, np.abs(r))
        # FP32: a few ulp of |Z| <= 5.8 after the log / sqrt / sincospi chain
        assert err.max() <= (2e-6 if precision == "fp32" else 1e-14), err.max()


# ---------------------------------------------------------------- sweeps
def _cases():
    c1 = wl.config("c1")
    c2 = wl.scaled(wl.config("c2"), M=3001)
    c3 = wl.scaled(wl.config("c3"), M=1500)
    c4 = wl.scaled(wl.config("c4"), M=777)
    gen3 = wl.Workload(wl.general_problem(3, 120, seed=5, cubic=0.1, lam=6.0), M=1300, seed=9)
    gen5 = wl.Workload(wl.general_problem(5, 64, seed=6, cubic=0.05, lam=2.0), M=513, seed=10)
    return {"c1": (c1, 50), "c2": (c2, 32), "c3": (c3, 64), "c4": (c4, 64), "gen3": (gen3, 16),
            "gen5": (gen5, 8)}


CASES = _cases()


@pytest.fixture(scope="module")
def oracle_runs():
    """Oracle per-path data and (J, g) per case and iteration word (cached)."""
    cache = {}

    def get(name, it, u):
        key = (name, it, u.tobytes())
        if key not in cache:
            w, _ = CASES[name]
            p = w.problem
            X, lam, C = ref.paths(p, w.seed, it, 0, w.M, u)
            J, g = ref.cost_grad(p, w.M, w.seed, it, u)
            s = ref.grad_scale(p, w.M, w.seed, it, u)
            cache[key] = (X, lam, C, J, g, s)
        return cache[key]

    return get


def _control(p, name):
    return np.zeros((p.N, p.d)) if name in ("c1", "c2") else wl.random_control(p, 3, 0.3)


@pytest.mark.parametrize("noise", ["table", "inline"])
@pytest.mark.parametrize("mode", ["store", "recompute"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_cost_grad_and_paths(dev, oracle_runs, name, precision, mode, noise):
    w, K = CASES[name]
    p = w.problem
    say(name, precision, mode, noise, f"M={w.M} N={p.N} d={p.d} K={K}")
    u = _control(p, name)
    it = 3
    X, lam, C, J_ref, g_ref, s_ref = oracle_runs(name, it, u)
    eng = B.Engine(p, M=w.M, seed=w.seed, precision=precision, mode=mode, K=K, device=dev,
                   noise=noise)
    tol = TOL[precision]
    # forward with per-path cost dump
    dp, dumps = eng.path_dump(0, w.M)
    J = eng.forward(u, it=it, dump=dp)
    eng.adjoint(u, it=it, dump=dp)
    Jc, gc = eng.cost_grad(u, it=it)
    import torch
    torch.cuda.synchronize()
    assert eng.check_finite()
    Xg = dump_to_paths(dumps["X"], w.M)
    Lg = dump_to_paths(dumps["lam"], w.M)
    e_x = per_path_error(Xg, X[:, 1:, :])
    e_l = per_path_error(Lg, lam[:, 1:, :])
    e_c = float(np.max(np.abs(dumps["cost"].cpu().numpy() - C) / np.abs(C)))
    e_J = rel_err(float(J), J_ref)
    e_J2 = rel_err(float(Jc), J_ref)
    e_g, e_ge = grad_errors(gc.cpu().numpy(), g_ref, s_ref)
    say(f"   errors: X {e_x:.2e} lam {e_l:.2e} C {e_c:.2e} J {e_J:.2e} g {e_g:.2e} "
        f"(per entry {e_ge:.2e})")
    assert e_x <= tol["path"]
    assert e_l <= tol["path"]
    assert e_c <= tol["path"]
    assert e_J <= tol["J"] and e_J2 <= tol["J"]
    assert e_g <= tol["g"] and e_ge <= tol["g"]
    if mode == "store":
        traj = eng.trajectory().double().cpu().numpy()  # (N, d, M)
        assert per_path_error(np.transpose(traj, (2, 0, 1)), X[:, 1:, :]) <= tol["path"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["c2", "c4", "gen3", "gen5"])
def test_store_and_recompute_bitwise_equal(dev, name, precision):
    w, K = CASES[name]
    p = w.problem
    say("bitwise", name, precision, K)
    u = _control(p, name)
    a = B.Engine(p, M=w.M, seed=w.seed, precision=precision, mode="store", device=dev)
    b = B.Engine(p, M=w.M, seed=w.seed, precision=precision, mode="recompute", K=K, device=dev)
    Ja, ga = a.cost_grad(u, it=1)
    Jb, gb = b.cost_grad(u, it=1)
    assert float(Ja) == float(Jb)
    assert np.array_equal(ga.cpu().numpy(), gb.cpu().numpy())


@pytest.mark.parametrize("name", ["c2", "gen3"])
def test_repeatable_bitwise(dev, name):
    w, K = CASES[name]
    p = w.problem
    say("repeat", name)
    eng = B.Engine(p, M=w.M, seed=w.seed, precision="fp32", mode="recompute", K=K, device=dev)
    u = _control(p, name)
    J1, g1 = eng.cost_grad(u, it=4)
    J1, g1 = float(J1), g1.cpu().numpy()
    J2, g2 = eng.cost_grad(u, it=4)
    assert J1 == float(J2) and np.array_equal(g1, g2.cpu().numpy())
    J3, _ = eng.cost_grad(u, it=5)
    assert float(J3) != J1


# ---------------------------------------------------------------- edges
EDGE = [
    # (label, d, N, M, K)
    ("one path", 1, 50, 1, 7),
    ("one block minus one", 2, 40, 255, 8),
    ("one block plus one", 4, 33, 257, 5),
    ("one step", 3, 1, 300, 1),
    ("two steps", 8, 2, 300, 2),
    ("K = N", 1, 64, 600, 64),
    ("K = 1", 2, 30, 400, 1),
    ("K not dividing N", 8, 70, 300, 64),
    ("d = 6 padded", 6, 45, 700, 9),
    ("d = 7 padded", 7, 25, 260, 25),
]


@pytest.mark.parametrize("label,d,N,M,K", EDGE)
@pytest.mark.parametrize("mode", ["store", "recompute"])
def test_edge_shapes(dev, label, d, N, M, K, mode):
    say("edge", label, mode)
    p = wl.general_problem(d, N, seed=100 + d + N, cubic=0.07, lam=min(4.0, 1.5 * N))
    u = wl.random_control(p, 8, 0.2)
    eng = B.Engine(p, M=M, seed=77, precision="fp32", mode=mode, K=K, device=dev)
    dp, dumps = eng.path_dump(0, M)
    eng.forward(u, it=2, dump=dp)
    eng.adjoint(u, it=2, dump=dp)
    J, g = eng.cost_grad(u, it=2)
    X, lam, C = ref.paths(p, 77, 2, 0, M, u)
    J_ref, g_ref = ref.cost_grad(p, M, 77, 2, u)
    s_ref = ref.grad_scale(p, M, 77, 2, u)
    tol = TOL["fp32"]
    assert per_path_error(dump_to_paths(dumps["X"], M), X[:, 1:, :]) <= tol["path"]
    assert per_path_error(dump_to_paths(dumps["lam"], M), lam[:, 1:, :]) <= tol["path"]
    assert rel_err(float(J), J_ref) <= tol["J"]
    assert_grad(g.cpu().numpy(), g_ref, s_ref, tol["g"])


def test_zero_rate_and_zero_noise(dev):
    """lam = 0 and s = 0: every path is the deterministic Euler path."""
    p = wl.general_problem(3, 50, seed=4, lam=0.0)
    p = dataclasses.replace(p, s=np.zeros(3))
    u = wl.random_control(p, 2, 0.5)
    eng = B.Engine(p, M=500, seed=3, precision="fp64", device=dev)
    dp, dumps = eng.path_dump(0, 500)
    eng.forward(u, it=0, dump=dp)
    eng.adjoint(u, it=0, dump=dp)
    X = dump_to_paths(dumps["X"], 500)
    assert np.all(X == X[:1])
    from oracle import closed_form as cf
    np.testing.assert_allclose(X[0], cf.deterministic_path(p, u)[1:], rtol=1e-12, atol=1e-13)


def test_nonfinite_flag(dev):
    """A divergent cubic drift overflows: the reduction raises the flag."""
    p = wl.general_problem(1, 200, seed=1, cubic=-50.0, lam=0.0)
    p = dataclasses.replace(p, x0=np.array([3.0]), T=5.0)
    eng = B.Engine(p, M=300, seed=1, precision="fp32", device=dev)
    eng.cost_grad(np.zeros((p.N, 1)), it=0)
    assert not eng.check_finite()
    assert eng.check_finite()  # the flag clears once read


# ---------------------------------------------------------------- segment recompute, rate limit
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_segment_recompute_many_groups_per_block(dev, precision):
    """d = 8 with checkpoints every 24 steps runs the persistent segment
    kernel; 2^19 + 77 paths make 2049 groups of 256, more than the blocks
    resident at once, so blocks sweep several groups; K = 24 does not divide
    N = 60 and the last segment is short.  Bitwise equal to the stored
    variant, and J, g against the oracle."""
    import torch
    p = wl.general_problem(8, 60, seed=31, cubic=0.05, lam=3.0)
    M = (1 << 19) + 77
    u = wl.random_control(p, 4, 0.3)
    say("segment recompute", precision, M)
    a = B.Engine(p, M=M, seed=7, precision=precision, mode="store", device=dev)
    Ja, ga = a.cost_grad(u, it=1)
    Ja, ga = float(Ja), ga.cpu().numpy()
    del a
    torch.cuda.empty_cache()
    b = B.Engine(p, M=M, seed=7, precision=precision, mode="recompute", K=24, device=dev)
    Jb, gb = b.cost_grad(u, it=1)
    assert float(Jb) == Ja and np.array_equal(gb.cpu().numpy(), ga)
    J_ref, g_ref = ref.cost_grad(p, M, 7, 1, u)
    s_ref = ref.grad_scale(p, M, 7, 1, u)
    tol = TOL[precision]
    assert rel_err(Ja, J_ref) <= tol["J"]
    en, ee = assert_grad(ga, g_ref, s_ref, tol["g"])
    say(f"   J {rel_err(Ja, J_ref):.2e} g {en:.2e} (per entry {ee:.2e})")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_rate_at_the_abi_limit(dev, precision):
    """lambda dt = 2, the largest rate the ABI takes: counts reach deep into
    the threshold table; the draws (counts bit-exact) and a full sweep against
    the oracle, stored and recomputed."""
    p = wl.general_problem(4, 100, seed=8, cubic=0.05, lam=200.0, T=1.0)
    assert p.lam * p.dt == pytest.approx(2.0)
    say("rate limit", precision)
    eng = B.Engine(p, M=3000, seed=21, precision=precision, device=dev)
    _, _, n = eng.draws(m0=0, mc=3000, k0=0, kc=100, it=5)
    _, _, rn = ref.draws(21, 5, p.d, p.lam * p.dt, 0, 3000, 0, 100)
    n = n.cpu().numpy()
    np.testing.assert_array_equal(n, rn)
    assert n.max() >= 9 and abs(n.mean() - 2.0) < 0.02
    u = wl.random_control(p, 5, 0.3)
    J_ref, g_ref = ref.cost_grad(p, 3000, 21, 5, u)
    s_ref = ref.grad_scale(p, 3000, 21, 5, u)
    tol = TOL[precision]
    for mode, K in (("store", 0), ("recompute", 16)):
        e = B.Engine(p, M=3000, seed=21, precision=precision, mode=mode, K=K, device=dev)
        J, g = e.cost_grad(u, it=5)
        assert e.check_finite()
        assert rel_err(float(J), J_ref) <= tol["J"]
        assert_grad(g.cpu().numpy(), g_ref, s_ref, tol["g"], f"{mode}")


@pytest.mark.parametrize("d,mode,K", [(1, "store", 0), (1, "recompute", 16), (2, "store", 0),
                                      (8, "store", 0), (8, "recompute", 64)])
def test_sweeps_without_cubic_term_are_bitwise_the_term_times_zero(dev, d, mode, K):
    """The sweeps are compiled without the cubic term when c3 = 0.  A cubic
    coefficient of 1e-300 is non-zero on the host, so it takes the
    instantiation with the term, but it rounds to 0 in FP32: the term then
    adds -0 * X^3, and every bit of J, g and the paths must equal the run
    without it."""
    say("cubic term compiled out", d, mode, K)
    base = wl.general_problem(d, 96, seed=40 + d, cubic=0.0, lam=3.0)
    tiny = dataclasses.replace(base, cubic=1e-300)
    out = []
    for p in (base, tiny):
        eng = B.Engine(p, M=700, seed=3, precision="fp32", mode=mode, K=K, device=dev)
        dp, dd = eng.path_dump(0, 700)
        J, g = eng.cost_grad(np.zeros((p.N, p.d)), it=2)
        eng.forward(np.zeros((p.N, p.d)), it=2, dump=dp)
        eng.adjoint(np.zeros((p.N, p.d)), it=2, dump=dp)
        out.append((float(J), g.cpu().numpy(), dd["X"].cpu().numpy(), dd["lam"].cpu().numpy()))
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1:], out[1][1:]):
        np.testing.assert_array_equal(a, b)


# (label, d, N, M, K, cubic): N on both sides of the table's register tile
# (16 / padded d steps), ragged blocks, padded dimensions
NOISE_SHAPES = [
    ("d1 one path", 1, 50, 1, 7, 0.07),
    ("d1 N = tile", 1, 16, 300, 4, 0.0),
    ("d1 N = tile + 1", 1, 17, 513, 17, 0.07),
    ("d2 one step", 2, 1, 255, 1, 0.07),
    ("d3 ragged", 3, 37, 1300, 9, 0.1),
    ("d4 two tiles", 4, 8, 257, 3, 0.0),
    ("d6 padded", 6, 45, 700, 9, 0.05),
    ("d8 N = 2 tiles + 1", 8, 5, 300, 5, 0.07),
    ("d8 c4-like", 8, 64, 600, 16, 0.0),
    # the sweeps copy the per-step table into LDS 16 KB at a time: 128 steps
    # at d = 8 in FP64 (256 in FP32), 256 at d = 3 (FP64), 1024 at d = 1 (FP64)
    ("d8 three table chunks", 8, 300, 257, 32, 0.05),
    ("d3 two table chunks", 3, 300, 200, 50, 0.1),
    ("d1 two table chunks", 1, 1100, 300, 64, 0.0),
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("mode", ["store", "recompute"])
@pytest.mark.parametrize("label,d,N,M,K,cubic", NOISE_SHAPES)
def test_noise_table_is_bitwise_the_inline_draws(dev, label, d, N, M, K, cubic, mode, precision):
    """The forward sweeps read the iteration's draws from the noise table or
    compute them in the sweep; every bit of J, g, the per-path states, adjoints
    and costs and the stored trajectory must agree."""
    say("noise table", label, mode, precision)
    p = wl.general_problem(d, N, seed=200 + d + N, cubic=cubic, lam=min(5.0, 2.0 * N))
    u = wl.random_control(p, 4, 0.3)
    out = []
    for noise in ("table", "inline"):
        eng = B.Engine(p, M=M, seed=11, precision=precision, mode=mode, K=K, device=dev,
                       noise=noise)
        dp, dd = eng.path_dump(0, M)
        J, g = eng.cost_grad(u, it=6)
        Jf = eng.forward(u, it=6, dump=dp)
        eng.adjoint(u, it=6, dump=dp)
        Jf2 = eng.forward(u, it=6, store=False)
        out.append((float(J), float(Jf), float(Jf2), g.cpu().numpy(), dd["X"].cpu().numpy(),
                    dd["lam"].cpu().numpy(), dd["cost"].cpu().numpy(),
                    eng.trajectory().cpu().numpy()))
    a, b = out
    assert a[:3] == b[:3]
    for x, y in zip(a[3:], b[3:]):
        np.testing.assert_array_equal(x, y)
