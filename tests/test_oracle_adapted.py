"""Pins of the oracle's jump-adapted grid (Section 3 of Bartsch, Borzi,
Ciaramella, Reichle, arXiv 2505.04328: the grid is the union of the uniform
points and each particle's jump times, integrated with Euler between them and
the jump law at the jump times, Algorithms 5.1-5.2), each against something
other than the oracle's own formulas:

* jump times: the gaps between consecutive jumps of one particle, across
  uniform intervals, follow the exponential law of the paper's sampling rule
  (mean 1/sigma, Kolmogorov-Smirnov against Exp(sigma)), and the counts per
  interval are Poisson(sigma dtau);
* with no jumps (beta tiny) the adapted grid is the (separately pinned) fixed
  grid, bit for bit;
* free flight (no spring, noise or control): between jumps the velocity is
  constant, so the position at every uniform point and jump time has a closed
  form from the jump times and jump normals alone, and so has the cost's
  quadrature over the sub-steps;
* the adjoint gradient agrees with central differences of J and with the
  forward-mode tangent, with several jumps per interval, noise, gamma = 0.9, a
  moving target and the ellipse cost.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ref
from paper_2505_04328_amd import workloads as wl


def _adapted(**kw):
    kw.setdefault("grid", "adapted")
    return wl.feedback_problem(**kw)


def test_jump_times_have_exponential_gaps():
    """One particle over 400 intervals of length 1: sigma = sqrt(beta/pi)."""
    p = _adapted(N=400, T=400.0, beta=10.0)
    sigma = math.sqrt(p.beta / math.pi)
    gaps, counts, offs = [], [], []
    for m in range(6):
        last = None
        for k in range(p.N):
            n, a, Z, S = ref.fb_adapted_draws(p, 3, m, k, 1)
            counts.append(n)
            assert a[0] == 0.0 and a[-1] == 1.0 and np.all(np.diff(a) >= 0.0)
            for r in range(1, n + 1):
                t = k * p.dt + a[r] * p.dt
                offs.append(a[r])
                if last is not None:
                    gaps.append(t - last)
                last = t
    gaps = np.array(gaps)
    counts = np.array(counts)
    assert abs(gaps.mean() * sigma - 1.0) < 4.0 / math.sqrt(len(gaps))
    assert stats.kstest(gaps, "expon", args=(0, 1.0 / sigma)).pvalue > 1e-3
    assert abs(counts.mean() - sigma * p.dt) < 4.0 * math.sqrt(sigma * p.dt / len(counts))
    assert abs(counts.var() / (sigma * p.dt) - 1.0) < 0.15
    assert stats.kstest(np.array(offs), "uniform").pvalue > 1e-3


def test_adapted_normals_are_standard():
    p = _adapted(N=200, T=200.0, beta=10.0)
    zs, ss = [], []
    for m in range(4):
        for k in range(p.N):
            n, a, Z, S = ref.fb_adapted_draws(p, 5, m, k, 0)
            zs.append(Z.reshape(-1))
            ss.append(S)
    zs, ss = np.concatenate(zs), np.concatenate(ss)
    for x in (zs, ss):
        assert abs(x.mean()) < 4.0 / math.sqrt(len(x))
        assert abs(x.std() - 1.0) < 0.05
    assert stats.kstest(ss, "norm").pvalue > 1e-3


@pytest.mark.parametrize("cost", ["track", "ellipse"])
def test_adapted_without_jumps_is_the_fixed_grid(cost):
    kw = dict(N=20, T=2.0, beta=1e-12, alpha=0.2, cost=cost, zd=np.tile([0.3, -0.2], (21, 1)))
    fixed = wl.feedback_problem(**kw)
    adapted = _adapted(**kw)
    mu = wl.random_feedback_control(fixed, 3, 0.5)
    a = ref.fb_paths(adapted, 4, 2, 0, 200, mu)
    f = ref.fb_paths(fixed, 4, 2, 0, 200, mu)
    assert a[3].sum() == 0
    for x, y in zip(a, f):
        np.testing.assert_array_equal(x, y)
    Ja, ga = ref.fb_cost_grad(adapted, 300, 4, 2, mu)
    Jf, gf = ref.fb_cost_grad(fixed, 300, 4, 2, mu)
    assert Ja == Jf
    np.testing.assert_array_equal(ga, gf)


def test_free_flight_closed_form():
    """eta = 0, no noise, no control: v is piecewise constant, jumping to
    gamma v + S / sqrt(2 beta) at each jump time; x integrates it exactly."""
    N, T = 30, 6.0
    zd = np.stack([np.linspace(0.0, 1.0, N + 1), np.linspace(0.5, -0.5, N + 1)], axis=1)
    p = _adapted(N=N, T=T, eta=0.0, b1=0.0, b2=0.0, beta=6.0, gamma=0.7, alpha=0.0,
                 init="gauss", z0=(0.2, 0.9), s0=(0.0, 0.0), zd=zd, sigJ=0.6)
    mu = np.zeros((p.N, p.L))
    M = 20
    z, _, _, n, C = ref.fb_paths(p, 8, 0, 0, M, mu)
    assert n.sum() > 2 * M
    dt = p.dt
    for m in range(M):
        x, v = 0.2, 0.9
        cost = 0.0
        for k in range(N):
            nk, a, _, S = ref.fb_adapted_draws(p, 8, m, k, 0)
            assert nk == n[m, k]
            assert abs(z[m, k, 0] - x) <= 1e-12 and abs(z[m, k, 1] - v) <= 1e-12
            for r in range(nk + 1):
                h = (a[r + 1] - a[r]) * dt
                x = x + h * v
                if r < nk:
                    v = p.gamma * v + S[r] / math.sqrt(2.0 * p.beta)
                frac = a[r + 1]
                tgt = (1.0 - frac) * zd[k] + frac * zd[k + 1]
                cost += h * -math.exp(-((x - tgt[0]) ** 2 + (v - tgt[1]) ** 2) / (2 * 0.36))
        assert abs(z[m, N, 0] - x) <= 1e-12 and abs(z[m, N, 1] - v) <= 1e-12
        assert abs(C[m] - cost) <= 1e-12 * abs(cost)


def _grad_case(cost):
    N, T = 12, 3.0
    t = np.arange(N + 1) * (T / N)
    zd = np.stack([0.5 * np.sin(t), 0.3 * np.cos(2 * t)], axis=1)
    return _adapted(N=N, T=T, beta=10.0, gamma=0.9, alpha=0.3, b1=0.1, b2=0.2, cost=cost,
                    zd=zd, sigJ=0.5, init="gauss", s0=(0.3, 0.3), z0=(0.2, -0.1))


@pytest.mark.parametrize("cost", ["track", "ellipse"])
def test_adapted_gradient_matches_differences_and_tangent(cost):
    p = _grad_case(cost)
    mu = wl.random_feedback_control(p, 13, 0.5)
    M, seed, it = 60, 6, 1
    _, _, _, n, _ = ref.fb_paths(p, seed, it, 0, M, mu)
    assert n.sum() > M and n.max() >= 2
    J, g = ref.fb_cost_grad(p, M, seed, it, mu)
    rng = np.random.default_rng(9)
    h = 1e-5
    for _ in range(3):
        d = rng.normal(size=mu.shape)
        Jp, _ = ref.fb_cost_grad(p, M, seed, it, mu + h * d, grad=False)
        Jm, _ = ref.fb_cost_grad(p, M, seed, it, mu - h * d, grad=False)
        fd = (Jp - Jm) / (2 * h)
        adj = p.dt * float(np.sum(g * d))
        tan = ref.fb_tangent(p, M, seed, it, mu, d)
        assert abs(adj - fd) <= 1e-6 * abs(fd), (adj, fd)
        assert abs(tan - fd) <= 1e-6 * abs(fd), (tan, fd)
        assert abs(adj - tan) <= 1e-11 * abs(tan), (adj, tan)


def test_adapted_adjoint_terminal_and_uniform_points():
    """lam_N = d_last grad Jt(z_N), d_last the length of the last sub-step."""
    p = _grad_case("track")
    mu = wl.random_feedback_control(p, 2, 0.5)
    z, lam, _, n, _ = ref.fb_paths(p, 3, 0, 0, 40, mu)
    for m in range(40):
        nk, a, _, _ = ref.fb_adapted_draws(p, 3, m, p.N - 1, 0)
        dl = (1.0 - a[nk]) * p.dt
        rx, rv = z[m, -1] - p.zd[-1]
        e = math.exp(-(rx * rx + rv * rv) / (2 * p.sigJ ** 2)) / p.sigJ ** 2
        np.testing.assert_allclose(lam[m, -1], [dl * rx * e, dl * rv * e], rtol=1e-13, atol=1e-16)


def test_position_noise_is_brownian_at_the_uniform_points():
    """No spring, control or velocity noise: x with b1 > 0 minus x with b1 = 0
    (same draws) is b1 times a Brownian motion sampled at the uniform points,
    however the jumps split the intervals: increments N(0, b1^2 dtau)."""
    kw = dict(N=40, T=40.0, eta=0.0, b2=0.0, beta=10.0, alpha=0.0, init="gauss",
              s0=(0.0, 0.0), z0=(0.0, 0.5))
    noisy, quiet = _adapted(b1=0.3, **kw), _adapted(b1=0.0, **kw)
    mu = np.zeros((noisy.N, noisy.L))
    zn, _, _, n, _ = ref.fb_paths(noisy, 2, 0, 0, 150, mu)
    zq, _, _, _, _ = ref.fb_paths(quiet, 2, 0, 0, 150, mu)
    assert n.mean() > 1.0
    inc = np.diff(zn[:, :, 0] - zq[:, :, 0], axis=1).reshape(-1) / (0.3 * math.sqrt(noisy.dt))
    assert abs(inc.mean()) < 4.0 / math.sqrt(len(inc))
    assert abs(inc.var() - 1.0) < 0.06
    assert stats.kstest(inc, "norm").pvalue > 1e-3
