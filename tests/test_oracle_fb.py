"""Pins of the FP64 oracle for the paper's model problem (oracle/fb_oracle.c):
the controlled oscillator with Keilson-Storer velocity jumps and radial-basis
feedback (Section 5, model equation, shape functions, jump process; Section 6).

Each pin checks the oracle against something other than itself: special values
of the bump (eq. Gaussian_RBF) and its derivative by central differences; the
exact mean / second-moment recursions of the uncontrolled dynamics
(closed_form.fb_moments); which grid points the cost covers (targets placed far
away except at one step); the control's index structure (a single non-zero
coefficient against the paper's cell-centre formula, Section 5,
discretization); central differences of J under common random numbers and the
tangent-linear duality for the adjoint and the gradient (Section 4,
eq. definition_Gradient); a replay of the Armijo iteration (Algorithm 5.4); and
for the surrogate gradient of Section 6.5, the law of the surrogate states, the
exact gradient recovered when the surrogate states land on a particle's own
path, and the one-step definition.
"""
import math

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import ref
from paper_2505_04328_amd import workloads as wl


def small_problem(**kw):
    base = dict(N=20, T=2.0, nx=6, nv=6, alpha=0.1, sigJ=0.7, b1=0.1, b2=0.2, gamma=0.8, beta=10.0)
    base.update(kw)
    zd = kw.pop("zd", None)
    N = base["N"]
    if zd is None:
        t = np.arange(N + 1) * (base["T"] / N)
        zd = np.stack([0.3 * np.cos(t), -0.2 * np.sin(t)], axis=1)
    base["zd"] = zd
    return wl.feedback_problem(**base)


# ---------------------------------------------------------------- bump
def test_bump_special_values():
    assert ref.fb_bump(0.0, 0.5) == pytest.approx(math.exp(-1.0), rel=1e-15)
    # eps |r| = 1/2: exp(-1/(1 - 1/4)) = exp(-4/3)
    assert ref.fb_bump(1.0, 0.5) == pytest.approx(math.exp(-4.0 / 3.0), rel=1e-15)
    assert ref.fb_bump(-1.0, 0.5) == ref.fb_bump(1.0, 0.5)
    for r in (2.0, -2.0, 2.5, 17.0):
        assert ref.fb_bump(r, 0.5) == 0.0
        assert ref.fb_bump_deriv(r, 0.5) == 0.0
    assert ref.fb_bump_deriv(0.0, 0.5) == 0.0


@pytest.mark.parametrize("eps", [0.5, 1.3])
def test_bump_derivative_by_differences(eps):
    h = 1e-6
    for r in np.linspace(-0.97 / eps, 0.97 / eps, 41):
        fd = (ref.fb_bump(r + h, eps) - ref.fb_bump(r - h, eps)) / (2 * h)
        d = ref.fb_bump_deriv(r, eps)
        assert abs(fd - d) <= 1e-7 * max(1.0, abs(d)), (r, fd, d)


# ---------------------------------------------------------------- dynamics
@pytest.mark.parametrize("init", ["gauss", "uniform"])
def test_uncontrolled_moments(init):
    """mu = 0: sample means and raw second moments of (x, v) against the exact
    recursions, within 5 standard errors, at several steps including k = 0."""
    p = wl.feedback_problem(N=50, T=5.0, init=init, b1=0.4, b2=0.4)
    M = 20000
    z, _, _, n, _ = ref.fb_paths(p, 3, 0, 0, M, np.zeros((p.N, p.L)))
    ref_m = cf.fb_moments(p)
    for k in (0, 1, 5, 25, 50):
        x, v = z[:, k, 0], z[:, k, 1]
        for q, samp in enumerate((x, v, x * x, x * v, v * v)):
            se = samp.std(ddof=1) / math.sqrt(M)
            assert abs(samp.mean() - ref_m[k, q]) <= 5 * se + 1e-12, (init, k, q, samp.mean(), ref_m[k, q], se)
    lam = p.rate * p.dt
    assert abs(n.mean() - lam) <= 5 * math.sqrt(lam / n.size)


def test_jump_counts_are_poisson():
    p = wl.feedback_problem(N=50, T=5.0)
    _, _, _, n, _ = ref.fb_paths(p, 5, 2, 0, 4000, np.zeros((p.N, p.L)))
    lam = p.rate * p.dt
    counts = np.bincount(n.ravel(), minlength=6)[:4]
    total = n.size
    exp = np.array([math.exp(-lam) * lam ** j / math.factorial(j) for j in range(4)]) * total
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert chi2 < 25.0, (counts, exp)


# ---------------------------------------------------------------- cost
def test_tracking_cost_covers_steps_1_to_N():
    """Targets far away everywhere except one step: with the target only at
    t_N the cost is dt E[-exp(...)] < 0; with it only at t_0 the cost is 0."""
    p0 = wl.feedback_problem(N=20, T=2.0)
    far = np.full((p0.N + 1, 2), 1e3)
    only_N = far.copy()
    only_N[-1] = (0.0, 0.0)
    only_0 = far.copy()
    only_0[0] = (0.75, 0.75)
    mu = np.zeros((p0.N, p0.L))
    J_N, _ = ref.fb_cost_grad(wl.feedback_problem(N=20, T=2.0, zd=only_N), 2000, 1, 0, mu, grad=False)
    J_0, _ = ref.fb_cost_grad(wl.feedback_problem(N=20, T=2.0, zd=only_0), 2000, 1, 0, mu, grad=False)
    assert J_N < -0.1 * p0.dt
    assert J_0 == 0.0


def test_control_cost_identity():
    """With the targets out of reach the cost is dt alpha/2 sum_k u_k^2 per path,
    the controls being the ones the oracle reports."""
    p = wl.feedback_problem(N=20, T=2.0, zd=np.full((21, 2), 1e3), alpha=0.3)
    mu = wl.random_feedback_control(p, 4, 1.0)
    _, _, u, _, C = ref.fb_paths(p, 2, 1, 0, 64, mu)
    np.testing.assert_allclose(C, p.dt * 0.5 * p.alpha * np.sum(u * u, axis=1), rtol=1e-13)
    J, _ = ref.fb_cost_grad(p, 64, 2, 1, mu, grad=False)
    assert J == pytest.approx(C.mean(), rel=1e-13)


@pytest.mark.parametrize("i0,l0", [(1, 4), (3, 0)])
def test_control_index_structure(i0, l0):
    """A single non-zero coefficient (i0, l0): u = mu b(x - x^{i0}) b(v - v^{l0})
    with the cell centres x^i = (i - 1/2) dx - xmax (1-based i), dx = 2 xmax/nx."""
    p = wl.feedback_problem(N=10, T=1.0, nx=5, nv=7, xmax=2.0, vmax=3.0, eps=0.6, init="uniform")
    mu = np.zeros((p.N, p.L))
    mu[:, i0 * p.nv + l0] = 1.7
    z, _, u, _, _ = ref.fb_paths(p, 6, 0, 0, 50, mu)
    xc = (i0 + 0.5) * (2 * p.xmax / p.nx) - p.xmax
    vc = (l0 + 0.5) * (2 * p.vmax / p.nv) - p.vmax
    for m in range(50):
        for k in range(p.N):
            want = 1.7 * ref.fb_bump(z[m, k, 0] - xc, p.eps) * ref.fb_bump(z[m, k, 1] - vc, p.eps)
            assert u[m, k] == pytest.approx(want, rel=1e-13, abs=1e-300)


def test_cost_independent_of_threads():
    p = small_problem()
    mu = wl.random_feedback_control(p, 1, 0.8)
    a = ref.fb_cost_grad(p, 9000, 3, 2, mu, nthreads=1)
    b = ref.fb_cost_grad(p, 9000, 3, 2, mu, nthreads=5)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- adjoint
def _directions(p, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = rng.normal(size=(p.N, p.L))
        out.append(d / math.sqrt(p.dt * np.sum(d * d)))
    return out


@pytest.mark.parametrize("gamma", [0.8, -0.5])
def test_gradient_by_central_differences(gamma):
    """J is smooth in mu (the draws and jump counts do not depend on it):
    central differences under common random numbers against dt <g, delta>."""
    p = small_problem(gamma=gamma)
    M = 400
    mu = wl.random_feedback_control(p, 7, 1.0)
    _, g = ref.fb_cost_grad(p, M, 11, 4, mu)
    gn = math.sqrt(p.dt * np.sum(g * g))
    h = 1e-5
    for d in _directions(p, 6, 3):
        jp, _ = ref.fb_cost_grad(p, M, 11, 4, mu + h * d, grad=False)
        jm, _ = ref.fb_cost_grad(p, M, 11, 4, mu - h * d, grad=False)
        fd = (jp - jm) / (2 * h)
        ad = p.dt * float(np.sum(g * d))
        assert abs(fd - ad) <= 1e-6 * gn, (fd, ad, gn)


def test_tangent_adjoint_duality():
    p = small_problem()
    M = 300
    mu = wl.random_feedback_control(p, 8, 1.0)
    _, g = ref.fb_cost_grad(p, M, 2, 9, mu)
    for d in _directions(p, 4, 5):
        dJ = ref.fb_tangent(p, M, 2, 9, mu, d)
        ad = p.dt * float(np.sum(g * d))
        assert abs(dJ - ad) <= 1e-12 * max(1.0, abs(dJ)), (dJ, ad)


def test_adjoint_terminal_and_zero_row():
    p = small_problem()
    mu = wl.random_feedback_control(p, 2, 0.5)
    z, lam, _, _, _ = ref.fb_paths(p, 4, 0, 0, 8, mu)
    s2 = p.sigJ ** 2
    r = z[:, -1, :] - p.zd[-1]
    e = np.exp(-np.sum(r * r, axis=1) / (2 * s2))
    np.testing.assert_allclose(lam[:, -1, :], p.dt * r / s2 * e[:, None], rtol=1e-13)
    assert np.all(lam[:, 0, :] == 0.0)


# ---------------------------------------------------------------- iteration
def test_armijo_replay():
    """Algorithm 5.4 replayed from fb_cost_grad: iteration n uses counter n for
    the gradient and for every trial, steps along -g, accepts the first zeta in
    zeta0 rho^j with J(mu - zeta g) <= J(mu) - c zeta ||g||^2."""
    p = small_problem()
    M, seed = 600, 5
    mu0 = wl.random_feedback_control(p, 9, 0.5)
    mu_o, logs, n = ref.fb_optimize(p, M, seed, 0, mu0, n_max=3, zeta0=64.0, rho=0.5, c_armijo=0.3)
    assert n == 3
    mu = mu0.copy()
    for it in range(3):
        J, g = ref.fb_cost_grad(p, M, seed, it, mu)
        gg = p.dt * float(np.sum(g * g))
        zeta = 64.0
        for _ in range(30):
            Jt, _ = ref.fb_cost_grad(p, M, seed, it, mu - zeta * g, grad=False)
            if Jt <= J - 0.3 * zeta * gg:
                break
            zeta *= 0.5
        assert logs[it]["zeta"] == zeta
        assert logs[it]["J"] == J
        mu = mu - zeta * g
    np.testing.assert_array_equal(mu, mu_o)


def test_descent_on_the_paper_setting():
    """A few iterations on the Section 6.1 setting lower the cost on fresh draws."""
    w = wl.feedback_config("f1")
    p = w.problem
    mu, logs, n = ref.fb_optimize(p, w.M, w.seed, 0, np.zeros((p.N, p.L)), n_max=4)
    assert n == 4
    J0, _ = ref.fb_cost_grad(p, 20000, 77, 1000, np.zeros((p.N, p.L)), grad=False)
    J1, _ = ref.fb_cost_grad(p, 20000, 77, 1000, mu, grad=False)
    assert J1 < J0


# ---------------------------------------------------------------- surrogate adjoint (Section 6.5)
def test_surrogate_states_law():
    """zs_k ~ N(zd_k, diag(svar0 + svar1 t_k)), components uncorrelated, and
    one sample per particle and realization (Section 6.5): the standardised
    offset (zs_k - zd_k) / sqrt(var(t_k)) is the same at every step, and
    differs between particles and between realizations."""
    p = wl.feedback_problem(N=10, T=2.0, zd=_moving_target(10, 2.0), svar0=(0.04, 0.09),
                            svar1=(0.3, 0.05))
    M = 20000
    xi = {}
    for k in (0, 4, 10):
        zs = np.array([ref.fb_surrogate_state(p, 7, m, k, 3) for m in range(M)])
        t = k * p.dt
        var = np.array([0.04 + 0.3 * t, 0.09 + 0.05 * t])
        mean_err = np.abs(zs.mean(axis=0) - p.zd[k])
        assert np.all(mean_err <= 5 * np.sqrt(var / M)), (k, mean_err)
        v = zs.var(axis=0, ddof=1)
        assert np.all(np.abs(v - var) <= 5 * var * np.sqrt(2.0 / M)), (k, v, var)
        c = np.corrcoef(zs[:, 0], zs[:, 1])[0, 1]
        assert abs(c) <= 5 / np.sqrt(M)
        xi[k] = (zs - p.zd[k]) / np.sqrt(var)
    np.testing.assert_allclose(xi[4], xi[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(xi[10], xi[0], rtol=0, atol=1e-12)
    other = np.array([ref.fb_surrogate_state(p, 7, m, 4, 4) for m in range(200)])
    assert np.all(np.abs(other - np.array([ref.fb_surrogate_state(p, 7, m, 4, 3)
                                             for m in range(200)])).max(axis=1) > 0)


def _moving_target(N, T):
    t = np.arange(N + 1) * (T / N)
    return np.stack([0.5 * np.cos(t), -0.4 * np.sin(t)], axis=1)


@pytest.mark.parametrize("gamma", [0.8, -0.5])
def test_surrogate_on_own_path_equals_exact(gamma):
    """One particle, and a target shifted so that the surrogate states land on
    the particle's own realised path: the surrogate offsets sigma_k Z_k come
    from the counters and do not depend on the target, so with
    zd'_k = z_k - sigma_k Z_k the surrogate states are z_k while the tracking
    sources grad Jt(z_k; zd'_k) stay non-zero.  The surrogate gradient must then
    be the exact (difference-pinned) gradient.  Noise and jumps included."""
    kw = dict(gamma=gamma, b1=0.3, b2=0.4, beta=40.0, svar0=(0.05, 0.08), svar1=(0.2, 0.1))
    base = small_problem(**kw)
    mu = wl.random_feedback_control(base, 3, 1.0)
    seed, it = 5, 2
    z, _, _, n, _ = ref.fb_paths(base, seed, it, 0, 1, mu)
    assert n.sum() > 0  # the particle jumps
    zero = small_problem(zd=np.zeros((base.N + 1, 2)), **kw)
    offs = np.array([ref.fb_surrogate_state(zero, seed, 0, k, it) for k in range(base.N + 1)])
    p = small_problem(zd=z[0] - offs, **kw)
    zs = np.array([ref.fb_surrogate_state(p, seed, 0, k, it) for k in range(p.N + 1)])
    np.testing.assert_allclose(zs, z[0], rtol=0, atol=1e-14)
    J, g = ref.fb_cost_grad(p, 1, seed, it, mu)
    Js, gs = ref.fb_cost_grad_surrogate(p, 1, seed, it, mu)
    assert Js == J
    np.testing.assert_allclose(gs, g, rtol=1e-10, atol=1e-12 * np.abs(g).max())
    # the tracking sources are active: the same particle against the unshifted
    # target has a different gradient
    _, g0 = ref.fb_cost_grad(base, 1, seed, it, mu)
    assert np.abs(g0 - g).max() > 1e-3 * np.abs(g).max()


def test_surrogate_fit_matches_the_ensemble():
    """Fitted surrogate variance (Section 6.5: a variance that grows linearly
    and follows the forward model's own): the per-step variance is numpy's
    population variance of the oracle's particle states, and the line is
    numpy's least-squares fit through it."""
    p = small_problem(b1=0.3, b2=0.4, beta=40.0, svar="fit")
    mu = wl.random_feedback_control(p, 3, 1.0)
    M, seed, it = 3000, 5, 2
    var, a, b = ref.fb_surrogate_fit(p, M, seed, it, mu)
    z, _, _, n, _ = ref.fb_paths(p, seed, it, 0, M, mu)
    assert n.sum() > 0
    want = z.var(axis=0)
    np.testing.assert_allclose(var, want, rtol=1e-12, atol=1e-15)
    t = np.arange(p.N + 1) * p.dt
    for c in range(2):
        bb, aa = np.polyfit(t, want[:, c], 1)
        assert abs(b[c] - bb) <= 1e-12 * abs(bb)
        assert abs(a[c] - aa) <= 1e-12 * (abs(aa) + abs(bb) * p.T)


def test_surrogate_fit_two_points_is_their_line():
    """N = 1: the least-squares line through two points passes through both."""
    p = small_problem(N=1, T=0.5, b1=0.3, b2=0.4, svar="fit")
    mu = wl.random_feedback_control(p, 2, 1.0)
    var, a, b = ref.fb_surrogate_fit(p, 4000, 3, 1, mu)
    np.testing.assert_allclose(a, var[0], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(b, (var[1] - var[0]) / p.dt, rtol=1e-12, atol=1e-15)


def test_surrogate_fit_velocity_random_walk():
    """Closed form: without the spring, control and position noise, and with
    gamma = 1, the velocity is a random walk with Gaussian steps and jumps that
    add 1/(2 beta) each at the rate sqrt(beta/pi): Var v(t) = s0_v^2 +
    (b2^2 + sqrt(beta/pi)/(2 beta)) t exactly in expectation, so the fitted
    velocity line recovers it within the Monte Carlo error."""
    p = wl.feedback_problem(N=20, T=2.0, eta=0.0, b1=0.0, b2=0.4, beta=40.0, gamma=1.0, nx=4,
                            nv=4, s0=(0.1, 0.2), svar="fit")
    _, a, b = ref.fb_surrogate_fit(p, 50000, 5, 2, np.zeros((p.N, p.L)))
    slope = 0.4 ** 2 + math.sqrt(40.0 / math.pi) / 80.0
    assert abs(b[1] - slope) <= 0.03 * slope, (b[1], slope)
    assert abs(a[1] - 0.04) <= 0.03 * 0.04, a[1]
    # the position variance grows faster than linearly (its integral of a
    # random walk): the line through it starts below zero
    assert a[0] < 0 < b[0]


def test_surrogate_fit_gradient_is_the_given_line_at_the_fit():
    """svar_kind 1 is svar_kind 0 at the fitted line, also where the line is
    negative near t = 0 (the variance is 0 there: the surrogate state is the
    target)."""
    kw = dict(eta=0.0, b1=0.0, b2=0.4, beta=40.0, gamma=1.0, s0=(0.1, 0.2))
    pf = small_problem(svar="fit", **kw)
    mu = wl.random_feedback_control(pf, 3, 1.0)
    M, seed, it = 2000, 4, 1
    _, a, b = ref.fb_surrogate_fit(pf, M, seed, it, mu)
    assert a[0] < 0
    pg = small_problem(svar0=a, svar1=b, **kw)
    Jf, gf = ref.fb_cost_grad_surrogate(pf, M, seed, it, mu)
    Jg, gg = ref.fb_cost_grad_surrogate(pg, M, seed, it, mu)
    assert Jf == Jg
    np.testing.assert_array_equal(gf, gg)
    z0 = ref.fb_surrogate_state(pg, seed, 3, 0, it)
    assert z0[0] == pg.zd[0, 0] and z0[1] != pg.zd[0, 1]
    # the given line the defaults use is another direction
    _, gd = ref.fb_cost_grad_surrogate(small_problem(**kw), M, seed, it, mu)
    assert np.abs(gd - gf).max() > 1e-3 * np.abs(gf).max()


def test_surrogate_fit_one_particle_is_exact():
    """One particle has zero ensemble variance, so the fitted surrogate states
    are the target itself; with the target set to the particle's own realised
    path the surrogate gradient is the exact (difference-pinned) gradient."""
    kw = dict(gamma=0.8, b1=0.3, b2=0.4, beta=40.0)
    base = small_problem(**kw)
    mu = wl.random_feedback_control(base, 3, 1.0)
    seed, it = 5, 2
    z, _, _, n, _ = ref.fb_paths(base, seed, it, 0, 1, mu)
    assert n.sum() > 0
    p = small_problem(zd=z[0], svar="fit", **kw)
    var, a, b = ref.fb_surrogate_fit(p, 1, seed, it, mu)
    assert np.all(var == 0) and np.all(a == 0) and np.all(b == 0)
    J, g = ref.fb_cost_grad(p, 1, seed, it, mu)
    Js, gs = ref.fb_cost_grad_surrogate(p, 1, seed, it, mu)
    assert Js == J
    np.testing.assert_allclose(gs, g, rtol=1e-10, atol=1e-12 * np.abs(g).max())


def test_surrogate_one_step_definition():
    """N = 1: gs_0 = (1/M) sum_m [alpha u_0 phi(z_0) + gamma^n dt dJt/dv(zs_1) phi(zs_0)]."""
    p = wl.feedback_problem(N=1, T=0.5, zd=np.array([[0.2, -0.1], [0.4, 0.3]]), alpha=0.3,
                            sigJ=0.6, nx=4, nv=5, svar0=(0.05, 0.02), svar1=(0.1, 0.2))
    mu = wl.random_feedback_control(p, 2, 1.0)
    M, seed, it = 5, 8, 1
    z, _, u, n, _ = ref.fb_paths(p, seed, it, 0, M, mu)
    _, gs = ref.fb_cost_grad_surrogate(p, M, seed, it, mu)
    dx, dv = 2 * p.xmax / p.nx, 2 * p.vmax / p.nv
    xc = (np.arange(p.nx) + 0.5) * dx - p.xmax
    vc = (np.arange(p.nv) + 0.5) * dv - p.vmax

    def phi(zz):
        bx = np.array([ref.fb_bump(zz[0] - c, p.eps) for c in xc])
        bv = np.array([ref.fb_bump(zz[1] - c, p.eps) for c in vc])
        return np.outer(bx, bv).reshape(-1)

    want = np.zeros(p.L)
    for m in range(M):
        zs0 = ref.fb_surrogate_state(p, seed, m, 0, it)
        zs1 = ref.fb_surrogate_state(p, seed, m, 1, it)
        r = zs1 - p.zd[1]
        dJv = r[1] / p.sigJ ** 2 * np.exp(-np.sum(r * r) / (2 * p.sigJ ** 2))
        gn = p.gamma ** n[m, 0]
        want += p.alpha * u[m, 0] * phi(z[m, 0]) + gn * p.dt * dJv * phi(zs0)
    np.testing.assert_allclose(gs[0], want / M, rtol=1e-12, atol=1e-15)


def test_gradient_scale_diagnostic_fb():
    """The feedback model's per-entry summand scale: never below |g| (fixed
    grid, jump-adapted grid, surrogate), and equal to |g| for one particle."""
    p = wl.feedback_problem(N=12, T=1.2, zd=np.zeros((13, 2)), alpha=0.2)
    mu = wl.random_feedback_control(p, 4, 0.5)
    for kw in (dict(), dict(grid="adapted")):
        q = wl.feedback_problem(N=12, T=1.2, zd=np.zeros((13, 2)), alpha=0.2, **kw)
        _, g = ref.fb_cost_grad(q, 2000, 1, 0, mu)
        s = ref.fb_grad_scale(q, 2000, 1, 0, mu)
        assert np.all(s >= np.abs(g) * (1 - 1e-14))
        _, g1 = ref.fb_cost_grad(q, 1, 1, 0, mu)
        np.testing.assert_allclose(ref.fb_grad_scale(q, 1, 1, 0, mu), np.abs(g1), rtol=1e-13,
                                   atol=1e-300)
    _, gs = ref.fb_cost_grad_surrogate(p, 2000, 1, 0, mu)
    ss = ref.fb_grad_scale(p, 2000, 1, 0, mu, surrogate=True)
    assert np.all(ss >= np.abs(gs) * (1 - 1e-14))
