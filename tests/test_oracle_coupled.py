"""Pins of the oracle's coupled-particle model (Section 6.4 of Bartsch, Borzi,
Ciaramella, Reichle, arXiv 2505.04328: eq. interacting_model, the start on the
ellipse of eq. coupled_ellipse and the ellipse cost of
eq. phonon_functional_tracking), each against something other than the oracle's
own formulas:

* the noise-free, jump-free, uncontrolled ring is linear: its Euler steps are
  powers of I + dt A with A assembled here from the ring's graph Laplacian
  2 I - S - S^T (S the cyclic shift), and the start is read off the unit
  circle's roots of unity;
* with omega = 0 a ring of np particles is np independent particles of the
  (separately pinned) single-particle model with the same counters;
* the adjoint gradient agrees with central differences of J and with the
  forward-mode tangent, with coupling, jumps, noise and the ellipse cost;
* the ellipse cost at points where it has a closed value.
"""
import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import workloads as wl

AX, AV = 1.5, 1.7071067811865475


def _quiet_ring(np_, N=40, T=4.0, eta=1.0, omega=0.5):
    """No noise, no control, jumps so rare that none is drawn (checked)."""
    return wl.ring_problem(N=N, T=T, np_=np_, omega=omega, eta=eta, b1=0.0, b2=0.0, beta=1e-12)


def _ring_matrix(np_, eta, omega):
    """Drift matrix of the uncontrolled ring, state (x_0, v_0, x_1, v_1, ...)."""
    S = np.roll(np.eye(np_), 1, axis=1)           # cyclic shift
    lap = 2.0 * np.eye(np_) - S - S.T             # ring graph Laplacian
    A = np.zeros((2 * np_, 2 * np_))
    A[0::2, 1::2] = np.eye(np_)                    # x' = v
    A[1::2, 0::2] = -eta * np.eye(np_) - omega * lap   # v' = -eta x - omega (L x)
    return A


@pytest.mark.parametrize("np_", [1, 2, 3, 7])
def test_quiet_ring_is_matrix_power(np_):
    p = _quiet_ring(np_)
    mu = np.zeros((p.N, p.L))
    M = 3
    z, _, u, n, _ = ref.fb_paths(p, 5, 0, 0, M, mu)
    assert n.sum() == 0 and np.all(u == 0.0)
    roots = np.exp(2j * np.pi * np.arange(np_) / np_)
    z0 = np.empty(2 * np_)
    z0[0::2], z0[1::2] = AX * roots.real, AV * roots.imag
    B = np.eye(2 * np_) + p.dt * _ring_matrix(np_, p.eta, p.omega)
    want = np.empty((p.N + 1, 2 * np_))
    want[0] = z0
    for k in range(p.N):
        want[k + 1] = B @ want[k]
    for m in range(M):
        got = z[m * np_:(m + 1) * np_]                       # (np, N+1, 2)
        got = got.transpose(1, 0, 2).reshape(p.N + 1, 2 * np_)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_quiet_ring_uniform_mode_feels_no_coupling():
    """All particles in the same state: the Laplacian term vanishes and each
    follows the single oscillator x'' = -eta x (Euler: powers of [[1, dt], [-eta dt, 1]])."""
    p = wl.feedback_problem(N=30, T=3.0, np_=6, omega=0.7, b1=0.0, b2=0.0, beta=1e-12,
                            init="gauss", z0=(0.4, -0.3), s0=(0.0, 0.0), cost="ellipse")
    z, _, _, n, _ = ref.fb_paths(p, 3, 0, 0, 2, np.zeros((p.N, p.L)))
    assert n.sum() == 0
    B = np.array([[1.0, p.dt], [-p.eta * p.dt, 1.0]])
    want = [np.array([0.4, -0.3])]
    for _ in range(p.N):
        want.append(B @ want[-1])
    for q in range(12):
        np.testing.assert_allclose(z[q], np.array(want), rtol=1e-13, atol=1e-15)


def test_uncoupled_ring_is_independent_particles():
    """omega = 0: ring m's particle j is particle m np + j of the one-particle
    model (same counters), and J, g are its means over all particles."""
    kw = dict(N=15, T=1.5, alpha=0.2, zd=np.tile([0.2, -0.1], (16, 1)), init="gauss",
              s0=(0.2, 0.3))
    ring = wl.feedback_problem(np_=4, omega=0.0, **kw)
    single = wl.feedback_problem(**kw)
    mu = wl.random_feedback_control(ring, 3, 0.5)
    zr, lr, ur, nr, cr = ref.fb_paths(ring, 9, 1, 2, 6, mu)
    zs, ls, us, ns, cs = ref.fb_paths(single, 9, 1, 8, 24, mu)
    assert nr.sum() > 0
    for a, b in ((zr, zs), (lr, ls), (ur, us), (nr, ns), (cr, cs)):
        np.testing.assert_array_equal(a, b)
    Jr, gr = ref.fb_cost_grad(ring, 40, 9, 1, mu)
    Js, gs = ref.fb_cost_grad(single, 160, 9, 1, mu)
    assert abs(Jr - Js) <= 1e-13 * abs(Js)
    np.testing.assert_allclose(gr, gs, rtol=0, atol=1e-13 * np.abs(gs).max())


def _coupled_case(np_):
    p = wl.ring_problem(N=20, T=2.0, np_=np_, omega=0.5, alpha=0.3, s0=(0.05, 0.05), sigJ=0.4)
    return p, wl.random_feedback_control(p, 11, 0.5)


@pytest.mark.parametrize("np_", [2, 5])
def test_coupled_gradient_matches_differences_and_tangent(np_):
    p, mu = _coupled_case(np_)
    M, seed, it = 12, 4, 3
    _, _, _, n, _ = ref.fb_paths(p, seed, it, 0, M, mu)
    assert n.sum() > 10 and p.gamma != 1.0
    J, g = ref.fb_cost_grad(p, M, seed, it, mu)
    rng = np.random.default_rng(5)
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


def test_coupled_J_is_mean_of_particle_costs():
    p, mu = _coupled_case(3)
    M = 7
    _, _, _, _, c = ref.fb_paths(p, 2, 0, 0, M, mu)
    J, _ = ref.fb_cost_grad(p, M, 2, 0, mu, grad=False)
    assert c.shape == (M * 3,)
    assert abs(J - c.mean()) <= 1e-13 * abs(J)


def _one_step(z0, sigJ=0.5, T=0.5):
    """One particle, one step, no noise, jumps, spring or control: z_1 = (x0 + dt v0, v0)."""
    p = wl.feedback_problem(N=1, T=T, eta=0.0, b1=0.0, b2=0.0, beta=1e-12, init="gauss", z0=z0,
                            s0=(0.0, 0.0), cost="ellipse", sigJ=sigJ)
    J, _ = ref.fb_cost_grad(p, 1, 1, 0, np.zeros((1, p.L)), grad=False)
    return J, p.dt


def test_ellipse_cost_closed_values():
    s = 0.5
    J, dt = _one_step((AX, 0.0))             # on the ellipse: -1 per unit time
    assert J == -dt
    J, dt = _one_step((0.0, 0.0))            # centre: q = -1
    assert abs(J + dt * np.exp(-1.0 / (2 * s * s))) <= 1e-15
    J, dt = _one_step((AX * np.sqrt(3.0), 0.0))   # q = 2
    assert abs(J + dt * np.exp(-4.0 / (2 * s * s))) <= 1e-15
    J, dt = _one_step((-AX * np.sqrt(0.5), 0.0), sigJ=0.3)   # q = -1/2
    assert abs(J + dt * np.exp(-0.25 / (2 * 0.09))) <= 1e-15
    # the top of the ellipse moves to (dt av, av): q = (dt av / ax)^2
    J, dt = _one_step((0.0, AV), T=0.01)
    q = (dt * AV / AX) ** 2
    assert abs(J + dt * np.exp(-q * q / (2 * s * s))) <= 1e-17


def test_ellipse_start():
    np_ = 8
    p = wl.ring_problem(N=4, T=0.4, np_=np_)
    for m in (0, 5):
        for j in range(np_):
            z = ref.fb_initial(p, 7, m * np_ + j, 0)
            ang = np.arctan2(z[1] / AV, z[0] / AX) % (2 * np.pi)
            assert abs((z[0] / AX) ** 2 + (z[1] / AV) ** 2 - 1.0) <= 1e-14
            assert abs(ang - (2 * np.pi * j / np_) % (2 * np.pi)) <= 1e-12 or \
                abs(abs(ang - 2 * np.pi * j / np_) - 2 * np.pi) <= 1e-12
    # jitter s0: Gaussian around the ellipse point
    pj = wl.ring_problem(N=4, T=0.4, np_=np_, s0=(0.1, 0.2))
    pts = np.array([ref.fb_initial(pj, 7, m * np_ + 3, 0) for m in range(4000)])
    base = np.array([AX * np.cos(2 * np.pi * 3 / np_), AV * np.sin(2 * np.pi * 3 / np_)])
    assert np.all(np.abs(pts.mean(0) - base) < 4 * np.array([0.1, 0.2]) / np.sqrt(4000))
    assert np.all(np.abs(pts.std(0) / np.array([0.1, 0.2]) - 1.0) < 0.05)
