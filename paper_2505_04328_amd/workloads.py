"""Seeded synthetic problem generators.

This module only builds inputs: problem coefficients, desired trajectories and
seeds.  It holds none of the method's arithmetic, so both the GPU path and the
FP64 oracle may take their inputs from it.

The model is the controlled jump-diffusion of the paper's Section 2
(eq. SDE_constraint) reduced to an open-loop, piecewise-constant control on the
fixed grid t_k = k*T/N (Section 3, eq. piecewise_constant_control):

    dX = (A X - c3 X^3 + B u(t)) dt + diag(s) dW + dJ,

with J a compound Poisson process of rate ``lam`` whose jump sizes are
N(jump_mean, diag(jump_std^2)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Problem:
    """One optimal-control problem instance (all arrays FP64, host memory)."""

    d: int
    N: int
    T: float
    lam: float
    cubic: float
    nu: float
    x0: np.ndarray
    A: np.ndarray  # d x d
    B: np.ndarray  # d x d
    s: np.ndarray  # d
    jump_mean: np.ndarray  # d
    jump_std: np.ndarray  # d
    xT: np.ndarray  # d
    xd: np.ndarray  # N x d, row k = x_d(t_k)
    name: str = ""

    def __post_init__(self):
        d, N = int(self.d), int(self.N)
        self.d, self.N = d, N
        self.T, self.lam, self.cubic, self.nu = (float(self.T), float(self.lam),
                                                 float(self.cubic), float(self.nu))
        def vec(a):
            return np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (d,)))
        self.x0, self.s = vec(self.x0), vec(self.s)
        self.jump_mean, self.jump_std, self.xT = vec(self.jump_mean), vec(self.jump_std), vec(self.xT)
        self.A = np.ascontiguousarray(np.asarray(self.A, np.float64).reshape(d, d))
        self.B = np.ascontiguousarray(np.asarray(self.B, np.float64).reshape(d, d))
        self.xd = np.ascontiguousarray(np.asarray(self.xd, np.float64).reshape(N, d))

    @property
    def dt(self) -> float:
        return self.T / self.N

    def zeros_u(self) -> np.ndarray:
        return np.zeros((self.N, self.d), np.float64)


@dataclasses.dataclass
class Workload:
    """A problem plus the Monte Carlo run parameters it is quoted with."""

    problem: Problem
    M: int
    seed: int = 1
    precision: str = "fp32"  # "fp32" path arithmetic with FP64 reductions, or "fp64"
    K: int = 0  # checkpoint interval of the recompute variant (0 = stored)
    iters: int = 0
    name: str = ""


def sine_target(N: int, T: float, d: int) -> np.ndarray:
    """x_d(t_k) = sin(2 pi t_k) in every component, t_k = k T / N."""
    t = np.arange(N, dtype=np.float64) * (T / N)
    return np.repeat(np.sin(2.0 * math.pi * t)[:, None], d, axis=1)


def stable_symmetric(d: int, seed: int, lo: float = -2.0, hi: float = -0.2):
    """Random symmetric A with eigenvalues uniform in [lo, hi] and diffusion
    scales s ~ U(0.1, 0.5), from numpy's default_rng(seed): eigenvalues first,
    then an orthogonal Q from the QR of a Gaussian matrix (signs fixed by
    diag R), A = Q diag(eig) Q^T, then s."""
    rng = np.random.default_rng(seed)
    eig = rng.uniform(lo, hi, d)
    Q, R = np.linalg.qr(rng.standard_normal((d, d)))
    Q = Q * np.sign(np.diag(R))[None, :]
    A = (Q * eig[None, :]) @ Q.T
    s = rng.uniform(0.1, 0.5, d)
    return A, s


def ou_1d(N: int, lam: float, jump_mean: float, jump_std: float, T: float = 1.0,
          a: float = 1.0, s: float = 0.3, nu: float = 1e-3, name: str = "") -> Problem:
    """dX = (u_k - a X) dt + s dW + dJ with X0 = 0, x_T = 1, x_d = sin 2 pi t."""
    return Problem(d=1, N=N, T=T, lam=lam, cubic=0.0, nu=nu, x0=[0.0], A=[[-a]], B=[[1.0]],
                   s=[s], jump_mean=[jump_mean], jump_std=[jump_std], xT=[1.0],
                   xd=sine_target(N, T, 1), name=name)


def coupled_8d(N: int, T: float = 2.0, lam: float = 3.0, cubic: float = 0.0,
               nu: float = 1e-3, name: str = "") -> Problem:
    """d = 8 coupled linear drift, A random stable (seed 7), B = I, jumps
    N(0, 0.2^2 I), X0 = 0, x_T = 1, x_d = sin(2 pi t) 1."""
    A, s = stable_symmetric(8, 7)
    return Problem(d=8, N=N, T=T, lam=lam, cubic=cubic, nu=nu, x0=np.zeros(8), A=A,
                   B=np.eye(8), s=s, jump_mean=np.zeros(8), jump_std=np.full(8, 0.2),
                   xT=np.ones(8), xd=sine_target(N, T, 8), name=name)


def config(name: str) -> Workload:
    """The five benchmark configurations.

    c1: 1-D OU, N=100, lam=2, jumps N(0,0.2^2), M=10^4, FP64, 20 iterations.
    c2: same model, M=2^20, N=1000, lam=5, jumps N(-0.1,0.3^2), FP32, K=32, 50 iterations.
    c3: d=8 linear, M=2^20, N=500, T=2, lam=3, FP32.
    c4: c3 with cubic drift 0.1, M=2^18, N=2000, K=64 (differentiation).
    c5: serving mix (see ``serving_requests``); the Workload returned is the largest
        request shape, for sizing only.
    """
    if name == "c1":
        return Workload(ou_1d(100, 2.0, 0.0, 0.2, name="c1"), M=10_000, seed=1,
                        precision="fp64", iters=20, name="c1")
    if name == "c2":
        return Workload(ou_1d(1000, 5.0, -0.1, 0.3, name="c2"), M=1 << 20, seed=1,
                        precision="fp32", K=32, iters=50, name="c2")
    if name == "c3":
        return Workload(coupled_8d(500, name="c3"), M=1 << 20, seed=1, precision="fp32",
                        iters=20, name="c3")
    if name == "c4":
        return Workload(coupled_8d(2000, cubic=0.1, name="c4"), M=1 << 18, seed=1,
                        precision="fp32", K=64, name="c4")
    if name == "c5":
        return Workload(coupled_8d(2000, T=1.0, name="c5"), M=1 << 20, seed=1,
                        precision="fp32", iters=30, name="c5")
    raise KeyError(name)


def scaled(w: Workload, M: int | None = None, N: int | None = None) -> Workload:
    """The same problem at fewer paths and/or steps (x_d resampled on the new grid)."""
    p = w.problem
    if N is not None and N != p.N:
        p = dataclasses.replace(p, N=N, xd=sine_target(N, p.T, p.d))
    return dataclasses.replace(w, problem=p, M=w.M if M is None else M)


def general_problem(d: int, N: int, seed: int, cubic: float = 0.0, lam: float = 3.0,
                    T: float = 1.0, nu: float = 1e-2, jump_mean: float = 0.05,
                    jump_std: float = 0.2) -> Problem:
    """A test problem with a non-symmetric A and a non-identity B, so that a
    transposed operand anywhere in an implementation changes the results."""
    rng = np.random.default_rng(seed)
    A = -1.0 * np.eye(d) + 0.4 * rng.standard_normal((d, d)) / math.sqrt(d)
    B = np.eye(d) + 0.3 * rng.standard_normal((d, d)) / math.sqrt(d)
    s = rng.uniform(0.1, 0.5, d)
    x0 = 0.3 * rng.standard_normal(d)
    xT = 1.0 + 0.2 * rng.standard_normal(d)
    t = np.arange(N) * (T / N)
    ph = rng.uniform(0, 2 * math.pi, d)
    xd = np.sin(2 * math.pi * t[:, None] / T + ph[None, :])
    jm = jump_mean * (1 + rng.standard_normal(d))
    js = jump_std * rng.uniform(0.5, 1.5, d)
    return Problem(d=d, N=N, T=T, lam=lam, cubic=cubic, nu=nu, x0=x0, A=A, B=B, s=s,
                   jump_mean=jm, jump_std=js, xT=xT, xd=xd, name=f"general{d}")


def random_control(p: Problem, seed: int, scale: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((p.N, p.d))


def fd_directions(p: Problem, count: int = 16, seed: int = 2) -> np.ndarray:
    """Random directions normalised in L2(0,T): dt * sum_k |delta_k|^2 = 1."""
    rng = np.random.default_rng(seed)
    out = rng.standard_normal((count, p.N, p.d))
    nrm = np.sqrt(p.dt * np.sum(out * out, axis=(1, 2)))
    return out / nrm[:, None, None]


@dataclasses.dataclass
class Request:
    """One optimisation request of the serving mix."""

    rid: int
    arrival: float  # seconds after the start
    problem: Problem
    M: int
    seed: int
    iters: int


def serving_requests(count: int = 256, rate: float = 50.0, seed: int = 11, M_lo: int = 1 << 14,
                     M_hi: int = 1 << 20, N_lo: int = 100, N_hi: int = 2000,
                     lam_hi: float = 10.0, iters: int = 30) -> list:
    """Poisson arrivals (exponential gaps of mean 1/rate, default_rng(seed)), d in
    {1,2,4,8}, M uniform integer in [M_lo, M_hi], N uniform integer in [N_lo, N_hi],
    lam ~ U(0, lam_hi), T = 1, A and s from ``stable_symmetric(d, 1000 + r)``,
    jumps N(0, 0.2^2 I), cost as c1, nu = 1e-3, Philox seed r + 1."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        d = int(rng.choice([1, 2, 4, 8]))
        M = int(rng.integers(M_lo, M_hi + 1))
        N = int(rng.integers(N_lo, N_hi + 1))
        lam = float(rng.uniform(0.0, lam_hi))
        A, s = stable_symmetric(d, 1000 + r)
        p = Problem(d=d, N=N, T=1.0, lam=lam, cubic=0.0, nu=1e-3, x0=np.zeros(d), A=A,
                    B=np.eye(d), s=s, jump_mean=np.zeros(d), jump_std=np.full(d, 0.2),
                    xT=np.ones(d), xd=sine_target(N, 1.0, d), name=f"req{r}")
        out.append(Request(rid=r, arrival=float(arrivals[r]), problem=p, M=M, seed=r + 1,
                           iters=iters))
    return out


# ---------------------------------------------------------------------------
# The paper's own model problem (Section 5, model equation; Section 6): one
# particle z = (x, v) per path in a harmonic oscillator with Brownian noise,
# Keilson-Storer velocity jumps v <- gamma v + N(0, 1/(2 beta)) at rate
# sqrt(beta/pi), and the feedback control u(z, t_k) = sum_l mu_k[l] phi_l(z)
# over nx x nv products of compact bump functions on the cell centres of
# (-xmax, xmax) x (-vmax, vmax).


@dataclasses.dataclass
class FeedbackProblem:
    """One instance of the paper's model problem (FP64, host memory)."""

    N: int
    T: float
    eta: float
    b1: float
    b2: float
    gamma: float
    beta: float
    nx: int
    nv: int
    xmax: float
    vmax: float
    eps: float
    alpha: float
    sigJ: float
    init_kind: int  # 0: Gaussian z0 + s0 * Z, 1: uniform on [z0 - s0, z0 + s0], 2: ellipse
    z0: np.ndarray  # 2
    s0: np.ndarray  # 2
    zd: np.ndarray  # (N+1) x 2, row k = desired (x, v) at t_k
    name: str = ""
    # variance of the surrogate adjoint states, var_c(t) = svar0[c] + svar1[c] t
    # (Section 6.5); None: the initial variance plus the noise and jump
    # variance rates (b1^2, b2^2 + rate / (2 beta))
    svar0: np.ndarray | None = None
    svar1: np.ndarray | None = None
    # coupled particles (Section 6.4): rings of np particles with
    # nearest-neighbour coupling omega; cost_kind 1 is the ellipse cost with
    # half-axes (ax, av), which init_kind 2 also starts the particles on
    np: int = 1
    omega: float = 0.0
    cost_kind: int = 0
    ax: float = 1.0
    av: float = 1.0
    # time grid: 0 the fixed grid with Poisson jump counts per step, 1 the
    # jump-adapted grid (uniform points and each particle's jump times)
    grid: int = 0
    # surrogate variance: 0 the line svar0 + svar1 t, 1 the least-squares line
    # through the forward ensemble's own per-step variance (Section 6.5)
    svar_kind: int = 0

    def __post_init__(self):
        self.N, self.nx, self.nv, self.init_kind = int(self.N), int(self.nx), int(self.nv), int(self.init_kind)
        self.np, self.cost_kind, self.grid = int(self.np), int(self.cost_kind), int(self.grid)
        self.svar_kind = int(self.svar_kind)
        for f in ("T", "eta", "b1", "b2", "gamma", "beta", "xmax", "vmax", "eps", "alpha", "sigJ",
                  "omega", "ax", "av"):
            setattr(self, f, float(getattr(self, f)))
        self.z0 = np.ascontiguousarray(np.broadcast_to(np.asarray(self.z0, np.float64), (2,)))
        self.s0 = np.ascontiguousarray(np.broadcast_to(np.asarray(self.s0, np.float64), (2,)))
        self.zd = np.ascontiguousarray(np.asarray(self.zd, np.float64).reshape(self.N + 1, 2))
        if self.svar0 is None:
            self.svar0 = self.s0 ** 2 if self.init_kind == 0 else self.s0 ** 2 / 3.0
        if self.svar1 is None:
            self.svar1 = (self.b1 ** 2, self.b2 ** 2 + math.sqrt(self.beta / math.pi) / (2.0 * self.beta))
        self.svar0 = np.ascontiguousarray(np.broadcast_to(np.asarray(self.svar0, np.float64), (2,)))
        self.svar1 = np.ascontiguousarray(np.broadcast_to(np.asarray(self.svar1, np.float64), (2,)))

    @property
    def dt(self) -> float:
        return self.T / self.N

    @property
    def L(self) -> int:
        return self.nx * self.nv

    @property
    def rate(self) -> float:
        """Keilson-Storer jump frequency sqrt(beta/pi) (eq. collision_frequency)."""
        return math.sqrt(self.beta / math.pi)


@dataclasses.dataclass
class FeedbackWorkload:
    problem: FeedbackProblem
    M: int
    seed: int = 1


def feedback_problem(N: int = 50, T: float = 5.0, init: str = "gauss", zd=None, eta: float = 1.0,
                     b1: float = 0.05, b2: float = 0.1, gamma: float = 0.9, beta: float = 10.0,
                     nx: int = 10, nv: int = 10, xmax: float = 2.0, vmax: float = 2.0,
                     eps: float = 0.5, alpha: float = 1e-2, sigJ: float = 0.5,
                     name: str = "", s0=None, z0=None, svar0=None, svar1=None, np_: int = 1,
                     omega: float = 0.0, cost: str = "track", ax: float = 1.5,
                     av: float = 1.7071067811865475, grid: str = "fixed",
                     svar: str = "given") -> FeedbackProblem:
    """The setting of the paper's Section 6 (xmax = vmax = 2, nx = nv = 10,
    eps = 0.5, beta = 10, gamma = 0.9, eta = 1, T = 5, N = 50).  The paper does
    not state alpha, sigma_J, b1, b2; the defaults here are readings.  init
    'gauss' is N((0.75, 0.75), 0.01 I) (Section 6.1), 'uniform' is [-1, 1]^2,
    'ellipse' the ring's particles equally spaced in angle on the ellipse
    (Section 6.4); z0 and s0 override the law's centre and scale.  np_ > 1
    couples rings of np_ particles with strength omega; cost 'ellipse' is the
    cost of Section 6.4 with the half-axes ax = 1.5, av = 1.7071067811865475
    printed there.  grid 'adapted' integrates on the jump-adapted grid of
    Section 3 (Algorithms 5.1-5.2) instead of the fixed grid.  svar 'fit' takes
    the surrogate variance of Section 6.5 from a least-squares line through the
    forward ensemble's per-step variance instead of svar0 + svar1 t."""
    if init == "gauss":
        kind, z0d, s0d = 0, (0.75, 0.75), (0.1, 0.1)
    elif init == "uniform":
        kind, z0d, s0d = 1, (0.0, 0.0), (1.0, 1.0)
    elif init == "ellipse":
        kind, z0d, s0d = 2, (0.0, 0.0), (0.0, 0.0)
    else:
        raise ValueError(init)
    if cost not in ("track", "ellipse"):
        raise ValueError(cost)
    if grid not in ("fixed", "adapted"):
        raise ValueError(grid)
    if svar not in ("given", "fit"):
        raise ValueError(svar)
    z0 = z0d if z0 is None else z0
    s0 = s0d if s0 is None else s0
    if zd is None:
        zd = np.zeros((N + 1, 2))
    return FeedbackProblem(N=N, T=T, eta=eta, b1=b1, b2=b2, gamma=gamma, beta=beta, nx=nx, nv=nv,
                           xmax=xmax, vmax=vmax, eps=eps, alpha=alpha, sigJ=sigJ, init_kind=kind,
                           z0=z0, s0=s0, zd=zd, name=name, svar0=svar0, svar1=svar1, np=np_,
                           omega=omega, cost_kind=0 if cost == "track" else 1, ax=ax, av=av,
                           grid=0 if grid == "fixed" else 1, svar_kind=0 if svar == "given" else 1)


def ring_problem(N: int = 50, T: float = 5.0, np_: int = 2000, omega: float = 0.5, name: str = "",
                 **kw) -> FeedbackProblem:
    """Section 6.4: rings of np_ nearest-neighbour coupled oscillators (eta = 1,
    omega = 0.5) started on the ellipse with ax = 1.5, av = 1.7071067811865475,
    and the ellipse cost; the other settings as in Section 6."""
    return feedback_problem(N=N, T=T, init="ellipse", np_=np_, omega=omega, cost="ellipse",
                            name=name, **kw)


def switching_target(N: int, T: float, amp: float = 0.5) -> np.ndarray:
    """A non-smooth desired trajectory (Section 6.3 follows one; its formula is
    not printed): x_d jumps between +amp and -amp at t = T/2, v_d = 0."""
    t = np.arange(N + 1) * (T / N)
    zd = np.zeros((N + 1, 2))
    zd[:, 0] = np.where(t < 0.5 * T, amp, -amp)
    return zd


def feedback_config(name: str) -> FeedbackWorkload:
    """f1: Section 6.1 centering from a Gaussian cloud, the paper's size
    (2000 particles, 50 steps).  f2: centering from the uniform box.  f3: the
    switching target.  f4: the measured size, 2^20 particles and 500 steps
    (dt = 0.01) of the f1 setting."""
    if name == "f1":
        return FeedbackWorkload(feedback_problem(name="f1"), M=2000, seed=1)
    if name == "f2":
        return FeedbackWorkload(feedback_problem(init="uniform", name="f2"), M=2000, seed=1)
    if name == "f3":
        return FeedbackWorkload(feedback_problem(zd=switching_target(50, 5.0), name="f3"), M=2000,
                                seed=1)
    if name == "f4":
        return FeedbackWorkload(feedback_problem(N=500, name="f4"), M=1 << 20, seed=1)
    raise KeyError(name)


def adapted_config(name: str) -> FeedbackWorkload:
    """The jump-adapted grid (Section 3).  ja1: the paper's setting (Section
    6.1, 2000 particles, 50 steps of 0.1).  ja2: the measured size of f4, 2^20
    particles and 500 steps of 0.01 (a jump in about one interval of 56).  ja3:
    2^20 particles at the paper's step, 50 steps of 0.1 (a jump in about one
    interval of six, several in some)."""
    if name == "ja1":
        return FeedbackWorkload(feedback_problem(name="ja1", grid="adapted"), M=2000, seed=1)
    if name == "ja2":
        return FeedbackWorkload(feedback_problem(N=500, name="ja2", grid="adapted"), M=1 << 20,
                                seed=1)
    if name == "ja3":
        return FeedbackWorkload(feedback_problem(name="ja3", grid="adapted"), M=1 << 20, seed=1)
    raise KeyError(name)


def ring_config(name: str) -> FeedbackWorkload:
    """ring1: Section 6.4 at the paper's size, one ring of 2000 particles, 50
    steps.  ring2: the measured size, 512 independent rings of 2000 particles
    (1,024,000 particles), 500 steps (dt = 0.01).  M counts rings."""
    if name == "ring1":
        return FeedbackWorkload(ring_problem(name="ring1"), M=1, seed=1)
    if name == "ring2":
        return FeedbackWorkload(ring_problem(N=500, name="ring2"), M=512, seed=1)
    raise KeyError(name)


def random_feedback_control(p: FeedbackProblem, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded control mu (N x L), entries N(0, scale^2)."""
    return np.random.default_rng(seed).normal(0.0, scale, (p.N, p.L))
