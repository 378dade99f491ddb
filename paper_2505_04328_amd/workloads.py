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
