"""Closed forms of the linear-drift, quadratic-cost case (cubic = 0), in numpy FP64.

Test infrastructure only.  With c3 = 0 the Euler-Maruyama recursion of the
paper's fully discrete problem (Section 3, eq. model_approximation) is affine in
the state with additive noise and additive compound-Poisson jumps, so its mean
and covariance follow exact recursions, the expected discrete functional
(Section 3, discrete functional) is an explicit quadratic in u, and its
gradient follows the adjoint recursion of Section 4 (eq. AdjointModel) applied
to the mean path.  These pin the Monte Carlo oracle statistically and give the
linear-quadratic optimum.

With Phi = I + dt A, mu = lam*dt:
    m_{k+1} = Phi m_k + dt B u_k + mu m_J
    P_{k+1} = Phi P_k Phi^T + dt diag(s^2) + mu (diag(s_J^2) + m_J m_J^T)
    E[J]    = sum_{k<N} dt/2 (|m_k - xd_k|^2 + tr P_k) + 1/2 (|m_N - xT|^2 + tr P_N)
              + nu dt/2 sum_k |u_k|^2
    lbar_N  = m_N - xT,  lbar_k = Phi^T lbar_{k+1} + dt (m_k - xd_k)
    E-grad  = nu u_k + B^T lbar_{k+1}

The end of the file holds the same kind of moment recursion for the paper's
own model problem (oscillator, Keilson-Storer jumps) without control.
"""
from __future__ import annotations

import math

import numpy as np


def _check(p):
    if p.cubic != 0.0:
        raise ValueError("closed forms hold for the linear drift only (cubic = 0)")


def moments(p, u=None):
    """Mean m (N+1 x d) and covariance P (N+1 x d x d) of X_k."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    u = np.zeros((N, d)) if u is None else np.asarray(u, np.float64)
    mu = p.lam * dt
    Phi = np.eye(d) + dt * p.A
    Q = dt * np.diag(p.s ** 2) + mu * (np.diag(p.jump_std ** 2) + np.outer(p.jump_mean, p.jump_mean))
    m = np.zeros((N + 1, d))
    P = np.zeros((N + 1, d, d))
    m[0] = p.x0
    for k in range(N):
        m[k + 1] = Phi @ m[k] + dt * (p.B @ u[k]) + mu * p.jump_mean
        P[k + 1] = Phi @ P[k] @ Phi.T + Q
    return m, P


def expected_cost(p, u=None) -> float:
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    u = np.zeros((N, d)) if u is None else np.asarray(u, np.float64)
    m, P = moments(p, u)
    run = sum(0.5 * dt * (np.sum((m[k] - p.xd[k]) ** 2) + np.trace(P[k])) for k in range(N))
    term = 0.5 * (np.sum((m[N] - p.xT) ** 2) + np.trace(P[N]))
    return float(run + term + 0.5 * p.nu * dt * np.sum(u * u))


def expected_grad(p, u=None) -> np.ndarray:
    """L2 representative g (N x d) of the gradient of E[J]: dE[J]/du_k = dt g_k."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    u = np.zeros((N, d)) if u is None else np.asarray(u, np.float64)
    m, _ = moments(p, u)
    Phi = np.eye(d) + dt * p.A
    lb = np.zeros((N + 1, d))
    lb[N] = m[N] - p.xT
    for k in range(N - 1, 0, -1):
        lb[k] = Phi.T @ lb[k + 1] + dt * (m[k] - p.xd[k])
    return p.nu * u + lb[1:] @ p.B


def mean_control_map(p):
    """Affine map u -> (m_1..m_N): m_flat = m_free + G u_flat, with m_free the mean
    path at u = 0.  Built column by column from the mean recursion."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    m0, _ = moments(p, None)
    Phi = np.eye(d) + dt * p.A
    G = np.zeros((N * d, N * d))
    # effect of u_j on m_{k+1} (k >= j) is Phi^{k-j} dt B
    blk = dt * p.B
    for j in range(N):
        cur = blk
        for k in range(j, N):
            G[k * d:(k + 1) * d, j * d:(j + 1) * d] = cur
            cur = Phi @ cur
    return m0[1:].reshape(-1), G


def _weights_targets(p):
    d, N, dt = p.d, p.N, p.dt
    w = np.full(N * d, dt)
    w[(N - 1) * d:] = 1.0  # m_N carries the terminal weight; m_1..m_{N-1} the running weight
    target = np.concatenate([p.xd[1:].reshape(-1), p.xT])
    return w, target


def expected_grad_dense(p, u=None) -> np.ndarray:
    """Same quantity as ``expected_grad`` by a different route: differentiate the
    quadratic E[J](u) through the assembled matrix G of ``mean_control_map``,
    dE[J]/du = G^T W (m - target) + nu dt u, then divide by dt."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    u = np.zeros((N, d)) if u is None else np.asarray(u, np.float64)
    mfree, G = mean_control_map(p)
    w, target = _weights_targets(p)
    m = mfree + G @ u.reshape(-1)
    grad = G.T @ (w * (m - target)) + p.nu * dt * u.reshape(-1)
    return (grad / dt).reshape(N, d)


def lq_optimum(p) -> np.ndarray:
    """Minimiser of E[J] over u (N x d) from the dense normal equations."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    mfree, G = mean_control_map(p)
    w, target = _weights_targets(p)
    H = G.T @ (w[:, None] * G) + p.nu * dt * np.eye(N * d)
    rhs = G.T @ (w * (target - mfree))
    return np.linalg.solve(H, rhs).reshape(N, d)


def deterministic_path(p, u=None) -> np.ndarray:
    """X_k of the noise-free, jump-free recursion via matrix powers:
    X_k = Phi^k x0 + sum_{j<k} Phi^{k-1-j} dt B u_j  (valid for cubic = 0)."""
    _check(p)
    d, N, dt = p.d, p.N, p.dt
    u = np.zeros((N, d)) if u is None else np.asarray(u, np.float64)
    Phi = np.eye(d) + dt * p.A
    X = np.zeros((N + 1, d))
    for k in range(N + 1):
        x = np.linalg.matrix_power(Phi, k) @ p.x0
        for j in range(k):
            x = x + np.linalg.matrix_power(Phi, k - 1 - j) @ (dt * (p.B @ u[j]))
        X[k] = x
    return X


# ---------------------------------------------------------------------------
# The paper's model problem (fb_oracle.c) without control (mu = 0): the Euler
# step is linear in z, the jump count n ~ Poisson(lam = sqrt(beta/pi) dt) is
# independent of the state and of the Brownian normals, so the means and raw
# second moments follow exact recursions.  With n Keilson-Storer jumps the
# velocity becomes gamma^n v + N(0, V_n), V_n = (1 - gamma^{2n}) / ((1 - gamma^2) 2 beta),
# and for a Poisson count E[gamma^n] = exp(-lam (1 - gamma)),
# E[gamma^{2n}] = exp(-lam (1 - gamma^2)).

def fb_moments(p):
    """Arrays (N+1) of E[x], E[v], E[x^2], E[x v], E[v^2] for mu = 0."""
    dt, eta, lam = p.dt, p.eta, p.rate * p.dt
    g1 = math.exp(-lam * (1.0 - p.gamma))
    g2 = math.exp(-lam * (1.0 - p.gamma * p.gamma))
    if abs(1.0 - p.gamma * p.gamma) > 1e-15:
        EV = (1.0 - g2) / ((1.0 - p.gamma * p.gamma) * 2.0 * p.beta)
    else:
        EV = lam / (2.0 * p.beta)
    if p.init_kind == 0:
        var = p.s0 ** 2
    else:
        var = p.s0 ** 2 / 3.0
    mx, mv = p.z0[0], p.z0[1]
    sxx, sxv, svv = mx * mx + var[0], mx * mv, mv * mv + var[1]
    out = np.zeros((p.N + 1, 5))
    out[0] = (mx, mv, sxx, sxv, svv)
    for k in range(p.N):
        mx, mv = mx + dt * mv, g1 * (mv - dt * eta * mx)
        sxx, sxv, svv = (sxx + 2 * dt * sxv + dt * dt * svv + p.b1 ** 2 * dt,
                         g1 * (sxv - dt * eta * sxx + dt * svv - dt * dt * eta * sxv),
                         g2 * (svv - 2 * dt * eta * sxv + dt * dt * eta * eta * sxx + p.b2 ** 2 * dt) + EV)
        out[k + 1] = (mx, mv, sxx, sxv, svv)
    return out
