"""ctypes wrapper of the FP64 C oracle (test infrastructure only).

Each function mirrors one routine of ``jd_oracle.c``; see that file for which
passage of the paper each follows.  Inputs are numpy arrays and
``Problem`` instances from the seeded workload generators.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class _Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("N", C.c_int32), ("T", C.c_double), ("lambda_", C.c_double),
                ("cubic", C.c_double), ("nu", C.c_double),
                ("x0", C.c_void_p), ("A", C.c_void_p), ("B", C.c_void_p), ("s", C.c_void_p),
                ("jump_mean", C.c_void_p), ("jump_std", C.c_void_p), ("xT", C.c_void_p),
                ("xd", C.c_void_p)]


class _Opt(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("tol", C.c_double), ("zeta0", C.c_double),
                ("rho", C.c_double), ("c_armijo", C.c_double), ("max_backtracks", C.c_int32)]


def lib():
    """Load the oracle shared library, building it first if absent.  The
    environment variable JD_ORACLE_LIB names another build of the same source
    (the mutation tests use it to run the pins against planted mistakes)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("JD_ORACLE_LIB")
        if alt:
            _lib = _bind(C.CDLL(alt))
        else:
            if not os.path.exists(_build.LIB):
                _build.build()
            _lib = _bind(C.CDLL(_build.LIB))
    return _lib


def _bind(L):
    P = C.c_void_p
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_uniform.argtypes = [C.c_uint32]
    L.or_uniform.restype = C.c_double
    L.or_uniform_batch.argtypes = [P, C.c_int64, P]
    L.or_poisson_thresholds.argtypes = [C.c_double, P]
    L.or_poisson_count.argtypes = [C.c_uint32, P]
    L.or_poisson_count.restype = C.c_int
    L.or_draws_grid.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_int64,
                                C.c_int64, C.c_int32, C.c_int32, P, P, P]
    L.or_paths.argtypes = [P, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, P, P, P, P, C.c_int]
    L.or_paths.restype = C.c_int
    L.or_cost_grad.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, C.c_int]
    L.or_cost_grad.restype = C.c_int
    L.or_grad_scale.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, C.c_int]
    L.or_grad_scale.restype = C.c_int
    L.or_tangent.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, C.c_int]
    L.or_tangent.restype = C.c_int
    L.or_optimize.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, P, P, P, P, C.c_int]
    L.or_optimize.restype = C.c_int
    return L


def default_threads() -> int:
    n = os.environ.get("OMP_NUM_THREADS")
    if n and n.isdigit() and int(n) > 0:
        return int(n)
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class _ProblemRef:
    """Holds the ctypes struct and keeps the numpy arrays it points to alive."""

    def __init__(self, p):
        self.keep = [np.ascontiguousarray(x, np.float64) for x in
                     (p.x0, p.A, p.B, p.s, p.jump_mean, p.jump_std, p.xT, p.xd)]
        x0, A, B, s, jm, js, xT, xd = self.keep
        assert xd.shape == (p.N, p.d)
        self.st = _Problem(p.d, p.N, p.T, p.lam, p.cubic, p.nu, _ptr(x0), _ptr(A), _ptr(B),
                           _ptr(s), _ptr(jm), _ptr(js), _ptr(xT), _ptr(xd))

    @property
    def ref(self):
        return C.byref(self.st)


def _u(p, u):
    if u is None:
        return np.zeros((p.N, p.d))
    u = np.ascontiguousarray(u, np.float64)
    assert u.shape == (p.N, p.d)
    return u


def philox(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 blocks for counters ctr (n x 4 uint32) under key (2 uint32)."""
    L = lib()
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32).reshape(2)
    out = np.empty_like(ctr)
    o = np.empty(4, np.uint32)
    for i in range(ctr.shape[0]):
        c = np.ascontiguousarray(ctr[i])
        L.or_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
        out[i] = o
    return out


def uniform(w: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, np.uint32)
    out = np.empty(w.shape, np.float64)
    lib().or_uniform_batch(_ptr(w), w.size, _ptr(out))
    return out


def poisson_thresholds(mu: float) -> np.ndarray:
    t = np.zeros(32, np.uint64)
    lib().or_poisson_thresholds(float(mu), _ptr(t))
    return t


def poisson_count(P: int, thr: np.ndarray) -> int:
    thr = np.ascontiguousarray(thr, np.uint64)
    return lib().or_poisson_count(int(P), _ptr(thr))


def draws(seed: int, it: int, d: int, mu: float, m0: int, mc: int, k0: int, kc: int):
    """Brownian normals zw, jump normals zj (mc x kc x d) and counts (mc x kc)."""
    zw = np.empty((mc, kc, d))
    zj = np.empty((mc, kc, d))
    n = np.empty((mc, kc), np.int32)
    lib().or_draws_grid(seed, it, d, float(mu), m0, mc, k0, kc, _ptr(zw), _ptr(zj), _ptr(n))
    return zw, zj, n


def paths(p, seed: int, it: int, m0: int, count: int, u=None, nthreads: int | None = None):
    """Per-path X (count x (N+1) x d), lam (same; row 0 zero) and C (count)."""
    pr = _ProblemRef(p)
    u = _u(p, u)
    X = np.empty((count, p.N + 1, p.d))
    lam = np.empty((count, p.N + 1, p.d))
    Cm = np.empty(count)
    rc = lib().or_paths(pr.ref, seed, it, m0, count, _ptr(u), _ptr(X), _ptr(lam), _ptr(Cm),
                        nthreads or default_threads())
    if rc:
        raise ValueError(f"or_paths rejected the problem (rc={rc})")
    return X, lam, Cm


def cost_grad(p, M: int, seed: int, it: int, u=None, grad: bool = True,
              nthreads: int | None = None):
    """(J, g) with g of shape (N, d) (None when grad=False)."""
    pr = _ProblemRef(p)
    u = _u(p, u)
    J = np.zeros(1)
    g = np.empty((p.N, p.d)) if grad else None
    rc = lib().or_cost_grad(pr.ref, M, seed, it, _ptr(u), _ptr(J), _ptr(g) if grad else None,
                            nthreads or default_threads())
    if rc:
        raise ValueError(f"or_cost_grad failed (rc={rc})")
    return float(J[0]), g


def grad_scale(p, M: int, seed: int, it: int, u=None, nthreads: int | None = None):
    """Test diagnostic (N, d): per gradient entry, the mean over the paths of
    the absolute value of the path's summand, nu |u| + mean |B^T lam_{k+1}|."""
    pr = _ProblemRef(p)
    u = _u(p, u)
    s = np.empty((p.N, p.d))
    rc = lib().or_grad_scale(pr.ref, M, seed, it, _ptr(u), _ptr(s), nthreads or default_threads())
    if rc:
        raise ValueError(f"or_grad_scale failed (rc={rc})")
    return s


def tangent(p, M: int, seed: int, it: int, u, delta, nthreads: int | None = None) -> float:
    pr = _ProblemRef(p)
    u = _u(p, u)
    dl = _u(p, delta)
    out = np.zeros(1)
    rc = lib().or_tangent(pr.ref, M, seed, it, _ptr(u), _ptr(dl), _ptr(out),
                          nthreads or default_threads())
    if rc:
        raise ValueError(f"or_tangent failed (rc={rc})")
    return float(out[0])


def optimize(p, M: int, seed: int, it0: int, u0=None, n_max: int = 20, tol: float = 0.0,
             zeta0: float = 1.0, rho: float = 0.5, c_armijo: float = 1e-4,
             max_backtracks: int = 30, nthreads: int | None = None):
    """Returns (u_final, log dict, iterations done)."""
    pr = _ProblemRef(p)
    u = _u(p, u0).copy()
    opt = _Opt(n_max, tol, zeta0, rho, c_armijo, max_backtracks)
    logs = {k: np.zeros(max(n_max, 1)) for k in ("J", "gnorm", "zeta", "E")}
    bt = np.zeros(max(n_max, 1), np.int32)
    n = lib().or_optimize(pr.ref, M, seed, it0, C.byref(opt), _ptr(u), _ptr(logs["J"]),
                          _ptr(logs["gnorm"]), _ptr(logs["zeta"]), _ptr(bt), _ptr(logs["E"]),
                          nthreads or default_threads())
    if n < 0:
        raise RuntimeError(f"or_optimize failed (rc={n})")
    logs = {k: v[:n] for k, v in logs.items()}
    logs["backtracks"] = bt[:n]
    return u, logs, n


# ---------------------------------------------------------------------------
# The paper's model problem (fb_oracle.c): FeedbackProblem instances.

class _FbProblem(C.Structure):
    _fields_ = [("N", C.c_int32), ("nx", C.c_int32), ("nv", C.c_int32),
                ("T", C.c_double), ("eta", C.c_double), ("b1", C.c_double), ("b2", C.c_double),
                ("gamma", C.c_double), ("beta", C.c_double), ("xmax", C.c_double),
                ("vmax", C.c_double), ("eps", C.c_double), ("alpha", C.c_double),
                ("sigJ", C.c_double), ("init_kind", C.c_int32), ("z0", C.c_double * 2),
                ("s0", C.c_double * 2), ("svar0", C.c_double * 2), ("svar1", C.c_double * 2),
                ("zd", C.c_void_p), ("np", C.c_int32), ("omega", C.c_double),
                ("cost_kind", C.c_int32), ("ax", C.c_double), ("av", C.c_double),
                ("grid", C.c_int32), ("svar_kind", C.c_int32)]


def _bind_fb(L):
    if getattr(L, "_fb_bound", False):
        return L
    P = C.c_void_p
    L.fb_bump.argtypes = [C.c_double, C.c_double]
    L.fb_bump.restype = C.c_double
    L.fb_bump_deriv.argtypes = [C.c_double, C.c_double]
    L.fb_bump_deriv.restype = C.c_double
    L.fb_initial.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P]
    L.fb_step_draws.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P, P, P]
    L.fb_paths.argtypes = [P, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, P, P, P, P, P, P, C.c_int]
    L.fb_paths.restype = C.c_int
    L.fb_cost_grad.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, C.c_int]
    L.fb_cost_grad.restype = C.c_int
    L.fb_grad_scale.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, C.c_int]
    L.fb_grad_scale.restype = C.c_int
    L.fb_grad_scale_surrogate.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, C.c_int]
    L.fb_grad_scale_surrogate.restype = C.c_int
    L.fb_surrogate_state.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P]
    L.fb_cost_grad_surrogate.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, C.c_int]
    L.fb_cost_grad_surrogate.restype = C.c_int
    L.fb_tangent.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, C.c_int]
    L.fb_tangent.restype = C.c_int
    L.fb_optimize.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double,
                              C.c_double, C.c_double, C.c_double, C.c_int32, P, P, P, P, P, P,
                              C.c_int, C.c_int]
    L.fb_paths_surrogate.argtypes = [P, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, P, P, C.c_int]
    L.fb_paths_surrogate.restype = C.c_int
    L.fb_surrogate_fit.argtypes = [P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P, P, C.c_int]
    L.fb_surrogate_fit.restype = C.c_int
    L.fb_adapted_draws.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P, P, P, P, P]
    L.fb_optimize.restype = C.c_int
    L._fb_bound = True
    return L


def _fb():
    return _bind_fb(lib())


class _Fb:
    """Keeps the ctypes struct and the arrays it points to alive together."""

    def __init__(self, p):
        self.zd = np.ascontiguousarray(p.zd, np.float64)
        self.st = _FbProblem(p.N, p.nx, p.nv, p.T, p.eta, p.b1, p.b2, p.gamma, p.beta, p.xmax,
                             p.vmax, p.eps, p.alpha, p.sigJ, p.init_kind,
                             (C.c_double * 2)(*p.z0), (C.c_double * 2)(*p.s0),
                             (C.c_double * 2)(*p.svar0), (C.c_double * 2)(*p.svar1),
                             self.zd.ctypes.data, p.np, p.omega, p.cost_kind, p.ax, p.av, p.grid,
                             p.svar_kind)

    def ref(self):
        return C.byref(self.st)


def _mu(p, mu):
    return np.ascontiguousarray(np.asarray(mu, np.float64).reshape(p.N, p.L))


def fb_bump(r: float, eps: float) -> float:
    return _fb().fb_bump(float(r), float(eps))


def fb_bump_deriv(r: float, eps: float) -> float:
    return _fb().fb_bump_deriv(float(r), float(eps))


def fb_initial(p, seed: int, m: int, it: int) -> np.ndarray:
    z = np.zeros(2)
    fb = _Fb(p)
    _fb().fb_initial(fb.ref(), seed, m, it, _ptr(z))
    return z


def fb_step_draws(p, seed: int, m: int, k: int, it: int):
    """(Zx, Zv, ZJ), n for path m, step k."""
    thr = poisson_thresholds(p.rate * p.dt)
    Z = np.zeros(3)
    n = C.c_int()
    _fb().fb_step_draws(seed, m, k, it, _ptr(thr), _ptr(Z), C.byref(n))
    return Z, n.value


def fb_adapted_draws(p, seed: int, m: int, k: int, it: int):
    """Jump-adapted draws of interval k of particle m: (n, offsets a[0..n+1],
    sub-step normals (n+1, 2), jump normals S[1..n])."""
    thr = poisson_thresholds(p.rate * p.dt)
    n = C.c_int()
    a = np.zeros(33)
    Z = np.zeros(66)
    S = np.zeros(32)
    _fb().fb_adapted_draws(seed, m, k, it, _ptr(thr), C.byref(n), _ptr(a), _ptr(Z), _ptr(S))
    n = n.value
    return n, a[:n + 2].copy(), Z[:2 * (n + 1)].reshape(n + 1, 2).copy(), S[1:n + 1].copy()


def fb_paths(p, seed: int, it: int, m0: int, count: int, mu, nthreads: int | None = None):
    """Per-particle z (P, N+1, 2), lam (P, N+1, 2), u (P, N), jump counts (P, N)
    and costs (P) of systems m0..m0+count-1, P = count np (particle order)."""
    mu = _mu(p, mu)
    P = count * p.np
    z = np.zeros((P, p.N + 1, 2))
    lam = np.zeros((P, p.N + 1, 2))
    u = np.zeros((P, p.N))
    n = np.zeros((P, p.N), np.int32)
    c = np.zeros(P)
    fb = _Fb(p)
    rc = _fb().fb_paths(fb.ref(), seed, it, m0, count, _ptr(mu), _ptr(z), _ptr(lam), _ptr(u),
                        _ptr(n), _ptr(c), nthreads or default_threads())
    assert rc == 0, rc
    return z, lam, u, n, c


def fb_cost_grad(p, M: int, seed: int, it: int, mu, grad: bool = True,
                 nthreads: int | None = None):
    """(J, g) with g of shape (N, L) (None if grad is False)."""
    mu = _mu(p, mu)
    J = C.c_double()
    g = np.zeros((p.N, p.L)) if grad else None
    fb = _Fb(p)
    rc = _fb().fb_cost_grad(fb.ref(), M, seed, it, _ptr(mu), C.byref(J),
                            None if g is None else _ptr(g), nthreads or default_threads())
    assert rc == 0, rc
    return J.value, g


def fb_grad_scale(p, M: int, seed: int, it: int, mu, surrogate: bool = False,
                  nthreads: int | None = None) -> np.ndarray:
    """Test diagnostic (N, L): per gradient entry, the mean over the particles
    of the absolute value of the particle's summand (of the surrogate gradient
    when surrogate is set)."""
    mu = _mu(p, mu)
    s = np.zeros((p.N, p.L))
    fb = _Fb(p)
    fn = _fb().fb_grad_scale_surrogate if surrogate else _fb().fb_grad_scale
    rc = fn(fb.ref(), M, seed, it, _ptr(mu), _ptr(s), nthreads or default_threads())
    assert rc == 0, rc
    return s


def fb_surrogate_state(p, seed: int, m: int, k: int, it: int) -> np.ndarray:
    z = np.zeros(2)
    fb = _Fb(p)
    _fb().fb_surrogate_state(fb.ref(), seed, m, k, it, _ptr(z))
    return z


def fb_surrogate_fit(p, M: int, seed: int, it: int, mu, nthreads: int | None = None):
    """(var, a, b): the forward ensemble's per-step variance ((N+1, 2)) of M
    particles under mu and the least-squares line a + b t through it."""
    mu = _mu(p, mu)
    var = np.zeros((p.N + 1, 2))
    a, b = np.zeros(2), np.zeros(2)
    fb = _Fb(p)
    rc = _fb().fb_surrogate_fit(fb.ref(), M, seed, it, _ptr(mu), _ptr(var), _ptr(a), _ptr(b),
                                nthreads or default_threads())
    assert rc == 0, rc
    return var, a, b


def fb_paths_surrogate(p, seed: int, it: int, m0: int, count: int, mu) -> np.ndarray:
    """Per-path surrogate adjoints (count, N+1, 2)."""
    mu = _mu(p, mu)
    lam = np.zeros((count, p.N + 1, 2))
    fb = _Fb(p)
    rc = _fb().fb_paths_surrogate(fb.ref(), seed, it, m0, count, _ptr(mu), _ptr(lam), 1)
    assert rc == 0, rc
    return lam


def fb_cost_grad_surrogate(p, M: int, seed: int, it: int, mu, nthreads: int | None = None):
    """(J, gs): the exact cost and the surrogate gradient of Section 6.5."""
    mu = _mu(p, mu)
    J = C.c_double()
    g = np.zeros((p.N, p.L))
    fb = _Fb(p)
    rc = _fb().fb_cost_grad_surrogate(fb.ref(), M, seed, it, _ptr(mu), C.byref(J), _ptr(g),
                                      nthreads or default_threads())
    assert rc == 0, rc
    return J.value, g


def fb_tangent(p, M: int, seed: int, it: int, mu, dmu, nthreads: int | None = None) -> float:
    mu, dmu = _mu(p, mu), _mu(p, dmu)
    dJ = C.c_double()
    fb = _Fb(p)
    rc = _fb().fb_tangent(fb.ref(), M, seed, it, _ptr(mu), _ptr(dmu), C.byref(dJ),
                          nthreads or default_threads())
    assert rc == 0, rc
    return dJ.value


def fb_optimize(p, M: int, seed: int, it0: int, mu, n_max: int, tol: float = 0.0,
                zeta0: float = 1.0, rho: float = 0.5, c_armijo: float = 1e-4,
                max_backtracks: int = 30, surrogate: bool = False, nthreads: int | None = None):
    """Returns (mu, logs, n) like ``optimize``."""
    mu = _mu(p, mu).copy()
    nm = max(n_max, 1)
    lJ, lg, lz, lE = np.zeros(nm), np.zeros(nm), np.zeros(nm), np.zeros(nm)
    lb = np.zeros(nm, np.int32)
    fb = _Fb(p)
    n = _fb().fb_optimize(fb.ref(), M, seed, it0, n_max, tol, zeta0, rho, c_armijo,
                          max_backtracks, _ptr(mu), _ptr(lJ), _ptr(lg), _ptr(lz), _ptr(lb),
                          _ptr(lE), 1 if surrogate else 0, nthreads or default_threads())
    logs = [dict(J=lJ[i], gnorm=lg[i], zeta=lz[i], backtracks=int(lb[i]), E=lE[i])
            for i in range(max(n, 0))]
    return mu, logs, n
