"""ctypes binding of libjd (include/jd.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of ``libjd.so``; this module
turns torch device tensors into raw device pointers plus torch's current HIP
stream and back.  There is no fallback: if the library is missing the import
of ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjd.so")

JD_OK, JD_EINVAL, JD_EWORKSPACE, JD_EHIP, JD_ENONFINITE, JD_ELINESEARCH, JD_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
JD_EAGAIN = -7
JD_FP32, JD_FP64 = 0, 1
JD_STORE, JD_RECOMPUTE, JD_SURROGATE = 0, 1, 2
JD_NOISE_AUTO, JD_NOISE_INLINE, JD_NOISE_TABLE = 0, 1, 2

EXPORTED = ["jd_version", "jd_strerror", "jd_workspace_bytes", "jd_traj_bytes", "jd_forward",
            "jd_adjoint", "jd_cost_grad", "jd_optimize", "jd_check_finite", "jd_draws",
            "jd_philox", "jd_poisson_thresholds", "jd_noalloc_capacity", "jd_cost_grad_noalloc"]
# include/jd_feedback.h
EXPORTED_FB = ["jd_fb_workspace_bytes", "jd_fb_traj_bytes", "jd_fb_forward", "jd_fb_adjoint",
               "jd_fb_cost_grad", "jd_fb_optimize", "jd_fb_draws"]


class JdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib().jd_strerror(code).decode()} ({code})")


class jd_problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("N", C.c_int32), ("T", C.c_double), ("lambda_", C.c_double),
                ("cubic", C.c_double), ("nu", C.c_double), ("x0", C.c_void_p), ("A", C.c_void_p),
                ("B", C.c_void_p), ("s", C.c_void_p), ("jump_mean", C.c_void_p),
                ("jump_std", C.c_void_p), ("xT", C.c_void_p), ("xd", C.c_void_p)]


class jd_dump(C.Structure):
    _fields_ = [("m0", C.c_int64), ("count", C.c_int64), ("X", C.c_void_p), ("lam", C.c_void_p),
                ("cost", C.c_void_p)]


class jd_run(C.Structure):
    _fields_ = [("M", C.c_int64), ("seed", C.c_uint64), ("iter", C.c_uint32),
                ("precision", C.c_int32), ("mode", C.c_int32), ("K", C.c_int32),
                ("dump", C.POINTER(jd_dump)), ("noise", C.c_int32)]


class jd_opt(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("max_backtracks", C.c_int32), ("tol", C.c_double),
                ("zeta0", C.c_double), ("rho", C.c_double), ("c_armijo", C.c_double)]


class jd_iter_log(C.Structure):
    _fields_ = [("iter", C.c_uint32), ("backtracks", C.c_int32), ("J", C.c_double),
                ("gnorm", C.c_double), ("zeta", C.c_double), ("J_new", C.c_double),
                ("E", C.c_double)]


_lib = None


def lib():
    """The loaded libjd.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2505_04328_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.jd_version.restype = C.c_int
        L.jd_strerror.argtypes = [C.c_int]
        L.jd_strerror.restype = C.c_char_p
        L.jd_workspace_bytes.argtypes = [P, P]
        L.jd_workspace_bytes.restype = C.c_size_t
        L.jd_traj_bytes.argtypes = [P, P]
        L.jd_traj_bytes.restype = C.c_size_t
        L.jd_forward.argtypes = [P, P, P, P, P, P, C.c_size_t, P]
        L.jd_adjoint.argtypes = [P, P, P, P, P, P, C.c_size_t, P]
        L.jd_cost_grad.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P]
        L.jd_optimize.argtypes = [P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.jd_check_finite.argtypes = [P, C.c_size_t, P]
        L.jd_draws.argtypes = [P, P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, P, P, P, P]
        L.jd_philox.argtypes = [C.c_uint64, P, C.c_int64, P, P]
        L.jd_poisson_thresholds.argtypes = [C.c_double, P]
        L.jd_noalloc_capacity.argtypes = []
        L.jd_cost_grad_noalloc.argtypes = [P, P, P, P, P, P, P]
        for name in EXPORTED:
            if name not in ("jd_version", "jd_strerror", "jd_workspace_bytes", "jd_traj_bytes",
                            "jd_noalloc_capacity"):
                getattr(L, name).restype = C.c_int
        L.jd_noalloc_capacity.restype = C.c_size_t
        L.jd_fb_workspace_bytes.argtypes = [P, P]
        L.jd_fb_workspace_bytes.restype = C.c_size_t
        L.jd_fb_traj_bytes.argtypes = [P, P]
        L.jd_fb_traj_bytes.restype = C.c_size_t
        L.jd_fb_forward.argtypes = [P, P, P, P, P, P, C.c_size_t, P]
        L.jd_fb_adjoint.argtypes = [P, P, P, P, P, P, C.c_size_t, P]
        L.jd_fb_cost_grad.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P]
        L.jd_fb_optimize.argtypes = [P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.jd_fb_draws.argtypes = [P, P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, P, P, P, P]
        for name in EXPORTED_FB[2:]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(code: int, where: str):
    if code != JD_OK:
        raise JdError(code, where)


def _torch():
    import torch
    return torch


def _stream_ptr(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _dptr(t) -> int:
    return 0 if t is None else t.data_ptr()


class Problem:
    """Host problem data packed for the C ABI, with x_d on the device."""

    def __init__(self, p, device="cuda:0"):
        torch = _torch()
        self.p = p
        self.device = torch.device(device)
        self._keep = [np.ascontiguousarray(a, np.float64) for a in
                      (p.x0, p.A, p.B, p.s, p.jump_mean, p.jump_std, p.xT)]
        x0, A, B, s, jm, js, xT = self._keep
        self.xd = torch.from_numpy(np.ascontiguousarray(p.xd, np.float64)).to(self.device)
        self.st = jd_problem(p.d, p.N, p.T, p.lam, p.cubic, p.nu, x0.ctypes.data, A.ctypes.data,
                             B.ctypes.data, s.ctypes.data, jm.ctypes.data, js.ctypes.data,
                             xT.ctypes.data, self.xd.data_ptr())

    @property
    def ref(self):
        return C.byref(self.st)


NOISE = {"auto": JD_NOISE_AUTO, "inline": JD_NOISE_INLINE, "table": JD_NOISE_TABLE}


def make_run(M: int, seed: int = 1, it: int = 0, precision: str = "fp32", mode: str = "store",
             K: int = 0, dump: jd_dump | None = None, noise: str = "auto") -> jd_run:
    prec = {"fp32": JD_FP32, "fp64": JD_FP64}[precision]
    md = {"store": JD_STORE, "recompute": JD_RECOMPUTE, "surrogate": JD_SURROGATE}[mode]
    return jd_run(M, seed, it, prec, md, K, C.pointer(dump) if dump is not None else None,
                  NOISE[noise])


class Engine:
    """One problem + Monte Carlo configuration with its device buffers
    (workspace and trajectory/checkpoint buffer) allocated by torch."""

    def __init__(self, problem, M: int, seed: int = 1, precision: str = "fp32",
                 mode: str = "store", K: int = 0, device="cuda:0", noise: str = "auto"):
        torch = _torch()
        self.prob = problem if isinstance(problem, Problem) else Problem(problem, device)
        self.p = self.prob.p
        self.M, self.seed, self.precision, self.mode, self.K = M, seed, precision, mode, K
        self.noise = noise
        self.device = self.prob.device
        self.rdtype = torch.float32 if precision == "fp32" else torch.float64
        run = make_run(M, seed, 0, precision, mode, K, noise=noise)
        L = lib()
        self.ws_bytes = L.jd_workspace_bytes(self.prob.ref, C.byref(run))
        self.traj_bytes = L.jd_traj_bytes(self.prob.ref, C.byref(run))
        if self.ws_bytes == 0 or self.traj_bytes == 0:
            raise JdError(JD_EINVAL, "Engine")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        esz = 4 if precision == "fp32" else 8
        self.nblk = (M + 255) // 256
        self.traj = torch.empty(self.traj_bytes // esz, dtype=self.rdtype, device=self.device)

    def run(self, it: int = 0, dump: jd_dump | None = None) -> jd_run:
        return make_run(self.M, self.seed, it, self.precision, self.mode, self.K, dump,
                        self.noise)

    def _u(self, u):
        torch = _torch()
        if isinstance(u, np.ndarray):
            u = torch.from_numpy(np.ascontiguousarray(u, np.float64))
        u = u.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(u.shape) == (self.p.N, self.p.d), u.shape
        return u

    def trajectory(self):
        """The trajectory / checkpoint buffer as a (slots, d, M) tensor (a copy:
        the buffer is blocked by 256 paths, see jd_traj_bytes)."""
        slots = self.traj.numel() // (self.p.d * self.nblk * 256)
        t = self.traj.view(self.nblk, slots, self.p.d, 256).permute(1, 2, 0, 3)
        return t.reshape(slots, self.p.d, self.nblk * 256)[:, :, :self.M]

    def forward(self, u, it: int = 0, store: bool = True, dump: jd_dump | None = None):
        torch = _torch()
        u = self._u(u)
        J = torch.empty((), dtype=torch.float64, device=self.device)
        run = self.run(it, dump)
        check(lib().jd_forward(self.prob.ref, C.byref(run), u.data_ptr(),
                               self.traj.data_ptr() if store else None, J.data_ptr(),
                               self.ws.data_ptr(), self.ws_bytes, _stream_ptr(self.device)),
              "jd_forward")
        return J

    def adjoint(self, u, it: int = 0, dump: jd_dump | None = None):
        torch = _torch()
        u = self._u(u)
        g = torch.empty((self.p.N, self.p.d), dtype=torch.float64, device=self.device)
        run = self.run(it, dump)
        check(lib().jd_adjoint(self.prob.ref, C.byref(run), u.data_ptr(), self.traj.data_ptr(),
                               g.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                               _stream_ptr(self.device)), "jd_adjoint")
        return g

    def cost_grad(self, u, it: int = 0, J=None, g=None):
        torch = _torch()
        u = self._u(u)
        if J is None:
            J = torch.empty((), dtype=torch.float64, device=self.device)
        if g is None:
            g = torch.empty((self.p.N, self.p.d), dtype=torch.float64, device=self.device)
        run = self.run(it)
        check(lib().jd_cost_grad(self.prob.ref, C.byref(run), u.data_ptr(), J.data_ptr(),
                                 g.data_ptr(), self.traj.data_ptr(), self.ws.data_ptr(),
                                 self.ws_bytes, _stream_ptr(self.device)), "jd_cost_grad")
        return J, g

    def optimize(self, u, n_max: int, it0: int = 0, tol: float = 0.0, zeta0: float = 1.0,
                 rho: float = 0.5, c_armijo: float = 1e-4, max_backtracks: int = 30):
        """Runs the gradient iteration in place on the device tensor u; returns
        (u, list of per-iteration dicts)."""
        u = self._u(u)
        opt = jd_opt(n_max, max_backtracks, tol, zeta0, rho, c_armijo)
        logs = (jd_iter_log * max(n_max, 1))()
        done = C.c_int32(0)
        run = self.run(it0)
        rc = lib().jd_optimize(self.prob.ref, C.byref(run), C.byref(opt), u.data_ptr(), logs,
                               C.byref(done), self.traj.data_ptr(), self.ws.data_ptr(),
                               self.ws_bytes, _stream_ptr(self.device))
        out = [dict(iter=l.iter, backtracks=l.backtracks, J=l.J, gnorm=l.gnorm, zeta=l.zeta,
                    J_new=l.J_new, E=l.E) for l in logs[:done.value]]
        check(rc, "jd_optimize")
        return u, out

    def check_finite(self) -> bool:
        rc = lib().jd_check_finite(self.ws.data_ptr(), self.ws_bytes, _stream_ptr(self.device))
        if rc == JD_ENONFINITE:
            return False
        check(rc, "jd_check_finite")
        return True

    def draws(self, m0: int, mc: int, k0: int, kc: int, it: int = 0):
        torch = _torch()
        d = self.p.d
        zw = torch.empty((mc, kc, d), dtype=self.rdtype, device=self.device)
        zj = torch.empty((mc, kc, d), dtype=self.rdtype, device=self.device)
        n = torch.empty((mc, kc), dtype=torch.int32, device=self.device)
        run = self.run(it)
        check(lib().jd_draws(self.prob.ref, C.byref(run), m0, mc, k0, kc, zw.data_ptr(),
                             zj.data_ptr(), n.data_ptr(), _stream_ptr(self.device)), "jd_draws")
        return zw, zj, n

    def path_dump(self, m0: int, count: int):
        """Allocates a dump for paths [m0, m0+count): returns (jd_dump, tensors)."""
        torch = _torch()
        N, d = self.p.N, self.p.d
        X = torch.zeros((N, d, count), dtype=self.rdtype, device=self.device)
        lam = torch.zeros((N, d, count), dtype=self.rdtype, device=self.device)
        cost = torch.zeros(count, dtype=torch.float64, device=self.device)
        dp = jd_dump(m0, count, X.data_ptr(), lam.data_ptr(), cost.data_ptr())
        return dp, dict(X=X, lam=lam, cost=cost)


def philox(seed: int, ctr, device="cuda:0"):
    """Raw Philox4x32-10 blocks on the device for counters ctr (n x 4 uint32)."""
    torch = _torch()
    c = torch.as_tensor(np.ascontiguousarray(ctr, np.uint32).view(np.int32)).reshape(-1, 4)
    c = c.to(device)
    out = torch.empty_like(c)
    check(lib().jd_philox(seed, c.data_ptr(), c.shape[0], out.data_ptr(), _stream_ptr(device)),
          "jd_philox")
    return out.cpu().numpy().view(np.uint32)


def poisson_thresholds(mu: float) -> np.ndarray:
    t = np.zeros(32, np.uint64)
    check(lib().jd_poisson_thresholds(float(mu), t.ctypes.data), "jd_poisson_thresholds")
    return t


# ---------------------------------------------------------------------------
# The paper's model problem (include/jd_feedback.h).

JD_FB_INIT_GAUSS, JD_FB_INIT_UNIFORM, JD_FB_INIT_ELLIPSE = 0, 1, 2
JD_FB_COST_TRACK, JD_FB_COST_ELLIPSE = 0, 1
JD_FB_MAX_RING = 2048
JD_FB_GRID_FIXED, JD_FB_GRID_ADAPTED = 0, 1
JD_FB_SVAR_GIVEN, JD_FB_SVAR_FIT = 0, 1


class jd_fb_problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("nx", C.c_int32), ("nv", C.c_int32), ("T", C.c_double),
                ("eta", C.c_double), ("b1", C.c_double), ("b2", C.c_double),
                ("gamma", C.c_double), ("beta", C.c_double), ("xmax", C.c_double),
                ("vmax", C.c_double), ("eps", C.c_double), ("alpha", C.c_double),
                ("sigJ", C.c_double), ("init_kind", C.c_int32), ("z0", C.c_double * 2),
                ("s0", C.c_double * 2), ("svar0", C.c_double * 2), ("svar1", C.c_double * 2),
                ("zd", C.c_void_p), ("np", C.c_int32), ("omega", C.c_double),
                ("cost_kind", C.c_int32), ("ax", C.c_double), ("av", C.c_double),
                ("grid", C.c_int32), ("svar_kind", C.c_int32)]


class FbProblem:
    """A workloads.FeedbackProblem packed for the C ABI, z_d on the device."""

    def __init__(self, p, device="cuda:0"):
        torch = _torch()
        self.p = p
        self.device = torch.device(device)
        self.zd = torch.from_numpy(np.ascontiguousarray(p.zd, np.float64)).to(self.device)
        self.st = jd_fb_problem(p.N, p.nx, p.nv, p.T, p.eta, p.b1, p.b2, p.gamma, p.beta, p.xmax,
                                p.vmax, p.eps, p.alpha, p.sigJ, p.init_kind,
                                (C.c_double * 2)(*p.z0), (C.c_double * 2)(*p.s0),
                                (C.c_double * 2)(*p.svar0), (C.c_double * 2)(*p.svar1),
                                self.zd.data_ptr(), p.np, p.omega, p.cost_kind, p.ax, p.av, p.grid,
                                p.svar_kind)

    @property
    def ref(self):
        return C.byref(self.st)


class FbEngine:
    """Feedback-model problem + Monte Carlo configuration with its workspace and
    trajectory buffers (torch allocations).  M counts realizations: particles
    for independent particles, rings of np particles otherwise (M np
    particles); particle indices (dumps, draws) run over all of them."""

    def __init__(self, problem, M: int, seed: int = 1, precision: str = "fp32", device="cuda:0",
                 mode: str = "store"):
        """mode 'store' (exact gradient over the stored trajectory) or
        'surrogate' (the storage-free surrogate gradient of Section 6.5)."""
        torch = _torch()
        self.prob = problem if isinstance(problem, FbProblem) else FbProblem(problem, device)
        self.p = self.prob.p
        self.M, self.seed, self.precision, self.mode = M, seed, precision, mode
        self.device = self.prob.device
        self.rdtype = torch.float32 if precision == "fp32" else torch.float64
        run = make_run(M, seed, 0, precision, mode)
        L = lib()
        self.ws_bytes = L.jd_fb_workspace_bytes(self.prob.ref, C.byref(run))
        self.traj_bytes = L.jd_fb_traj_bytes(self.prob.ref, C.byref(run))
        if self.ws_bytes == 0 or self.traj_bytes == 0:
            raise JdError(JD_EINVAL, "FbEngine")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        esz = 4 if precision == "fp32" else 8
        self.particles = M * self.p.np
        npr = self.p.np
        if npr == 1:
            self.nblk = (M + 255) // 256
        else:
            G = 1 if npr <= 256 else 8
            R = 256 * G // npr
            self.nblk = (M + R - 1) // R * G
        self.traj = torch.empty(self.traj_bytes // esz, dtype=self.rdtype, device=self.device)

    def slots(self) -> np.ndarray:
        """Trajectory slot of every particle (the layout of include/jd_feedback.h)."""
        npr = self.p.np
        if npr == 1:
            return np.arange(self.M)
        G = 1 if npr <= 256 else 8
        R = 256 * G // npr
        r = np.repeat(np.arange(self.M), npr)
        j = np.tile(np.arange(npr), self.M)
        return (r // R) * 256 * G + (r % R) * npr + j

    def run(self, it: int = 0, dump: jd_dump | None = None) -> jd_run:
        return make_run(self.M, self.seed, it, self.precision, self.mode, 0, dump)

    def _mu(self, mu):
        torch = _torch()
        if isinstance(mu, np.ndarray):
            mu = torch.from_numpy(np.ascontiguousarray(mu, np.float64))
        mu = mu.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(mu.shape) == (self.p.N, self.p.L), mu.shape
        return mu

    def trajectory(self):
        """z_0..z_N as an (N+1, 2, particles) tensor (a copy of the blocked buffer)."""
        torch = _torch()
        n = self.nblk * (self.p.N + 1) * 2 * 256  # the states; jump data follows
        t = self.traj[:n].view(self.nblk, self.p.N + 1, 2, 256).permute(1, 2, 0, 3)
        t = t.reshape(self.p.N + 1, 2, self.nblk * 256)
        if self.p.np == 1:
            return t[:, :, :self.M]
        return t[:, :, torch.from_numpy(self.slots()).to(self.device)]

    def forward(self, mu, it: int = 0, store: bool = True, dump: jd_dump | None = None):
        torch = _torch()
        mu = self._mu(mu)
        J = torch.empty((), dtype=torch.float64, device=self.device)
        run = self.run(it, dump)
        check(lib().jd_fb_forward(self.prob.ref, C.byref(run), mu.data_ptr(),
                                  self.traj.data_ptr() if store else None, J.data_ptr(),
                                  self.ws.data_ptr(), self.ws_bytes, _stream_ptr(self.device)),
              "jd_fb_forward")
        return J

    def adjoint(self, mu, it: int = 0, dump: jd_dump | None = None):
        torch = _torch()
        mu = self._mu(mu)
        g = torch.empty((self.p.N, self.p.L), dtype=torch.float64, device=self.device)
        run = self.run(it, dump)
        check(lib().jd_fb_adjoint(self.prob.ref, C.byref(run), mu.data_ptr(),
                                  self.traj.data_ptr(), g.data_ptr(), self.ws.data_ptr(),
                                  self.ws_bytes, _stream_ptr(self.device)), "jd_fb_adjoint")
        return g

    def cost_grad(self, mu, it: int = 0, J=None, g=None, dump: jd_dump | None = None):
        torch = _torch()
        mu = self._mu(mu)
        if J is None:
            J = torch.empty((), dtype=torch.float64, device=self.device)
        if g is None:
            g = torch.empty((self.p.N, self.p.L), dtype=torch.float64, device=self.device)
        run = self.run(it, dump)
        check(lib().jd_fb_cost_grad(self.prob.ref, C.byref(run), mu.data_ptr(), J.data_ptr(),
                                    g.data_ptr(), self.traj.data_ptr(), self.ws.data_ptr(),
                                    self.ws_bytes, _stream_ptr(self.device)), "jd_fb_cost_grad")
        return J, g

    def optimize(self, mu, n_max: int, it0: int = 0, tol: float = 0.0, zeta0: float = 1.0,
                 rho: float = 0.5, c_armijo: float = 1e-4, max_backtracks: int = 30,
                 allow_stall: bool = False):
        """The gradient iteration; mu is updated in place.  allow_stall: a line
        search that finds no Armijo step ends the iteration (JD_ELINESEARCH,
        mu at the last accepted iterate) instead of raising."""
        mu = self._mu(mu)
        opt = jd_opt(n_max, max_backtracks, tol, zeta0, rho, c_armijo)
        logs = (jd_iter_log * max(n_max, 1))()
        done = C.c_int32(0)
        run = self.run(it0)
        rc = lib().jd_fb_optimize(self.prob.ref, C.byref(run), C.byref(opt), mu.data_ptr(), logs,
                                  C.byref(done), self.traj.data_ptr(), self.ws.data_ptr(),
                                  self.ws_bytes, _stream_ptr(self.device))
        out = [dict(iter=l.iter, backtracks=l.backtracks, J=l.J, gnorm=l.gnorm, zeta=l.zeta,
                    J_new=l.J_new, E=l.E) for l in logs[:done.value]]
        if not (allow_stall and rc == JD_ELINESEARCH):
            check(rc, "jd_fb_optimize")
        return mu, out

    def check_finite(self) -> bool:
        rc = lib().jd_check_finite(self.ws.data_ptr(), self.ws_bytes, _stream_ptr(self.device))
        if rc == JD_ENONFINITE:
            return False
        check(rc, "jd_check_finite")
        return True

    def draws(self, m0: int, mc: int, k0: int, kc: int, it: int = 0):
        """(z_init (mc, 2), Z (mc, kc, 3), counts (mc, kc))."""
        torch = _torch()
        zi = torch.empty((mc, 2), dtype=self.rdtype, device=self.device)
        Z = torch.empty((mc, kc, 3), dtype=self.rdtype, device=self.device)
        n = torch.empty((mc, kc), dtype=torch.int32, device=self.device)
        run = self.run(it)
        check(lib().jd_fb_draws(self.prob.ref, C.byref(run), m0, mc, k0, kc, zi.data_ptr(),
                                Z.data_ptr(), n.data_ptr(), _stream_ptr(self.device)),
              "jd_fb_draws")
        return zi, Z, n

    def path_dump(self, m0: int, count: int):
        """Dump buffers for particles [m0, m0+count): z and lam (N+1, 2, count), cost."""
        torch = _torch()
        N = self.p.N
        X = torch.zeros((N + 1, 2, count), dtype=self.rdtype, device=self.device)
        lam = torch.zeros((N + 1, 2, count), dtype=self.rdtype, device=self.device)
        cost = torch.zeros(count, dtype=torch.float64, device=self.device)
        dp = jd_dump(m0, count, X.data_ptr(), lam.data_ptr(), cost.data_ptr())
        return dp, dict(X=X, lam=lam, cost=cost)
