"""Request loop over the libjd request server (include/jd_server.h).

``Server`` wraps the C server: one device arena (a torch allocation), requests
submitted with their host data, a non-blocking progress call, results fetched
once.  ``run_mix`` replays a list of timed requests (Poisson arrivals) against
a server in wall-clock time and records each request's latency (completion
minus arrival) and the work done.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import time

import numpy as np

from . import binding as B


def _bind_server(L):
    P = C.c_void_p
    if getattr(L, "_server_bound", False):
        return L
    L.jd_server_request_bytes.argtypes = [P, P]
    L.jd_server_request_bytes.restype = C.c_size_t
    L.jd_server_create.argtypes = [P, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
    L.jd_server_create.restype = C.c_int
    L.jd_server_submit.argtypes = [P, P, P, P, P, P, C.POINTER(C.c_int64)]
    L.jd_server_submit.restype = C.c_int
    L.jd_server_progress.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64)]
    L.jd_server_progress.restype = C.c_int
    L.jd_server_result.argtypes = [P, C.c_int64, P, P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.jd_server_result.restype = C.c_int
    L.jd_server_times.argtypes = [P, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.jd_server_times.restype = C.c_int
    L.jd_server_destroy.argtypes = [P]
    L.jd_server_destroy.restype = C.c_int
    L._server_bound = True
    return L


def lib():
    return _bind_server(B.lib())


class _HostProblem:
    """jd_problem with host arrays only (the server copies x_d itself)."""

    def __init__(self, p):
        self.p = p
        self._keep = [np.ascontiguousarray(a, np.float64) for a in
                      (p.x0, p.A, p.B, p.s, p.jump_mean, p.jump_std, p.xT, p.xd)]
        x0, A, Bm, s, jm, js, xT, xd = self._keep
        self.xd = xd
        self.st = B.jd_problem(p.d, p.N, p.T, p.lam, p.cubic, p.nu, x0.ctypes.data, A.ctypes.data,
                               Bm.ctypes.data, s.ctypes.data, jm.ctypes.data, js.ctypes.data,
                               xT.ctypes.data, xd.ctypes.data)


def request_bytes(p, M: int, precision: str = "fp32", mode: str = "store", K: int = 0) -> int:
    hp = _HostProblem(p)
    run = B.make_run(M, 1, 0, precision, mode, K)
    return lib().jd_server_request_bytes(C.byref(hp.st), C.byref(run))


class Server:
    def __init__(self, arena_bytes: int, max_active: int = 32, n_streams: int = 4,
                 device="cuda:0"):
        import torch
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.h = C.c_void_p()
        B.check(lib().jd_server_create(self.arena.data_ptr(), arena_bytes, max_active, n_streams,
                                       C.byref(self.h)), "jd_server_create")
        self.n = {}
        self.max_active = max_active
        # what progress() has seen: the most requests admitted and queued at
        # once, and how many times requests waited in the queue while a slot
        # was free (that is, for arena memory)
        self.stats = dict(max_active=0, max_queued=0, waited_for_memory=0)

    def submit(self, p, M: int, seed: int, iters: int, precision: str = "fp32",
               mode: str = "store", K: int = 0, it0: int = 0, u0=None, tol: float = 0.0,
               zeta0: float = 1.0, rho: float = 0.5, c_armijo: float = 1e-4,
               max_backtracks: int = 30) -> int:
        hp = _HostProblem(p)
        run = B.make_run(M, seed, it0, precision, mode, K)
        opt = B.jd_opt(iters, max_backtracks, tol, zeta0, rho, c_armijo)
        u = None if u0 is None else np.ascontiguousarray(u0, np.float64)
        t = C.c_int64()
        B.check(lib().jd_server_submit(self.h, C.byref(hp.st), hp.xd.ctypes.data, C.byref(run),
                                       C.byref(opt), None if u is None else u.ctypes.data,
                                       C.byref(t)), "jd_server_submit")
        self.n[t.value] = (p.N, p.d, iters)
        return t.value

    def progress(self):
        a, q, c = C.c_int32(), C.c_int32(), C.c_int64()
        B.check(lib().jd_server_progress(self.h, C.byref(a), C.byref(q), C.byref(c)),
                "jd_server_progress")
        st = self.stats
        st["max_active"] = max(st["max_active"], a.value)
        st["max_queued"] = max(st["max_queued"], q.value)
        if q.value > 0 and a.value < self.max_active:
            st["waited_for_memory"] += 1
        return a.value, q.value, c.value

    def times(self, ticket: int):
        """(queued, service) seconds of a finished request whose result has
        not been taken, or None while it runs."""
        qd, sv = C.c_double(), C.c_double()
        rc = lib().jd_server_times(self.h, ticket, C.byref(qd), C.byref(sv))
        if rc == -7:  # JD_EAGAIN
            return None
        B.check(rc, "jd_server_times")
        return qd.value, sv.value

    def result(self, ticket: int):
        """None while running; else dict(u, log, status, queued, service)."""
        tm = self.times(ticket)
        if tm is None:
            return None
        N, d, iters = self.n[ticket]
        u = np.empty((N, d))
        logs = (B.jd_iter_log * max(iters, 1))()
        n, status = C.c_int32(), C.c_int32()
        rc = lib().jd_server_result(self.h, ticket, u.ctypes.data, logs, C.byref(n), C.byref(status))
        if rc == -7:  # JD_EAGAIN
            return None
        B.check(rc, "jd_server_result")
        del self.n[ticket]
        log = [dict(iter=l.iter, backtracks=l.backtracks, J=l.J, gnorm=l.gnorm, zeta=l.zeta,
                    J_new=l.J_new, E=l.E) for l in logs[:n.value]]
        return dict(u=u, log=log, status=status.value, queued=tm[0], service=tm[1])

    def close(self):
        if self.h:
            lib().jd_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Record:
    rid: int
    ticket: int
    arrival: float
    submitted: float = 0.0
    done: float = float("nan")
    queued: float = float("nan")   # the server's admission - submission
    service: float = float("nan")  # the server's completion - admission
    status: int = 0
    iterations: int = 0
    trials: int = 0
    path_steps: float = 0.0  # M * N per gradient evaluation (forward + adjoint)
    swept: float = 0.0       # M * N per sweep (forward, adjoint, every trial forward)
    u: np.ndarray | None = None
    log: list | None = None

    @property
    def latency(self):
        return self.done - self.arrival


def choose_mode(p, M: int, precision: str, store_limit: int):
    """Stored trajectory when it fits store_limit bytes, else checkpoints every
    64 steps (128 at d = 1)."""
    esz = 4 if precision == "fp32" else 8
    if p.N * p.d * ((M + 255) // 256 * 256) * esz <= store_limit:
        return "store", 0
    return "recompute", min(128 if p.d == 1 else 64, p.N)


def run_mix(server: Server, requests, precision: str = "fp32", store_limit: int = 8 << 30,
            time_scale: float = 1.0, timeout: float = 3600.0, on_done=None):
    """Submits each request at its arrival time (scaled), drives the server until
    all are done; returns (records, wall seconds)."""
    order = sorted(requests, key=lambda r: r.arrival)
    recs = []
    t0 = time.perf_counter()
    i = 0
    pending = {}
    while i < len(order) or pending:
        now = time.perf_counter() - t0
        while i < len(order) and order[i].arrival * time_scale <= now:
            r = order[i]
            mode, K = choose_mode(r.problem, r.M, precision, store_limit)
            tk = server.submit(r.problem, r.M, r.seed, r.iters, precision, mode, K)
            rec = Record(rid=r.rid, ticket=tk, arrival=r.arrival * time_scale, submitted=now)
            pending[tk] = (rec, r)
            recs.append(rec)
            i += 1
        server.progress()
        for tk in list(pending):
            res = server.result(tk)
            if res is None:
                continue
            rec, r = pending.pop(tk)
            rec.done = time.perf_counter() - t0
            rec.status = res["status"]
            rec.queued, rec.service = res["queued"], res["service"]
            rec.iterations = len(res["log"])
            rec.trials = sum(1 + l["backtracks"] for l in res["log"])
            rec.path_steps = rec.iterations * r.M * r.problem.N
            rec.swept = (2 * rec.iterations + rec.trials) * r.M * r.problem.N
            rec.u = res["u"]
            rec.log = res["log"]
            if on_done:
                on_done(rec)
        if time.perf_counter() - t0 > timeout:
            raise TimeoutError("serving mix did not finish")
    return recs, time.perf_counter() - t0
