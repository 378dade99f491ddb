"""The C-ABI library loads, exports every symbol include/jd.h declares, and
rejects invalid arguments before anything is enqueued.  Host-only: no call here
reaches the GPU (every call returns from validation or is host arithmetic)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import ref
from paper_2505_04328_amd import binding as B
from paper_2505_04328_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("jd.h", "jd_server.h", "jd_feedback.h")]


def _gpu_visible() -> bool:
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


# Validation tests hand fake device addresses to the entry points; they are
# meant for the host only and never run where a GPU is visible.
host_only = pytest.mark.skipif(_gpu_visible(), reason="host-only validation test")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_2505_04328_amd import build
        build.build()
    return B.lib()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(jd_[a-z_0-9]+)\s*\(", text,
                                flags=re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12, names
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(B.EXPORTED) | set(SERVER) | set(B.EXPORTED_FB) == set(names)


SERVER = ["jd_server_request_bytes", "jd_server_create", "jd_server_submit",
          "jd_server_progress", "jd_server_result", "jd_server_times", "jd_server_destroy"]


def test_version_and_strerror(L):
    assert L.jd_version() == 101
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(L.jd_strerror(code), bytes)


@pytest.mark.parametrize("mu", [0.0, 0.002, 0.005, 0.012, 0.02, 0.1, 1.0, 2.0])
def test_poisson_thresholds_match_oracle_bitwise(L, mu):
    """Two independent FP64 implementations of the same threshold sequence agree
    exactly (both are then pinned against scipy's CDF by the oracle tests)."""
    np.testing.assert_array_equal(B.poisson_thresholds(mu), ref.poisson_thresholds(mu))


class _Dummy:
    """A problem whose x_d pointer is a fake non-null address: only validation runs."""

    def __init__(self, p):
        self.p = p
        self._keep = [np.ascontiguousarray(a, np.float64) for a in
                      (p.x0, p.A, p.B, p.s, p.jump_mean, p.jump_std, p.xT)]
        x0, A, Bm, s, jm, js, xT = self._keep
        self.st = B.jd_problem(p.d, p.N, p.T, p.lam, p.cubic, p.nu, x0.ctypes.data,
                               A.ctypes.data, Bm.ctypes.data, s.ctypes.data, jm.ctypes.data,
                               js.ctypes.data, xT.ctypes.data, 0x1000)


def _sizes(L, prob, run):
    return L.jd_workspace_bytes(C.byref(prob.st), C.byref(run)), L.jd_traj_bytes(C.byref(prob.st), C.byref(run))


def test_workspace_and_traj_sizes(L):
    p = wl.config("c2").problem
    pr = _Dummy(p)
    M = 1 << 20
    ws, tb = _sizes(L, pr, B.make_run(M, precision="fp32"))
    assert tb == p.N * 1 * M * 4
    assert ws >= p.N * (M // 256) * 8  # per-block FP64 partials of the adjoint
    _, tb64 = _sizes(L, pr, B.make_run(M, precision="fp64"))
    assert tb64 == 2 * tb
    _, tck = _sizes(L, pr, B.make_run(M, precision="fp32", mode="recompute", K=32))
    assert tck == (p.N // 32 + (p.N % 32 > 0)) * M * 4
    # d = 8, K = 64: the segment scratch of the recompute adjoint, one region of
    # K d 256 elements for each of min(blocks, 1024) resident blocks
    p8 = wl.config("c4").problem
    ws8, _ = _sizes(L, _Dummy(p8), B.make_run(1 << 18, precision="fp32", mode="recompute", K=64))
    ws8s, _ = _sizes(L, _Dummy(p8), B.make_run(1 << 18, precision="fp32", mode="store"))
    assert ws8 - ws8s >= 1024 * 64 * 8 * 256 * 4
    assert ws8 - ws8s < 1024 * 64 * 8 * 256 * 4 + (1 << 20)
    ws8d, _ = _sizes(L, _Dummy(p8), B.make_run(1 << 18, precision="fp64", mode="recompute", K=64))
    assert ws8d > 1024 * 64 * 8 * 256 * 8
    # blocks of 256 paths
    _, t7 = _sizes(L, pr, B.make_run(7, precision="fp32"))
    assert t7 == p.N * 256 * 4
    _, t257 = _sizes(L, pr, B.make_run(257, precision="fp32"))
    assert t257 == p.N * 512 * 4


def test_noise_table_workspace(L):
    """The noise table adds 2 N d ldm values of the run precision to the
    workspace; JD_NOISE_AUTO takes it for grids of at most 256 (FP64) or 64
    (FP32) blocks of 256 paths, and the trajectory buffer does not change."""
    p = wl.config("c1").problem
    pr = _Dummy(p)
    for prec, esz, nmax in (("fp32", 4, 64), ("fp64", 8, 256)):
        for M in (10_000, 257, 256 * nmax):
            ldm = (M + 255) // 256 * 256
            wi, ti = _sizes(L, pr, B.make_run(M, precision=prec, noise="inline"))
            wt, tt = _sizes(L, pr, B.make_run(M, precision=prec, noise="table"))
            wa, ta = _sizes(L, pr, B.make_run(M, precision=prec))
            tab = 2 * p.N * p.d * ldm * esz
            assert wt - wi == (tab + 255) // 256 * 256
            assert wa == wt  # at most 256 blocks: the table
            assert ti == tt == ta
        # one block more: draws in the sweeps unless asked for
        M = 256 * nmax + 1
        wi, _ = _sizes(L, pr, B.make_run(M, precision=prec, noise="inline"))
        wa, _ = _sizes(L, pr, B.make_run(M, precision=prec))
        wt, _ = _sizes(L, pr, B.make_run(M, precision=prec, noise="table"))
        assert wa == wi < wt
    # a table beyond 1 GiB is not taken by the automatic choice: d = 8,
    # 5000 steps, 2^16 paths in FP64 would need 2 * 5000 * 8 * 65536 * 8 bytes
    q = _Dummy(wl.general_problem(8, 5000, seed=2))
    wi, _ = _sizes(L, q, B.make_run(1 << 16, precision="fp64", noise="inline"))
    wa, _ = _sizes(L, q, B.make_run(1 << 16, precision="fp64"))
    assert wa == wi


@host_only
def test_invalid_arguments_rejected_before_launch(L):
    p = wl.general_problem(3, 20, seed=1)
    pr = _Dummy(p)
    run = B.make_run(1000)
    P = C.byref(pr.st)
    fake = C.c_void_p(0x2000)
    ws = 1 << 30
    # null pointers
    assert L.jd_forward(None, C.byref(run), fake, fake, fake, fake, ws, None) == B.JD_EINVAL
    assert L.jd_forward(P, None, fake, fake, fake, fake, ws, None) == B.JD_EINVAL
    assert L.jd_forward(P, C.byref(run), None, fake, fake, fake, ws, None) == B.JD_EINVAL
    assert L.jd_cost_grad(P, C.byref(run), fake, fake, fake, None, fake, ws, None) == B.JD_EINVAL
    assert L.jd_adjoint(P, C.byref(run), fake, None, fake, fake, ws, None) == B.JD_EINVAL
    # workspace too small
    assert L.jd_forward(P, C.byref(run), fake, fake, fake, fake, 100, None) == B.JD_EWORKSPACE
    assert L.jd_forward(P, C.byref(run), fake, fake, fake, None, ws, None) == B.JD_EINVAL

    def bad(**kw):
        q = _Dummy(wl.general_problem(3, 20, seed=1))
        for k, v in kw.items():
            setattr(q.st, k, v)
        return L.jd_forward(C.byref(q.st), C.byref(run), fake, fake, fake, fake, ws, None)

    assert bad(d=0) == B.JD_EINVAL
    assert bad(d=9) == B.JD_EINVAL
    assert bad(N=0) == B.JD_EINVAL
    assert bad(T=0.0) == B.JD_EINVAL
    assert bad(T=float("nan")) == B.JD_EINVAL
    assert bad(lambda_=-1.0) == B.JD_EINVAL
    assert bad(lambda_=41.0 * 20) == B.JD_EINVAL  # lambda*dt > 2
    assert bad(nu=-1.0) == B.JD_EINVAL
    assert bad(xd=None) == B.JD_EINVAL
    assert bad(A=None) == B.JD_EINVAL

    def badrun(**kw):
        r = B.make_run(1000)
        for k, v in kw.items():
            setattr(r, k, v)
        return L.jd_forward(P, C.byref(r), fake, fake, fake, fake, ws, None)

    assert badrun(M=0) == B.JD_EINVAL
    assert badrun(M=(1 << 31) + 1) == B.JD_EINVAL
    assert badrun(precision=2) == B.JD_EINVAL
    assert badrun(mode=3) == B.JD_EINVAL
    assert badrun(mode=B.JD_RECOMPUTE, K=0) == B.JD_EINVAL
    assert badrun(mode=B.JD_RECOMPUTE, K=21) == B.JD_EINVAL
    assert badrun(noise=3) == B.JD_EINVAL
    assert badrun(noise=-1) == B.JD_EINVAL
    # a checkpoint interval whose segment scratch would exceed 8 GiB (1024
    # regions of K d 256 elements) is refused, not mis-run
    q = _Dummy(wl.general_problem(8, 2000, seed=2))
    r = B.make_run(1 << 20, precision="fp32", mode="recompute", K=1100)
    assert L.jd_forward(C.byref(q.st), C.byref(r), fake, fake, fake, fake, ws, None) == B.JD_EUNSUPPORTED
    r = B.make_run(1 << 20, precision="fp32", mode="recompute", K=1000)
    assert L.jd_workspace_bytes(C.byref(q.st), C.byref(r)) > 0
    # dump range outside [0, M)
    dp = B.jd_dump(990, 20, None, None, None)
    r = B.make_run(1000, dump=dp)
    assert L.jd_forward(P, C.byref(r), fake, fake, fake, fake, ws, None) == B.JD_EINVAL
    # non-finite coefficient
    q = _Dummy(wl.general_problem(3, 20, seed=1))
    q._keep[1][0, 0] = np.inf
    assert L.jd_forward(C.byref(q.st), C.byref(run), fake, fake, fake, fake, ws, None) == B.JD_EINVAL


@host_only
def test_optimizer_options_validated(L):
    pr = _Dummy(wl.general_problem(2, 10, seed=3))
    run = B.make_run(500)
    fake = C.c_void_p(0x2000)
    P = C.byref(pr.st)
    for kw in (dict(n_max=-1), dict(max_backtracks=0), dict(zeta0=0.0), dict(rho=1.0),
               dict(rho=0.0), dict(c_armijo=0.0), dict(tol=-1.0)):
        o = B.jd_opt(5, 30, 0.0, 1.0, 0.5, 1e-4)
        for k, v in kw.items():
            setattr(o, k, v)
        assert L.jd_optimize(P, C.byref(run), C.byref(o), fake, None, None, fake, fake, 1 << 30,
                             None) == B.JD_EINVAL
    assert L.jd_optimize(P, C.byref(run), None, fake, None, None, fake, fake, 1 << 30,
                         None) == B.JD_EINVAL


@host_only
def test_draws_and_philox_argument_checks(L):
    pr = _Dummy(wl.general_problem(2, 10, seed=3))
    run = B.make_run(500)
    assert L.jd_draws(C.byref(pr.st), C.byref(run), -1, 1, 0, 1, None, None, None, None) == B.JD_EINVAL
    assert L.jd_draws(C.byref(pr.st), C.byref(run), 0, 0, 0, 1, None, None, None, None) == B.JD_OK
    assert L.jd_philox(1, None, 5, None, None) == B.JD_EINVAL
    assert L.jd_philox(1, None, 0, None, None) == B.JD_OK
    assert L.jd_poisson_thresholds(-1.0, None) == B.JD_EINVAL


@host_only
def test_server_arguments_checked_on_host(L):
    from paper_2505_04328_amd import serving as S
    Ls = S.lib()
    h = C.c_void_p()
    assert Ls.jd_server_create(None, 1 << 20, 4, 2, C.byref(h)) == B.JD_EINVAL
    assert Ls.jd_server_create(C.c_void_p(0x1000), 1 << 20, 0, 2, C.byref(h)) == B.JD_EINVAL
    assert Ls.jd_server_create(C.c_void_p(0x1000), 1 << 20, 4, 17, C.byref(h)) == B.JD_EINVAL
    assert Ls.jd_server_progress(None, None, None, None) == B.JD_EINVAL
    assert Ls.jd_server_result(None, 1, None, None, None, None) == B.JD_EINVAL
    assert Ls.jd_server_submit(None, None, None, None, None, None, None) == B.JD_EINVAL


def test_server_request_bytes(L):
    from paper_2505_04328_amd import serving as S
    p = wl.general_problem(3, 100, seed=2)
    nb = S.request_bytes(p, 1000)
    # control + target + trajectory (100 steps x 3 comps x 1024 columns FP32) + workspace
    assert nb >= 2 * 100 * 3 * 8 + 100 * 3 * 1024 * 4
    assert S.request_bytes(p, 1000, mode="recompute", K=10) < nb


# ---------------------------------------------------------------- feedback model
class _FbDummy:
    """A feedback problem whose z_d pointer is a fake non-null address."""

    def __init__(self, p):
        self.p = p
        self.st = B.jd_fb_problem(p.N, p.nx, p.nv, p.T, p.eta, p.b1, p.b2, p.gamma, p.beta,
                                  p.xmax, p.vmax, p.eps, p.alpha, p.sigJ, p.init_kind,
                                  (C.c_double * 2)(*p.z0), (C.c_double * 2)(*p.s0),
                                  (C.c_double * 2)(*p.svar0), (C.c_double * 2)(*p.svar1), 0x1000,
                                  p.np, p.omega, p.cost_kind, p.ax, p.av, p.grid, p.svar_kind)


def test_fb_workspace_and_traj_sizes(L):
    p = wl.feedback_config("f4").problem
    pr = _FbDummy(p)
    M = 1 << 20
    run = B.make_run(M, precision="fp32")
    tb = L.jd_fb_traj_bytes(C.byref(pr.st), C.byref(run))
    # z_0..z_N, then one jump-count byte per particle and step
    assert tb == (p.N + 1) * 2 * M * 4 + p.N * M
    ws = L.jd_fb_workspace_bytes(C.byref(pr.st), C.byref(run))
    assert ws >= (M // 256) * p.N * p.L * 8  # per-block FP64 gradient partials
    run7 = B.make_run(7, precision="fp64")
    assert L.jd_fb_traj_bytes(C.byref(pr.st), C.byref(run7)) == (p.N + 1) * 2 * 256 * 8 + p.N * 256
    rec = B.make_run(1000, precision="fp32", mode="recompute", K=10)
    assert L.jd_fb_traj_bytes(C.byref(pr.st), C.byref(rec)) == 0


def test_fb_surrogate_fit_workspace(L):
    """The fitted surrogate variance ignores svar0/svar1 and adds the per-step
    moment partials of the forward's blocks ((N+1) x blocks x 4 FP64)."""
    p = wl.feedback_config("f4").problem
    M = 1 << 20
    sur = B.make_run(M, precision="fp32", mode="surrogate")
    given = _FbDummy(p)
    fit = _FbDummy(p)
    fit.st.svar_kind = B.JD_FB_SVAR_FIT
    fit.st.svar0 = (C.c_double * 2)(-1.0, float("nan"))
    wg = L.jd_fb_workspace_bytes(C.byref(given.st), C.byref(sur))
    wf = L.jd_fb_workspace_bytes(C.byref(fit.st), C.byref(sur))
    assert wg > 0 and wf >= wg + (p.N + 1) * (M // 256) * 4 * 8
    given.st.svar0 = (C.c_double * 2)(-1.0, 0.0)
    assert L.jd_fb_workspace_bytes(C.byref(given.st), C.byref(sur)) == 0


def test_fb_adapted_traj_size(L):
    """The jump-adapted grid adds 32 post-jump states with their jump times
    and a count per slot, then a count byte per slot and interval."""
    p = wl.adapted_config("ja2").problem
    pr = _FbDummy(p)
    for prec, es in (("fp32", 4), ("fp64", 8)):
        run = B.make_run(1000, precision=prec)
        slots = 4 * 256
        want = (p.N + 1) * 2 * slots * es + 32 * 3 * slots * es + slots * 4 + p.N * slots
        assert L.jd_fb_traj_bytes(C.byref(pr.st), C.byref(run)) == want


@pytest.mark.parametrize("np_,M,rows", [
    (3, 100, 2),      # 85 rings of 3 per 256-slot workgroup: 2 workgroups
    (256, 5, 5),      # one full ring per workgroup
    (257, 7, 8),      # 8 groups of 256 slots hold 7 rings of 257
    (2000, 3, 24),    # one ring of 2000 per 2048-slot workgroup
    (2048, 2, 16),
])
def test_fb_ring_traj_sizes(L, np_, M, rows):
    """Rings: whole rings per workgroup, 256 slots per trajectory row."""
    p = wl.ring_problem(N=10, T=1.0, np_=np_)
    pr = _FbDummy(p)
    run = B.make_run(M, precision="fp32")
    assert L.jd_fb_traj_bytes(C.byref(pr.st), C.byref(run)) == ((p.N + 1) * 2 * rows * 256 * 4
                                                                + p.N * rows * 256)
    assert L.jd_fb_workspace_bytes(C.byref(pr.st), C.byref(run)) >= rows * p.N * p.L * 8 // (
        1 if np_ <= 256 else 8)
    # the ellipse cost needs no target outside the surrogate mode
    pr.st.zd = None
    assert L.jd_fb_workspace_bytes(C.byref(pr.st), C.byref(run)) > 0


@host_only
def test_fb_invalid_arguments_rejected_before_launch(L):
    run = B.make_run(1000)
    fake = C.c_void_p(0x2000)
    ws = 1 << 30

    def call(**kw):
        q = _FbDummy(wl.feedback_problem(N=20, T=2.0))
        for k, v in kw.items():
            setattr(q.st, k, v)
        return L.jd_fb_forward(C.byref(q.st), C.byref(run), fake, fake, fake, fake, ws, None)

    for kw in (dict(N=0), dict(nx=0), dict(nx=17), dict(nv=17), dict(T=0.0), dict(beta=0.0),
               dict(eps=-1.0), dict(sigJ=0.0), dict(gamma=1.5), dict(b1=-0.1), dict(alpha=-1.0),
               dict(init_kind=3), dict(zd=None), dict(xmax=0.0), dict(T=float("nan"))):
        assert call(**kw) == B.JD_EINVAL, kw
    # rate * dt > 2
    assert call(beta=1e4, N=2, T=2.0) == B.JD_EINVAL
    assert call(svar0=(C.c_double * 2)(-1.0, 0.0)) == B.JD_EINVAL
    assert call(svar1=(C.c_double * 2)(0.0, float("inf"))) == B.JD_EINVAL
    assert call(svar_kind=2) == B.JD_EINVAL
    pr = _FbDummy(wl.feedback_problem(N=20, T=2.0))
    P = C.byref(pr.st)
    assert L.jd_fb_forward(P, C.byref(run), None, fake, fake, fake, ws, None) == B.JD_EINVAL
    assert L.jd_fb_forward(P, C.byref(run), fake, fake, fake, fake, 100, None) == B.JD_EWORKSPACE
    assert L.jd_fb_cost_grad(P, C.byref(run), fake, fake, fake, None, fake, ws, None) == B.JD_EINVAL
    assert L.jd_fb_adjoint(P, C.byref(run), fake, None, fake, fake, ws, None) == B.JD_EINVAL
    rec = B.make_run(1000, mode="recompute", K=5)
    assert L.jd_fb_forward(P, C.byref(rec), fake, fake, fake, fake, ws, None) == B.JD_EUNSUPPORTED
    sur = B.make_run(1000, mode="surrogate")
    assert L.jd_fb_adjoint(P, C.byref(sur), fake, fake, fake, fake, ws, None) == B.JD_EUNSUPPORTED
    # the storage-free surrogate gradient takes no trajectory, the exact one needs it
    assert L.jd_fb_cost_grad(P, C.byref(sur), fake, fake, fake, None, fake, 100, None) == B.JD_EWORKSPACE
    assert L.jd_fb_cost_grad(P, C.byref(run), fake, fake, fake, None, fake, 100, None) == B.JD_EINVAL
    bad_opt = B.jd_opt(3, 0, 0.0, 1.0, 0.5, 1e-4)
    assert L.jd_fb_optimize(P, C.byref(run), C.byref(bad_opt), fake, None, None, fake, fake, ws,
                            None) == B.JD_EINVAL
    assert L.jd_fb_draws(P, C.byref(run), -1, 4, 0, 4, fake, fake, fake, None) == B.JD_EINVAL
    # the noise policy is checked; every valid value leaves the workspace as is
    bad_noise = B.make_run(1000)
    bad_noise.noise = 3
    assert L.jd_fb_forward(P, C.byref(bad_noise), fake, fake, fake, fake, ws, None) == B.JD_EINVAL
    sizes = {L.jd_fb_workspace_bytes(P, C.byref(B.make_run(1000, noise=n)))
             for n in ("auto", "inline", "table")}
    assert len(sizes) == 1 and 0 not in sizes
    # rings (Section 6.4)
    for kw in (dict(np=0), dict(np=B.JD_FB_MAX_RING + 1), dict(omega=float("nan")),
               dict(cost_kind=2), dict(cost_kind=1, ax=0.0), dict(init_kind=2, av=-1.0),
               dict(cost_kind=0, zd=None), dict(grid=2)):
        assert call(**kw) == B.JD_EINVAL, kw
    # the jump-adapted grid: independent particles, exact gradient only
    assert call(grid=1, np=3) == B.JD_EUNSUPPORTED
    ad = _FbDummy(wl.feedback_problem(N=20, T=2.0, grid="adapted"))
    assert L.jd_fb_cost_grad(C.byref(ad.st), C.byref(sur), fake, fake, fake, None, fake, ws,
                             None) == B.JD_EUNSUPPORTED
    ring = _FbDummy(wl.ring_problem(N=20, T=2.0, np_=5))
    R = C.byref(ring.st)
    assert L.jd_fb_cost_grad(R, C.byref(sur), fake, fake, fake, None, fake, ws, None) == B.JD_EUNSUPPORTED
    ring.st.zd = None
    assert L.jd_fb_workspace_bytes(R, C.byref(sur)) == 0
    big = B.make_run((1 << 31) // 5 + 1)
    assert L.jd_fb_workspace_bytes(R, C.byref(big)) == 0
    dump = B.jd_dump(0, 5 * 1000 + 1, None, None, None)
    dr = B.make_run(1000, dump=dump)
    assert L.jd_fb_forward(R, C.byref(dr), fake, fake, fake, fake, ws, None) == B.JD_EINVAL
    assert L.jd_fb_draws(P, C.byref(run), 0, 0, 0, 4, fake, fake, fake, None) == B.JD_OK
