"""Shared helpers of the GPU parity tests: tolerances and comparisons.

Tolerances (written here once, used by every parity test):
  per-path states and adjoints:  |x - x_ref| <= TOL_PATH * (|x_ref| + rms_k), with
      rms_k the root mean square of the reference over the checked paths and
      components at step k (so values that cross zero are not judged by a
      vanishing denominator);
  J:   |J - J_ref| / |J_ref| <= TOL_J;
  g:   both normwise, ||g - g_ref||_L2 / ||g_ref||_L2 <= TOL_G, and entry by
       entry, |g_q - g_ref_q| <= TOL_G * (|g_ref_q| + rms_k + s_q), with rms_k
       the root mean square of g_ref over the components of step k and s_q the
       mean over the paths of the absolute value of each path's summand of
       entry q (the oracle's gradient-scale diagnostic).  Every entry, a late
       step or a component with little signal included, is held to the size
       of its step and of what it is the mean of: rounding in the per-path
       arithmetic moves an entry in proportion to s_q, so an entry whose
       summands cancel (|g_q| << s_q) cannot be held to its own size, and in
       d = 1 an entry that changes sign has only itself as its step.
FP32 path arithmetic uses the stated target of the method's GPU form (1e-5 per
path, 1e-6 for J and g).  The FP64 GPU form differs from the FP64 oracle only by
operation order (fused multiply-adds, sincospi instead of cos(2 pi u)), so its
bound is rounding-level.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

TOL = {
    "fp32": dict(path=1e-5, J=1e-6, g=1e-6),
    "fp64": dict(path=1e-11, J=1e-12, g=1e-12),
}


def gpu_device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2505_04328_amd import binding
    binding.lib()  # raises if the HIP library is missing: no fallback
    return torch.device("cuda:0")


def per_path_error(x: np.ndarray, ref: np.ndarray) -> float:
    """x, ref: (paths, steps, d).  Returns max_k,p,c |x-ref| / (|ref| + rms_k)."""
    rms = np.sqrt(np.mean(ref * ref, axis=(0, 2)))  # per step
    den = np.abs(ref) + rms[None, :, None]
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(x - ref) / den))


def rel_err(x: float, ref: float) -> float:
    return abs(x - ref) / abs(ref)


def norm_err(g: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


def per_entry_error(g: np.ndarray, ref: np.ndarray, scale: np.ndarray) -> float:
    """max_q |g_q - ref_q| / (|ref_q| + rms_k + scale_q): rms_k the RMS of ref
    over the components of entry q's step (rows of ref), scale the oracle's
    mean absolute summand per entry (ref.grad_scale / ref.fb_grad_scale).  An
    entry whose denominator is zero must match exactly (its error counts as
    infinite otherwise)."""
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        ref = ref[:, None]
    g = np.asarray(g, dtype=np.float64).reshape(ref.shape)
    scale = np.asarray(scale, dtype=np.float64).reshape(ref.shape)
    rms = np.sqrt(np.mean(ref * ref, axis=1))
    den = np.abs(ref) + rms[:, None] + scale
    err = np.abs(g - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, err / np.where(den > 0, den, 1.0), np.where(err > 0, np.inf, 0.0))
    return float(np.max(r)) if r.size else 0.0


def grad_errors(g, ref, scale) -> tuple[float, float]:
    """(normwise, per-entry) errors of a gradient against its reference."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return norm_err(g.reshape(ref.shape), ref), per_entry_error(g, ref, scale)


def assert_grad(g, ref, scale, tol: float, what: str = "g",
                tol_entry: float | None = None) -> tuple[float, float]:
    """Asserts both gradient bounds (the per-entry one at tol_entry, default
    tol); returns the two errors."""
    en, ee = grad_errors(g, ref, scale)
    te = tol if tol_entry is None else tol_entry
    assert en <= tol, f"{what}: normwise error {en:.3e} > {tol:.1e}"
    assert ee <= te, f"{what}: per-entry error {ee:.3e} > {te:.1e}"
    return en, ee


def dump_to_paths(t, count: int) -> np.ndarray:
    """GPU dump layout (N, d, count) -> (count, N, d) float64 numpy."""
    a = t.double().cpu().numpy()
    return np.transpose(a, (2, 0, 1))


def golden(name: str) -> dict:
    """The full-size FP64 oracle record of a workload (tests/golden/make_full_size.py)."""
    with open(os.path.join(GOLD, f"full_{name}_it0.json")) as f:
        return json.loads("".join(ln for ln in f if not ln.startswith("#")))


def golden_g(name: str) -> tuple[np.ndarray, np.ndarray]:
    """The whole FP64 oracle gradient of a full-size workload and its
    per-entry summand scale (steps x components each)."""
    with np.load(os.path.join(GOLD, f"full_{name}_it0_g.npz"), allow_pickle=False) as z:
        return np.array(z["g"]), np.array(z["scale"])
