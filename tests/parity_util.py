"""Shared helpers of the GPU parity tests: tolerances and comparisons.

Tolerances (written here once, used by every parity test):
  per-path states and adjoints:  |x - x_ref| <= TOL_PATH * (|x_ref| + rms_k), with
      rms_k the root mean square of the reference over the checked paths and
      components at step k (so values that cross zero are not judged by a
      vanishing denominator);
  J:   |J - J_ref| / |J_ref| <= TOL_J;
  g:   ||g - g_ref||_L2 / ||g_ref||_L2 <= TOL_G (normwise over all N*d entries).
FP32 path arithmetic uses the stated target of the method's GPU form (1e-5 per
path, 1e-6 for J and g).  The FP64 GPU form differs from the FP64 oracle only by
operation order (fused multiply-adds, sincospi instead of cos(2 pi u)), so its
bound is rounding-level.
"""
from __future__ import annotations

import numpy as np
import pytest

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


def dump_to_paths(t, count: int) -> np.ndarray:
    """GPU dump layout (N, d, count) -> (count, N, d) float64 numpy."""
    a = t.double().cpu().numpy()
    return np.transpose(a, (2, 0, 1))
