"""Writes the full-size expected values used by tests/test_gpu_full_size.py.

Calls only the FP64 oracle (oracle/) and the seeded workload generators: for
the c2, c3 and c4 workloads at their full path counts, iteration word 0, seed 1
and u = 0, it records J, ||g||_L2, the L2 projections <g, delta_i> on 16 fixed
random directions (numpy default_rng(2), L2-normalised) and 64 sampled entries
of g into full_<name>_it0.json, and the whole gradient (N x d, FP64) with the
oracle's per-entry summand scale (ref.grad_scale) into full_<name>_it0_g.npz.  For the paper's model problem at its
measured size (f4: 2^20 particles, 500 steps) the same record is written at the
control mu = random_feedback_control(p, 4, 0.5) (whole gradient N x L), and so
for the coupled rings of Section 6.4 at their measured size (ring2: 512 rings
of 2000 particles, 500 steps) and the jump-adapted grid at f4's size (ja2).  Run from the repository
root:

    python tests/golden/make_full_size.py            # every workload (minutes on 8 cores)
    python tests/golden/make_full_size.py c3 f4      # some of them
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
from paper_2505_04328_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_index(p, count=64, seed=5):
    rng = np.random.default_rng(seed)
    return rng.integers(0, p.N * p.d, count)


def fb_directions(p, count=16, seed=2):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = rng.normal(size=(p.N, p.L))
        out.append(d / np.sqrt(p.dt * np.sum(d * d)))
    return out


def write(name, rec, g, scale):
    path = os.path.join(HERE, f"full_{name}_it0.json")
    with open(path, "w") as f:
        f.write("# FP64 oracle, written by tests/golden/make_full_size.py\n")
        json.dump(rec, f, indent=None)
        f.write("\n")
    np.savez_compressed(os.path.join(HERE, f"full_{name}_it0_g.npz"), g=np.asarray(g, np.float64),
                        scale=np.asarray(scale, np.float64))
    return path


def feedback(name):
    if name.startswith("ring"):
        w = wl.ring_config(name)
    elif name.startswith("ja"):
        w = wl.adapted_config(name)
    else:
        w = wl.feedback_config(name)
    p = w.problem
    t0 = time.time()
    mu = wl.random_feedback_control(p, 4, 0.5)
    J, g = ref.fb_cost_grad(p, w.M, w.seed, 0, mu)
    scale = ref.fb_grad_scale(p, w.M, w.seed, 0, mu)
    proj = [float(p.dt * np.sum(g * dl)) for dl in fb_directions(p)]
    idx = np.random.default_rng(5).integers(0, p.N * p.L, 64)
    rec = {
        "config": name, "M": w.M, "N": p.N, "L": p.L, "seed": w.seed, "iter": 0,
        "mu": "random_feedback_control(p, 4, 0.5)", "J": J,
        "gnorm_L2": float(np.sqrt(p.dt * np.sum(g * g))), "projections": proj,
        "sample_index": [int(i) for i in idx], "sample_g": [float(g.reshape(-1)[i]) for i in idx],
        "oracle_seconds": time.time() - t0,
    }
    path = write(name, rec, g, scale)
    print(f"{name}: J = {J:.15g}  ({time.time() - t0:.1f} s) -> {path}", flush=True)


def main(names):
    for name in names:
        if name.startswith(("f", "ring", "ja")):
            feedback(name)
            continue
        w = wl.config(name)
        p = w.problem
        t0 = time.time()
        J, g = ref.cost_grad(p, w.M, w.seed, 0, np.zeros((p.N, p.d)))
        scale = ref.grad_scale(p, w.M, w.seed, 0, np.zeros((p.N, p.d)))
        dirs = wl.fd_directions(p, 16, seed=2)
        proj = [float(p.dt * np.sum(g * dl)) for dl in dirs]
        idx = sample_index(p)
        rec = {
            "config": name, "M": w.M, "N": p.N, "d": p.d, "seed": w.seed, "iter": 0, "u": "zeros",
            "J": J, "gnorm_L2": float(np.sqrt(p.dt * np.sum(g * g))), "projections": proj,
            "sample_index": [int(i) for i in idx], "sample_g": [float(g.reshape(-1)[i]) for i in idx],
            "oracle_seconds": time.time() - t0,
        }
        path = write(name, rec, g, scale)
        print(f"{name}: J = {J:.15g}  ({time.time() - t0:.1f} s) -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3", "c4", "f4", "ring2", "ja2"])
