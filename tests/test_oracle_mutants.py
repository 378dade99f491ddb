"""Strength of the oracle's pins: plant one plausible mistake at a time in a copy
of the oracle source (on the CPU), build it, and run the pin suites against the
mutant.  Every mutant must make at least one pin fail; the unmodified source
must pass them all (the pin suites themselves run that case).

Not listed: the byte layout of the Poisson word.  Which bits feed the count is a
convention, not a law: any layout using bits the uniforms do not read gives the
same distribution, so no pin of the law can see it.  It is fixed only by the
bit-exact agreement of the two independent implementations (oracle and GPU)."""
import concurrent.futures as cfut
import os
import subprocess
import sys

import pytest

from oracle import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_rng.py", "tests/test_oracle_model.py"]

# name: (exact text in jd_oracle.c, replacement)
MUTANTS = {
    "philox_multiplier": ("M0 = 0xD2511F53u", "M0 = 0xD2511F55u"),
    "philox_key_bump": ("k1 += W1;", "k1 += W0;"),
    "uniform_bits": ("(w >> 8) | 1u", "(w >> 9) | 1u"),
    "poisson_pmf_index": ("p = p * mu / (double)j;", "p = p * mu / (double)(j + 1);"),
    "jump_normal_is_brownian": ("zj[i] = R * sin(th);", "zj[i] = R * cos(th);"),
    "drift_without_dt": ("Xn[i] = Xk[i] + dt * f +", "Xn[i] = Xk[i] + f +"),
    "drift_A_transposed": ("f += pb->A[i * d + j] * Xk[j];", "f += pb->A[j * d + i] * Xk[j];"),
    "control_B_transposed": ("f += pb->B[i * d + j] * u[(size_t)k * d + j];",
                             "f += pb->B[j * d + i] * u[(size_t)k * d + j];"),
    "cubic_sign": ("f -= pb->cubic * Xk[i] * Xk[i] * Xk[i];", "f += pb->cubic * Xk[i] * Xk[i] * Xk[i];"),
    "noise_scale_dt": ("sqdt * pb->s[i] * zw[i]", "dt * pb->s[i] * zw[i]"),
    "jump_std_times_n": ("pb->jump_std[i] * sqrt((double)n) * zj[i]", "pb->jump_std[i] * (double)n * zj[i]"),
    "jump_mean_dropped": ("(double)n * pb->jump_mean[i] +", "0.0 * pb->jump_mean[i] +"),
    "running_cost_without_dt": ("C += 0.5 * dt * e;", "C += 0.5 * e;"),
    "terminal_cost_weight": ("    C += 0.5 * e;\n    return C;", "    C += e;\n    return C;"),
    "adjoint_A_not_transposed": ("a += pb->A[j * d + i] * ln[j];", "a += pb->A[i * d + j] * ln[j];"),
    "adjoint_cubic_factor": ("a -= 3.0 * pb->cubic * Xk[i] * Xk[i] * ln[i];",
                             "a -= pb->cubic * Xk[i] * Xk[i] * ln[i];"),
    "adjoint_without_dt": ("lam[(size_t)k * d + i] = ln[i] + dt * a;", "lam[(size_t)k * d + i] = ln[i] + a;"),
    "adjoint_source_sign": ("a += Xk[i] - pb->xd[(size_t)k * d + i];", "a -= Xk[i] - pb->xd[(size_t)k * d + i];"),
    "adjoint_source_index": ("a += Xk[i] - pb->xd[(size_t)k * d + i];",
                             "a += Xk[i] - pb->xd[(size_t)(k - 1) * d + i];"),
    "adjoint_terminal_sign": ("lam[(size_t)N * d + i] = X[(size_t)N * d + i] - pb->xT[i];",
                              "lam[(size_t)N * d + i] = pb->xT[i] - X[(size_t)N * d + i];"),
    "gradient_index_shift": ("const double* l1 = Ls + (size_t)(k + 1) * d;",
                             "const double* l1 = Ls + (size_t)(k + (k + 1 < N ? 2 : 1)) * d;"),
    "gradient_B_not_transposed": ("bl += pb->B[j * d + i] * l1[j];", "bl += pb->B[i * d + j] * l1[j];"),
    "gradient_without_control_term": ("g[q] = pb->nu * u[q] + t / (double)M;", "g[q] = t / (double)M;"),
    "cost_control_without_dt": ("0.5 * pb->nu * dt * uu", "0.5 * pb->nu * uu"),
    "armijo_sign": ("if (Jt <= J - opt->c_armijo * zeta * gg)", "if (Jt <= J + opt->c_armijo * zeta * gg)"),
    "descent_sign": ("ut[q] = u[q] - zeta * g[q];", "ut[q] = u[q] + zeta * g[q];"),
}


def _run_mutant(name, tmpdir):
    src = open(build.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutant {name}: pattern must occur exactly once"
    msrc = os.path.join(tmpdir, f"{name}.c")
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmpdir, f"{name}.so")
    build.build(src=msrc, out=lib, extra=["-I" + os.path.dirname(build.SRC)])
    env = dict(os.environ, JD_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_FILES], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_mutant_is_caught(tmp_path):
    workers = max(1, min(8, (os.cpu_count() or 2)))
    with cfut.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda n: _run_mutant(n, str(tmp_path)), MUTANTS))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, "mutants not caught by any pin: " + ", ".join(n for n, _ in survivors)
    for n, rc, out in results:
        assert rc == 1, f"mutant {n}: pytest ended abnormally (rc={rc}): {out}"
