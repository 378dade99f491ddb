"""Strength of the oracle's pins: plant one plausible mistake at a time in a copy
of the oracle source (on the CPU), build it, and run the pin suites against the
mutant.  Every mutant must make at least one pin fail; the unmodified source
must pass them all (the pin suites themselves run that case).

Not listed: the byte layout of the Poisson word, which Philox block feeds
the surrogate states of the feedback model, and which Box-Muller branch gives
the jump normal on the jump-adapted grid.  Which bits feed the count is a
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
# pin suites run against a mutant of each oracle source file
PIN_FILES = {
    "jd_oracle.c": ["tests/test_oracle_rng.py", "tests/test_oracle_model.py"],
    "fb_oracle.c": ["tests/test_oracle_fb.py", "tests/test_oracle_coupled.py",
                    "tests/test_oracle_adapted.py"],
}

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

# the paper's model problem (fb_oracle.c): name: (exact text, replacement)
FB_MUTANTS = {
    "fb_bump_exponent": ("return exp(-1.0 / (1.0 - q * q));", "return exp(-1.0 / (1.0 - q * q * q * q));"),
    "fb_bump_deriv_eps": ("(-2.0 * eps * eps * r) / (s * s)", "(-2.0 * eps * r) / (s * s)"),
    "fb_centre_offset": ("double r = z[0] - ((i + 0.5) * dx - pb->xmax);",
                         "double r = z[0] - ((i + 1.0) * dx - pb->xmax);"),
    "fb_velocity_centres_use_x": ("double r = z[1] - ((l + 0.5) * dv - pb->vmax);",
                                  "double r = z[1] - ((l + 0.5) * dx - pb->xmax);"),
    "fb_control_transposed": ("u += mu[i * pb->nv + l] * px[i] * pv[l];",
                              "u += mu[l * pb->nx + i] * px[i] * pv[l];"),
    "fb_position_without_dt": ("zn[0] = zk[0] + dt * zk[1] + pb->b1 * sq * Z[0];",
                               "zn[0] = zk[0] + zk[1] + pb->b1 * sq * Z[0];"),
    "fb_spring_sign": ("double vs = zk[1] + dt * (u - pb->eta * zk[0] -", "double vs = zk[1] + dt * (u + pb->eta * zk[0] -"),
    "fb_velocity_noise_is_x": ("+ pb->b2 * sq * Z[1];", "+ pb->b2 * sq * Z[0];"),
    "fb_jump_factor_once": ("zn[1] = gn * vs + sqrt(Vn) * Z[2];", "zn[1] = (w->n[k] ? pb->gamma : 1.0) * vs + sqrt(Vn) * Z[2];"),
    "fb_jump_variance": ("*Vn = s / (2.0 * pb->beta);", "*Vn = s / pb->beta;"),
    "fb_jump_rate": ("return sqrt(pb->beta / FB_PI) * (pb->T / (double)pb->N);",
                     "return sqrt(pb->beta * FB_PI) * (pb->T / (double)pb->N);"),
    "fb_initial_sine_to_x": ("z[1] = pb->z0[1] + pb->s0[1] * R * sin(FB_TWO_PI * ub);",
                             "z[1] = pb->z0[1] + pb->s0[1] * R * cos(FB_TWO_PI * ub);"),
    "fb_track_left_point": ("w->C[j] += dt * track(pb, zn, k + 1);", "w->C[j] += dt * track(pb, zk, k);"),
    "fb_control_cost_half": ("w->C[j] += dt * 0.5 * pb->alpha * u * u;", "w->C[j] += dt * pb->alpha * u * u;"),
    "fb_adjoint_terminal_without_dt": ("w->lam[2 * (N * np + j)] = dt * gz[0];", "w->lam[2 * (N * np + j)] = gz[0];"),
    "fb_adjoint_spring_sign": ("w->lam[2 * (k * np + j)] = lx + gn * dt * (ux - pb->eta) * lv",
                               "w->lam[2 * (k * np + j)] = lx + gn * dt * (ux + pb->eta) * lv"),
    "fb_adjoint_position_coupling": ("=\n                dt * lx + gn * (1.0 + dt * uv) * lv",
                                     "=\n                lx + gn * (1.0 + dt * uv) * lv"),
    "fb_adjoint_no_jump_factor": ("=\n                dt * lx + gn * (1.0 + dt * uv) * lv",
                                  "=\n                dt * lx + (1.0 + dt * uv) * lv"),
    "fb_adjoint_uv_dropped": ("=\n                dt * lx + gn * (1.0 + dt * uv) * lv", "=\n                dt * lx + gn * lv"),
    "fb_adjoint_track_sign": ("=\n                dt * lx + gn * (1.0 + dt * uv) * lv + dt * gz[1]",
                              "=\n                dt * lx + gn * (1.0 + dt * uv) * lv - dt * gz[1]"),
    "fb_adjoint_control_cost_dropped": ("+\n                                       dt * gz[0] + dt * pb->alpha * u * ux;",
                                        "+\n                                       dt * gz[0];"),
    "fb_gradient_no_jump_factor": ("double wk = pb->alpha * u + gn * lv;", "double wk = pb->alpha * u + lv;"),
    "fb_gradient_control_term_dropped": ("double wk = pb->alpha * u + gn * lv;", "double wk = gn * lv;"),
    "fb_track_grad_sign": ("gz[0] = rx / s2 * e;", "gz[0] = -rx / s2 * e;"),
    "fb_armijo_sign": ("if (Jt <= J - c_armijo * zeta * gg)", "if (Jt <= J + c_armijo * zeta * gg)"),
    "fb_surr_no_jump_factor": ("G[(size_t)k * L + i * pb->nv + l] += summand(w, w->px[i] * w->pv[l] * (gn * lv));",
                               "G[(size_t)k * L + i * pb->nv + l] += summand(w, w->px[i] * w->pv[l] * lv);"),
    "fb_surr_var_no_sqrt": ("z[0] = pb->zd[2 * k] + sqrt(vx) * R * cos(th);",
                            "z[0] = pb->zd[2 * k] + vx * R * cos(th);"),
    "fb_surr_var_no_clamp": ("return v > 0.0 ? v : 0.0;", "return v;"),
    "fb_fit_about_zero": ("double d = pass == 0 ? w.z[q] : w.z[q] - zbar[q];", "double d = w.z[q];"),
    "fb_fit_mean_not_divided": ("            zbar[q] /= (double)M;\n", ""),
    "fb_fit_sxx_uncentred": ("sxx += dtk * dtk;", "sxx += (double)k * dt * (double)k * dt;"),
    "fb_fit_intercept_sign": ("a[c] = vbar - b[c] * tbar;", "a[c] = vbar + b[c] * tbar;"),
    "fb_fit_components_swapped": ("vbar += V[2 * k + c];", "vbar += V[2 * k + 1 - c];"),
    "fb_fit_line_swapped": ("mu, NULL, fitted.svar0, fitted.svar1,", "mu, NULL, fitted.svar1, fitted.svar0,"),
    "fb_surr_fresh_sample_per_step": ("uint32_t ctr[4] = {m, FB_SURR_WORD, iter, 1u};",
                                      "uint32_t ctr[4] = {m, k, iter, 1u};"),
    "fb_surr_time_next_step": ("double t = (double)k * (pb->T / (double)pb->N);",
                               "double t = (double)(k + 1) * (pb->T / (double)pb->N);"),
    "fb_surr_track_sign": ("double nlv = dt * lx + gn * (1.0 + dt * uv) * lv + dt * gz[1]",
                           "double nlv = dt * lx + gn * (1.0 + dt * uv) * lv - dt * gz[1]"),
    "fb_surr_terminal_without_dt": ("double lx = dt * gz[0], lv = dt * gz[1];",
                                    "double lx = dt * gz[0], lv = gz[1];"),
    "fb_surr_forward_term_dropped": ("double au = pb->alpha * w.u[k];", "double au = 0.0 * w.u[k];"),
    # coupled particles (Section 6.4)
    "fb_coupling_sign": ("- pb->omega * (2.0 * zk[0] - xl - xr)", "+ pb->omega * (2.0 * zk[0] - xl - xr)"),
    "fb_coupling_one_neighbour": ("(2.0 * zk[0] - xl - xr)", "(2.0 * zk[0] - xl - xl)"),
    "fb_ring_not_closed": ("return (j + pb->np - 1) % pb->np;", "return j > 0 ? j - 1 : j;"),
    "fb_particle_counter_shared": ("fb_step_draws(seed, m * (uint32_t)np + (uint32_t)j,",
                                   "fb_step_draws(seed, m * (uint32_t)np,"),
    "fb_adjoint_coupling_sign": ("+ dt * pb->omega * cpl", "- dt * pb->omega * cpl"),
    "fb_adjoint_coupling_self": ("double cpl = w->w[left_of(pb, j)] + w->w[right_of(pb, j)] - 2.0 * w->w[j];",
                                 "double cpl = 2.0 * w->w[left_of(pb, j)] - 2.0 * w->w[j];"),
    "fb_adjoint_coupling_no_jump_factor": ("w->w[j] = gn * w->lam[2 * ((k + 1) * np + j) + 1];",
                                           "w->w[j] = w->lam[2 * ((k + 1) * np + j) + 1];"),
    "fb_mean_over_systems": ("const double P = (double)M * (double)pb->np;", "const double P = (double)M;"),
    "fb_ellipse_axes_swapped": ("z[0] * z[0] / (pb->ax * pb->ax) + z[1] * z[1] / (pb->av * pb->av) - 1.0",
                                "z[0] * z[0] / (pb->av * pb->av) + z[1] * z[1] / (pb->ax * pb->ax) - 1.0"),
    "fb_ellipse_q_not_squared": ("return -exp(-(q * q) / (2.0 * pb->sigJ * pb->sigJ));",
                                 "return -exp(-fabs(q) / (2.0 * pb->sigJ * pb->sigJ));"),
    "fb_ellipse_grad_factor": ("gz[0] = e * 2.0 * z[0] / (pb->ax * pb->ax);", "gz[0] = e * z[0] / (pb->ax * pb->ax);"),
    "fb_ellipse_grad_axis": ("gz[1] = e * 2.0 * z[1] / (pb->av * pb->av);", "gz[1] = e * 2.0 * z[1] / (pb->ax * pb->ax);"),
    "fb_ellipse_start_angle": ("(double)(m % (uint32_t)pb->np) / (double)pb->np;",
                               "(double)(m % (uint32_t)pb->np) / (double)(pb->np + 1);"),
    "fb_ellipse_start_axes": ("z[0] = pb->ax * cos(th)", "z[0] = pb->av * cos(th)"),
    "fb_tangent_coupling_neighbour": ("pb->omega * (2.0 * tx - txl - txr)", "pb->omega * (2.0 * tx - txl - txl)"),
    # jump-adapted grid (Section 3, Algorithms 5.1-5.2)
    "fb_adapted_offset_exponent": ("pow(V, 1.0 / (double)(*n - r + 1))", "pow(V, 1.0 / (double)(*n - r + 2))"),
    "fb_adapted_offset_not_ordered": ("a[r] = a[r - 1] + (1.0 - a[r - 1]) * (1.0 - pow(",
                                      "a[r] = a[r - 1] + (1.0 - a[r - 1]) * (0.5 - 0.5 * pow("),
    "fb_adapted_uniform_word": ("double V = or_uniform(W[(r - 1) % 4]);", "double V = or_uniform(W[0]);"),
    "fb_adapted_jump_scale": ("sb = 1.0 / sqrt(2.0 * pb->beta);", "sb = 1.0 / sqrt(pb->beta);"),
    "fb_adapted_jump_at_interval_end": ("            if (r < n)\n                vn = pb->gamma * vn + S[r + 1] * sb;",
                                        "            if (r > 0)\n                vn = pb->gamma * vn + S[r] * sb;"),
    "fb_adapted_substep_noise_dt": ("double xn = x + d * v + pb->b1 * sqrt(d) * Z[2 * r];",
                                    "double xn = x + d * v + pb->b1 * sqrt(dtau) * Z[2 * r];"),
    "fb_adapted_cost_weight": ("C += d * track_to(pb, ze, target_at(pb, k, a[r + 1], zt));",
                               "C += dtau * track_to(pb, ze, target_at(pb, k, a[r + 1], zt));"),
    "fb_adapted_target_reversed": ("buf[c] = (1.0 - a) * pb->zd[2 * k + c] + a * pb->zd[2 * (k + 1) + c];",
                                   "buf[c] = a * pb->zd[2 * k + c] + (1.0 - a) * pb->zd[2 * (k + 1) + c];"),
    "fb_adapted_adjoint_no_jump_factor": ("const double lxm = lx, lvm = r < n ? pb->gamma * lv : lv;",
                                          "const double lxm = lx, lvm = lv;"),
    "fb_adapted_adjoint_prev_weight": ("                dprev = w->sd[s - 1];", "                dprev = w->sd[s];"),
    "fb_adapted_adjoint_terminal_weight": ("double lx = dlast * gz[0], lv = dlast * gz[1];",
                                           "double lx = dtau * gz[0], lv = dtau * gz[1];"),
    "fb_adapted_gradient_weight": ("double wk = (d / dtau) * (pb->alpha * u + lvm);",
                                   "double wk = pb->alpha * u + lvm;"),
    "fb_adapted_tangent_jump": ("                nv *= pb->gamma;", "                nv *= 1.0;"),
    "fb_surr_control_cost_source_dropped": ("double nlx = lx + gn * dt * (ux - pb->eta) * lv + dt * gz[0] + dt * pb->alpha * u * ux;",
                                            "double nlx = lx + gn * dt * (ux - pb->eta) * lv + dt * gz[0];"),
}


ALL = [(n, "jd_oracle.c", old, new) for n, (old, new) in MUTANTS.items()] + \
      [(n, "fb_oracle.c", old, new) for n, (old, new) in FB_MUTANTS.items()]


def _run_mutant(case, tmpdir):
    name, target, old, new = case
    srcs = []
    for path in build.SRC:
        text = open(path).read()
        if os.path.basename(path) == target:
            assert text.count(old) == 1, f"mutant {name}: pattern must occur exactly once"
            text = text.replace(old, new)
        msrc = os.path.join(tmpdir, f"{name}__{os.path.basename(path)}")
        with open(msrc, "w") as f:
            f.write(text)
        srcs.append(msrc)
    lib = os.path.join(tmpdir, f"{name}.so")
    build.build(src=srcs, out=lib, extra=["-I" + os.path.dirname(build.SRC[0])])
    env = dict(os.environ, JD_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_FILES[target]], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    return name, r.returncode, r.stdout[-600:]


def test_every_mutant_is_caught(tmp_path):
    workers = max(1, min(8, (os.cpu_count() or 2)))
    with cfut.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda c: _run_mutant(c, str(tmp_path)), ALL))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, "mutants not caught by any pin: " + ", ".join(n for n, _ in survivors)
    for n, rc, out in results:
        assert rc == 1, f"mutant {n}: pytest ended abnormally (rc={rc}): {out}"
