/*
 * FP64 CPU oracle for the adjoint Monte Carlo method of Bartsch, Borzi,
 * Ciaramella and Reichle, "Adjoint-based optimal control of jump-diffusion
 * processes" (arXiv 2505.04328).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Plain, slow,
 * one path at a time, FP64 throughout, compiled with -ffp-contract=off and no
 * fast-math.  It shares no code with the GPU library.
 *
 * What is computed follows the paper's fully discrete problem (Section 3,
 * eq. model_approximation, discrete functional), its adjoint model (Section 4,
 * eq. AdjointModel), the reduced gradient (Section 4, eq. definition_Gradient)
 * and the gradient scheme with stochastic Armijo line search (Section 5,
 * Algorithms 5.3 and 5.4, eq. Stochastic_Armijo), specialised to the
 * fixed-grid, additive-jump, open-loop-control model of the header comment.
 * The random draws are a counter-based Philox4x32-10 stream (Salmon, Moraes,
 * Dror, Shaw, SC'11) so that the adjoint sweep sees the same increments and
 * jumps as the forward sweep, which the paper requires of the discretize-
 * before-optimize adjoint (Section 4, remark after the adjoint model).
 */
#include "jd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_CHUNK 4096
#define OR_TWO32 4294967296.0

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the published definition (SC'11, Section 5): each round
 * multiplies words 0 and 2 by fixed odd constants, splits the 64-bit products
 * into hi/lo halves and mixes them with words 1 and 3 and the round key; the
 * key is bumped by the Weyl increments between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform on [2^-24, 1-2^-24] from the top 24 bits of a word, lowest of them
 * forced to one: exact in FP32 and FP64, never 0 or 1. */
double or_uniform(uint32_t w)
{
    return (double)((w >> 8) | 1u) * (1.0 / 16777216.0);
}

void or_uniform_batch(const uint32_t* w, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_uniform(w[i]);
}

/* Inverse-CDF thresholds for a Poisson(mu) count against a 32-bit word:
 * p_0 = exp(-mu), p_j = (p_{j-1} * mu) / j, F_j = F_{j-1} + p_j,
 * thr_j = min(2^32, floor(2^32 F_j)) for j < 31, thr_31 = 2^32. */
void or_poisson_thresholds(double mu, uint64_t thr[32])
{
    double p = exp(-mu);
    double F = p;
    for (int j = 0; j < 31; ++j) {
        if (j > 0) {
            p = p * mu / (double)j;
            F = F + p;
        }
        double t = floor(ldexp(F, 32));
        thr[j] = (t >= OR_TWO32) ? (uint64_t)4294967296ull : (uint64_t)t;
    }
    thr[31] = (uint64_t)4294967296ull;
}

/* The count is the smallest j with P < thr_j. */
int or_poisson_count(uint32_t P, const uint64_t thr[32])
{
    int n = 0;
    while ((uint64_t)P >= thr[n])
        ++n;
    return n;
}

/* One path-step's draws.  Counter (m, k, iter, s) for Philox block s, key =
 * the two halves of the seed.  Component i takes words 2i and 2i+1 for a
 * Box-Muller pair: the cosine branch is the Brownian normal, the sine branch
 * the jump-size normal.  The Poisson word is built from the low bytes of the
 * four words of block 0 (bits the uniforms never read). */
void or_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, int d,
              const uint64_t thr[32], double* zw, double* zj, int* count)
{
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t W[16];
    int nblk = (d + 1) / 2;
    for (int s = 0; s < nblk; ++s) {
        uint32_t ctr[4] = {m, k, iter, (uint32_t)s};
        or_philox4x32_10(ctr, key, &W[4 * s]);
    }
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < d; ++i) {
        double ua = or_uniform(W[2 * i]);
        double ub = or_uniform(W[2 * i + 1]);
        double R = sqrt(-2.0 * log(ua));
        double th = two_pi * ub;
        zw[i] = R * cos(th);
        zj[i] = R * sin(th);
    }
    uint32_t P = (W[0] & 0xFFu) | ((W[1] & 0xFFu) << 8) | ((W[2] & 0xFFu) << 16) |
                 ((W[3] & 0xFFu) << 24);
    *count = or_poisson_count(P, thr);
}

void or_draws_grid(uint64_t seed, uint32_t iter, int d, double mu,
                   int64_t m0, int64_t mc, int32_t k0, int32_t kc,
                   double* zw, double* zj, int32_t* counts)
{
    uint64_t thr[32];
    or_poisson_thresholds(mu, thr);
    for (int64_t p = 0; p < mc; ++p) {
        for (int32_t q = 0; q < kc; ++q) {
            int n;
            size_t o = (size_t)(p * kc + q);
            or_draws(seed, (uint32_t)(m0 + p), (uint32_t)(k0 + q), iter, d, thr,
                     zw + o * d, zj + o * d, &n);
            counts[o] = n;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Forward Euler-Maruyama sweep of one path (Section 3, fully discrete problem;
 * Section 5, model equation) on the fixed grid t_k = k dt with a per-step
 * Poisson count of additive jumps.  Fills X[0..N][0..d) and returns the path
 * cost C^m: left-point running cost over k = 0..N-1 plus the terminal term. */
static double path_forward(const or_problem* pb, const uint64_t thr[32], uint64_t seed,
                           uint32_t iter, uint32_t m, const double* u, double* X)
{
    const int d = pb->d, N = pb->N;
    const double dt = pb->T / (double)N;
    const double sqdt = sqrt(dt);
    double zw[8], zj[8];
    for (int i = 0; i < d; ++i)
        X[i] = pb->x0[i];
    double C = 0.0;
    for (int k = 0; k < N; ++k) {
        const double* Xk = X + (size_t)k * d;
        double* Xn = X + (size_t)(k + 1) * d;
        double e = 0.0;
        for (int i = 0; i < d; ++i) {
            double r = Xk[i] - pb->xd[(size_t)k * d + i];
            e += r * r;
        }
        C += 0.5 * dt * e;
        int n;
        or_draws(seed, m, (uint32_t)k, iter, d, thr, zw, zj, &n);
        for (int i = 0; i < d; ++i) {
            double f = 0.0;
            for (int j = 0; j < d; ++j)
                f += pb->A[i * d + j] * Xk[j];
            f -= pb->cubic * Xk[i] * Xk[i] * Xk[i];
            for (int j = 0; j < d; ++j)
                f += pb->B[i * d + j] * u[(size_t)k * d + j];
            double jump = (double)n * pb->jump_mean[i] + pb->jump_std[i] * sqrt((double)n) * zj[i];
            Xn[i] = Xk[i] + dt * f + sqdt * pb->s[i] * zw[i] + jump;
        }
    }
    double e = 0.0;
    for (int i = 0; i < d; ++i) {
        double r = X[(size_t)N * d + i] - pb->xT[i];
        e += r * r;
    }
    C += 0.5 * e;
    return C;
}

/* Backward discrete adjoint of one path (Section 4, adjoint model, with the
 * dt factors of Section 5, adjoint equation).  The jump map is additive, so its
 * Jacobian is the identity and no jump condition acts on lam; the noise is
 * additive, so no noise term either.  Fills lam[k] for k = N..1. */
static void path_adjoint(const or_problem* pb, const double* X, double* lam)
{
    const int d = pb->d, N = pb->N;
    const double dt = pb->T / (double)N;
    for (int i = 0; i < d; ++i)
        lam[(size_t)N * d + i] = X[(size_t)N * d + i] - pb->xT[i];
    for (int k = N - 1; k >= 1; --k) {
        const double* ln = lam + (size_t)(k + 1) * d;
        const double* Xk = X + (size_t)k * d;
        for (int i = 0; i < d; ++i) {
            double a = 0.0;
            for (int j = 0; j < d; ++j)
                a += pb->A[j * d + i] * ln[j];
            a -= 3.0 * pb->cubic * Xk[i] * Xk[i] * ln[i];
            a += Xk[i] - pb->xd[(size_t)k * d + i];
            lam[(size_t)k * d + i] = ln[i] + dt * a;
        }
    }
    for (int i = 0; i < d; ++i)
        lam[i] = 0.0;
}

static int check_problem(const or_problem* pb)
{
    if (!pb || pb->d < 1 || pb->d > 8 || pb->N < 1 || !(pb->T > 0.0) || pb->lambda < 0.0)
        return -1;
    if (pb->lambda * (pb->T / (double)pb->N) > 2.0)
        return -1;
    return 0;
}

int or_paths(const or_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
             const double* u, double* X, double* lam, double* C, int nthreads)
{
    if (check_problem(pb) || m0 < 0 || count < 0)
        return -1;
    const int d = pb->d, N = pb->N;
    const size_t stride = (size_t)(N + 1) * d;
    uint64_t thr[32];
    or_poisson_thresholds(pb->lambda * (pb->T / (double)N), thr);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double* Xs = (double*)malloc(stride * sizeof(double));
        double* Ls = (double*)malloc(stride * sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < count; ++p) {
            double c = path_forward(pb, thr, seed, iter, (uint32_t)(m0 + p), u, Xs);
            if (C)
                C[p] = c;
            if (X)
                memcpy(X + (size_t)p * stride, Xs, stride * sizeof(double));
            if (lam) {
                path_adjoint(pb, Xs, Ls);
                memcpy(lam + (size_t)p * stride, Ls, stride * sizeof(double));
            }
        }
        free(Xs);
        free(Ls);
    }
    return 0;
}

/* Monte Carlo reduction (Section 3, discrete functional; Section 4, reduced
 * gradient).  Paths are summed in chunks of OR_CHUNK consecutive indices, each
 * chunk in index order, the chunks combined in index order, so the result does
 * not depend on the thread count. */
static int cost_grad_impl(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                          const double* u, double* J, double* g, int nthreads, int absval)
{
    if (check_problem(pb) || M < 1 || !u || !J)
        return -1;
    const int d = pb->d, N = pb->N;
    const double dt = pb->T / (double)N;
    const size_t stride = (size_t)(N + 1) * d;
    const size_t nd = (size_t)N * d;
    const int64_t nchunk = (M + OR_CHUNK - 1) / OR_CHUNK;
    uint64_t thr[32];
    or_poisson_thresholds(pb->lambda * dt, thr);
    double* csum = (double*)calloc((size_t)nchunk, sizeof(double));
    double* gsum = g ? (double*)calloc((size_t)nchunk * nd, sizeof(double)) : NULL;
    if (!csum || (g && !gsum)) {
        free(csum);
        free(gsum);
        return -2;
    }
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double* Xs = (double*)malloc(stride * sizeof(double));
        double* Ls = (double*)malloc(stride * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; ++c) {
            int64_t mb = c * OR_CHUNK, me = mb + OR_CHUNK < M ? mb + OR_CHUNK : M;
            double cs = 0.0;
            double* gs = g ? gsum + (size_t)c * nd : NULL;
            for (int64_t m = mb; m < me; ++m) {
                cs += path_forward(pb, thr, seed, iter, (uint32_t)m, u, Xs);
                if (gs) {
                    path_adjoint(pb, Xs, Ls);
                    for (int k = 0; k < N; ++k) {
                        const double* l1 = Ls + (size_t)(k + 1) * d;
                        for (int i = 0; i < d; ++i) {
                            double bl = 0.0;
                            for (int j = 0; j < d; ++j)
                                bl += pb->B[j * d + i] * l1[j];
                            gs[(size_t)k * d + i] += absval ? fabs(bl) : bl;
                        }
                    }
                }
            }
            csum[c] = cs;
        }
        free(Xs);
        free(Ls);
    }
    double ctot = 0.0;
    for (int64_t c = 0; c < nchunk; ++c)
        ctot += csum[c];
    double uu = 0.0;
    for (size_t q = 0; q < nd; ++q)
        uu += u[q] * u[q];
    *J = ctot / (double)M + 0.5 * pb->nu * dt * uu;
    if (g) {
        for (size_t q = 0; q < nd; ++q) {
            double t = 0.0;
            for (int64_t c = 0; c < nchunk; ++c)
                t += gsum[(size_t)c * nd + q];
            if (absval)
                g[q] = pb->nu * fabs(u[q]) + t / (double)M;
            else
                g[q] = pb->nu * u[q] + t / (double)M;
        }
    }
    free(csum);
    free(gsum);
    return 0;
}

int or_cost_grad(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                 const double* u, double* J, double* g, int nthreads)
{
    return cost_grad_impl(pb, M, seed, iter, u, J, g, nthreads, 0);
}

/* Test diagnostic, not part of the method: the size of what each gradient
 * entry is the mean of, s_q = nu |u_q| + (1/M) sum_m |(B^T lam^m_{k+1})_i|
 * (q = k d + i), from the same paths and the same loop as or_cost_grad.  An
 * entry whose summands cancel is small against s_q, and rounding in the
 * per-path arithmetic moves it in proportion to s_q, not to its own size. */
int or_grad_scale(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                  const double* u, double* s, int nthreads)
{
    double J;
    if (!s)
        return -1;
    return cost_grad_impl(pb, M, seed, iter, u, &J, s, nthreads, 1);
}

/* Forward-mode (tangent-linear) derivative of J along delta: differentiates the
 * Euler step and the cost directly, independently of the adjoint. */
int or_tangent(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
               const double* u, const double* delta, double* dJ, int nthreads)
{
    if (check_problem(pb) || M < 1 || !u || !delta || !dJ)
        return -1;
    const int d = pb->d, N = pb->N;
    const double dt = pb->T / (double)N;
    const size_t stride = (size_t)(N + 1) * d;
    const int64_t nchunk = (M + OR_CHUNK - 1) / OR_CHUNK;
    uint64_t thr[32];
    or_poisson_thresholds(pb->lambda * dt, thr);
    double* csum = (double*)calloc((size_t)nchunk, sizeof(double));
    if (!csum)
        return -2;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double* Xs = (double*)malloc(stride * sizeof(double));
        double* Ts = (double*)malloc(stride * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; ++c) {
            int64_t mb = c * OR_CHUNK, me = mb + OR_CHUNK < M ? mb + OR_CHUNK : M;
            double cs = 0.0;
            for (int64_t m = mb; m < me; ++m) {
                path_forward(pb, thr, seed, iter, (uint32_t)m, u, Xs);
                for (int i = 0; i < d; ++i)
                    Ts[i] = 0.0;
                double dc = 0.0;
                for (int k = 0; k < N; ++k) {
                    const double* Xk = Xs + (size_t)k * d;
                    const double* Tk = Ts + (size_t)k * d;
                    double* Tn = Ts + (size_t)(k + 1) * d;
                    for (int i = 0; i < d; ++i)
                        dc += dt * (Xk[i] - pb->xd[(size_t)k * d + i]) * Tk[i];
                    for (int i = 0; i < d; ++i) {
                        double f = 0.0;
                        for (int j = 0; j < d; ++j)
                            f += pb->A[i * d + j] * Tk[j];
                        f -= 3.0 * pb->cubic * Xk[i] * Xk[i] * Tk[i];
                        for (int j = 0; j < d; ++j)
                            f += pb->B[i * d + j] * delta[(size_t)k * d + j];
                        Tn[i] = Tk[i] + dt * f;
                    }
                }
                for (int i = 0; i < d; ++i)
                    dc += (Xs[(size_t)N * d + i] - pb->xT[i]) * Ts[(size_t)N * d + i];
                cs += dc;
            }
            csum[c] = cs;
        }
        free(Xs);
        free(Ts);
    }
    double tot = 0.0;
    for (int64_t c = 0; c < nchunk; ++c)
        tot += csum[c];
    double ud = 0.0;
    for (size_t q = 0; q < (size_t)N * d; ++q)
        ud += u[q] * delta[q];
    *dJ = tot / (double)M + pb->nu * dt * ud;
    free(csum);
    return 0;
}

/* Gradient descent with the stochastic Armijo rule (Section 5, optimization
 * procedure): iteration n draws with counter iter0+n; every line-search trial
 * of that iteration reuses the same counter (common random numbers).  The
 * step is along -g with the L2(0,T) norm ||v||^2 = dt sum_k |v_k|^2. */
int or_optimize(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter0,
                const or_opt* opt, double* u, double* logJ, double* log_gnorm,
                double* log_zeta, int32_t* log_bt, double* logE, int nthreads)
{
    if (check_problem(pb) || !opt || !u || opt->n_max < 0 || opt->max_backtracks < 1)
        return -1;
    const int d = pb->d, N = pb->N;
    const double dt = pb->T / (double)N;
    const size_t nd = (size_t)N * d;
    double* g = (double*)malloc(nd * sizeof(double));
    double* ut = (double*)malloc(nd * sizeof(double));
    if (!g || !ut) {
        free(g);
        free(ut);
        return -2;
    }
    int n;
    for (n = 0; n < opt->n_max; ++n) {
        uint32_t it = iter0 + (uint32_t)n;
        double J;
        if (or_cost_grad(pb, M, seed, it, u, &J, g, nthreads)) {
            n = -2;
            break;
        }
        double gg = 0.0;
        for (size_t q = 0; q < nd; ++q)
            gg += g[q] * g[q];
        gg *= dt;
        double zeta = opt->zeta0;
        int accepted = 0, bt;
        for (bt = 0; bt < opt->max_backtracks; ++bt) {
            for (size_t q = 0; q < nd; ++q)
                ut[q] = u[q] - zeta * g[q];
            double Jt;
            or_cost_grad(pb, M, seed, it, ut, &Jt, NULL, nthreads);
            if (Jt <= J - opt->c_armijo * zeta * gg) {
                accepted = 1;
                break;
            }
            zeta *= opt->rho;
        }
        if (!accepted) {
            n = -3;
            break;
        }
        double E = 0.0;
        for (size_t q = 0; q < nd; ++q) {
            double r = ut[q] - u[q];
            E += r * r;
            u[q] = ut[q];
        }
        E = sqrt(dt * E);
        if (logJ)
            logJ[n] = J;
        if (log_gnorm)
            log_gnorm[n] = sqrt(gg);
        if (log_zeta)
            log_zeta[n] = zeta;
        if (log_bt)
            log_bt[n] = bt;
        if (logE)
            logE[n] = E;
        if (E <= opt->tol) {
            ++n;
            break;
        }
    }
    free(g);
    free(ut);
    return n;
}
