/*
 * FP64 CPU oracle for the paper's model problem (arXiv 2505.04328): the
 * controlled oscillator with Keilson-Storer velocity jumps and radial-basis
 * feedback control.  The definitions are in fb_oracle.h.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite and the benchmark's CPU
 * baseline, never by the product path.  Plain, one path at a time, FP64,
 * -ffp-contract=off.  It shares no code with the GPU library; it reuses this
 * directory's Philox, uniform map and Poisson thresholds (jd_oracle.c).
 *
 * Sources in the paper:
 *   control     eq. control_structure, shape functions as products of a
 *               position and a velocity bump (Section 5, shape functions,
 *               eq. Gaussian_RBF) on the cell centres of Section 5,
 *               discretization;
 *   dynamics    eq. coefficients and eq. SDE_splitted_drift_Euler (h = 0);
 *   jumps       eq. jump_law (v <- gamma v + N(0, 1/(2 beta))) at the rate
 *               of eq. collision_frequency;
 *   cost        eq. discrete_functional with the tracking cost of
 *               eq. tracking_cost;
 *   adjoint     eq. adjoint_eq_approximation with lam = -r and the jump
 *               condition p <- gamma p (Section 4, adjoint model);
 *   gradient    eq. definition_Gradient (Psi^T r = phi p);
 *   iteration   Algorithm 5.4 with eq. Stochastic_Armijo;
 *   coupling    eq. interacting_model on a ring, the ellipse cost of
 *               eq. phonon_functional_tracking and the start on the ellipse
 *               of eq. coupled_ellipse (Section 6.4);
 *   grid        the jump-adapted grid of Section 3 (uniform points and jump
 *               times) integrated as in Algorithms 5.1-5.2.
 */
#include "fb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "jd_oracle.h"

#define FB_CHUNK 4096
#define FB_INIT_STEP 0xFFFFFFFFu
#define FB_SURR_WORD 0xFFFFFFFEu
#define FB_SUB 32 /* sub-steps of a uniform interval on the jump-adapted grid: <= 31 jumps + 1 */

static const double FB_TWO_PI = 6.283185307179586476925286766559;
static const double FB_PI = 3.141592653589793238462643383280;

double fb_bump(double r, double eps)
{
    double q = eps * r;
    if (fabs(q) >= 1.0)
        return 0.0;
    return exp(-1.0 / (1.0 - q * q));
}

/* d/dr exp(-1/(1 - eps^2 r^2)) = b(r) * (-2 eps^2 r) / (1 - eps^2 r^2)^2. */
double fb_bump_deriv(double r, double eps)
{
    double q = eps * r;
    if (fabs(q) >= 1.0)
        return 0.0;
    double s = 1.0 - q * q;
    return exp(-1.0 / s) * (-2.0 * eps * eps * r) / (s * s);
}

static void key_of(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* Initial state from Philox block (m, 0xFFFFFFFF, iter, 0): a Box-Muller pair
 * of words 0 and 1 (cosine -> x, sine -> v) for the Gaussian law, or the two
 * uniforms for the box. */
void fb_initial(const fb_problem* pb, uint64_t seed, uint32_t m, uint32_t iter, double z[2])
{
    uint32_t key[2], W[4];
    uint32_t ctr[4] = {m, FB_INIT_STEP, iter, 0u};
    key_of(seed, key);
    or_philox4x32_10(ctr, key, W);
    double ua = or_uniform(W[0]), ub = or_uniform(W[1]);
    if (pb->init_kind == 0) {
        double R = sqrt(-2.0 * log(ua));
        z[0] = pb->z0[0] + pb->s0[0] * R * cos(FB_TWO_PI * ub);
        z[1] = pb->z0[1] + pb->s0[1] * R * sin(FB_TWO_PI * ub);
    } else if (pb->init_kind == 2) {
        /* particle j = m mod np of its ring, at parameter angle 2 pi j / np */
        double th = FB_TWO_PI * (double)(m % (uint32_t)pb->np) / (double)pb->np;
        double R = sqrt(-2.0 * log(ua));
        z[0] = pb->ax * cos(th) + pb->s0[0] * R * cos(FB_TWO_PI * ub);
        z[1] = pb->av * sin(th) + pb->s0[1] * R * sin(FB_TWO_PI * ub);
    } else {
        z[0] = pb->z0[0] + pb->s0[0] * (2.0 * ua - 1.0);
        z[1] = pb->z0[1] + pb->s0[1] * (2.0 * ub - 1.0);
    }
}

/* Step draws from Philox block (m, k, iter, 0): Box-Muller of words 0 and 1
 * gives the two Brownian normals (cosine -> x, sine -> v), the cosine branch
 * of words 2 and 3 the jump normal, the low bytes of the four words the
 * Poisson word. */
void fb_step_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, const uint64_t thr[32],
                   double Z[3], int* n)
{
    uint32_t key[2], W[4];
    uint32_t ctr[4] = {m, k, iter, 0u};
    key_of(seed, key);
    or_philox4x32_10(ctr, key, W);
    double R = sqrt(-2.0 * log(or_uniform(W[0])));
    double th = FB_TWO_PI * or_uniform(W[1]);
    Z[0] = R * cos(th);
    Z[1] = R * sin(th);
    double R2 = sqrt(-2.0 * log(or_uniform(W[2])));
    Z[2] = R2 * cos(FB_TWO_PI * or_uniform(W[3]));
    uint32_t P = (W[0] & 0xFFu) | ((W[1] & 0xFFu) << 8) | ((W[2] & 0xFFu) << 16) |
                 ((W[3] & 0xFFu) << 24);
    *n = or_poisson_count(P, thr);
}

/* Jump-adapted draws of interval k (see fb_oracle.h): the count and the
 * sub-step-0 normals of block (m, k, iter, 0); for jump r = 1..n the
 * Box-Muller pair of words 0, 1 of block (m, k, iter, r) (normals of sub-step
 * r) and the cosine branch of its words 2, 3 (the jump normal); the offsets as
 * successive minima of the n uniforms V_r. */
void fb_adapted_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, const uint64_t thr[32],
                      int* n, double* a, double* Z, double* S)
{
    uint32_t key[2], W[4];
    double Z3[3];
    key_of(seed, key);
    fb_step_draws(seed, m, k, iter, thr, Z3, n);
    Z[0] = Z3[0];
    Z[1] = Z3[1];
    a[0] = 0.0;
    for (int r = 1; r <= *n; ++r) {
        uint32_t c1[4] = {m, k, iter, (uint32_t)r};
        or_philox4x32_10(c1, key, W);
        double R = sqrt(-2.0 * log(or_uniform(W[0])));
        double th = FB_TWO_PI * or_uniform(W[1]);
        Z[2 * r] = R * cos(th);
        Z[2 * r + 1] = R * sin(th);
        double R2 = sqrt(-2.0 * log(or_uniform(W[2])));
        S[r] = R2 * cos(FB_TWO_PI * or_uniform(W[3]));
        uint32_t c2[4] = {m, k, iter, 64u + (uint32_t)((r - 1) / 4)};
        or_philox4x32_10(c2, key, W);
        double V = or_uniform(W[(r - 1) % 4]);
        /* the smallest of the n - r + 1 remaining uniforms on (a_{r-1}, 1) */
        a[r] = a[r - 1] + (1.0 - a[r - 1]) * (1.0 - pow(V, 1.0 / (double)(*n - r + 1)));
    }
    a[*n + 1] = 1.0;
}

/* Surrogate variance of component c at time t: the line svar0 + svar1 t, or 0
 * where the line is negative (a fitted line may start below zero). */
static double surr_var(const fb_problem* pb, int c, double t)
{
    double v = pb->svar0[c] + pb->svar1[c] * t;
    return v > 0.0 ? v : 0.0;
}

/* Surrogate state (Section 6.5: one position and velocity sampled for each
 * particle and realization): zd_k + sqrt(var(t_k)) (R cos, R sin) with the
 * Box-Muller pair of words 0 and 1 of block (m, 0xFFFFFFFE, iter, 1), the same
 * pair at every step k. */
void fb_surrogate_state(const fb_problem* pb, uint64_t seed, uint32_t m, uint32_t k, uint32_t iter,
                        double z[2])
{
    uint32_t key[2], W[4];
    uint32_t ctr[4] = {m, FB_SURR_WORD, iter, 1u};
    key_of(seed, key);
    or_philox4x32_10(ctr, key, W);
    double R = sqrt(-2.0 * log(or_uniform(W[0])));
    double th = FB_TWO_PI * or_uniform(W[1]);
    double t = (double)k * (pb->T / (double)pb->N);
    double vx = surr_var(pb, 0, t), vv = surr_var(pb, 1, t);
    z[0] = pb->zd[2 * k] + sqrt(vx) * R * cos(th);
    z[1] = pb->zd[2 * k + 1] + sqrt(vv) * R * sin(th);
}

static int check_problem(const fb_problem* pb)
{
    if (!pb || pb->N < 1 || pb->nx < 1 || pb->nv < 1 || pb->nx > 16 || pb->nv > 16 || pb->np < 1)
        return -1;
    if ((pb->grid != 0 && pb->grid != 1) || (pb->grid == 1 && pb->np != 1))
        return -1;
    if (!(pb->T > 0.0) || !(pb->beta > 0.0) || !(pb->eps > 0.0) || !(pb->sigJ > 0.0))
        return -1;
    if (pb->cost_kind != 0 && pb->cost_kind != 1)
        return -1;
    if ((pb->cost_kind == 0 && !pb->zd) || pb->init_kind < 0 || pb->init_kind > 2)
        return -1;
    if ((pb->cost_kind == 1 || pb->init_kind == 2) && !(pb->ax > 0.0 && pb->av > 0.0))
        return -1;
    if (!(pb->xmax > 0.0) || !(pb->vmax > 0.0) || pb->gamma < -1.0 || pb->gamma > 1.0)
        return -1;
    if (sqrt(pb->beta / FB_PI) * (pb->T / (double)pb->N) > 2.0)
        return -1;
    if (pb->svar_kind != 0 && pb->svar_kind != 1)
        return -1;
    for (int c = 0; c < 2; ++c)
        if (!isfinite(pb->svar0[c]) || !isfinite(pb->svar1[c]))
            return -1;
    return 0;
}

static double rate_dt(const fb_problem* pb)
{
    return sqrt(pb->beta / FB_PI) * (pb->T / (double)pb->N);
}

/* Shape-function values at z: px[i] = b(x - xc_i), pv[l] = b(v - vc_l) and,
 * if dpx/dpv are given, their derivatives. */
static void shapes(const fb_problem* pb, const double z[2], double* px, double* pv, double* dpx,
                   double* dpv)
{
    double dx = 2.0 * pb->xmax / (double)pb->nx, dv = 2.0 * pb->vmax / (double)pb->nv;
    for (int i = 0; i < pb->nx; ++i) {
        double r = z[0] - ((i + 0.5) * dx - pb->xmax);
        px[i] = fb_bump(r, pb->eps);
        if (dpx)
            dpx[i] = fb_bump_deriv(r, pb->eps);
    }
    for (int l = 0; l < pb->nv; ++l) {
        double r = z[1] - ((l + 0.5) * dv - pb->vmax);
        pv[l] = fb_bump(r, pb->eps);
        if (dpv)
            dpv[l] = fb_bump_deriv(r, pb->eps);
    }
}

/* u = sum_{i,l} mu[i nv + l] px[i] pv[l]. */
static double control(const fb_problem* pb, const double* mu, const double* px, const double* pv)
{
    double u = 0.0;
    for (int i = 0; i < pb->nx; ++i)
        for (int l = 0; l < pb->nv; ++l)
            u += mu[i * pb->nv + l] * px[i] * pv[l];
    return u;
}

/* Ellipse defect q = x^2/ax^2 + v^2/av^2 - 1 (zero on the ellipse). */
static double ellipse_q(const fb_problem* pb, const double z[2])
{
    return z[0] * z[0] / (pb->ax * pb->ax) + z[1] * z[1] / (pb->av * pb->av) - 1.0;
}

/* Running cost against the target zd (ignored by the ellipse cost): the
 * tracking cost -exp(-|z - zd|^2/(2 sigJ^2)), or the ellipse cost
 * -exp(-q^2/(2 sigJ^2)). */
static double track_to(const fb_problem* pb, const double z[2], const double* zd)
{
    if (pb->cost_kind == 1) {
        double q = ellipse_q(pb, z);
        return -exp(-(q * q) / (2.0 * pb->sigJ * pb->sigJ));
    }
    double rx = z[0] - zd[0], rv = z[1] - zd[1];
    return -exp(-(rx * rx + rv * rv) / (2.0 * pb->sigJ * pb->sigJ));
}

/* Its gradient: (z - zd)/sigJ^2 * exp(-|z - zd|^2/(2 sigJ^2)), or
 * q/sigJ^2 * exp(-q^2/(2 sigJ^2)) * (2x/ax^2, 2v/av^2). */
static void track_grad_to(const fb_problem* pb, const double z[2], const double* zd, double gz[2])
{
    double s2 = pb->sigJ * pb->sigJ;
    if (pb->cost_kind == 1) {
        double q = ellipse_q(pb, z);
        double e = q / s2 * exp(-(q * q) / (2.0 * s2));
        gz[0] = e * 2.0 * z[0] / (pb->ax * pb->ax);
        gz[1] = e * 2.0 * z[1] / (pb->av * pb->av);
        return;
    }
    double rx = z[0] - zd[0], rv = z[1] - zd[1];
    double e = exp(-(rx * rx + rv * rv) / (2.0 * s2));
    gz[0] = rx / s2 * e;
    gz[1] = rv / s2 * e;
}

/* The target at uniform point k (none for the ellipse cost). */
static const double* target(const fb_problem* pb, int k)
{
    return pb->cost_kind == 1 ? NULL : pb->zd + 2 * k;
}

static double track(const fb_problem* pb, const double z[2], int k)
{
    return track_to(pb, z, target(pb, k));
}

static void track_grad(const fb_problem* pb, const double z[2], int k, double gz[2])
{
    track_grad_to(pb, z, target(pb, k), gz);
}

/* The target at fraction a in (0, 1] of uniform interval k: linear between the
 * uniform targets, zd_{k+1} itself at a = 1. */
static const double* target_at(const fb_problem* pb, int k, double a, double buf[2])
{
    if (pb->cost_kind == 1)
        return NULL;
    if (a == 1.0)
        return pb->zd + 2 * (k + 1);
    for (int c = 0; c < 2; ++c)
        buf[c] = (1.0 - a) * pb->zd[2 * k + c] + a * pb->zd[2 * (k + 1) + c];
    return buf;
}

/* gamma^n and V_n = (1/(2 beta)) sum_{i<n} gamma^{2i}: n Keilson-Storer jumps
 * v <- gamma v + s_i composed (a Gaussian with that variance). */
static void ks_factors(const fb_problem* pb, int n, double* gn, double* Vn)
{
    double g = 1.0, s = 0.0;
    for (int i = 0; i < n; ++i) {
        s += g * g;
        g *= pb->gamma;
    }
    *gn = g;
    *Vn = s / (2.0 * pb->beta);
}

/* Work arrays of one system of np particles; z and lam are indexed
 * [(k np + j) 2 + c], u and n [k np + j]. */
typedef struct {
    double *z, *u, *px, *pv, *dpx, *dpv, *lam, *C, *w;
    int *n;
    /* jump-adapted grid, per interval k and sub-step r (index k FB_SUB + r):
     * start states sz (x, v), controls su, lengths sd, start offsets sa */
    double *sz, *su, *sd, *sa;
    int absval; /* gradient-scale diagnostic: accumulate |summand| */
} work;

/* A particle's gradient summand as accumulated: itself, or its absolute value
 * for the gradient-scale diagnostic. */
static double summand(const work* w, double v) { return w->absval ? fabs(v) : v; }

static int work_alloc(const fb_problem* pb, work* w)
{
    size_t N = (size_t)pb->N, np = (size_t)pb->np;
    w->z = (double*)malloc((N + 1) * np * 2 * sizeof(double));
    w->lam = (double*)malloc((N + 1) * np * 2 * sizeof(double));
    w->u = (double*)malloc(N * np * sizeof(double));
    w->n = (int*)malloc(N * np * sizeof(int));
    w->C = (double*)malloc(np * sizeof(double));
    w->w = (double*)malloc(np * sizeof(double));
    w->px = (double*)malloc(16 * sizeof(double));
    w->pv = (double*)malloc(16 * sizeof(double));
    w->dpx = (double*)malloc(16 * sizeof(double));
    w->dpv = (double*)malloc(16 * sizeof(double));
    const size_t ns = pb->grid == 1 ? N * FB_SUB : 1;
    w->sz = (double*)malloc(ns * 2 * sizeof(double));
    w->su = (double*)malloc(ns * sizeof(double));
    w->sd = (double*)malloc(ns * sizeof(double));
    w->sa = (double*)malloc(ns * sizeof(double));
    w->absval = 0;
    return (w->z && w->lam && w->u && w->n && w->C && w->w && w->px && w->pv && w->dpx && w->dpv &&
            w->sz && w->su && w->sd && w->sa)
               ? 0
               : -2;
}

static void work_free(work* w)
{
    free(w->z);
    free(w->lam);
    free(w->u);
    free(w->n);
    free(w->C);
    free(w->w);
    free(w->px);
    free(w->pv);
    free(w->dpx);
    free(w->dpv);
    free(w->sz);
    free(w->su);
    free(w->sd);
    free(w->sa);
}

/* Ring neighbours of particle j. */
static int left_of(const fb_problem* pb, int j) { return (j + pb->np - 1) % pb->np; }
static int right_of(const fb_problem* pb, int j) { return (j + 1) % pb->np; }

/* Forward sweep of system m (eq. SDE_splitted_drift_Euler on the fixed grid,
 * with the nearest-neighbour force of eq. interacting_model; the step's n
 * jumps applied after its Euler update): fills w->z, w->u, w->n and the
 * particle costs w->C, and returns their sum. */
static double path_forward_fixed(const fb_problem* pb, const uint64_t thr[32], uint64_t seed,
                                 uint32_t iter, uint32_t m, const double* mu, work* w)
{
    const int N = pb->N, L = pb->nx * pb->nv, np = pb->np;
    const double dt = pb->T / (double)N, sq = sqrt(dt);
    for (int j = 0; j < np; ++j) {
        fb_initial(pb, seed, m * (uint32_t)np + (uint32_t)j, iter, w->z + 2 * j);
        w->C[j] = 0.0;
    }
    for (int k = 0; k < N; ++k) {
        for (int j = 0; j < np; ++j) {
            const double* zk = w->z + 2 * (k * np + j);
            double* zn = w->z + 2 * ((k + 1) * np + j);
            const double xl = w->z[2 * (k * np + left_of(pb, j))];
            const double xr = w->z[2 * (k * np + right_of(pb, j))];
            shapes(pb, zk, w->px, w->pv, NULL, NULL);
            double u = control(pb, mu + (size_t)k * L, w->px, w->pv);
            w->u[k * np + j] = u;
            w->C[j] += dt * 0.5 * pb->alpha * u * u;
            double Z[3];
            int n;
            fb_step_draws(seed, m * (uint32_t)np + (uint32_t)j, (uint32_t)k, iter, thr, Z, &n);
            w->n[k * np + j] = n;
            double gn, Vn;
            ks_factors(pb, n, &gn, &Vn);
            zn[0] = zk[0] + dt * zk[1] + pb->b1 * sq * Z[0];
            double vs = zk[1] + dt * (u - pb->eta * zk[0] - pb->omega * (2.0 * zk[0] - xl - xr))
                        + pb->b2 * sq * Z[1];
            zn[1] = gn * vs + sqrt(Vn) * Z[2];
            w->C[j] += dt * track(pb, zn, k + 1);
        }
    }
    double C = 0.0;
    for (int j = 0; j < np; ++j)
        C += w->C[j];
    return C;
}

/* Backward adjoint of the system held in w (eq. adjoint_eq_approximation,
 * lam_j = dC/dz_j for C the sum of the particle costs, lam = -r): fills
 * w->lam for k = N..1 and, if G is given, adds each particle's gradient
 * summand phi(z_k) (alpha u_k + gamma^{n_k} lam^v_{k+1}) to G[k*L + l]. */
static void path_adjoint_fixed(const fb_problem* pb, const double* mu, work* w, double* G)
{
    const int N = pb->N, L = pb->nx * pb->nv, np = pb->np;
    const double dt = pb->T / (double)N;
    double gz[2];
    for (int j = 0; j < np; ++j) {
        track_grad(pb, w->z + 2 * (N * np + j), N, gz);
        w->lam[2 * (N * np + j)] = dt * gz[0];
        w->lam[2 * (N * np + j) + 1] = dt * gz[1];
    }
    for (int k = N - 1; k >= 0; --k) {
        const double* mk = mu + (size_t)k * L;
        /* w_j = gamma^{n_j} lam^v_{j,k+1}: what the velocity update passes back */
        for (int j = 0; j < np; ++j) {
            double gn, Vn;
            ks_factors(pb, w->n[k * np + j], &gn, &Vn);
            w->w[j] = gn * w->lam[2 * ((k + 1) * np + j) + 1];
        }
        for (int j = 0; j < np; ++j) {
            const double* zk = w->z + 2 * (k * np + j);
            const double lx = w->lam[2 * ((k + 1) * np + j)], lv = w->lam[2 * ((k + 1) * np + j) + 1];
            shapes(pb, zk, w->px, w->pv, w->dpx, w->dpv);
            double u = w->u[k * np + j];
            double gn, Vn;
            ks_factors(pb, w->n[k * np + j], &gn, &Vn);
            if (G) {
                double wk = pb->alpha * u + gn * lv;
                for (int i = 0; i < pb->nx; ++i)
                    for (int l = 0; l < pb->nv; ++l)
                        G[(size_t)k * L + i * pb->nv + l] += summand(w, w->px[i] * w->pv[l] * wk);
            }
            if (k == 0)
                continue;
            double ux = control(pb, mk, w->dpx, w->pv);
            double uv = control(pb, mk, w->px, w->dpv);
            double cpl = w->w[left_of(pb, j)] + w->w[right_of(pb, j)] - 2.0 * w->w[j];
            track_grad(pb, zk, k, gz);
            w->lam[2 * (k * np + j)] = lx + gn * dt * (ux - pb->eta) * lv + dt * pb->omega * cpl +
                                       dt * gz[0] + dt * pb->alpha * u * ux;
            w->lam[2 * (k * np + j) + 1] =
                dt * lx + gn * (1.0 + dt * uv) * lv + dt * gz[1] + dt * pb->alpha * u * uv;
        }
    }
    for (int j = 0; j < np; ++j) {
        w->lam[2 * j] = 0.0;
        w->lam[2 * j + 1] = 0.0;
    }
}

/* Forward sweep of particle m on the jump-adapted grid (Algorithms 5.1-5.2):
 * in each uniform interval, Euler sub-steps up to each jump time, the jump
 * v <- gamma v + S/sqrt(2 beta) there, and on to the interval's end; the
 * running cost on every sub-step.  Fills w->z, w->u (at the uniform points),
 * w->n, the sub-step arrays and w->C[0]; returns the cost. */
static double path_forward_adapted(const fb_problem* pb, const uint64_t thr[32], uint64_t seed,
                                   uint32_t iter, uint32_t m, const double* mu, work* w)
{
    const int N = pb->N, L = pb->nx * pb->nv;
    const double dtau = pb->T / (double)N, sb = 1.0 / sqrt(2.0 * pb->beta);
    double a[FB_SUB + 1], Z[2 * FB_SUB], S[FB_SUB], zt[2];
    fb_initial(pb, seed, m, iter, w->z);
    double C = 0.0;
    for (int k = 0; k < N; ++k) {
        int n;
        fb_adapted_draws(seed, m, (uint32_t)k, iter, thr, &n, a, Z, S);
        w->n[k] = n;
        double x = w->z[2 * k], v = w->z[2 * k + 1];
        for (int r = 0; r <= n; ++r) {
            const int s = k * FB_SUB + r;
            const double d = (a[r + 1] - a[r]) * dtau;
            const double zs[2] = {x, v};
            w->sz[2 * s] = x;
            w->sz[2 * s + 1] = v;
            w->sd[s] = d;
            w->sa[s] = a[r];
            shapes(pb, zs, w->px, w->pv, NULL, NULL);
            double u = control(pb, mu + (size_t)k * L, w->px, w->pv);
            w->su[s] = u;
            if (r == 0)
                w->u[k] = u;
            C += d * 0.5 * pb->alpha * u * u;
            double xn = x + d * v + pb->b1 * sqrt(d) * Z[2 * r];
            double vn = v + d * (u - pb->eta * x) + pb->b2 * sqrt(d) * Z[2 * r + 1];
            if (r < n)
                vn = pb->gamma * vn + S[r + 1] * sb;
            x = xn;
            v = vn;
            const double ze[2] = {x, v};
            C += d * track_to(pb, ze, target_at(pb, k, a[r + 1], zt));
        }
        w->z[2 * (k + 1)] = x;
        w->z[2 * (k + 1) + 1] = v;
    }
    w->C[0] = C;
    return C;
}

/* The exact adjoint of path_forward_adapted, sub-step by sub-step backwards:
 * at the end of sub-step r the adjoint of the pre-jump state is
 * (lam^x, gamma lam^v) if a jump ends it, and the start state z_r receives the
 * Euler transpose, its control cost and the running cost of the sub-step that
 * ends at it.  Adds d_r/dtau phi(z_r) (alpha u_r + lam^v_-) to G[k L + l]. */
static void path_adjoint_adapted(const fb_problem* pb, const double* mu, work* w, double* G)
{
    const int N = pb->N, L = pb->nx * pb->nv;
    const double dtau = pb->T / (double)N;
    double gz[2], zt[2];
    const double dlast = w->sd[(N - 1) * FB_SUB + w->n[N - 1]];
    track_grad(pb, w->z + 2 * N, N, gz);
    double lx = dlast * gz[0], lv = dlast * gz[1];
    w->lam[2 * N] = lx;
    w->lam[2 * N + 1] = lv;
    for (int k = N - 1; k >= 0; --k) {
        const double* mk = mu + (size_t)k * L;
        const int n = w->n[k];
        for (int r = n; r >= 0; --r) {
            const int s = k * FB_SUB + r;
            const double* zs = w->sz + 2 * s;
            const double d = w->sd[s], u = w->su[s];
            const double lxm = lx, lvm = r < n ? pb->gamma * lv : lv;
            shapes(pb, zs, w->px, w->pv, w->dpx, w->dpv);
            if (G) {
                double wk = (d / dtau) * (pb->alpha * u + lvm);
                for (int i = 0; i < pb->nx; ++i)
                    for (int l = 0; l < pb->nv; ++l)
                        G[(size_t)k * L + i * pb->nv + l] += summand(w, w->px[i] * w->pv[l] * wk);
            }
            if (k == 0 && r == 0)
                break;
            /* the sub-step ending at z_r: r - 1 of this interval, or the last of k - 1 */
            double dprev;
            const double* tz;
            if (r > 0) {
                dprev = w->sd[s - 1];
                tz = target_at(pb, k, w->sa[s], zt);
            } else {
                dprev = w->sd[(k - 1) * FB_SUB + w->n[k - 1]];
                tz = target(pb, k);
            }
            double ux = control(pb, mk, w->dpx, w->pv);
            double uv = control(pb, mk, w->px, w->dpv);
            track_grad_to(pb, zs, tz, gz);
            lx = lxm + d * (ux - pb->eta) * lvm + dprev * gz[0] + d * pb->alpha * u * ux;
            lv = d * lxm + (1.0 + d * uv) * lvm + dprev * gz[1] + d * pb->alpha * u * uv;
        }
        if (k >= 1) {
            w->lam[2 * k] = lx;
            w->lam[2 * k + 1] = lv;
        }
    }
    w->lam[0] = 0.0;
    w->lam[1] = 0.0;
}

static double path_forward(const fb_problem* pb, const uint64_t thr[32], uint64_t seed,
                           uint32_t iter, uint32_t m, const double* mu, work* w)
{
    return pb->grid == 1 ? path_forward_adapted(pb, thr, seed, iter, m, mu, w)
                         : path_forward_fixed(pb, thr, seed, iter, m, mu, w);
}

static void path_adjoint(const fb_problem* pb, const double* mu, work* w, double* G)
{
    if (pb->grid == 1)
        path_adjoint_adapted(pb, mu, w, G);
    else
        path_adjoint_fixed(pb, mu, w, G);
}

/* Copies the system's per-particle rows into particle-major outputs. */
static void copy_rows(const fb_problem* pb, const work* w, int64_t p0, double* z, double* lam,
                      double* u, int32_t* jumps, double* C)
{
    const int N = pb->N, np = pb->np;
    for (int j = 0; j < np; ++j) {
        const size_t p = (size_t)p0 + (size_t)j;
        for (int k = 0; k <= N; ++k)
            for (int c = 0; c < 2; ++c) {
                if (z)
                    z[(p * (N + 1) + k) * 2 + c] = w->z[2 * (k * np + j) + c];
                if (lam)
                    lam[(p * (N + 1) + k) * 2 + c] = w->lam[2 * (k * np + j) + c];
            }
        for (int k = 0; k < N; ++k) {
            if (u)
                u[p * N + k] = w->u[k * np + j];
            if (jumps)
                jumps[p * N + k] = w->n[k * np + j];
        }
        if (C)
            C[p] = w->C[j];
    }
}

int fb_paths(const fb_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
             const double* mu, double* z, double* lam, double* u, int32_t* jumps, double* C,
             int nthreads)
{
    if (check_problem(pb) || !mu || m0 < 0 || count < 0)
        return -1;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : rc)
    {
        work w;
        const int ok = work_alloc(pb, &w) == 0;
        rc |= ok ? 0 : 1;
        {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < count; ++p) {
                if (!ok)
                    continue;
                path_forward(pb, thr, seed, iter, (uint32_t)(m0 + p), mu, &w);
                if (lam)
                    path_adjoint(pb, mu, &w, NULL);
                copy_rows(pb, &w, p * pb->np, z, lam, u, jumps, C);
            }
        }
        work_free(&w);
    }
    return rc ? -2 : 0;
}

/* Systems per reduction chunk: FB_CHUNK particles' worth, at least one. */
static int64_t chunk_systems(const fb_problem* pb)
{
    return pb->np >= FB_CHUNK ? 1 : FB_CHUNK / pb->np;
}

/* Monte Carlo reductions in chunks of consecutive systems, each chunk in
 * system order and the chunks in index order (thread-count independent);
 * the means are over the M np particles. */
static int cost_grad_impl(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                          const double* mu, double* J, double* g, int nthreads, int absval)
{
    if (check_problem(pb) || M < 1 || !mu || !J)
        return -1;
    const int N = pb->N, L = pb->nx * pb->nv;
    const size_t nl = (size_t)N * L;
    const int64_t cs_sys = chunk_systems(pb);
    const int64_t nchunk = (M + cs_sys - 1) / cs_sys;
    const double P = (double)M * (double)pb->np;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    double* csum = (double*)calloc((size_t)nchunk, sizeof(double));
    double* gsum = g ? (double*)calloc((size_t)nchunk * nl, sizeof(double)) : NULL;
    if (!csum || (g && !gsum)) {
        free(csum);
        free(gsum);
        return -2;
    }
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : rc)
    {
        work w;
        const int ok = work_alloc(pb, &w) == 0;
        rc |= ok ? 0 : 1;
        w.absval = absval;
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < nchunk; ++c) {
                if (!ok)
                    continue;
                int64_t mb = c * cs_sys, me = mb + cs_sys < M ? mb + cs_sys : M;
                double cs = 0.0;
                for (int64_t m = mb; m < me; ++m) {
                    cs += path_forward(pb, thr, seed, iter, (uint32_t)m, mu, &w);
                    if (g)
                        path_adjoint(pb, mu, &w, gsum + (size_t)c * nl);
                }
                csum[c] = cs;
            }
        }
        work_free(&w);
    }
    if (rc) {
        free(csum);
        free(gsum);
        return -2;
    }
    double ctot = 0.0;
    for (int64_t c = 0; c < nchunk; ++c)
        ctot += csum[c];
    *J = ctot / P;
    if (g) {
        for (size_t q = 0; q < nl; ++q) {
            double t = 0.0;
            for (int64_t c = 0; c < nchunk; ++c)
                t += gsum[(size_t)c * nl + q];
            g[q] = t / P;
        }
    }
    free(csum);
    free(gsum);
    return 0;
}

int fb_cost_grad(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                 const double* mu, double* J, double* g, int nthreads)
{
    return cost_grad_impl(pb, M, seed, iter, mu, J, g, nthreads, 0);
}

int fb_grad_scale(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                  const double* mu, double* s, int nthreads)
{
    double J;
    if (!s)
        return -1;
    return cost_grad_impl(pb, M, seed, iter, mu, &J, s, nthreads, 1);
}

/* The surrogate adjoint of path m (forward jump counts in w->n): the recursion
 * of path_adjoint at the states zs_k; adds gamma^{n_k} ls^v_{k+1} phi(zs_k) to
 * G.  Writes the surrogate adjoint into w->lam.  Independent particles only. */
static void path_adjoint_surrogate(const fb_problem* pb, const double* mu, uint64_t seed,
                                   uint32_t iter, uint32_t m, work* w, double* G)
{
    const int N = pb->N, L = pb->nx * pb->nv;
    const double dt = pb->T / (double)N;
    double zs[2], gz[2];
    fb_surrogate_state(pb, seed, m, (uint32_t)N, iter, zs);
    track_grad(pb, zs, N, gz);
    double lx = dt * gz[0], lv = dt * gz[1];
    w->lam[2 * N] = lx;
    w->lam[2 * N + 1] = lv;
    for (int k = N - 1; k >= 0; --k) {
        const double* mk = mu + (size_t)k * L;
        fb_surrogate_state(pb, seed, m, (uint32_t)k, iter, zs);
        shapes(pb, zs, w->px, w->pv, w->dpx, w->dpv);
        double gn, Vn;
        ks_factors(pb, w->n[k], &gn, &Vn);
        for (int i = 0; i < pb->nx; ++i)
            for (int l = 0; l < pb->nv; ++l)
                G[(size_t)k * L + i * pb->nv + l] += summand(w, w->px[i] * w->pv[l] * (gn * lv));
        if (k == 0)
            break;
        double u = control(pb, mk, w->px, w->pv);
        double ux = control(pb, mk, w->dpx, w->pv);
        double uv = control(pb, mk, w->px, w->dpv);
        track_grad(pb, zs, k, gz);
        double nlx = lx + gn * dt * (ux - pb->eta) * lv + dt * gz[0] + dt * pb->alpha * u * ux;
        double nlv = dt * lx + gn * (1.0 + dt * uv) * lv + dt * gz[1] + dt * pb->alpha * u * uv;
        lx = nlx;
        lv = nlv;
        w->lam[2 * k] = lx;
        w->lam[2 * k + 1] = lv;
    }
    w->lam[0] = 0.0;
    w->lam[1] = 0.0;
}

static int check_surrogate(const fb_problem* pb)
{
    return check_problem(pb) || pb->np != 1 || pb->grid != 0 || !pb->zd ? -1 : 0;
}

int fb_paths_surrogate(const fb_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
                       const double* mu, double* lam, int nthreads)
{
    if (check_surrogate(pb) || pb->svar_kind != 0 || !mu || !lam || m0 < 0 || count < 0)
        return -1;
    const int N = pb->N, L = pb->nx * pb->nv;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    double* G = (double*)calloc((size_t)N * L, sizeof(double));
    if (!G)
        return -2;
    int rc = 0;
    work w;
    if (work_alloc(pb, &w) == 0) {
        for (int64_t p = 0; p < count; ++p) {
            path_forward(pb, thr, seed, iter, (uint32_t)(m0 + p), mu, &w);
            path_adjoint_surrogate(pb, mu, seed, iter, (uint32_t)(m0 + p), &w, G);
            memcpy(lam + (size_t)p * (N + 1) * 2, w.lam, (size_t)(N + 1) * 2 * sizeof(double));
        }
    } else {
        rc = -2;
    }
    work_free(&w);
    free(G);
    (void)nthreads;
    return rc;
}

/* Per-step sums over the particles, in chunks of FB_CHUNK consecutive
 * particles (each chunk in particle order, the chunks in index order):
 * pass 0 sums z_k,c, pass 1 sums (z_k,c - zbar[k,c])^2. */
static int ensemble_sums(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                         const double* mu, int pass, const double* zbar, double* out,
                         int nthreads)
{
    const int N = pb->N;
    const size_t nk = (size_t)(N + 1) * 2;
    const int64_t nchunk = (M + FB_CHUNK - 1) / FB_CHUNK;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    double* part = (double*)calloc((size_t)nchunk * nk, sizeof(double));
    if (!part)
        return -2;
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : rc)
    {
        work w;
        const int ok = work_alloc(pb, &w) == 0;
        rc |= ok ? 0 : 1;
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < nchunk; ++c) {
                if (!ok)
                    continue;
                int64_t mb = c * FB_CHUNK, me = mb + FB_CHUNK < M ? mb + FB_CHUNK : M;
                double* S = part + (size_t)c * nk;
                for (int64_t m = mb; m < me; ++m) {
                    path_forward(pb, thr, seed, iter, (uint32_t)m, mu, &w);
                    for (size_t q = 0; q < nk; ++q) {
                        double d = pass == 0 ? w.z[q] : w.z[q] - zbar[q];
                        S[q] += pass == 0 ? d : d * d;
                    }
                }
            }
        }
        work_free(&w);
    }
    if (!rc) {
        for (size_t q = 0; q < nk; ++q) {
            double t = 0.0;
            for (int64_t c = 0; c < nchunk; ++c)
                t += part[(size_t)c * nk + q];
            out[q] = t;
        }
    }
    free(part);
    return rc ? -2 : 0;
}

/* The forward ensemble's variance per step and component (the population
 * variance about the per-step mean, in two passes) and the ordinary
 * least-squares line through the points (t_k, V_k,c), k = 0..N, equal weights:
 * b = sum (t_k - tbar)(V_k - Vbar) / sum (t_k - tbar)^2, a = Vbar - b tbar.
 * Section 6.5 asks for a surrogate variance that grows linearly in time and
 * follows the forward model's own variance. */
int fb_surrogate_fit(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                     const double* mu, double* var, double a[2], double b[2], int nthreads)
{
    if (check_surrogate(pb) || M < 1 || !mu || !a || !b)
        return -1;
    const int N = pb->N;
    const size_t nk = (size_t)(N + 1) * 2;
    const double dt = pb->T / (double)N;
    double* zbar = (double*)malloc(nk * sizeof(double));
    double* V = (double*)malloc(nk * sizeof(double));
    int rc = (zbar && V) ? 0 : -2;
    if (!rc)
        rc = ensemble_sums(pb, M, seed, iter, mu, 0, NULL, zbar, nthreads);
    if (!rc) {
        for (size_t q = 0; q < nk; ++q)
            zbar[q] /= (double)M;
        rc = ensemble_sums(pb, M, seed, iter, mu, 1, zbar, V, nthreads);
    }
    if (!rc) {
        for (size_t q = 0; q < nk; ++q)
            V[q] /= (double)M;
        double tbar = 0.0;
        for (int k = 0; k <= N; ++k)
            tbar += (double)k * dt;
        tbar /= (double)(N + 1);
        for (int c = 0; c < 2; ++c) {
            double vbar = 0.0;
            for (int k = 0; k <= N; ++k)
                vbar += V[2 * k + c];
            vbar /= (double)(N + 1);
            double sxy = 0.0, sxx = 0.0;
            for (int k = 0; k <= N; ++k) {
                double dtk = (double)k * dt - tbar;
                sxy += dtk * (V[2 * k + c] - vbar);
                sxx += dtk * dtk;
            }
            b[c] = sxy / sxx;
            a[c] = vbar - b[c] * tbar;
        }
        if (var)
            memcpy(var, V, nk * sizeof(double));
    }
    free(zbar);
    free(V);
    return rc;
}

/* Surrogate gradient (Section 6.5): the forward adds alpha u_k phi(z_k) as it
 * goes, the adjoint runs on the surrogate states; nothing is stored.  With
 * svar_kind 1 the variance line is first fitted to the forward ensemble. */
static int surrogate_impl(const fb_problem* pb_in, int64_t M, uint64_t seed, uint32_t iter,
                          const double* mu, double* J, double* g, int nthreads, int absval)
{
    if (check_surrogate(pb_in) || M < 1 || !mu || !J || !g)
        return -1;
    fb_problem fitted = *pb_in;
    if (pb_in->svar_kind == 1) {
        int frc = fb_surrogate_fit(pb_in, M, seed, iter, mu, NULL, fitted.svar0, fitted.svar1,
                                   nthreads);
        if (frc)
            return frc;
        fitted.svar_kind = 0;
    }
    const fb_problem* pb = &fitted;
    const int N = pb->N, L = pb->nx * pb->nv;
    const size_t nl = (size_t)N * L;
    const int64_t nchunk = (M + FB_CHUNK - 1) / FB_CHUNK;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    double* csum = (double*)calloc((size_t)nchunk, sizeof(double));
    double* gsum = (double*)calloc((size_t)nchunk * nl, sizeof(double));
    if (!csum || !gsum) {
        free(csum);
        free(gsum);
        return -2;
    }
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : rc)
    {
        work w;
        const int ok = work_alloc(pb, &w) == 0;
        rc |= ok ? 0 : 1;
        w.absval = absval;
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < nchunk; ++c) {
                if (!ok)
                    continue;
                int64_t mb = c * FB_CHUNK, me = mb + FB_CHUNK < M ? mb + FB_CHUNK : M;
                double cs = 0.0;
                double* G = gsum + (size_t)c * nl;
                for (int64_t m = mb; m < me; ++m) {
                    cs += path_forward(pb, thr, seed, iter, (uint32_t)m, mu, &w);
                    for (int k = 0; k < N; ++k) {
                        shapes(pb, w.z + 2 * k, w.px, w.pv, NULL, NULL);
                        double au = pb->alpha * w.u[k];
                        for (int i = 0; i < pb->nx; ++i)
                            for (int l = 0; l < pb->nv; ++l)
                                G[(size_t)k * L + i * pb->nv + l] += summand(&w, w.px[i] * w.pv[l] * au);
                    }
                    path_adjoint_surrogate(pb, mu, seed, iter, (uint32_t)m, &w, G);
                }
                csum[c] = cs;
            }
        }
        work_free(&w);
    }
    if (rc) {
        free(csum);
        free(gsum);
        return -2;
    }
    double ctot = 0.0;
    for (int64_t c = 0; c < nchunk; ++c)
        ctot += csum[c];
    *J = ctot / (double)M;
    for (size_t q = 0; q < nl; ++q) {
        double t = 0.0;
        for (int64_t c = 0; c < nchunk; ++c)
            t += gsum[(size_t)c * nl + q];
        g[q] = t / (double)M;
    }
    free(csum);
    free(gsum);
    return 0;
}

int fb_cost_grad_surrogate(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                           const double* mu, double* J, double* g, int nthreads)
{
    return surrogate_impl(pb, M, seed, iter, mu, J, g, nthreads, 0);
}

int fb_grad_scale_surrogate(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                            const double* mu, double* s, int nthreads)
{
    double J;
    if (!s)
        return -1;
    return surrogate_impl(pb, M, seed, iter, mu, &J, s, nthreads, 1);
}

/* Tangent of particle m's cost on the jump-adapted grid (path in w): each
 * Euler sub-step and jump differentiated directly. */
static double tangent_adapted(const fb_problem* pb, const double* mu, const double* dmu, work* w)
{
    const int N = pb->N, L = pb->nx * pb->nv;
    double tx = 0.0, tv = 0.0, dc = 0.0, gz[2], zt[2];
    for (int k = 0; k < N; ++k) {
        const double* mk = mu + (size_t)k * L;
        const int n = w->n[k];
        for (int r = 0; r <= n; ++r) {
            const int s = k * FB_SUB + r;
            const double* zs = w->sz + 2 * s;
            const double d = w->sd[s], u = w->su[s];
            shapes(pb, zs, w->px, w->pv, w->dpx, w->dpv);
            double du = control(pb, mk, w->dpx, w->pv) * tx + control(pb, mk, w->px, w->dpv) * tv +
                        control(pb, dmu + (size_t)k * L, w->px, w->pv);
            dc += d * pb->alpha * u * du;
            double nx = tx + d * tv;
            double nv = tv + d * (du - pb->eta * tx);
            if (r < n)
                nv *= pb->gamma;
            tx = nx;
            tv = nv;
            /* the state at the sub-step's end */
            const double* ze = r < n ? w->sz + 2 * (s + 1) : w->z + 2 * (k + 1);
            const double a_end = r < n ? w->sa[s + 1] : 1.0;
            track_grad_to(pb, ze, target_at(pb, k, a_end, zt), gz);
            dc += d * (gz[0] * tx + gz[1] * tv);
        }
    }
    return dc;
}

/* Forward-mode derivative of J along dmu: differentiates the Euler step with
 * its coupling, the jump composition and the cost directly, independently of
 * the adjoint.  t holds the tangents (dx_j, dv_j) of the current step. */
int fb_tangent(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
               const double* mu, const double* dmu, double* dJ, int nthreads)
{
    if (check_problem(pb) || M < 1 || !mu || !dmu || !dJ)
        return -1;
    const int N = pb->N, L = pb->nx * pb->nv, np = pb->np;
    const double dt = pb->T / (double)N;
    const int64_t cs_sys = chunk_systems(pb);
    const int64_t nchunk = (M + cs_sys - 1) / cs_sys;
    uint64_t thr[32];
    or_poisson_thresholds(rate_dt(pb), thr);
    double* csum = (double*)calloc((size_t)nchunk, sizeof(double));
    if (!csum)
        return -2;
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : rc)
    {
        work w;
        double* t = (double*)malloc((size_t)np * 4 * sizeof(double));
        const int ok = work_alloc(pb, &w) == 0 && t;
        rc |= ok ? 0 : 1;
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < nchunk; ++c) {
                if (!ok)
                    continue;
                int64_t mb = c * cs_sys, me = mb + cs_sys < M ? mb + cs_sys : M;
                double cs = 0.0;
                for (int64_t m = mb; m < me; ++m) {
                    path_forward(pb, thr, seed, iter, (uint32_t)m, mu, &w);
                    if (pb->grid == 1) {
                        cs += tangent_adapted(pb, mu, dmu, &w);
                        continue;
                    }
                    double* tn = t + 2 * np;
                    for (int j = 0; j < 2 * np; ++j)
                        t[j] = 0.0;
                    double dc = 0.0;
                    for (int k = 0; k < N; ++k) {
                        const double* mk = mu + (size_t)k * L;
                        for (int j = 0; j < np; ++j) {
                            const double* zk = w.z + 2 * (k * np + j);
                            const double tx = t[2 * j], tv = t[2 * j + 1];
                            shapes(pb, zk, w.px, w.pv, w.dpx, w.dpv);
                            double u = w.u[k * np + j];
                            double du = control(pb, mk, w.dpx, w.pv) * tx +
                                        control(pb, mk, w.px, w.dpv) * tv +
                                        control(pb, dmu + (size_t)k * L, w.px, w.pv);
                            dc += dt * pb->alpha * u * du;
                            double gn, Vn;
                            ks_factors(pb, w.n[k * np + j], &gn, &Vn);
                            double txl = t[2 * left_of(pb, j)], txr = t[2 * right_of(pb, j)];
                            tn[2 * j] = tx + dt * tv;
                            tn[2 * j + 1] = gn * (tv + dt * (du - pb->eta * tx -
                                                             pb->omega * (2.0 * tx - txl - txr)));
                        }
                        for (int j = 0; j < np; ++j) {
                            t[2 * j] = tn[2 * j];
                            t[2 * j + 1] = tn[2 * j + 1];
                            double gz[2];
                            track_grad(pb, w.z + 2 * ((k + 1) * np + j), k + 1, gz);
                            dc += dt * (gz[0] * t[2 * j] + gz[1] * t[2 * j + 1]);
                        }
                    }
                    cs += dc;
                }
                csum[c] = cs;
            }
        }
        free(t);
        work_free(&w);
    }
    double tot = 0.0;
    for (int64_t c = 0; c < nchunk; ++c)
        tot += csum[c];
    *dJ = tot / ((double)M * (double)np);
    free(csum);
    return rc ? -2 : 0;
}

/* Algorithm 5.4: iteration n draws with counter iter0 + n, every Armijo trial
 * of the iteration reuses it; descent along -g with ||v||^2 = dt sum |v_k|^2. */
int fb_optimize(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter0, int32_t n_max,
                double tol, double zeta0, double rho, double c_armijo, int32_t max_backtracks,
                double* mu, double* logJ, double* log_gnorm, double* log_zeta, int32_t* log_bt,
                double* logE, int surrogate, int nthreads)
{
    if (check_problem(pb) || !mu || n_max < 0 || max_backtracks < 1)
        return -1;
    const int N = pb->N, L = pb->nx * pb->nv;
    const double dt = pb->T / (double)N;
    const size_t nl = (size_t)N * L;
    double* g = (double*)malloc(nl * sizeof(double));
    double* mt = (double*)malloc(nl * sizeof(double));
    if (!g || !mt) {
        free(g);
        free(mt);
        return -2;
    }
    int n;
    for (n = 0; n < n_max; ++n) {
        uint32_t it = iter0 + (uint32_t)n;
        double J;
        int grc = surrogate ? fb_cost_grad_surrogate(pb, M, seed, it, mu, &J, g, nthreads)
                            : fb_cost_grad(pb, M, seed, it, mu, &J, g, nthreads);
        if (grc) {
            n = -2;
            break;
        }
        double gg = 0.0;
        for (size_t q = 0; q < nl; ++q)
            gg += g[q] * g[q];
        gg *= dt;
        double zeta = zeta0;
        int accepted = 0, bt;
        for (bt = 0; bt < max_backtracks; ++bt) {
            for (size_t q = 0; q < nl; ++q)
                mt[q] = mu[q] - zeta * g[q];
            double Jt;
            fb_cost_grad(pb, M, seed, it, mt, &Jt, NULL, nthreads);
            if (Jt <= J - c_armijo * zeta * gg) {
                accepted = 1;
                break;
            }
            zeta *= rho;
        }
        if (!accepted) {
            n = -3;
            break;
        }
        double E = 0.0;
        for (size_t q = 0; q < nl; ++q) {
            double r = mt[q] - mu[q];
            E += r * r;
            mu[q] = mt[q];
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
        if (E <= tol) {
            ++n;
            break;
        }
    }
    free(g);
    free(mt);
    return n;
}
