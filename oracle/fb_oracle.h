/*
 * FP64 CPU oracle for the paper's own model problem (Bartsch, Borzi,
 * Ciaramella, Reichle, arXiv 2505.04328, Sections 2 and 5): a particle in
 * phase space z = (x, v) driven by a harmonic oscillator, Brownian noise,
 * Keilson-Storer velocity jumps and a feedback control built from
 * radial-basis shape functions, with a Gaussian tracking cost.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory.
 *
 * Conventions (paths m, steps k = 0..N-1, dt = T/N, t_k = k dt):
 *   centres   xc_i = (i + 1/2) 2 xmax/nx - xmax,  vc_l = (l + 1/2) 2 vmax/nv - vmax
 *   bump      b(r) = exp(-1/(1 - (eps r)^2)) for |r| < 1/eps, else 0
 *   shape     phi_{i nv + l}(x, v) = b(x - xc_i) b(v - vc_l),  L = nx nv
 *   control   u_k = sum_l mu_k[l] phi_l(z_k)              (mu is N x L)
 *   forward   x_{k+1} = x_k + dt v_k + b1 sqrt(dt) Zx
 *             v*      = v_k + dt (u_k - eta x_k) + b2 sqrt(dt) Zv
 *             v_{k+1} = gamma^n v* + sqrt(V_n) ZJ,  V_n = (1/(2 beta)) sum_{i<n} gamma^{2i}
 *             (n ~ Poisson(sigma dt) Keilson-Storer jumps in the step, sigma = sqrt(beta/pi))
 *   cost      C = dt sum_{k=1..N} Jt(z_k, zd_k) + dt alpha/2 sum_{k=0..N-1} u_k^2
 *             Jt(z, zd) = -exp(-|z - zd|^2 / (2 sigJ^2))
 *   adjoint   lam = dC/dz:  lam_N = dt grad Jt(z_N)
 *             lam^x_k = lam^x_{k+1} + gamma^n dt (u_x - eta) lam^v_{k+1} + dt dJt/dx + dt alpha u u_x
 *             lam^v_k = dt lam^x_{k+1} + gamma^n (1 + dt u_v) lam^v_{k+1} + dt dJt/dv + dt alpha u u_v
 *   gradient  g_k[l] = (1/M) sum_m phi_l(z_k) (alpha u_k + gamma^{n_k} lam^v_{k+1})
 *             (dJ/dmu_k = dt g_k)
 *
 * Coupled particles (Section 6.4, eq. interacting_model): a system is a ring of
 * np particles j = 0..np-1 (np = 1: the independent particles above); particle
 * j of system m is particle p = m np + j and draws with counter word 0 = p.
 * The velocity update of particle j adds the nearest-neighbour force
 *   v* = v_k + dt (u_k - eta x_k - omega (2 x_{j,k} - x_{j-1,k} - x_{j+1,k})) + ...
 * (indices mod np).  The cost of a system is the mean of its particles' costs,
 * J the mean over all M np particles, and the adjoint of particle j gains
 *   lam^x_{j,k} += dt omega (w_{j-1} + w_{j+1} - 2 w_j),  w_i = gamma^{n_{i,k}} lam^v_{i,k+1}.
 * Ellipse cost (eq. phonon_functional_tracking): Jt(z) = -exp(-q^2/(2 sigJ^2)),
 * q = x^2/ax^2 + v^2/av^2 - 1.  Ellipse start (eq. coupled_ellipse): particle j
 * at (ax cos th_j, av sin th_j), th_j = 2 pi j / np, plus s0 . (Z1, Z2).
 *
 * Jump-adapted grid (grid = 1; Section 3, the union of the uniform points and
 * each particle's jump times, integrated as in Algorithms 5.1-5.2; independent
 * particles).  In uniform interval k the particle has n ~ Poisson(sigma dtau)
 * jumps (the count of block (m, k, iter, 0)) at offsets a_1 < ... < a_n (in
 * units of dtau) drawn as the ordered minima of uniforms,
 *   a_r = a_{r-1} + (1 - a_{r-1}) (1 - V_r^{1/(n-r+1)}),  a_0 = 0, a_{n+1} = 1,
 * V_r = word (r-1) mod 4 of block (m, k, iter, 64 + (r-1)/4)  (the order
 * statistics of n uniforms: a Poisson process on the interval).  Sub-step r
 * (r = 0..n) spans [a_r, a_{r+1}] dtau with length d_r and normals (Zx_r, Zv_r):
 * the Box-Muller pair of words 0, 1 of block (m, k, iter, r).  Sub-step r < n
 * ends at jump r+1: v <- gamma v + S_{r+1} / sqrt(2 beta), S_r the cosine branch
 * of words 2, 3 of block (m, k, iter, r).  Euler on each sub-step with the
 * interval's control mu_k; the cost is
 *   C = sum over sub-steps [ d_r Jt(z_end, zd(t_end)) + d_r alpha/2 u_r^2 ]
 * (z_end the post-jump state, zd linear between the uniform targets), the
 * adjoint the exact transpose (p <- gamma p at the jumps) and
 *   g_k[l] = (1/(M dtau)) sum_m sum_r d_r phi_l(z_r) (alpha u_r + lam^v_-(end of r)),
 * lam^v_- the adjoint of the pre-jump velocity.  With no jumps this is the
 * fixed-grid model exactly.
 *
 * Surrogate gradient (Section 6.5, the adjoint independent of the forward
 * trajectories): the adjoint runs on states zs_k ~ N(zd_k, diag(var(t_k))),
 * one sample per particle and realization, zs_k = zd_k + sqrt(var(t_k)) Z with
 * Z the Box-Muller pair of words 0, 1 of Philox block (m, 0xFFFFFFFE, iter, 1)
 * at every step, with the forward's jump counts; no trajectory is stored:
 *   gs_k[l] = (1/M) sum_m [ alpha u_k phi_l(z_k) + gamma^{n_k} ls^v_{k+1} phi_l(zs_k) ]
 * where ls is the adjoint recursion above evaluated at zs (u, u_x, u_v and
 * grad Jt at zs_k).  The variance is var_c(t) = max(0, svar0[c] + svar1[c] t):
 * with svar_kind 0 the line as given; with svar_kind 1 the ordinary
 * least-squares line through the points (t_k, V_k,c), k = 0..N, where
 *   V_k,c = (1/M) sum_m (z^m_k,c - zbar_k,c)^2,  zbar_k,c = (1/M) sum_m z^m_k,c
 * is the forward ensemble's own per-step variance under the same mu and draws
 * (svar0 and svar1 are then ignored).
 */
#ifndef FB_ORACLE_H
#define FB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t N, nx, nv;
    double T, eta, b1, b2, gamma, beta;
    double xmax, vmax, eps, alpha, sigJ;
    int32_t init_kind;     /* 0: Gaussian z0 + s0 * Z, 1: uniform on [z0 - s0, z0 + s0],
                              2: ellipse points + s0 * Z */
    double z0[2], s0[2];
    double svar0[2], svar1[2]; /* surrogate-state variance line var_c(t) = svar0[c] + svar1[c] t
                                  (finite; evaluated as max(0, .)) */
    const double* zd;      /* (N+1) x 2, row k = desired (x, v) at t_k (tracking cost) */
    int32_t np;            /* particles per system (ring), >= 1 */
    double omega;          /* nearest-neighbour coupling */
    int32_t cost_kind;     /* 0: tracking cost around zd, 1: ellipse cost */
    double ax, av;         /* ellipse half-axes (cost_kind 1, init_kind 2) */
    int32_t grid;          /* 0: fixed grid with Poisson counts, 1: jump-adapted grid */
    int32_t svar_kind;     /* surrogate variance: 0 the given line, 1 fitted to the forward ensemble */
} fb_problem;

/* Bump b(r) and its derivative b'(r). */
double fb_bump(double r, double eps);
double fb_bump_deriv(double r, double eps);

/* Draws of particle m under iteration iter: initial state (x, v), and for step k
 * the normals (Zx, Zv, ZJ) and the jump count n. */
void fb_initial(const fb_problem* pb, uint64_t seed, uint32_t m, uint32_t iter, double z[2]);
void fb_step_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, const uint64_t thr[32],
                   double Z[3], int* n);

/* Jump-adapted draws of interval k of particle m: the count n, the offsets
 * a[0..n+1], the sub-step normals Z[2r], Z[2r+1] (r = 0..n) and the jump
 * normals S[r] (r = 1..n).  Arrays hold 33, 33 x 2 and 32 entries. */
void fb_adapted_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, const uint64_t thr[32],
                      int* n, double* a, double* Z, double* S);

/* Per-particle states z (P x (N+1) x 2), adjoints lam (P x (N+1) x 2, row 0
 * zero), controls u (P x N), jump counts (P x N) and costs C (P) of the
 * P = count np particles of systems m0..m0+count-1, in particle order.  Any
 * output may be NULL. */
int fb_paths(const fb_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
             const double* mu, double* z, double* lam, double* u, int32_t* jumps, double* C,
             int nthreads);

/* J and g (N x L) over M systems (M np particles), fixed-order chunked FP64
 * sums.  g may be NULL. */
int fb_cost_grad(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                 const double* mu, double* J, double* g, int nthreads);

/* Test diagnostic, not part of the method: s (N x L), the mean over the
 * particles of the absolute value of each particle's gradient summand, from
 * the same paths and loops as fb_cost_grad / fb_cost_grad_surrogate.  A
 * gradient entry whose summands cancel is small against s, and rounding in the
 * per-particle arithmetic moves it in proportion to s, not to its own size. */
int fb_grad_scale(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                  const double* mu, double* s, int nthreads);
int fb_grad_scale_surrogate(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                            const double* mu, double* s, int nthreads);

/* Surrogate state of path m at step k. */
void fb_surrogate_state(const fb_problem* pb, uint64_t seed, uint32_t m, uint32_t k, uint32_t iter,
                        double z[2]);

/* The forward ensemble's per-step variance var ((N+1) x 2, may be NULL) of
 * the M particles under mu, and the least-squares line a[c] + b[c] t through
 * it (the fitted surrogate variance, svar_kind 1; computed whatever svar_kind
 * holds). */
int fb_surrogate_fit(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                     const double* mu, double* var, double a[2], double b[2], int nthreads);

/* Per-path surrogate adjoints ls (count x (N+1) x 2, row 0 zero); svar_kind 0
 * only (a fitted line depends on all M particles: pass it as the given line).
 * The surrogate functions take independent particles only (np = 1). */
int fb_paths_surrogate(const fb_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
                       const double* mu, double* lam, int nthreads);

/* J (exact) and the surrogate gradient gs (N x L). */
int fb_cost_grad_surrogate(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                           const double* mu, double* J, double* g, int nthreads);

/* Tangent-linear directional derivative dJ[dmu]. */
int fb_tangent(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
               const double* mu, const double* dmu, double* dJ, int nthreads);

/* Gradient iteration with stochastic Armijo backtracking on the same draws
 * (Section 5, Algorithm 5.4); mu in/out.  Logs may be NULL.  surrogate != 0
 * steps along the surrogate gradient (the Armijo test uses the exact cost). */
int fb_optimize(const fb_problem* pb, int64_t M, uint64_t seed, uint32_t iter0, int32_t n_max,
                double tol, double zeta0, double rho, double c_armijo, int32_t max_backtracks,
                double* mu, double* logJ, double* log_gnorm, double* log_zeta, int32_t* log_bt,
                double* logE, int surrogate, int nthreads);

#ifdef __cplusplus
}
#endif

#endif
