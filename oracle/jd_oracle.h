/*
 * FP64 CPU oracle for the discretize-then-optimize adjoint Monte Carlo method for
 * controlled jump-diffusions (Bartsch, Borzi, Ciaramella, Reichle, "Adjoint-based
 * optimal control of jump-diffusion processes", arXiv 2505.04328).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  It shares no code, header,
 * table or constant generator with the GPU library: every piece here (Philox,
 * uniform map, Box-Muller, Poisson thresholds, Euler step, adjoint, reductions,
 * optimizer) is written independently from the published definitions.
 *
 * Conventions (state X in R^d, paths m = 0..M-1, steps k = 0..N-1, dt = T/N):
 *   X_{k+1} = X_k + dt*(A X_k - c3 X_k^3 + B u_k) + sqrt(dt) s.Z^W_k + dJ_k
 *   C^m     = sum_{k<N} dt/2 |X_k - xd_k|^2 + 1/2 |X_N - xT|^2
 *   J       = (1/M) sum_m C^m + nu*dt/2 sum_k |u_k|^2
 *   lam_N   = X_N - xT,
 *   lam_k   = lam_{k+1} + dt*[(A - 3 c3 diag(X_k^2))^T lam_{k+1} + (X_k - xd_k)]
 *   g_k     = nu u_k + (1/M) sum_m B^T lam^m_{k+1}          (dJ/du_k = dt*g_k)
 * lam = dC/dX is minus the paper's adjoint r (Section 4, adjoint model).
 */
#ifndef JD_ORACLE_H
#define JD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem data, all host memory, FP64.  A and B are d*d row-major; xd is N*d
 * (row k = x_d(t_k)). */
typedef struct {
    int32_t d, N;
    double T, lambda, cubic, nu;
    const double *x0, *A, *B, *s, *jump_mean, *jump_std, *xT, *xd;
} or_problem;

typedef struct {
    int32_t n_max;
    double tol, zeta0, rho, c_armijo;
    int32_t max_backtracks;
} or_opt;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint32_t w);
void or_uniform_batch(const uint32_t* w, int64_t n, double* out);
void or_poisson_thresholds(double mu, uint64_t thr[32]);
int or_poisson_count(uint32_t P, const uint64_t thr[32]);

/* Draws of the (m,k) path-step under iteration counter iter: zw, zj have d
 * entries; *count is the Poisson jump count. */
void or_draws(uint64_t seed, uint32_t m, uint32_t k, uint32_t iter, int d,
              const uint64_t thr[32], double* zw, double* zj, int* count);

/* Grid of draws for paths m0..m0+mc-1 and steps k0..k0+kc-1, path-major:
 * zw[((p*kc)+q)*d + i], counts[p*kc + q]. */
void or_draws_grid(uint64_t seed, uint32_t iter, int d, double mu,
                   int64_t m0, int64_t mc, int32_t k0, int32_t kc,
                   double* zw, double* zj, int32_t* counts);

/* Per-path states X (count x (N+1) x d), adjoints lam (count x (N+1) x d, row 0
 * unused and zeroed) and path costs C (count), for paths m0..m0+count-1.  Any
 * output pointer may be NULL. */
int or_paths(const or_problem* pb, uint64_t seed, uint32_t iter, int64_t m0, int64_t count,
             const double* u, double* X, double* lam, double* C, int nthreads);

/* J and g (N*d) over M paths, chunked fixed-order FP64 sums. g may be NULL. */
int or_cost_grad(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                 const double* u, double* J, double* g, int nthreads);

/* Test diagnostic: s (N*d) = nu |u| + (1/M) sum_m |B^T lam^m_{k+1}| per entry,
 * the scale of each gradient entry's Monte Carlo summands. */
int or_grad_scale(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
                  const double* u, double* s, int nthreads);

/* Tangent-linear directional derivative dJ[delta]. */
int or_tangent(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter,
               const double* u, const double* delta, double* dJ, int nthreads);

/* Gradient iteration with stochastic Armijo backtracking (Section 5, optimization
 * procedure).  u is in/out.  Per-iteration log arrays (n_max entries each) may be
 * NULL.  Returns number of iterations done (>= 0) or a negative error. */
int or_optimize(const or_problem* pb, int64_t M, uint64_t seed, uint32_t iter0,
                const or_opt* opt, double* u, double* logJ, double* log_gnorm,
                double* log_zeta, int32_t* log_bt, double* logE, int nthreads);

#ifdef __cplusplus
}
#endif

#endif
