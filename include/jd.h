/*
 * jd.h -- C ABI of libjd, the MI355X (gfx950) hot path of the adjoint Monte
 * Carlo method for optimal control of jump-diffusion processes of Bartsch,
 * Borzi, Ciaramella and Reichle, "Adjoint-based optimal control of
 * jump-diffusion processes" (arXiv 2505.04328).
 *
 * Model (the paper's Section 2, eq. SDE_constraint, with an open-loop control
 * that is piecewise constant on the grid t_k = k dt, dt = T/N, Section 3,
 * eq. piecewise_constant_control; fixed-grid Euler-Maruyama with a Poisson
 * number of additive jumps per step, Section 3, eq. model_approximation and
 * Section 5, model equation):
 *
 *   X_0     = x0
 *   X_{k+1} = X_k + dt (A X_k - c3 X_k.X_k.X_k + B u_k) + sqrt(dt) s.Z^W_k + dJ_k
 *   dJ_k    = n_k jump_mean + jump_std.sqrt(n_k).Z^J_k,   n_k ~ Poisson(lambda dt)
 *
 * Cost (Section 3, discrete functional; left-point running cost and a
 * terminal term):
 *   C^m = sum_{k<N} dt/2 |X_k - xd_k|^2 + 1/2 |X_N - xT|^2
 *   J   = (1/M) sum_m C^m + nu dt/2 sum_k |u_k|^2
 *
 * Adjoint (Section 4, eq. AdjointModel, with the dt factors of Section 5,
 * adjoint equation; lam = dC/dX = -r in the paper's sign):
 *   lam_N = X_N - xT
 *   lam_k = lam_{k+1} + dt [ (A - 3 c3 diag(X_k^2))^T lam_{k+1} + (X_k - xd_k) ]
 * Gradient (Section 4, eq. definition_Gradient), L2(0,T) representative:
 *   g_k = nu u_k + B^T (1/M) sum_m lam^m_{k+1},   dJ/du_k = dt g_k.
 *
 * Draws: Philox4x32-10 (Salmon et al., SC'11) with counter (m, k, iter, s) and
 * key (seed low, seed high); block s supplies components 2s and 2s+1; the
 * uniform of a word w is ((w >> 8) | 1) 2^-24; component i takes the Box-Muller
 * pair of words 2i, 2i+1 (cosine branch -> Z^W_i, sine branch -> Z^J_i); the
 * Poisson count compares the word built from the low bytes of block 0's four
 * words with inverse-CDF thresholds floor(2^32 F_j) of Poisson(lambda dt).
 * Every path can therefore be regenerated from (seed, m, iter) alone, which the
 * discretize-then-optimize adjoint needs (same increments and jump times as the
 * forward sweep, Section 4, remark after the adjoint model).
 *
 * Conventions for every entry point:
 *  - Return 0 on success, a negative JD_E* code on error; nothing throws.
 *  - Arguments are validated before anything is enqueued; an error return has
 *    no side effect on device memory.
 *  - Device buffers are owned by the caller and passed as raw device pointers;
 *    the library allocates no device memory.  Host arrays inside jd_problem
 *    are read during the call only.
 *  - All work is enqueued on `stream` and the call returns without waiting,
 *    except jd_optimize, which runs the line search on the device and
 *    synchronizes the stream once per batch of up to 64 iterations (see
 *    jd_optimize).  Kernel faults surface as JD_EHIP from a later call on the
 *    stream.
 *  - d in 1..8 (internally padded to 1, 2, 4 or 8 with inert components).
 *  - u and g are FP64, row-major N x d (u[k*d + c]).  J is one FP64.
 *  - Calls on different streams with different workspaces may run
 *    concurrently; calls sharing a workspace must be ordered by the caller.
 */
#ifndef JD_H
#define JD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JD_VERSION 101

/* Error codes. */
#define JD_OK 0
#define JD_EINVAL (-1)       /* invalid argument */
#define JD_EWORKSPACE (-2)   /* workspace smaller than jd_workspace_bytes() */
#define JD_EHIP (-3)         /* HIP launch or runtime error */
#define JD_ENONFINITE (-4)   /* J or g not finite */
#define JD_ELINESEARCH (-5)  /* no Armijo step within max_backtracks; u unchanged */
#define JD_EUNSUPPORTED (-6) /* valid but not built (e.g. checkpoint interval too long) */
#define JD_EAGAIN (-7)       /* result not ready yet (request server) */

/* Path arithmetic.  Reductions, J, g and the line search are FP64 in both. */
#define JD_FP32 0
#define JD_FP64 1

/* Trajectory handling between the forward and the adjoint sweep. */
#define JD_STORE 0     /* store X_1..X_N */
#define JD_RECOMPUTE 1 /* store X every K steps, regenerate segments in the adjoint */
#define JD_SURROGATE 2 /* feedback model only (jd_feedback.h): storage-free surrogate gradient */

/* Problem data (the paper's Section 2 problem statement reduced to the model
 * above).  All pointers except xd are HOST memory read during the call. */
typedef struct jd_problem {
    int32_t d;          /* state dimension, 1..8 */
    int32_t N;          /* time steps, >= 1 */
    double T;           /* horizon, > 0; dt = T/N */
    double lambda;      /* Poisson jump rate, >= 0, lambda*dt <= 2 */
    double cubic;       /* c3 of the drift term -c3 X^3 (elementwise) */
    double nu;          /* control weight, >= 0 */
    const double* x0;        /* host, d: initial state */
    const double* A;         /* host, d*d row-major: linear drift */
    const double* B;         /* host, d*d row-major: control matrix */
    const double* s;         /* host, d: diffusion scales (diagonal) */
    const double* jump_mean; /* host, d: mean of one jump */
    const double* jump_std;  /* host, d: std of one jump (per component) */
    const double* xT;        /* host, d: terminal target */
    const double* xd;        /* DEVICE, N*d FP64: x_d(t_k), row k */
} jd_problem;

/* Where the forward sweeps take the draws of a path-step from.  Every choice
 * gives bitwise the same results; they differ in speed only.  A sweep runs one
 * path per lane, so a run of few paths leaves most of the GPU idle and waits on
 * the latency of each step's draw chain (Philox, Box-Muller, the Poisson
 * count).  The table moves that chain into one launch over all path-steps per
 * gradient iteration, which the line-search trials of the iteration reuse
 * (they run on the iteration's draws). */
#define JD_NOISE_AUTO 0   /* the table for M <= 65536 paths in FP64 and
                             M <= 16384 in FP32 if it takes at most 1 GiB
                             (N*d*2 values per path), inline otherwise */
#define JD_NOISE_INLINE 1 /* each sweep computes its draws */
#define JD_NOISE_TABLE 2  /* the table, whatever the size: the workspace grows by
                             2*N*d*ceil(M/256)*256 values of the run precision */

/* One Monte Carlo evaluation. */
typedef struct jd_dump jd_dump;
typedef struct jd_run {
    int64_t M;          /* paths, 1..2^31 */
    uint64_t seed;      /* Philox key */
    uint32_t iter;      /* Philox counter word 2: fresh draws per gradient iteration */
    int32_t precision;  /* JD_FP32 or JD_FP64 */
    int32_t mode;       /* JD_STORE or JD_RECOMPUTE */
    int32_t K;          /* checkpoint interval for JD_RECOMPUTE (1..N); ignored for JD_STORE */
    const jd_dump* dump;/* optional per-path diagnostics, NULL normally */
    int32_t noise;      /* JD_NOISE_*; the feedback model (jd_feedback.h) checks the
                           value and always draws in the sweep */
} jd_run;

/* Per-path diagnostics for paths [m0, m0+count) (DEVICE pointers, each may be
 * NULL).  Written by jd_forward (cost) and jd_adjoint (X, lam), time-major:
 *   X[((k-1)*d + c)*count + p]   = X_k,c of path m0+p, k = 1..N, run precision
 *   lam[((k-1)*d + c)*count + p] = lam_k,c,                k = 1..N, run precision
 *   cost[p]                      = C^(m0+p), FP64. */
struct jd_dump {
    int64_t m0, count;
    void* X;
    void* lam;
    double* cost;
};

/* Line-search gradient iteration (Section 5, Algorithm 5.4 with the stochastic
 * Armijo rule eq. Stochastic_Armijo). */
typedef struct jd_opt {
    int32_t n_max;          /* iterations, >= 0 */
    int32_t max_backtracks; /* trials per iteration, >= 1 */
    double tol;             /* stop when ||u^{n+1} - u^n||_L2 <= tol (0: run n_max) */
    double zeta0;           /* first trial step, > 0 */
    double rho;             /* backtracking factor, in (0,1) */
    double c_armijo;        /* sufficient-decrease constant, > 0 */
} jd_opt;

/* Per-iteration record written by jd_optimize (host memory). */
typedef struct jd_iter_log {
    uint32_t iter;      /* Philox counter word used */
    int32_t backtracks; /* rejected trials before the accepted one */
    double J;           /* J(u^n) */
    double gnorm;       /* ||g^n||_L2 = sqrt(dt sum |g_k|^2) */
    double zeta;        /* accepted step */
    double J_new;       /* J(u^{n+1}) on the same draws */
    double E;           /* ||u^{n+1} - u^n||_L2 */
} jd_iter_log;

/* Library version (JD_VERSION). */
int jd_version(void);

/* Static text for an error code. */
const char* jd_strerror(int code);

/* Device workspace bytes needed by any entry point for this problem and run
 * (partial sums, per-step tables, line-search state).  0 if arguments are
 * invalid.  The same workspace serves every entry point. */
size_t jd_workspace_bytes(const jd_problem* prob, const jd_run* run);

/* Bytes of the trajectory buffer.  The buffer holds S slots (JD_STORE: S = N,
 * slot k-1 = X_k for k = 1..N; JD_RECOMPUTE: S = ceil(N/K), slot j-1 = X_{jK}
 * for j < S and slot S-1 = X_N) in blocks of 256 paths, elements of the run
 * precision: component c of slot q of path m is at
 *   ((m / 256) * S + q) * d * 256 + c * 256 + (m % 256),
 * i.e. each block of 256 paths owns a contiguous time-major region.  Its size
 * is S * d * ceil(M/256) * 256 elements.  0 if arguments are invalid. */
size_t jd_traj_bytes(const jd_problem* prob, const jd_run* run);

/* Forward sweep of all M paths (Section 3, eq. model_approximation; Section 5,
 * Algorithms 5.1-5.2 on the fixed grid): writes the trajectory (JD_STORE) or
 * the checkpoints (JD_RECOMPUTE) into traj, and J(u) into *J (device FP64).
 * traj may be NULL for a cost-only sweep.  u: device FP64 N*d. */
int jd_forward(const jd_problem* prob, const jd_run* run, const double* u, void* traj,
               double* J, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward adjoint sweep of all M paths (Section 4, eq. AdjointModel) over the
 * trajectory written by jd_forward with the same prob/run/u, and the Monte
 * Carlo gradient (Section 4, eq. definition_Gradient): grad (device FP64 N*d)
 * receives g (no dt factor).  In JD_RECOMPUTE mode each K-step segment is
 * regenerated from its checkpoint with the same counters, bit-identical to
 * the forward sweep. */
int jd_adjoint(const jd_problem* prob, const jd_run* run, const double* u, const void* traj,
               double* grad, void* ws, size_t ws_bytes, hipStream_t stream);

/* Forward + adjoint + reductions (Section 5, Algorithm 5.3): J -> *J,
 * g -> grad.  traj must hold jd_traj_bytes(). */
int jd_cost_grad(const jd_problem* prob, const jd_run* run, const double* u, double* J,
                 double* grad, void* traj, void* ws, size_t ws_bytes, hipStream_t stream);

/* Gradient iteration (Section 5, Algorithm 5.4): for n = 0, 1, ...: evaluate
 * J(u^n), g^n with counter word run->iter + n, then try u' = u^n - zeta g^n for
 * zeta = zeta0, rho zeta0, ... with the same counter word (common random
 * numbers) until J(u') is finite and J(u') <= J(u^n) - c zeta ||g^n||^2_L2
 * (eq. Stochastic_Armijo; a trial whose cost overflows is rejected like any
 * other); stop after n_max iterations or when ||u' - u^n||_L2 <= tol.  u
 * (device FP64 N*d) is updated in place; log (host, n_max entries, may be
 * NULL) gets one record per iteration and *iters_done (host, may be NULL) the
 * number done.
 * The Armijo decisions, the step and the stopping test are taken on the
 * device: the library enqueues the evaluation and a few trials of each of up
 * to 64 iterations, each gated by a phase word in the workspace header that
 * the device advances, then synchronizes `stream` once to read the outcome
 * and the iterations' log (and again only when an iteration needed more
 * trials than were enqueued).  The results are those of taking one trial at a
 * time.  Returns JD_ELINESEARCH (u at the last accepted iterate) when no
 * trial of max_backtracks is accepted, JD_ENONFINITE when J(u^n) or g^n is not
 * finite. */
int jd_optimize(const jd_problem* prob, const jd_run* run, const jd_opt* opt, double* u,
                jd_iter_log* log, int32_t* iters_done, void* traj, void* ws,
                size_t ws_bytes, hipStream_t stream);

/* jd_cost_grad without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that forbid
 * allocation): the workspace comes from a static device array of
 * jd_noalloc_capacity() bytes (64 MiB) that the library holds on every GPU it
 * runs on until the process ends.  The caller passes u, J, grad and traj as
 * for jd_cost_grad (traj: jd_traj_bytes()); results are bitwise those of
 * jd_cost_grad.  Returns JD_EWORKSPACE, before touching the device, when the
 * problem's workspace (jd_workspace_bytes() less 256 bytes of alignment
 * slack) exceeds the capacity: the 1-D workloads up to 2^20 paths x 1000 steps
 * fit.  A noise table chosen by JD_NOISE_AUTO that does not fit is left out
 * (the sweeps draw inline; the results do not change), so the check is on the
 * workspace without it.  The call allocates nothing (the first call on a device looks up the
 * array's device address once).  All calls on one GPU share the array: calls
 * that overlap in time on one device (different streams, or host threads)
 * race on it and must be ordered by the caller; the array keeps the last
 * call's contents, and every call initialises what it reads. */
size_t jd_noalloc_capacity(void);
int jd_cost_grad_noalloc(const jd_problem* prob, const jd_run* run, const double* u, double* J,
                         double* grad, void* traj, hipStream_t stream);

/* Reads the non-finite flag of the most recent entry-point call on this
 * workspace (each call clears it first; its reductions raise it when J or g is
 * not finite), then clears it.  Synchronizes `stream`.  Returns JD_OK or
 * JD_ENONFINITE. */
int jd_check_finite(void* ws, size_t ws_bytes, hipStream_t stream);

/* The draws of paths [m0, m0+mc) and steps [k0, k0+kc) under run->seed and
 * run->iter, exactly as the sweeps use them: zw, zj (device, run precision,
 * mc*kc*d, path-major: ((p*kc + q)*d + i)), counts (device int32, mc*kc).
 * Any output may be NULL. */
int jd_draws(const jd_problem* prob, const jd_run* run, int64_t m0, int64_t mc, int32_t k0,
             int32_t kc, void* zw, void* zj, int32_t* counts, hipStream_t stream);

/* Raw Philox4x32-10 blocks: out[4i..4i+3] for counter ctr[4i..4i+3] and key
 * (seed low, seed high).  ctr, out: device uint32, n >= 0 blocks. */
int jd_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t stream);

/* The Poisson thresholds the sweeps use for rate*dt = mu (host output, 32
 * entries): thr_j = min(2^32, floor(2^32 F_j)), F_j the Poisson(mu) CDF
 * accumulated in FP64 as p_0 = exp(-mu), p_j = (p_{j-1} mu)/j; thr_31 = 2^32. */
int jd_poisson_thresholds(double mu, uint64_t* thr);

#ifdef __cplusplus
}
#endif

#endif /* JD_H */
