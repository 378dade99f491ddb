/*
 * jd_feedback.h -- C ABI of libjd for the paper's own model problem
 * (Bartsch, Borzi, Ciaramella, Reichle, arXiv 2505.04328, Section 5 model
 * equation, shape functions and jump process; Section 6): one particle
 * z = (x, v) per path in a harmonic oscillator with Brownian noise and
 * Keilson-Storer velocity jumps, steered by a feedback control built from
 * radial-basis shape functions, with a Gaussian tracking cost.
 *
 *   centres   x^i = (i + 1/2) 2 xmax/nx - xmax,  v^l = (l + 1/2) 2 vmax/nv - vmax
 *             (0-based i, l; the cell centres of Section 5, discretization)
 *   bump      b(r) = exp(-1/(1 - (eps r)^2)) for |r| < 1/eps, else 0 (eq. Gaussian_RBF)
 *   control   u_k = sum_{i,l} mu_k[i nv + l] b(x_k - x^i) b(v_k - v^l)  (eq. control_structure)
 *   forward   (eq. SDE_splitted_drift_Euler, h = 0, on the fixed grid t_k = k dt)
 *             x_{k+1} = x_k + dt v_k + b1 sqrt(dt) Zx_k
 *             v*      = v_k + dt (u_k - eta x_k) + b2 sqrt(dt) Zv_k
 *             v_{k+1} = gamma^n v* + sqrt(V_n) ZJ_k,  V_n = (1/(2 beta)) sum_{i<n} gamma^{2i}
 *             n = n_k ~ Poisson(sqrt(beta/pi) dt): the step's Keilson-Storer jumps
 *             v <- gamma v + N(0, 1/(2 beta)) (eq. jump_law, eq. collision_frequency),
 *             composed exactly after the step's Euler update
 *   cost      C = dt sum_{k=1..N} Jt(z_k, zd_k) + dt alpha/2 sum_{k=0..N-1} u_k^2,
 *             Jt(z, zd) = -exp(-|z - zd|^2/(2 sigJ^2))  (eq. discrete_functional,
 *             eq. tracking_cost);  J = (1/M) sum_m C^m
 *   adjoint   lam = dC/dz = -r (eq. adjoint_eq_approximation, jump condition p <- gamma p):
 *             lam_N   = dt grad Jt(z_N)
 *             lam^x_k = lam^x_{k+1} + gamma^n dt (u_x - eta) lam^v_{k+1} + dt dJt/dx + dt alpha u u_x
 *             lam^v_k = dt lam^x_{k+1} + gamma^n (1 + dt u_v) lam^v_{k+1} + dt dJt/dv + dt alpha u u_v
 *   gradient  g_k[i nv + l] = (1/M) sum_m b(x_k - x^i) b(v_k - v^l) (alpha u_k + gamma^{n_k} lam^v_{k+1})
 *             (eq. definition_Gradient; dJ/dmu_k = dt g_k)
 *
 * Draws (counter-based, like jd.h): Philox4x32-10 block (m, k, iter, 0) per
 * path-step; the Box-Muller pair of words 0 and 1 gives Zx (cosine) and Zv
 * (sine), the cosine branch of words 2 and 3 gives ZJ, the low bytes of the
 * four words the Poisson word.  The initial state uses block
 * (m, 0xFFFFFFFF, iter, 0): Gaussian z0 + s0 (R cos, R sin) of words 0 and 1,
 * or uniform z0 + s0 (2 u - 1) (fresh initial particles every iteration,
 * Section 5, optimization procedure).
 *
 * Coupled particles (Section 6.4, eq. interacting_model): with np > 1 the
 * M = run->M realizations are rings of np particles (particle j of ring r is
 * particle p = r np + j, which draws with counter word 0 = p); the velocity
 * update of particle j gains the nearest-neighbour force
 *   v* = ... + dt (u_k - eta x_k - omega (2 x_{j,k} - x_{j-1,k} - x_{j+1,k}))
 * (indices mod np), the adjoint passes w_i = gamma^{n_i} lam^v_{i,k+1} back to
 * the neighbours,
 *   lam^x_{j,k} += dt omega (w_{j-1} + w_{j+1} - 2 w_j),
 * and J and g are means over all M np particles.  Ellipse cost (cost_kind =
 * JD_FB_COST_ELLIPSE, eq. phonon_functional_tracking): Jt(z) =
 * -exp(-q^2/(2 sigJ^2)), q = x^2/ax^2 + v^2/av^2 - 1.  Ellipse start
 * (JD_FB_INIT_ELLIPSE, eq. coupled_ellipse): particle j of its ring at
 * (ax cos th_j, av sin th_j) + s0 . (Z1, Z2), th_j = 2 pi j / np, (Z1, Z2) the
 * Gaussian pair of the initial-state block.  One ring runs inside one
 * workgroup, its neighbours exchanged through LDS.
 *
 * Jump-adapted grid (grid = JD_FB_GRID_ADAPTED; Section 3 and Algorithms
 * 5.1-5.2; independent particles, JD_STORE): each particle's grid is the
 * uniform points t_k plus its jump times.  Interval k holds the n jumps
 * counted by Philox block (m, k, iter, 0) (the count above), at offsets
 * a_1 < ... < a_n (units of dt) drawn as successive minima of uniforms,
 *   a_r = a_{r-1} + (1 - a_{r-1}) (1 - V_r^{1/(n-r+1)}),  a_0 = 0, a_{n+1} = 1,
 * V_r = word (r-1) mod 4 of block (m, k, iter, 64 + (r-1)/4) (a Poisson process
 * on the interval).  Sub-step r spans [a_r, a_{r+1}] dt (length d_r) with the
 * Box-Muller pair of words 0, 1 of block (m, k, iter, r) and the control mu_k;
 * sub-step r < n ends at jump r+1: v <- gamma v + S / sqrt(2 beta), S the
 * cosine normal of words 2, 3 of block (m, k, iter, r+1).  The cost is
 *   C = sum over sub-steps d_r (Jt(z_end, zd(t_end)) + alpha/2 u_r^2)
 * (z_end post-jump; zd linear between the uniform targets), the adjoint its
 * exact transpose (lam^v <- gamma lam^v across a jump), and
 *   g_k[l] = (1/M) sum_m sum_r (d_r/dt) phi_l(z_r) (alpha u_r + lam^v_-(end of r)).
 * The trajectory, dumps and lam rows hold the uniform points; with no jumps
 * the model is the fixed-grid one.
 *
 * Surrogate gradient (run->mode = JD_SURROGATE; Section 6.5, the adjoint
 * independent of the forward trajectories): nothing is stored.  The forward
 * adds alpha u_k phi(z_k) to the gradient as it goes; the adjoint recursion
 * above runs on surrogate states zs_k = zd_k + sqrt(svar0 + svar1 t_k) . (Z1, Z2)
 * with one sample (Z1, Z2) per particle and realization (Box-Muller pair of
 * words 0, 1 of Philox block (m, 0xFFFFFFFE, iter, 1), the same at every
 * step) and the forward's jump counts, and adds gamma^{n_k} ls^v_{k+1} phi(zs_k).  J is the
 * exact cost.  The gradient is biased (it is not the derivative of J).  The
 * variance is max(0, a + b t) per component: with svar_kind JD_FB_SVAR_GIVEN
 * the line a = svar0, b = svar1; with JD_FB_SVAR_FIT the ordinary
 * least-squares line through the points (t_k, V_k), k = 0..N, where V_k is
 * the population variance over the M particles of the forward sweep's own
 * z_k (same mu and draws), so that the surrogate variance follows the forward
 * model's (the forward sums z_k - zd_k and its square per step in FP64; a
 * short reduction and the fit run between the two sweeps).
 *
 * Conventions are those of jd.h (return codes, caller-owned device buffers,
 * asynchronous calls on `stream`, validation before any launch).  mu and g
 * are FP64 device arrays, row-major N x L with L = nx nv.  Modes: JD_STORE
 * (exact gradient over the stored trajectory) and JD_SURROGATE (jd_fb_forward,
 * jd_fb_cost_grad, jd_fb_optimize; traj may be NULL; independent particles
 * only, np = 1, else JD_EUNSUPPORTED); JD_RECOMPUTE returns JD_EUNSUPPORTED.
 * Particle indices (dumps, jd_fb_draws) count M np particles; M np < 2^32.
 */
#ifndef JD_FEEDBACK_H
#define JD_FEEDBACK_H

#include "jd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define JD_FB_INIT_GAUSS 0   /* z_0 = z0 + s0 . (Z1, Z2) */
#define JD_FB_INIT_UNIFORM 1 /* z_0 uniform on [z0 - s0, z0 + s0] */
#define JD_FB_INIT_ELLIPSE 2 /* z_0 = ring position on the ellipse + s0 . (Z1, Z2) */

#define JD_FB_COST_TRACK 0   /* tracking cost around zd */
#define JD_FB_COST_ELLIPSE 1 /* ellipse cost with half-axes ax, av */

#define JD_FB_MAX_RING 2048  /* largest np: one ring per workgroup */

#define JD_FB_GRID_FIXED 0   /* fixed grid, Poisson jump counts composed per step */
#define JD_FB_GRID_ADAPTED 1 /* jump-adapted grid: uniform points plus jump times */

#define JD_FB_SVAR_GIVEN 0   /* surrogate variance svar0 + svar1 t */
#define JD_FB_SVAR_FIT 1     /* surrogate variance fitted to the forward ensemble */

typedef struct jd_fb_problem {
    int32_t N;          /* time steps, >= 1 */
    int32_t nx, nv;     /* shape-function grid, 1..16 each; L = nx nv */
    double T;           /* horizon, > 0 */
    double eta;         /* oscillator stiffness (H = [[0, 1], [-eta, 0]]) */
    double b1, b2;      /* noise scales of x and v, >= 0 */
    double gamma;       /* Keilson-Storer gamma in [-1, 1] */
    double beta;        /* Keilson-Storer beta > 0; jump rate sqrt(beta/pi), rate*dt <= 2 */
    double xmax, vmax;  /* shape-function domain (-xmax, xmax) x (-vmax, vmax), > 0 */
    double eps;         /* bump shape parameter, > 0 */
    double alpha;       /* control-cost weight, >= 0 */
    double sigJ;        /* tracking-cost width, > 0 */
    int32_t init_kind;  /* JD_FB_INIT_GAUSS or JD_FB_INIT_UNIFORM */
    double z0[2], s0[2];/* initial law: centre and scale (s0 >= 0) */
    double svar0[2], svar1[2]; /* surrogate-state variance svar0 + svar1 t (>= 0), JD_SURROGATE
                                  with JD_FB_SVAR_GIVEN (ignored with JD_FB_SVAR_FIT) */
    const double* zd;   /* DEVICE, (N+1) x 2 FP64: desired (x, v) at t_0..t_N; may be
                           NULL with the ellipse cost outside JD_SURROGATE */
    int32_t np;         /* particles per ring, 1..JD_FB_MAX_RING (1: independent particles) */
    double omega;       /* nearest-neighbour coupling (finite) */
    int32_t cost_kind;  /* JD_FB_COST_TRACK or JD_FB_COST_ELLIPSE */
    double ax, av;      /* ellipse half-axes, > 0 (ellipse cost or start) */
    int32_t grid;       /* JD_FB_GRID_FIXED or JD_FB_GRID_ADAPTED (np = 1, JD_STORE) */
    int32_t svar_kind;  /* JD_FB_SVAR_GIVEN or JD_FB_SVAR_FIT (JD_SURROGATE) */
} jd_fb_problem;

/* Per-path diagnostics for the feedback model, as jd_dump with these layouts
 * (DEVICE pointers, run precision for z and lam):
 *   X[(k*2 + c)*count + p]   = z_k,c of path m0+p, k = 0..N   (jd_fb_forward)
 *   lam[(k*2 + c)*count + p] = lam_k,c,                k = 1..N (jd_fb_adjoint)
 *   cost[p]                  = C^(m0+p), FP64                  (jd_fb_forward) */

/* Workspace and trajectory bytes (0 if the arguments are invalid).  The
 * trajectory holds z_0..z_N in rows of 256 slots: component c of z_k of the
 * particle in slot s is element ((s / 256) (N+1) + k) 2 256 + c 256 + (s % 256).
 * With np = 1 particle m sits in slot m.  With np > 1 a workgroup holds
 * R = floor(256 G / np) rings in 256 G slots (G = 1 for np <= 256, else 8):
 * particle j of ring r sits in slot (r / R) 256 G + (r % R) np + j.  On the
 * fixed grid the buffer continues with one byte per slot and step, the jump
 * count n_k of step k = 0..N-1 of slot s at byte
 * B + ((s / 256) N + k) 256 + (s % 256), B the byte length of the states;
 * jd_fb_forward writes them and jd_fb_adjoint reads them instead of
 * regenerating the draws.  On the jump-adapted grid the buffer continues with
 * the states after each of a slot's first 32 jumps and the jump times (entry e
 * of slot s, component c = 0, 1 for x, v and 2 for the jump's offset in its
 * interval in units of dt: element T + ((s / 256) 32 + e) 3 256 + c 256 +
 * (s % 256), T the trajectory's length), one int32 jump count per slot, and
 * then one byte per
 * slot and interval k, the interval's jump count (byte
 * C + ((s / 256) N + k) 256 + (s % 256), C where the int32 counts end), all
 * of which the adjoint reads. */
size_t jd_fb_workspace_bytes(const jd_fb_problem* prob, const jd_run* run);
size_t jd_fb_traj_bytes(const jd_fb_problem* prob, const jd_run* run);

/* Forward sweep (Algorithms 5.1-5.2 on the fixed grid) of all M particles:
 * stores the trajectory (traj may be NULL for a cost-only sweep) and J(mu)
 * into *J (device FP64).  mu: device FP64 N x L. */
int jd_fb_forward(const jd_fb_problem* prob, const jd_run* run, const double* mu, void* traj,
                  double* J, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward adjoint sweep over the trajectory of jd_fb_forward (same prob,
 * run, mu) and the Monte Carlo gradient g (device FP64 N x L, no dt factor);
 * JD_STORE only (JD_SURROGATE: JD_EUNSUPPORTED, use jd_fb_cost_grad).
 * The per-step sum over particles of phi(z) (alpha u + gamma^n lam^v) is a
 * dense 16 x 16 contraction over paths and runs on the matrix cores (FP64, or
 * FP32 products with FP64 sums beyond one wave's step for FP32 paths). */
int jd_fb_adjoint(const jd_fb_problem* prob, const jd_run* run, const double* mu,
                  const void* traj, double* grad, void* ws, size_t ws_bytes, hipStream_t stream);

/* Forward + adjoint + reductions (Algorithm 5.3): J -> *J, g -> grad (the
 * surrogate gradient under JD_SURROGATE, where traj may be NULL). */
int jd_fb_cost_grad(const jd_fb_problem* prob, const jd_run* run, const double* mu, double* J,
                    double* grad, void* traj, void* ws, size_t ws_bytes, hipStream_t stream);

/* Gradient iteration (Algorithm 5.4 with eq. Stochastic_Armijo), exactly as
 * jd_optimize (the line search decided on the device, one synchronization per
 * batch of up to 64 iterations, a trial whose cost overflows rejected):
 * iteration n uses counter word run->iter + n for the gradient and every
 * trial; mu (device FP64 N x L) is updated in place. */
int jd_fb_optimize(const jd_fb_problem* prob, const jd_run* run, const jd_opt* opt, double* mu,
                   jd_iter_log* log, int32_t* iters_done, void* traj, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* The draws of paths [m0, m0+mc): initial states z_init (mc x 2) and, for steps
 * [k0, k0+kc), the normals Z ((p kc + q) 3 + {0: Zx, 1: Zv, 2: ZJ}) and jump
 * counts counts[p kc + q] (device buffers, run precision for z_init and Z,
 * each may be NULL), for checking the draws against an independent
 * implementation. */
int jd_fb_draws(const jd_fb_problem* prob, const jd_run* run, int64_t m0, int64_t mc, int32_t k0,
                int32_t kc, void* z_init, void* Z, int32_t* counts, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif
