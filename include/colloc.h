/*
 * colloc.h -- C ABI of the MI355X collocation interior-point Newton step.
 *
 * The library evaluates and differentiates the simultaneous-method NLP of an ODE
 * parameter-estimation problem (problem statement eq. 1a-1d; discretized NLP eq. 2a-2e with
 * the collocation equation in the form of eq. 3), assembles the condensed primal-dual KKT
 * matrix W + Sx + dw I + J^T Ds J, factors it without pivoting, solves it, and runs the
 * filter line-search interior-point iteration around it (the solver stack in the benchmark
 * setup: a filter line-search interior-point method on a pivoting-free KKT form, relative
 * KKT tolerance 1e-6, acceptable level 1e-4 over 15 iterations).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A problem handle is a batch of n_inst >= 1 instances with the same shape class
 *    (n_s species, n_r reactions, n_p parameters, K collocation points); the number of finite
 *    elements N and the reaction network may differ per instance.
 *  - Right-Radau collocation points (last point at tau = 1), so continuity (eq. 2c) links
 *    node K of element i-1 to node 0 of element i.
 *  - Vector layouts (per instance, instances stored back to back in handle order):
 *      x (primal, length N*b + n_p, b = (K+1) n_s):  z[i][j][s] at i*b + j*n_s + s, then theta.
 *      g, y, s, v (constraints, length N*b):  row (i, j, s) at i*b + j*n_s + s, where j = 0 is
 *        the initial-condition row (i = 0, eq. 2d) or the continuity row (i >= 1, eq. 2c), and
 *        j = k >= 1 is the collocation row at point k (eq. 2b / eq. 3), written as
 *        sum_j a_jk z_ij - h_i f(z_ik, theta), the sign used by the paper's constraint listing.
 *    colloc_layout() returns the per-instance offsets.
 *  - Objective: Phi = 1/2 sum_m ((sum_j l_j(tau_m) z[e_m][j][s_m] - y_m) / sigma_m)^2.
 *  - Mass-action kinetics: f_s = sum_r nu_sr rho_r, rho_r = kappa_r prod_(filled slots) u,
 *    kappa_r = exp(theta[param_r]) or exp(logk_fixed_r) when param_r = -1.
 *  - Pointers named *_dev are device memory (hipMalloc or torch CUDA tensors) owned by the
 *    caller; the library never allocates device memory after colloc_create.  Host pointers
 *    are only read during the call.
 *  - All device work is enqueued asynchronously on the given stream; no call synchronizes
 *    except colloc_create/colloc_upload.  A handle must not be used from two threads at once.
 *  - Argument and shape errors are detected on the host before anything is enqueued and
 *    return a negative COLLOC_E* code; numerical outcomes are reported per instance in
 *    device status words.  A failed kernel launch returns COLLOC_EHIP.
 */
#ifndef COLLOC_H
#define COLLOC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Host return codes. */
enum {
  COLLOC_OK = 0,
  COLLOC_EINVAL = -1,      /* bad argument, shape or pointer */
  COLLOC_ENOMEM = -2,      /* host allocation failed */
  COLLOC_EHIP = -3,        /* a HIP call or kernel launch failed */
  COLLOC_EUNSUPPORTED = -4 /* shape class outside what the kernels support (see colloc_create) */
};

/* Per-instance device status of the interior-point iteration (the paper's solve statuses,
 * Table 1 keys: solve succeeded, solved to acceptable level, timeout/iteration cap,
 * restoration failed, error). */
enum {
  COLLOC_RUNNING = 0,
  COLLOC_SOLVED = 1,
  COLLOC_ACCEPTABLE = 2,
  COLLOC_MAXITER = 3,
  COLLOC_TIMEOUT = 4,
  COLLOC_ENOTPD = 5,              /* inertia correction exceeded delta_max */
  COLLOC_ENONFINITE = 6,          /* NaN/Inf in the optimality error */
  COLLOC_RESTORATION_REQUIRED = 7, /* line search reached alpha_min (no restoration phase) */
  COLLOC_EFILTER = 8              /* the filter's COLLOC_FILTER_CAP entries were all taken */
};

/* Factor precision of kkt_factor / ipm_step. */
enum {
  COLLOC_FP64 = 0,    /* FP64 block factors */
  COLLOC_FP32_IR = 1  /* FP32 block factors, FP64 parameter Schur complement, FP64 refinement */
};

/* One estimation instance (eq. 1 with mass-action right-hand side).  Host pointers, copied by
 * colloc_create.  react/prod hold two species slots per reaction (-1 = empty slot; a
 * bimolecular 2A reaction lists A twice); nu_sr = (count of s in prod) - (count in react). */
typedef struct colloc_instance_desc {
  int32_t n_s, n_r, n_p, N;
  const int32_t* react;       /* [n_r][2] */
  const int32_t* prod;        /* [n_r][2] */
  const int32_t* param;       /* [n_r], index into theta or -1 (rate fixed) */
  const double* logk_fixed;   /* [n_r], natural-log rate where param == -1 */
  const double* h;            /* [N] element widths, > 0 */
  const double* z0;           /* [n_s] initial state (eq. 2d) */
  int32_t n_meas;
  const int32_t* meas_elem;   /* [n_meas] element index in [0, N) */
  const int32_t* meas_species;/* [n_meas] */
  const double* meas_tau;     /* [n_meas] local time in [0, 1] inside the element */
  const double* meas_y;       /* [n_meas] observed value */
  const double* meas_sigma;   /* [n_meas] noise scale, > 0 */
  const double* theta_lo;     /* [n_p] bounds (eq. 1a), theta_lo < theta_hi */
  const double* theta_hi;     /* [n_p] */
} colloc_instance_desc;

/* Interior-point options (defaults from colloc_ipm_default_opts). */
typedef struct colloc_ipm_opts {
  double tol, acceptable_tol;  /* 1e-6, 1e-4 */
  int32_t acceptable_iter;     /* 15 consecutive acceptable iterations */
  int32_t max_iter;            /* 3000 */
  double mu_init;              /* 0.1 */
  double tau_r;                /* equality relaxation half-width, 1e-8 */
  double kappa_eps, kappa_mu, theta_mu, tau_min, kappa_sigma, s_max;
  double bound_push, bound_frac;
  double delta_w0, delta_min, delta_max, kappa_w_minus, kappa_w_plus, kappa_w_plus_bar;
  double gamma_theta, gamma_phi, s_theta, s_phi, eta_phi, delta_sw, gamma_alpha;
  int32_t max_ls;              /* backtracking trials per iteration, <= COLLOC_MAX_LS */
  int32_t precision;           /* COLLOC_FP64 or COLLOC_FP32_IR */
  int32_t ir_max;              /* refinement sweeps in FP32_IR mode (default 10) */
  int32_t pad_;
  double ir_tol;               /* normwise backward-error target of the refinement (1e-14), see
                                  kkt_solve */
  double max_wall_s;           /* wall-clock limit per instance in seconds from ipm_init, read
                                  from the device clock at each iteration's decision; 0 = none
                                  (default).  Exceeding it ends the instance with COLLOC_TIMEOUT */
} colloc_ipm_opts;

#define COLLOC_MAX_LS 48
#define COLLOC_FILTER_CAP 128

/* Per-instance iteration record, device-resident inside the state buffer. */
typedef struct colloc_ipm_info {
  int32_t status, iter, phase, ls_trials;
  int32_t factor_tries, acc_count, filter_len, ir_sweeps;
  double mu, tau, delta_w, delta_last;
  double alpha_pr, alpha_du, obj, inf_pr;
  double inf_du, E0, theta_cv, phi;
  double theta_max, theta_min, dphi, alpha_min;
  double Emu, s_d, s_c;
  int32_t ir_fallbacks, pad_;  /* FP32_IR: iterations factored in FP64 (after the first
                                * fallback an instance stays on FP64 factors) */
  double t_start;              /* device wall clock at ipm_init, seconds */
} colloc_ipm_info;

/* Sizes and per-instance offsets of a handle (host arrays owned by the handle). */
typedef struct colloc_layout {
  int32_t n_inst, n_s, n_r, n_p, K, b;
  int64_t n_elem;            /* total elements over the batch */
  int64_t n_total;           /* total primal length */
  int64_t m_total;           /* total constraint length */
  int64_t jac_len, hess_len; /* lengths (doubles) of the derivative value arrays */
  const int64_t* x_off;      /* [n_inst] start of instance in x */
  const int64_t* g_off;      /* [n_inst] start of instance in g/y/s */
  const int64_t* elem_off;   /* [n_inst] first global element of the instance */
  const int32_t* N;          /* [n_inst] */
} colloc_layout;

typedef struct colloc_problem colloc_problem; /* opaque host handle */

/* Validate a batch and build its host tables (collocation weights l_j'(tau_k) of eq. 3,
 * continuity weights, measurement interpolation weights, work lists).  K in [1, 5].
 * Returns COLLOC_EUNSUPPORTED for shapes beyond the kernels' LDS budget.  Host only. */
int colloc_create(const colloc_instance_desc* inst, int32_t n_inst, int32_t K,
                  colloc_problem** out);
int colloc_destroy(colloc_problem* p);
int colloc_layout_get(const colloc_problem* p, colloc_layout* out);

/* Device table bytes; colloc_upload copies the tables into caller memory of that size
 * (256-byte aligned) and synchronizes the stream.  Must precede every device call. */
size_t colloc_table_bytes(const colloc_problem* p);
int colloc_upload(colloc_problem* p, void* table_dev, hipStream_t stream);

/* Workspace for colloc_eval/kkt_assemble/kkt_factor/kkt_solve/kkt_matvec/ipm_step (KKT blocks,
 * factors, solve vectors, reduction partials) and the interior-point state buffer.  Every call
 * that touches factor blocks takes the precision explicitly.  The FP32_IR size equals the FP64
 * size: an interior-point iteration whose FP32 factor fails or whose refinement does not
 * converge re-factors that instance in FP64 in the same workspace. */
size_t colloc_workspace_bytes(const colloc_problem* p, int32_t precision);
size_t colloc_state_bytes(const colloc_problem* p);

/* a1 -- pattern values (eq. 2a-2d): obj[n_inst] = Phi per instance, g[m_total].
 * x_dev: primal point.  Deterministic (fixed reduction order). */
int colloc_eval(const colloc_problem* p, const double* x_dev, double* obj_dev, double* g_dev,
                void* ws_dev, hipStream_t stream);

/* colloc_eval without a workspace, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same inputs and
 * outputs as colloc_eval, bitwise the same results.  The per-element partial objective sums live
 * in a library-owned static device array of COLLOC_NOALLOC_SCRATCH_DOUBLES doubles per GPU
 * (4 MiB, held until the process ends), so the call handles at most
 * COLLOC_NOALLOC_MAX_ELEMS finite elements over the batch; larger handles return COLLOC_EINVAL
 * before anything is enqueued.  The call allocates nothing.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams or threads) race and must be
 * serialized by the caller.  Nothing in the array needs clearing: each call writes every entry
 * it reads. */
#define COLLOC_NOALLOC_SCRATCH_DOUBLES (1 << 19)
#define COLLOC_NOALLOC_MAX_ELEMS (COLLOC_NOALLOC_SCRATCH_DOUBLES / 13)
int colloc_eval_noalloc(const colloc_problem* p, const double* x_dev, double* obj_dev,
                        double* g_dev, hipStream_t stream);

/* a2 -- derivatives of every expression pattern (the paper's per-pattern parallel AD):
 *   grad[n_total]  = grad Phi
 *   jac[jac_len]   = per (element i, collocation point k=1..K, reaction r), three values
 *                    (d rho_r/d slot0, d rho_r/d slot1, d rho_r/d theta) at z[i][k]; the
 *                    constraint Jacobian is sum_j a_jk I - h_i nu (these), plus the constant
 *                    continuity/initial rows.  Index ((e*K + k-1)*n_r + r)*3 + t, e global.
 *   hess[hess_len] = per (e, k, r), w_ikr * (d2rho/dslot0 dslot1, d2rho/dslot0 dtheta,
 *                    d2rho/dslot1 dtheta, d2rho/dtheta2) with w_ikr = -h_i sum_s y[i][k][s] nu_sr,
 *                    the weight of rho_r in y^T g.  Index ((e*K + k-1)*n_r + r)*4 + t.
 *   The objective's Hessian is constant and applied inside kkt_assemble. */
int colloc_derivs(const colloc_problem* p, const double* x_dev, const double* y_dev,
                  double* grad_dev, double* jac_dev, double* hess_dev, hipStream_t stream);

/* a3 -- condensed KKT assembly: K = W + Sx + dw I + J^T (Ss + dw I) J into the workspace
 * block storage, and rhs = -r_x - J^T ((Ss + dw) r_y + r_s) (relaxed-equality primal-dual
 * system; W = Hessian of Phi + y^T g from hess and the measurement weights).
 *   sigma_x[n_inst*n_p] (theta entries), sigma_s[m_total], delta_w[n_inst] (device),
 *   r_x[n_total], r_s[m_total], r_y[m_total], rhs[n_total] output.  precision selects the
 *   block storage (must match the following kkt_factor). */
int kkt_assemble(const colloc_problem* p, const double* jac_dev, const double* hess_dev,
                 const double* sigma_x_dev, const double* sigma_s_dev, const double* delta_w_dev,
                 const double* r_x_dev, const double* r_s_dev, const double* r_y_dev,
                 void* ws_dev, int32_t precision, double* rhs_dev, hipStream_t stream);

/* a4 -- pivoting-free factorization of the assembled matrix: per-element static condensation
 * of the interior collocation points, cyclic reduction of the separator chain (element-end
 * states) level by level, then the dense parameter Schur complement.  info[n_inst] (device):
 * 0 = positive definite, 1 = a non-positive or non-finite pivot was met. */
int kkt_factor(const colloc_problem* p, void* ws_dev, int32_t precision, int32_t* info_dev,
               hipStream_t stream);

/* a5 -- solve K dx = rhs with the factor (forward through the elimination levels, parameter
 * block, back substitution).  With ir_max > 0, up to ir_max refinement sweeps follow: the
 * residual r = rhs - K dx is formed matrix-free in FP64 from the derivative values, Ds, Sx and
 * dw of the last assembly (kkt_matvec), the correction d solves with the same factor and
 * dx += d.  An instance converges once the dx its residual was taken at has normwise backward
 * error ||r||_inf <= ir_tol (||K||_inf ||dx||_inf + ||rhs||_inf), ||K||_inf bounded above by the
 * largest row sum of |J|^T Ds |J| + |W| + the diagonal terms (formed once per call); it fails
 * when ir_max sweeps are spent or a correction is more than half the previous one (the factor
 * no longer contracts the error).
 * ir_sweeps[n_inst] (device, may be NULL): the sweeps taken by a converged instance, minus the
 * sweeps taken by a failed one, 0 without refinement or where the factor failed.  Refinement is
 * what makes COLLOC_FP32_IR factors reach FP64 accuracy; in ipm_step a failed refinement makes
 * the instance re-factor in FP64 (counted in ir_fallbacks). */
int kkt_solve(const colloc_problem* p, void* ws_dev, int32_t precision, const double* rhs_dev,
              double* dx_dev, int32_t ir_max, double ir_tol, int32_t* ir_sweeps_dev,
              hipStream_t stream);

/* out = K v with the assembled matrix, evaluated matrix-free in FP64 from the derivative
 * values, Ds, Sx and dw stored by the last kkt_assemble or ipm_step (the residual of the
 * refinement).  v and out must not alias. */
int kkt_matvec(const colloc_problem* p, void* ws_dev, const double* v_dev, double* out_dev,
               hipStream_t stream);

/* Collocation-consistent starting states (forward implicit Runge-Kutta sweep at fixed
 * parameters; the paper's initial state guesses come from a forward solve at the nominal
 * parameters, numerical-results section, benchmark setup).  For every instance, element by element
 * in mesh order, the K stage values solve the collocation equations of eq. 2b / eq. 3 at
 * theta from the element's first node (z0, eq. 2d; then the previous element's last node,
 * eq. 2c) by Newton's method with the dense K n_s x K n_s Jacobian, factored on chip.
 * theta_dev [n_inst][n_p] (device): the parameters; x_dev [n_total] (device, written): every
 * instance's [z | theta], ready for ipm_init.  status_dev [n_inst] (device, written): 0, or
 * 1 + the first element whose Newton iteration did not converge (its values are the last
 * iterate).  Allocates nothing.  COLLOC_EUNSUPPORTED when K n_s > 96 (the Newton system must
 * fit in LDS). */
int colloc_forward_init(const colloc_problem* p, const double* theta_dev, double* x_dev,
                        int32_t* status_dev, hipStream_t stream);

/* a6 -- interior-point iteration.  ipm_init pushes theta into its bounds, sets the slacks,
 * multipliers, mu and filter (state buffer of colloc_state_bytes).  ipm_step performs one
 * iteration for every running instance: evaluate, test convergence, update mu, assemble and
 * factor (an indefinite matrix makes the step a retry with a larger delta_w), solve, fraction
 * to the boundary, filter line search over the backtracking candidates, update.  Finished
 * instances are left unchanged. */
void colloc_ipm_default_opts(colloc_ipm_opts* o);
int ipm_init(const colloc_problem* p, const double* x0_dev, void* state_dev, void* ws_dev,
             const colloc_ipm_opts* opts, hipStream_t stream);
int ipm_step(const colloc_problem* p, void* state_dev, void* ws_dev, const colloc_ipm_opts* opts,
             hipStream_t stream);

/* Graph-captured interior-point iterations (batched instances run as one replayed graph per
 * step instead of one launch per kernel).  ipm_graph_create captures `steps` consecutive
 * ipm_step calls on (state, ws, opts) by stream capture on `stream` (not the null stream) and
 * instantiates the graph; nothing is executed during capture.  ipm_graph_launch replays them:
 * each replay performs exactly what `steps` ipm_step calls would.  The graph is bound to the
 * given buffers and options; phase timing is not recorded inside it.  Host-only errors:
 * COLLOC_EINVAL, COLLOC_EHIP when capture or instantiation fails. */
typedef struct colloc_graph colloc_graph;
int ipm_graph_create(const colloc_problem* p, void* state_dev, void* ws_dev,
                     const colloc_ipm_opts* opts, int32_t steps, hipStream_t stream,
                     colloc_graph** out);
int ipm_graph_launch(colloc_graph* g, hipStream_t stream);
int ipm_graph_destroy(colloc_graph* g);

/* Byte offsets of the state buffer's fields: x[n_total], s, y, vL, vU [m_total], zL, zU
 * [n_inst*n_p], dx[n_total], ds, dy [m_total], info[n_inst] (colloc_ipm_info), and the filter
 * entries fth, fph [n_inst][COLLOC_FILTER_CAP].  An instance's iterate between two ipm_step
 * calls (status RUNNING with no pending inertia retry, or finished) is its segments of x, s, y,
 * vL, vU, zL, zU, fth, fph and its info record: copying them into another state buffer moves
 * the instance to another batch (continuous batching). */
typedef struct colloc_state_layout {
  size_t x, s, y, vL, vU, zL, zU, dx, ds, dy, info, fth, fph;
} colloc_state_layout;
int colloc_state_layout_get(const colloc_problem* p, colloc_state_layout* out);

/* Per-phase timing with HIP events recorded on the call's stream around each phase launch:
 * enable, then read accumulated milliseconds and launch counts per phase.  LEVEL0 is the element
 * condensation (with the fused assembly on the register path); on the tiled path ASSEMBLY is the
 * element assembly, LEVEL0 the interior-column panel factorization and SCHUR the element Schur
 * complement tiles. */
enum {
  COLLOC_PH_EVAL = 0, COLLOC_PH_LEVEL0 = 1, COLLOC_PH_CR = 2, COLLOC_PH_BORDER = 3,
  COLLOC_PH_SOLVE = 4, COLLOC_PH_STEP = 5, COLLOC_PH_LINESEARCH = 6, COLLOC_PH_ASSEMBLY = 7,
  COLLOC_PH_SCHUR = 8, COLLOC_N_PHASES = 9
};
int colloc_timing_enable(colloc_problem* p, int32_t enable);
int colloc_timing_read(colloc_problem* p, double* ms, int64_t* launches, int32_t n);

/* Thread-grid choice of the register-resident elimination kernels (the tuning hook of
 * paper_2607_12201_amd.autotune).  which: 0 = element (level-0) kernel, 1 = separator-chain
 * kernel, 2 = border kernel.  A kernel runs on a TS x TS thread grid holding its matrix in
 * registers, ceil(rows / TS) blocks per side.  colloc_tile_options writes the usable TS for this
 * handle's shape into ts[0..cap) and returns their count (negative on bad arguments);
 * colloc_tile_set selects one (0 = built-in rule) and returns COLLOC_EINVAL for a TS the shape
 * cannot use; colloc_tile_get returns the current choice (0 = built-in rule).  For the chain
 * kernel TS = 1 selects its blocked LDS variant (FP64 factors only), whose
 * arithmetic differs from the register-resident one in rounding only.  Among the TS x TS grids the
 * choice changes which thread computes an entry, not the arithmetic: results are identical. */
int colloc_tile_options(const colloc_problem* p, int32_t which, int32_t* ts, int32_t cap);
int colloc_tile_set(colloc_problem* p, int32_t which, int32_t ts);
int colloc_tile_get(const colloc_problem* p, int32_t which);

/* Collocation tables computed by the library (tau[K+1], a[(K+1)*(K+1)] with a[j*(K+1)+k] =
 * l_j'(tau_k)), for inspection. */
int colloc_tables(int32_t K, double* tau, double* a);

#ifdef __cplusplus
}
#endif
#endif /* COLLOC_H */
