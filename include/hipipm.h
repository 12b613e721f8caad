/*
 * hipipm -- batched primal-dual interior-point NLP solver for one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libhipipm.so.  The library solves batches of the parametric NLP
 *     min_x f(x, theta)  s.t.  c(x, theta) = 0,  x_L <= x <= x_U           (Sec. III, eq. (1))
 * whose instances share f, c and the bounds and differ only in theta (eq. (2)), with the
 * IPOPT-style barrier method of Sec. IV: log-barrier subproblems (eq. (3)), Newton steps on
 * the augmented KKT system (eq. (7)) with inertia correction, fraction-to-the-boundary, a
 * backtracking filter line search with second-order correction, the tiny-step rule, hard
 * feasibility restoration and the monotone barrier update (Table I rows 1, 2, 4, 6, 7).
 * Finished instances are replaced by new ones at iteration boundaries (iteration-level
 * batching, Sec. V and Fig. 2); every instance takes its own branch inside the same launches.
 *
 * f, c and the bounds are compiled problem families (quadrotor multiple-shooting NMPC); the
 * caller supplies theta.  Decision vector layout (FP64), per instance:
 *     v = (x_0, u_0, x_1, u_1, ..., x_{N-1}, u_{N-1}, x_N, s)
 * with 13 states and 4 rotor thrusts per stage and s the inequality slacks ordered
 * (k = 1..N) x (row j).  Constraint / multiplier order:
 *     y = (x_0 - xbar0 [13], x_{k+1} - F(x_k, u_k) [13 each, k = 0..N-1], g_kj - s_kj).
 * Bounds: 0 <= u <= 2 u_hover, s >= 0; every other component is free.
 *
 * Conventions for every call:
 *   - return 0 on success, a negative HIPIPM_ERR_* code otherwise; no call aborts.
 *     hipipm_last_error() describes the last failure of a context.
 *   - "device pointer" arguments point to memory on the context's device that the caller
 *     owns and keeps alive for the duration of the call (and, for the workspace, until it
 *     is unbound or the context is destroyed).  The library never frees caller memory.
 *   - work is enqueued on the HIP stream passed as `stream` (a hipStream_t; NULL = the
 *     default stream) and the call returns when it has finished (hipipm_solve synchronizes
 *     the stream to poll its completion counter).
 *   - per-instance numerical failures are statuses (HIPIPM_STATUS_*), not call errors.
 */
#ifndef HIPIPM_H
#define HIPIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define HIPIPM_OK 0
#define HIPIPM_ERR_INVALID_ARG (-1)
#define HIPIPM_ERR_HIP (-2)
#define HIPIPM_ERR_UNSUPPORTED (-3)
#define HIPIPM_ERR_WORKSPACE (-4)

/* ---- per-instance status ---- */
#define HIPIPM_STATUS_RUNNING 0
#define HIPIPM_STATUS_CONVERGED 1       /* scaled KKT error E_0 <= tol */
#define HIPIPM_STATUS_MAX_ITER 2
#define HIPIPM_STATUS_RESTO_FAILED 3    /* restoration could not start or its line search failed */
#define HIPIPM_STATUS_INFEASIBLE 4      /* restoration converged to a point that is not feasible */
#define HIPIPM_STATUS_NUMERICAL 5       /* non-finite values in the iterate */

/* ---- problem families ---- */
#define HIPIPM_FAMILY_QUAD_OBS 0   /* point-to-point with spherical obstacles;
                                      theta = [xbar0 (13), target (3), n_obs x (cx, cy, cz, r)] */
#define HIPIPM_FAMILY_QUAD_TRACK 1 /* figure-eight tracking with spherical obstacles;
                                      theta = [xbar0 (13), A, omega, n_obs x (cx, cy, cz, r)] */
#define HIPIPM_FAMILY_QUAD_TRACK_MOVING 3 /* figure-eight tracking with spheres moving at constant
                                      velocity, trajectories known in advance (the tracking task
                                      with time-varying obstacles, Sec. VI);
                                      theta = [xbar0 (13), A, omega, n_obs x (cx, cy, cz, r, vx, vy, vz)],
                                      centre of sphere j at stage k: (cx, cy, cz) + k dt (vx, vy, vz) */

/* Problem descriptor (Sec. VI quadrotor NMPC; constants are inputs, not baked in). */
typedef struct {
    int32_t family;   /* HIPIPM_FAMILY_* */
    int32_t N;        /* shooting intervals, 1..64 */
    int32_t n_agents; /* must be 1 */
    int32_t n_obs;    /* spheres, 0..64 */
    double dt, mass, jxx, jyy, jzz, arm, ctau, grav;
    double q_weight, r_weight, d_min;
} hipipm_problem_desc;

/* Algorithm options.  hipipm_default_options() fills the published IPOPT defaults. */
typedef struct {
    double tol;
    int32_t max_iter;
    double mu_init, kappa_eps, kappa_mu, theta_mu, tau_min;
    double kappa1, kappa2, lam_max, s_max;
    double delta_min, delta_0, delta_max, delta_c_bar, kappa_c;
    double kappa_minus, kappa_plus, kappa_plus_bar;
    double gamma_theta, gamma_phi, delta_sw, s_theta, s_phi, eta_phi, gamma_alpha;
    int32_t max_soc;
    double kappa_soc, kappa_sigma, rho_resto, kappa_resto, bound_mult_reset;
    int32_t poll_every;   /* iterations between completion polls (>= 1) */
    int32_t timing;       /* 1: time every kernel launch with HIP events (hipipm_kernel_times) */
    int32_t fuse_below;   /* once at most this many instances are unfinished, each pass runs the
                             per-slot phases in one fused launch (0: never); default 2^30,
                             i.e. always */
    int32_t precision;    /* KKT factor and solve: 0 FP64 (default); 1 FP32 with FP64 iterative
                             refinement on the full system, FP64 refactorization when refinement
                             fails (runs every pass fused) */
    int32_t refine_max;   /* refinement sweeps per solve in precision 1 (default 3) */
    double refine_tol;    /* refinement stops when |b - K x|_inf <= refine_tol |b|_inf (default 1e-10) */
    double warm_mu0;      /* barrier parameter of a warm start (default 1e-3) */
    double warm_push;     /* bound push (kappa_1 = kappa_2) of a warm start (default 1e-3) */
    int32_t warm_iter_cap; /* a warm-started instance still running after this many iterations, or
                              entering restoration, restarts cold in its slot (0: only restoration) */
    int32_t warm_gate;    /* 1 (default): a warm point is kept only if its scaled error E_mu0 at
                             mu0 = warm_mu0 does not exceed that of the cold start (cold start with
                             least-squares y, z = 1), which costs the cold start's least-squares
                             pass; 0: every finite warm point is used */
    int32_t watchdog_trigger; /* watchdog (Table I row 3): after this many consecutive shortened
                             steps of the original problem (the first trial of the line search
                             rejected) the next steps are full steps (alpha_max) without the
                             line-search test; 0 (default): no watchdog */
    int32_t watchdog_max; /* full steps the watchdog takes (default 3): a step acceptable with respect
                             to the iterate where it started ends it as an ordinary acceptance; if
                             the last one is not, the iterate goes back to that point */
    int32_t soft_resto_max; /* soft feasibility restoration (Table I row 5): when the line search of the
                             original problem fails, take up to this many soft steps (primal-dual
                             Newton steps with one step size min(alpha_max primal, alpha_max dual),
                             accepted when they lower the primal-dual error by soft_resto_factor)
                             before hard restoration; 0 (default): straight to hard restoration */
    double soft_resto_factor; /* required reduction of the primal-dual error per soft step (0.9999) */
    int32_t mu_strategy;  /* barrier update (Table I row 7): 0 (default) monotone; 1 adaptive: mu from
                             the complementarity by the LOQO rule every iteration (free mode) while
                             the scaled KKT error keeps falling (E_0 <= 0.9999 x the largest of the
                             last four), otherwise the monotone rule from mu = 0.8 x the mean
                             complementarity until its barrier problem is solved with progress */
    int32_t async_passes; /* > 0: asynchronous slots -- each launch lets every slot run up to this many
                             whole passes back to back (its own derivatives included), refilling from
                             the device queue, with no wait for other slots between passes; the host
                             polls after each launch.  0 (default): one launch per phase or one fused
                             launch per pass, every slot advancing one pass per launch.  Results are
                             the same either way; best with slots = the number of resident
                             workgroups (hipipm_resident_slots) and a pass count large enough
                             for the whole solve to be one launch */
    int32_t nested_resto; /* nested hard restoration (Table I row 6): when the restoration phase cannot
                             make progress (its line search or inertia correction fails) at a point
                             where its own constraints c(x) - p + n = 0 are violated by more than tol,
                             restore them -- at fixed x, p and n take the closed form that starts the
                             restoration phase, at its current mu -- and continue restoring; 1
                             (default) on, 0: the restoration fails there (status RESTO_FAILED) */
    int32_t resto_ls_max; /* most backtracking halvings of a restoration-phase line search (default 60,
                             as in the main phase; 0: a rejected full step fails at once) */
} hipipm_options;

typedef struct {
    int32_t n, m, n_w, n_s, n_theta, n_lower, n_upper, N, nx, nu, n_ineq;
} hipipm_dims;

typedef struct {
    int64_t iterations, resto_iterations, soc_tried, soc_accepted, factorizations, resto_entries,
        tiny_steps, passes, instances_done;
    int64_t solves;                  /* step solves with a stored factor (incl. least-squares y, not SOC) */
    int64_t fused_factorizations;    /* factorizations done inside the fused pass kernel */
    int64_t fused_solves;            /* solves (step and SOC) done inside the fused pass kernel */
    int64_t refine_sweeps;           /* precision 1: refinement sweeps (each one FP32 solve) */
    int64_t fp64_fallbacks;          /* precision 1: iterations refactored in FP64 after refinement failed */
    int64_t warm_started;            /* instances started from a warm point */
    int64_t warm_rejected;           /* warm points rejected (non-finite, or by the gate) -> cold */
    int64_t warm_restarts;           /* warm starts that diverged and restarted cold */
    int64_t fp32_retakes;            /* precision 1: FP32 inertia verdicts (wrong inertia, or a pivot
                                        too close to zero for FP32) taken again in FP64 */
    int64_t watchdog_starts;         /* watchdog activations */
    int64_t watchdog_reverts;        /* watchdog sequences that went back to their starting point */
    int64_t soft_resto_steps;        /* accepted soft-restoration steps */
    int64_t soft_resto_fails;        /* soft restorations that ended in hard restoration */
    int64_t mu_fallbacks;            /* adaptive barrier update: switches to the monotone mode */
    int64_t nested_restorations;     /* nested restorations of the restoration phase */
    int64_t cycles_eval, cycles_pre, cycles_factor, cycles_solve, cycles_linesearch;
                                     /* shader-clock cycles summed over slots in the derivatives (asynchronous
                                        slots only) and the four phases of the fused kernels */
} hipipm_stats;

typedef struct hipipm_ctx hipipm_ctx;

/* Fill *o with the default options (tol 1e-8, max_iter 1000, mu_init 0.1, ...). */
int hipipm_default_options(hipipm_options* o);

/* Create a context for `slots` concurrently iterating instances on the current HIP device.
 * Validates the descriptor; performs no device allocation (see hipipm_bind_workspace).
 * *out receives the context; destroy it with hipipm_destroy. */
int hipipm_create(const hipipm_problem_desc* d, const hipipm_options* o, int32_t slots, hipipm_ctx** out);

/* Sizes of one instance (n variables incl. slacks, m constraints, theta length, ...). */
int hipipm_get_dims(const hipipm_ctx* ctx, hipipm_dims* out);

/* Slots the context's device runs at once in the asynchronous-slot kernel (options.async_passes >
 * 0) for this problem and precision: the kernel's workgroups per compute unit (registers, LDS)
 * times the compute units.  A context with this many slots and a large async_passes keeps every
 * slot resident for the whole solve, in one launch: no slot's instance waits for a compute unit
 * and no launch ends with some units idle while the last slots finish.  Queries the device;
 * allocates nothing.  For callers sizing a persistent solve. */
int hipipm_resident_slots(const hipipm_ctx* ctx, int32_t* slots);

/* Device workspace needed for the context's slot count, in bytes (256-byte aligned base). */
int hipipm_workspace_bytes(const hipipm_ctx* ctx, size_t* bytes);

/* Bind caller-owned device memory of at least hipipm_workspace_bytes() bytes, 256-byte
 * aligned.  The library uses it for all slot state and scratch; the caller frees it after
 * hipipm_destroy (or after binding another buffer). */
int hipipm_bind_workspace(hipipm_ctx* ctx, void* dev_ptr, size_t bytes);

/* Solve n_inst instances with iteration-level batching over the context's slots.
 *   theta   : device, [n_inst][n_theta] FP64, read only
 *   warm    : device, [n_inst][n_w + m] FP64 warm points (the primal w = (x_0, u_0, ..., x_N)
 *             without slacks, then the equality multipliers y), or NULL for the cold start
 *             (x_k = xbar0, u_k = hover thrust, s = g(x), z = 1, least-squares y).  A warm
 *             instance starts at w pushed into the bounds by options.warm_push, s = max(g(w),
 *             warm_push), its y, bound multipliers from stationarity floored at mu0 / slack,
 *             mu0 = options.warm_mu0; a warm point with a non-finite entry is rejected and the
 *             instance starts cold (see also options.warm_iter_cap)
 *   x_out   : device, [n_inst][n];  y_out: [n_inst][m];  zl_out, zu_out: [n_inst][n]
 *             (bound multipliers, zero on unbounded components)
 *   obj_out, kkt_out : device, [n_inst] objective and scaled KKT error E_0 at the result
 *   status_out, iters_out : device, [n_inst] int32
 * Output pointers may be NULL to skip that output (theta may not).
 * The call returns when every instance has finished (it waits on `stream` for the completion
 * counter, which it polls every options.poll_every passes; one chunk of passes over empty slots
 * may still be queued and is finished before the return).  One context runs one solve at a time:
 * its workspace and its pinned counter copies (allocated at the first solve, freed by
 * hipipm_destroy) are shared by all its calls.  Errors: HIPIPM_ERR_INVALID_ARG (NULL context or
 * theta, n_inst < 0), HIPIPM_ERR_WORKSPACE (no workspace bound), HIPIPM_ERR_HIP (a HIP call
 * failed, or the solve exceeded its pass bound; the stream is synchronised first). */
int hipipm_solve(hipipm_ctx* ctx, int32_t n_inst, const double* theta, const double* warm, double* x_out,
                 double* y_out, double* zl_out, double* zu_out, double* obj_out, double* kkt_out,
                 int32_t* status_out, int32_t* iters_out, void* stream);

/* For callers that cannot allocate device or pinned host memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): hipipm_solve with the library's own
 * static device workspace of HIPIPM_STATIC_WORKSPACE_BYTES (64 MiB) per GPU instead of the bound
 * workspace.  Arguments, outputs and results are those of hipipm_solve (same kernels); the
 * context needs no bound workspace, but hipipm_workspace_bytes() of the context must not exceed
 * the static size (HIPIPM_ERR_WORKSPACE otherwise: create it with fewer slots; e.g. up to about
 * 120 slots of the N = 30, 8-sphere tracking family, 350 of the N = 10, 3-sphere point-to-point
 * family).
 * The call allocates nothing: no hipMalloc/hipFree, no pinned host buffer, no events (kernel timing
 * is not recorded); it polls the completion counter with a copy into host stack memory and a wait
 * on `stream` every options.poll_every passes.  All calls on one GPU share that GPU's static
 * workspace: calls that overlap in time on one GPU (from several threads or streams) race and
 * must be serialised by the caller.  The array keeps the last call's contents; the call re-arms
 * what must start from known values (the counter block, every slot it uses). */
#define HIPIPM_STATIC_WORKSPACE_BYTES (64ull << 20)
int hipipm_solve_noalloc(hipipm_ctx* ctx, int32_t n_inst, const double* theta, const double* warm, double* x_out,
                         double* y_out, double* zl_out, double* zu_out, double* obj_out, double* kkt_out,
                         int32_t* status_out, int32_t* iters_out, void* stream);

/* Counters accumulated over all solves since creation (or the last hipipm_reset_stats). */
int hipipm_stats_get(const hipipm_ctx* ctx, hipipm_stats* out);
int hipipm_reset_stats(hipipm_ctx* ctx);

/* Kernel timing (options.timing = 1): total milliseconds and launch counts per kernel since the
 * last reset, in the order "eval", "pre", "factor", "solve", "linesearch", "fused", "setup",
 * "async" (the five kernels of a pass, the fused pass kernel used for the last options.fuse_below
 * instances, the per-solve setup, the asynchronous-slot kernel).  *n_kernels: capacity of the
 * arrays on input, number of timed kernels (8) on output. */
int hipipm_kernel_times(const hipipm_ctx* ctx, int32_t* n_kernels, double* total_ms, int64_t* launches);

/* ---- test hooks (one-step replay, Sec. VI "Correctness") ----
 * A flat FP64 state per slot in the oracle's field order:
 *   header[16]: phase, iter, status, init_filter, theta_R, warm, warm-gate stage, 0...
 *   main : mu, tau, dx_last, theta_max, theta_min, tiny, nf, 0 | x[n] y[m] zl[n] zu[n] | fth[F] fph[F]
 *   resto: same with n + 2m variables (x, p, n)
 *   x_R[n], DR2[n]
 *   watchdog: shortened-step count, active, steps taken, theta, phi_mu, grad phi^T d, alpha_max, mu
 *             of the reference iteration | its x[n] y[m] zl[n] zu[n]
 *   soft restoration: active, steps taken, theta, phi_mu of its starting point
 *   adaptive barrier update: free mode, references held, references[4], mu ceiling, 0
 * with F = max_iter + 2 filter pairs (the filter is never full: each pair comes from an accepted
 * iteration or a restoration entry).  A warm start's gate data are not part of the state.
 * hipipm_state_len gives its length.  hipipm_state_import loads `count` states (host pointer,
 * [count][len]) into slots 0..count-1 (theta from the device pointer, [count][n_theta]);
 * hipipm_start instead starts instances 0..count-1 of theta (device, [count][n_theta]) and warm
 * (device, [count][n_w + m] or NULL; as in hipipm_solve) in slots 0..count-1 without running a
 * pass; hipipm_step runs `passes` passes of the iteration pipeline on those slots without refill,
 * with the kernels a solve uses (the fused pass kernel when options.precision = 1 or
 * options.fuse_below > 0, the per-phase kernels otherwise); theta and warm (device, may be NULL
 * for warm) are the rows of slot i's instance i, read by a cold restart and by the warm-start gate;
 * hipipm_state_export copies the slot states back (host pointer).  Errors: INVALID_ARG for a NULL
 * context, count outside [0, slots], negative passes, NULL theta (count > 0) or states; WORKSPACE
 * without a bound workspace; HIP when a HIP call fails. */
int hipipm_state_len(const hipipm_ctx* ctx, int32_t* len);
int hipipm_state_import(hipipm_ctx* ctx, int32_t count, const double* states_host, const double* theta_dev,
                        void* stream);
int hipipm_start(hipipm_ctx* ctx, int32_t count, const double* theta, const double* warm, void* stream);
int hipipm_step(hipipm_ctx* ctx, int32_t count, int32_t passes, const double* theta, const double* warm,
                void* stream);
int hipipm_state_export(hipipm_ctx* ctx, int32_t count, double* states_host, void* stream);

/* Raw structured KKT factor + solve for kernel parity: for `count` instances (device pointers)
 * at primal-dual points v [count][n], y [count][m], zl/zu [count][n] with barrier mu, factor
 * the augmented matrix of eq. (7) with perturbations delta_x, delta_c, solve it for the
 * right-hand side rhs [count][n + m] (v rows then y rows) into sol [count][n + m], and write
 * inertia_ok [count] (1 when every pivot block had the required sign, i.e. inertia (n, m, 0)).
 * theta: [count][n_theta]. */
int hipipm_kkt_factor_solve(hipipm_ctx* ctx, int32_t count, const double* theta, const double* v,
                            const double* y, const double* zl, const double* zu, double mu, double delta_x,
                            double delta_c, const double* rhs, double* sol, int32_t* inertia_ok, void* stream);

/* Stage derivatives for kernel parity: for `count` stages, F (13), G = dF/d(x,u) (13 x 17, row
 * major) and H = sum_r lam_r d2F_r/d(x,u)^2 (17 x 17) of the RK4 step; x [count][13],
 * u [count][4], lam [count][13] device pointers. */
int hipipm_stage_derivs(hipipm_ctx* ctx, int32_t count, const double* x, const double* u, const double* lam,
                        double* F, double* G, double* H, void* stream);

const char* hipipm_last_error(const hipipm_ctx* ctx);
void hipipm_destroy(hipipm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
