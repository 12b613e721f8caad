/*
 * CPU FP64 ORACLE -- test infrastructure only.
 *
 * A plain, slow, dense implementation of the batched primal-dual interior-point
 * method of "Scaling Nonlinear Optimization: Many Problems One GPU" (Sec. IV and
 * Table I), used only by the tests, the smoke check and the CPU-baseline leg of
 * the benchmark to check the HIP solver.  It shares no code with the HIP
 * library: its own problem descriptor, derivatives (hyper-dual numbers), dense
 * KKT assembly and dense Bunch-Kaufman LDL^T.  Nothing in the product path may
 * link, import or call it.
 */
#ifndef IPM_ORACLE_H
#define IPM_ORACLE_H

#include <stdint.h>

/* ---------------- dense symmetric indefinite LDL^T (Bunch-Kaufman) ---------------- */
/* Factor the symmetric n x n matrix A (row-major, full storage; only the lower
 * triangle is read) as P A P^T = L D L^T.  On return A holds L (strict lower
 * part, unit diagonal implied) and D (diagonal and, for 2x2 pivots, the
 * subdiagonal entry).  perm[k] = original index of position k; blk[k] = 1 for a
 * 1x1 pivot, 2 for the first row of a 2x2 pivot, 0 for its second row.
 * inertia = (n_plus, n_minus, n_zero) counted from the pivot blocks; a pivot is
 * "zero" only if it is exactly 0.  Returns 0. */
int bk_factor(int n, double* A, int* perm, int* blk, int inertia[3]);
/* Solve A x = b with the factor from bk_factor; b is overwritten with x. */
void bk_solve(int n, const double* F, const int* perm, const int* blk, double* b, double* work);

/* ---------------- generic NLP (eq. (1)) ---------------- */
typedef struct nlp_s {
    int n, m;
    const double* xl; /* length n; -INFINITY where no lower bound */
    const double* xu; /* length n; +INFINITY where no upper bound */
    void* ud;
    void (*f)(void* ud, const double* x, double* out);
    void (*grad)(void* ud, const double* x, double* g);
    void (*c)(void* ud, const double* x, double* c);
    void (*jac)(void* ud, const double* x, double* J); /* m x n dense, row-major */
    /* n x n dense full: objf * Hess f + sum_i y_i Hess c_i */
    void (*hess)(void* ud, const double* x, double objf, const double* y, double* H);
} nlp_t;

/* ---------------- algorithm options (IPOPT published defaults, readings) ---------------- */
typedef struct {
    double tol;            /* 1e-8 : scaled KKT error E_0 at convergence */
    int32_t max_iter;      /* 1000 */
    double mu_init;        /* 0.1 */
    double kappa_eps;      /* 10 */
    double kappa_mu;       /* 0.2 */
    double theta_mu;       /* 1.5 */
    double tau_min;        /* 0.99 */
    double kappa1, kappa2; /* 1e-2, 1e-2 : bound push */
    double lam_max;        /* 1e3 : least-squares multiplier cap */
    double s_max;          /* 100 */
    double delta_min, delta_0, delta_max;          /* 1e-20, 1e-4, 1e40 */
    double delta_c_bar, kappa_c;                   /* 1e-8, 0.25 */
    double kappa_minus, kappa_plus, kappa_plus_bar;/* 1/3, 8, 100 */
    double gamma_theta, gamma_phi, delta_sw;       /* 1e-5, 1e-8, 1 */
    double s_theta, s_phi, eta_phi, gamma_alpha;   /* 1.1, 2.3, 1e-8, 0.05 */
    int32_t max_soc; double kappa_soc;             /* 4, 0.99 */
    double kappa_sigma;                            /* 1e10 */
    double rho_resto, kappa_resto;                 /* 1000, 0.9 */
    double bound_mult_reset;                       /* 1e3 */
    /* learned warm start (step 14 of the method as built here): bound push, barrier parameter,
     * divergence cap (0: only restoration counts as divergence), E_mu0 gate on/off */
    double warm_mu0, warm_push;                    /* 1e-3, 1e-3 */
    int32_t warm_iter_cap;                         /* 0 */
    int32_t warm_gate;                             /* 1 */
    /* watchdog (Table I row 3): consecutive shortened iterations that start it (0: off), full
     * steps it takes without the line-search test before reverting */
    int32_t watchdog_trigger, watchdog_max;        /* 0, 3 */
    /* soft feasibility restoration (Table I row 5): soft steps before hard restoration (0: off),
     * required reduction factor of the primal-dual error */
    int32_t soft_resto_max;                        /* 0 */
    double soft_resto_factor;                      /* 0.9999 */
    /* barrier update (Table I row 7): 0 monotone, 1 adaptive (free mode, monotone fallback) */
    int32_t mu_strategy;                           /* 0 */
    /* nested hard restoration (Table I row 6): when the restoration phase cannot make progress,
     * restore its own constraints (1) or fail (0); most backtracking halvings of a restoration
     * line search (the main phase allows 60) */
    int32_t nested_resto;                          /* 1 */
    int32_t resto_ls_max;                          /* 60 */
} ipmo_opts;

/* ---------------- quadrotor NMPC problem family ---------------- */
typedef struct {
    int32_t family;   /* 0 point-to-point with spheres, 1 figure-eight tracking, 2 multi-quadrotor,
                         3 figure-eight tracking with spheres moving at constant velocity */
    int32_t N;        /* shooting intervals */
    int32_t n_agents;
    int32_t n_obs;
    double dt, mass, jxx, jyy, jzz, arm, ctau, grav;
    double q_weight, r_weight, d_min;
} ipmo_quad_desc;

enum { PH_INIT_Y = 0, PH_REGULAR = 1, PH_RESTO = 2, PH_DONE = 3 };
enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAX_ITER = 2, ST_RESTO_FAILED = 3,
       ST_INFEASIBLE = 4, ST_NUMERICAL = 5 };

#endif
