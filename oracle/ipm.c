/*
 * CPU FP64 ORACLE -- test infrastructure only (see oracle.h).
 *
 * Primal-dual interior-point method for the parametric NLP of Sec. III eq. (1),
 * in the order of Sec. IV:
 *   barrier problem (eq. (3)), Lagrangian (eq. (4)), perturbed KKT conditions
 *   (eq. (5)), Newton system (eq. (6)) reduced to the augmented system (eq. (7))
 *   by eliminating the bound-multiplier steps, LDL^T with inertia and the
 *   delta_x / delta_c inertia correction (Sec. IV "Step direction"), and the
 *   fallback branches of Table I: backtracking filter line search (row 1),
 *   second-order correction (row 2), tiny-step rule (row 4), hard feasibility
 *   restoration (row 6, one level) and the monotone barrier update (row 7).
 * The paper hands the constants and sub-rules of these branches to the IPOPT
 * paper (Waechter & Biegler 2006); the published defaults are used, listed in
 * ipmo_opts.
 *
 * Everything is dense: the full (n+m) x (n+m) matrix of eq. (7) is assembled
 * with slacks (and, in restoration, the p/n elastic variables) as ordinary
 * variables and factored by bk_factor.
 *
 * The method is run as a sequence of "passes" so that its state can be saved
 * and replayed one step at a time (Sec. VI "Correctness"):
 *   PH_INIT_Y  : least-squares equality multipliers at the current point;
 *   PH_REGULAR : one iteration on the original problem;
 *   PH_RESTO   : one iteration on the feasibility-restoration problem.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void* quad_nlp_new(const ipmo_quad_desc* d, const double* theta, nlp_t* out);
void quad_nlp_free(void* p);
void quad_cold_start(const ipmo_quad_desc* d, const double* theta, double* v);
void quad_warm_point(const ipmo_quad_desc* d, const double* theta, const double* w, double* v);
int quad_nw(const ipmo_quad_desc* d);

#define EPS DBL_EPSILON

struct solver_s;
static void grow_buffers(struct solver_s* S, int nv);

/* ------------------------------------------------------------------ */
/* one barrier-problem iterate (original problem or restoration problem) */
typedef struct {
    int n, m;
    double *x, *y, *zl, *zu; /* zl/zu full length, zero on unbounded components */
    double mu, tau, dx_last, theta_max, theta_min;
    int tiny;
    int nf, fcap;     /* filter entries in use, allocated capacity (grows without limit) */
    double *fth, *fph;
} sub_t;

/* restoration NLP: min rho sum(p+n) + zeta/2 |D_R (x - x_R)|^2 s.t. c(x) - p + n = 0 */
typedef struct {
    nlp_t* P;
    int n, m;
    double *xR, *DR2;
    double zeta, rho;
    double *xl, *xu;
    double *cb, *Jb, *Hb;
} resto_ud;

typedef struct solver_s {
    nlp_t* P;
    ipmo_opts o;
    int phase, status, iter, init_filter;
    /* learned warm start: warm = 1 while the iterate comes from a warm point (a divergence then
     * restarts cold); wstage = 1 while the gate's cold reference is being computed, 2 while the
     * warm point waits for its multipliers and the gate's comparison */
    int warm, wstage;
    double e_cold;                      /* gate: E_mu0 of the cold start */
    double *warm_w, *warm_y;            /* the warm row (copied), NULL for a cold start */
    double *x_cold, *y_cold;            /* the cold start (before the bound push); gate: its least-squares y */
    double thmax_cold, thmin_cold;
    int scap;                           /* filter pairs kept in the flat state (max_iter + 2) */
    sub_t main, rs;
    nlp_t RP;
    resto_ud RU;
    double theta_R;
    /* evaluation buffers, sized for the restoration problem */
    double *g, *c, *J, *Hm, *K, *rhs, *wk, *dx, *dy, *dzl, *dzu, *xt, *ct, *csoc, *gphi, *rx;
    double *dxs, *dys, *dzls, *dzus;
    int *perm, *blk;
    int cap_n;
    double f;
    /* statistics */
    int st_resto_iter, st_soc_try, st_soc_acc, st_fact, st_resto_entries, st_tiny, st_passes;
    int st_warm_started, st_warm_rejected, st_warm_restarts, st_wd_starts, st_wd_reverts;
    /* watchdog (Table I row 3) on the original problem: consecutive shortened iterations, active
     * flag, unconditional steps taken, and the reference iterate where it started with that
     * iteration's theta, phi_mu, directional derivative, step size alpha_max and mu */
    int wd_short, wd_active, wd_iter;
    double wd_thk, wd_phk, wd_gphi, wd_amax, wd_mu;
    double *wd_x, *wd_y, *wd_zl, *wd_zu;
    /* soft feasibility restoration (Table I row 5): active flag, soft steps taken, theta and phi_mu
     * of the iterate where it started; trial buffers of a soft step */
    int soft, soft_iter, st_soft_steps, st_soft_fails;
    double soft_thk, soft_phk;
    /* adaptive barrier update (Table I row 7): mode (1 free, 0 monotone fallback), the last
     * MU_REFS scaled KKT errors E_0 that the free mode must improve on, how many are held, the
     * barrier-parameter ceiling, switches to the monotone mode */
    int mu_free, n_refs, st_mu_fallbacks;
    int st_nested;                      /* nested restorations of the restoration phase */
    double refs[4], mu_max;
    double *sf_y, *sf_zl, *sf_zu, *sf_g, *sf_J;
    double last_dx, last_dc, last_alpha, last_alpha_z;
    int last_soc;
    /* second-order corrections of the last pass: count, c_soc and step of each, theta of each trial */
    int soc_n;
    double *soc_c, *soc_d, *soc_th;
} solver_t;

/* ------------------------------------------------------------------ */
static void sub_alloc(sub_t* T, int n, int m) {
    T->n = n; T->m = m;
    T->x = (double*)calloc(n, sizeof(double));
    T->y = (double*)calloc(m > 0 ? m : 1, sizeof(double));
    T->zl = (double*)calloc(n, sizeof(double));
    T->zu = (double*)calloc(n, sizeof(double));
    T->fcap = 16;
    T->fth = (double*)calloc(T->fcap, sizeof(double));
    T->fph = (double*)calloc(T->fcap, sizeof(double));
    T->nf = 0;
}

static void sub_free(sub_t* T) {
    free(T->x); free(T->y); free(T->zl); free(T->zu); free(T->fth); free(T->fph);
}

/* filter F = {(theta_F, phi_F)} (Table I row 1): a point is rejected if theta >= theta_F and
 * phi >= phi_F for some entry.  Entries dominated by a new entry are dropped (their forbidden
 * region is contained in the new one), so the semantics do not change.  The filter has no
 * capacity limit: the storage grows as needed. */
static void filter_add(sub_t* T, double th, double ph) {
    int w = 0;
    for (int i = 0; i < T->nf; ++i)
        if (!(T->fth[i] >= th && T->fph[i] >= ph)) { T->fth[w] = T->fth[i]; T->fph[w] = T->fph[i]; ++w; }
    T->nf = w;
    if (T->nf >= T->fcap) {
        T->fcap *= 2;
        T->fth = (double*)realloc(T->fth, (size_t)T->fcap * sizeof(double));
        T->fph = (double*)realloc(T->fph, (size_t)T->fcap * sizeof(double));
    }
    T->fth[T->nf] = th;
    T->fph[T->nf] = ph;
    T->nf++;
}

static int filter_ok(const sub_t* T, double th, double ph) {
    for (int i = 0; i < T->nf; ++i)
        if (th >= T->fth[i] && ph >= T->fph[i]) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* restoration NLP callbacks */
static void r_f(void* ud, const double* x, double* out) {
    resto_ud* R = (resto_ud*)ud;
    double s = 0, q = 0;
    for (int i = 0; i < R->m; ++i) s += x[R->n + i] + x[R->n + R->m + i];
    for (int i = 0; i < R->n; ++i) { double e = x[i] - R->xR[i]; q += R->DR2[i] * e * e; }
    *out = R->rho * s + 0.5 * R->zeta * q;
}
static void r_grad(void* ud, const double* x, double* g) {
    resto_ud* R = (resto_ud*)ud;
    for (int i = 0; i < R->n; ++i) g[i] = R->zeta * R->DR2[i] * (x[i] - R->xR[i]);
    for (int i = 0; i < 2 * R->m; ++i) g[R->n + i] = R->rho;
}
static void r_c(void* ud, const double* x, double* c) {
    resto_ud* R = (resto_ud*)ud;
    R->P->c(R->P->ud, x, c);
    for (int i = 0; i < R->m; ++i) c[i] += -x[R->n + i] + x[R->n + R->m + i];
}
static void r_jac(void* ud, const double* x, double* J) {
    resto_ud* R = (resto_ud*)ud;
    int n = R->n, m = R->m, N = n + 2 * m;
    R->P->jac(R->P->ud, x, R->Jb);
    memset(J, 0, (size_t)m * N * sizeof(double));
    for (int i = 0; i < m; ++i) {
        memcpy(J + (size_t)i * N, R->Jb + (size_t)i * n, n * sizeof(double));
        J[(size_t)i * N + n + i] = -1.0;
        J[(size_t)i * N + n + m + i] = 1.0;
    }
}
static void r_hess(void* ud, const double* x, double objf, const double* y, double* Hm) {
    resto_ud* R = (resto_ud*)ud;
    int n = R->n, N = n + 2 * R->m;
    R->P->hess(R->P->ud, x, 0.0, y, R->Hb);
    memset(Hm, 0, (size_t)N * N * sizeof(double));
    for (int i = 0; i < n; ++i) {
        memcpy(Hm + (size_t)i * N, R->Hb + (size_t)i * n, n * sizeof(double));
        Hm[(size_t)i * N + i] += objf * R->zeta * R->DR2[i];
    }
}

/* ------------------------------------------------------------------ */
static double dot(int n, const double* a, const double* b) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}
static double nrm1(int n, const double* a) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += fabs(a[i]);
    return s;
}
static double nrmi(int n, const double* a) {
    double s = 0;
    for (int i = 0; i < n; ++i) if (fabs(a[i]) > s) s = fabs(a[i]);
    return s;
}

/* barrier objective phi_mu (eq. (3)) restricted to the finite bounds; NaN outside the interior */
static double barrier_obj(const nlp_t* P, const double* x, double f, double mu) {
    double b = 0;
    for (int i = 0; i < P->n; ++i) {
        if (isfinite(P->xl[i])) { double s = x[i] - P->xl[i]; if (!(s > 0)) return NAN; b += log(s); }
        if (isfinite(P->xu[i])) { double s = P->xu[i] - x[i]; if (!(s > 0)) return NAN; b += log(s); }
    }
    return f - mu * b;
}

/* scaled KKT error E_mu of the perturbed optimality conditions (eq. (5)) with the IPOPT
 * scaling s_d, s_c (s_max = 100).  g = grad f, c, J at T->x. */
static double kkt_error(const nlp_t* P, const sub_t* T, const double* g, const double* c, const double* J,
                        double mu, const ipmo_opts* o, double* wk) {
    int n = P->n, m = P->m;
    int nL = 0, nU = 0;
    double s1 = nrm1(m, T->y), z1 = 0, comp = 0;
    for (int i = 0; i < n; ++i) wk[i] = g[i] - T->zl[i] + T->zu[i];
    for (int r = 0; r < m; ++r) {
        double yr = T->y[r];
        if (yr == 0.0) continue;
        const double* Jr = J + (size_t)r * n;
        for (int i = 0; i < n; ++i) wk[i] += Jr[i] * yr;
    }
    for (int i = 0; i < n; ++i) {
        if (isfinite(P->xl[i])) {
            nL++; z1 += fabs(T->zl[i]);
            double e = fabs((T->x[i] - P->xl[i]) * T->zl[i] - mu);
            if (e > comp) comp = e;
        }
        if (isfinite(P->xu[i])) {
            nU++; z1 += fabs(T->zu[i]);
            double e = fabs((P->xu[i] - T->x[i]) * T->zu[i] - mu);
            if (e > comp) comp = e;
        }
    }
    double sd = 1.0, sc = 1.0;
    if (m + nL + nU > 0) sd = fmax(o->s_max, (s1 + z1) / (double)(m + nL + nU)) / o->s_max;
    if (nL + nU > 0) sc = fmax(o->s_max, z1 / (double)(nL + nU)) / o->s_max;
    double e = nrmi(n, wk) / sd;
    double pr = nrmi(m, c);
    if (pr > e) e = pr;
    if (comp / sc > e) e = comp / sc;
    return e;
}

/* fraction-to-the-boundary rule on the bounded primal components */
static double ftb_primal(const nlp_t* P, const double* x, const double* dx, double tau) {
    double a = 1.0;
    for (int i = 0; i < P->n; ++i) {
        if (isfinite(P->xl[i]) && dx[i] < 0) { double t = -tau * (x[i] - P->xl[i]) / dx[i]; if (t < a) a = t; }
        if (isfinite(P->xu[i]) && dx[i] > 0) { double t = tau * (P->xu[i] - x[i]) / dx[i]; if (t < a) a = t; }
    }
    return a;
}
static double ftb_dual(const nlp_t* P, const double* zl, const double* zu, const double* dzl,
                       const double* dzu, double tau) {
    double a = 1.0;
    for (int i = 0; i < P->n; ++i) {
        if (isfinite(P->xl[i]) && dzl[i] < 0) { double t = -tau * zl[i] / dzl[i]; if (t < a) a = t; }
        if (isfinite(P->xu[i]) && dzu[i] < 0) { double t = -tau * zu[i] / dzu[i]; if (t < a) a = t; }
    }
    return a;
}

/* bound-multiplier steps eliminated from eq. (6) (Sec. IV):
 *   dz_L = S_L^{-1}(mu e - S_L z_L - Z_L dx),  dz_U = S_U^{-1}(mu e - S_U z_U + Z_U dx) */
static void dz_recover(const nlp_t* P, const sub_t* T, const double* dx, double* dzl, double* dzu) {
    for (int i = 0; i < P->n; ++i) {
        dzl[i] = dzu[i] = 0.0;
        if (isfinite(P->xl[i])) { double s = T->x[i] - P->xl[i]; dzl[i] = (T->mu - s * T->zl[i] - T->zl[i] * dx[i]) / s; }
        if (isfinite(P->xu[i])) { double s = P->xu[i] - T->x[i]; dzu[i] = (T->mu - s * T->zu[i] + T->zu[i] * dx[i]) / s; }
    }
}

/* assemble the lower triangle of K(delta_x, delta_c) = [[W + Sigma + dx I, A^T], [A, -dc I]] (eq. (7)) */
static void assemble_K(const nlp_t* P, const sub_t* T, const double* Hm, const double* J, double dxp, double dcp,
                       double* K) {
    int n = P->n, m = P->m, N = n + m;
    for (int i = 0; i < n; ++i) {
        double* Ki = K + (size_t)i * N;
        memcpy(Ki, Hm + (size_t)i * n, (i + 1) * sizeof(double));
        double sig = 0;
        if (isfinite(P->xl[i])) sig += T->zl[i] / (T->x[i] - P->xl[i]);
        if (isfinite(P->xu[i])) sig += T->zu[i] / (P->xu[i] - T->x[i]);
        Ki[i] += sig + dxp;
    }
    for (int r = 0; r < m; ++r) {
        double* Ki = K + (size_t)(n + r) * N;
        memcpy(Ki, J + (size_t)r * n, n * sizeof(double));
        memset(Ki + n, 0, (r + 1) * sizeof(double));
        Ki[n + r] = -dcp;
    }
}

/* ------------------------------------------------------------------ */
enum { R_ACCEPT = 0, R_CONVERGED, R_MAXITER, R_LSFAIL, R_ICFAIL, R_NUMERICAL };

static void eval_point(solver_t* S, const nlp_t* P, const sub_t* T) {
    P->f(P->ud, T->x, &S->f);
    P->grad(P->ud, T->x, S->g);
    P->c(P->ud, T->x, S->c);
    P->jac(P->ud, T->x, S->J);
}

static void set_zeta(solver_t* S, const sub_t* T, int is_resto) {
    if (is_resto) S->RU.zeta = sqrt(T->mu);
}

/* evaluate c, f, theta = |c|_1 and phi_mu at a trial point; returns 1 if all finite */
static int trial_eval(const nlp_t* P, const sub_t* T, const double* xt, double* ct, double* th, double* ph) {
    double f;
    P->c(P->ud, xt, ct);
    P->f(P->ud, xt, &f);
    *th = nrm1(P->m, ct);
    *ph = barrier_obj(P, xt, f, T->mu);
    return isfinite(*th) && isfinite(*ph);
}

/* filter acceptance of a trial (theta_t, phi_t) for step size alpha (Table I row 1). */
static int acceptable(const sub_t* T, const ipmo_opts* o, double thk, double phk, double gphi, double alpha,
                      double tht, double pht, int* sw_out, int* arm_out) {
    if (!(isfinite(tht) && isfinite(pht))) return 0;
    if (tht > T->theta_max) return 0;
    int sw = gphi < 0 && alpha * pow(-gphi, o->s_phi) > o->delta_sw * pow(thk, o->s_theta);
    double slack = 10.0 * EPS * fabs(phk);
    int arm = (pht - (phk + o->eta_phi * alpha * gphi)) <= slack;
    int ok;
    if (sw && thk <= T->theta_min) ok = arm;
    else ok = (tht <= (1.0 - o->gamma_theta) * thk) || ((pht - (phk - o->gamma_phi * thk)) <= slack);
    if (!ok) return 0;
    if (!filter_ok(T, tht, pht)) return 0;
    *sw_out = sw;
    *arm_out = arm;
    return 1;
}

/* smallest step size the backtracking tries before falling back to restoration (Table I row 1,
 * constants of the filter method): gamma_alpha times the least of gamma_theta, the step that
 * would give the required phi decrease, and (when the switching condition can apply) the step
 * at which the switching condition starts to hold */
static double alpha_min(const ipmo_opts* o, double thk, double gphi, double theta_min) {
    if (!(gphi < 0)) return o->gamma_alpha * o->gamma_theta;
    double t = fmin(o->gamma_theta, o->gamma_phi * thk / (-gphi));
    if (thk <= theta_min) t = fmin(t, o->delta_sw * pow(thk, o->s_theta) / pow(-gphi, o->s_phi));
    return o->gamma_alpha * t;
}

/* monotone barrier update (Table I row 7): decrease mu while the barrier problem is solved to
 * kappa_eps * mu, or once after a tiny step; reset the filter on every decrease. */
static void mu_update(solver_t* S, const nlp_t* P, sub_t* T, int is_resto) {
    const ipmo_opts* o = &S->o;
    double mu_min = o->tol / 10.0;
    for (;;) {
        double Emu = kkt_error(P, T, S->g, S->c, S->J, T->mu, o, S->wk);
        if (!(Emu <= o->kappa_eps * T->mu || T->tiny)) break;
        T->tiny = 0;
        double nm = fmax(mu_min, fmin(o->kappa_mu * T->mu, pow(T->mu, o->theta_mu)));
        if (!(nm < T->mu)) break;
        T->mu = nm;
        T->tau = fmax(o->tau_min, 1.0 - T->mu);
        T->nf = 0;
        if (is_resto) {                 /* the restoration objective depends on mu through zeta */
            set_zeta(S, T, 1);
            P->f(P->ud, T->x, &S->f);
            P->grad(P->ud, T->x, S->g);
        }
    }
}

/* Adaptive barrier update (Table I row 7), original problem only.  Free mode: mu from the
 * current complementarity by the LOQO rule, mu = sigma * avg with avg = mean of the products
 * s_i z_i over the bounded components, xi = min_i(s_i z_i) / avg and
 * sigma = 0.1 min(0.05 (1 - xi) / xi, 2)^3, kept in [tol / 10, mu_max]; the free mode continues
 * while the scaled KKT error E_0 of each new iterate is at most kappa_red = 0.9999 times the
 * largest of the last four accepted ones.  Otherwise the monotone mode takes over, starting from
 * mu = 0.8 avg; once its barrier problem is solved (E_mu <= kappa_eps mu) and E_0 has come down
 * by kappa_red against the references, the free mode resumes, else mu decreases monotonically.
 * The filter is reset whenever mu changes. */
#define MU_REFS 4
static void mu_refs_push(solver_t* S, double e0) {
    if (S->n_refs == MU_REFS) {
        for (int i = 1; i < MU_REFS; ++i) S->refs[i - 1] = S->refs[i];
        S->n_refs--;
    }
    S->refs[S->n_refs++] = e0;
}
static int mu_progress(const solver_t* S, double e0) {
    if (S->n_refs == 0) return 1;
    double mx = S->refs[0];
    for (int i = 1; i < S->n_refs; ++i) mx = fmax(mx, S->refs[i]);
    return e0 <= 0.9999 * mx;
}
static void compl_stats(const nlp_t* P, const sub_t* T, double* avg, double* mn) {
    double sum = 0, lo = INFINITY;
    int cnt = 0;
    for (int i = 0; i < P->n; ++i) {
        if (isfinite(P->xl[i])) { double p = (T->x[i] - P->xl[i]) * T->zl[i]; sum += p; lo = fmin(lo, p); cnt++; }
        if (isfinite(P->xu[i])) { double p = (P->xu[i] - T->x[i]) * T->zu[i]; sum += p; lo = fmin(lo, p); cnt++; }
    }
    *avg = cnt ? sum / cnt : 0.0;
    *mn = cnt ? lo : 0.0;
}
static void mu_update_adaptive(solver_t* S, const nlp_t* P, sub_t* T, double e0) {
    const ipmo_opts* o = &S->o;
    double mu_min = o->tol / 10.0;
    double avg, mn;
    compl_stats(P, T, &avg, &mn);
    if (S->mu_max == 0.0) S->mu_max = 1e3 * fmax(avg, mu_min);     /* set at the first iteration */
    if (S->mu_free && !mu_progress(S, e0)) {
        /* not enough progress: the monotone mode takes over */
        S->mu_free = 0;
        S->st_mu_fallbacks++;
        double nm = fmin(S->mu_max, fmax(mu_min, 0.8 * avg));
        if (nm != T->mu) { T->mu = nm; T->nf = 0; }
        T->tau = fmax(o->tau_min, 1.0 - T->mu);
        return;
    }
    if (!S->mu_free) {
        double Emu = kkt_error(P, T, S->g, S->c, S->J, T->mu, o, S->wk);
        if (!(Emu <= o->kappa_eps * T->mu || T->tiny)) return;      /* barrier problem not solved yet */
        if (mu_progress(S, e0)) {
            S->mu_free = 1;                                          /* progress: back to free mode */
            S->n_refs = 0;
        } else {
            T->tiny = 0;
            double nm = fmax(mu_min, fmin(o->kappa_mu * T->mu, pow(T->mu, o->theta_mu)));
            if (nm < T->mu) { T->mu = nm; T->nf = 0; }
            T->tau = fmax(o->tau_min, 1.0 - T->mu);
            return;
        }
    }
    mu_refs_push(S, e0);
    T->tiny = 0;
    double xi = avg > 0 ? mn / avg : 1.0;
    double t = fmin(0.05 * (1.0 - xi) / xi, 2.0);
    double nm = 0.1 * t * t * t * avg;
    nm = fmin(S->mu_max, fmax(mu_min, nm));
    if (nm != T->mu) { T->mu = nm; T->nf = 0; }
    T->tau = fmax(o->tau_min, 1.0 - T->mu);
}

/* factor K with the delta_x / delta_c inertia correction; returns 0 on success */
static int factor_ic(solver_t* S, const nlp_t* P, sub_t* T) {
    const ipmo_opts* o = &S->o;
    int n = P->n, m = P->m, N = n + m, in[3];
    double dxp = 0.0, dcp = 0.0;
    assemble_K(P, T, S->Hm, S->J, 0.0, 0.0, S->K);
    bk_factor(N, S->K, S->perm, S->blk, in);
    S->st_fact++;
    if (in[0] == n && in[1] == m && in[2] == 0) { S->last_dx = 0; S->last_dc = 0; return 0; }
    if (in[2] > 0) dcp = o->delta_c_bar * pow(T->mu, o->kappa_c);
    dxp = (T->dx_last == 0.0) ? o->delta_0 : fmax(o->delta_min, o->kappa_minus * T->dx_last);
    for (;;) {
        assemble_K(P, T, S->Hm, S->J, dxp, dcp, S->K);
        bk_factor(N, S->K, S->perm, S->blk, in);
        S->st_fact++;
        if (in[0] == n && in[1] == m && in[2] == 0) {
            T->dx_last = dxp;
            S->last_dx = dxp; S->last_dc = dcp;
            return 0;
        }
        if (in[2] > 0 && dcp == 0.0) dcp = o->delta_c_bar * pow(T->mu, o->kappa_c);
        dxp *= (T->dx_last == 0.0) ? o->kappa_plus_bar : o->kappa_plus;
        if (dxp > o->delta_max) return 1;
    }
}

static void kkt_solve(solver_t* S, int N, double* d) { bk_solve(N, S->K, S->perm, S->blk, d, S->wk); }

/* keep c_soc, the step and the trial theta of a second-order correction for inspection */
static void soc_record(solver_t* S, int n, int m, double tht) {
    int k = S->soc_n;
    if (k >= S->o.max_soc) return;
    int nmax = S->P->n + 2 * S->P->m, mm = S->P->m > 0 ? S->P->m : 1;
    memcpy(S->soc_c + (size_t)k * mm, S->csoc, m * sizeof(double));
    memcpy(S->soc_d + (size_t)k * nmax, S->dxs, n * sizeof(double));
    S->soc_th[k] = tht;
    S->soc_n++;
}

/* primal-dual error of the barrier problem at mu (the residual of the perturbed optimality
 * conditions, eq. (5), in the 1-norm): |grad f + A^T y - z_L + z_U|_1 + |c|_1 + the
 * complementarity deviations |S_L z_L - mu e|_1 + |S_U z_U - mu e|_1 */
static double pd_error(const nlp_t* P, const double* x, const double* y, const double* zl, const double* zu,
                       const double* g, const double* c, const double* J, double mu) {
    int n = P->n, m = P->m;
    double e = nrm1(m, c);
    for (int i = 0; i < n; ++i) {
        double d = g[i] - zl[i] + zu[i];
        for (int r = 0; r < m; ++r) d += J[(size_t)r * n + i] * y[r];
        e += fabs(d);
        if (isfinite(P->xl[i])) e += fabs((x[i] - P->xl[i]) * zl[i] - mu);
        if (isfinite(P->xu[i])) e += fabs((P->xu[i] - x[i]) * zu[i] - mu);
    }
    return e;
}

/* Soft feasibility restoration step (Table I row 5): the primal-dual Newton step with one step
 * size for primal and dual variables, alpha = min(alpha_max primal, alpha_max dual), accepted when
 * it lowers the primal-dual error of the barrier problem by the factor soft_resto_factor; the
 * original acceptance test is not applied.  Returns 1 (accepted, iterate updated) or 0. */
static int soft_step(solver_t* S, const nlp_t* P, sub_t* T, double amax) {
    const ipmo_opts* o = &S->o;
    int n = P->n, m = P->m;
    double ad = ftb_dual(P, T->zl, T->zu, S->dzl, S->dzu, T->tau);
    double as = fmin(amax, ad);
    double e0 = pd_error(P, T->x, T->y, T->zl, T->zu, S->g, S->c, S->J, T->mu);
    for (int i = 0; i < n; ++i) {
        S->xt[i] = T->x[i] + as * S->dx[i];
        S->sf_zl[i] = T->zl[i] + as * S->dzl[i];
        S->sf_zu[i] = T->zu[i] + as * S->dzu[i];
    }
    for (int r = 0; r < m; ++r) S->sf_y[r] = T->y[r] + as * S->dy[r];
    P->grad(P->ud, S->xt, S->sf_g);
    P->c(P->ud, S->xt, S->ct);
    P->jac(P->ud, S->xt, S->sf_J);
    double e1 = pd_error(P, S->xt, S->sf_y, S->sf_zl, S->sf_zu, S->sf_g, S->ct, S->sf_J, T->mu);
    if (!(e1 <= o->soft_resto_factor * e0)) return 0;
    memcpy(T->x, S->xt, n * sizeof(double));
    memcpy(T->y, S->sf_y, m * sizeof(double));
    for (int i = 0; i < n; ++i) {
        if (isfinite(P->xl[i])) {
            double s = T->x[i] - P->xl[i];
            T->zl[i] = fmax(fmin(S->sf_zl[i], o->kappa_sigma * T->mu / s), T->mu / (o->kappa_sigma * s));
        }
        if (isfinite(P->xu[i])) {
            double s = P->xu[i] - T->x[i];
            T->zu[i] = fmax(fmin(S->sf_zu[i], o->kappa_sigma * T->mu / s), T->mu / (o->kappa_sigma * s));
        }
    }
    S->last_alpha = as;
    S->last_alpha_z = as;
    return 1;
}

/* one iteration of the barrier method on problem P with iterate T */
static int core_iter(solver_t* S, const nlp_t* P, sub_t* T, int is_resto) {
    const ipmo_opts* o = &S->o;
    int n = P->n, m = P->m, N = n + m;
    set_zeta(S, T, is_resto);
    eval_point(S, P, T);
    double E0 = kkt_error(P, T, S->g, S->c, S->J, 0.0, o, S->wk);
    if (!isfinite(E0)) return R_NUMERICAL;
    if (E0 <= o->tol) return R_CONVERGED;
    if (S->iter >= o->max_iter) return R_MAXITER;
    if (!is_resto && o->mu_strategy == 1) mu_update_adaptive(S, P, T, E0);
    else mu_update(S, P, T, is_resto);
    P->hess(P->ud, T->x, 1.0, T->y, S->Hm);

    /* gradient of the barrier objective and the right-hand side of eq. (7) */
    for (int i = 0; i < n; ++i) {
        double gp = S->g[i];
        if (isfinite(P->xl[i])) gp -= T->mu / (T->x[i] - P->xl[i]);
        if (isfinite(P->xu[i])) gp += T->mu / (P->xu[i] - T->x[i]);
        S->gphi[i] = gp;
        S->rx[i] = gp;
    }
    for (int r = 0; r < m; ++r) {
        const double* Jr = S->J + (size_t)r * n;
        for (int i = 0; i < n; ++i) S->rx[i] += Jr[i] * T->y[r];
    }
    if (factor_ic(S, P, T)) return R_ICFAIL;
    for (int i = 0; i < n; ++i) S->rhs[i] = -S->rx[i];
    for (int r = 0; r < m; ++r) S->rhs[n + r] = -S->c[r];
    kkt_solve(S, N, S->rhs);
    memcpy(S->dx, S->rhs, n * sizeof(double));
    memcpy(S->dy, S->rhs + n, m * sizeof(double));
    dz_recover(P, T, S->dx, S->dzl, S->dzu);

    double amax = ftb_primal(P, T->x, S->dx, T->tau);
    double thk = nrm1(m, S->c);
    double phk = barrier_obj(P, T->x, S->f, T->mu);
    double gphi = dot(n, S->gphi, S->dx);

    /* tiny step (Table I row 4): at a nearly feasible point (|c|_inf <= 1e-4), a step that changes
     * no component by more than 10 eps (relative) is accepted without the line search */
    double tmax = 0;
    for (int i = 0; i < n; ++i) { double t = fabs(S->dx[i]) / (1.0 + fabs(T->x[i])); if (t > tmax) tmax = t; }
    const double *ady = S->dy, *adzl = S->dzl, *adzu = S->dzu;
    double ap = amax;
    int augment = 0, accepted = 0, shortened = 0;
    double aug_th = thk, aug_ph = phk;       /* the point whose (theta, phi) enters the filter */
    S->last_soc = 0;
    S->soc_n = 0;
    const int use_wd = !is_resto && o->watchdog_trigger > 0;
    const int use_soft = !is_resto && o->soft_resto_max > 0;
    if (use_wd && S->wd_active && T->mu != S->wd_mu) S->wd_active = 0;   /* new barrier problem */
    int try_soft = use_soft && S->soft;
    if (try_soft) {
        /* in soft restoration: no line search, the soft step or (after soft_resto_max of them, or
         * when it fails) hard restoration */
    } else if (tmax < 10.0 * EPS && nrmi(m, S->c) <= 1e-4) {
        for (int i = 0; i < n; ++i) S->xt[i] = T->x[i] + ap * S->dx[i];
        T->tiny = 1;
        S->st_tiny++;
        accepted = 1;
        if (use_wd) S->wd_active = 0;
    } else if (use_wd && (S->wd_active || S->wd_short >= o->watchdog_trigger)) {
        /* watchdog (Table I row 3): after watchdog_trigger consecutive shortened steps, take up to
         * watchdog_max full steps (alpha_max) without the line-search test; a step that is
         * acceptable with respect to the iterate where the watchdog started ends it as an ordinary
         * acceptance, and if the last of them is not, the iterate goes back to that reference
         * point (the next iteration starts there with the ordinary backtracking line search) */
        if (!S->wd_active) {
            S->wd_active = 1;
            S->wd_iter = 0;
            S->wd_thk = thk; S->wd_phk = phk; S->wd_gphi = gphi; S->wd_amax = amax; S->wd_mu = T->mu;
            memcpy(S->wd_x, T->x, n * sizeof(double));
            memcpy(S->wd_y, T->y, m * sizeof(double));
            memcpy(S->wd_zl, T->zl, n * sizeof(double));
            memcpy(S->wd_zu, T->zu, n * sizeof(double));
            S->st_wd_starts++;
        }
        for (int i = 0; i < n; ++i) S->xt[i] = T->x[i] + amax * S->dx[i];
        double tht, pht;
        trial_eval(P, T, S->xt, S->ct, &tht, &pht);
        int sw = 0, arm = 0;
        S->wd_iter++;
        if (acceptable(T, o, S->wd_thk, S->wd_phk, S->wd_gphi, S->wd_amax, tht, pht, &sw, &arm)) {
            augment = !(sw && arm);
            aug_th = S->wd_thk;
            aug_ph = S->wd_phk;
            S->wd_active = 0;
            S->wd_short = 0;
        } else if (S->wd_iter >= o->watchdog_max) {
            /* revert: the reference iterate, no step accepted in this pass */
            memcpy(T->x, S->wd_x, n * sizeof(double));
            memcpy(T->y, S->wd_y, m * sizeof(double));
            memcpy(T->zl, S->wd_zl, n * sizeof(double));
            memcpy(T->zu, S->wd_zu, n * sizeof(double));
            S->wd_active = 0;
            S->wd_short = 0;
            S->st_wd_reverts++;
            return R_ACCEPT;
        }
        accepted = 1;
    } else {
        /* backtracking filter line search (Table I rows 1-2) */
        double amin = alpha_min(o, thk, gphi, T->theta_min);
        double alpha = amax;
        for (int l = 0;; ++l) {
            /* alpha_min, or 60 halvings (alpha_min is 0 at an exactly feasible point; the
             * restoration phase takes at most resto_ls_max) */
            if (alpha < amin || l >= (is_resto ? o->resto_ls_max : 60)) {
                if (!use_soft) return R_LSFAIL;
                try_soft = 1;
                break;
            }
            for (int i = 0; i < n; ++i) S->xt[i] = T->x[i] + alpha * S->dx[i];
            double tht, pht;
            int fin = trial_eval(P, T, S->xt, S->ct, &tht, &pht);
            int sw = 0, arm = 0;
            if (acceptable(T, o, thk, phk, gphi, alpha, tht, pht, &sw, &arm)) {
                ap = alpha;
                augment = !(sw && arm);
                accepted = 1;
                shortened = l > 0;
                break;
            }
            if (l == 0 && fin && o->max_soc > 0 && tht >= thk) {
                /* second-order correction: c_soc <- a_soc c_soc + c(x_trial), same factor */
                double asoc = alpha, th_old = 0;
                memcpy(S->csoc, S->c, m * sizeof(double));
                for (int p = 0; p < o->max_soc; ++p) {
                    if (p > 0 && !(tht <= o->kappa_soc * th_old)) break;
                    th_old = tht;
                    for (int r = 0; r < m; ++r) S->csoc[r] = asoc * S->csoc[r] + S->ct[r];
                    for (int i = 0; i < n; ++i) S->rhs[i] = -S->rx[i];
                    for (int r = 0; r < m; ++r) S->rhs[n + r] = -S->csoc[r];
                    kkt_solve(S, N, S->rhs);
                    S->st_soc_try++;
                    memcpy(S->dxs, S->rhs, n * sizeof(double));
                    memcpy(S->dys, S->rhs + n, m * sizeof(double));
                    asoc = ftb_primal(P, T->x, S->dxs, T->tau);
                    for (int i = 0; i < n; ++i) S->xt[i] = T->x[i] + asoc * S->dxs[i];
                    fin = trial_eval(P, T, S->xt, S->ct, &tht, &pht);
                    soc_record(S, n, m, tht);
                    /* acceptance uses the original step size and direction derivative */
                    if (acceptable(T, o, thk, phk, gphi, alpha, tht, pht, &sw, &arm)) {
                        dz_recover(P, T, S->dxs, S->dzls, S->dzus);
                        ady = S->dys; adzl = S->dzls; adzu = S->dzus;
                        ap = asoc;
                        augment = !(sw && arm);
                        accepted = 1;
                        shortened = 1;
                        S->st_soc_acc++;
                        S->last_soc = 1;
                        break;
                    }
                    if (!fin) break;
                }
                if (accepted) break;
            }
            alpha *= 0.5;
        }
    }
    if (try_soft) {
        if (!S->soft) {
            /* the line search failed: start soft restoration at this iterate */
            S->soft = 1;
            S->soft_iter = 0;
            S->soft_thk = thk;
            S->soft_phk = phk;
            S->wd_active = 0;
            S->wd_short = 0;
        }
        if (S->soft_iter >= o->soft_resto_max || !soft_step(S, P, T, amax)) {
            S->soft = 0;
            S->st_soft_fails++;
            return R_LSFAIL;                /* hard restoration */
        }
        S->soft_iter++;
        S->st_soft_steps++;
        /* back to the ordinary iteration once the point is acceptable to the filter with a
         * sufficient decrease of theta or phi_mu over the point where soft restoration started
         * (which then enters the filter) */
        double tht = nrm1(m, S->ct), f;
        P->f(P->ud, T->x, &f);
        double pht = barrier_obj(P, T->x, f, T->mu);
        if (isfinite(tht) && isfinite(pht) && tht <= T->theta_max && filter_ok(T, tht, pht) &&
            (tht <= (1.0 - o->gamma_theta) * S->soft_thk ||
             pht - (S->soft_phk - o->gamma_phi * S->soft_thk) <= 10.0 * EPS * fabs(S->soft_phk))) {
            S->soft = 0;
            filter_add(T, (1.0 - o->gamma_theta) * S->soft_thk, S->soft_phk - o->gamma_phi * S->soft_thk);
        }
        S->iter++;
        return R_ACCEPT;
    }
    (void)accepted;
    /* accept: primal and equality multipliers with the primal step, bound multipliers with the
     * dual fraction-to-boundary step, then the kappa_sigma safeguard */
    double az = ftb_dual(P, T->zl, T->zu, adzl, adzu, T->tau);
    S->last_alpha = ap;
    S->last_alpha_z = az;
    if (augment) filter_add(T, (1.0 - o->gamma_theta) * aug_th, aug_ph - o->gamma_phi * aug_th);
    if (use_wd && !S->wd_active) S->wd_short = shortened ? S->wd_short + 1 : 0;
    for (int r = 0; r < m; ++r) T->y[r] += ap * ady[r];
    for (int i = 0; i < n; ++i) T->x[i] = S->xt[i];
    for (int i = 0; i < n; ++i) {
        if (isfinite(P->xl[i])) {
            double z = T->zl[i] + az * adzl[i], s = T->x[i] - P->xl[i];
            T->zl[i] = fmax(fmin(z, o->kappa_sigma * T->mu / s), T->mu / (o->kappa_sigma * s));
        }
        if (isfinite(P->xu[i])) {
            double z = T->zu[i] + az * adzu[i], s = P->xu[i] - T->x[i];
            T->zu[i] = fmax(fmin(z, o->kappa_sigma * T->mu / s), T->mu / (o->kappa_sigma * s));
        }
    }
    S->iter++;
    if (is_resto) S->st_resto_iter++;
    return R_ACCEPT;
}

/* ------------------------------------------------------------------ */
/* least-squares equality multipliers: [[I, A^T], [A, 0]] [d; y] = -[grad f - z_L + z_U; 0] */
static void init_y(solver_t* S) {
    nlp_t* P = S->P;
    sub_t* T = &S->main;
    int n = P->n, m = P->m, N = n + m, in[3];
    eval_point(S, P, T);
    memset(S->K, 0, (size_t)N * N * sizeof(double));
    for (int i = 0; i < n; ++i) S->K[(size_t)i * N + i] = 1.0;
    for (int r = 0; r < m; ++r) memcpy(S->K + (size_t)(n + r) * N, S->J + (size_t)r * n, n * sizeof(double));
    for (int i = 0; i < n; ++i) S->rhs[i] = -(S->g[i] - T->zl[i] + T->zu[i]);
    for (int r = 0; r < m; ++r) S->rhs[n + r] = 0.0;
    bk_factor(N, S->K, S->perm, S->blk, in);
    kkt_solve(S, N, S->rhs);
    double ym = nrmi(m, S->rhs + n);
    if (!(ym <= S->o.lam_max)) memset(T->y, 0, m * sizeof(double));
    else memcpy(T->y, S->rhs + n, m * sizeof(double));
    if (S->init_filter) {
        double th0 = nrm1(m, S->c);
        T->theta_max = 1e4 * fmax(1.0, th0);
        T->theta_min = 1e-4 * fmax(1.0, th0);
        T->nf = 0;
        S->init_filter = 0;
    }
}

/* push a starting point into the bounds (bound push kappa_1, kappa_2) and set z = 1 on the
 * bounded components, y = 0 and the barrier parameter mu0 */
static void init_point(const nlp_t* P, const ipmo_opts* o, sub_t* T, const double* x0, double k1, double k2,
                       double mu0) {
    for (int i = 0; i < P->n; ++i) {
        double x = x0[i], l = P->xl[i], u = P->xu[i];
        if (isfinite(l) && isfinite(u)) {
            double pl = fmin(k1 * fmax(1.0, fabs(l)), k2 * (u - l));
            double pu = fmin(k1 * fmax(1.0, fabs(u)), k2 * (u - l));
            x = fmax(x, l + pl);
            x = fmin(x, u - pu);
        } else if (isfinite(l)) {
            x = fmax(x, l + k1 * fmax(1.0, fabs(l)));
        } else if (isfinite(u)) {
            x = fmin(x, u - k1 * fmax(1.0, fabs(u)));
        }
        T->x[i] = x;
        T->zl[i] = isfinite(l) ? 1.0 : 0.0;
        T->zu[i] = isfinite(u) ? 1.0 : 0.0;
    }
    memset(T->y, 0, (P->m > 0 ? P->m : 1) * sizeof(double));
    T->mu = mu0;
    T->tau = fmax(o->tau_min, 1.0 - T->mu);
    T->dx_last = 0.0;
    T->tiny = 0;
    T->nf = 0;
    T->theta_max = T->theta_min = 0.0;
}

static void cold_point(solver_t* S) {
    init_point(S->P, &S->o, &S->main, S->x_cold, S->o.kappa1, S->o.kappa2, S->o.mu_init);
}

/* the warm point: w (with its slacks) pushed into the bounds by warm_push, its multipliers y,
 * barrier parameter warm_mu0; the bound multipliers are set in the next INIT_Y pass */
static void warm_point(solver_t* S) {
    init_point(S->P, &S->o, &S->main, S->warm_w, S->o.warm_push, S->o.warm_push, S->o.warm_mu0);
    memcpy(S->main.y, S->warm_y, S->P->m * sizeof(double));
}

/* Warm start, INIT_Y pass at the warm point: bound multipliers from the stationarity residual
 * r = grad f + A^T y (z_L = max(r, mu0 / (x - x_L)), z_U = max(-r, mu0 / (x_U - x))), filter
 * bounds from theta at the warm point.  With the gate, the warm start is kept only if
 * E_mu0(warm) <= E_mu0(cold start) (both at mu0 = warm_mu0); otherwise the cold start computed
 * in the previous pass takes its place. */
static void warm_init_pass(solver_t* S) {
    nlp_t* P = S->P;
    sub_t* T = &S->main;
    int n = P->n, m = P->m;
    eval_point(S, P, T);
    for (int i = 0; i < n; ++i) S->wk[i] = S->g[i];
    for (int r = 0; r < m; ++r)
        for (int i = 0; i < n; ++i) S->wk[i] += S->J[(size_t)r * n + i] * T->y[r];
    const double mu0 = T->mu;
    for (int i = 0; i < n; ++i) {
        double r = S->wk[i];
        T->zl[i] = isfinite(P->xl[i]) ? fmax(r, mu0 / (T->x[i] - P->xl[i])) : 0.0;
        T->zu[i] = isfinite(P->xu[i]) ? fmax(-r, mu0 / (P->xu[i] - T->x[i])) : 0.0;
    }
    double th0 = nrm1(m, S->c);
    int keep = 1;
    if (S->wstage == 2) {
        double e_warm = kkt_error(P, T, S->g, S->c, S->J, S->o.warm_mu0, &S->o, S->wk);
        keep = e_warm <= S->e_cold;
    }
    if (keep) {
        T->theta_max = 1e4 * fmax(1.0, th0);
        T->theta_min = 1e-4 * fmax(1.0, th0);
    } else {
        /* rejected by the gate: the cold start of the previous pass */
        cold_point(S);
        memcpy(T->y, S->y_cold, m * sizeof(double));
        T->theta_max = S->thmax_cold;
        T->theta_min = S->thmin_cold;
        S->warm = 0;
        S->st_warm_rejected++;
    }
    T->nf = 0;
    S->wstage = 0;
    S->init_filter = 0;
    S->phase = PH_REGULAR;
}

/* Gate, first pass done (least-squares y at the cold start): record E_mu0 of the cold start and
 * move to the warm point (the phase stays INIT_Y) */
static void gate_cold_done(solver_t* S) {
    nlp_t* P = S->P;
    sub_t* T = &S->main;
    int m = P->m;
    eval_point(S, P, T);
    S->e_cold = kkt_error(P, T, S->g, S->c, S->J, S->o.warm_mu0, &S->o, S->wk);
    memcpy(S->y_cold, T->y, m * sizeof(double));
    S->thmax_cold = T->theta_max;
    S->thmin_cold = T->theta_min;
    warm_point(S);
    S->warm = 1;
    S->wstage = 2;
}

/* a warm start that diverged (it needs restoration, or runs past warm_iter_cap iterations)
 * starts again from the cold start; the iteration count carries on */
static void cold_restart(solver_t* S) {
    cold_point(S);
    S->mu_free = 1;
    S->n_refs = 0;
    S->mu_max = 0.0;
    S->wd_active = 0;
    S->wd_short = 0;
    S->soft = 0;
    S->init_filter = 1;
    S->theta_R = 0.0;
    S->warm = 0;
    S->wstage = 0;
    S->phase = PH_INIT_Y;
    S->st_warm_restarts++;
}

/* enter feasibility restoration (Table I row 6) from the main iterate */
static int resto_enter(solver_t* S) {
    const ipmo_opts* o = &S->o;
    nlp_t* P = S->P;
    sub_t* T = &S->main;
    sub_t* R = &S->rs;
    int n = P->n, m = P->m;
    grow_buffers(S, n + 2 * m);
    eval_point(S, P, T);
    double thk = nrm1(m, S->c);
    double phk = barrier_obj(P, T->x, S->f, T->mu);
    if (thk <= o->tol) return 1;           /* no infeasibility to remove */
    S->wd_active = 0;
    S->wd_short = 0;
    S->soft = 0;
    filter_add(T, (1.0 - o->gamma_theta) * thk, phk - o->gamma_phi * thk);
    S->theta_R = thk;
    double muR = fmax(T->mu, nrmi(m, S->c));
    double rho = o->rho_resto;
    memcpy(S->RU.xR, T->x, n * sizeof(double));
    for (int i = 0; i < n; ++i) {
        double d = fmin(1.0, 1.0 / fabs(T->x[i]));
        S->RU.DR2[i] = d * d;
    }
    memcpy(R->x, T->x, n * sizeof(double));
    for (int r = 0; r < m; ++r) {
        double c = S->c[r];
        double a = (muR - rho * c) / (2.0 * rho);
        double nn = a + sqrt(a * a + muR * c / (2.0 * rho));
        double pp = c + nn;
        R->x[n + r] = pp;
        R->x[n + m + r] = nn;
        R->zl[n + r] = muR / pp;
        R->zl[n + m + r] = muR / nn;
        R->zu[n + r] = R->zu[n + m + r] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        R->zl[i] = isfinite(P->xl[i]) ? fmin(rho, T->zl[i]) : 0.0;
        R->zu[i] = isfinite(P->xu[i]) ? fmin(rho, T->zu[i]) : 0.0;
    }
    memset(R->y, 0, (m > 0 ? m : 1) * sizeof(double));
    R->mu = muR;
    R->tau = fmax(o->tau_min, 1.0 - muR);
    R->dx_last = 0.0;
    R->tiny = 0;
    R->nf = 0;
    S->RP.c(S->RP.ud, R->x, S->ct);
    double th0 = nrm1(m, S->ct);
    R->theta_max = 1e4 * fmax(1.0, th0);
    R->theta_min = 1e-4 * fmax(1.0, th0);
    S->st_resto_entries++;
    return 0;
}

/* Nested hard restoration (Table I row 6): the restoration phase cannot make progress at
 * (x, p, n).  Its own restoration problem -- minimise the violation of c(x) - p + n = 0 -- is
 * solved at once: the elastic pair (p, n) is free in it and enters that constraint linearly, so
 * its minimiser keeps x and takes, for every row, the (p, n) that minimises rho (p + n) -
 * mu (ln p + ln n) subject to c(x) - p + n = 0 (the closed form that starts the restoration phase,
 * at the restoration phase's current mu), with z_p = mu / p, z_n = mu / n.  The failing point enters
 * the restoration filter, as an iterate does when it leaves for restoration.  Counts as a
 * restoration iteration.  Returns 0 (nothing done) when the restoration constraints already hold
 * within tol, i.e. when restoring them cannot help. */
static int nested_resto(solver_t* S) {
    const ipmo_opts* o = &S->o;
    nlp_t* P = S->P;
    sub_t* R = &S->rs;
    int n = P->n, m = P->m;
    double fR;
    S->RP.c(S->RP.ud, R->x, S->ct);
    S->RP.f(S->RP.ud, R->x, &fR);
    double th = nrm1(m, S->ct);
    double ph = barrier_obj(&S->RP, R->x, fR, R->mu);
    if (!(th > o->tol)) return 0;
    filter_add(R, (1.0 - o->gamma_theta) * th, ph - o->gamma_phi * th);
    P->c(P->ud, R->x, S->c);
    double mu = R->mu, rho = o->rho_resto;
    for (int r = 0; r < m; ++r) {
        double c = S->c[r];
        double a = (mu - rho * c) / (2.0 * rho);
        double nn = a + sqrt(a * a + mu * c / (2.0 * rho));
        double pp = c + nn;
        R->x[n + r] = pp;
        R->x[n + m + r] = nn;
        R->zl[n + r] = mu / pp;
        R->zl[n + m + r] = mu / nn;
    }
    S->iter++;
    S->st_resto_iter++;
    S->st_nested++;
    return 1;
}

/* after an accepted restoration step: return to the original problem when the point is
 * acceptable to the original filter and theta <= kappa_resto theta(x_R) */
static int resto_try_exit(solver_t* S) {
    const ipmo_opts* o = &S->o;
    nlp_t* P = S->P;
    sub_t* T = &S->main;
    sub_t* R = &S->rs;
    int n = P->n, m = P->m;
    double f;
    P->c(P->ud, R->x, S->ct);
    P->f(P->ud, R->x, &f);
    double th = nrm1(m, S->ct);
    double ph = barrier_obj(P, R->x, f, T->mu);
    if (!(isfinite(th) && isfinite(ph))) return 0;
    if (!(th <= o->kappa_resto * S->theta_R)) return 0;
    if (!filter_ok(T, th, ph)) return 0;
    memcpy(T->x, R->x, n * sizeof(double));
    double zmax = 0;
    for (int i = 0; i < n; ++i) {
        T->zl[i] = R->zl[i];
        T->zu[i] = R->zu[i];
        if (T->zl[i] > zmax) zmax = T->zl[i];
        if (T->zu[i] > zmax) zmax = T->zu[i];
    }
    if (zmax > o->bound_mult_reset)
        for (int i = 0; i < n; ++i) {
            T->zl[i] = isfinite(P->xl[i]) ? 1.0 : 0.0;
            T->zu[i] = isfinite(P->xu[i]) ? 1.0 : 0.0;
        }
    T->tiny = 0;
    S->n_refs = 0;                           /* the adaptive update restarts its progress record */
    return 1;
}

/* one pass of the phase machine */
static void solver_pass(solver_t* S) {
    S->st_passes++;
    if (S->phase == PH_DONE) return;
    if (S->phase == PH_INIT_Y) {
        if (S->warm) { warm_init_pass(S); return; }
        init_y(S);                                   /* least-squares y at the cold start */
        if (S->wstage == 1) { gate_cold_done(S); return; }
        S->phase = PH_REGULAR;
        return;
    }
    if (S->warm && (S->phase == PH_RESTO || (S->o.warm_iter_cap > 0 && S->iter >= S->o.warm_iter_cap))) {
        cold_restart(S);
        return;
    }
    if (S->phase == PH_REGULAR) {
        int r = core_iter(S, S->P, &S->main, 0);
        switch (r) {
        case R_ACCEPT: return;
        case R_CONVERGED: S->status = ST_CONVERGED; S->phase = PH_DONE; return;
        case R_MAXITER: S->status = ST_MAX_ITER; S->phase = PH_DONE; return;
        case R_NUMERICAL: S->status = ST_NUMERICAL; S->phase = PH_DONE; return;
        default:
            if (resto_enter(S)) { S->status = ST_RESTO_FAILED; S->phase = PH_DONE; return; }
            S->phase = PH_RESTO;
            return;
        }
    }
    if (S->phase == PH_RESTO) {
        int r = core_iter(S, &S->RP, &S->rs, 1);
        switch (r) {
        case R_ACCEPT:
            if (resto_try_exit(S)) S->phase = PH_INIT_Y;
            return;
        case R_CONVERGED: S->status = ST_INFEASIBLE; S->phase = PH_DONE; return;
        case R_MAXITER: S->status = ST_MAX_ITER; S->phase = PH_DONE; return;
        case R_NUMERICAL: S->status = ST_NUMERICAL; S->phase = PH_DONE; return;
        default:
            if (S->o.nested_resto && nested_resto(S)) return;
            S->status = ST_RESTO_FAILED; S->phase = PH_DONE; return;
        }
    }
}


/* evaluation and KKT buffers for a problem with nv variables and m constraints */
static void grow_buffers(solver_t* S, int nv) {
    if (nv <= S->cap_n) return;
    int m = S->P->m, NK = nv + m;
    free(S->g); free(S->J); free(S->Hm); free(S->K); free(S->rhs); free(S->wk); free(S->dx);
    free(S->dzl); free(S->dzu); free(S->dxs); free(S->dzls); free(S->dzus); free(S->xt); free(S->gphi);
    free(S->rx); free(S->perm); free(S->blk);
    free(S->c); free(S->dy); free(S->dys); free(S->ct); free(S->csoc);
    S->g = (double*)calloc(nv, sizeof(double));
    S->J = (double*)calloc((size_t)(m + 1) * nv, sizeof(double));
    S->Hm = (double*)calloc((size_t)nv * nv, sizeof(double));
    S->K = (double*)calloc((size_t)NK * NK, sizeof(double));
    S->rhs = (double*)calloc(NK, sizeof(double));
    S->wk = (double*)calloc(NK, sizeof(double));
    S->dx = (double*)calloc(nv, sizeof(double));
    S->dzl = (double*)calloc(nv, sizeof(double));
    S->dzu = (double*)calloc(nv, sizeof(double));
    S->dxs = (double*)calloc(nv, sizeof(double));
    S->dzls = (double*)calloc(nv, sizeof(double));
    S->dzus = (double*)calloc(nv, sizeof(double));
    S->xt = (double*)calloc(nv, sizeof(double));
    S->gphi = (double*)calloc(nv, sizeof(double));
    S->rx = (double*)calloc(nv, sizeof(double));
    S->perm = (int*)calloc(NK, sizeof(int));
    S->blk = (int*)calloc(NK, sizeof(int));
    S->c = (double*)calloc(m + 1, sizeof(double));
    S->dy = (double*)calloc(m + 1, sizeof(double));
    S->dys = (double*)calloc(m + 1, sizeof(double));
    S->ct = (double*)calloc(m + 1, sizeof(double));
    S->csoc = (double*)calloc(m + 1, sizeof(double));
    S->cap_n = nv;
}

/* ------------------------------------------------------------------ */
/* x_cold: the cold starting point; x_warm / y_warm (or NULL): a warm point (all n primal
 * values) and its equality multipliers.  A warm point with a non-finite entry is rejected and the
 * solve starts cold. */
static solver_t* solver_new(nlp_t* P, const ipmo_opts* o, const double* x_cold, const double* x_warm,
                            const double* y_warm) {
    solver_t* S = (solver_t*)calloc(1, sizeof(solver_t));
    S->P = P;
    S->o = *o;
    int n = P->n, m = P->m;
    int NR = n + 2 * m;                 /* restoration variables */
    sub_alloc(&S->main, n, m);
    sub_alloc(&S->rs, NR, m);
    S->scap = o->max_iter + 2;
    S->cap_n = 0;
    grow_buffers(S, n);                 /* grown to the restoration size on first entry */
    /* restoration NLP */
    resto_ud* U = &S->RU;
    U->P = P; U->n = n; U->m = m; U->rho = o->rho_resto;
    U->xR = (double*)calloc(n, sizeof(double));
    U->DR2 = (double*)calloc(n, sizeof(double));
    U->xl = (double*)calloc(NR, sizeof(double));
    U->xu = (double*)calloc(NR, sizeof(double));
    U->Jb = (double*)calloc((size_t)(m + 1) * n, sizeof(double));
    U->Hb = (double*)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i) { U->xl[i] = P->xl[i]; U->xu[i] = P->xu[i]; }
    for (int i = n; i < NR; ++i) { U->xl[i] = 0.0; U->xu[i] = INFINITY; }
    S->RP.n = NR; S->RP.m = m; S->RP.xl = U->xl; S->RP.xu = U->xu; S->RP.ud = U;
    S->RP.f = r_f; S->RP.grad = r_grad; S->RP.c = r_c; S->RP.jac = r_jac; S->RP.hess = r_hess;
    S->sf_y = (double*)calloc(m > 0 ? m : 1, sizeof(double));
    S->sf_zl = (double*)calloc(n, sizeof(double));
    S->sf_zu = (double*)calloc(n, sizeof(double));
    S->sf_g = (double*)calloc(n, sizeof(double));
    S->sf_J = (double*)calloc((size_t)(m > 0 ? m : 1) * n, sizeof(double));
    S->wd_x = (double*)calloc(n, sizeof(double));
    S->wd_y = (double*)calloc(m > 0 ? m : 1, sizeof(double));
    S->wd_zl = (double*)calloc(n, sizeof(double));
    S->wd_zu = (double*)calloc(n, sizeof(double));
    S->x_cold = (double*)malloc(n * sizeof(double));
    S->y_cold = (double*)calloc(m > 0 ? m : 1, sizeof(double));
    memcpy(S->x_cold, x_cold, n * sizeof(double));
    S->soc_c = (double*)calloc((size_t)(o->max_soc > 0 ? o->max_soc : 1) * (m > 0 ? m : 1), sizeof(double));
    S->soc_d = (double*)calloc((size_t)(o->max_soc > 0 ? o->max_soc : 1) * NR, sizeof(double));
    S->soc_th = (double*)calloc(o->max_soc > 0 ? o->max_soc : 1, sizeof(double));
    int use_warm = x_warm != NULL && y_warm != NULL;
    if (use_warm) {
        for (int i = 0; i < n; ++i) if (!isfinite(x_warm[i])) use_warm = 0;
        for (int r = 0; r < m; ++r) if (!isfinite(y_warm[r])) use_warm = 0;
        if (use_warm) {
            S->warm_w = (double*)malloc(n * sizeof(double));
            S->warm_y = (double*)calloc(m > 0 ? m : 1, sizeof(double));
            memcpy(S->warm_w, x_warm, n * sizeof(double));
            memcpy(S->warm_y, y_warm, m * sizeof(double));
            S->st_warm_started = 1;
        } else {
            S->st_warm_rejected = 1;
        }
    }
    S->phase = PH_INIT_Y;
    S->status = ST_RUNNING;
    S->init_filter = 1;
    S->mu_free = 1;
    if (use_warm && !o->warm_gate) {
        warm_point(S);
        S->warm = 1;
    } else {
        cold_point(S);
        if (use_warm) S->wstage = 1;    /* the gate's cold reference first */
    }
    return S;
}

static void solver_free(solver_t* S) {
    if (!S) return;
    sub_free(&S->main); sub_free(&S->rs);
    free(S->g); free(S->c); free(S->J); free(S->Hm); free(S->K); free(S->rhs); free(S->wk);
    free(S->dx); free(S->dy); free(S->dzl); free(S->dzu); free(S->dxs); free(S->dys); free(S->dzls);
    free(S->dzus); free(S->xt); free(S->ct); free(S->csoc); free(S->gphi); free(S->rx);
    free(S->perm); free(S->blk);
    free(S->RU.xR); free(S->RU.DR2); free(S->RU.xl); free(S->RU.xu); free(S->RU.Jb); free(S->RU.Hb);
    free(S->x_cold); free(S->y_cold); free(S->warm_w); free(S->warm_y);
    free(S->soc_c); free(S->soc_d); free(S->soc_th);
    free(S->wd_x); free(S->wd_y); free(S->wd_zl); free(S->wd_zu);
    free(S->sf_y); free(S->sf_zl); free(S->sf_zu); free(S->sf_g); free(S->sf_J);
    free(S);
}

static void solver_run(solver_t* S) {
    while (S->phase != PH_DONE) solver_pass(S);
}

/* =================================================================== */
/* exported C ABI (host pointers only)                                  */
/* =================================================================== */
void ipmo_default_opts(ipmo_opts* o) {
    o->tol = 1e-8; o->max_iter = 1000; o->mu_init = 0.1; o->kappa_eps = 10.0; o->kappa_mu = 0.2;
    o->theta_mu = 1.5; o->tau_min = 0.99; o->kappa1 = 1e-2; o->kappa2 = 1e-2; o->lam_max = 1e3;
    o->s_max = 100.0; o->delta_min = 1e-20; o->delta_0 = 1e-4; o->delta_max = 1e40;
    o->delta_c_bar = 1e-8; o->kappa_c = 0.25; o->kappa_minus = 1.0 / 3.0; o->kappa_plus = 8.0;
    o->kappa_plus_bar = 100.0; o->gamma_theta = 1e-5; o->gamma_phi = 1e-8; o->delta_sw = 1.0;
    o->s_theta = 1.1; o->s_phi = 2.3; o->eta_phi = 1e-8; o->gamma_alpha = 0.05; o->max_soc = 4;
    o->kappa_soc = 0.99; o->kappa_sigma = 1e10; o->rho_resto = 1000.0; o->kappa_resto = 0.9;
    o->bound_mult_reset = 1e3;
    o->warm_mu0 = 1e-3; o->warm_push = 1e-3; o->warm_iter_cap = 0; o->warm_gate = 1;
    o->watchdog_trigger = 0; o->watchdog_max = 3;
    o->soft_resto_max = 0; o->soft_resto_factor = 0.9999;
    o->mu_strategy = 0;
    o->nested_resto = 1;
    o->resto_ls_max = 60;
}

int ipmo_sizeof_opts(void) { return (int)sizeof(ipmo_opts); }
int ipmo_sizeof_desc(void) { return (int)sizeof(ipmo_quad_desc); }

int ipmo_bk_factor(int n, double* A, int* perm, int* blk, int* inertia) { return bk_factor(n, A, perm, blk, inertia); }
void ipmo_bk_solve(int n, const double* F, const int* perm, const int* blk, double* b) {
    double* w = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    bk_solve(n, F, perm, blk, b, w);
    free(w);
}

/* outputs of one solve */
typedef struct {
    double* x; double* y; double* zl; double* zu; double* obj; double* kkt; int32_t* status; int32_t* iters;
    int32_t* stats; /* NSTAT ints per instance */
} outs_t;
#define NSTAT 17

static void write_outputs(solver_t* S, int idx, const outs_t* O) {
    nlp_t* P = S->P;
    int n = P->n, m = P->m;
    sub_t* T = &S->main;
    if (O->x) memcpy(O->x + (size_t)idx * n, T->x, n * sizeof(double));
    if (O->y) memcpy(O->y + (size_t)idx * m, T->y, m * sizeof(double));
    if (O->zl) memcpy(O->zl + (size_t)idx * n, T->zl, n * sizeof(double));
    if (O->zu) memcpy(O->zu + (size_t)idx * n, T->zu, n * sizeof(double));
    if (O->obj || O->kkt) {
        eval_point(S, P, T);
        if (O->obj) O->obj[idx] = S->f;
        if (O->kkt) O->kkt[idx] = kkt_error(P, T, S->g, S->c, S->J, 0.0, &S->o, S->wk);
    }
    if (O->status) O->status[idx] = S->status;
    if (O->iters) O->iters[idx] = S->iter;
    if (O->stats) {
        int32_t* s = O->stats + (size_t)idx * NSTAT;
        s[0] = S->iter; s[1] = S->st_resto_iter; s[2] = S->st_soc_try; s[3] = S->st_soc_acc;
        s[4] = S->st_fact; s[5] = S->st_resto_entries; s[6] = S->st_tiny; s[7] = S->st_passes;
        s[8] = S->st_warm_started; s[9] = S->st_warm_rejected; s[10] = S->st_warm_restarts;
        s[11] = S->st_wd_starts; s[12] = S->st_wd_reverts; s[13] = S->st_soft_steps; s[14] = S->st_soft_fails;
        s[15] = S->st_mu_fallbacks;
        s[16] = S->st_nested;
    }
}

typedef struct {
    const ipmo_quad_desc* d;
    const ipmo_opts* o;
    int n_inst, n_theta, n;
    const double* theta;
    const double* warm;     /* [n_inst][n_w + m] rows (w, y), or NULL */
    outs_t O;
    int next;
    pthread_mutex_t lock;
} batch_t;

static void solve_one_quad(batch_t* B, int i) {
    nlp_t P;
    const double* th = B->theta + (size_t)i * B->n_theta;
    void* Q = quad_nlp_new(B->d, th, &P);
    double* x0 = (double*)malloc(P.n * sizeof(double));
    double* xw = (double*)malloc(P.n * sizeof(double));
    quad_cold_start(B->d, th, x0);
    const double* row = B->warm ? B->warm + (size_t)i * (quad_nw(B->d) + P.m) : NULL;
    if (row) quad_warm_point(B->d, th, row, xw);
    solver_t* S = solver_new(&P, B->o, x0, row ? xw : NULL, row ? row + quad_nw(B->d) : NULL);
    solver_run(S);
    write_outputs(S, i, &B->O);
    solver_free(S);
    free(x0);
    free(xw);
    quad_nlp_free(Q);
}

static void* batch_worker(void* arg) {
    batch_t* B = (batch_t*)arg;
    for (;;) {
        pthread_mutex_lock(&B->lock);
        int i = B->next++;
        pthread_mutex_unlock(&B->lock);
        if (i >= B->n_inst) break;
        solve_one_quad(B, i);
    }
    return NULL;
}

static int desc_n_theta(const ipmo_quad_desc* d) {
    if (d->family == 0) return 16 + 4 * d->n_obs;
    if (d->family == 1) return 15 + 4 * d->n_obs;
    if (d->family == 3) return 15 + 7 * d->n_obs;
    return 16 * d->n_agents;
}

/* Solve n_inst quadrotor NMPC instances with `threads` workers: cold start, or warm from the rows
 * of `warm` ([n_inst][n_w + m]: primal w without slacks, then the equality multipliers y). */
int ipmo_solve_quad(const ipmo_quad_desc* d, const ipmo_opts* o, int n_inst, const double* theta,
                    const double* warm, int threads, double* x, double* y, double* zl, double* zu,
                    double* obj, double* kkt, int32_t* status, int32_t* iters, int32_t* stats) {
    batch_t B;
    memset(&B, 0, sizeof(B));
    B.d = d; B.o = o; B.n_inst = n_inst; B.n_theta = desc_n_theta(d); B.theta = theta;
    B.warm = warm;
    B.O.x = x; B.O.y = y; B.O.zl = zl; B.O.zu = zu; B.O.obj = obj; B.O.kkt = kkt;
    B.O.status = status; B.O.iters = iters; B.O.stats = stats;
    pthread_mutex_init(&B.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > n_inst) threads = n_inst;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (threads > 0 ? threads : 1));
    for (int t = 0; t < threads; ++t) pthread_create(&th[t], NULL, batch_worker, &B);
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&B.lock);
    return 0;
}

/* ------------------------------------------------------------------ */
/* handle API: pass-by-pass stepping and flat state export/import for the
 * one-step replay test (Sec. VI "Correctness") */
typedef struct {
    nlp_t P;
    void* Q;          /* quad user data, or NULL for a generic problem */
    solver_t* S;
} handle_t;

/* one instance; warm_row (or NULL): [n_w + m] = (w, y) as in ipmo_solve_quad */
void* ipmo_create_quad(const ipmo_quad_desc* d, const ipmo_opts* o, const double* theta, const double* warm_row) {
    handle_t* Hd = (handle_t*)calloc(1, sizeof(handle_t));
    Hd->Q = quad_nlp_new(d, theta, &Hd->P);
    double* x0 = (double*)malloc(Hd->P.n * sizeof(double));
    double* xw = (double*)malloc(Hd->P.n * sizeof(double));
    quad_cold_start(d, theta, x0);
    if (warm_row) quad_warm_point(d, theta, warm_row, xw);
    Hd->S = solver_new(&Hd->P, o, x0, warm_row ? xw : NULL, warm_row ? warm_row + quad_nw(d) : NULL);
    free(x0);
    free(xw);
    return Hd;
}

/* generic problem from callbacks; xl/xu are copied */
void* ipmo_create_generic(int n, int m, const double* xl, const double* xu,
                          void (*f)(void*, const double*, double*), void (*grad)(void*, const double*, double*),
                          void (*c)(void*, const double*, double*), void (*jac)(void*, const double*, double*),
                          void (*hess)(void*, const double*, double, const double*, double*),
                          const ipmo_opts* o, const double* x0) {
    handle_t* Hd = (handle_t*)calloc(1, sizeof(handle_t));
    double* l = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    double* u = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    memcpy(l, xl, n * sizeof(double));
    memcpy(u, xu, n * sizeof(double));
    Hd->P.n = n; Hd->P.m = m; Hd->P.xl = l; Hd->P.xu = u; Hd->P.ud = NULL;
    Hd->P.f = f; Hd->P.grad = grad; Hd->P.c = c; Hd->P.jac = jac; Hd->P.hess = hess;
    Hd->S = solver_new(&Hd->P, o, x0, NULL, NULL);
    return Hd;
}

void ipmo_destroy(void* h) {
    handle_t* Hd = (handle_t*)h;
    if (!Hd) return;
    solver_free(Hd->S);
    if (Hd->Q) quad_nlp_free(Hd->Q);
    else { free((void*)Hd->P.xl); free((void*)Hd->P.xu); }
    free(Hd);
}

int ipmo_pass(void* h) { handle_t* Hd = (handle_t*)h; solver_pass(Hd->S); return Hd->S->phase; }
int ipmo_run(void* h) { handle_t* Hd = (handle_t*)h; solver_run(Hd->S); return Hd->S->status; }
int ipmo_phase(void* h) { return ((handle_t*)h)->S->phase; }
int ipmo_status(void* h) { return ((handle_t*)h)->S->status; }
int ipmo_iter(void* h) { return ((handle_t*)h)->S->iter; }

void ipmo_outputs(void* h, double* x, double* y, double* zl, double* zu, double* obj, double* kkt,
                  int32_t* status, int32_t* iters, int32_t* stats) {
    handle_t* Hd = (handle_t*)h;
    outs_t O = {x, y, zl, zu, obj, kkt, status, iters, stats};
    write_outputs(Hd->S, 0, &O);
}

/* last pass diagnostics: [delta_x, delta_c, alpha_primal, alpha_dual, soc_accepted, mu, tau, nf] */
void ipmo_last_info(void* h, double* out) {
    solver_t* S = ((handle_t*)h)->S;
    sub_t* T = S->phase == PH_RESTO ? &S->rs : &S->main;
    out[0] = S->last_dx; out[1] = S->last_dc; out[2] = S->last_alpha; out[3] = S->last_alpha_z;
    out[4] = S->last_soc; out[5] = T->mu; out[6] = T->tau; out[7] = T->nf;
}

/* Flat state (FP64), field order:
 *   header[16] = phase, iter, status, init_filter, theta_R, warm, wstage, 0...
 *   main sub-state  : mu, tau, dx_last, theta_max, theta_min, tiny, nf, 0 | x[n] y[m] zl[n] zu[n] | fth[F] fph[F]
 *   resto sub-state : same with n_R = n + 2m variables
 *   x_R[n], DR2[n]
 *   watchdog: short, active, iter, theta, phi, grad phi^T d, alpha_max, mu | x[n] y[m] zl[n] zu[n]
 *   soft restoration: active, steps taken, theta, phi of its starting point
 *   adaptive barrier update: free mode, references held, references[4], mu_max, 0
 * F = max_iter + 2 filter pairs: every entry of the original problem's filter comes from an
 * accepted iteration or a restoration entry (each entry but the last followed by an accepted
 * restoration iteration), every entry of the restoration filter from an accepted restoration
 * iteration, so neither holds more than max_iter + 1 pairs. */
static int sub_len(const solver_t* S, const sub_t* T) { return 8 + 3 * T->n + T->m + 2 * S->scap; }

int ipmo_state_len(void* h) {
    solver_t* S = ((handle_t*)h)->S;
    return 16 + sub_len(S, &S->main) + sub_len(S, &S->rs) + 2 * S->P->n + 8 + 3 * S->P->n + S->P->m + 4 + 8;
}

static double* sub_put(const solver_t* S, const sub_t* T, double* p) {
    p[0] = T->mu; p[1] = T->tau; p[2] = T->dx_last; p[3] = T->theta_max; p[4] = T->theta_min;
    p[5] = T->tiny; p[6] = T->nf; p[7] = 0; p += 8;
    memcpy(p, T->x, T->n * sizeof(double)); p += T->n;
    memcpy(p, T->y, T->m * sizeof(double)); p += T->m;
    memcpy(p, T->zl, T->n * sizeof(double)); p += T->n;
    memcpy(p, T->zu, T->n * sizeof(double)); p += T->n;
    for (int i = 0; i < S->scap; ++i) p[i] = i < T->nf ? T->fth[i] : 0.0;
    p += S->scap;
    for (int i = 0; i < S->scap; ++i) p[i] = i < T->nf ? T->fph[i] : 0.0;
    return p + S->scap;
}
static const double* sub_get(const solver_t* S, sub_t* T, const double* p) {
    T->mu = p[0]; T->tau = p[1]; T->dx_last = p[2]; T->theta_max = p[3]; T->theta_min = p[4];
    T->tiny = (int)p[5]; T->nf = (int)p[6]; p += 8;
    memcpy(T->x, p, T->n * sizeof(double)); p += T->n;
    memcpy(T->y, p, T->m * sizeof(double)); p += T->m;
    memcpy(T->zl, p, T->n * sizeof(double)); p += T->n;
    memcpy(T->zu, p, T->n * sizeof(double)); p += T->n;
    if (T->fcap < S->scap) {
        T->fcap = S->scap;
        T->fth = (double*)realloc(T->fth, (size_t)T->fcap * sizeof(double));
        T->fph = (double*)realloc(T->fph, (size_t)T->fcap * sizeof(double));
    }
    memcpy(T->fth, p, S->scap * sizeof(double)); p += S->scap;
    memcpy(T->fph, p, S->scap * sizeof(double));
    return p + S->scap;
}

void ipmo_state_get(void* h, double* out) {
    solver_t* S = ((handle_t*)h)->S;
    memset(out, 0, 16 * sizeof(double));
    out[0] = S->phase; out[1] = S->iter; out[2] = S->status; out[3] = S->init_filter; out[4] = S->theta_R;
    out[5] = S->warm; out[6] = S->wstage;
    double* p = sub_put(S, &S->main, out + 16);
    p = sub_put(S, &S->rs, p);
    int n = S->P->n, m = S->P->m;
    memcpy(p, S->RU.xR, n * sizeof(double)); p += n;
    memcpy(p, S->RU.DR2, n * sizeof(double)); p += n;
    p[0] = S->wd_short; p[1] = S->wd_active; p[2] = S->wd_iter; p[3] = S->wd_thk; p[4] = S->wd_phk;
    p[5] = S->wd_gphi; p[6] = S->wd_amax; p[7] = S->wd_mu; p += 8;
    memcpy(p, S->wd_x, n * sizeof(double)); p += n;
    memcpy(p, S->wd_y, m * sizeof(double)); p += m;
    memcpy(p, S->wd_zl, n * sizeof(double)); p += n;
    memcpy(p, S->wd_zu, n * sizeof(double)); p += n;
    p[0] = S->soft; p[1] = S->soft_iter; p[2] = S->soft_thk; p[3] = S->soft_phk; p += 4;
    p[0] = S->mu_free; p[1] = S->n_refs;
    for (int i = 0; i < 4; ++i) p[2 + i] = S->refs[i];
    p[6] = S->mu_max; p[7] = 0.0;
}

/* load a flat state (a warm start's gate data are not part of it: load states of cold solves) */
void ipmo_state_set(void* h, const double* in) {
    solver_t* S = ((handle_t*)h)->S;
    grow_buffers(S, S->P->n + 2 * S->P->m);     /* the state may be in the restoration phase */
    S->phase = (int)in[0]; S->iter = (int)in[1]; S->status = (int)in[2]; S->init_filter = (int)in[3];
    S->theta_R = in[4];
    S->warm = (int)in[5]; S->wstage = (int)in[6];
    const double* p = sub_get(S, &S->main, in + 16);
    p = sub_get(S, &S->rs, p);
    int n = S->P->n, m = S->P->m;
    memcpy(S->RU.xR, p, n * sizeof(double)); p += n;
    memcpy(S->RU.DR2, p, n * sizeof(double)); p += n;
    S->wd_short = (int)p[0]; S->wd_active = (int)p[1]; S->wd_iter = (int)p[2]; S->wd_thk = p[3];
    S->wd_phk = p[4]; S->wd_gphi = p[5]; S->wd_amax = p[6]; S->wd_mu = p[7]; p += 8;
    memcpy(S->wd_x, p, n * sizeof(double)); p += n;
    memcpy(S->wd_y, p, m * sizeof(double)); p += m;
    memcpy(S->wd_zl, p, n * sizeof(double)); p += n;
    memcpy(S->wd_zu, p, n * sizeof(double)); p += n;
    S->soft = (int)p[0]; S->soft_iter = (int)p[1]; S->soft_thk = p[2]; S->soft_phk = p[3]; p += 4;
    S->mu_free = (int)p[0]; S->n_refs = (int)p[1];
    for (int i = 0; i < 4; ++i) S->refs[i] = p[2 + i];
    S->mu_max = p[6];
}

/* E_mu of the original problem at an arbitrary primal-dual point (used to re-check GPU results) */
double ipmo_quad_kkt_error(const ipmo_quad_desc* d, const ipmo_opts* o, const double* theta, const double* x,
                           const double* y, const double* zl, const double* zu, double mu) {
    nlp_t P;
    void* Q = quad_nlp_new(d, theta, &P);
    sub_t T;
    T.n = P.n; T.m = P.m;
    T.x = (double*)x; T.y = (double*)y; T.zl = (double*)zl; T.zu = (double*)zu;
    double* g = (double*)malloc(P.n * sizeof(double));
    double* c = (double*)malloc((P.m + 1) * sizeof(double));
    double* J = (double*)malloc((size_t)(P.m + 1) * P.n * sizeof(double));
    double* wk = (double*)malloc(P.n * sizeof(double));
    P.grad(P.ud, x, g);
    P.c(P.ud, x, c);
    P.jac(P.ud, x, J);
    double e = kkt_error(&P, &T, g, c, J, mu, o, wk);
    free(g); free(c); free(J); free(wk);
    quad_nlp_free(Q);
    return e;
}

/* Newton direction of the last regular pass (dx[n], dy[m], dzl[n], dzu[n]) and the gradient of
 * the barrier objective used for it (for the eq. (6) == eq. (7) + elimination invariant test) */
void ipmo_last_step(void* h, double* dx, double* dy, double* dzl, double* dzu) {
    solver_t* S = ((handle_t*)h)->S;
    int n = S->P->n, m = S->P->m;
    memcpy(dx, S->dx, n * sizeof(double));
    memcpy(dy, S->dy, m * sizeof(double));
    memcpy(dzl, S->dzl, n * sizeof(double));
    memcpy(dzu, S->dzu, n * sizeof(double));
}

/* f, grad f, c, dense Jacobian (m x n) and dense Hessian of objf f + y^T c at v (any may be NULL) */
void ipmo_quad_eval(const ipmo_quad_desc* d, const double* theta, const double* v, const double* y, double objf,
                    double* f, double* g, double* c, double* J, double* Hm) {
    nlp_t P;
    void* Q = quad_nlp_new(d, theta, &P);
    if (f) P.f(P.ud, v, f);
    if (g) P.grad(P.ud, v, g);
    if (c) P.c(P.ud, v, c);
    if (J) P.jac(P.ud, v, J);
    if (Hm) P.hess(P.ud, v, objf, y, Hm);
    quad_nlp_free(Q);
}


/* ------------------------------------------------------------------ */
/* pieces of the method on plain arrays, for hand-computed pins          */
double ipmo_ftb_primal(int n, const double* x, const double* dx, const double* xl, const double* xu, double tau) {
    nlp_t P;
    memset(&P, 0, sizeof(P));
    P.n = n; P.xl = xl; P.xu = xu;
    return ftb_primal(&P, x, dx, tau);
}

double ipmo_ftb_dual(int n, const double* zl, const double* zu, const double* dzl, const double* dzu,
                     const double* xl, const double* xu, double tau) {
    nlp_t P;
    memset(&P, 0, sizeof(P));
    P.n = n; P.xl = xl; P.xu = xu;
    return ftb_dual(&P, zl, zu, dzl, dzu, tau);
}

/* acceptance of a trial point against filter entries (fth, fph)[nf] and theta_max / theta_min;
 * out[0] = accepted, out[1] = switching condition, out[2] = Armijo condition */
void ipmo_acceptable(const ipmo_opts* o, double theta_max, double theta_min, int nf, const double* fth,
                     const double* fph, double thk, double phk, double gphi, double alpha, double tht, double pht,
                     int32_t* out) {
    sub_t T;
    memset(&T, 0, sizeof(T));
    T.theta_max = theta_max; T.theta_min = theta_min; T.nf = nf;
    T.fth = (double*)fth; T.fph = (double*)fph;
    int sw = -1, arm = -1;
    out[0] = acceptable(&T, o, thk, phk, gphi, alpha, tht, pht, &sw, &arm);
    out[1] = sw; out[2] = arm;
}

double ipmo_alpha_min(const ipmo_opts* o, double thk, double gphi, double theta_min) {
    return alpha_min(o, thk, gphi, theta_min);
}

/* E_mu of the handle's current original-problem iterate */
/* the unperturbed matrix of eq. (7) (delta_x = delta_c = 0) of the sub-problem the current phase
 * works on (the restoration problem in PH_RESTO), at the current iterate and mu, written in full
 * (both triangles) into K [N][N]; returns N = n_v + m (0 outside the regular and restoration
 * phases).  For conditioning checks in the tests. */
int ipmo_kkt_dense(void* h, double* K) {
    solver_t* S = ((handle_t*)h)->S;
    if (S->phase != PH_REGULAR && S->phase != PH_RESTO) return 0;
    const int is_resto = S->phase == PH_RESTO;
    const nlp_t* P = is_resto ? &S->RP : S->P;
    sub_t* T = is_resto ? &S->rs : &S->main;
    grow_buffers(S, S->P->n + 2 * S->P->m);
    set_zeta(S, T, is_resto);
    eval_point(S, P, T);
    P->hess(P->ud, T->x, 1.0, T->y, S->Hm);
    int N = P->n + P->m;
    assemble_K(P, T, S->Hm, S->J, 0.0, 0.0, K);
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) K[(size_t)i * N + j] = K[(size_t)j * N + i];
    return N;
}

double ipmo_handle_kkt_error(void* h, double mu) {
    solver_t* S = ((handle_t*)h)->S;
    eval_point(S, S->P, &S->main);
    return kkt_error(S->P, &S->main, S->g, S->c, S->J, mu, &S->o, S->wk);
}

/* the second-order corrections of the last pass: returns their number; c_soc [k][m], step [k][n_v]
 * (n_v the variables of the phase's problem), theta of each corrected trial point */
int ipmo_last_soc(void* h, double* csoc, double* dxs, double* th) {
    solver_t* S = ((handle_t*)h)->S;
    int nmax = S->P->n + 2 * S->P->m, mm = S->P->m > 0 ? S->P->m : 1;
    for (int k = 0; k < S->soc_n; ++k) {
        if (csoc) memcpy(csoc + (size_t)k * S->P->m, S->soc_c + (size_t)k * mm, S->P->m * sizeof(double));
        if (dxs) memcpy(dxs + (size_t)k * nmax, S->soc_d + (size_t)k * nmax, nmax * sizeof(double));
        if (th) th[k] = S->soc_th[k];
    }
    return S->soc_n;
}
