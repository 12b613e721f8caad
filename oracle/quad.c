/*
 * CPU FP64 ORACLE -- test infrastructure only (see oracle.h).
 *
 * Quadrotor multiple-shooting NMPC transcription of the parametric NLP of
 * Sec. III eq. (1): decision vector v = (w, s) with
 *   w = (x_0, u_0, x_1, u_1, ..., x_{N-1}, u_{N-1}, x_N)   (stage-interleaved)
 *   s = inequality slacks, (k = 1..N) x (row j)
 * constraints c = [x_0 - xbar0 ; x_{k+1} - F(x_k, u_k), k = 0..N-1 ; g_kj(x_k) - s_kj]
 * (general inequalities enter through slacks, Sec. III) and bounds
 * 0 <= u <= 2 u_hover, s >= 0, every other component free.
 *
 * The 13-state rigid body (Sec. VI: position, attitude quaternion, linear and
 * angular velocity) is integrated with classical RK4 under zero-order hold.
 * All first and second derivatives come from hyper-dual numbers
 * (a + b e1 + c e2 + d e1 e2, e1^2 = e2^2 = 0): seeding e1 along z_i and e2
 * along z_j gives dF/dz_i in b and d2F/dz_i dz_j in d, exactly (no truncation).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct { double a, b, c, d; } hd;

static inline hd H(double a) { hd r = {a, 0, 0, 0}; return r; }
static inline hd hadd(hd x, hd y) { hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; return r; }
static inline hd hsub(hd x, hd y) { hd r = {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d}; return r; }
static inline hd hmul(hd x, hd y) {
    hd r = {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a,
            x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a};
    return r;
}
static inline hd hsc(double s, hd x) { hd r = {s * x.a, s * x.b, s * x.c, s * x.d}; return r; }

typedef struct {
    double mass, jxx, jyy, jzz, arm, ctau, grav;
} qparams;

/* continuous rigid-body dynamics xdot = f(x, u) (one agent, 13 states, 4 thrusts) */
static void quad_f(const qparams* P, const hd* x, const hd* u, hd* xd) {
    const hd *q = x + 3, *v = x + 7, *w = x + 10;
    (void)v;
    /* pdot = v (world frame) */
    xd[0] = x[7]; xd[1] = x[8]; xd[2] = x[9];
    /* qdot = 1/2 q (x) (0, omega) */
    xd[3] = hsc(0.5, hsub(hsub(hsc(-1.0, hmul(q[1], w[0])), hmul(q[2], w[1])), hmul(q[3], w[2])));
    xd[4] = hsc(0.5, hsub(hadd(hmul(q[0], w[0]), hmul(q[2], w[2])), hmul(q[3], w[1])));
    xd[5] = hsc(0.5, hsub(hadd(hmul(q[0], w[1]), hmul(q[3], w[0])), hmul(q[1], w[2])));
    xd[6] = hsc(0.5, hsub(hadd(hmul(q[0], w[2]), hmul(q[1], w[1])), hmul(q[2], w[0])));
    /* vdot = R(q) (0, 0, T)/m - (0, 0, g); third column of the unit-quaternion rotation */
    hd T = hadd(hadd(u[0], u[1]), hadd(u[2], u[3]));
    hd Tm = hsc(1.0 / P->mass, T);
    hd r13 = hsc(2.0, hadd(hmul(q[1], q[3]), hmul(q[0], q[2])));
    hd r23 = hsc(2.0, hsub(hmul(q[2], q[3]), hmul(q[0], q[1])));
    hd r33 = hsub(H(1.0), hsc(2.0, hadd(hmul(q[1], q[1]), hmul(q[2], q[2]))));
    xd[7] = hmul(r13, Tm);
    xd[8] = hmul(r23, Tm);
    xd[9] = hsub(hmul(r33, Tm), H(P->grav));
    /* omegadot = J^{-1} (tau - omega x J omega), "+" rotor layout */
    hd tx = hsc(P->arm, hsub(u[1], u[3]));
    hd ty = hsc(P->arm, hsub(u[2], u[0]));
    hd tz = hsc(P->ctau, hsub(hadd(u[0], u[2]), hadd(u[1], u[3])));
    xd[10] = hsc(1.0 / P->jxx, hsub(tx, hsc(P->jzz - P->jyy, hmul(w[1], w[2]))));
    xd[11] = hsc(1.0 / P->jyy, hsub(ty, hsc(P->jxx - P->jzz, hmul(w[2], w[0]))));
    xd[12] = hsc(1.0 / P->jzz, hsub(tz, hsc(P->jyy - P->jxx, hmul(w[0], w[1]))));
}

/* classical RK4 over one interval with zero-order-hold inputs */
static void quad_rk4(const qparams* P, double dt, const hd* x, const hd* u, hd* out) {
    hd k1[13], k2[13], k3[13], k4[13], t[13];
    quad_f(P, x, u, k1);
    for (int i = 0; i < 13; ++i) t[i] = hadd(x[i], hsc(0.5 * dt, k1[i]));
    quad_f(P, t, u, k2);
    for (int i = 0; i < 13; ++i) t[i] = hadd(x[i], hsc(0.5 * dt, k2[i]));
    quad_f(P, t, u, k3);
    for (int i = 0; i < 13; ++i) t[i] = hadd(x[i], hsc(dt, k3[i]));
    quad_f(P, t, u, k4);
    for (int i = 0; i < 13; ++i)
        out[i] = hadd(x[i], hsc(dt / 6.0, hadd(hadd(k1[i], hsc(2.0, k2[i])), hadd(hsc(2.0, k3[i]), k4[i]))));
}

/* F, dF/d(x,u) (13 x 17) and sum_r lam_r d2F_r/d(x,u)^2 (17 x 17) for one agent */
static void agent_derivs(const qparams* P, double dt, const double* x, const double* u, const double* lam,
                         double* F, double* G, double* HL) {
    hd z[17], out[13];
    for (int i = 0; i < 17; ++i) z[i] = H(i < 13 ? x[i] : u[i - 13]);
    if (F) {
        quad_rk4(P, dt, z, z + 13, out);
        for (int r = 0; r < 13; ++r) F[r] = out[r].a;
    }
    if (!G && !HL) return;
    for (int i = 0; i < 17; ++i) {
        for (int j = i; j < 17; ++j) {
            if (!HL && j != i) continue;
            for (int t = 0; t < 17; ++t) z[t].b = z[t].c = z[t].d = 0.0;
            z[i].b = 1.0;
            z[j].c = 1.0;
            quad_rk4(P, dt, z, z + 13, out);
            if (G && j == i)
                for (int r = 0; r < 13; ++r) G[r * 17 + i] = out[r].b;
            if (HL) {
                double acc = 0.0;
                for (int r = 0; r < 13; ++r) acc += lam[r] * out[r].d;
                HL[i * 17 + j] = acc;
                HL[j * 17 + i] = acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
typedef struct {
    ipmo_quad_desc d;
    qparams P;
    int nx, nu, nineq, nw, ns, n, m;
    const double* theta;
    double* xl;
    double* xu;
} quad_nlp;

static int xo(const quad_nlp* Q, int k) { return k * (Q->nx + Q->nu); }       /* x_k offset */
static int uo(const quad_nlp* Q, int k) { return k * (Q->nx + Q->nu) + Q->nx; } /* u_k offset */
static int so(const quad_nlp* Q, int k, int j) { return Q->nw + (k - 1) * Q->nineq + j; } /* k >= 1 */
static int go(const quad_nlp* Q, int k, int j) { return (Q->d.N + 1) * Q->nx + (k - 1) * Q->nineq + j; }

/* reference state of agent a at stage k (13) */
static void ref_state(const quad_nlp* Q, int a, int k, double* xr) {
    memset(xr, 0, 13 * sizeof(double));
    xr[3] = 1.0;
    const double* th = Q->theta;
    if (Q->d.family == 0) {
        xr[0] = th[13]; xr[1] = th[14]; xr[2] = th[15];
    } else if (Q->d.family == 1 || Q->d.family == 3) {
        double A = th[13], om = th[14], t = k * Q->d.dt;
        xr[0] = A * sin(om * t);
        xr[1] = 0.5 * A * sin(2.0 * om * t);
        xr[7] = A * om * cos(om * t);
        xr[8] = A * om * cos(2.0 * om * t);
    } else {
        const double* ag = th + a * 16;
        xr[0] = ag[13]; xr[1] = ag[14]; xr[2] = ag[15];
    }
}

static const double* xbar0(const quad_nlp* Q, int a) {
    return Q->d.family == 2 ? Q->theta + a * 16 : Q->theta;
}

/* sphere j at stage k: centre (o[0..2]) and radius (o[3]).  Families 0 and 1 hold fixed spheres
 * (cx, cy, cz, r); family 3 holds spheres moving at constant velocity (cx, cy, cz, r, vx, vy, vz),
 * centre c + t_k v at t_k = k dt (the obstacle trajectories are known in advance). */
static void obs_at(const quad_nlp* Q, int j, int k, double* o) {
    if (Q->d.family == 3) {
        const double* b = Q->theta + 15 + 7 * j;
        double t = k * Q->d.dt;
        for (int i = 0; i < 3; ++i) o[i] = b[i] + t * b[4 + i];
        o[3] = b[3];
    } else {
        const double* b = Q->theta + (Q->d.family == 0 ? 16 : 15) + 4 * j;
        for (int i = 0; i < 4; ++i) o[i] = b[i];
    }
}

/* pair index -> (a, b), a < b */
static void pair_of(int n_agents, int j, int* a, int* b) {
    int t = 0;
    for (int i = 0; i < n_agents; ++i)
        for (int l = i + 1; l < n_agents; ++l) {
            if (t == j) { *a = i; *b = l; return; }
            ++t;
        }
}

/* inequality g_kj(x_k) >= 0 at stage k: value; *pa, *pb = position offsets of the agents involved
 * (*pb < 0 for a sphere) */
static double ineq_val(const quad_nlp* Q, const double* xk, int k, int j, int* pa, int* pb) {
    if (Q->d.family == 2) {
        int a = 0, b = 0;
        pair_of(Q->d.n_agents, j, &a, &b);
        *pa = 13 * a; *pb = 13 * b;
        double s = 0;
        for (int t = 0; t < 3; ++t) { double e = xk[13 * a + t] - xk[13 * b + t]; s += e * e; }
        return s - Q->d.d_min * Q->d.d_min;
    }
    double o[4];
    obs_at(Q, j, k, o);
    *pa = 0; *pb = -1;
    double s = 0;
    for (int t = 0; t < 3; ++t) { double e = xk[t] - o[t]; s += e * e; }
    return s - o[3] * o[3];
}

static void q_f(void* ud, const double* v, double* out) {
    quad_nlp* Q = (quad_nlp*)ud;
    double f = 0, xr[13];
    double uh = Q->P.mass * Q->P.grav / 4.0;
    for (int k = 0; k <= Q->d.N; ++k) {
        for (int a = 0; a < Q->d.n_agents; ++a) {
            ref_state(Q, a, k, xr);
            const double* x = v + xo(Q, k) + 13 * a;
            for (int i = 0; i < 13; ++i) f += Q->d.q_weight * (x[i] - xr[i]) * (x[i] - xr[i]);
            if (k < Q->d.N) {
                const double* u = v + uo(Q, k) + 4 * a;
                for (int i = 0; i < 4; ++i) f += Q->d.r_weight * (u[i] - uh) * (u[i] - uh);
            }
        }
    }
    *out = f;
}

static void q_grad(void* ud, const double* v, double* g) {
    quad_nlp* Q = (quad_nlp*)ud;
    double xr[13];
    double uh = Q->P.mass * Q->P.grav / 4.0;
    memset(g, 0, Q->n * sizeof(double));
    for (int k = 0; k <= Q->d.N; ++k) {
        for (int a = 0; a < Q->d.n_agents; ++a) {
            ref_state(Q, a, k, xr);
            int ox = xo(Q, k) + 13 * a;
            for (int i = 0; i < 13; ++i) g[ox + i] = 2.0 * Q->d.q_weight * (v[ox + i] - xr[i]);
            if (k < Q->d.N) {
                int ou = uo(Q, k) + 4 * a;
                for (int i = 0; i < 4; ++i) g[ou + i] = 2.0 * Q->d.r_weight * (v[ou + i] - uh);
            }
        }
    }
}

static void q_c(void* ud, const double* v, double* c) {
    quad_nlp* Q = (quad_nlp*)ud;
    int nx = Q->nx;
    for (int a = 0; a < Q->d.n_agents; ++a) {
        const double* xb = xbar0(Q, a);
        for (int i = 0; i < 13; ++i) c[13 * a + i] = v[13 * a + i] - xb[i];
    }
    for (int k = 0; k < Q->d.N; ++k) {
        for (int a = 0; a < Q->d.n_agents; ++a) {
            double F[13];
            agent_derivs(&Q->P, Q->d.dt, v + xo(Q, k) + 13 * a, v + uo(Q, k) + 4 * a, NULL, F, NULL, NULL);
            for (int i = 0; i < 13; ++i) c[(k + 1) * nx + 13 * a + i] = v[xo(Q, k + 1) + 13 * a + i] - F[i];
        }
    }
    for (int k = 1; k <= Q->d.N; ++k)
        for (int j = 0; j < Q->nineq; ++j) {
            int pa, pb;
            c[go(Q, k, j)] = ineq_val(Q, v + xo(Q, k), k, j, &pa, &pb) - v[so(Q, k, j)];
        }
}

static void q_jac(void* ud, const double* v, double* J) {
    quad_nlp* Q = (quad_nlp*)ud;
    int n = Q->n, nx = Q->nx;
    memset(J, 0, (size_t)Q->m * n * sizeof(double));
    for (int i = 0; i < nx; ++i) J[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < Q->d.N; ++k) {
        for (int a = 0; a < Q->d.n_agents; ++a) {
            double G[13 * 17];
            agent_derivs(&Q->P, Q->d.dt, v + xo(Q, k) + 13 * a, v + uo(Q, k) + 4 * a, NULL, NULL, G, NULL);
            for (int r = 0; r < 13; ++r) {
                size_t row = (size_t)((k + 1) * nx + 13 * a + r) * n;
                J[row + xo(Q, k + 1) + 13 * a + r] = 1.0;
                for (int t = 0; t < 13; ++t) J[row + xo(Q, k) + 13 * a + t] = -G[r * 17 + t];
                for (int t = 0; t < 4; ++t) J[row + uo(Q, k) + 4 * a + t] = -G[r * 17 + 13 + t];
            }
        }
    }
    for (int k = 1; k <= Q->d.N; ++k)
        for (int j = 0; j < Q->nineq; ++j) {
            int pa, pb;
            const double* xk = v + xo(Q, k);
            ineq_val(Q, xk, k, j, &pa, &pb);
            double o[4];
            obs_at(Q, j, k, o);
            size_t row = (size_t)go(Q, k, j) * n;
            for (int t = 0; t < 3; ++t) {
                if (pb < 0) {
                    J[row + xo(Q, k) + t] = 2.0 * (xk[t] - o[t]);
                } else {
                    double e = xk[pa + t] - xk[pb + t];
                    J[row + xo(Q, k) + pa + t] = 2.0 * e;
                    J[row + xo(Q, k) + pb + t] = -2.0 * e;
                }
            }
            J[row + so(Q, k, j)] = -1.0;
        }
}

static void q_hess(void* ud, const double* v, double objf, const double* y, double* Hm) {
    quad_nlp* Q = (quad_nlp*)ud;
    int n = Q->n, nx = Q->nx;
    memset(Hm, 0, (size_t)n * n * sizeof(double));
    for (int k = 0; k <= Q->d.N; ++k) {
        for (int i = 0; i < nx; ++i) Hm[(size_t)(xo(Q, k) + i) * n + xo(Q, k) + i] += objf * 2.0 * Q->d.q_weight;
        if (k < Q->d.N)
            for (int i = 0; i < Q->nu; ++i) Hm[(size_t)(uo(Q, k) + i) * n + uo(Q, k) + i] += objf * 2.0 * Q->d.r_weight;
    }
    /* dynamics rows x_{k+1} - F(x_k, u_k): Hessian -sum_r y_r d2F_r */
    for (int k = 0; k < Q->d.N; ++k) {
        for (int a = 0; a < Q->d.n_agents; ++a) {
            double HL[17 * 17], lam[13];
            for (int r = 0; r < 13; ++r) lam[r] = -y[(k + 1) * nx + 13 * a + r];
            agent_derivs(&Q->P, Q->d.dt, v + xo(Q, k) + 13 * a, v + uo(Q, k) + 4 * a, lam, NULL, NULL, HL);
            for (int i = 0; i < 17; ++i) {
                int gi = i < 13 ? xo(Q, k) + 13 * a + i : uo(Q, k) + 4 * a + (i - 13);
                for (int j = 0; j < 17; ++j) {
                    int gj = j < 13 ? xo(Q, k) + 13 * a + j : uo(Q, k) + 4 * a + (j - 13);
                    Hm[(size_t)gi * n + gj] += HL[i * 17 + j];
                }
            }
        }
    }
    /* inequality rows: Hessian of |p - o|^2 is 2 I; of |p_a - p_b|^2 is [[2I, -2I], [-2I, 2I]] */
    for (int k = 1; k <= Q->d.N; ++k)
        for (int j = 0; j < Q->nineq; ++j) {
            double yg = y[go(Q, k, j)];
            int pa, pb;
            ineq_val(Q, v + xo(Q, k), k, j, &pa, &pb);
            for (int t = 0; t < 3; ++t) {
                int ia = xo(Q, k) + pa + t;
                Hm[(size_t)ia * n + ia] += 2.0 * yg;
                if (pb >= 0) {
                    int ib = xo(Q, k) + pb + t;
                    Hm[(size_t)ib * n + ib] += 2.0 * yg;
                    Hm[(size_t)ia * n + ib] -= 2.0 * yg;
                    Hm[(size_t)ib * n + ia] -= 2.0 * yg;
                }
            }
        }
}

/* --------------------------- construction --------------------------- */
void* quad_nlp_new(const ipmo_quad_desc* d, const double* theta, nlp_t* out) {
    quad_nlp* Q = (quad_nlp*)calloc(1, sizeof(quad_nlp));
    Q->d = *d;
    Q->P.mass = d->mass; Q->P.jxx = d->jxx; Q->P.jyy = d->jyy; Q->P.jzz = d->jzz;
    Q->P.arm = d->arm; Q->P.ctau = d->ctau; Q->P.grav = d->grav;
    Q->nx = 13 * d->n_agents;
    Q->nu = 4 * d->n_agents;
    Q->nineq = d->family == 2 ? d->n_agents * (d->n_agents - 1) / 2 : d->n_obs;
    Q->nw = (d->N + 1) * Q->nx + d->N * Q->nu;
    Q->ns = d->N * Q->nineq;
    Q->n = Q->nw + Q->ns;
    Q->m = (d->N + 1) * Q->nx + Q->ns;
    Q->theta = theta;
    Q->xl = (double*)malloc(Q->n * sizeof(double));
    Q->xu = (double*)malloc(Q->n * sizeof(double));
    double uh = d->mass * d->grav / 4.0;
    for (int i = 0; i < Q->n; ++i) { Q->xl[i] = -INFINITY; Q->xu[i] = INFINITY; }
    for (int k = 0; k < d->N; ++k)
        for (int i = 0; i < Q->nu; ++i) { Q->xl[uo(Q, k) + i] = 0.0; Q->xu[uo(Q, k) + i] = 2.0 * uh; }
    for (int i = Q->nw; i < Q->n; ++i) Q->xl[i] = 0.0;
    out->n = Q->n; out->m = Q->m; out->xl = Q->xl; out->xu = Q->xu; out->ud = Q;
    out->f = q_f; out->grad = q_grad; out->c = q_c; out->jac = q_jac; out->hess = q_hess;
    return Q;
}

void quad_nlp_free(void* p) {
    quad_nlp* Q = (quad_nlp*)p;
    if (!Q) return;
    free(Q->xl);
    free(Q->xu);
    free(Q);
}

/* cold start: x_k = xbar0 for every k, u_k = hover thrust, s = g(x) (pushed into the bounds later) */
void quad_cold_start(const ipmo_quad_desc* d, const double* theta, double* v) {
    nlp_t tmp;
    quad_nlp* Q = (quad_nlp*)quad_nlp_new(d, theta, &tmp);
    double uh = d->mass * d->grav / 4.0;
    for (int k = 0; k <= d->N; ++k) {
        for (int a = 0; a < d->n_agents; ++a) {
            const double* xb = xbar0(Q, a);
            for (int i = 0; i < 13; ++i) v[xo(Q, k) + 13 * a + i] = xb[i];
            if (k < d->N)
                for (int i = 0; i < 4; ++i) v[uo(Q, k) + 4 * a + i] = uh;
        }
    }
    for (int k = 1; k <= d->N; ++k)
        for (int j = 0; j < Q->nineq; ++j) {
            int pa, pb;
            v[so(Q, k, j)] = ineq_val(Q, v + xo(Q, k), k, j, &pa, &pb);
        }
    quad_nlp_free(Q);
}

/* single-agent stage evaluation exported for model tests */
void quad_stage_derivs(const ipmo_quad_desc* d, const double* x, const double* u, const double* lam,
                       double* F, double* G, double* HL) {
    qparams P = {d->mass, d->jxx, d->jyy, d->jzz, d->arm, d->ctau, d->grav};
    agent_derivs(&P, d->dt, x, u, lam, F, G, HL);
}

void quad_xdot(const ipmo_quad_desc* d, const double* x, const double* u, double* xd) {
    qparams P = {d->mass, d->jxx, d->jyy, d->jzz, d->arm, d->ctau, d->grav};
    hd hx[13], hu[4], out[13];
    for (int i = 0; i < 13; ++i) hx[i] = H(x[i]);
    for (int i = 0; i < 4; ++i) hu[i] = H(u[i]);
    quad_f(&P, hx, hu, out);
    for (int i = 0; i < 13; ++i) xd[i] = out[i].a;
}

/* primal values w without slacks (stage-interleaved), as in the decision vector */
int quad_nw(const ipmo_quad_desc* d) {
    int nx = 13 * d->n_agents, nu = 4 * d->n_agents;
    return (d->N + 1) * nx + d->N * nu;
}

/* warm point: v = (w, s) with the slacks at s = g(w) (pushed into the bounds later) */
void quad_warm_point(const ipmo_quad_desc* d, const double* theta, const double* w, double* v) {
    nlp_t tmp;
    quad_nlp* Q = (quad_nlp*)quad_nlp_new(d, theta, &tmp);
    memcpy(v, w, Q->nw * sizeof(double));
    for (int k = 1; k <= d->N; ++k)
        for (int j = 0; j < Q->nineq; ++j) {
            int pa, pb;
            v[so(Q, k, j)] = ineq_val(Q, v + xo(Q, k), k, j, &pa, &pb);
        }
    quad_nlp_free(Q);
}
