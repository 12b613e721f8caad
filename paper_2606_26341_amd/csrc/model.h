// Quadrotor NMPC model on the device: 13-state rigid body (position, attitude quaternion,
// world-frame velocity, body rates) with 4 rotor thrusts (Sec. VI), classical RK4 under
// zero-order hold, and exact first/second derivatives of one RK4 step.
//
// Derivatives: each lane seeds one input direction e_j of z = (x, u) as a dual number
// (value + tangent).  The forward RK4 sweep carries the tangents, giving column j of
// G = dF/dz; a hand-written adjoint (vector-Jacobian product) sweep of lam^T F, also in dual
// arithmetic, gives in its tangent column j of sum_r lam_r d2F_r/dz^2 (forward-over-reverse).
#pragma once
#include "common.h"

namespace hipipm {

struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual dconst(double v) { return {v, 0.0}; }
__device__ __forceinline__ double dval(double a) { return a; }
__device__ __forceinline__ double dval(Dual a) { return a.v; }
template <class T> __device__ __forceinline__ T mkconst(double v);
template <> __device__ __forceinline__ double mkconst<double>(double v) { return v; }
template <> __device__ __forceinline__ Dual mkconst<Dual>(double v) { return {v, 0.0}; }

// continuous dynamics xdot = f(x, u)
template <class T>
__device__ __forceinline__ void quad_f(const Cfg& c, const T* x, const T* u, T* xd) {
  const T *q = x + 3, *w = x + 10;
  xd[0] = x[7];
  xd[1] = x[8];
  xd[2] = x[9];
  // qdot = 1/2 q (x) (0, omega)
  xd[3] = 0.5 * (-(q[1] * w[0]) - q[2] * w[1] - q[3] * w[2]);
  xd[4] = 0.5 * (q[0] * w[0] - q[3] * w[1] + q[2] * w[2]);
  xd[5] = 0.5 * (q[3] * w[0] + q[0] * w[1] - q[1] * w[2]);
  xd[6] = 0.5 * (-(q[2] * w[0]) + q[1] * w[1] + q[0] * w[2]);
  // vdot = R(q) e_z T/m - g e_z
  T Tm = (1.0 / c.mass) * ((u[0] + u[1]) + (u[2] + u[3]));
  T r13 = 2.0 * (q[1] * q[3] + q[0] * q[2]);
  T r23 = 2.0 * (q[2] * q[3] - q[0] * q[1]);
  T r33 = mkconst<T>(1.0) - 2.0 * (q[1] * q[1] + q[2] * q[2]);
  xd[7] = r13 * Tm;
  xd[8] = r23 * Tm;
  xd[9] = r33 * Tm - mkconst<T>(c.grav);
  // omegadot = J^{-1}(tau - omega x J omega), "+" layout
  T tx = c.arm * (u[1] - u[3]);
  T ty = c.arm * (u[2] - u[0]);
  T tz = c.ctau * ((u[0] + u[2]) - (u[1] + u[3]));
  xd[10] = (1.0 / c.jxx) * (tx - (c.jzz - c.jyy) * (w[1] * w[2]));
  xd[11] = (1.0 / c.jyy) * (ty - (c.jxx - c.jzz) * (w[2] * w[0]));
  xd[12] = (1.0 / c.jzz) * (tz - (c.jyy - c.jxx) * (w[0] * w[1]));
}

// adjoint of f: xb = (df/dx)^T a, ub = (df/du)^T a, given q, omega of the evaluation point and u
template <class T>
__device__ __forceinline__ void quad_vjp(const Cfg& c, const T* q, const T* w, const T* u, const T* a, T* xb,
                                         T* ub) {
  const T zero = mkconst<T>(0.0);
  xb[0] = zero; xb[1] = zero; xb[2] = zero;
  // pdot = v
  xb[7] = a[0]; xb[8] = a[1]; xb[9] = a[2];
  // quaternion kinematics
  const T aw = a[3], ax = a[4], ay = a[5], az = a[6];
  T bqw = 0.5 * (ax * w[0] + ay * w[1] + az * w[2]);
  T bqx = 0.5 * (-(aw * w[0]) - ay * w[2] + az * w[1]);
  T bqy = 0.5 * (-(aw * w[1]) + ax * w[2] - az * w[0]);
  T bqz = 0.5 * (-(aw * w[2]) - ax * w[1] + ay * w[0]);
  T bwx = 0.5 * (-(aw * q[1]) + ax * q[0] + ay * q[3] - az * q[2]);
  T bwy = 0.5 * (-(aw * q[2]) - ax * q[3] + ay * q[0] + az * q[1]);
  T bwz = 0.5 * (-(aw * q[3]) + ax * q[2] - ay * q[1] + az * q[0]);
  // thrust rotation: s = b . (r13, r23, r33),  vdot = s T/m
  const T bx = a[7], by = a[8], bz = a[9];
  T Tm = (1.0 / c.mass) * ((u[0] + u[1]) + (u[2] + u[3]));
  T r13 = 2.0 * (q[1] * q[3] + q[0] * q[2]);
  T r23 = 2.0 * (q[2] * q[3] - q[0] * q[1]);
  T r33 = mkconst<T>(1.0) - 2.0 * (q[1] * q[1] + q[2] * q[2]);
  T s = bx * r13 + by * r23 + bz * r33;
  bqw = bqw + Tm * (2.0 * (bx * q[2] - by * q[1]));
  bqx = bqx + Tm * (2.0 * (bx * q[3] - by * q[0]) - 4.0 * (bz * q[1]));
  bqy = bqy + Tm * (2.0 * (bx * q[0] + by * q[3]) - 4.0 * (bz * q[2]));
  bqz = bqz + Tm * (2.0 * (bx * q[1] + by * q[2]));
  T sm = (1.0 / c.mass) * s;
  // rotational dynamics
  T ex = (1.0 / c.jxx) * a[10], ey = (1.0 / c.jyy) * a[11], ez = (1.0 / c.jzz) * a[12];
  bwx = bwx - (c.jxx - c.jzz) * (ey * w[2]) - (c.jyy - c.jxx) * (ez * w[1]);
  bwy = bwy - (c.jzz - c.jyy) * (ex * w[2]) - (c.jyy - c.jxx) * (ez * w[0]);
  bwz = bwz - (c.jzz - c.jyy) * (ex * w[1]) - (c.jxx - c.jzz) * (ey * w[0]);
  xb[3] = bqw; xb[4] = bqx; xb[5] = bqy; xb[6] = bqz;
  xb[10] = bwx; xb[11] = bwy; xb[12] = bwz;
  ub[0] = sm - c.arm * ey + c.ctau * ez;
  ub[1] = sm + c.arm * ex - c.ctau * ez;
  ub[2] = sm + c.arm * ey + c.ctau * ez;
  ub[3] = sm - c.arm * ex - c.ctau * ez;
}

// one RK4 step, primal only
__device__ __forceinline__ void rk4(const Cfg& c, const double* x, const double* u, double* out) {
  double k[NX], t[NX], acc[NX];
  const double h = c.dt;
  quad_f<double>(c, x, u, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] = k[i]; t[i] = x[i] + 0.5 * h * k[i]; }
  quad_f<double>(c, t, u, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] += 2.0 * k[i]; t[i] = x[i] + 0.5 * h * k[i]; }
  quad_f<double>(c, t, u, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] += 2.0 * k[i]; t[i] = x[i] + h * k[i]; }
  quad_f<double>(c, t, u, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) out[i] = x[i] + (h / 6.0) * (acc[i] + k[i]);
}

// Column j of G = dF/d(x, u) of the RK4 step only (forward tangent sweep, no Hessian)
__device__ __forceinline__ void rk4_tangent(const Cfg& c, const double* x, const double* u, int j, double* Gcol) {
  Dual z[NZ], k[NX], t[NX], acc[NX];
#pragma unroll
  for (int i = 0; i < NZ; ++i) z[i] = {i < NX ? x[i] : u[i - NX], i == j ? 1.0 : 0.0};
  const Dual* xs = z;
  const Dual* us = z + NX;
  const double h = c.dt;
  quad_f<Dual>(c, xs, us, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] = k[i]; t[i] = xs[i] + (0.5 * h) * k[i]; }
  quad_f<Dual>(c, t, us, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] = acc[i] + 2.0 * k[i]; t[i] = xs[i] + (0.5 * h) * k[i]; }
  quad_f<Dual>(c, t, us, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) { acc[i] = acc[i] + 2.0 * k[i]; t[i] = xs[i] + h * k[i]; }
  quad_f<Dual>(c, t, us, k);
#pragma unroll
  for (int i = 0; i < NX; ++i) Gcol[i] = ((h / 6.0) * (acc[i] + k[i])).d + (i == j ? 1.0 : 0.0);
}

// Direction j of the RK4 step derivatives: F (optional), column j of G and of H = d2(lam^T F)/dz2.
__device__ __forceinline__ void rk4_deriv_dir(const Cfg& c, const double* x, const double* u, const double* lam,
                                              int j, double* F, double* Gcol, double* Hcol) {
  Dual z[NZ];
#pragma unroll
  for (int i = 0; i < NZ; ++i) z[i] = {i < NX ? x[i] : u[i - NX], i == j ? 1.0 : 0.0};
  const Dual* xs = z;
  const Dual* us = z + NX;
  const double h = c.dt;
  // forward sweep, keeping q and omega of the four stage points
  Dual qs[4][4], ws[4][3], k[NX], t[NX], acc[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) t[i] = xs[i];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) qs[st][i] = t[3 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) ws[st][i] = t[10 + i];
    quad_f<Dual>(c, t, us, k);
    const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
    const double hn = (st < 2) ? 0.5 * h : h;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      acc[i] = (st == 0) ? k[i] : acc[i] + wgt * k[i];
      if (st < 3) t[i] = xs[i] + hn * k[i];
    }
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    Dual Fi = xs[i] + (h / 6.0) * acc[i];
    if (F) F[i] = Fi.v;
    Gcol[i] = Fi.d;
  }
  // adjoint sweep of lam^T F (lam constant), in dual arithmetic
  Dual xbar[NX], ubar[NU], xi[NX], ui[NU], kb[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) xbar[i] = dconst(lam[i]);
#pragma unroll
  for (int i = 0; i < NU; ++i) ubar[i] = dconst(0.0);
#pragma unroll
  for (int i = 0; i < NX; ++i) xi[i] = dconst(0.0);   // adjoint of the previous stage point
#pragma unroll
  for (int st = 3; st >= 0; --st) {
    const double cw = (st == 0 || st == 3) ? h / 6.0 : h / 3.0;
    const double cn = (st == 2) ? h : 0.5 * h;        // coefficient of k_st in the next stage point
#pragma unroll
    for (int i = 0; i < NX; ++i) kb[i] = (st == 3) ? dconst(cw * lam[i]) : dconst(cw * lam[i]) + cn * xi[i];
    quad_vjp<Dual>(c, qs[st], ws[st], us, kb, xi, ui);
#pragma unroll
    for (int i = 0; i < NX; ++i) xbar[i] = xbar[i] + xi[i];
#pragma unroll
    for (int i = 0; i < NU; ++i) ubar[i] = ubar[i] + ui[i];
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) Hcol[i] = xbar[i].d;
#pragma unroll
  for (int i = 0; i < NU; ++i) Hcol[NX + i] = ubar[i].d;
}

// reference state at knot k
__device__ __forceinline__ void ref_state(const Cfg& c, const double* th, int k, double* xr) {
#pragma unroll
  for (int i = 0; i < NX; ++i) xr[i] = 0.0;
  xr[3] = 1.0;
  if (c.family == 0) {
    xr[0] = th[13]; xr[1] = th[14]; xr[2] = th[15];
  } else {   // figure-eight tracking (fixed or moving spheres)
    double A = th[13], om = th[14], t = k * c.dt;
    xr[0] = A * sin(om * t);
    xr[1] = 0.5 * A * sin(2.0 * om * t);
    xr[7] = A * om * cos(om * t);
    xr[8] = A * om * cos(2.0 * om * t);
  }
}

// sphere j at knot k: centre o[0..2], radius o[3].  The point-to-point and tracking families hold
// fixed spheres (cx, cy, cz, r); the moving-sphere tracking family holds (cx, cy, cz, r, vx, vy, vz),
// centre c + t_k v at t_k = k dt (obstacle trajectories known in advance).
__device__ __forceinline__ void obs_at(const Cfg& c, const double* th, int j, int k, double (&o)[4]) {
  if (c.family == 3) {
    const double* b = th + 15 + 7 * j;
    const double t = k * c.dt;
#pragma unroll
    for (int i = 0; i < 3; ++i) o[i] = b[i] + t * b[4 + i];
    o[3] = b[3];
  } else {
    const double* b = th + (c.family == 0 ? 16 : 15) + 4 * j;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = b[i];
  }
}

}  // namespace hipipm
