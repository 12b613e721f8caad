// Structured KKT factorization and solve for one slot, executed by one 64-lane wavefront
// (one workgroup), working set in LDS.
//
// The augmented system of eq. (7) for the multiple-shooting NMPC is block-tridiagonal in the
// stage blocks (lambda_k, x_k, u_k), lambda_k being the multiplier of the rows that define x_k.
// Inequality slacks (and, in restoration, the elastic p/n variables) are eliminated first;
// each slack pivot is positive and its row pivot negative, so with Haynsworth inertia
// additivity the reduced system must have one positive eigenvalue per primal and one negative
// per dynamics row.  The stages are then eliminated backward (k = N..0):
//   Hbar_k = H_k + G_k^T S_{k+1} G_k,  R_k = Hbar_k^uu = L_R L_R^T (Cholesky),
//   P_k = Hbar^xx - Y^T Y  (Y = L_R^{-1} Hbar^ux),
//   pair pivot [[-Delta, I], [I, P_k]]: with Delta = 0 its inertia is always (n_x, n_x) and
//   S_k = P_k; with Delta > 0 it needs C = I + Delta^1/2 P Delta^1/2 positive definite and
//   S_k = P - V^T V, V = L_C^{-1} Delta^1/2 P.
// The inertia is (n, m, 0) iff every Cholesky succeeds; a pivot that is exactly zero marks the
// matrix singular (Sec. IV "Step direction": inertia-controlled LDL^T).
#pragma once
#include "common.h"

namespace hipipm {

struct Slot {
  double* sc;
  double *v, *y, *zlu, *zuu, *zls, *th, *fm, *fr;
  double *yr, *rzlu, *rzuu, *rzls, *xr, *p, *nn, *zp, *zn;
  double *F, *G, *HW, *fac, *rb;
  double *dv, *dy, *dzlu, *dzuu, *dzls, *dp, *dn, *dzp, *dzn;
  double *rv, *rc, *rp, *rn, *vt, *ct, *pt, *nt, *csoc, *dvs, *dys, *dps, *dns, *g, *ref;
};

__device__ __forceinline__ Slot make_slot(const Cfg& c, double* ws, int slot) {
  double* R = ws + (long long)slot * c.stride;
  Slot s;
  s.sc = R + c.o_sc;
  s.v = R + c.o_v; s.y = R + c.o_y; s.zlu = R + c.o_zlu; s.zuu = R + c.o_zuu; s.zls = R + c.o_zls;
  s.th = R + c.o_th; s.fm = R + c.o_fm; s.fr = R + c.o_fr;
  s.yr = R + c.o_yr; s.rzlu = R + c.o_rzlu; s.rzuu = R + c.o_rzuu; s.rzls = R + c.o_rzls;
  s.xr = R + c.o_xr; s.p = R + c.o_p; s.nn = R + c.o_nn; s.zp = R + c.o_zp; s.zn = R + c.o_zn;
  s.F = R + c.o_F; s.G = R + c.o_G; s.HW = R + c.o_HW; s.fac = R + c.o_fac; s.rb = R + c.o_rb;
  s.dv = R + c.o_dv; s.dy = R + c.o_dy; s.dzlu = R + c.o_dzlu; s.dzuu = R + c.o_dzuu; s.dzls = R + c.o_dzls;
  s.dp = R + c.o_dp; s.dn = R + c.o_dn; s.dzp = R + c.o_dzp; s.dzn = R + c.o_dzn;
  s.rv = R + c.o_rv; s.rc = R + c.o_rc; s.rp = R + c.o_rp; s.rn = R + c.o_rn;
  s.vt = R + c.o_vt; s.ct = R + c.o_ct; s.pt = R + c.o_pt; s.nt = R + c.o_nt; s.csoc = R + c.o_csoc;
  s.dvs = R + c.o_dvs; s.dys = R + c.o_dys; s.dps = R + c.o_dps; s.dns = R + c.o_dns; s.g = R + c.o_g;
  s.ref = R + c.o_ref;
  return s;
}

// index helpers (decision vector and constraint rows)
__device__ __forceinline__ int xo(int k) { return k * NZ; }
__device__ __forceinline__ int uo(int k) { return k * NZ + NX; }
__device__ __forceinline__ int so(const Cfg& c, int k, int j) { return c.n_w + (k - 1) * c.NI + j; }
__device__ __forceinline__ int go(const Cfg& c, int k, int j) { return (c.N + 1) * NX + (k - 1) * c.NI + j; }

// the iterate the current phase works on (main problem or restoration problem)
struct Iter {
  double *y, *zlu, *zuu, *zls, *sub, *filt;
  bool resto;
};
__device__ __forceinline__ Iter cur_iter(const Slot& s, bool resto) {
  Iter it;
  it.resto = resto;
  if (resto) { it.y = s.yr; it.zlu = s.rzlu; it.zuu = s.rzuu; it.zls = s.rzls; it.sub = s.sc + SC_RMU; it.filt = s.fr; }
  else { it.y = s.y; it.zlu = s.zlu; it.zuu = s.zuu; it.zls = s.zls; it.sub = s.sc + SC_MU; it.filt = s.fm; }
  return it;
}

// ----------------------------------------------------------------------------- wave reductions
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wor(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}

// ----------------------------------------------------------------------------- LDS workspace
struct KktLds {
  double S[NX * NX];
  double H[NZ * NZ];
  double T[NX * NZ];
  double Gs[NX * NZ];
  double LR[NU * NU];
  double Y[NU * NX];
  double P[NX * NX];
  double C[NX * NX];
  double V[NX * NX];
  double dh[NX];
  double jg[MAX_OBS * 3];
  double Dg[MAX_OBS];
  double vec[8][32];
  double fr[FR_LEN];
  int bad;
};

enum : int { MODE_STEP = 0, MODE_LSQ = 1 };

// diagonal data of the eliminated variables
struct Elim {
  bool lsq, resto;
  double dxp, dcp, zeta;
};

// sigma of slack (k, j) and the row regularisation d of constraint row r
__device__ __forceinline__ double slack_sigma(const Cfg& c, const Slot& s, const Iter& it, const Elim& e, int k,
                                              int j) {
  if (e.lsq) return 1.0;
  const int si = so(c, k, j);
  double sv = s.v[si];
  double sig = it.zls[(k - 1) * c.NI + j] / sv + e.dxp;
  if (e.resto) {
    double d = fmin(1.0, 1.0 / fabs(s.xr[si]));
    sig += e.zeta * d * d;
  }
  return sig;
}
__device__ __forceinline__ void row_elastic(const Slot& s, const Elim& e, int r, double& sp, double& sn) {
  sp = s.zp[r] / s.p[r] + e.dxp;
  sn = s.zn[r] / s.nn[r] + e.dxp;
}
__device__ __forceinline__ double row_d(const Slot& s, const Elim& e, int r) {
  if (e.lsq) return 0.0;
  double d = e.dcp;
  if (e.resto) {
    double sp, sn;
    row_elastic(s, e, r, sp, sn);
    d += 1.0 / sp + 1.0 / sn;
  }
  return d;
}

// Cholesky of an n x n matrix in LDS (in place, lower), executed cooperatively; returns 0 ok,
// 1 non-positive pivot, 2 exactly-zero pivot.
__device__ __forceinline__ int chol_lds(double* A, int n, int ld, int lane) {
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    double d = A[j * ld + j];
    if (!(d > 0.0)) return d == 0.0 ? 2 : 1;
    double r = sqrt(d);
    __syncthreads();
    if (lane == 0) A[j * ld + j] = r;
    for (int i = j + 1 + lane; i < n; i += WAVE) A[i * ld + j] /= r;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = lane; e < m * m; e += WAVE) {
      int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) A[i * ld + l] -= A[i * ld + j] * A[l * ld + j];
    }
  }
  __syncthreads();
  return 0;
}

// ----------------------------------------------------------------------------- factorization
// Assemble and factor all stage blocks; returns 0 (inertia correct), 1 (wrong), 2 (singular).
// Per-stage factor records are written to s.fac.
__device__ __forceinline__ int kkt_factor(const Cfg& c, const Slot& s, const Iter& it, const Elim& e, double zeta, KktLds& L,
                          int lane) {
  const int N = c.N, NI = c.NI;
  for (int i = lane; i < NX * NX; i += WAVE) L.S[i] = 0.0;
  int status = 0;
  for (int k = N; k >= 0; --k) {
    const int nz = (k < N) ? NZ : NX;
    __syncthreads();
    // ---- stage Hessian H_k = W_k + Sigma + delta_x I (+ condensed slacks) ----
    for (int q = lane; q < nz * nz; q += WAVE) {
      int i = q / nz, j = q % nz;
      double h = 0.0;
      if (!e.lsq && k < N) h = s.HW[(long long)k * NZ * NZ + i * NZ + j];
      if (i == j) {
        if (e.lsq) {
          h += 1.0;
        } else {
          int vi = (i < NX) ? xo(k) + i : uo(k) + (i - NX);
          if (e.resto) {
            double d = fmin(1.0, 1.0 / fabs(s.xr[vi]));
            h += zeta * d * d;
          } else {
            h += (i < NX) ? 2.0 * c.qw : 2.0 * c.rw;
          }
          if (i >= NX) {
            double u = s.v[vi];
            int b = k * NU + (i - NX);
            h += it.zlu[b] / u + it.zuu[b] / (c.umax - u);
          }
          h += e.dxp;
        }
      }
      L.H[i * nz + j] = h;
    }
    // slack condensation data of stage k (k >= 1)
    if (k >= 1) {
      for (int j = lane; j < NI; j += WAVE) {
        const double* o = obs_ptr(c, s.th) + 4 * j;
        double sig = slack_sigma(c, s, it, e, k, j);
        double d = row_d(s, e, go(c, k, j));
        L.Dg[j] = sig / (1.0 + sig * d);
        for (int t = 0; t < 3; ++t) L.jg[3 * j + t] = 2.0 * (s.v[xo(k) + t] - o[t]);
      }
    }
    __syncthreads();
    if (k >= 1) {
      for (int q = lane; q < 9; q += WAVE) {
        int a = q / 3, b = q % 3;
        double acc = 0.0;
        for (int j = 0; j < NI; ++j) {
          acc += L.Dg[j] * L.jg[3 * j + a] * L.jg[3 * j + b];
          if (a == b && !e.lsq) acc += 2.0 * it.y[go(c, k, j)];
        }
        L.H[a * nz + b] += acc;
      }
    }
    // ---- Schur update H += G^T S_{k+1} G ----
    if (k < N) {
      const double* Gk = s.G + (long long)k * NX * NZ;
      for (int q = lane; q < NX * NZ; q += WAVE) L.Gs[q] = Gk[q];
      __syncthreads();
      for (int q = lane; q < NX * NZ; q += WAVE) {
        int i = q / NZ, j = q % NZ;
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) acc += L.S[i * NX + l] * L.Gs[l * NZ + j];
        L.T[q] = acc;
      }
      __syncthreads();
      for (int q = lane; q < NZ * NZ; q += WAVE) {
        int i = q / NZ, j = q % NZ;
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) acc += L.Gs[l * NZ + i] * L.T[l * NZ + j];
        L.H[q] += acc;
      }
    }
    __syncthreads();
    double* fr = s.fac + (long long)k * FR_LEN;
    // ---- control block: Cholesky of Hbar^uu, Y, P ----
    if (k < N) {
      if (lane == 0) {
        int bad = 0;
        for (int j = 0; j < NU && !bad; ++j) {
          double d = L.H[(NX + j) * NZ + NX + j];
          for (int l = 0; l < j; ++l) d -= L.LR[j * NU + l] * L.LR[j * NU + l];
          if (!(d > 0.0)) { bad = (d == 0.0) ? 2 : 1; break; }
          double r = sqrt(d);
          L.LR[j * NU + j] = r;
          for (int i = j + 1; i < NU; ++i) {
            double a = L.H[(NX + i) * NZ + NX + j];
            for (int l = 0; l < j; ++l) a -= L.LR[i * NU + l] * L.LR[j * NU + l];
            L.LR[i * NU + j] = a / r;
          }
          for (int i = 0; i < j; ++i) L.LR[i * NU + j] = 0.0;
        }
        L.bad = bad;
      }
      __syncthreads();
      if (L.bad) { status = L.bad; break; }
      for (int b = lane; b < NX; b += WAVE) {
        for (int a = 0; a < NU; ++a) {
          double acc = L.H[(NX + a) * NZ + b];
          for (int l = 0; l < a; ++l) acc -= L.LR[a * NU + l] * L.Y[l * NX + b];
          L.Y[a * NX + b] = acc / L.LR[a * NU + a];
        }
      }
      __syncthreads();
      for (int q = lane; q < NX * NX; q += WAVE) {
        int i = q / NX, j = q % NX;
        double acc = L.H[i * NZ + j];
#pragma unroll
        for (int a = 0; a < NU; ++a) acc -= L.Y[a * NX + i] * L.Y[a * NX + j];
        L.P[q] = acc;
      }
    } else {
      for (int q = lane; q < NX * NX; q += WAVE) L.P[q] = L.H[q];
    }
    // ---- pair pivot with the dual regularisation Delta_k of the rows defining x_k ----
    for (int i = lane; i < NX; i += WAVE) L.dh[i] = sqrt(row_d(s, e, k * NX + i));
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < NX; ++i) dmax = fmax(dmax, L.dh[i]);
    if (dmax > 0.0) {
      for (int q = lane; q < NX * NX; q += WAVE) {
        int i = q / NX, j = q % NX;
        L.C[q] = L.dh[i] * L.P[q] * L.dh[j] + (i == j ? 1.0 : 0.0);
      }
      int r = chol_lds(L.C, NX, NX, lane);
      if (r) { status = r; break; }
      for (int col = lane; col < NX; col += WAVE) {
        for (int i = 0; i < NX; ++i) {
          double acc = L.dh[i] * L.P[i * NX + col];
          for (int l = 0; l < i; ++l) acc -= L.C[i * NX + l] * L.V[l * NX + col];
          L.V[i * NX + col] = acc / L.C[i * NX + i];
        }
      }
      __syncthreads();
      for (int q = lane; q < NX * NX; q += WAVE) {
        int i = q / NX, j = q % NX;
        double acc = L.P[q];
        for (int l = 0; l < NX; ++l) acc -= L.V[l * NX + i] * L.V[l * NX + j];
        L.S[q] = acc;
      }
      for (int q = lane; q < NX * NX; q += WAVE) fr[FR_LC + q] = L.C[q];
    } else {
      for (int q = lane; q < NX * NX; q += WAVE) L.S[q] = L.P[q];
    }
    // ---- store the stage factor ----
    for (int q = lane; q < NU * NU; q += WAVE) fr[FR_LR + q] = L.LR[q];
    for (int q = lane; q < NU * NX; q += WAVE) fr[FR_Y + q] = L.Y[q];
    for (int q = lane; q < NX * NX; q += WAVE) fr[FR_P + q] = L.P[q];
    for (int q = lane; q < NX; q += WAVE) fr[FR_DH + q] = L.dh[q];
    if (lane == 0) fr[FR_FLAG] = dmax > 0.0 ? 1.0 : 0.0;
  }
  __syncthreads();
  return status;
}

// ----------------------------------------------------------------------------- solve
// Apply M_k^{-1} to (ra, rx, ru) of stage k with its factor record: on entry L.vec[1] = ra,
// L.vec[2] = rx, L.vec[3][0..3] = ru; on exit L.vec[0] = lambda part a and, if `full`,
// L.vec[2] = x part b and L.vec[3] = u part.  The record is first staged into LDS with
// coalesced loads; the small products are spread over lanes.
__device__ __forceinline__ void stage_apply(const Cfg& c, const double* fr, bool has_u, KktLds& L, bool full,
                                            int lane) {
  double* F = L.fr;
  for (int q = lane; q < FR_LEN; q += WAVE) F[q] = fr[q];
  __syncthreads();
  const double* LR = F + FR_LR;
  const double* Y = F + FR_Y;
  const double* P = F + FR_P;
  const double* LC = F + FR_LC;
  const double* dh = F + FR_DH;
  const bool reg = F[FR_FLAG] != 0.0;
  double* wu = L.vec[4];
  double* t = L.vec[5];
  // wu = L_R^{-1} ru
  if (has_u && lane == 0) {
    for (int a2 = 0; a2 < NU; ++a2) {
      double acc = L.vec[3][a2];
      for (int l = 0; l < a2; ++l) acc -= LR[a2 * NU + l] * wu[l];
      wu[a2] = acc / LR[a2 * NU + a2];
    }
  }
  __syncthreads();
  // t = rx - Y^T wu - P ra
  if (lane < NX) {
    double acc = L.vec[2][lane];
    if (has_u)
      for (int a2 = 0; a2 < NU; ++a2) acc -= Y[a2 * NX + lane] * wu[a2];
    for (int l = 0; l < NX; ++l) acc -= P[lane * NX + l] * L.vec[1][l];
    t[lane] = acc;
  }
  __syncthreads();
  if (reg) {
    // a = Delta^{-1/2} C^{-1} Delta^{1/2} t  with C = L_C L_C^T
    if (lane == 0) {
      double* z = L.vec[6];
      for (int i = 0; i < NX; ++i) {
        double acc = dh[i] * t[i];
        for (int l = 0; l < i; ++l) acc -= LC[i * NX + l] * z[l];
        z[i] = acc / LC[i * NX + i];
      }
      for (int i = NX - 1; i >= 0; --i) {
        double acc = z[i];
        for (int l = i + 1; l < NX; ++l) acc -= LC[l * NX + i] * z[l];
        z[i] = acc / LC[i * NX + i];
      }
      for (int i = 0; i < NX; ++i) L.vec[0][i] = z[i] / dh[i];
    }
  } else {
    if (lane < NX) L.vec[0][lane] = t[lane];
  }
  __syncthreads();
  if (!full) return;
  // b = ra + Delta a
  if (lane < NX) L.vec[2][lane] = L.vec[1][lane] + (reg ? dh[lane] * dh[lane] * L.vec[0][lane] : 0.0);
  __syncthreads();
  if (has_u) {
    // u = L_R^{-T} (wu - Y b)
    if (lane < NU) {
      double acc = wu[lane];
      for (int i = 0; i < NX; ++i) acc -= Y[lane * NX + i] * L.vec[2][i];
      L.vec[6][lane] = acc;
    }
    __syncthreads();
    if (lane == 0) {
      double* cu = L.vec[6];
      for (int a2 = NU - 1; a2 >= 0; --a2) {
        double acc = cu[a2];
        for (int l = a2 + 1; l < NU; ++l) acc -= LR[l * NU + a2] * cu[l];
        cu[a2] = acc / LR[a2 * NU + a2];
      }
      for (int a2 = 0; a2 < NU; ++a2) L.vec[3][a2] = cu[a2];
    }
    __syncthreads();
  }
}

// Solve K [dv; dy] = [bv; bc] (and the eliminated p/n rows bp, bn in restoration) with the
// factor in s.fac.  Outputs xv (n), xc (m), xp, xn (m; restoration only).
__device__ __forceinline__ void kkt_solve(const Cfg& c, const Slot& s, const Iter& it, const Elim& e, const double* bv,
                          const double* bc, const double* bp, const double* bn, double* xv, double* xc, double* xp,
                          double* xn, KktLds& L, int lane) {
  const int N = c.N, NI = c.NI;
  // 1. condensed stage right-hand sides into s.rb (lambda 13, x 13, u 4 per knot)
  for (int q = lane; q < (N + 1) * RB_LEN; q += WAVE) {
    int k = q / RB_LEN, i = q % RB_LEN;
    double val = 0.0;
    if (i < NX) {
      int r = k * NX + i;
      val = bc[r];
      if (e.resto) {
        double sp, sn;
        row_elastic(s, e, r, sp, sn);
        val += bp[r] / sp - bn[r] / sn;
      }
    } else if (i < 2 * NX) {
      val = bv[xo(k) + i - NX];
    } else if (i < 2 * NX + NU && k < N) {
      val = bv[uo(k) + i - 2 * NX];
    }
    s.rb[q] = val;
  }
  __syncthreads();
  // position rows of x_k gather the slack rows of stage k
  for (int q = lane; q < N * 3; q += WAVE) {
    int k = 1 + q / 3, t = q % 3;
    double acc = 0.0;
    for (int j = 0; j < NI; ++j) {
      const double* o = obs_ptr(c, s.th) + 4 * j;
      int r = go(c, k, j);
      double sig = slack_sigma(c, s, it, e, k, j);
      double d = row_d(s, e, r);
      double D = sig / (1.0 + sig * d);
      double bg = bc[r];
      if (e.resto) {
        double sp, sn;
        row_elastic(s, e, r, sp, sn);
        bg += bp[r] / sp - bn[r] / sn;
      }
      double jg = 2.0 * (s.v[xo(k) + t] - o[t]);
      acc += jg * D * (bv[so(c, k, j)] / sig + bg);
    }
    s.rb[(long long)k * RB_LEN + NX + t] += acc;
  }
  __syncthreads();
  // 2. backward sweep: rbar_k = r_k + G_k^T a_{k+1}
  for (int k = N; k >= 0; --k) {
    double* rb = s.rb + (long long)k * RB_LEN;
    const double* fr = s.fac + (long long)k * FR_LEN;
    for (int i = lane; i < NX; i += WAVE) {
      L.vec[1][i] = rb[i];
      L.vec[2][i] = rb[NX + i];
    }
    if (k < N)
      for (int i = lane; i < NU; i += WAVE) L.vec[3][i] = rb[2 * NX + i];
    __syncthreads();
    stage_apply(c, fr, k < N, L, false, lane);
    if (k > 0) {
      const double* Gp = s.G + (long long)(k - 1) * NX * NZ;
      double* rbp = s.rb + (long long)(k - 1) * RB_LEN;
      for (int j = lane; j < NZ; j += WAVE) {
        double acc = 0.0;
        for (int l = 0; l < NX; ++l) acc += Gp[l * NZ + j] * L.vec[0][l];
        rbp[NX + j] += acc;
      }
    }
    __syncthreads();
  }
  // 3. forward sweep
  for (int k = 0; k <= N; ++k) {
    const double* rb = s.rb + (long long)k * RB_LEN;
    const double* fr = s.fac + (long long)k * FR_LEN;
    for (int i = lane; i < NX; i += WAVE) {
      double w = 0.0;
      if (k > 0) {
        const double* Gp = s.G + (long long)(k - 1) * NX * NZ;
        for (int l = 0; l < NZ; ++l) w += Gp[i * NZ + l] * xv[(k - 1) * NZ + l];
      }
      L.vec[1][i] = rb[i] + w;
      L.vec[2][i] = rb[NX + i];
    }
    if (k < N)
      for (int i = lane; i < NU; i += WAVE) L.vec[3][i] = rb[2 * NX + i];
    __syncthreads();
    stage_apply(c, fr, k < N, L, true, lane);
    for (int i = lane; i < NX; i += WAVE) {
      xc[k * NX + i] = L.vec[0][i];
      xv[xo(k) + i] = L.vec[2][i];
    }
    if (k < N)
      for (int i = lane; i < NU; i += WAVE) xv[uo(k) + i] = L.vec[3][i];
    __syncthreads();
  }
  // 4. recover slack steps, inequality multiplier steps and elastic steps
  for (int q = lane; q < N * NI; q += WAVE) {
    int k = 1 + q / NI, j = q % NI;
    const double* o = obs_ptr(c, s.th) + 4 * j;
    int r = go(c, k, j);
    double sig = slack_sigma(c, s, it, e, k, j);
    double d = row_d(s, e, r);
    double D = sig / (1.0 + sig * d);
    double bg = bc[r];
    if (e.resto) {
      double sp, sn;
      row_elastic(s, e, r, sp, sn);
      bg += bp[r] / sp - bn[r] / sn;
    }
    double jdx = 0.0;
    for (int t = 0; t < 3; ++t) jdx += 2.0 * (s.v[xo(k) + t] - o[t]) * xv[xo(k) + t];
    int si = so(c, k, j);
    double bs = bv[si];
    double dyg = D * (jdx - bs / sig - bg);
    xc[r] = dyg;
    xv[si] = (bs + dyg) / sig;
  }
  __syncthreads();
  if (e.resto) {
    for (int r = lane; r < c.m; r += WAVE) {
      double sp, sn;
      row_elastic(s, e, r, sp, sn);
      xp[r] = (bp[r] + xc[r]) / sp;
      xn[r] = (bn[r] - xc[r]) / sn;
    }
  }
  __syncthreads();
}

}  // namespace hipipm
