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
//
// Memory schedule: the per-stage inputs (derivative blocks G_k, W_k and the perturbation-free
// diagonal data) are read from HBM one stage ahead into registers while the current stage is
// computed, then parked in an LDS double buffer; the wave synchronises on LDS only, so those
// loads stay in flight across the stage's barriers.  The solve keeps all stage right-hand sides
// and the running step in LDS.
#pragma once
#include "common.h"

namespace hipipm {

struct Slot {
  double* sc;
  double *v, *y, *zlu, *zuu, *zls, *th, *fm, *fr;
  double *yr, *rzlu, *rzuu, *rzls, *xr, *p, *nn, *zp, *zn;
  double *F, *G, *HW, *fac, *rb;
  double *dv, *dy, *dzlu, *dzuu, *dzls, *dp, *dn, *dzp, *dzn;
  double *rv, *rc, *rp, *rn, *vt, *ct, *pt, *nt, *csoc, *dvs, *dys, *dps, *dns, *g, *ref, *sd;
  double *qv, *qc, *qp, *qn, *ev, *ec, *ep, *en;
  double *wdv, *wdy, *wdzlu, *wdzuu, *wdzls;
  double *syt, *szlu, *szuu, *szls;
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
  s.sd = R + c.o_sd;
  s.qv = R + c.o_qv; s.qc = R + c.o_qc; s.qp = R + c.o_qp; s.qn = R + c.o_qn;
  s.ev = R + c.o_ev; s.ec = R + c.o_ec; s.ep = R + c.o_ep; s.en = R + c.o_en;
  s.wdv = R + c.o_wdv; s.wdy = R + c.o_wdy; s.wdzlu = R + c.o_wdzlu; s.wdzuu = R + c.o_wdzuu; s.wdzls = R + c.o_wdzls;
  s.syt = R + c.o_syt; s.szlu = R + c.o_szlu; s.szuu = R + c.o_szuu; s.szls = R + c.o_szls;
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
// value of v on lane src (src uniform), delivered to every lane through the scalar unit
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// value of x on the lane chosen by the DPP pattern CTRL (within rows of 16 lanes)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
// reduction over each row of 16 lanes with a commutative op, the same bits on every lane of the
// row: partners lane ^ 1, lane ^ 2 (quad permutations), then the mirrored lane within 8 and 16
template <typename T, typename Op>
__device__ __forceinline__ T row16_reduce(T x, Op op) {
  x = op(x, dpp_mov<0xB1>(x));
  x = op(x, dpp_mov<0x4E>(x));
  x = op(x, dpp_mov<0x141>(x));
  x = op(x, dpp_mov<0x140>(x));
  return x;
}
template <typename T>
__device__ __forceinline__ T row16_sum(T x) {
  return row16_reduce(x, [](T a, T b) { return a + b; });
}
// whole-wavefront reductions (every lane active): rows by DPP, the four row results combined in a
// fixed order from the scalar unit, so every lane returns the same bits

__device__ __forceinline__ double wsum(double v) {
  v = row16_sum(v);
  return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}
__device__ __forceinline__ double wmax(double v) {
  v = row16_reduce(v, [](double a, double b) { return fmax(a, b); });
  return fmax(fmax(lane_bcast(v, 0), lane_bcast(v, 16)), fmax(lane_bcast(v, 32), lane_bcast(v, 48)));
}
__device__ __forceinline__ double wmin(double v) {
  v = row16_reduce(v, [](double a, double b) { return fmin(a, b); });
  return fmin(fmin(lane_bcast(v, 0), lane_bcast(v, 16)), fmin(lane_bcast(v, 32), lane_bcast(v, 48)));
}
__device__ __forceinline__ int wor(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}

// ----------------------------------------------------------------------------- lane loops
// One wavefront per slot leaves no other wave on the SIMD to hide memory latency behind, and a
// plain `for (i = lane; i < n; i += WAVE)` loop that loads, waits and stores pays one memory
// round trip per trip (a store to the slot record may alias the next trip's loads, so the
// compiler cannot hoist them).  lanes_for runs the same trips in groups: the group's loads (ld,
// which must not store) are all issued first, from a clamped index so that every lane loads a
// valid word without a branch, then use(i, value) runs for each trip in order.  A group holds up
// to 4 trips and at most 32 loaded words per lane unless LB0 sets its size: the loops over all
// constraint rows or variables that load one to three words per trip and sit on a slot's critical
// path (theta sums, trial points, the accept update) use 12, one group for a few hundred entries;
// a larger default for every loop measured slower (registers).  Results, and the order of every
// accumulation, are those of the plain loop.
template <int LB0 = 0, class Ld, class Use>
__device__ __forceinline__ void lanes_for(int n, int lane, Ld ld, Use use) {
  using V = decltype(ld(0));
  constexpr int K = (int)(sizeof(V) / sizeof(double));
  constexpr int LB = LB0 > 0 ? LB0 : (K >= 32 ? 1 : (32 / K > 4 ? 4 : 32 / K));
  for (int b = lane; b < n; b += LB * WAVE) {
    V v[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) v[u] = ld(min(b + u * WAVE, n - 1));
#pragma unroll
    for (int u = 0; u < LB; ++u)
      if (b + u * WAVE < n) use(b + u * WAVE, v[u]);
  }
}
// inequality rows of one knot whose loads are issued together
constexpr int OBS_CHUNK = 8;
// a compile-time case of a stage body (the first and last knots of a sweep)
template <bool B>
struct Flag {
  static constexpr bool value = B;
};
// the loaded values of one trip
template <int K>
struct DV {
  double v[K];
};

// Workgroup barrier whose fences cover LDS only, so outstanding global loads (prefetches) stay in
// flight across it.  Used only where no lane reads global memory written by another lane since
// the last full __syncthreads.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Scheduling fence: the compiler moves no instruction across it.  The factorization and the
// sweeps load a step's words from LDS into registers, then fence, so that the loads are issued as
// one group and the dependent products after it wait once for the group instead of once per
// pair of words (left to itself, the scheduler interleaves each read with its use).
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// ----------------------------------------------------------------------------- stage data
// Perturbation-free diagonal data of knot k (written once per factorization request):
//   [0, NZ)            objective Hessian diagonal + bound Sigma of (x_k, u_k) (identity in LSQ mode)
//   [NZ, NZ+NX)        z_p/p of the rows defining x_k   (restoration only)
//   [NZ+NX, NZ+2NX)    z_n/n of those rows              (restoration only)
//   [NZ+2NX, NZ+2NX+9) condensed inequality block Hc of the position rows (3x3), see kkt_condense
//   then per inequality row j of the knot: sigma0 (z_s/s [+ zeta D_R^2]), z_p/p, z_n/n, J_g (3),
//   2 y_g (Hessian of the row).
constexpr int SD_HC = NZ + 2 * NX;
constexpr int SD_HEAD = SD_HC + 9;
constexpr int SD_OBS = 7;
__device__ __host__ __forceinline__ int sd_len_of(int NI) { return ((SD_HEAD + SD_OBS * NI + 7) / 8) * 8; }
__device__ __forceinline__ int sd_len(const Cfg& c) { return sd_len_of(c.NI); }

struct Elim {
  bool lsq, resto;
  double dxp, dcp, zeta;
};

// row regularisation d = delta_c + 1/(z_p/p + delta_x) + 1/(z_n/n + delta_x) (elastic part in restoration)
__device__ __forceinline__ double row_dreg(const Elim& e, double sp0, double sn0) {
  if (e.lsq) return 0.0;
  double d = e.dcp;
  if (e.resto) d += 1.0 / (sp0 + e.dxp) + 1.0 / (sn0 + e.dxp);
  return d;
}

// Condensed inequality block of every knot k >= 1 for the perturbations in e:
//   Hc_k = sum_j D_kj J_kj^T J_kj + diag(sum_j 2 y_kj) (position rows),
//   D_kj = sigma / (1 + sigma d),  sigma = sigma0 + delta_x,  d = delta_c + elastic part,
// which is what eliminating the slack s_kj and its row (and the elastic p/n) leaves on x_k.
// One knot per lane: the knot's inequality rows are loaded once and D_kj computed once for the six
// upper-triangle entries.  Reads and rewrites the stage data.
__device__ __forceinline__ void kkt_condense(const Cfg& c, const Slot& s, const Elim& e, int lane) {
  const int N = c.N, NI = c.NI, SL = sd_len(c);
  for (int q = lane; q < N; q += WAVE) {
    const int k = 1 + q;
    double* sdk = s.sd + (long long)k * SL;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int j = 0; j < NI; ++j) {
      const double* o7 = sdk + SD_HEAD + SD_OBS * j;
      const double sig = o7[0] + (e.lsq ? 0.0 : e.dxp);
      const double d = row_dreg(e, o7[1], o7[2]);
      const double D = sig / (1.0 + sig * d);
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int a = p < 3 ? 0 : (p < 5 ? 1 : 2), b = p < 3 ? p : (p < 5 ? p - 2 : 2);
        acc[p] += D * o7[3 + a] * o7[3 + b];
        if (a == b) acc[p] += o7[6];
      }
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int a = p < 3 ? 0 : (p < 5 ? 1 : 2), b = p < 3 ? p : (p < 5 ? p - 2 : 2);
      sdk[SD_HC + a * 3 + b] = acc[p];
      if (a != b) sdk[SD_HC + b * 3 + a] = acc[p];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void kkt_stage_data(const Cfg& c, const Slot& s, const Iter& it, const Elim& e,
                                               int lane) {
  const int N = c.N, NI = c.NI, L = sd_len(c);
  if (!e.resto && !e.lsq) {
    // regular iterations: every knot entry but the controls' is a constant, stored without loads;
    // the control entries (v, z_L, z_U) in one group of loads
    for (int q = lane; q < (N + 1) * SD_HC; q += WAVE) {
      const int k = q / SD_HC, i = q % SD_HC;
      if (i >= NX && i < NZ && k < N) continue;
      s.sd[(long long)k * L + i] = (i < NX) ? 2.0 * c.qw : 0.0;
    }
    lanes_for(N * NU, lane, [&](int b) {
      const int k = b / NU, a = b % NU;
      return DV<3>{{s.v[uo(k) + a], it.zlu[b], it.zuu[b]}};
    }, [&](int b, const DV<3>& t) {
      const int k = b / NU, a = b % NU;
      double val = 2.0 * c.rw;
      double u = t.v[0];
      val += t.v[1] / u + t.v[2] / (c.umax - u);
      s.sd[(long long)k * L + NX + a] = val;
    });
  } else {
    // knot entries: the loads of a trip are the control bounds' (v, z_L, z_U), the regulariser's
    // x_R, or the elastic pair's (z, p) -- whichever the entry needs
    lanes_for<8>((N + 1) * SD_HC, lane, [&](int q) {
      const int k = q / SD_HC, i = q % SD_HC;
      DV<4> t{{0.0, 1.0, 0.0, 0.0}};
      if (i < NZ) {
        if ((k < N || i < NX) && !e.lsq) {
          const int vi = (i < NX) ? xo(k) + i : uo(k) + (i - NX);
          if (e.resto) t.v[0] = s.xr[vi];
          if (i >= NX) {
            const int b = k * NU + (i - NX);
            t.v[1] = s.v[vi];
            t.v[2] = it.zlu[b];
            t.v[3] = it.zuu[b];
          }
        }
      } else if (e.resto) {
        const int r = k * NX + (i - NZ) % NX;
        t.v[0] = (i < NZ + NX) ? s.zp[r] : s.zn[r];
        t.v[1] = (i < NZ + NX) ? s.p[r] : s.nn[r];
      }
      return t;
    }, [&](int q, const DV<4>& t) {
      const int k = q / SD_HC, i = q % SD_HC;
      double* sd = s.sd + (long long)k * L;
      double val = 0.0;
      if (i < NZ) {
        if (k < N || i < NX) {
          if (e.lsq) {
            val = 1.0;
          } else {
            if (e.resto) {
              double d = fmin(1.0, 1.0 / fabs(t.v[0]));
              val = e.zeta * d * d;
            } else {
              val = (i < NX) ? 2.0 * c.qw : 2.0 * c.rw;
            }
            if (i >= NX) {
              double u = t.v[1];
              val += t.v[2] / u + t.v[3] / (c.umax - u);
            }
          }
        }
      } else if (e.resto) {
        val = t.v[0] / t.v[1];
      }
      sd[i] = val;
    });
  }
  lanes_for(N * NI, lane, [&](int q) {
    const int k = 1 + q / NI, j = q % NI;
    DV<14> t;
    double o[4];
    obs_at(c, s.th, j, k, o);
    const int si = so(c, k, j), r = go(c, k, j);
#pragma unroll
    for (int a = 0; a < 3; ++a) t.v[a] = o[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) t.v[3 + a] = s.v[xo(k) + a];
    t.v[6] = it.zls[q];
    t.v[7] = s.v[si];
    t.v[8] = e.resto ? s.xr[si] : 1.0;
    t.v[9] = it.y[r];
    t.v[10] = e.resto ? s.zp[r] : 0.0;
    t.v[11] = e.resto ? s.p[r] : 1.0;
    t.v[12] = e.resto ? s.zn[r] : 0.0;
    t.v[13] = e.resto ? s.nn[r] : 1.0;
    return t;
  }, [&](int q, const DV<14>& t) {
    const int k = 1 + q / NI, j = q % NI;
    double* o7 = s.sd + (long long)k * L + SD_HEAD + SD_OBS * j;
    double sig0 = 1.0;
    if (!e.lsq) {
      sig0 = t.v[6] / t.v[7];
      if (e.resto) {
        double d = fmin(1.0, 1.0 / fabs(t.v[8]));
        sig0 += e.zeta * d * d;
      }
    }
    o7[0] = sig0;
    o7[1] = e.resto ? t.v[10] / t.v[11] : 0.0;
    o7[2] = e.resto ? t.v[12] / t.v[13] : 0.0;
    for (int a = 0; a < 3; ++a) o7[3 + a] = 2.0 * (t.v[3 + a] - t.v[a]);
    o7[6] = e.lsq ? 0.0 : 2.0 * t.v[9];
  });
  __syncthreads();
  kkt_condense(c, s, e, lane);
}

// ----------------------------------------------------------------------------- LDS workspaces
constexpr int PF = 16;   // prefetch registers per lane (one stage of inputs)
static_assert(NZ * NZ + NX * NZ + SD_HEAD + SD_OBS * MAX_OBS + 8 <= PF * WAVE, "stage inputs exceed the prefetch");

// The unrolled loops below give every lane the same number of entries and no per-entry
// branch, so that the entries' dependency chains overlap; the arrays are padded so that the
// surplus lanes read and write harmless words.
constexpr int TILE_T = (NX * NZ + WAVE - 1) / WAVE;    // 4 entries of T = S G per lane
constexpr int TILE_H = (NZ * NZ + WAVE - 1) / WAVE;    // 5 entries of H per lane
constexpr int TILE_P = (NX * NX + WAVE - 1) / WAVE;    // 3 entries of P, S per lane

template <typename T>
struct FacLdsT {
  T S[16 * NX];          // rows read up to (TILE_T * WAVE - 1) / NZ
  T H[TILE_H * WAVE];
  T Y[WAVE];
  T P[TILE_P * WAVE];
  T CV[TILE_T * WAVE + 96];   // T = S G during the Schur update, then L_C | V (+ read-only pad)
  T LI[NX * NX];              // L_C^{-1}
  T dh[NX];
  T rdh[NX];
  T buf[PF * WAVE];      // stage inputs: W (NZ*NZ) | G (NX*NZ) | stage data
};
using FacLds = FacLdsT<double>;

constexpr int SPF = (FR_LEN + NX * NZ + WAVE - 1) / WAVE;
static_assert(FR_LEN + NX * NZ <= SPF * WAVE, "solve stage inputs exceed the prefetch");

// solve workspace, carved from dynamic LDS (its size depends on the horizon; sized in doubles)
template <typename T>
struct SolLdsT {
  T* rb;                             // condensed stage right-hand sides, (N+1) x RB_LEN
  T* buf;                            // factor record of the knot | G of the coupling interval
  T* tmp;                            // 32 words: x part of the current stage
};
using SolLds = SolLdsT<double>;
__device__ __host__ __forceinline__ int sol_lds_doubles(int N) { return (N + 1) * RB_LEN + SPF * WAVE + 32; }
template <typename T>
__device__ __forceinline__ SolLdsT<T> sol_lds(const Cfg& c, double* dyn) {
  SolLdsT<T> V;
  V.rb = reinterpret_cast<T*>(dyn);
  V.buf = V.rb + (c.N + 1) * RB_LEN;
  V.tmp = V.buf + SPF * WAVE;
  return V;
}

// 1/sqrt(d) for finite d > 0: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double d) {
  const double h = 0.5 * d;
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
// 1/x for finite nonzero x: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

__device__ __forceinline__ float rsqrt_nr(float d) {
  const float y = __builtin_amdgcn_rsqf(d);
  return y * fmaf(-0.5f * d * y, y, 1.5f);
}
__device__ __forceinline__ float rcp_nr(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, y, 1.0f), y, y);
}


// FP64 matrix-core product D = A B + C on 16 x 16 tiles with K = 4 (v_mfma_f64_16x16x4f64), one
// call per wavefront.  Lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16) and holds
// D(4 r + l / 16, l % 16) in item r.
typedef double dbl4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// The FP32 product v_mfma_f32_16x16x4f32 takes A and B the same way but holds D(4 (l / 16) + r,
// l % 16) in item r.
typedef float flt4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ flt4 mfma32(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// the 16 x 16 x 4 product in the factor's precision T: accumulator type, product, and the row of
// the result that item r of a lane in lane group kq = l / 16 holds
template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef dbl4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) { return mfma64(a, b, c); }
  static __device__ __forceinline__ int row(int r, int kq) { return 4 * r + kq; }
};
template <>
struct Mma<float> {
  typedef flt4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) { return mfma32(a, b, c); }
  static __device__ __forceinline__ int row(int r, int kq) { return 4 * kq + r; }
};

// An FP32 pivot that keeps less than this fraction of the diagonal entry it started from has
// lost most of its significant digits to cancellation: its sign is not a reliable inertia verdict,
// and the factorization reports status 3 so that the decision is taken again in FP64.
constexpr float F32_PIVOT_REL = 1e-4f;

// In-register Cholesky of an NX x NX SPD candidate held one row per lane (lane i < NX holds
// c[l] = A_il; the lower part is used).  Right-looking, column j broadcast from lane j.  On
// success row `lane` of L is in c (lower part) and rinv[j] = 1 / L_jj on every lane.  Returns 0,
// 1 (a non-positive pivot), 2 (an exactly-zero pivot) or, in FP32 only, 3 (a positive pivot
// below F32_PIVOT_REL times its starting diagonal entry); the result is wave-uniform.
template <typename T>
__device__ __forceinline__ int chol_rows(T (&c)[NX], T (&rinv)[NX], int lane) {
  T dg = 0.0;
  if constexpr (sizeof(T) == sizeof(float)) {
#pragma unroll
    for (int j = 0; j < NX; ++j) dg = (lane == j) ? c[j] : dg;
  }
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const T d = lane_bcast(c[j], j);
    if (!(d > 0.0)) return d == 0.0 ? 2 : 1;
    if constexpr (sizeof(T) == sizeof(float))
      if (d <= F32_PIVOT_REL * lane_bcast(dg, j)) return 3;
    rinv[j] = rsqrt_nr(d);
    c[j] = (lane == j) ? d * rinv[j] : c[j] * rinv[j];
#pragma unroll
    for (int l = j + 1; l < NX; ++l) {
      const T ljl = lane_bcast(c[j], l);     // L_lj
      if (lane >= l) c[l] -= c[j] * ljl;
    }
  }
  return 0;
}

// stage k inputs as one flat range: [W_k (k < N) | G_k (k < N) | stage data].  Every lane loads
// from a valid address (lanes past the end re-read the last word) so that no load sits behind a
// branch: the registers are consumed only by stage_park, where the wait for the loads lands.
// Which range the t-th word of every lane falls in is known at compile time once the loop is
// unrolled; only the groups of 64 words that straddle a boundary select an address per lane.
__device__ __forceinline__ void stage_prefetch(const Cfg& c, const Slot& s, int k, int lane, double* reg) {
  const int nS = sd_len(c);
  const double* D = s.sd + (long long)k * nS;
  if (k < c.N) {
    constexpr int EW = NZ * NZ, EG = NZ * NZ + NX * NZ;   // ends of the W_k and G_k words
    const double* W = s.HW + (long long)k * NZ * NZ;
    const double* G = s.G + (long long)k * NX * NZ;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int q = lane + WAVE * t, lo = WAVE * t, hi = WAVE * t + WAVE;
      if (hi <= EW) {
        reg[t] = W[q];
      } else if (lo >= EW && hi <= EG) {
        reg[t] = G[q - EW];
      } else if (lo >= EG) {
        reg[t] = D[min(q - EG, nS - 1)];
      } else {
        const double* a = (q < EW) ? W + q : (q < EG) ? G + (q - EW) : D + min(q - EG, nS - 1);
        reg[t] = *a;
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < PF; ++t) reg[t] = D[min(lane + WAVE * t, nS - 1)];
  }
}
template <typename T>
__device__ __forceinline__ void stage_park(T* buf, int lane, const double* reg) {
#pragma unroll
  for (int t = 0; t < PF; ++t) buf[lane + WAVE * t] = (T)reg[t];
}

// ----------------------------------------------------------------------------- factorization
// Factor all stage blocks with perturbations (e.dxp, e.dcp); stage data from kkt_stage_data.
// Returns 0 (inertia correct), 1 (wrong), 2 (singular) or, in FP32, 3 (a pivot too close to zero
// for an FP32 verdict).  Writes the per-knot factor records.
template <typename T, bool FENCE = true>
__device__ __forceinline__ int kkt_factor(const Cfg& c, const Slot& s, const Elim& e, FacLdsT<T>& L, int lane) {
  const int N = c.N;
  double reg[PF];   // FP64 inputs, rounded to T when parked
  if (!e.lsq && (e.dxp != 0.0 || e.dcp != 0.0)) kkt_condense(c, s, e, lane);
  for (int i = lane; i < 16 * NX; i += WAVE) L.S[i] = 0.0;
  stage_prefetch(c, s, N, lane, reg);
  stage_park(L.buf, lane, reg);
  lds_barrier();
  const T dx = e.lsq ? T(0) : T(e.dxp);
  int status = 0;
  // one knot; the knots with a control (k < N) and with a predecessor (k > 0) are compile-time
  // cases: knot N, knots N-1..1, knot 0.  Returns true when the factorization stops (status set).
  auto knot = [&](int k, auto has_u_tag, auto more_tag) -> bool {
    constexpr bool HAS_U = decltype(has_u_tag)::value, MORE = decltype(more_tag)::value;
    double reg[PF];          // the next knot's inputs, in flight during this knot
    const T* B = L.buf;      // dead after the barrier that follows the dh read
    const T* Wk = B;
    const T* Gk = B + (HAS_U ? NZ * NZ : 0);
    const T* SD = B + (HAS_U ? NZ * NZ + NX * NZ : 0);
    T* fr = reinterpret_cast<T*>(s.fac) + (long long)k * FR_LEN;
    if (MORE) stage_prefetch(c, s, k - 1, lane, reg);   // in flight during this stage
    // ---- Schur update, first half: T = S_{k+1} G_k (13 x 17) ----
    // columns 0..15 on the matrix cores (K = 13 padded to 16; one 16 x 16 x 4 product costs about
    // as much as eleven FMAs of a wavefront), column 16 on the vector ALUs, row i on lane i
    const int r16 = lane & 15, kq = lane >> 4, li0 = lane < NX ? lane : NX - 1;
    // In FP64 the product's item st on lane l is T(4 st + l/16, l%16), the B operand of step st of
    // G^T T below, so T stays in registers (column 16 is broadcast from its lanes); the FP32
    // product's items are laid out differently and pass through LDS, as they do in the unfenced
    // FP64 fallback of the mixed kernels (fewer registers).
    constexpr bool REG_T = sizeof(T) == sizeof(double) && FENCE;
    typename Mma<T>::acc t0 = {T(0), T(0), T(0), T(0)};
    T t16 = 0.0;
    if (HAS_U) {
      // operands first, as one group of LDS reads
      T sr[NX], gc[NX], sv[4], g0[4];
#pragma unroll
      for (int l = 0; l < NX; ++l) {
        sr[l] = L.S[li0 * NX + l];
        gc[l] = Gk[l * NZ + 16];
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int kk = 4 * st + kq, kc = kk < NX ? kk : 0;
        sv[st] = L.S[(r16 < NX ? r16 : 0) * NX + kc];
        g0[st] = Gk[kc * NZ + r16];
      }
      if constexpr (FENCE) sched_fence();
#pragma unroll
      for (int l = 0; l < NX; ++l) t16 += sr[l] * gc[l];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int kk = 4 * st + kq;
        const T a = (kk < NX && r16 < NX) ? sv[st] : T(0);
        t0 = Mma<T>::mma(a, kk < NX ? g0[st] : T(0), t0);
      }
      if constexpr (!REG_T) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq);
          if (i < NX) L.CV[i * NZ + r16] = t0[r];
        }
        if (lane < NX) L.CV[lane * NZ + 16] = t16;
        lds_barrier();
      }
    }
    // ---- stage Hessian (NZ stride): W_k + diag + delta_x I + Hc_k + G_k^T T ----
    // the words of entry (i, j): W_ij, the diagonal term of column j, the condensed block's entry
    struct HW3 {
      T w, d, hc;
    };
    auto h_words = [&](int i, int j) -> HW3 {
      return {(!e.lsq && HAS_U) ? Wk[i * NZ + j] : T(0), SD[j], SD[SD_HC + 3 * (i < 3 ? i : 0) + (j < 3 ? j : 0)]};
    };
    auto h_base = [&](int i, int j, const HW3& b) -> T {
      T h = b.w;
      h += (i == j && (HAS_U || i < NX)) ? b.d + dx : T(0);
      h += (MORE && i < 3 && j < 3) ? b.hc : T(0);
      return h;
    };
    {
      // the leading 16 x 16 tile of the symmetric 17 x 17 result on the matrix cores (the
      // additive terms as the accumulator's start); column 16 on the vector ALUs, entry i on
      // lane i, also written as row 16.  Operands first, as one group of LDS reads.
      const int ih = lane < NZ ? lane : NZ - 1;
      HW3 hb[4], hb16 = h_words(ih, 16);
#pragma unroll
      for (int r = 0; r < 4; ++r) hb[r] = h_words(Mma<T>::row(r, kq), r16);
      T gi[NX], cv[NX], g0[4], c0[4];
      if (HAS_U) {
#pragma unroll
        for (int l = 0; l < NX; ++l) {
          gi[l] = Gk[l * NZ + ih];
          if constexpr (REG_T) cv[l] = lane_bcast(t16, l);
          else cv[l] = L.CV[l * NZ + 16];
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + kq, kc = kk < NX ? kk : 0;
          g0[st] = Gk[kc * NZ + r16];
          if constexpr (REG_T) c0[st] = t0[st];
          else c0[st] = L.CV[kc * NZ + r16];
        }
      }
      if constexpr (FENCE) sched_fence();
      typename Mma<T>::acc h00;
#pragma unroll
      for (int r = 0; r < 4; ++r) h00[r] = h_base(Mma<T>::row(r, kq), r16, hb[r]);
      T h16 = h_base(ih, 16, hb16);
      if (HAS_U) {
#pragma unroll
        for (int l = 0; l < NX; ++l) h16 += gi[l] * cv[l];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + kq;
          h00 = Mma<T>::mma(kk < NX ? g0[st] : T(0), kk < NX ? c0[st] : T(0), h00);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) L.H[Mma<T>::row(r, kq) * NZ + r16] = h00[r];
      if (lane < NZ) {
        L.H[lane * NZ + 16] = h16;
        L.H[16 * NZ + lane] = h16;
      }
    }
    lds_barrier();
    // ---- control block: Cholesky of Hbar^uu (on every lane, in registers), Y, P ----
    const int li = lane < NX ? lane : NX - 1;
    // pair pivot with the dual regularisation Delta_k of the rows defining x_k (Delta > 0 on every
    // row exactly when delta_c > 0 or the elastic variables are eliminated); without it S_k = P_k,
    // written where P is formed
    const bool pair = !e.lsq && (e.resto || e.dcp > 0.0);
    if (HAS_U) {
      T lr[NU * NU], rr[NU];
      // the control block's lower triangle and this lane's column of H_ux, as one group of reads
      T huu[NU * NU], hux[NU];
#pragma unroll
      for (int j = 0; j < NU; ++j) {
#pragma unroll
        for (int i = j; i < NU; ++i) huu[i * NU + j] = L.H[(NX + i) * NZ + NX + j];
        hux[j] = L.H[(NX + j) * NZ + li];
      }
      if constexpr (FENCE) sched_fence();
      int bad = 0;
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        T d = huu[j * NU + j];
        const T d0 = d;
#pragma unroll
        for (int l = 0; l < j; ++l) d -= lr[j * NU + l] * lr[j * NU + l];
        if (bad == 0 && !(d > 0.0)) bad = (d == 0.0) ? 2 : 1;
        if constexpr (sizeof(T) == sizeof(float))
          if (bad == 0 && d <= F32_PIVOT_REL * d0) bad = 3;
        rr[j] = rsqrt_nr(d);
        lr[j * NU + j] = d * rr[j];
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          if (i < j) lr[i * NU + j] = 0.0;
          if (i <= j) continue;
          T a = huu[i * NU + j];
#pragma unroll
          for (int l = 0; l < j; ++l) a -= lr[i * NU + l] * lr[j * NU + l];
          lr[i * NU + j] = a * rr[j];
        }
      }
      if (bad) { status = bad; return true; }
      {
        T v = 0.0, w = 0.0;
#pragma unroll
        for (int t = 0; t < NU * NU; ++t) v = (lane == t) ? lr[t] : v;
#pragma unroll
        for (int t = 0; t < NU; ++t) w = (lane == t) ? rr[t] : w;
        if (lane < NU * NU) fr[FR_LR + lane] = v;
        if (lane < NU) fr[FR_RR + lane] = w;
      }
      if (lane < NX) {
        T y[NU];
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          T acc = hux[a];
#pragma unroll
          for (int l = 0; l < a; ++l) acc -= lr[a * NU + l] * y[l];
          y[a] = acc * rr[a];
          L.Y[a * NX + lane] = y[a];
          fr[FR_Y + a * NX + lane] = y[a];
        }
      }
      lds_barrier();
      {
        // P = H_xx - Y^T Y: one matrix-core product with K = NU
        const T yv = L.Y[kq * NX + (r16 < NX ? r16 : 0)];
        const T y = r16 < NX ? yv : T(0);
        typename Mma<T>::acc p;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq);
          const T hv = L.H[(i < NX ? i : 0) * NZ + (r16 < NX ? r16 : 0)];
          p[r] = (i < NX && r16 < NX) ? hv : T(0);
        }
        p = Mma<T>::mma(-y, y, p);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq);
          if (i < NX && r16 < NX) {
            L.P[i * NX + r16] = p[r];
            fr[FR_P + i * NX + r16] = p[r];
            if (!pair) L.S[i * NX + r16] = p[r];
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < TILE_P; ++t) {
        const int q = lane + WAVE * t;
        const T pv = L.H[(q / NX) * NZ + q % NX];
        L.P[q] = pv;
        if (q < NX * NX) fr[FR_P + q] = pv;
        if (!pair) L.S[q] = pv;
      }
      if (lane < NU * NX) fr[FR_Y + lane] = T(0);
    }
    // ---- pair pivot with the dual regularisation Delta_k of the rows defining x_k ----
    const T dhl = pair ? T(sqrt(row_dreg(e, SD[NZ + li], SD[NZ + NX + li]))) : T(0);
    if (lane < NX) L.dh[lane] = dhl;
    lds_barrier();
    T* LC = L.CV;
    T* VV = L.CV + NX * NX;
    if (pair) {
      // C = I + Delta^1/2 P Delta^1/2, one row per lane, factored in registers
      T cr[NX], ri[NX], pr[NX], dhv[NX];
#pragma unroll
      for (int l = 0; l < NX; ++l) {
        pr[l] = L.P[li * NX + l];
        dhv[l] = L.dh[l];
      }
      if constexpr (FENCE) sched_fence();
#pragma unroll
      for (int l = 0; l < NX; ++l) cr[l] = dhl * pr[l] * dhv[l] + (lane == l ? 1.0 : 0.0);
      const int r = chol_rows(cr, ri, lane);
      if (r) { status = r; return true; }
      if (lane < NX) {
#pragma unroll
        for (int l = 0; l < NX; ++l) LC[lane * NX + l] = (l <= lane) ? cr[l] : 0.0;
        L.rdh[lane] = rcp_nr(dhl);
      }
      lds_barrier();
      // lanes 0..12: column `lane` of V = L_C^{-1} Delta^1/2 P; lanes 32..44: column `lane - 32` of
      // L_C^{-1}; forward substitutions in registers
      if (lane < NX || (lane >= 32 && lane < 32 + NX)) {
        const bool inv = lane >= 32;
        const int col = inv ? lane - 32 : lane;
        T v[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          // row i of L_C and the right-hand side entry, as one group of reads
          T lc[NX];
          const T di = L.dh[i], pic = L.P[i * NX + col];
#pragma unroll
          for (int l = 0; l < i; ++l) lc[l] = LC[i * NX + l];
          if constexpr (FENCE) sched_fence();
          T acc = inv ? (i == col ? 1.0 : 0.0) : di * pic;
#pragma unroll
          for (int l = 0; l < i; ++l) acc -= lc[l] * v[l];
          v[i] = acc * ri[i];
          if (inv) L.LI[i * NX + col] = v[i];
          else VV[i * NX + col] = v[i];
        }
      }
      lds_barrier();
      // S = P - V^T V and M = Delta^{-1/2} C^{-1} Delta^{1/2}, C^{-1} = L_C^{-T} L_C^{-1}
      {
        // both Gram products on the matrix cores (K = 13 padded to 16)
        const int jc = r16 < NX ? r16 : 0;
        typename Mma<T>::acc sa, ma = {T(0), T(0), T(0), T(0)};
        T pv[4], vv[4], lv[4], dr[4], rd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq), ic = i < NX ? i : 0;
          pv[r] = L.P[ic * NX + jc];
          dr[r] = L.dh[jc];
          rd[r] = L.rdh[ic];
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int l = 4 * st + kq, lc = l < NX ? l : 0;
          vv[st] = VV[lc * NX + jc];
          lv[st] = L.LI[lc * NX + jc];
        }
        if constexpr (FENCE) sched_fence();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq);
          sa[r] = (i < NX && r16 < NX) ? pv[r] : T(0);
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int l = 4 * st + kq;
          const bool ok = l < NX && r16 < NX;
          const T v = ok ? vv[st] : T(0), w = ok ? lv[st] : T(0);
          sa = Mma<T>::mma(-v, v, sa);
          ma = Mma<T>::mma(w, w, ma);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = Mma<T>::row(r, kq);
          if (i < NX && r16 < NX) {
            L.S[i * NX + r16] = sa[r];
            fr[FR_M + i * NX + r16] = ma[r] * dr[r] * rd[r];
          }
        }
      }
    }
    // ---- store the rest of the stage factor (Y and P were stored where formed) ----
    if (lane < NX) fr[FR_DH + lane] = dhl;
    if (lane == 0) fr[FR_FLAG] = pair ? 1.0 : 0.0;
    if (MORE) stage_park(L.buf, lane, reg);
    lds_barrier();
    return false;
  };
  if (!knot(N, Flag<false>{}, Flag<true>{})) {
    int k = N - 1;
    for (; k >= 1; --k)
      if (knot(k, Flag<true>{}, Flag<true>{})) break;
    if (k == 0) knot(0, Flag<true>{}, Flag<false>{});
  }
  __syncthreads();
  return status;
}

// ----------------------------------------------------------------------------- solve
// Apply M_k^{-1} of stage k (factor record F in LDS) to the stage right-hand side
// (ra, rx, ru): ra[] holds the lambda part on every lane, rx the x component of row `lane`,
// ru[] the control part on every lane.  Returns the lambda component a of row `lane`; with
// `full` also the x component b of row `lane` and the control part cu[] on every lane.
// Lanes >= NX compute throw-away values.  Ends with an LDS barrier after the last read of F.
//   w_u = L_R^{-1} r_u,  t = r_x - Y^T w_u - P r_a,
//   a = t (Delta = 0)  or  a = M t,  M = Delta^{-1/2} C^{-1} Delta^{1/2} from the factor record,
//   b = r_a + Delta a,  c_u = L_R^{-T} (w_u - Y b)
// the words of a factor record that lane `li` reads in stage_apply: L_R (strict lower part),
// the reciprocal pivots, column li of Y, row li of P, Delta^{1/2}_li and the pair-pivot flag
template <typename T>
struct StageWords {
  T lr[NU * NU], rr[NU], yl[NU], pr[NX], dh;
  bool reg;
};
template <typename T>
__device__ __forceinline__ StageWords<T> stage_words(const T* F, int li) {
  StageWords<T> W;
#pragma unroll
  for (int a2 = 0; a2 < NU; ++a2) {
#pragma unroll
    for (int l = 0; l < a2; ++l) W.lr[a2 * NU + l] = F[FR_LR + a2 * NU + l];
    W.rr[a2] = F[FR_RR + a2];
    W.yl[a2] = F[FR_Y + a2 * NX + li];
  }
#pragma unroll
  for (int l = 0; l < NX; ++l) W.pr[l] = F[FR_P + li * NX + l];
  W.reg = F[FR_FLAG] != 0.0;
  W.dh = F[FR_DH + li];
  return W;
}
template <typename T>
__device__ __forceinline__ T stage_apply(const T* F, const StageWords<T>& W, bool has_u, const T (&ra)[NX], T rx,
                                         const T (&ru)[NU], bool full, int lane, T& b, T (&cu)[NU], SolLdsT<T>& V) {
  const int li = lane < NX ? lane : NX - 1;
  const auto& lr = W.lr;
  const auto& rr = W.rr;
  const auto& yl = W.yl;
  const auto& pr = W.pr;
  const bool reg = W.reg;
  const T dh = W.dh;
  T wu[NU];
#pragma unroll
  for (int a2 = 0; a2 < NU; ++a2) {
    T acc = ru[a2];
#pragma unroll
    for (int l = 0; l < a2; ++l) acc -= lr[a2 * NU + l] * wu[l];
    wu[a2] = has_u ? acc * rr[a2] : 0.0;
  }
  T t = rx;
  if (has_u)
#pragma unroll
    for (int a2 = 0; a2 < NU; ++a2) t -= yl[a2] * wu[a2];
#pragma unroll
  for (int l = 0; l < NX; ++l) t -= pr[l] * ra[l];
  T av = t;
  if (reg) {
    T mr[NX];
#pragma unroll
    for (int l = 0; l < NX; ++l) mr[l] = F[FR_M + li * NX + l];
    sched_fence();
    T tl[NX];
#pragma unroll
    for (int l = 0; l < NX; ++l) tl[l] = lane_bcast(t, l);
    T acc = 0.0;
#pragma unroll
    for (int l = 0; l < NX; ++l) acc += mr[l] * tl[l];
    av = acc;
  }
  if (full) {
    b = ra[li] + (reg ? dh * dh * av : 0.0);
    if (has_u) {
      if (lane < NX) V.tmp[lane] = b;
      lds_barrier();
      // (Y b)_a: lane 16 a + i forms Y_ai b_i, each row of 16 lanes sums its four products
      const int i16 = lane & 15, ic = i16 < NX ? i16 : 0;
      const T yv = F[FR_Y + (lane >> 4) * NX + ic], tv = V.tmp[ic];
      const T yb = row16_sum(i16 < NX ? T(yv * tv) : T(0));
      T c2[NU];
#pragma unroll
      for (int a2 = 0; a2 < NU; ++a2) c2[a2] = wu[a2] - lane_bcast(yb, 16 * a2);
#pragma unroll
      for (int a2 = NU - 1; a2 >= 0; --a2) {
        T acc = c2[a2];
#pragma unroll
        for (int l = a2 + 1; l < NU; ++l) acc -= lr[l * NU + a2] * cu[l];
        cu[a2] = acc * rr[a2];
      }
    } else {
#pragma unroll
      for (int a2 = 0; a2 < NU; ++a2) cu[a2] = 0.0;
    }
  }
  lds_barrier();
  return av;
}

// flat prefetch of [factor record of knot kf | G of interval kg]; out-of-range kf / kg load a
// valid record whose words the sweeps never read (branch-free loads, see stage_prefetch)
template <typename T>
__device__ __forceinline__ void sol_prefetch(const Cfg& c, const Slot& s, int kf, int kg, int lane, T* reg) {
  const bool hf = kf >= 0 && kf <= c.N, hg = kg >= 0 && kg < c.N;
  const T* Fp = reinterpret_cast<const T*>(s.fac) + (long long)(hf ? kf : 0) * FR_LEN;
  const double* Gp = s.G + (long long)(hg ? kg : 0) * NX * NZ;
#pragma unroll
  for (int t = 0; t < SPF; ++t) {
    // as in stage_prefetch, only the group that straddles the record's end selects per lane
    const int q = lane + WAVE * t, lo = WAVE * t, hi = WAVE * t + WAVE;
    if (hi <= FR_LEN) {
      reg[t] = Fp[q];
    } else if (lo >= FR_LEN) {
      reg[t] = T(Gp[min(q - FR_LEN, NX * NZ - 1)]);
    } else if constexpr (sizeof(T) == sizeof(double)) {
      const double* a = (q < FR_LEN) ? reinterpret_cast<const double*>(Fp) + q : Gp + min(q - FR_LEN, NX * NZ - 1);
      reg[t] = *a;
    } else {
      const T fv = Fp[q < FR_LEN ? q : FR_LEN - 1];
      const double gv = Gp[q < FR_LEN ? 0 : min(q - FR_LEN, NX * NZ - 1)];
      reg[t] = q < FR_LEN ? fv : T(gv);
    }
  }
}
template <typename T>
__device__ __forceinline__ void sol_park(T* buf, int lane, const T* reg) {
#pragma unroll
  for (int t = 0; t < SPF; ++t) buf[lane + WAVE * t] = reg[t];
}

// Solve K [dv; dy] = [bv; bc] (and the eliminated p/n rows bp, bn in restoration) with the factor
// in s.fac and the stage data in s.sd.  Outputs xv (n), xc (m), xp, xn (m; restoration only).
template <typename T>
__device__ __forceinline__ void kkt_solve(const Cfg& c, const Slot& s, const Elim& e, const double* bv,
                                          const double* bc, const double* bp, const double* bn, double* xv,
                                          double* xc, double* xp, double* xn, SolLdsT<T>& V, int lane) {
  const int N = c.N, NI = c.NI, SL = sd_len(c);
  T reg[SPF];
  sol_prefetch(c, s, N, N - 1, lane, reg);      // first backward stage
  // 1. condensed stage right-hand sides (lambda 13, x 13, u 4 per knot) into LDS; outside
  //    restoration an entry is one word of b, all of them in one or two groups of loads
  if (!e.resto) {
    lanes_for<16>((N + 1) * RB_LEN, lane, [&](int q) {
      const int k = q / RB_LEN, i = q % RB_LEN;
      double v = 0.0;
      if (i < NX) v = bc[k * NX + i];
      else if (i < 2 * NX) v = bv[xo(k) + i - NX];
      else if (i < 2 * NX + NU && k < N) v = bv[uo(k) + i - 2 * NX];
      return DV<1>{{v}};
    }, [&](int q, const DV<1>& t) { V.rb[q] = T(t.v[0]); });
  } else {
    lanes_for<8>((N + 1) * RB_LEN, lane, [&](int q) {
      const int k = q / RB_LEN, i = q % RB_LEN;
      DV<5> t{{0.0, 0.0, 0.0, 1.0, 1.0}};
      if (i < NX) {
        const int r = k * NX + i;
        const double* sdk = s.sd + (long long)k * SL;
        t.v[0] = bc[r];
        t.v[1] = bp[r];
        t.v[2] = bn[r];
        t.v[3] = sdk[NZ + i];
        t.v[4] = sdk[NZ + NX + i];
      } else if (i < 2 * NX) {
        t.v[0] = bv[xo(k) + i - NX];
      } else if (i < 2 * NX + NU && k < N) {
        t.v[0] = bv[uo(k) + i - 2 * NX];
      }
      return t;
    }, [&](int q, const DV<5>& t) {
      const int i = q % RB_LEN;
      double val = t.v[0];
      if (i < NX) val += t.v[1] / (t.v[3] + e.dxp) - t.v[2] / (t.v[4] + e.dxp);
      V.rb[q] = T(val);
    });
  }
  lds_barrier();
  // position rows of x_k gather the slack rows of knot k, one knot per lane (each row's D and
  // right-hand side once for the three positions)
  for (int q = lane; q < N; q += WAVE) {
    const int k = 1 + q;
    const double* sdk = s.sd + (long long)k * SL;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
    for (int j = 0; j < NI; ++j) {
      const double* o7 = sdk + SD_HEAD + SD_OBS * j;
      const int r = go(c, k, j);
      const double sig = o7[0] + (e.lsq ? 0.0 : e.dxp);
      const double d = row_dreg(e, o7[1], o7[2]);
      const double D = sig / (1.0 + sig * d);
      double bg = bc[r];
      if (e.resto) bg += bp[r] / (o7[1] + e.dxp) - bn[r] / (o7[2] + e.dxp);
      const double bj = bv[so(c, k, j)];
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[t] += o7[3 + t] * D * (bj / sig + bg);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) V.rb[k * RB_LEN + NX + t] += T(acc[t]);
  }
  sol_park(V.buf, lane, reg);
  lds_barrier();
  // 2. backward sweep: rbar_k = r_k + G_k^T a_{k+1}.  The knots with a control (k < N) and with a
  //    predecessor (k > 0) are compile-time cases of the stage body: knot N, knots N-1..1, knot 0.
  const int li = lane < NX ? lane : NX - 1;
  auto bwd = [&](int k, auto has_u_tag, auto more_tag) {
    constexpr bool HAS_U = decltype(has_u_tag)::value, MORE = decltype(more_tag)::value;
    T reg[SPF];              // the next knot's record, in flight during this knot
    const T* B = V.buf;                  // factor of knot k | G_{k-1}
    if (MORE) sol_prefetch(c, s, k - 1, k - 2, lane, reg);
    const T* rbk = V.rb + k * RB_LEN;
    T ra[NX], ru[NU], cu[NU], bx;
#pragma unroll
    for (int l = 0; l < NX; ++l) ra[l] = rbk[l];
#pragma unroll
    for (int a2 = 0; a2 < NU; ++a2) ru[a2] = HAS_U ? rbk[2 * NX + a2] : T(0.0);
    const T rx = rbk[NX + li];
    const StageWords<T> W = stage_words(B, li);
    // column lz of G_{k-1} and the right-hand side entry it updates
    const int lz = lane < NZ ? lane : NZ - 1;
    T gc[NX], rbn = 0.0;
    if (MORE) {
#pragma unroll
      for (int l = 0; l < NX; ++l) gc[l] = B[FR_LEN + l * NZ + lz];
      rbn = V.rb[(k - 1) * RB_LEN + NX + lz];
    }
    sched_fence();
    const T av = stage_apply(B, W, HAS_U, ra, rx, ru, false, lane, bx, cu, V);
    if (MORE) {
      T al[NX];
#pragma unroll
      for (int l = 0; l < NX; ++l) al[l] = lane_bcast(av, l);
      if (lane < NZ) {
        T acc = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) acc += gc[l] * al[l];
        V.rb[(k - 1) * RB_LEN + NX + lane] = rbn + acc;
      }
      lds_barrier();
      sol_park(V.buf, lane, reg);
    }
    lds_barrier();
  };
  bwd(N, Flag<false>{}, Flag<true>{});
  for (int k = N - 1; k >= 1; --k) bwd(k, Flag<true>{}, Flag<true>{});
  bwd(0, Flag<true>{}, Flag<false>{});
  // 3. forward sweep with the lambda rows fed by G_{k-1} (dx_{k-1}, du_{k-1}); the buffer still
  //    holds the record of knot 0 from the last backward stage.  Cases: knot 0, knots 1..N-1, knot N.
  T dz[NZ];
#pragma unroll
  for (int l = 0; l < NZ; ++l) dz[l] = 0.0;
  auto fwd = [&](int k, auto has_u_tag, auto prev_tag) {
    constexpr bool HAS_U = decltype(has_u_tag)::value, PREV = decltype(prev_tag)::value;
    T reg[SPF];              // the next knot's record, in flight during this knot
    const T* B = V.buf;                  // factor of knot k | G_{k-1}
    if (HAS_U) sol_prefetch(c, s, k + 1, k, lane, reg);
    const T* rbk = V.rb + k * RB_LEN;
    T rai = rbk[li];
    T gr[NZ];                 // row li of G_{k-1}
    if (PREV) {
#pragma unroll
      for (int l = 0; l < NZ; ++l) gr[l] = B[FR_LEN + li * NZ + l];
    }
    T ra[NX], ru[NU], cu[NU], bx = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < NU; ++a2) ru[a2] = HAS_U ? rbk[2 * NX + a2] : T(0.0);
    const T rx = rbk[NX + li];
    const StageWords<T> W = stage_words(B, li);
    sched_fence();
    if (PREV) {
      T w = 0.0;
#pragma unroll
      for (int l = 0; l < NZ; ++l) w += gr[l] * dz[l];
      rai += w;
    }
#pragma unroll
    for (int l = 0; l < NX; ++l) ra[l] = lane_bcast(rai, l);
    const T av = stage_apply(B, W, HAS_U, ra, rx, ru, true, lane, bx, cu, V);
    if (lane < NX) {
      xc[k * NX + lane] = av;
      xv[xo(k) + lane] = bx;
    }
    if (HAS_U) {
      T u = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < NU; ++a2) u = (lane == a2) ? cu[a2] : u;
      if (lane < NU) xv[uo(k) + lane] = u;
    }
#pragma unroll
    for (int l = 0; l < NX; ++l) dz[l] = lane_bcast(bx, l);
#pragma unroll
    for (int a2 = 0; a2 < NU; ++a2) dz[NX + a2] = cu[a2];
    if (HAS_U) sol_park(V.buf, lane, reg);    // stage_apply ended with a barrier after its last read
    lds_barrier();
  };
  fwd(0, Flag<true>{}, Flag<false>{});
  for (int k = 1; k < N; ++k) fwd(k, Flag<true>{}, Flag<true>{});
  fwd(N, Flag<false>{}, Flag<true>{});
  __syncthreads();   // xv is read back by other lanes below
  // 4. recover slack steps, inequality multiplier steps and elastic steps
  lanes_for(N * NI, lane, [&](int q) {
    const int k = 1 + q / NI, j = q % NI;
    const double* o7 = s.sd + (long long)k * SL + SD_HEAD + SD_OBS * j;
    const int r = go(c, k, j);
    DV<13> t;
#pragma unroll
    for (int a = 0; a < 6; ++a) t.v[a] = o7[a];
    t.v[12] = bv[so(c, k, j)];
    t.v[6] = bc[r];
    t.v[7] = e.resto ? bp[r] : 0.0;
    t.v[8] = e.resto ? bn[r] : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) t.v[9 + a] = xv[xo(k) + a];
    return t;
  }, [&](int q, const DV<13>& t) {
    const int k = 1 + q / NI, j = q % NI;
    const double* o7 = t.v;
    const int r = go(c, k, j);
    const double sig = o7[0] + (e.lsq ? 0.0 : e.dxp);
    const double d = row_dreg(e, o7[1], o7[2]);
    const double D = sig / (1.0 + sig * d);
    double bg = t.v[6];
    if (e.resto) bg += t.v[7] / (o7[1] + e.dxp) - t.v[8] / (o7[2] + e.dxp);
    double jdx = 0.0;
    for (int a = 0; a < 3; ++a) jdx += o7[3 + a] * t.v[9 + a];
    const int si = so(c, k, j);
    const double bs = t.v[12];
    const double dyg = D * (jdx - bs / sig - bg);
    xc[r] = dyg;
    xv[si] = (bs + dyg) / sig;
  });
  __syncthreads();
  if (e.resto) {
    lanes_for(c.m, lane, [&](int r) { return DV<7>{{s.zp[r], s.p[r], s.zn[r], s.nn[r], bp[r], bn[r], xc[r]}}; },
              [&](int r, const DV<7>& t) {
                const double sp = t.v[0] / t.v[1] + e.dxp, sn = t.v[2] / t.v[3] + e.dxp;
                xp[r] = (t.v[4] + t.v[6]) / sp;
                xn[r] = (t.v[5] - t.v[6]) / sn;
              });
  }
  __syncthreads();
}

}  // namespace hipipm
