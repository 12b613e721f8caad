// Per-slot device bodies of one batched interior-point iteration (Sec. V): every slot runs its
// own branch of Table I, one 64-lane wavefront per slot.  The phases of a pass are
//
//   pre_body   phase dispatch, result write-out + slot refill (iteration-level batching, Sec. V),
//              convergence test (E_0), monotone barrier update (Table I row 7), right-hand side
//              of eq. (7), perturbation-free stage data of the KKT matrix
//   fac_body   inertia-correcting structured LDL^T of eq. (7) with slack condensation
//   sol_body   step, bound-multiplier steps, fraction to the boundary; least-squares multipliers
//   ls_body    tiny step (row 4), backtracking filter line search (row 1) with second-order
//              correction (row 2), acceptance, restoration entry/exit (row 6)
//
// The kernels that run them are in kernels.hip (one launch per phase, and the derivative
// kernel), iter_fp64.hip and iter_mixed.hip (all four phases of a slot in one launch).
#pragma once
#include "common.h"
#include "model.h"
#include "kkt.h"

namespace hipipm {

// ============================================================================ per-slot helpers
__device__ __forceinline__ double fdiv_safe(double a, double b) { return a / b; }

// The same value, opaque to the optimiser.  A loop body that takes its lane index through this
// computes everything derived from the index inside the body, instead of having it hoisted out
// of the loop and kept live (in registers) across all of the loop.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// -c at the current point into rc (restoration: -(c - p + n))
__device__ __forceinline__ void eval_c(const Cfg& c, const Slot& s, bool resto, int lane) {
  const int N = c.N, NI = c.NI;
  lanes_for((N + 1) * NX, lane, [&](int r) {
    const int k = r / NX, i = r % NX;
    return DV<2>{{s.v[xo(k) + i], (k == 0) ? s.th[i] : s.F[(k - 1) * NX + i]}};
  }, [&](int r, const DV<2>& t) { s.rc[r] = -(t.v[0] - t.v[1]); });
  lanes_for(N * NI, lane, [&](int q) {
    const int k = 1 + q / NI, j = q % NI;
    DV<8> t;
    double o[4];
    obs_at(c, s.th, j, k, o);
#pragma unroll
    for (int a = 0; a < 4; ++a) t.v[a] = o[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) t.v[4 + a] = s.v[xo(k) + a];
    t.v[7] = s.v[so(c, k, j)];
    return t;
  }, [&](int q, const DV<8>& t) {
    const int k = 1 + q / NI, j = q % NI;
    double g = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) { double e = t.v[4 + a] - t.v[a]; g += e * e; }
    s.rc[go(c, k, j)] = -(g - t.v[3] * t.v[3] - t.v[7]);
  });
  __syncthreads();
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<3>{{s.rc[r], s.p[r], s.nn[r]}}; },
              [&](int r, const DV<3>& t) { s.rc[r] = t.v[0] + (t.v[1] - t.v[2]); });
  __syncthreads();
}

// objective gradient g = grad f (regular) or grad f_R (restoration, v part) and A^T y into aty
__device__ __forceinline__ void eval_grad(const Cfg& c, const Slot& s, const double* yv, bool resto, double zeta, double* aty,
                          int lane) {
  const int N = c.N, NI = c.NI;
  // grad f (into g) and A^T y (into aty) in one lane loop.  Every load of a trip (v_i and its
  // reference or restoration point, the identity row, column r of G_k with y_{k+1}, the first
  // OBS_CHUNK inequality rows of knot k) is issued before the first use, from valid addresses on
  // every lane, two trips at a time, so that a pair of trips waits for memory once.
  struct AtyIn {
    double ys, vi, wi, gc[NX], yn[NX], oc[OBS_CHUNK], yg[OBS_CHUNK];
  };
  auto load_obs = [&](int j0, int ko, int ro, double* oc, double* yg) {
#pragma unroll
    for (int u = 0; u < OBS_CHUNK; ++u) {
      const int j = min(j0 + u, NI - 1);
      double o[4];
      obs_at(c, s.th, j, ko, o);
      oc[u] = ro == 0 ? o[0] : (ro == 1 ? o[1] : o[2]);
      yg[u] = yv[go(c, ko, j)];
    }
  };
  lanes_for<2>(c.n, lane, [&](int i) {
    AtyIn t;
    t.vi = s.v[i];
    t.wi = 0.0;
    if (resto) {
      t.wi = s.xr[i];
    } else if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      if (r < NX) t.wi = s.ref[k * NX + r];
    }
    if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      const int kg = k < N ? k : N - 1, ko = k >= 1 ? k : 1, ro = r < 3 ? r : 0;
      const double* Gk = s.G + (long long)kg * NX * NZ;
      t.ys = yv[k * NX + (r < NX ? r : 0)];
#pragma unroll
      for (int l = 0; l < NX; ++l) {
        t.gc[l] = Gk[l * NZ + r];
        t.yn[l] = yv[(kg + 1) * NX + l];
      }
      if (NI > 0) load_obs(0, ko, ro, t.oc, t.yg);
    } else {
      const int q = i - c.n_w;
      t.ys = yv[go(c, 1 + q / NI, q % NI)];
    }
    return t;
  }, [&](int i, const AtyIn& t) {
    double gi = 0.0;
    if (resto) {
      double d = fmin(1.0, 1.0 / fabs(t.wi));
      gi = zeta * d * d * (t.vi - t.wi);
    } else if (i < c.n_w) {
      int r = i % NZ;
      if (r < NX) {
        gi = 2.0 * c.qw * (t.vi - t.wi);
      } else {
        gi = 2.0 * c.rw * (t.vi - c.uh);
      }
    }
    s.g[i] = gi;
    double a = 0.0;
    if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      if (r < NX) a += t.ys;        // +I of the rows defining x_k
      if (k < N) {
#pragma unroll
        for (int l = 0; l < NX; ++l) a -= t.gc[l] * t.yn[l];
      }
      if (r < 3 && k >= 1) {
#pragma unroll
        for (int u = 0; u < OBS_CHUNK; ++u)
          if (u < NI) a += 2.0 * (t.vi - t.oc[u]) * t.yg[u];
        for (int j0 = OBS_CHUNK; j0 < NI; j0 += OBS_CHUNK) {
          double oc[OBS_CHUNK], yg[OBS_CHUNK];
          load_obs(j0, k, r, oc, yg);
#pragma unroll
          for (int u = 0; u < OBS_CHUNK; ++u)
            if (j0 + u < NI) a += 2.0 * (t.vi - oc[u]) * yg[u];
        }
      }
    } else {
      a = -t.ys;
    }
    aty[i] = a;
  });
  __syncthreads();
}

// z_L / z_U of v component i (0 if unbounded)
__device__ __forceinline__ void z_of(const Cfg& c, const Iter& it, int i, double& zl, double& zu) {
  zl = zu = 0.0;
  if (i < c.n_w) {
    int k = i / NZ, r = i % NZ;
    if (r >= NX && k < c.N) { zl = it.zlu[k * NU + r - NX]; zu = it.zuu[k * NU + r - NX]; }
  } else {
    zl = it.zls[i - c.n_w];
  }
}

struct ErrParts {
  double dual, prim, y1, z1;
  int nL, nU;
};

__device__ __forceinline__ ErrParts err_parts(const Cfg& c, const Slot& s, const Iter& it, const double* aty, int lane) {
  double dual = 0.0, nanf = 0.0, z1 = 0.0, y1 = 0.0, prim = 0.0;
  lanes_for(c.n, lane, [&](int i) {
    double zl, zu;
    z_of(c, it, i, zl, zu);
    return DV<4>{{s.g[i], aty[i], zl, zu}};
  }, [&](int i, const DV<4>& t) {
    const double zl = t.v[2], zu = t.v[3];
    double d = t.v[0] + t.v[1] - zl + zu;
    if (!isfinite(d)) nanf = 1.0;
    dual = fmax(dual, fabs(d));
    z1 += fabs(zl) + fabs(zu);
  });
  lanes_for(c.m, lane, [&](int r) {
    return DV<4>{{it.y[r], s.rc[r], it.resto ? s.zp[r] : 0.0, it.resto ? s.zn[r] : 0.0}};
  }, [&](int r, const DV<4>& t) {
    y1 += fabs(t.v[0]);
    double pr = fabs(t.v[1]);
    if (!isfinite(pr)) nanf = 1.0;
    prim = fmax(prim, pr);
    if (it.resto) {
      double dp = c.rho_resto - t.v[0] - t.v[2];
      double dn = c.rho_resto + t.v[0] - t.v[3];
      dual = fmax(dual, fmax(fabs(dp), fabs(dn)));
      z1 += fabs(t.v[2]) + fabs(t.v[3]);
    }
  });
  ErrParts e;
  e.dual = wmax(dual);
  e.prim = wmax(prim);
  e.y1 = wsum(y1);
  e.z1 = wsum(z1);
  if (wmax(nanf) > 0.0) e.dual = NAN;
  e.nL = c.N * NU + c.N * c.NI + (it.resto ? 2 * c.m : 0);
  e.nU = c.N * NU;
  return e;
}

// max |s z - mu| over the bounded components
__device__ __forceinline__ double compl_max(const Cfg& c, const Slot& s, const Iter& it, double mu, int lane) {
  double cm = 0.0;
  lanes_for(c.N * NU, lane, [&](int b) {
    const int k = b / NU, i = b % NU;
    return DV<3>{{s.v[uo(k) + i], it.zlu[b], it.zuu[b]}};
  }, [&](int b, const DV<3>& t) {
    const double u = t.v[0];
    cm = fmax(cm, fabs(u * t.v[1] - mu));
    cm = fmax(cm, fabs((c.umax - u) * t.v[2] - mu));
  });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<2>{{s.v[c.n_w + q], it.zls[q]}}; },
            [&](int q, const DV<2>& t) { cm = fmax(cm, fabs(t.v[0] * t.v[1] - mu)); });
  if (it.resto)
    lanes_for(c.m, lane, [&](int r) { return DV<4>{{s.p[r], s.zp[r], s.nn[r], s.zn[r]}}; },
              [&](int r, const DV<4>& t) {
                cm = fmax(cm, fabs(t.v[0] * t.v[1] - mu));
                cm = fmax(cm, fabs(t.v[2] * t.v[3] - mu));
              });
  return wmax(cm);
}

__device__ __forceinline__ double kkt_err(const Cfg& c, const ErrParts& e, double cm, int m) {
  double sd = 1.0, sc = 1.0;
  if (m + e.nL + e.nU > 0) sd = fmax(c.s_max, (e.y1 + e.z1) / (double)(m + e.nL + e.nU)) / c.s_max;
  if (e.nL + e.nU > 0) sc = fmax(c.s_max, e.z1 / (double)(e.nL + e.nU)) / c.s_max;
  double r = e.dual / sd;
  if (isnan(e.dual)) return NAN;
  r = fmax(r, e.prim);
  r = fmax(r, cm / sc);
  return r;
}

// reference value that entry i < n_w of v is weighed against (state rows), 0 for controls
__device__ __forceinline__ double obj_ref(const Slot& s, int i) {
  const int k = i / NZ, r = i % NZ;
  return r < NX ? s.ref[k * NX + r] : 0.0;
}
// term of entry i < n_w of the regular objective, added to a lane's partial sum (the lane takes
// its entries in increasing order, so every caller forms the same partial sums)
__device__ __forceinline__ void obj_term(const Cfg& c, int i, double vi, double ref, double& f) {
  if (i % NZ < NX) {
    double e = vi - ref;
    f += c.qw * e * e;
  } else {
    double e = vi - c.uh;
    f += c.rw * e * e;
  }
}
// lane partial sum of the regular objective at v
__device__ __forceinline__ double obj_regular_lane(const Cfg& c, const Slot& s, const double* v, int lane) {
  double f = 0.0;
  lanes_for(c.n_w, lane, [&](int i) { return DV<2>{{v[i], obj_ref(s, i)}}; },
            [&](int i, const DV<2>& t) { obj_term(c, i, t.v[0], t.v[1], f); });
  return f;
}
// objective value at v (regular) -- wave sum
__device__ __forceinline__ double obj_regular(const Cfg& c, const Slot& s, const double* v, int lane) {
  return wsum(obj_regular_lane(c, s, v, lane));
}

// restoration objective rho sum(p + n) + zeta/2 |D_R (v - x_R)|^2
__device__ __forceinline__ double obj_resto(const Cfg& c, const Slot& s, const double* v, const double* p, const double* nn,
                            double zeta, int lane) {
  double a = 0.0, q = 0.0;
  lanes_for(c.m, lane, [&](int r) { return DV<2>{{p[r], nn[r]}}; },
            [&](int r, const DV<2>& t) { a += t.v[0] + t.v[1]; });
  lanes_for(c.n, lane, [&](int i) { return DV<2>{{s.xr[i], v[i]}}; }, [&](int i, const DV<2>& t) {
    double d = fmin(1.0, 1.0 / fabs(t.v[0]));
    double e = t.v[1] - t.v[0];
    q += d * d * e * e;
  });
  return c.rho_resto * wsum(a) + 0.5 * zeta * wsum(q);
}

// sum of log-slacks of the bounded components; NaN if one is not positive
__device__ __forceinline__ double log_barrier(const Cfg& c, const double* v, const double* p, const double* nn, bool resto,
                              int lane) {
  double b = 0.0, bad = 0.0;
  lanes_for(c.N * NU, lane, [&](int bb) {
    const int k = bb / NU, i = bb % NU;
    return DV<1>{{v[uo(k) + i]}};
  }, [&](int bb, const DV<1>& t) {
    double u = t.v[0];
    double sl = u, su = c.umax - u;
    if (!(sl > 0.0) || !(su > 0.0)) bad = 1.0;
    else b += log(sl) + log(su);
  });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<1>{{v[c.n_w + q]}}; }, [&](int q, const DV<1>& t) {
    double sv = t.v[0];
    if (!(sv > 0.0)) bad = 1.0;
    else b += log(sv);
  });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<2>{{p[r], nn[r]}}; }, [&](int r, const DV<2>& t) {
      if (!(t.v[0] > 0.0) || !(t.v[1] > 0.0)) bad = 1.0;
      else b += log(t.v[0]) + log(t.v[1]);
    });
  if (wmax(bad) > 0.0) return NAN;
  return wsum(b);
}

// primal fraction to the boundary over the bounded components of (dv, dp, dn)
__device__ __forceinline__ double ftb_primal(const Cfg& c, const Slot& s, const double* dv, const double* dp, const double* dn,
                             bool resto, double tau, int lane) {
  double a = 1.0;
  lanes_for(c.N * NU, lane, [&](int bb) {
    const int k = bb / NU, i = bb % NU;
    return DV<2>{{s.v[uo(k) + i], dv[uo(k) + i]}};
  }, [&](int bb, const DV<2>& t) {
    double u = t.v[0], d = t.v[1];
    if (d < 0) a = fmin(a, -tau * u / d);
    if (d > 0) a = fmin(a, tau * (c.umax - u) / d);
  });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<2>{{dv[c.n_w + q], s.v[c.n_w + q]}}; },
            [&](int q, const DV<2>& t) {
              double d = t.v[0];
              if (d < 0) a = fmin(a, -tau * t.v[1] / d);
            });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<4>{{dp[r], s.p[r], dn[r], s.nn[r]}}; },
              [&](int r, const DV<4>& t) {
                if (t.v[0] < 0) a = fmin(a, -tau * t.v[1] / t.v[0]);
                if (t.v[2] < 0) a = fmin(a, -tau * t.v[3] / t.v[2]);
              });
  return wmin(a);
}

// bound-multiplier steps (eq. (6) rows 3-4 eliminated): into dzlu, dzuu, dzls, dzp, dzn
__device__ __forceinline__ void dz_recover(const Cfg& c, const Slot& s, const Iter& it, double mu, const double* dv,
                           const double* dp, const double* dn, int lane) {
  lanes_for(c.N * NU, lane, [&](int bb) {
    const int k = bb / NU, i = bb % NU;
    return DV<4>{{s.v[uo(k) + i], dv[uo(k) + i], it.zlu[bb], it.zuu[bb]}};
  }, [&](int bb, const DV<4>& t) {
    double u = t.v[0], d = t.v[1], zl = t.v[2], zu = t.v[3];
    double sl = u, su = c.umax - u;
    s.dzlu[bb] = (mu - sl * zl - zl * d) / sl;
    s.dzuu[bb] = (mu - su * zu + zu * d) / su;
  });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<3>{{s.v[c.n_w + q], dv[c.n_w + q], it.zls[q]}}; },
            [&](int q, const DV<3>& t) {
              double sv = t.v[0], d = t.v[1], z = t.v[2];
              s.dzls[q] = (mu - sv * z - z * d) / sv;
            });
  if (it.resto)
    lanes_for(c.m, lane, [&](int r) { return DV<6>{{s.p[r], s.zp[r], dp[r], s.nn[r], s.zn[r], dn[r]}}; },
              [&](int r, const DV<6>& t) {
                s.dzp[r] = (mu - t.v[0] * t.v[1] - t.v[1] * t.v[2]) / t.v[0];
                s.dzn[r] = (mu - t.v[3] * t.v[4] - t.v[4] * t.v[5]) / t.v[3];
              });
  __syncthreads();
}

__device__ __forceinline__ double ftb_dual(const Cfg& c, const Slot& s, const Iter& it, double tau, int lane) {
  double a = 1.0;
  lanes_for(c.N * NU, lane, [&](int bb) { return DV<4>{{s.dzlu[bb], it.zlu[bb], s.dzuu[bb], it.zuu[bb]}}; },
            [&](int bb, const DV<4>& t) {
              if (t.v[0] < 0) a = fmin(a, -tau * t.v[1] / t.v[0]);
              if (t.v[2] < 0) a = fmin(a, -tau * t.v[3] / t.v[2]);
            });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<2>{{s.dzls[q], it.zls[q]}}; }, [&](int q, const DV<2>& t) {
    if (t.v[0] < 0) a = fmin(a, -tau * t.v[1] / t.v[0]);
  });
  if (it.resto)
    lanes_for(c.m, lane, [&](int r) { return DV<4>{{s.dzp[r], s.zp[r], s.dzn[r], s.zn[r]}}; },
              [&](int r, const DV<4>& t) {
                if (t.v[0] < 0) a = fmin(a, -tau * t.v[1] / t.v[0]);
                if (t.v[2] < 0) a = fmin(a, -tau * t.v[3] / t.v[2]);
              });
  return wmin(a);
}

// Filter of a sub-problem: fc theta values, then fc phi values, in the slot record.  Its
// capacity fc = max_iter + 2 is never reached: every entry comes from an accepted iteration or a
// restoration entry.
// reject if theta >= theta_F and phi >= phi_F for some entry
__device__ __forceinline__ bool filter_ok(const Cfg& c, const double* filt, int nf, double th, double ph, int lane) {
  int bad = 0;
  lanes_for(nf, lane, [&](int i) { return DV<2>{{filt[i], filt[c.fc + i]}}; }, [&](int i, const DV<2>& t) {
    if (th >= t.v[0] && ph >= t.v[1]) bad = 1;
  });
  return wor(bad) == 0;
}

// add an entry, dropping the entries it dominates (which does not change what the filter
// rejects); returns the new count.  A stable compaction, 64 entries at a time: each lane keeps
// or drops its entry, a ballot gives the kept entries their new places (never above their old
// ones, so no entry of a later chunk is overwritten before it is read).
__device__ __forceinline__ int filter_add(const Cfg& c, double* filt, int nf, double th, double ph, int lane) {
  int w = 0;
  for (int base = 0; base < nf; base += WAVE) {
    const int i = base + lane;
    double a = 0.0, b = 0.0;
    bool keep = false;
    if (i < nf) {
      a = filt[i];
      b = filt[c.fc + i];
      keep = !(a >= th && b >= ph);
    }
    const unsigned long long kept = __ballot(keep);
    if (keep) {
      const int at = w + __popcll(kept & ((1ull << lane) - 1ull));
      filt[at] = a;
      filt[c.fc + at] = b;
    }
    w += __popcll(kept);
  }
  if (w < c.fc) {
    if (lane == 0) {
      filt[w] = th;
      filt[c.fc + w] = ph;
    }
    ++w;
  }
  __syncthreads();
  return w;
}

// ============================================================================ slot initialisation
// reference states x_ref,k (k = 0..N) of the cost, tabulated once per instance
__device__ __forceinline__ void fill_ref(const Cfg& c, const Slot& s, int lane) {
  for (int k = lane; k <= c.N; k += WAVE) {
    double xr[NX];
    ref_state(c, s.th, k, xr);
#pragma unroll
    for (int r = 0; r < NX; ++r) s.ref[k * NX + r] = xr[r];
  }
  __syncthreads();
}


// the scalar-block words a cold restart of a diverged warm start keeps: iterations and counters
__device__ __forceinline__ bool kept_on_restart(int q) {
  return q == SC_ITER || (q >= SC_ST_RESTO && q <= SC_ST_PASS) || q == SC_ST_SOLV || q == SC_ST_FFACT ||
         q == SC_ST_FSOLV || q == SC_ST_REF || q == SC_ST_FB || q == SC_ST_WSTART || q == SC_ST_RTK ||
         q == SC_ST_WDS || q == SC_ST_WDR || q == SC_ST_SOFTS || q == SC_ST_SOFTF || q == SC_ST_MUFB ||
         q == SC_ST_NEST ||
         (q >= SC_CYC_EVAL && q <= SC_CYC_LS);
}

// Starting point of the main sub-problem: cold (wp == nullptr: x_k = xbar0, u_k = hover thrust,
// slacks s = g(xbar0), y = 0) or the warm row wp (n_w primal values without slacks, then the m
// equality multipliers; slacks s = g(w)).  Pushed into the bounds by kappa_1, kappa_2 (warm_push
// for a warm point); z = 1 on the bounded components; mu0 = mu_init (warm_mu0); tau, empty filter.
// The reference trajectory must be tabulated.
__device__ __forceinline__ void start_point(const Cfg& c, const Slot& s, const double* wp, int lane) {
  const bool use_warm = wp != nullptr;
  // the cold and warm constants are loaded unconditionally and blended by value
  const double kc1 = c.kappa1, kc2 = c.kappa2, kw = c.warm_push, mc = c.mu_init, mw = c.warm_mu0;
  const double k1 = use_warm ? kw : kc1, k2 = use_warm ? kw : kc2;
  for (int i = lane; i < c.n; i += WAVE) {
    double x;
    if (i < c.n_w) {
      const int r = i % NZ;
      x = use_warm ? wp[i] : ((r < NX) ? s.th[r] : c.uh);
    } else {
      const int q = i - c.n_w, k = 1 + q / c.NI, j = q % c.NI;
      double o[4];
      obs_at(c, s.th, j, k, o);
      double g = 0.0;
      for (int t = 0; t < 3; ++t) {
        const double e = (use_warm ? wp[xo(k) + t] : s.th[t]) - o[t];
        g += e * e;
      }
      x = g - o[3] * o[3];
    }
    // push into the bounds
    if (i < c.n_w) {
      int k = i / NZ, r = i % NZ;
      if (r >= NX && k < c.N) {
        double l = 0.0, u = c.umax;
        double pl = fmin(k1 * fmax(1.0, fabs(l)), k2 * (u - l));
        double pu = fmin(k1 * fmax(1.0, fabs(u)), k2 * (u - l));
        x = fmax(x, l + pl);
        x = fmin(x, u - pu);
      }
    } else {
      x = fmax(x, 0.0 + k1 * 1.0);
    }
    s.v[i] = x;
  }
  for (int r = lane; r < c.m; r += WAVE) s.y[r] = use_warm ? wp[c.n_w + r] : 0.0;
  for (int b = lane; b < c.N * NU; b += WAVE) { s.zlu[b] = 1.0; s.zuu[b] = 1.0; }
  for (int q = lane; q < c.N * c.NI; q += WAVE) s.zls[q] = 1.0;
  __syncthreads();
  if (lane == 0) {
    const double mu0 = use_warm ? mw : mc;
    s.sc[SC_MU] = mu0;
    s.sc[SC_TAU] = fmax(c.tau_min, 1.0 - mu0);
    s.sc[SC_DXL] = 0.0;
    s.sc[SC_TINY] = 0.0;
    s.sc[SC_NF] = 0.0;
    s.sc[SC_THMAX] = 0.0;
    s.sc[SC_THMIN] = 0.0;
  }
  __syncthreads();
}

// Start an instance in a slot: cold, or from its row of `warm` (a row with a non-finite entry is
// rejected: cold start, counted).  With the warm-start gate the cold start is set up first (its
// least-squares multipliers give the reference E_mu0) and the warm point replaces it after that
// (sol_init_y); without it the warm point is the start.  Bound multipliers of a warm point come
// from stationarity in its INIT_Y pass (pre_init_y).  `restart`: the cold restart of a diverged
// warm start (warm is ignored, iterations and counters are kept).
__device__ __forceinline__ void init_instance(const Cfg& c, const Slot& s, int inst, const double* theta, const double* warm,
                              int lane, bool restart = false) {
  const double* th = theta + (long long)inst * c.n_theta;
  for (int i = lane; i < c.n_theta; i += WAVE) s.th[i] = th[i];
  const double* wp = (warm && !restart) ? warm + (long long)inst * (c.n_w + c.m) : nullptr;
  int bad = 0;
  if (wp)
    for (int i = lane; i < c.n_w + c.m; i += WAVE)
      if (!isfinite(wp[i])) bad = 1;
  const bool use_warm = wp && wor(bad) == 0;
  const bool gate = use_warm && c.warm_gate != 0;
  __syncthreads();
  fill_ref(c, s, lane);
  for (int q = lane; q < SC_LEN; q += WAVE)
    if (!(restart && kept_on_restart(q))) s.sc[q] = 0.0;
  __syncthreads();
  start_point(c, s, (use_warm && !gate) ? wp : nullptr, lane);
  if (lane == 0) {
    s.sc[SC_PHASE] = PH_INIT_Y;
    s.sc[SC_STATUS] = ST_RUNNING;
    s.sc[SC_INST] = inst;
    s.sc[SC_INITF] = 1.0;
    s.sc[SC_WARM] = (use_warm && !gate) ? 1.0 : 0.0;
    s.sc[SC_WSTAGE] = gate ? 1.0 : 0.0;
    s.sc[SC_MUFREE] = 1.0;
    if (!restart) s.sc[SC_ST_WSTART] = use_warm ? 1.0 : 0.0;
    s.sc[SC_ST_WREJ] = (wp && !use_warm) ? 1.0 : 0.0;
  }
  __syncthreads();
}


// ============================================================================ factor kernel
// finished instance: write the results (main problem, E_0 at the point), pop the next one
__device__ __forceinline__ void finish_slot(const Cfg& c, const Slot& s, const double* theta, const double* warm, Outs out,
                            Counters* cnt, bool refill, int lane) {
  Iter it = cur_iter(s, false);
  eval_c(c, s, false, lane);
  eval_grad(c, s, s.y, false, 0.0, s.vt, lane);
  ErrParts ep = err_parts(c, s, it, s.vt, lane);
  double E0 = kkt_err(c, ep, compl_max(c, s, it, 0.0, lane), c.m);
  double f = obj_regular(c, s, s.v, lane);
  const int inst = (int)s.sc[SC_INST];
  const long long b = (long long)inst;
  for (int i = lane; i < c.n; i += WAVE) {
    double zl, zu;
    z_of(c, it, i, zl, zu);
    if (out.x) out.x[b * c.n + i] = s.v[i];
    if (out.zl) out.zl[b * c.n + i] = zl;
    if (out.zu) out.zu[b * c.n + i] = zu;
  }
  if (out.y)
    for (int r = lane; r < c.m; r += WAVE) out.y[b * c.m + r] = s.y[r];
  __shared__ int next;
  if (lane == 0) {
    if (out.obj) out.obj[inst] = f;
    if (out.kkt) out.kkt[inst] = E0;
    if (out.status) out.status[inst] = (int)s.sc[SC_STATUS];
    if (out.iters) out.iters[inst] = (int)s.sc[SC_ITER];
    if (cnt) {
      atomicAdd(&cnt->st[0], (unsigned long long)s.sc[SC_ITER]);
      atomicAdd(&cnt->st[1], (unsigned long long)s.sc[SC_ST_RESTO]);
      atomicAdd(&cnt->st[2], (unsigned long long)s.sc[SC_ST_SOCT]);
      atomicAdd(&cnt->st[3], (unsigned long long)s.sc[SC_ST_SOCA]);
      atomicAdd(&cnt->st[4], (unsigned long long)s.sc[SC_ST_FACT]);
      atomicAdd(&cnt->st[5], (unsigned long long)s.sc[SC_ST_RENT]);
      atomicAdd(&cnt->st[6], (unsigned long long)s.sc[SC_ST_TINY]);
      atomicAdd(&cnt->st[7], (unsigned long long)s.sc[SC_ST_PASS]);
      atomicAdd(&cnt->st[8], 1ull);
      atomicAdd(&cnt->st[9], (unsigned long long)s.sc[SC_ST_SOLV]);
      atomicAdd(&cnt->st[10], (unsigned long long)s.sc[SC_ST_FFACT]);
      atomicAdd(&cnt->st[11], (unsigned long long)s.sc[SC_ST_FSOLV]);
      atomicAdd(&cnt->st[12], (unsigned long long)s.sc[SC_ST_REF]);
      atomicAdd(&cnt->st[13], (unsigned long long)s.sc[SC_ST_FB]);
      atomicAdd(&cnt->st[14], (unsigned long long)s.sc[SC_ST_WSTART]);
      atomicAdd(&cnt->st[15], (unsigned long long)s.sc[SC_ST_WREJ]);
      atomicAdd(&cnt->st[16], (unsigned long long)s.sc[SC_ST_WRST]);
      atomicAdd(&cnt->st[17], (unsigned long long)s.sc[SC_ST_RTK]);
      atomicAdd(&cnt->st[18], (unsigned long long)s.sc[SC_ST_WDS]);
      atomicAdd(&cnt->st[19], (unsigned long long)s.sc[SC_ST_WDR]);
      atomicAdd(&cnt->st[20], (unsigned long long)s.sc[SC_ST_SOFTS]);
      atomicAdd(&cnt->st[21], (unsigned long long)s.sc[SC_ST_SOFTF]);
      atomicAdd(&cnt->st[22], (unsigned long long)s.sc[SC_ST_MUFB]);
#pragma unroll
      for (int q = 0; q < 5; ++q) atomicAdd(&cnt->st[23 + q], (unsigned long long)s.sc[SC_CYC_EVAL + q]);
      atomicAdd(&cnt->st[28], (unsigned long long)s.sc[SC_ST_NEST]);
      atomicAdd(&cnt->done, 1);
      next = refill ? atomicAdd(&cnt->head, 1) : INT_MAX;
    } else {
      next = INT_MAX;
    }
  }
  __syncthreads();
  const int nx = next;
  if (cnt && nx < cnt->n_inst) {
    init_instance(c, s, nx, theta, warm, lane);
  } else {
    __syncthreads();
    if (lane == 0) s.sc[SC_PHASE] = PH_EMPTY;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------- mixed precision
// y = K x for the system of eq. (7) with the perturbations of e, slacks (and, in restoration, the
// elastic p, n) kept as variables of their own: the un-condensed system the condensed factor
// solves, assembled on the fly from W_k, G_k and the stage data.
__device__ __forceinline__ void kkt_matvec(const Cfg& c, const Slot& s, const Elim& e, const double* xv,
                                           const double* xc, const double* xp, const double* xn, double* yv,
                                           double* yc, double* yp, double* yn, int lane) {
  const int N = c.N, NI = c.NI, SL = sd_len(c);
  const double dx = e.lsq ? 0.0 : e.dxp, dc = e.lsq ? 0.0 : e.dcp;
  // primal rows of the knots
  for (int q = lane; q < (N + 1) * NZ; q += WAVE) {
    const int k = q / NZ, i = q % NZ;
    if (k == N && i >= NX) continue;
    const double* sdk = s.sd + (long long)k * SL;
    const int vi = k * NZ + i;
    double acc = (sdk[i] + dx) * xv[vi];
    if (k < N) {
      if (!e.lsq) {
        const double* W = s.HW + (long long)k * NZ * NZ + i * NZ;
        for (int j = 0; j < NZ; ++j) acc += W[j] * xv[k * NZ + j];
      }
      const double* G = s.G + (long long)k * NX * NZ;
      for (int l = 0; l < NX; ++l) acc -= G[l * NZ + i] * xc[(k + 1) * NX + l];
    }
    if (i < NX) acc += xc[k * NX + i];
    if (k >= 1 && i < 3)
      for (int j = 0; j < NI; ++j) {
        const double* o7 = sdk + SD_HEAD + SD_OBS * j;
        acc += o7[6] * xv[vi] + o7[3 + i] * xc[go(c, k, j)];
      }
    yv[vi] = acc;
  }
  // slack rows and inequality rows
  for (int q = lane; q < N * NI; q += WAVE) {
    const int k = 1 + q / NI, j = q % NI;
    const double* o7 = s.sd + (long long)k * SL + SD_HEAD + SD_OBS * j;
    const int si = so(c, k, j), r = go(c, k, j);
    yv[si] = (o7[0] + dx) * xv[si] - xc[r];
    double acc = -xv[si] - dc * xc[r];
    for (int t = 0; t < 3; ++t) acc += o7[3 + t] * xv[xo(k) + t];
    if (e.resto) {
      acc += xn[r] - xp[r];
      yp[r] = (o7[1] + dx) * xp[r] - xc[r];
      yn[r] = (o7[2] + dx) * xn[r] + xc[r];
    }
    yc[r] = acc;
  }
  // rows defining the states
  for (int r = lane; r < (N + 1) * NX; r += WAVE) {
    const int k = r / NX, i = r % NX;
    double acc = xv[xo(k) + i] - dc * xc[r];
    if (k >= 1) {
      const double* G = s.G + (long long)(k - 1) * NX * NZ + i * NZ;
      for (int l = 0; l < NZ; ++l) acc -= G[l] * xv[(k - 1) * NZ + l];
    }
    if (e.resto) {
      const double* sdk = s.sd + (long long)k * SL;
      acc += xn[r] - xp[r];
      yp[r] = (sdk[NZ + i] + dx) * xp[r] - xc[r];
      yn[r] = (sdk[NZ + NX + i] + dx) * xn[r] + xc[r];
    }
    yc[r] = acc;
  }
  __syncthreads();
}

// Solve K x = b with the stored factor.  FP64 factor: one solve.  FP32 factor: one FP32 solve,
// then sweeps of r = b - K x (FP64, full system) and x += K^{-1} r (FP32 solve) until
// |r|_inf <= refine_tol |b|_inf, at most refine_max sweeps; false if that was not reached.
__device__ __forceinline__ bool solve_refined(const Cfg& c, const Slot& s, const Elim& e, const double* bv,
                                              const double* bc, const double* bp, const double* bn, double* xv,
                                              double* xc, double* xp, double* xn, double* dyn, bool mixed, int lane) {
  if (!mixed || s.sc[SC_FPREC] == 0.0) {
    SolLdsT<double> V = sol_lds<double>(c, dyn);
    kkt_solve(c, s, e, bv, bc, bp, bn, xv, xc, xp, xn, V, lane);
    return true;
  }
  SolLdsT<float> V = sol_lds<float>(c, dyn);
  kkt_solve(c, s, e, bv, bc, bp, bn, xv, xc, xp, xn, V, lane);
  const int n = c.n, m = c.m;
  double bmax = 0.0;
  for (int i = lane; i < n; i += WAVE) bmax = fmax(bmax, fabs(bv[i]));
  for (int r = lane; r < m; r += WAVE) {
    bmax = fmax(bmax, fabs(bc[r]));
    if (e.resto) bmax = fmax(bmax, fmax(fabs(bp[r]), fabs(bn[r])));
  }
  bmax = wmax(bmax);
  int sweeps = 0;
  bool ok = false;
  for (;;) {
    kkt_matvec(c, s, e, xv, xc, xp, xn, s.qv, s.qc, s.qp, s.qn, lane);
    double rmax = 0.0;
    for (int i = lane; i < n; i += WAVE) {
      const double r = bv[i] - s.qv[i];
      s.qv[i] = r;
      rmax = fmax(rmax, fabs(r));
    }
    for (int r = lane; r < m; r += WAVE) {
      const double rc = bc[r] - s.qc[r];
      s.qc[r] = rc;
      rmax = fmax(rmax, fabs(rc));
      if (e.resto) {
        const double rp = bp[r] - s.qp[r], rn = bn[r] - s.qn[r];
        s.qp[r] = rp;
        s.qn[r] = rn;
        rmax = fmax(rmax, fmax(fabs(rp), fabs(rn)));
      }
    }
    rmax = wmax(rmax);
    __syncthreads();
    if (rmax <= c.refine_tol * bmax) { ok = true; break; }
    if (!isfinite(rmax) || sweeps >= c.refine_max) break;
    kkt_solve(c, s, e, s.qv, s.qc, s.qp, s.qn, s.ev, s.ec, s.ep, s.en, V, lane);
    for (int i = lane; i < n; i += WAVE) xv[i] += s.ev[i];
    for (int r = lane; r < m; r += WAVE) {
      xc[r] += s.ec[r];
      if (e.resto) { xp[r] += s.ep[r]; xn[r] += s.en[r]; }
    }
    __syncthreads();
    ++sweeps;
  }
  if (lane == 0) s.sc[SC_ST_REF] += sweeps;
  __syncthreads();
  return ok;
}

// the structured factorization in the precision of this iteration.  FENCE64: the FP64 factor
// groups its LDS reads behind scheduling fences (the mixed kernels, whose FP64 factor is the
// fallback path, leave its scheduling to the compiler: the fences cost them registers)
template <bool FENCE64 = true>
__device__ __forceinline__ int factor_any(const Cfg& c, const Slot& s, const Elim& e, FacLds& L, bool f32, int lane) {
  if (f32) return kkt_factor(c, s, e, *reinterpret_cast<FacLdsT<float>*>(&L), lane);   // only mixed kernels
  return kkt_factor<double, FENCE64>(c, s, e, L, lane);
}

// ---------------------------------------------------------------------------- k_pre
// Phase dispatch of one slot: result write-out and refill (FINISH), convergence and iteration
// limit tests (E_0), the monotone barrier update (Table I row 7), grad phi_mu, the right-hand
// side of eq. (7), theta_k and phi_k, and the perturbation-free stage data for the factorization.
// INIT_Y slots set up the least-squares multiplier system [[I, A^T], [A, 0]] instead.
__device__ __forceinline__ void pre_init_y(const Cfg& c, const Slot& s, int lane) {
  Iter it = cur_iter(s, false);
  eval_c(c, s, false, lane);
  eval_grad(c, s, s.y, false, 0.0, s.vt, lane);
  if (s.sc[SC_WARM] != 0.0) {
    // warm start: keep y; bound multipliers from stationarity grad f + A^T y - z_L + z_U = 0,
    // floored at mu0 / slack; filter bounds from theta_0; no least-squares system
    const double mu0 = s.sc[SC_MU];
    for (int b = lane; b < c.N * NU; b += WAVE) {
      const int vi = uo(b / NU) + b % NU;
      const double u = s.v[vi], r = s.g[vi] + s.vt[vi];
      s.zlu[b] = fmax(r, mu0 / u);
      s.zuu[b] = fmax(-r, mu0 / (c.umax - u));
    }
    for (int q = lane; q < c.N * c.NI; q += WAVE) {
      const int si = c.n_w + q;
      s.zls[q] = fmax(s.g[si] + s.vt[si], mu0 / s.v[si]);
    }
    double th0 = 0.0;
    for (int r = lane; r < c.m; r += WAVE) th0 += fabs(s.rc[r]);
    th0 = wsum(th0);
    __syncthreads();
    bool keep = true;
    if (s.sc[SC_WSTAGE] == 2.0) {
      // gate: keep the warm point only if E_mu0(warm) <= E_mu0(cold start)
      ErrParts ep = err_parts(c, s, it, s.vt, lane);
      const double ew = kkt_err(c, ep, compl_max(c, s, it, mu0, lane), c.m);
      keep = ew <= s.sc[SC_ECOLD];
      __syncthreads();
      if (!keep) {
        // rejected: back to the cold start and its least-squares multipliers (kept in y_R)
        start_point(c, s, nullptr, lane);
        for (int r = lane; r < c.m; r += WAVE) s.y[r] = s.yr[r];
      }
    }
    __syncthreads();
    if (lane == 0) {
      s.sc[SC_THMAX] = keep ? 1e4 * fmax(1.0, th0) : s.sc[SC_CTHMAX];
      s.sc[SC_THMIN] = keep ? 1e-4 * fmax(1.0, th0) : s.sc[SC_CTHMIN];
      if (!keep) { s.sc[SC_WARM] = 0.0; s.sc[SC_ST_WREJ] = 1.0; }
      s.sc[SC_WSTAGE] = 0.0;
      s.sc[SC_NF] = 0.0;
      s.sc[SC_INITF] = 0.0;
      s.sc[SC_PHASE] = PH_REGULAR;
    }
    __syncthreads();
    return;
  }
  for (int i = lane; i < c.n; i += WAVE) {
    double zl, zu;
    z_of(c, it, i, zl, zu);
    s.rv[i] = -(s.g[i] - zl + zu);
  }
  for (int r = lane; r < c.m; r += WAVE) s.dvs[r] = 0.0;   // zero constraint right-hand side
  Elim e{true, false, 0.0, 0.0, 0.0};
  kkt_stage_data(c, s, it, e, lane);
  if (lane == 0) s.sc[SC_WORK] = W_LSQ;
}

// Adaptive barrier update of the original problem (Table I row 7).  Free mode: mu from the
// complementarity by the LOQO rule, mu = sigma * avg with avg the mean of the products s_i z_i over
// the bounded components, xi = min_i(s_i z_i) / avg, sigma = 0.1 min(0.05 (1 - xi) / xi, 2)^3, kept in
// [tol / 10, mu_max]; it continues while E_0 of each new iterate is at most 0.9999 times the largest
// of the last four accepted ones.  Otherwise the monotone mode takes over from mu = 0.8 avg; once
// its barrier problem is solved (E_mu <= kappa_eps mu) with that progress the free mode resumes,
// else mu decreases monotonically.  A change of mu resets the filter.
__device__ __forceinline__ void mu_adaptive(const Cfg& c, const Slot& s, const Iter& it, const ErrParts& ep,
                                            double E0, double& mu, int lane) {
  double* sub = it.sub;
  const double mu_min = c.tol / 10.0;
  double sum = 0.0, mn = INFINITY;
  for (int b = lane; b < c.N * NU; b += WAVE) {
    const double u = s.v[uo(b / NU) + b % NU];
    const double p1 = u * it.zlu[b], p2 = (c.umax - u) * it.zuu[b];
    sum += p1 + p2;
    mn = fmin(mn, fmin(p1, p2));
  }
  for (int q = lane; q < c.N * c.NI; q += WAVE) {
    const double p = s.v[c.n_w + q] * it.zls[q];
    sum += p;
    mn = fmin(mn, p);
  }
  sum = wsum(sum);
  mn = wmin(mn);
  const int cnt = 2 * c.N * NU + c.N * c.NI;
  const double avg = cnt ? sum / cnt : 0.0, mnv = cnt ? mn : 0.0;
  double mumax = s.sc[SC_MUMAX];
  if (mumax == 0.0) mumax = 1e3 * fmax(avg, mu_min);           // set at the first iteration
  bool free = s.sc[SC_MUFREE] != 0.0, tiny = sub[5] != 0.0;
  int nrefs = (int)s.sc[SC_NREFS];
  double refs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) refs[i] = s.sc[SC_REFS + i];
  double nf = sub[6];
  double fb = 0.0;
  auto progress = [&](double e) {
    if (nrefs == 0) return true;
    double mx = refs[0];
    for (int i = 1; i < nrefs; ++i) mx = fmax(mx, refs[i]);
    return e <= 0.9999 * mx;
  };
  bool done = false;
  if (free && !progress(E0)) {
    // not enough progress: the monotone mode takes over
    free = false;
    fb = 1.0;
    const double nm = fmin(mumax, fmax(mu_min, 0.8 * avg));
    if (nm != mu) { mu = nm; nf = 0.0; }
    done = true;
  }
  if (!done && !free) {
    const double Emu = kkt_err(c, ep, compl_max(c, s, it, mu, lane), c.m);
    if (!(Emu <= c.kappa_eps * mu || tiny)) {
      done = true;                                               // barrier problem not solved yet
    } else if (progress(E0)) {
      free = true;                                               // progress: back to the free mode
      nrefs = 0;
    } else {
      tiny = false;
      const double nm = fmax(mu_min, fmin(c.kappa_mu * mu, pow(mu, c.theta_mu)));
      if (nm < mu) { mu = nm; nf = 0.0; }
      done = true;
    }
  }
  if (!done) {
    if (nrefs == 4) {
#pragma unroll
      for (int i = 1; i < 4; ++i) refs[i - 1] = refs[i];
      --nrefs;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) refs[i] = (i == nrefs) ? E0 : refs[i];
    ++nrefs;
    tiny = false;
    const double xi = avg > 0.0 ? mnv / avg : 1.0;
    const double t = fmin(0.05 * (1.0 - xi) / xi, 2.0);
    double nm = 0.1 * t * t * t * avg;
    nm = fmin(mumax, fmax(mu_min, nm));
    if (nm != mu) { mu = nm; nf = 0.0; }
  }
  __syncthreads();
  if (lane == 0) {
    sub[0] = mu;
    sub[1] = fmax(c.tau_min, 1.0 - mu);
    sub[5] = tiny ? 1.0 : 0.0;
    sub[6] = nf;
    s.sc[SC_MUMAX] = mumax;
    s.sc[SC_MUFREE] = free ? 1.0 : 0.0;
    s.sc[SC_NREFS] = nrefs;
#pragma unroll
    for (int i = 0; i < 4; ++i) s.sc[SC_REFS + i] = refs[i];
    s.sc[SC_ST_MUFB] += fb;
  }
  __syncthreads();
}

__device__ __forceinline__ void pre_body(const Cfg& c, const Slot& s, const double* theta, const double* warm,
                                         Outs out, Counters* cnt, int refill, int lane) {
  const int ph = (int)s.sc[SC_PHASE];
  if (ph == PH_EMPTY) return;
  __syncthreads();
  if (lane == 0) { s.sc[SC_ST_PASS] += 1.0; s.sc[SC_WORK] = W_NONE; s.sc[SC_FORCE64] = 0.0; }
  if (ph == PH_FINISH) { finish_slot(c, s, theta, warm, out, cnt, refill != 0, lane); return; }
  if (ph == PH_INIT_Y) { pre_init_y(c, s, lane); return; }

  const bool resto = (ph == PH_RESTO);
  if (s.sc[SC_WARM] != 0.0 && (resto || (c.warm_cap > 0 && s.sc[SC_ITER] >= c.warm_cap))) {
    // the warm start diverged (restoration, or too many iterations): restart cold in this slot,
    // keeping the iterations and counters spent so far
    __syncthreads();
    init_instance(c, s, (int)s.sc[SC_INST], theta, warm, lane, true);
    if (lane == 0) s.sc[SC_ST_WRST] = 1.0;
    __syncthreads();
    return;
  }
  Iter it = cur_iter(s, resto);
  double* sub = it.sub;   // mu, tau, dx_last, theta_max, theta_min, tiny, nf
  double mu = sub[0];
  double zeta = resto ? sqrt(mu) : 0.0;
  eval_c(c, s, resto, lane);
  eval_grad(c, s, it.y, resto, zeta, s.vt, lane);
  ErrParts ep = err_parts(c, s, it, s.vt, lane);
  const double E0 = kkt_err(c, ep, compl_max(c, s, it, 0.0, lane), c.m);
  __syncthreads();
  if (!isfinite(E0)) {
    if (lane == 0) { s.sc[SC_STATUS] = ST_NUMERICAL; s.sc[SC_PHASE] = PH_FINISH; }
    if (resto) for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.xr[i];
    return;
  }
  if (E0 <= c.tol) {
    if (!resto) {
      if (lane == 0) s.sc[SC_STATUS] = ST_CONVERGED;
      __syncthreads();
      finish_slot(c, s, theta, warm, out, cnt, refill != 0, lane);
    } else {
      for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.xr[i];
      if (lane == 0) { s.sc[SC_STATUS] = ST_INFEASIBLE; s.sc[SC_PHASE] = PH_FINISH; }
    }
    return;
  }
  if (s.sc[SC_ITER] >= c.max_iter) {
    if (!resto) {
      if (lane == 0) s.sc[SC_STATUS] = ST_MAX_ITER;
      __syncthreads();
      finish_slot(c, s, theta, warm, out, cnt, refill != 0, lane);
    } else {
      for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.xr[i];
      if (lane == 0) { s.sc[SC_STATUS] = ST_MAX_ITER; s.sc[SC_PHASE] = PH_FINISH; }
    }
    return;
  }
  // ---- barrier update (Table I row 7): adaptive with monotone fallback, or monotone ----
  if (!resto && c.mu_strategy == 1) {
    mu_adaptive(c, s, it, ep, E0, mu, lane);
  } else {
    const double mu_min = c.tol / 10.0;
    double tau = sub[1];
    double nf = sub[6];
    bool tiny = sub[5] != 0.0;
    for (;;) {
      double Emu = kkt_err(c, ep, compl_max(c, s, it, mu, lane), c.m);
      if (!(Emu <= c.kappa_eps * mu || tiny)) break;
      tiny = false;
      double nm = fmax(mu_min, fmin(c.kappa_mu * mu, pow(mu, c.theta_mu)));
      if (!(nm < mu)) break;
      mu = nm;
      tau = fmax(c.tau_min, 1.0 - mu);
      nf = 0.0;
      if (resto) {
        zeta = sqrt(mu);
        eval_grad(c, s, it.y, resto, zeta, s.vt, lane);
        ep = err_parts(c, s, it, s.vt, lane);
      }
    }
    __syncthreads();
    if (lane == 0) { sub[0] = mu; sub[1] = tau; sub[5] = tiny ? 1.0 : 0.0; sub[6] = nf; }
    __syncthreads();
  }
  // ---- barrier gradient, right-hand side of eq. (7), theta_k, phi_k ----
  // (the same lane loop forms this lane's partial sum of the regular objective at v)
  double freg = 0.0;
  lanes_for(c.n, lane, [&](int i) {
    return DV<4>{{s.g[i], s.v[i], s.vt[i], !resto && i < c.n_w ? obj_ref(s, i) : 0.0}};
  }, [&](int i, const DV<4>& t) {
    double gp = t.v[0];
    if (i < c.n_w) {
      int k = i / NZ, r = i % NZ;
      if (r >= NX && k < c.N) {
        double u = t.v[1];
        gp += -mu / u + mu / (c.umax - u);
      }
      if (!resto) obj_term(c, i, t.v[1], t.v[3], freg);
    } else {
      gp -= mu / t.v[1];
    }
    s.g[i] = gp;                       // now grad phi_mu
    s.rv[i] = -(gp + t.v[2]);
  });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<3>{{s.p[r], s.nn[r], it.y[r]}}; }, [&](int r, const DV<3>& t) {
      s.rp[r] = -(c.rho_resto - mu / t.v[0] - t.v[2]);
      s.rn[r] = -(c.rho_resto - mu / t.v[1] + t.v[2]);
    });
  double thk = 0.0;
  lanes_for<12>(c.m, lane, [&](int r) { return DV<1>{{s.rc[r]}}; }, [&](int r, const DV<1>& t) { thk += fabs(t.v[0]); });
  thk = wsum(thk);
  double fk = resto ? obj_resto(c, s, s.v, s.p, s.nn, zeta, lane) : wsum(freg);
  double phk = fk - mu * log_barrier(c, s.v, s.p, s.nn, resto, lane);
  Elim e{false, resto, 0.0, 0.0, zeta};
  kkt_stage_data(c, s, it, e, lane);
  if (lane == 0) {
    s.sc[SC_THK] = thk; s.sc[SC_PHK] = phk; s.sc[SC_FK] = fk; s.sc[SC_STEPMU] = mu;
    s.sc[SC_WORK] = W_STEP;
  }
}

// ---------------------------------------------------------------------------- k_fac
// Inertia-correcting factorization (Sec. IV "Inertia correction"): first without
// perturbation; on a singular matrix add delta_c = delta_c_bar mu^kappa_c; then grow delta_x
// from delta_0 (or kappa_minus times the last used value) by kappa_plus_bar / kappa_plus until
// the inertia is (n, m, 0) or delta_x exceeds delta_max.
template <bool FENCE64 = true>
__device__ __forceinline__ void fac_body(const Cfg& c, const Slot& s, FacLds& L, bool fused, bool mixed, int lane) {
  const int work = (int)s.sc[SC_WORK];
  if (work == W_NONE) return;
  bool f32 = mixed && c.prec == 1 && s.sc[SC_FORCE64] == 0.0;
  // the least-squares multiplier system (INIT_Y): one attempt, its status as the verdict
  const bool lsq = work == W_LSQ;
  const bool resto = !lsq && (int)s.sc[SC_PHASE] == PH_RESTO;
  double* sub = s.sc + (resto ? SC_RMU : SC_MU);
  const double mu = sub[0];
  // an FP64 redo of this iteration's factorization starts from the same delta_x^last
  const double dxl = (s.sc[SC_FORCE64] != 0.0) ? s.sc[SC_DXLSAVE] : sub[2];
  Elim e{lsq, resto, 0.0, 0.0, resto ? sqrt(mu) : 0.0};
  // one factorization call site (one inlined copy of the factor): the first attempt, the FP64
  // retake of an FP32 verdict, then the corrections
  int nfact = 0, st = 0;
  bool ok = false, corr = false;
  const int lane0 = lane;
  for (;;) {
    const int lane = opaque(lane0);
    st = factor_any<FENCE64>(c, s, e, L, f32, lane);
    ++nfact;
    if (lsq) break;
    if (st == 0) { ok = true; break; }
    if (f32) {
      // the inertia-correction decisions are FP64 ones: an FP32 verdict of wrong inertia, or a
      // pivot too close to zero for FP32 to tell its sign (status 3), is taken again in FP64, and
      // the rest of this iteration's correction runs in FP64
      f32 = false;
      if (lane == 0) s.sc[SC_ST_RTK] += 1.0;
      continue;
    }
    if (!corr) {
      corr = true;
      if (st == 2) e.dcp = c.delta_c_bar * pow(mu, c.kappa_c);
      e.dxp = (dxl == 0.0) ? c.delta_0 : fmax(c.delta_min, c.kappa_minus * dxl);
      continue;
    }
    if (st == 2 && e.dcp == 0.0) e.dcp = c.delta_c_bar * pow(mu, c.kappa_c);
    e.dxp *= (dxl == 0.0) ? c.kappa_plus_bar : c.kappa_plus;
    if (e.dxp > c.delta_max) break;
  }
  if (lsq) {
    if (lane == 0) { s.sc[SC_FSTAT] = st; s.sc[SC_FPREC] = f32 ? 1.0 : 0.0; }
    __syncthreads();
    return;
  }
  __syncthreads();
  if (lane == 0) {
    s.sc[SC_ST_FACT] += nfact;
    if (fused) s.sc[SC_ST_FFACT] += nfact;
    s.sc[SC_DXLSAVE] = dxl;
    if (ok && (e.dxp != 0.0)) sub[2] = e.dxp;
    s.sc[SC_FPREC] = f32 ? 1.0 : 0.0;
    s.sc[SC_LDX] = e.dxp;
    s.sc[SC_LDC] = e.dcp;
    s.sc[SC_FSTAT] = ok ? 0.0 : 1.0;
    s.sc[SC_STEP] = ok ? STEP_READY : STEP_ICFAIL;
  }
}

// ---------------------------------------------------------------------------- k_sol
// least-squares multipliers: keep y if finite and |y|_inf <= lambda_max, else y = 0; the first
// one also initialises the filter bounds theta_max, theta_min.  At the cold start of a gated warm
// start, E_mu0 of the cold start is recorded as the gate's reference and the warm point (row of
// `warm`) is loaded for the next INIT_Y pass.
template <bool FENCE64 = true>
__device__ __forceinline__ void sol_init_y(const Cfg& c, const Slot& s, const double* warm, double* sol_dyn,
                                           FacLds* L, bool fused, bool mixed, int lane) {
  Elim e{true, false, 0.0, 0.0, 0.0};
  bool fok = s.sc[SC_FSTAT] == 0.0;
  if (fok) fok = solve_refined(c, s, e, s.rv, s.dvs, nullptr, nullptr, s.dv, s.dy, nullptr, nullptr, sol_dyn, mixed, lane);
  if (mixed && !fok && L && s.sc[SC_FPREC] != 0.0) {
    // FP32 refinement failed: the least-squares system again in FP64
    if (lane == 0) { s.sc[SC_FORCE64] = 1.0; s.sc[SC_ST_FB] += 1.0; }
    __syncthreads();
    fac_body<FENCE64>(c, s, *L, fused, mixed, lane);
    fok = s.sc[SC_FSTAT] == 0.0;
    if (fok) fok = solve_refined(c, s, e, s.rv, s.dvs, nullptr, nullptr, s.dv, s.dy, nullptr, nullptr, sol_dyn, mixed, lane);
  }
  double ym = 0.0, bad = fok ? 0.0 : 1.0;
  if (fok)
    for (int r = lane; r < c.m; r += WAVE) {
      ym = fmax(ym, fabs(s.dy[r]));
      if (!isfinite(s.dy[r])) bad = 1.0;
    }
  ym = wmax(ym);
  const bool keep = wmax(bad) == 0.0 && ym <= c.lam_max;
  for (int r = lane; r < c.m; r += WAVE) s.y[r] = keep ? s.dy[r] : 0.0;
  double th0 = 0.0;
  for (int r = lane; r < c.m; r += WAVE) th0 += fabs(s.rc[r]);
  th0 = wsum(th0);
  __syncthreads();
  if (lane == 0) {
    if (s.sc[SC_INITF] != 0.0) {
      s.sc[SC_THMAX] = 1e4 * fmax(1.0, th0);
      s.sc[SC_THMIN] = 1e-4 * fmax(1.0, th0);
      s.sc[SC_NF] = 0.0;
      s.sc[SC_INITF] = 0.0;
    }
    s.sc[SC_PHASE] = PH_REGULAR;
    s.sc[SC_WORK] = W_NONE;
    if (fok) {
      s.sc[SC_ST_SOLV] += 1.0;
      if (fused) s.sc[SC_ST_FSOLV] += 1.0;
    }
  }
  __syncthreads();
  if (s.sc[SC_WSTAGE] == 1.0) {
    if (!warm) {
      // no warm rows in this call (replay): the gate cannot run, the cold start stays
      if (lane == 0) s.sc[SC_WSTAGE] = 0.0;
      __syncthreads();
      return;
    }
    // gate reference: E_mu0 at the cold start (least-squares y, z = 1; c and grad f of this pass)
    Iter it = cur_iter(s, false);
    eval_grad(c, s, s.y, false, 0.0, s.vt, lane);
    ErrParts ep = err_parts(c, s, it, s.vt, lane);
    const double ecold = kkt_err(c, ep, compl_max(c, s, it, c.warm_mu0, lane), c.m);
    for (int r = lane; r < c.m; r += WAVE) s.yr[r] = s.y[r];
    __syncthreads();
    if (lane == 0) {
      s.sc[SC_ECOLD] = ecold;
      s.sc[SC_CTHMAX] = s.sc[SC_THMAX];
      s.sc[SC_CTHMIN] = s.sc[SC_THMIN];
    }
    __syncthreads();
    start_point(c, s, warm + (long long)(int)s.sc[SC_INST] * (c.n_w + c.m), lane);
    if (lane == 0) {
      s.sc[SC_WARM] = 1.0;
      s.sc[SC_WSTAGE] = 2.0;
      s.sc[SC_PHASE] = PH_INIT_Y;
    }
    __syncthreads();
  }
}

// Step of eq. (7) from the stored factor, bound-multiplier steps, fraction to the boundary
// (primal) and the directional derivative of phi_mu.
template <bool FENCE64 = true>
__device__ __forceinline__ void sol_body(const Cfg& c, const Slot& s, const double* warm, double* sol_dyn, FacLds* L,
                                         bool fused, bool mixed, int lane) {
  const int work = (int)s.sc[SC_WORK];
  if (work == W_NONE) return;
  if (work == W_LSQ) { sol_init_y<FENCE64>(c, s, warm, sol_dyn, L, fused, mixed, lane); return; }
  if ((int)s.sc[SC_STEP] != STEP_READY) {
    __syncthreads();
    if (lane == 0) s.sc[SC_WORK] = W_NONE;
    return;
  }
  const bool resto = (int)s.sc[SC_PHASE] == PH_RESTO;
  Iter it = cur_iter(s, resto);
  const double mu = it.sub[0], tau = it.sub[1];
  Elim e{false, resto, s.sc[SC_LDX], s.sc[SC_LDC], resto ? sqrt(mu) : 0.0};
  if (!solve_refined(c, s, e, s.rv, s.rc, s.rp, s.rn, s.dv, s.dy, s.dp, s.dn, sol_dyn, mixed, lane) && L) {
    // FP32 refinement failed: factor this iteration again in FP64 (same inertia-correction start)
    if (lane == 0) { s.sc[SC_FORCE64] = 1.0; s.sc[SC_ST_FB] += 1.0; }
    __syncthreads();
    fac_body<FENCE64>(c, s, *L, fused, mixed, lane);
    __syncthreads();
    if ((int)s.sc[SC_STEP] != STEP_READY) {
      if (lane == 0) s.sc[SC_WORK] = W_NONE;
      return;
    }
    e.dxp = s.sc[SC_LDX];
    e.dcp = s.sc[SC_LDC];
    solve_refined(c, s, e, s.rv, s.rc, s.rp, s.rn, s.dv, s.dy, s.dp, s.dn, sol_dyn, mixed, lane);
  }
  dz_recover(c, s, it, mu, s.dv, s.dp, s.dn, lane);
  double amax = ftb_primal(c, s, s.dv, s.dp, s.dn, resto, tau, lane);
  double gphi = 0.0;
  lanes_for<12>(c.n, lane, [&](int i) { return DV<2>{{s.g[i], s.dv[i]}}; },
            [&](int i, const DV<2>& t) { gphi += t.v[0] * t.v[1]; });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<4>{{s.p[r], s.dp[r], s.nn[r], s.dn[r]}}; },
              [&](int r, const DV<4>& t) {
                gphi += (c.rho_resto - mu / t.v[0]) * t.v[1] + (c.rho_resto - mu / t.v[2]) * t.v[3];
              });
  gphi = wsum(gphi);
  __syncthreads();
  if (lane == 0) {
    s.sc[SC_AMAX] = amax;
    s.sc[SC_GPHI] = gphi;
    s.sc[SC_WORK] = W_NONE;
    s.sc[SC_ST_SOLV] += 1.0;
    if (fused) s.sc[SC_ST_FSOLV] += 1.0;
  }
}

// ============================================================================ line search kernel
struct Trial {
  double th, ph;
  bool fin;
};

// evaluate the trial point vt (pt, nt): constraints into ct, theta = |ct|_1, phi_mu.  The
// initial-state rows and the first inequality rows are loaded before the RK4 of each lane's
// interval, so that their memory round trip overlaps it.  freg: this lane's partial sum of the
// regular objective at vt (make_trial forms it; unused in restoration).
__device__ __forceinline__ Trial eval_trial(const Cfg& c, const Slot& s, bool resto, double mu, double zeta, double freg,
                                            int lane) {
  const int N = c.N, NI = c.NI;
  // rows defining x_0 and the first inequality group: loads issued first
  const int l0 = lane < NX ? lane : 0;
  const double x0v = s.vt[l0], x0t = s.th[l0];
  auto obs_ld = [&](int q) {
    const int k = 1 + q / NI, j = q % NI;
    DV<8> t;
    double o[4];
    obs_at(c, s.th, j, k, o);
#pragma unroll
    for (int a = 0; a < 4; ++a) t.v[a] = o[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) t.v[4 + a] = s.vt[xo(k) + a];
    t.v[7] = s.vt[so(c, k, j)];
    return t;
  };
  auto obs_use = [&](int q, const DV<8>& t) {
    const int k = 1 + q / NI, j = q % NI;
    double g = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) { double e = t.v[4 + a] - t.v[a]; g += e * e; }
    const double cv = g - t.v[3] * t.v[3] - t.v[7];
    s.ct[go(c, k, j)] = cv;
  };
  constexpr int OG = 4;                 // inequality trips per lane loaded ahead
  const int nq = N * NI;
  DV<8> og[OG];
  if (nq > 0) {
#pragma unroll
    for (int u = 0; u < OG; ++u) og[u] = obs_ld(min(lane + u * WAVE, nq - 1));
  }
  if (lane < N) {
    double x[NX], u[NU], F[NX], xn[NX];
    for (int i = 0; i < NX; ++i) x[i] = s.vt[xo(lane) + i];
    for (int i = 0; i < NU; ++i) u[i] = s.vt[uo(lane) + i];
    for (int i = 0; i < NX; ++i) xn[i] = s.vt[xo(lane + 1) + i];
    rk4(c, x, u, F);
    for (int i = 0; i < NX; ++i) {
      const double cv = xn[i] - F[i];
      s.ct[(lane + 1) * NX + i] = cv;
    }
  }
  if (lane < NX) s.ct[lane] = x0v - x0t;
#pragma unroll
  for (int u = 0; u < OG; ++u)
    if (lane + u * WAVE < nq) obs_use(lane + u * WAVE, og[u]);
  if (nq > OG * WAVE) {
    const int rest = nq - OG * WAVE;
    lanes_for(rest, lane, [&](int q) { return obs_ld(OG * WAVE + q); },
              [&](int q, const DV<8>& t) { obs_use(OG * WAVE + q, t); });
  }
  __syncthreads();
  if (resto) {
    lanes_for(c.m, lane, [&](int r) { return DV<3>{{s.ct[r], s.pt[r], s.nt[r]}}; },
              [&](int r, const DV<3>& t) { s.ct[r] = t.v[0] + (-t.v[1] + t.v[2]); });
    __syncthreads();
  }
  double th = 0.0;
  lanes_for<12>(c.m, lane, [&](int r) { return DV<1>{{s.ct[r]}}; }, [&](int r, const DV<1>& t) { th += fabs(t.v[0]); });
  th = wsum(th);
  double f = resto ? obj_resto(c, s, s.vt, s.pt, s.nt, zeta, lane) : wsum(freg);
  double ph = f - mu * log_barrier(c, s.vt, s.pt, s.nt, resto, lane);
  Trial t;
  t.th = th;
  t.ph = ph;
  t.fin = isfinite(th) && isfinite(ph);
  return t;
}

// trial point v + a dv (p + a dp, n + a dn); returns this lane's partial sum of the regular
// objective at it (0 in restoration)
__device__ __forceinline__ double make_trial(const Cfg& c, const Slot& s, bool resto, double a, const double* dv,
                                             const double* dp, const double* dn, int lane) {
  const int nw = c.n_w;
  double f = 0.0;
  lanes_for<12>(c.n, lane, [&](int i) { return DV<3>{{s.v[i], dv[i], !resto && i < nw ? obj_ref(s, i) : 0.0}}; },
            [&](int i, const DV<3>& t) {
              const double vt = t.v[0] + a * t.v[1];
              s.vt[i] = vt;
              if (!resto && i < nw) obj_term(c, i, vt, t.v[2], f);
            });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<4>{{s.p[r], dp[r], s.nn[r], dn[r]}}; }, [&](int r, const DV<4>& t) {
      s.pt[r] = t.v[0] + a * t.v[1];
      s.nt[r] = t.v[2] + a * t.v[3];
    });
  __syncthreads();
  return f;
}

struct Acc {
  bool ok, sw, arm;
};

__device__ __forceinline__ Acc acceptable(const Cfg& c, const double* sub, const double* filt, double thk, double phk, double gphi,
                          double alpha, const Trial& t, int lane) {
  Acc r{false, false, false};
  if (!t.fin) return r;
  if (t.th > sub[3]) return r;
  bool sw = gphi < 0 && alpha * pow(-gphi, c.s_phi) > c.delta_sw * pow(thk, c.s_theta);
  double slack = 10.0 * 2.220446049250313e-16 * fabs(phk);
  bool arm = (t.ph - (phk + c.eta_phi * alpha * gphi)) <= slack;
  bool ok;
  if (sw && thk <= sub[4]) ok = arm;
  else ok = (t.th <= (1.0 - c.gamma_theta) * thk) || ((t.ph - (phk - c.gamma_phi * thk)) <= slack);
  if (!ok) return r;
  if (!filter_ok(c, filt, (int)sub[6], t.th, t.ph, lane)) return r;
  r.ok = true;
  r.sw = sw;
  r.arm = arm;
  return r;
}

// enter feasibility restoration from the main iterate; false if it cannot start
__device__ __forceinline__ bool resto_enter(const Cfg& c, const Slot& s, int lane) {
  const double thk = s.sc[SC_THK], phk = s.sc[SC_PHK];
  if (thk <= c.tol) return false;
  if (lane == 0) { s.sc[SC_WD_ACTIVE] = 0.0; s.sc[SC_WD_SHORT] = 0.0; s.sc[SC_SOFT] = 0.0; }
  const int nf = filter_add(c, s.fm, (int)s.sc[SC_NF], (1.0 - c.gamma_theta) * thk, phk - c.gamma_phi * thk, lane);
  double cmax = 0.0;
  for (int r = lane; r < c.m; r += WAVE) cmax = fmax(cmax, fabs(s.rc[r]));
  cmax = wmax(cmax);
  const double mu = s.sc[SC_MU];
  const double muR = fmax(mu, cmax);
  const double rho = c.rho_resto;
  for (int i = lane; i < c.n; i += WAVE) s.xr[i] = s.v[i];
  double th0 = 0.0;
  for (int r = lane; r < c.m; r += WAVE) {
    double cv = -s.rc[r];
    double a = (muR - rho * cv) / (2.0 * rho);
    double nn = a + sqrt(a * a + muR * cv / (2.0 * rho));
    double pp = cv + nn;
    s.p[r] = pp;
    s.nn[r] = nn;
    s.zp[r] = muR / pp;
    s.zn[r] = muR / nn;
    s.yr[r] = 0.0;
    th0 += fabs(cv - pp + nn);
  }
  th0 = wsum(th0);
  for (int b = lane; b < c.N * NU; b += WAVE) { s.rzlu[b] = fmin(rho, s.zlu[b]); s.rzuu[b] = fmin(rho, s.zuu[b]); }
  for (int q = lane; q < c.N * c.NI; q += WAVE) s.rzls[q] = fmin(rho, s.zls[q]);
  __syncthreads();
  if (lane == 0) {
    s.sc[SC_NF] = nf;
    s.sc[SC_THR] = thk;
    s.sc[SC_RMU] = muR;
    s.sc[SC_RTAU] = fmax(c.tau_min, 1.0 - muR);
    s.sc[SC_RDXL] = 0.0;
    s.sc[SC_RTINY] = 0.0;
    s.sc[SC_RNF] = 0.0;
    s.sc[SC_RTHMAX] = 1e4 * fmax(1.0, th0);
    s.sc[SC_RTHMIN] = 1e-4 * fmax(1.0, th0);
    s.sc[SC_ST_RENT] += 1.0;
    s.sc[SC_PHASE] = PH_RESTO;
  }
  __syncthreads();
  return true;
}

// Nested hard restoration (Table I row 6): the restoration phase cannot make progress at
// (x, p, n).  Its own restoration problem -- minimise the violation of c(x) - p + n = 0 -- has
// (p, n) free and entering that constraint linearly, so its minimiser keeps x and takes, row by
// row, the (p, n) that minimises rho (p + n) - mu (ln p + ln n) subject to c(x) - p + n = 0 (the
// closed form that starts the restoration phase, at the restoration phase's current mu), with
// z_p = mu / p, z_n = mu / n.  The failing point enters the restoration filter, as an iterate
// does when it leaves for restoration.  Counts as a restoration iteration.  false (nothing done)
// when the restoration constraints already hold within tol, where restoring them cannot help.
__device__ __forceinline__ bool nested_resto(const Cfg& c, const Slot& s, const Iter& it, int lane) {
  const double thk = s.sc[SC_THK], phk = s.sc[SC_PHK];
  if (!(thk > c.tol)) return false;
  double* sub = it.sub;
  const int nf = filter_add(c, it.filt, (int)sub[6], (1.0 - c.gamma_theta) * thk, phk - c.gamma_phi * thk, lane);
  eval_c(c, s, false, lane);   // rc = -c(x)
  const double mu = sub[0], rho = c.rho_resto;
  for (int r = lane; r < c.m; r += WAVE) {
    double cv = -s.rc[r];
    double a = (mu - rho * cv) / (2.0 * rho);
    double nn = a + sqrt(a * a + mu * cv / (2.0 * rho));
    double pp = cv + nn;
    s.p[r] = pp;
    s.nn[r] = nn;
    s.zp[r] = mu / pp;
    s.zn[r] = mu / nn;
  }
  __syncthreads();
  if (lane == 0) {
    sub[6] = nf;
    s.sc[SC_ITER] += 1.0;
    s.sc[SC_ST_RESTO] += 1.0;
    s.sc[SC_ST_NEST] += 1.0;
  }
  __syncthreads();
  return true;
}

// after an accepted restoration step: return to the original problem if possible
__device__ __forceinline__ void resto_try_exit(const Cfg& c, const Slot& s, int lane) {
  // original constraints and barrier objective at v (main mu)
  for (int i = lane; i < c.n; i += WAVE) s.vt[i] = s.v[i];
  __syncthreads();
  const double mu = s.sc[SC_MU];
  Trial t = eval_trial(c, s, false, mu, 0.0, obj_regular_lane(c, s, s.vt, lane), lane);
  if (!t.fin) return;
  if (!(t.th <= c.kappa_resto * s.sc[SC_THR])) return;
  if (!filter_ok(c, s.fm, (int)s.sc[SC_NF], t.th, t.ph, lane)) return;
  double zmax = 0.0;
  for (int b = lane; b < c.N * NU; b += WAVE) zmax = fmax(zmax, fmax(s.rzlu[b], s.rzuu[b]));
  for (int q = lane; q < c.N * c.NI; q += WAVE) zmax = fmax(zmax, s.rzls[q]);
  zmax = wmax(zmax);
  const bool reset = zmax > c.bound_mult_reset;
  for (int b = lane; b < c.N * NU; b += WAVE) {
    s.zlu[b] = reset ? 1.0 : s.rzlu[b];
    s.zuu[b] = reset ? 1.0 : s.rzuu[b];
  }
  for (int q = lane; q < c.N * c.NI; q += WAVE) s.zls[q] = reset ? 1.0 : s.rzls[q];
  __syncthreads();
  if (lane == 0) {
    s.sc[SC_TINY] = 0.0;
    s.sc[SC_NREFS] = 0.0;   // the adaptive update restarts its progress record
    s.sc[SC_PHASE] = PH_INIT_Y;
  }
  __syncthreads();
}

// A^T y of the original problem at the point v (Jacobian evaluated there) into out
__device__ __forceinline__ void aty_at(const Cfg& c, const Slot& s, const double* v, const double* y, double* out,
                                       int lane) {
  const int N = c.N, NI = c.NI;
  for (int i = lane; i < c.n; i += WAVE) {
    double a = 0.0;
    if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      if (r < NX) a += y[k * NX + r];        // +I of the rows defining x_k
      if (r < 3 && k >= 1)
        for (int j = 0; j < NI; ++j) {
          double o[4];
          obs_at(c, s.th, j, k, o);
          a += 2.0 * (v[i] - o[r]) * y[go(c, k, j)];
        }
    } else {
      const int q = i - c.n_w, k = 1 + q / NI, j = q % NI;
      a = -y[go(c, k, j)];
    }
    out[i] = a;
  }
  __syncthreads();
  // -G_k^T y_{k+1}: one (interval, column) per item, the column from a forward tangent sweep
  for (int q = lane; q < N * NZ; q += WAVE) {
    const int k = q / NZ, j = q % NZ;
    double x[NX], u[NU], g[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = v[xo(k) + i];
#pragma unroll
    for (int i = 0; i < NU; ++i) u[i] = v[uo(k) + i];
    rk4_tangent(c, x, u, j, g);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < NX; ++l) acc += g[l] * y[(k + 1) * NX + l];
    out[k * NZ + j] -= acc;
  }
  __syncthreads();
}

// primal-dual error of the barrier problem at mu in the 1-norm: |grad f + A^T y - z_L + z_U|_1 +
// |c|_1 + |S_L z_L - mu e|_1 + |S_U z_U - mu e|_1.  g = grad f, aty = A^T y, cv = +-c (only |c|).
__device__ __forceinline__ double pd_error(const Cfg& c, const double* v, const double* g, const double* aty,
                                           const double* cv, const double* zlu, const double* zuu,
                                           const double* zls, double mu, int lane) {
  double e = 0.0;
  for (int i = lane; i < c.n; i += WAVE) {
    double zl = 0.0, zu = 0.0;
    if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      if (r >= NX && k < c.N) { zl = zlu[k * NU + r - NX]; zu = zuu[k * NU + r - NX]; }
    } else {
      zl = zls[i - c.n_w];
    }
    e += fabs(g[i] + aty[i] - zl + zu);
  }
  for (int r = lane; r < c.m; r += WAVE) e += fabs(cv[r]);
  for (int b = lane; b < c.N * NU; b += WAVE) {
    const double u = v[uo(b / NU) + b % NU];
    e += fabs(u * zlu[b] - mu) + fabs((c.umax - u) * zuu[b] - mu);
  }
  for (int q = lane; q < c.N * c.NI; q += WAVE) e += fabs(v[c.n_w + q] * zls[q] - mu);
  return wsum(e);
}

// objective gradient of the original problem at v into g
__device__ __forceinline__ void grad_f_at(const Cfg& c, const Slot& s, const double* v, double* g, int lane) {
  for (int i = lane; i < c.n; i += WAVE) {
    double gi = 0.0;
    if (i < c.n_w) {
      const int k = i / NZ, r = i % NZ;
      gi = (r < NX) ? 2.0 * c.qw * (v[i] - s.ref[k * NX + r]) : 2.0 * c.rw * (v[i] - c.uh);
    }
    g[i] = gi;
  }
  __syncthreads();
}

// Soft feasibility restoration step (Table I row 5): the primal-dual Newton step with one step size
// alpha = min(alpha_max primal, alpha_max dual) for primal and dual variables, accepted when it
// lowers the primal-dual error of the barrier problem by the factor soft_factor (the line-search
// test is not applied).  The trial point is left in vt / ct (its theta and phi in *t).  Returns
// true when accepted (iterate updated, kappa_Sigma safeguard on z).
__device__ __forceinline__ bool soft_step(const Cfg& c, const Slot& s, const Iter& it, double mu, double tau,
                                          double amax, Trial* t, int lane) {
  const double ad = ftb_dual(c, s, it, tau, lane);
  const double as = fmin(amax, ad);
  // error at the current point: grad f, A^T y (Jacobian of this pass), c (-c in rc)
  grad_f_at(c, s, s.v, s.qv, lane);
  aty_at(c, s, s.v, s.y, s.ev, lane);
  const double e0 = pd_error(c, s.v, s.qv, s.ev, s.rc, s.zlu, s.zuu, s.zls, mu, lane);
  // the trial
  const double freg = make_trial(c, s, false, as, s.dv, s.dp, s.dn, lane);
  for (int r = lane; r < c.m; r += WAVE) s.syt[r] = s.y[r] + as * s.dy[r];
  for (int b = lane; b < c.N * NU; b += WAVE) {
    s.szlu[b] = s.zlu[b] + as * s.dzlu[b];
    s.szuu[b] = s.zuu[b] + as * s.dzuu[b];
  }
  for (int q = lane; q < c.N * c.NI; q += WAVE) s.szls[q] = s.zls[q] + as * s.dzls[q];
  __syncthreads();
  *t = eval_trial(c, s, false, mu, 0.0, freg, lane);
  grad_f_at(c, s, s.vt, s.qv, lane);
  aty_at(c, s, s.vt, s.syt, s.ev, lane);
  const double e1 = pd_error(c, s.vt, s.qv, s.ev, s.ct, s.szlu, s.szuu, s.szls, mu, lane);
  if (!(e1 <= c.soft_factor * e0)) return false;
  const double ks = c.kappa_sigma;
  for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.vt[i];
  for (int r = lane; r < c.m; r += WAVE) s.y[r] = s.syt[r];
  __syncthreads();
  for (int b = lane; b < c.N * NU; b += WAVE) {
    const double u = s.v[uo(b / NU) + b % NU], su = c.umax - u;
    s.zlu[b] = fmax(fmin(s.szlu[b], ks * mu / u), mu / (ks * u));
    s.zuu[b] = fmax(fmin(s.szuu[b], ks * mu / su), mu / (ks * su));
  }
  for (int q = lane; q < c.N * c.NI; q += WAVE) {
    const double sv = s.v[c.n_w + q];
    s.zls[q] = fmax(fmin(s.szls[q], ks * mu / sv), mu / (ks * sv));
  }
  __syncthreads();
  if (lane == 0) { s.sc[SC_LALPHA] = as; s.sc[SC_LALPHAZ] = as; s.sc[SC_LSOC] = 0.0; }
  return true;
}

__device__ __forceinline__ void ls_body(const Cfg& c, const Slot& s, double* sol_dyn, bool fused, bool mixed,
                                        int lane) {
  const int ph = (int)s.sc[SC_PHASE];
  if (ph != PH_REGULAR && ph != PH_RESTO) return;
  const int step = (int)s.sc[SC_STEP];
  if (step == STEP_NONE) return;
  __syncthreads();
  if (lane == 0) s.sc[SC_STEP] = STEP_NONE;
  const bool resto = (ph == PH_RESTO);
  Iter it = cur_iter(s, resto);
  double* sub = it.sub;
  const double mu = sub[0], tau = sub[1];
  const double zeta = resto ? sqrt(mu) : 0.0;
  const double thk = s.sc[SC_THK], phk = s.sc[SC_PHK], gphi = s.sc[SC_GPHI], amax = s.sc[SC_AMAX];
  bool accepted = false, augment = false, soc_dir = false, tiny = false, shortened = false;
  double ap = amax;
  double aug_th = thk, aug_ph = phk;        // the point whose (theta, phi) enters the filter
  const bool use_wd = !resto && c.wd_trigger > 0;
  const bool use_soft = !resto && c.soft_max > 0;
  if (use_wd && s.sc[SC_WD_ACTIVE] != 0.0 && mu != s.sc[SC_WD_MU]) {
    // a new barrier problem ends the watchdog (its reference belongs to the previous one)
    __syncthreads();
    if (lane == 0) s.sc[SC_WD_ACTIVE] = 0.0;
    __syncthreads();
  }
  // in soft restoration there is no line search: the soft step, or hard restoration
  bool try_soft = use_soft && s.sc[SC_SOFT] != 0.0;
  if (step == STEP_READY && !try_soft) {
    // tiny step (Table I row 4) at a nearly feasible point
    double tmax = 0.0, cmax = 0.0;
    lanes_for(c.n, lane, [&](int i) { return DV<2>{{s.dv[i], s.v[i]}}; },
              [&](int i, const DV<2>& t) { tmax = fmax(tmax, fabs(t.v[0]) / (1.0 + fabs(t.v[1]))); });
    if (resto)
      lanes_for(c.m, lane, [&](int r) { return DV<4>{{s.dp[r], s.p[r], s.dn[r], s.nn[r]}}; },
                [&](int r, const DV<4>& t) {
                  tmax = fmax(tmax, fabs(t.v[0]) / (1.0 + fabs(t.v[1])));
                  tmax = fmax(tmax, fabs(t.v[2]) / (1.0 + fabs(t.v[3])));
                });
    lanes_for<12>(c.m, lane, [&](int r) { return DV<1>{{s.rc[r]}}; },
              [&](int r, const DV<1>& t) { cmax = fmax(cmax, fabs(t.v[0])); });
    tmax = wmax(tmax);
    cmax = wmax(cmax);
    if (tmax < 10.0 * 2.220446049250313e-16 && cmax <= 1e-4) {
      make_trial(c, s, resto, amax, s.dv, s.dp, s.dn, lane);
      tiny = true;
      accepted = true;
      if (use_wd && lane == 0) s.sc[SC_WD_ACTIVE] = 0.0;
    } else if (use_wd && (s.sc[SC_WD_ACTIVE] != 0.0 || s.sc[SC_WD_SHORT] >= c.wd_trigger)) {
      // watchdog (Table I row 3): full steps without the line-search test after wd_trigger
      // shortened steps; a step acceptable with respect to the iterate where the watchdog started
      // ends it as an ordinary acceptance; if the wd_max-th is not, the iterate goes back to that
      // reference point and the next pass takes the ordinary line search from there
      if (s.sc[SC_WD_ACTIVE] == 0.0) {
        for (int i = lane; i < c.n; i += WAVE) s.wdv[i] = s.v[i];
        for (int r = lane; r < c.m; r += WAVE) s.wdy[r] = s.y[r];
        for (int b = lane; b < c.N * NU; b += WAVE) { s.wdzlu[b] = s.zlu[b]; s.wdzuu[b] = s.zuu[b]; }
        for (int q = lane; q < c.N * c.NI; q += WAVE) s.wdzls[q] = s.zls[q];
        __syncthreads();
        if (lane == 0) {
          s.sc[SC_WD_ACTIVE] = 1.0;
          s.sc[SC_WD_ITER] = 0.0;
          s.sc[SC_WD_THK] = thk; s.sc[SC_WD_PHK] = phk; s.sc[SC_WD_GPHI] = gphi; s.sc[SC_WD_AMAX] = amax;
          s.sc[SC_WD_MU] = mu;
          s.sc[SC_ST_WDS] += 1.0;
        }
        __syncthreads();
      }
      const double freg = make_trial(c, s, resto, amax, s.dv, s.dp, s.dn, lane);
      Trial t = eval_trial(c, s, resto, mu, zeta, freg, lane);
      const double wthk = s.sc[SC_WD_THK], wphk = s.sc[SC_WD_PHK];
      Acc a = acceptable(c, sub, it.filt, wthk, wphk, s.sc[SC_WD_GPHI], s.sc[SC_WD_AMAX], t, lane);
      const double wit = s.sc[SC_WD_ITER] + 1.0;
      __syncthreads();
      if (a.ok) {
        augment = !(a.sw && a.arm);
        aug_th = wthk;
        aug_ph = wphk;
        if (lane == 0) { s.sc[SC_WD_ACTIVE] = 0.0; s.sc[SC_WD_SHORT] = 0.0; s.sc[SC_WD_ITER] = wit; }
      } else if (wit >= c.wd_max) {
        // revert to the reference iterate; no step is accepted in this pass
        for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.wdv[i];
        for (int r = lane; r < c.m; r += WAVE) s.y[r] = s.wdy[r];
        for (int b = lane; b < c.N * NU; b += WAVE) { s.zlu[b] = s.wdzlu[b]; s.zuu[b] = s.wdzuu[b]; }
        for (int q = lane; q < c.N * c.NI; q += WAVE) s.zls[q] = s.wdzls[q];
        if (lane == 0) {
          s.sc[SC_WD_ACTIVE] = 0.0;
          s.sc[SC_WD_SHORT] = 0.0;
          s.sc[SC_WD_ITER] = wit;
          s.sc[SC_ST_WDR] += 1.0;
        }
        __syncthreads();
        return;
      } else if (lane == 0) {
        s.sc[SC_WD_ITER] = wit;
      }
      accepted = true;
      __syncthreads();
    } else {
      double amin;
      if (gphi < 0) {
        double t = fmin(c.gamma_theta, c.gamma_phi * thk / (-gphi));
        if (thk <= sub[4]) t = fmin(t, c.delta_sw * pow(thk, c.s_theta) / pow(-gphi, c.s_phi));
        amin = c.gamma_alpha * t;
      } else {
        amin = c.gamma_alpha * c.gamma_theta;
      }
      double alpha = amax;
      const int lane0 = lane;
      for (int l = 0;; ++l) {
        const int lane = opaque(lane0);
        // alpha_min, or 60 halvings (alpha_min is 0 at an exactly feasible point; the restoration
        // phase takes at most resto_ls_max)
        if (alpha < amin || l >= (resto ? c.resto_ls_max : 60)) {
          try_soft = use_soft;          // the line search failed: soft restoration, if enabled
          break;
        }
        const double freg = make_trial(c, s, resto, alpha, s.dv, s.dp, s.dn, lane);
        Trial t = eval_trial(c, s, resto, mu, zeta, freg, lane);
        Acc a = acceptable(c, sub, it.filt, thk, phk, gphi, alpha, t, lane);
        if (a.ok) {
          ap = alpha;
          augment = !(a.sw && a.arm);
          accepted = true;
          shortened = l > 0;
          break;
        }
        if (l == 0 && t.fin && c.max_soc > 0 && t.th >= thk) {
          // second-order correction with the stored factor (Table I row 2)
          double asoc = alpha, th_old = 0.0, tht = t.th;
          bool fin = true;
          lanes_for<12>(c.m, lane, [&](int r) { return DV<1>{{s.rc[r]}}; },
                    [&](int r, const DV<1>& t) { s.csoc[r] = -t.v[0]; });
          __syncthreads();
          Elim e{false, resto, s.sc[SC_LDX], s.sc[SC_LDC], zeta};
          for (int p = 0; p < c.max_soc; ++p) {
            const int lane = opaque(lane0);
            if (p > 0 && !(tht <= c.kappa_soc * th_old)) break;
            th_old = tht;
            lanes_for<12>(c.m, lane, [&](int r) { return DV<2>{{s.csoc[r], s.ct[r]}}; }, [&](int r, const DV<2>& t) {
              const double cs = asoc * t.v[0] + t.v[1];
              s.csoc[r] = cs;
              s.ct[r] = -cs;      // right-hand side rows of the constraints
            });
            __syncthreads();
            if (!solve_refined(c, s, e, s.rv, s.ct, s.rp, s.rn, s.dvs, s.dys, s.dps, s.dns, sol_dyn, mixed, lane)) break;
            if (lane == 0) {
              s.sc[SC_ST_SOCT] += 1.0;
              if (fused) s.sc[SC_ST_FSOLV] += 1.0;
            }
            asoc = ftb_primal(c, s, s.dvs, s.dps, s.dns, resto, tau, lane);
            const double fsoc = make_trial(c, s, resto, asoc, s.dvs, s.dps, s.dns, lane);
            Trial ts = eval_trial(c, s, resto, mu, zeta, fsoc, lane);
            tht = ts.th;
            fin = ts.fin;
            Acc as = acceptable(c, sub, it.filt, thk, phk, gphi, alpha, ts, lane);
            if (as.ok) {
              ap = asoc;
              augment = !(as.sw && as.arm);
              accepted = true;
              soc_dir = true;
              shortened = true;
              if (lane == 0) s.sc[SC_ST_SOCA] += 1.0;
              break;
            }
            if (!fin) break;
          }
          if (accepted) break;
        }
        alpha *= 0.5;
      }
    }
  }
  __syncthreads();
  if (try_soft && step == STEP_READY) {
    if (s.sc[SC_SOFT] == 0.0) {
      // the line search failed: soft restoration starts at this iterate
      if (lane == 0) {
        s.sc[SC_SOFT] = 1.0;
        s.sc[SC_SOFT_IT] = 0.0;
        s.sc[SC_SOFT_THK] = thk;
        s.sc[SC_SOFT_PHK] = phk;
        s.sc[SC_WD_ACTIVE] = 0.0;
        s.sc[SC_WD_SHORT] = 0.0;
      }
      __syncthreads();
    }
    Trial t{0.0, 0.0, false};
    const bool ok = s.sc[SC_SOFT_IT] < c.soft_max && soft_step(c, s, it, mu, tau, amax, &t, lane);
    if (ok) {
      // back to the ordinary iteration once the point is acceptable to the filter with a
      // sufficient decrease of theta or phi_mu over the point where soft restoration started
      // (which then enters the filter)
      const double rth = s.sc[SC_SOFT_THK], rph = s.sc[SC_SOFT_PHK];
      const bool dec = t.th <= (1.0 - c.gamma_theta) * rth ||
                       (t.ph - (rph - c.gamma_phi * rth)) <= 10.0 * 2.220446049250313e-16 * fabs(rph);
      const bool leave = t.fin && t.th <= sub[3] && dec && filter_ok(c, it.filt, (int)sub[6], t.th, t.ph, lane);
      if (leave) {
        const int nf = filter_add(c, it.filt, (int)sub[6], (1.0 - c.gamma_theta) * rth, rph - c.gamma_phi * rth,
                                  lane);
        if (lane == 0) sub[6] = nf;
      }
      if (lane == 0) {
        if (leave) s.sc[SC_SOFT] = 0.0;
        s.sc[SC_SOFT_IT] += 1.0;
        s.sc[SC_ST_SOFTS] += 1.0;
        s.sc[SC_ITER] += 1.0;
      }
      __syncthreads();
      return;
    }
    if (lane == 0) { s.sc[SC_SOFT] = 0.0; s.sc[SC_ST_SOFTF] += 1.0; }
    __syncthreads();
  }
  if (!accepted) {
    // line search or inertia correction failed
    if (!resto) {
      if (!resto_enter(c, s, lane))
        if (lane == 0) { s.sc[SC_STATUS] = ST_RESTO_FAILED; s.sc[SC_PHASE] = PH_FINISH; }
    } else if (!(c.nested_resto && nested_resto(c, s, it, lane))) {
      for (int i = lane; i < c.n; i += WAVE) s.v[i] = s.xr[i];
      if (lane == 0) { s.sc[SC_STATUS] = ST_RESTO_FAILED; s.sc[SC_PHASE] = PH_FINISH; }
    }
    __syncthreads();
    return;
  }
  // ---- accept: (Table I) primal and y with the primal step, z with the dual fraction to the boundary
  if (soc_dir) dz_recover(c, s, it, mu, s.dvs, s.dps, s.dns, lane);
  const double az = ftb_dual(c, s, it, tau, lane);
  const double* ady = soc_dir ? s.dys : s.dy;
  if (augment) {
    const int nf = filter_add(c, it.filt, (int)sub[6], (1.0 - c.gamma_theta) * aug_th, aug_ph - c.gamma_phi * aug_th,
                              lane);
    if (lane == 0) sub[6] = nf;
  }
  if (use_wd && lane == 0 && s.sc[SC_WD_ACTIVE] == 0.0)
    s.sc[SC_WD_SHORT] = shortened ? s.sc[SC_WD_SHORT] + 1.0 : 0.0;
  lanes_for<12>(c.m, lane, [&](int r) { return DV<2>{{it.y[r], ady[r]}}; },
            [&](int r, const DV<2>& t) { it.y[r] = t.v[0] + ap * t.v[1]; });
  lanes_for<12>(c.n, lane, [&](int i) { return DV<1>{{s.vt[i]}}; }, [&](int i, const DV<1>& t) { s.v[i] = t.v[0]; });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<2>{{s.pt[r], s.nt[r]}}; }, [&](int r, const DV<2>& t) {
      s.p[r] = t.v[0];
      s.nn[r] = t.v[1];
    });
  __syncthreads();
  const double ks = c.kappa_sigma;
  lanes_for(c.N * NU, lane, [&](int b) {
    const int k = b / NU, i = b % NU;
    return DV<5>{{s.v[uo(k) + i], it.zlu[b], s.dzlu[b], it.zuu[b], s.dzuu[b]}};
  }, [&](int b, const DV<5>& t) {
    double u = t.v[0];
    double z = t.v[1] + az * t.v[2];
    it.zlu[b] = fmax(fmin(z, ks * mu / u), mu / (ks * u));
    double su = c.umax - u;
    z = t.v[3] + az * t.v[4];
    it.zuu[b] = fmax(fmin(z, ks * mu / su), mu / (ks * su));
  });
  lanes_for(c.N * c.NI, lane, [&](int q) { return DV<3>{{s.v[c.n_w + q], it.zls[q], s.dzls[q]}}; },
            [&](int q, const DV<3>& t) {
              double sv = t.v[0];
              double z = t.v[1] + az * t.v[2];
              it.zls[q] = fmax(fmin(z, ks * mu / sv), mu / (ks * sv));
            });
  if (resto)
    lanes_for(c.m, lane, [&](int r) { return DV<6>{{s.zp[r], s.dzp[r], s.p[r], s.zn[r], s.dzn[r], s.nn[r]}}; },
              [&](int r, const DV<6>& t) {
                double z = t.v[0] + az * t.v[1];
                s.zp[r] = fmax(fmin(z, ks * mu / t.v[2]), mu / (ks * t.v[2]));
                z = t.v[3] + az * t.v[4];
                s.zn[r] = fmax(fmin(z, ks * mu / t.v[5]), mu / (ks * t.v[5]));
              });
  __syncthreads();
  if (lane == 0) {
    if (tiny) { sub[5] = 1.0; s.sc[SC_ST_TINY] += 1.0; }
    s.sc[SC_ITER] += 1.0;
    if (resto) s.sc[SC_ST_RESTO] += 1.0;
    s.sc[SC_LALPHA] = ap;
    s.sc[SC_LALPHAZ] = az;
    s.sc[SC_LSOC] = soc_dir ? 1.0 : 0.0;
  }
  __syncthreads();
  if (resto) resto_try_exit(c, s, lane);
}

__host__ __device__ __forceinline__ size_t sol_bytes(const Cfg& c) { return (size_t)sol_lds_doubles(c.N) * sizeof(double); }
// The fused kernels' one dynamic LDS region: the factorization's workspace and the solve's, which
// no phase uses at the same time (the factor records go to the slot record, not LDS).
__host__ __device__ __forceinline__ size_t pass_lds_bytes(const Cfg& c) {
  const size_t f = sizeof(FacLds), v = sol_bytes(c);
  return f > v ? f : v;
}

// The four per-slot phases of one pass back to back, with the shader-clock cycles of each added to
// the slot's counters (the fused and asynchronous-slot kernels).
template <bool MIXED>
__device__ __forceinline__ void pass_phases(const Cfg& c, const Slot& s, const double* theta, const double* warm,
                                            Outs out, Counters* cnt, int refill, FacLds& L, double* sol_dyn,
                                            int lane) {
  const long long t0 = clock64();
  pre_body(c, s, theta, warm, out, cnt, refill, lane);
  __syncthreads();
  const long long t1 = clock64();
  fac_body<!MIXED>(c, s, L, true, MIXED, lane);
  __syncthreads();
  const long long t2 = clock64();
  sol_body<!MIXED>(c, s, warm, sol_dyn, &L, true, MIXED, lane);
  __syncthreads();
  const long long t3 = clock64();
  ls_body(c, s, sol_dyn, true, MIXED, lane);
  __syncthreads();
  const long long t4 = clock64();
  if (lane == 0 && (int)s.sc[SC_PHASE] != PH_EMPTY) {
    s.sc[SC_CYC_PRE] += (double)(t1 - t0);
    s.sc[SC_CYC_FAC] += (double)(t2 - t1);
    s.sc[SC_CYC_SOL] += (double)(t3 - t2);
    s.sc[SC_CYC_LS] += (double)(t4 - t3);
  }
}

// Derivatives of one slot at its current point (what the derivative kernel computes for it): RK4
// step F_k, G_k = dF/d(x, u) and W_k = -sum_r y_r Hess F_r per interval, one (interval, direction)
// item per lane.
// The stage points (x_k, u_k) and the multipliers y_{k+1}, k < N, are first copied into LDS (lds:
// the pass's dynamic LDS region, free before the factorization) in a few groups of loads, so that
// each of the directions a lane evaluates in turn reads its inputs from LDS, not from memory.
constexpr int EVAL_LDS_DOUBLES = MAX_N * (NZ + NX);
static_assert(EVAL_LDS_DOUBLES * sizeof(double) <= sizeof(FacLds), "derivative inputs exceed the pass LDS region");
__device__ __forceinline__ void eval_slot(const Cfg& c, const Slot& s, double* lds, int lane) {
  const int ph = (int)s.sc[SC_PHASE];
  const double* yv = (ph == PH_RESTO) ? s.yr : s.y;
  const int nz = c.N * NZ, ny = c.N * NX;
  double* lv = lds;            // v[0, N NZ): x_k, u_k
  double* ly = lds + nz;       // y[NX, (N+1) NX): y_{k+1}
  lanes_for(nz, lane, [&](int q) { return DV<2>{{s.v[q], yv[NX + min(q, ny - 1)]}}; },
            [&](int q, const DV<2>& t) {
              lv[q] = t.v[0];
              if (q < ny) ly[q] = t.v[1];
            });
  __syncthreads();
  for (int q = lane; q < c.N * NZ; q += WAVE) {
    const int k = q / NZ, j = q % NZ;
    double x[NX], u[NU], lam[NX], Fv[NX], Gc[NX], Hc[NZ];
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = lv[xo(k) + i];
#pragma unroll
    for (int i = 0; i < NU; ++i) u[i] = lv[uo(k) + i];
#pragma unroll
    for (int i = 0; i < NX; ++i) lam[i] = -ly[k * NX + i];
    rk4_deriv_dir(c, x, u, lam, j, j == 0 ? Fv : nullptr, Gc, Hc);
    double* G = s.G + (long long)k * NX * NZ;
    double* H = s.HW + (long long)k * NZ * NZ;
#pragma unroll
    for (int i = 0; i < NX; ++i) G[i * NZ + j] = Gc[i];
#pragma unroll
    for (int i = 0; i < NZ; ++i) H[i * NZ + j] = Hc[i];
    if (j == 0) {
#pragma unroll
      for (int i = 0; i < NX; ++i) s.F[k * NX + i] = Fv[i];
    }
  }
  __syncthreads();
}

// Asynchronous slots: each workgroup owns one slot and runs up to `passes` whole passes of it
// back to back (its derivatives, then the four phases), taking new instances from the device queue
// as its own finish; no slot waits for another between passes.  A slot that finds nothing left
// leaves at once, so every wave ends after at most `passes` passes.
template <bool MIXED>
__global__ __launch_bounds__(64) void k_run(Cfg c0, double* ws, const double* theta, const double* warm, Outs out,
                                            Counters* cnt, int passes) {
  HIP_DYNAMIC_SHARED(double, sol_dyn)
  FacLds& L = *reinterpret_cast<FacLds*>(sol_dyn);
#pragma nounroll
  for (int p = 0; p < passes; ++p) {
    // the slot's addresses are rebuilt every pass from an index the compiler cannot see through,
    // so that nothing derived from them is hoisted out of the loop and kept live across the
    // derivative evaluation and the four phases
    int b = blockIdx.x, lane = threadIdx.x;
    asm volatile("" : "+s"(b), "+v"(lane));
    typedef const char __attribute__((address_space(4)))* KPtr;
    KPtr kp = (KPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(kp));
    const Cfg& c = *(const Cfg*)(const Cfg __attribute__((address_space(4)))*)kp;
    const Slot s = make_slot(c, ws, b);
    if ((int)s.sc[SC_PHASE] == PH_EMPTY) return;
    const long long t0 = clock64();
    eval_slot(c, s, sol_dyn, lane);
    const long long t1 = clock64();
    pass_phases<MIXED>(c, s, theta, warm, out, cnt, 1, L, sol_dyn, lane);
    if (lane == 0) s.sc[SC_CYC_EVAL] += (double)(t1 - t0);
    __syncthreads();
  }
}

// The four per-slot phases of one iteration in a single launch: each slot runs its phases back
// to back, instead of every phase waiting for the slowest slot of the previous one, and a pass
// costs two launches instead of five.  MIXED: the FP32 factor / FP64 refinement variant.
template <bool MIXED>
__global__ __launch_bounds__(64) void k_iter(Cfg c, double* ws, const double* theta, const double* warm, Outs out,
                                             Counters* cnt, int refill) {
  HIP_DYNAMIC_SHARED(double, sol_dyn)
  FacLds& L = *reinterpret_cast<FacLds*>(sol_dyn);
  const int lane = threadIdx.x;
  const Slot s = make_slot(c, ws, blockIdx.x);
  if ((int)s.sc[SC_PHASE] == PH_EMPTY) return;
  pass_phases<MIXED>(c, s, theta, warm, out, cnt, refill, L, sol_dyn, lane);
}

}  // namespace hipipm
