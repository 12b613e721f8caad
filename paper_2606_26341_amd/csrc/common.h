// Internal layout and configuration shared by the host driver and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hipipm {

constexpr int NX = 13;   // states per quadrotor
constexpr int NU = 4;    // rotor thrusts
constexpr int NZ = NX + NU;
constexpr int WAVE = 64;
constexpr int MAX_N = 64;
constexpr int MAX_OBS = 64;

// slot phases
enum : int { PH_INIT_Y = 0, PH_REGULAR = 1, PH_RESTO = 2, PH_FINISH = 3, PH_EMPTY = 4 };
// instance statuses (same values as the public HIPIPM_STATUS_*)
enum : int { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAX_ITER = 2, ST_RESTO_FAILED = 3, ST_INFEASIBLE = 4,
             ST_NUMERICAL = 5 };
// step flags handed from the factor kernel to the line-search kernel
enum : int { STEP_NONE = 0, STEP_READY = 1, STEP_ICFAIL = 2 };
// factorization request of the current pass (k_pre -> k_fac -> k_sol)
enum : int { W_NONE = 0, W_STEP = 1, W_LSQ = 2 };

// scalar block of a slot record (doubles)
enum : int {
  SC_MU = 0, SC_TAU, SC_DXL, SC_THMAX, SC_THMIN, SC_TINY, SC_NF,           // main sub-problem
  SC_RMU = 8, SC_RTAU, SC_RDXL, SC_RTHMAX, SC_RTHMIN, SC_RTINY, SC_RNF,  // restoration sub-problem
  SC_PHASE = 16, SC_STATUS, SC_ITER, SC_INST, SC_INITF, SC_THR,
  SC_STEP = 24, SC_AMAX, SC_THK, SC_PHK, SC_GPHI, SC_FK, SC_STEPMU,
  SC_ST_RESTO = 32, SC_ST_SOCT, SC_ST_SOCA, SC_ST_FACT, SC_ST_RENT, SC_ST_TINY, SC_ST_PASS,
  SC_LDX = 40, SC_LDC, SC_LALPHA, SC_LALPHAZ, SC_LSOC, SC_WORK, SC_FSTAT,
  SC_ST_SOLV, SC_ST_FFACT, SC_ST_FSOLV, SC_FPREC, SC_FORCE64, SC_ST_REF, SC_ST_FB, SC_DXLSAVE,
  SC_WARM, SC_ST_WSTART, SC_ST_WREJ, SC_ST_WRST,
  // warm-start gate: stage (1 cold reference running, 2 warm point waiting for the comparison),
  // E_mu0 of the cold start, the cold start's filter bounds
  SC_WSTAGE, SC_ECOLD, SC_CTHMAX, SC_CTHMIN,
  SC_ST_RTK,   // FP32 inertia verdicts taken again in FP64
  // watchdog (Table I row 3): consecutive shortened steps, active flag, unconditional steps taken,
  // the reference iteration's theta, phi_mu, grad phi^T d, alpha_max and mu; activations, reverts
  SC_WD_SHORT = 64, SC_WD_ACTIVE, SC_WD_ITER, SC_WD_THK, SC_WD_PHK, SC_WD_GPHI, SC_WD_AMAX, SC_WD_MU,
  SC_ST_WDS, SC_ST_WDR,
  // soft feasibility restoration (Table I row 5): active flag, soft steps taken, theta and phi_mu
  // of its starting point; soft steps, failures
  SC_SOFT, SC_SOFT_IT, SC_SOFT_THK, SC_SOFT_PHK, SC_ST_SOFTS, SC_ST_SOFTF,
  // adaptive barrier update (Table I row 7): free mode flag, references held, the last four E_0
  // references, the mu ceiling; switches to the monotone mode
  SC_MUFREE = 80, SC_NREFS, SC_REFS, SC_MUMAX = SC_REFS + 4, SC_ST_MUFB,
  // shader-clock cycles this slot spent in the derivatives (asynchronous-slot kernel) and in the
  // four phases of the fused kernels
  SC_CYC_EVAL, SC_CYC_PRE, SC_CYC_FAC, SC_CYC_SOL, SC_CYC_LS,
  SC_ST_NEST,   // nested restorations of the restoration phase
  SC_LEN = 96
};

// per-stage factor record (doubles)
//   L_R (4x4 lower), Y = L_R^{-1} Hbar^ux, P, M = Delta^{-1/2} C^{-1} Delta^{1/2} (only when
//   Delta > 0), Delta^1/2, 1 / diag(L_R), flag (Delta > 0)
enum : int { FR_LR = 0, FR_Y = 16, FR_P = 16 + NU * NX, FR_M = FR_P + NX * NX, FR_DH = FR_M + NX * NX,
             FR_RR = FR_DH + NX, FR_FLAG = FR_RR + NU, FR_LEN = ((FR_FLAG + 1 + 7) / 8) * 8 };
// per-stage condensed right-hand side (lambda 13, x 13, u 4) padded
constexpr int RB_LEN = 32;

struct Cfg {
  // problem
  int family, N, NI, n_theta, n, m, n_w, n_s, n_lower, n_upper;
  double dt, mass, jxx, jyy, jzz, arm, ctau, grav, qw, rw, uh, umax;
  // options
  double tol; int max_iter;
  double mu_init, kappa_eps, kappa_mu, theta_mu, tau_min, kappa1, kappa2, lam_max, s_max;
  double delta_min, delta_0, delta_max, delta_c_bar, kappa_c, kappa_minus, kappa_plus, kappa_plus_bar;
  double gamma_theta, gamma_phi, delta_sw, s_theta, s_phi, eta_phi, gamma_alpha;
  int max_soc; double kappa_soc, kappa_sigma, rho_resto, kappa_resto, bound_mult_reset;
  int fc;                                    // filter capacity: max_iter + 2 pairs (never reached)
  int prec, refine_max; double refine_tol;   // KKT factor precision (1: FP32 + FP64 refinement)
  double warm_mu0, warm_push; int warm_cap;  // warm start: barrier parameter, bound push, iteration cap
  int warm_gate;                             // keep a warm point only if E_mu0(warm) <= E_mu0(cold)
  int wd_trigger, wd_max;                    // watchdog: shortened steps that start it (0: off), its steps
  int soft_max; double soft_factor;          // soft restoration: steps before hard restoration (0: off),
                                             // required primal-dual error reduction
  int mu_strategy;                           // 0 monotone, 1 adaptive with monotone fallback
  int async_passes;
  int nested_resto, resto_ls_max;            // nested restoration on/off; restoration backtracking cap                          // > 0: asynchronous slots, passes per launch
  // slot record layout, offsets in doubles
  long long stride;
  int o_v, o_y, o_zlu, o_zuu, o_zls, o_th, o_sc, o_fm, o_fr;
  int o_yr, o_rzlu, o_rzuu, o_rzls, o_xr, o_p, o_nn, o_zp, o_zn;
  int o_F, o_G, o_HW, o_fac, o_rb;
  int o_dv, o_dy, o_dzlu, o_dzuu, o_dzls, o_dp, o_dn, o_dzp, o_dzn;
  int o_rv, o_rc, o_rp, o_rn, o_vt, o_ct, o_pt, o_nt, o_csoc, o_dvs, o_dys, o_dps, o_dns;
  int o_g, o_ref, o_sd;
  int o_qv, o_qc, o_qp, o_qn, o_ev, o_ec, o_ep, o_en;   // refinement residual and correction
  int o_wdv, o_wdy, o_wdzlu, o_wdzuu, o_wdzls;          // watchdog reference iterate
  int o_syt, o_szlu, o_szuu, o_szls;                    // soft-restoration trial multipliers
};

// caller-owned output arrays of a solve
struct Outs {
  double *x, *y, *zl, *zu, *obj, *kkt;
  int32_t *status, *iters;
};

// global counters (device): queue head, finished count, stats
constexpr int N_STATS = 29;
struct Counters {
  int32_t head, done, n_inst, pad;
  unsigned long long st[N_STATS];
};

}  // namespace hipipm
