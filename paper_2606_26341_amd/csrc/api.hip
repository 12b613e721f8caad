// Host side of libhipipm.so: the C ABI of include/hipipm.h, the slot-record layout and the
// iteration-level batching driver (Sec. V, Fig. 2): each pass launches the derivative,
// preparation, factor, solve and line-search kernels over all slots; finished slots are
// refilled from a device-side instance counter inside the preparation kernel, and the host
// polls the completion counter every `poll_every` passes.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hipipm.h"
#include "common.h"

namespace hipipm {
void launch_eval(const Cfg& c, double* ws, int slots, hipStream_t st);
void launch_pre(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                Counters* cnt, int refill, hipStream_t st);
void launch_fac(const Cfg& c, double* ws, int slots, hipStream_t st);
void launch_sol(const Cfg& c, double* ws, int slots, const double* warm, hipStream_t st);
void launch_ls(const Cfg& c, double* ws, int slots, hipStream_t st);
void launch_iter(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                 Counters* cnt, int refill, hipStream_t st);
void launch_run_fp64(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                     Counters* cnt, int passes, hipStream_t st);
void launch_run_mixed(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                      Counters* cnt, int passes, hipStream_t st);
int occupancy_run_fp64(const Cfg& c);
int occupancy_run_mixed(const Cfg& c);
void launch_setup(const Cfg& c, double* ws, int slots, int n_active, const double* theta, const double* warm,
                  hipStream_t st);
void launch_stage_derivs(const Cfg& c, int count, const double* x, const double* u, const double* lam, double* F,
                         double* G, double* H, hipStream_t st);
void launch_kkt_test(const Cfg& c, double* ws, int count, double dxp, double dcp, const double* rhs, double* sol,
                     int* inertia_ok, hipStream_t st);
void launch_prepare(const Cfg& c, double* ws, int count, hipStream_t st);
void launch_counters_init(Counters* cnt, int head, int n_inst, hipStream_t st);
int sd_len_host(int NI);
}  // namespace hipipm

using namespace hipipm;

// timed kernels: eval, pre, factor, solve, linesearch (one launch each per pass), fused pass
// kernel, setup, asynchronous-slot kernel
static constexpr int NKT = 8;
static constexpr int NPK = 5;
static constexpr int KT_FUSED = 5;
static constexpr int KT_SETUP = 6;
static constexpr int KT_ASYNC = 7;

struct hipipm_ctx {
  hipipm_problem_desc desc;
  hipipm_options opts;
  Cfg cfg;
  int slots;
  int device;
  double* ws;
  size_t ws_bound;
  size_t need;
  size_t cnt_off;
  std::string err;
  hipipm_stats stats;
  double t_ms[NKT];
  long long t_n[NKT];
  // pinned copies of the device counter block, one per chunk of passes in flight, and the
  // events that mark each copy complete (allocated at the first solve)
  Counters* hcnt = nullptr;
  hipEvent_t cev[2] = {nullptr, nullptr};
};

static int fail(hipipm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ctx, HIPIPM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static int rup(int a, int b) { return (a + b - 1) / b * b; }

static void layout(Cfg& c) {
  int o = 0;
  auto take = [&](int len) {
    int r = o;
    o += rup(len > 0 ? len : 1, 8);
    return r;
  };
  const int n = c.n, m = c.m, N = c.N, NI = c.NI;
  c.o_sc = take(SC_LEN);
  c.o_v = take(n); c.o_y = take(m); c.o_zlu = take(N * NU); c.o_zuu = take(N * NU); c.o_zls = take(N * NI);
  c.o_th = take(c.n_theta); c.o_fm = take(2 * c.fc); c.o_fr = take(2 * c.fc);
  c.o_yr = take(m); c.o_rzlu = take(N * NU); c.o_rzuu = take(N * NU); c.o_rzls = take(N * NI);
  c.o_xr = take(n); c.o_p = take(m); c.o_nn = take(m); c.o_zp = take(m); c.o_zn = take(m);
  c.o_F = take(N * NX); c.o_G = take(N * NX * NZ); c.o_HW = take(N * NZ * NZ);
  c.o_fac = take((N + 1) * FR_LEN); c.o_rb = take((N + 1) * RB_LEN);
  c.o_dv = take(n); c.o_dy = take(m); c.o_dzlu = take(N * NU); c.o_dzuu = take(N * NU); c.o_dzls = take(N * NI);
  c.o_dp = take(m); c.o_dn = take(m); c.o_dzp = take(m); c.o_dzn = take(m);
  c.o_rv = take(n); c.o_rc = take(m); c.o_rp = take(m); c.o_rn = take(m);
  c.o_vt = take(n); c.o_ct = take(m); c.o_pt = take(m); c.o_nt = take(m); c.o_csoc = take(m);
  c.o_dvs = take(n); c.o_dys = take(m); c.o_dps = take(m); c.o_dns = take(m); c.o_g = take(n);
  c.o_ref = take((N + 1) * NX);
  c.o_sd = take((N + 1) * sd_len_host(NI));
  c.o_qv = take(n); c.o_qc = take(m); c.o_qp = take(m); c.o_qn = take(m);
  c.o_ev = take(n); c.o_ec = take(m); c.o_ep = take(m); c.o_en = take(m);
  c.o_wdv = take(n); c.o_wdy = take(m); c.o_wdzlu = take(N * NU); c.o_wdzuu = take(N * NU); c.o_wdzls = take(N * NI);
  c.o_syt = take(m); c.o_szlu = take(N * NU); c.o_szuu = take(N * NU); c.o_szls = take(N * NI);
  c.stride = rup(o, 64);
}

// ------------------------------------------------------------------ allocation-free solve
// The workspace of hipipm_solve_noalloc: one array per GPU, part of the library's code object
// (each GPU the library runs on holds it until the process ends).  In host code `scratch` is only
// a stand-in for the symbol; its device address on each GPU comes from hipGetSymbolAddress, taken
// once per device with that device current (at hipipm_create) and kept in g_scratch.
static constexpr size_t STATIC_WS_BYTES = (size_t)HIPIPM_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];
static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[MAX_DEVICES];

// device address of the static workspace on the current device `dev` (set up on first use)
static int scratch_setup(hipipm_ctx* c, int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(c, HIPIPM_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, HIPIPM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  if (out) *out = g_scratch[dev];
  return HIPIPM_OK;
}

extern "C" {

int hipipm_default_options(hipipm_options* o) {
  if (!o) return HIPIPM_ERR_INVALID_ARG;
  o->tol = 1e-8; o->max_iter = 1000; o->mu_init = 0.1; o->kappa_eps = 10.0; o->kappa_mu = 0.2;
  o->theta_mu = 1.5; o->tau_min = 0.99; o->kappa1 = 1e-2; o->kappa2 = 1e-2; o->lam_max = 1e3; o->s_max = 100.0;
  o->delta_min = 1e-20; o->delta_0 = 1e-4; o->delta_max = 1e40; o->delta_c_bar = 1e-8; o->kappa_c = 0.25;
  o->kappa_minus = 1.0 / 3.0; o->kappa_plus = 8.0; o->kappa_plus_bar = 100.0;
  o->gamma_theta = 1e-5; o->gamma_phi = 1e-8; o->delta_sw = 1.0; o->s_theta = 1.1; o->s_phi = 2.3;
  o->eta_phi = 1e-8; o->gamma_alpha = 0.05; o->max_soc = 4; o->kappa_soc = 0.99; o->kappa_sigma = 1e10;
  o->rho_resto = 1000.0; o->kappa_resto = 0.9; o->bound_mult_reset = 1e3;
  o->poll_every = 4; o->timing = 0; o->fuse_below = 1 << 30;
  o->precision = 0; o->refine_max = 3; o->refine_tol = 1e-10;
  o->warm_mu0 = 1e-3; o->warm_push = 1e-3; o->warm_iter_cap = 0; o->warm_gate = 1;
  o->watchdog_trigger = 0; o->watchdog_max = 3;
  o->soft_resto_max = 0; o->soft_resto_factor = 0.9999;
  o->mu_strategy = 0; o->async_passes = 0;
  o->nested_resto = 1; o->resto_ls_max = 60;
  return HIPIPM_OK;
}

int hipipm_create(const hipipm_problem_desc* d, const hipipm_options* o, int32_t slots, hipipm_ctx** out) {
  if (!d || !o || !out || slots <= 0) return HIPIPM_ERR_INVALID_ARG;
  *out = nullptr;
  if (d->family != HIPIPM_FAMILY_QUAD_OBS && d->family != HIPIPM_FAMILY_QUAD_TRACK &&
      d->family != HIPIPM_FAMILY_QUAD_TRACK_MOVING)
    return HIPIPM_ERR_UNSUPPORTED;
  if (d->n_agents != 1) return HIPIPM_ERR_UNSUPPORTED;
  if (d->N < 1 || d->N > MAX_N || d->n_obs < 0 || d->n_obs > MAX_OBS) return HIPIPM_ERR_INVALID_ARG;
  if (!(d->dt > 0) || !(d->mass > 0) || !(d->jxx > 0) || !(d->jyy > 0) || !(d->jzz > 0)) return HIPIPM_ERR_INVALID_ARG;
  if (o->max_iter < 0 || o->max_iter > (1 << 24) || o->poll_every < 1 || !(o->tol > 0) ||
      o->fuse_below < 0 || o->precision < 0 || o->precision > 1 || o->refine_max < 0 || !(o->refine_tol > 0) ||
      !(o->warm_mu0 > 0) || !(o->warm_push > 0) || o->warm_iter_cap < 0 || o->warm_gate < 0 || o->warm_gate > 1 ||
      o->watchdog_trigger < 0 || o->watchdog_max < 1 || o->soft_resto_max < 0 ||
      !(o->soft_resto_factor > 0 && o->soft_resto_factor <= 1) || o->mu_strategy < 0 || o->mu_strategy > 1 ||
      o->async_passes < 0 || o->nested_resto < 0 || o->nested_resto > 1 || o->resto_ls_max < 0)
    return HIPIPM_ERR_INVALID_ARG;
  hipipm_ctx* c = new hipipm_ctx();
  c->desc = *d;
  c->opts = *o;
  c->slots = slots;
  c->ws = nullptr;
  c->ws_bound = 0;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return HIPIPM_ERR_HIP; }
  // device address of the allocation-free solve's static workspace on this device
  if (scratch_setup(c, c->device, nullptr) != HIPIPM_OK) { delete c; return HIPIPM_ERR_HIP; }
  Cfg& g = c->cfg;
  memset(&g, 0, sizeof(g));
  g.family = d->family; g.N = d->N; g.NI = d->n_obs;
  g.n_theta = d->family == HIPIPM_FAMILY_QUAD_OBS ? 16 + 4 * d->n_obs
              : d->family == HIPIPM_FAMILY_QUAD_TRACK ? 15 + 4 * d->n_obs
                                                      : 15 + 7 * d->n_obs;
  g.n_w = (d->N + 1) * NX + d->N * NU;
  g.n_s = d->N * d->n_obs;
  g.n = g.n_w + g.n_s;
  g.m = (d->N + 1) * NX + g.n_s;
  g.n_lower = d->N * NU + g.n_s;
  g.n_upper = d->N * NU;
  g.dt = d->dt; g.mass = d->mass; g.jxx = d->jxx; g.jyy = d->jyy; g.jzz = d->jzz; g.arm = d->arm;
  g.ctau = d->ctau; g.grav = d->grav; g.qw = d->q_weight; g.rw = d->r_weight;
  g.uh = d->mass * d->grav / 4.0;
  g.umax = 2.0 * g.uh;
  g.tol = o->tol; g.max_iter = o->max_iter; g.mu_init = o->mu_init; g.kappa_eps = o->kappa_eps;
  g.kappa_mu = o->kappa_mu; g.theta_mu = o->theta_mu; g.tau_min = o->tau_min; g.kappa1 = o->kappa1;
  g.kappa2 = o->kappa2; g.lam_max = o->lam_max; g.s_max = o->s_max; g.delta_min = o->delta_min;
  g.delta_0 = o->delta_0; g.delta_max = o->delta_max; g.delta_c_bar = o->delta_c_bar; g.kappa_c = o->kappa_c;
  g.kappa_minus = o->kappa_minus; g.kappa_plus = o->kappa_plus; g.kappa_plus_bar = o->kappa_plus_bar;
  g.gamma_theta = o->gamma_theta; g.gamma_phi = o->gamma_phi; g.delta_sw = o->delta_sw; g.s_theta = o->s_theta;
  g.s_phi = o->s_phi; g.eta_phi = o->eta_phi; g.gamma_alpha = o->gamma_alpha; g.max_soc = o->max_soc;
  g.kappa_soc = o->kappa_soc; g.kappa_sigma = o->kappa_sigma; g.rho_resto = o->rho_resto;
  g.kappa_resto = o->kappa_resto; g.bound_mult_reset = o->bound_mult_reset; g.fc = o->max_iter + 2;
  g.prec = o->precision; g.refine_max = o->refine_max; g.refine_tol = o->refine_tol;
  g.warm_mu0 = o->warm_mu0; g.warm_push = o->warm_push; g.warm_cap = o->warm_iter_cap; g.warm_gate = o->warm_gate;
  g.wd_trigger = o->watchdog_trigger; g.wd_max = o->watchdog_max;
  g.soft_max = o->soft_resto_max; g.soft_factor = o->soft_resto_factor;
  g.mu_strategy = o->mu_strategy; g.async_passes = o->async_passes;
  g.nested_resto = o->nested_resto; g.resto_ls_max = o->resto_ls_max;
  layout(g);
  size_t rec = (size_t)g.stride * sizeof(double) * (size_t)slots;
  c->cnt_off = (rec + 255) / 256 * 256;
  c->need = c->cnt_off + (sizeof(Counters) + 255) / 256 * 256;
  memset(&c->stats, 0, sizeof(c->stats));
  memset(c->t_ms, 0, sizeof(c->t_ms));
  memset(c->t_n, 0, sizeof(c->t_n));
  *out = c;
  return HIPIPM_OK;
}

int hipipm_get_dims(const hipipm_ctx* c, hipipm_dims* out) {
  if (!c || !out) return HIPIPM_ERR_INVALID_ARG;
  out->n = c->cfg.n; out->m = c->cfg.m; out->n_w = c->cfg.n_w; out->n_s = c->cfg.n_s;
  out->n_theta = c->cfg.n_theta; out->n_lower = c->cfg.n_lower; out->n_upper = c->cfg.n_upper;
  out->N = c->cfg.N; out->nx = NX; out->nu = NU; out->n_ineq = c->cfg.NI;
  return HIPIPM_OK;
}

int hipipm_resident_slots(const hipipm_ctx* c, int32_t* slots) {
  if (!c || !slots) return HIPIPM_ERR_INVALID_ARG;
  const int per_cu = c->opts.precision == 1 ? occupancy_run_mixed(c->cfg) : occupancy_run_fp64(c->cfg);
  hipDeviceProp_t p;
  if (per_cu < 0 || hipGetDeviceProperties(&p, c->device) != hipSuccess) return HIPIPM_ERR_HIP;
  *slots = per_cu * p.multiProcessorCount;
  return HIPIPM_OK;
}

int hipipm_workspace_bytes(const hipipm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return HIPIPM_ERR_INVALID_ARG;
  *bytes = c->need;
  return HIPIPM_OK;
}

int hipipm_bind_workspace(hipipm_ctx* c, void* p, size_t bytes) {
  if (!c) return HIPIPM_ERR_INVALID_ARG;
  if (!p || bytes < c->need) return fail(c, HIPIPM_ERR_WORKSPACE, "workspace missing or smaller than hipipm_workspace_bytes()");
  if (((uintptr_t)p) % 256 != 0) return fail(c, HIPIPM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  c->ws = (double*)p;
  c->ws_bound = bytes;
  return HIPIPM_OK;
}

static Counters* counters(hipipm_ctx* c) { return (Counters*)((char*)c->ws + c->cnt_off); }

// the device counter block of a finished solve into the context's totals
static void add_stats(hipipm_ctx* c, const Counters& h, long long passes) {
  c->stats.iterations += (int64_t)h.st[0];
  c->stats.resto_iterations += (int64_t)h.st[1];
  c->stats.soc_tried += (int64_t)h.st[2];
  c->stats.soc_accepted += (int64_t)h.st[3];
  c->stats.factorizations += (int64_t)h.st[4];
  c->stats.resto_entries += (int64_t)h.st[5];
  c->stats.tiny_steps += (int64_t)h.st[6];
  c->stats.passes += passes;
  c->stats.instances_done += (int64_t)h.st[8];
  c->stats.solves += (int64_t)h.st[9];
  c->stats.fused_factorizations += (int64_t)h.st[10];
  c->stats.fused_solves += (int64_t)h.st[11];
  c->stats.refine_sweeps += (int64_t)h.st[12];
  c->stats.fp64_fallbacks += (int64_t)h.st[13];
  c->stats.warm_started += (int64_t)h.st[14];
  c->stats.warm_rejected += (int64_t)h.st[15];
  c->stats.warm_restarts += (int64_t)h.st[16];
  c->stats.fp32_retakes += (int64_t)h.st[17];
  c->stats.watchdog_starts += (int64_t)h.st[18];
  c->stats.watchdog_reverts += (int64_t)h.st[19];
  c->stats.soft_resto_steps += (int64_t)h.st[20];
  c->stats.soft_resto_fails += (int64_t)h.st[21];
  c->stats.mu_fallbacks += (int64_t)h.st[22];
  c->stats.nested_restorations += (int64_t)h.st[28];
  c->stats.cycles_eval += (int64_t)h.st[23];
  c->stats.cycles_pre += (int64_t)h.st[24];
  c->stats.cycles_factor += (int64_t)h.st[25];
  c->stats.cycles_solve += (int64_t)h.st[26];
  c->stats.cycles_linesearch += (int64_t)h.st[27];
}

int hipipm_solve(hipipm_ctx* c, int32_t n_inst, const double* theta, const double* warm, double* x_out,
                 double* y_out, double* zl_out, double* zu_out, double* obj_out, double* kkt_out,
                 int32_t* status_out, int32_t* iters_out, void* stream) {
  if (!c) return HIPIPM_ERR_INVALID_ARG;
  if (n_inst < 0) return fail(c, HIPIPM_ERR_INVALID_ARG, "n_inst < 0");
  if (n_inst == 0) return HIPIPM_OK;
  if (!theta) return fail(c, HIPIPM_ERR_INVALID_ARG, "theta is NULL");
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int active = n_inst < c->slots ? n_inst : c->slots;
  Counters h;
  memset(&h, 0, sizeof(h));
  h.head = active;
  h.done = 0;
  h.n_inst = n_inst;
  Counters* dcnt = counters(c);
  HIPCHK(c, hipMemcpyAsync(dcnt, &h, sizeof(h), hipMemcpyHostToDevice, st));
  Outs out{x_out, y_out, zl_out, zu_out, obj_out, kkt_out, status_out, iters_out};
  if (!c->hcnt) {
    void* p = nullptr;
    HIPCHK(c, hipHostMalloc(&p, 2 * sizeof(Counters), hipHostMallocDefault));
    c->hcnt = (Counters*)p;
    for (auto& e : c->cev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  const int poll = c->opts.poll_every;
  const bool timing = c->opts.timing != 0;
  // timing events: setup (2), then one set of (NPK + 1) per pass for each of the two chunks in flight
  const int per_chunk = (NPK + 1) * poll;
  std::vector<hipEvent_t> ev;
  if (timing) {
    ev.resize(2 + 2 * per_chunk);
    for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(ev[0], st));
  }
  launch_setup(c->cfg, c->ws, active, active, theta, warm, st);
  if (timing) {
    HIPCHK(c, hipEventRecord(ev[1], st));
    HIPCHK(c, hipEventSynchronize(ev[1]));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    c->t_ms[KT_SETUP] += ms;
    c->t_n[KT_SETUP] += 1;
  }
  HIPCHK(c, hipGetLastError());
  // every pass advances each running slot by at most one pipeline step; bound the loop
  const long long max_passes = ((long long)c->opts.max_iter + 8) * 3 * ((n_inst + active - 1) / active) + 64;
  long long passes = 0;
  bool fused_of[2] = {false, false}, async_of[2] = {false, false};
  const int apasses = c->opts.async_passes;
  // Passes go out in chunks of `poll`; each chunk ends with an asynchronous copy of the counter
  // block into pinned memory.  The next chunk is queued before the host waits for the previous
  // chunk's copy, so the GPU never idles on the poll.  Passes queued after the last instance
  // finished find every slot empty and return at once.
  auto launch_chunk = [&](int par, bool fused) -> int {
    async_of[par] = apasses > 0;
    if (apasses > 0) {
      // asynchronous slots: one launch in which every slot runs up to apasses whole passes
      hipEvent_t* e = timing ? &ev[2 + par * per_chunk] : nullptr;
      if (timing) HIPCHK(c, hipEventRecord(e[0], st));
      if (c->cfg.prec == 1) launch_run_mixed(c->cfg, c->ws, active, theta, warm, out, dcnt, apasses, st);
      else launch_run_fp64(c->cfg, c->ws, active, theta, warm, out, dcnt, apasses, st);
      if (timing) HIPCHK(c, hipEventRecord(e[1], st));
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(&c->hcnt[par], dcnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipEventRecord(c->cev[par], st));
      fused_of[par] = true;
      passes += apasses;
      return HIPIPM_OK;
    }
    for (int p = 0; p < poll; ++p) {
      hipEvent_t* e = timing ? &ev[2 + par * per_chunk + (NPK + 1) * p] : nullptr;
      if (timing) HIPCHK(c, hipEventRecord(e[0], st));
      launch_eval(c->cfg, c->ws, active, st);
      if (timing) HIPCHK(c, hipEventRecord(e[1], st));
      if (fused) {
        launch_iter(c->cfg, c->ws, active, theta, warm, out, dcnt, 1, st);
        if (timing) HIPCHK(c, hipEventRecord(e[2], st));
      } else {
        launch_pre(c->cfg, c->ws, active, theta, warm, out, dcnt, 1, st);
        if (timing) HIPCHK(c, hipEventRecord(e[2], st));
        launch_fac(c->cfg, c->ws, active, st);
        if (timing) HIPCHK(c, hipEventRecord(e[3], st));
        launch_sol(c->cfg, c->ws, active, warm, st);
        if (timing) HIPCHK(c, hipEventRecord(e[4], st));
        launch_ls(c->cfg, c->ws, active, st);
        if (timing) HIPCHK(c, hipEventRecord(e[5], st));
      }
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&c->hcnt[par], dcnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipEventRecord(c->cev[par], st));
    fused_of[par] = fused;
    passes += poll;
    return HIPIPM_OK;
  };
  // wait for chunk `par`: its counters into h, its kernel times into the buckets
  auto finish_chunk = [&](int par) -> int {
    HIPCHK(c, hipEventSynchronize(c->cev[par]));
    h = c->hcnt[par];
    if (timing && async_of[par]) {
      const hipEvent_t* e = &ev[2 + par * per_chunk];
      float ms = 0;
      HIPCHK(c, hipEventElapsedTime(&ms, e[0], e[1]));
      c->t_ms[KT_ASYNC] += ms;
      c->t_n[KT_ASYNC] += 1;
    } else if (timing) {
      for (int p = 0; p < poll; ++p) {
        const hipEvent_t* e = &ev[2 + par * per_chunk + (NPK + 1) * p];
        const int nk = fused_of[par] ? 2 : NPK;
        for (int q = 0; q < nk; ++q) {
          float ms = 0;
          HIPCHK(c, hipEventElapsedTime(&ms, e[q], e[q + 1]));
          const int bucket = (fused_of[par] && q == 1) ? KT_FUSED : q;
          c->t_ms[bucket] += ms;
          c->t_n[bucket] += 1;
        }
      }
    }
    return HIPIPM_OK;
  };
  // few unfinished instances left: fused pass kernel (every launch still covers all slots); the
  // count seen is one chunk old
  auto use_fused = [&]() {
    return c->opts.precision == 1 || (c->opts.fuse_below > 0 && n_inst - h.done <= c->opts.fuse_below);
  };
  auto bail = [&](int rc) {
    (void)hipStreamSynchronize(st);
    if (timing) for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
  };
  int rc = launch_chunk(0, use_fused());
  if (rc) return bail(rc);
  for (int cur = 0;; cur ^= 1) {
    const int nxt = cur ^ 1;
    const bool more = passes <= max_passes;
    if (more && (rc = launch_chunk(nxt, use_fused()))) return bail(rc);
    if ((rc = finish_chunk(cur))) return bail(rc);
    if (h.done >= n_inst) {
      if (more && (rc = finish_chunk(nxt))) return bail(rc);
      break;
    }
    if (!more) return bail(fail(c, HIPIPM_ERR_HIP, "solve did not finish within the pass bound"));
  }
  if (timing) for (auto& e : ev) (void)hipEventDestroy(e);
  add_stats(c, h, passes);
  return HIPIPM_OK;
}

int hipipm_solve_noalloc(hipipm_ctx* c, int32_t n_inst, const double* theta, const double* warm, double* x_out,
                         double* y_out, double* zl_out, double* zu_out, double* obj_out, double* kkt_out,
                         int32_t* status_out, int32_t* iters_out, void* stream) {
  if (!c) return HIPIPM_ERR_INVALID_ARG;
  if (n_inst < 0) return fail(c, HIPIPM_ERR_INVALID_ARG, "n_inst < 0");
  if (n_inst == 0) return HIPIPM_OK;
  if (!theta) return fail(c, HIPIPM_ERR_INVALID_ARG, "theta is NULL");
  if (c->need > STATIC_WS_BYTES)
    return fail(c, HIPIPM_ERR_WORKSPACE,
                "hipipm_solve_noalloc: the context needs " + std::to_string(c->need) +
                    " workspace bytes, more than the static workspace of " + std::to_string(STATIC_WS_BYTES) +
                    " bytes; create the context with fewer slots");
  HIPCHK(c, hipSetDevice(c->device));
  void* base = nullptr;
  if (int rc = scratch_setup(c, c->device, &base)) return rc;
  double* ws = (double*)base;
  Counters* dcnt = (Counters*)((char*)base + c->cnt_off);
  hipStream_t st = (hipStream_t)stream;
  const int active = n_inst < c->slots ? n_inst : c->slots;
  // the counter block is the only part of the workspace that must start from known values (every
  // slot record is written by the setup kernel before it is read); a kernel clears it
  launch_counters_init(dcnt, active, n_inst, st);
  launch_setup(c->cfg, ws, active, active, theta, warm, st);
  HIPCHK(c, hipGetLastError());
  Outs out{x_out, y_out, zl_out, zu_out, obj_out, kkt_out, status_out, iters_out};
  const long long max_passes = ((long long)c->opts.max_iter + 8) * 3 * ((n_inst + active - 1) / active) + 64;
  const int poll = c->opts.poll_every;
  long long passes = 0;
  Counters h;
  memset(&h, 0, sizeof(h));
  // chunks of `poll` passes, each followed by a copy of the counter block into host memory (the
  // stack, no pinned buffer) and a wait on the stream
  for (;;) {
    const bool fused = c->opts.precision == 1 || (c->opts.fuse_below > 0 && n_inst - h.done <= c->opts.fuse_below);
    for (int p = 0; p < poll; ++p) {
      launch_eval(c->cfg, ws, active, st);
      if (fused) {
        launch_iter(c->cfg, ws, active, theta, warm, out, dcnt, 1, st);
      } else {
        launch_pre(c->cfg, ws, active, theta, warm, out, dcnt, 1, st);
        launch_fac(c->cfg, ws, active, st);
        launch_sol(c->cfg, ws, active, warm, st);
        launch_ls(c->cfg, ws, active, st);
      }
    }
    passes += poll;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&h, dcnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (h.done >= n_inst) break;
    if (passes > max_passes) return fail(c, HIPIPM_ERR_HIP, "solve did not finish within the pass bound");
  }
  add_stats(c, h, passes);
  return HIPIPM_OK;
}

int hipipm_stats_get(const hipipm_ctx* c, hipipm_stats* out) {
  if (!c || !out) return HIPIPM_ERR_INVALID_ARG;
  *out = c->stats;
  return HIPIPM_OK;
}

int hipipm_reset_stats(hipipm_ctx* c) {
  if (!c) return HIPIPM_ERR_INVALID_ARG;
  memset(&c->stats, 0, sizeof(c->stats));
  memset(c->t_ms, 0, sizeof(c->t_ms));
  memset(c->t_n, 0, sizeof(c->t_n));
  return HIPIPM_OK;
}

int hipipm_kernel_times(const hipipm_ctx* c, int32_t* n_kernels, double* total_ms, int64_t* launches) {
  if (!c || !n_kernels) return HIPIPM_ERR_INVALID_ARG;
  int n = *n_kernels < NKT ? *n_kernels : NKT;
  for (int i = 0; i < n; ++i) {
    if (total_ms) total_ms[i] = c->t_ms[i];
    if (launches) launches[i] = c->t_n[i];
  }
  *n_kernels = NKT;
  return HIPIPM_OK;
}

// ------------------------------------------------------------------ state replay hooks
static int state_len_of(const Cfg& g) {
  int n = g.n, m = g.m;
  int sub_main = 8 + 3 * n + m + 2 * g.fc;
  int sub_resto = 8 + 3 * (n + 2 * m) + m + 2 * g.fc;
  int watchdog = 8 + 3 * n + m, soft = 4, adaptive = 8;
  return 16 + sub_main + sub_resto + 2 * n + watchdog + soft + adaptive;
}

int hipipm_state_len(const hipipm_ctx* c, int32_t* len) {
  if (!c || !len) return HIPIPM_ERR_INVALID_ARG;
  *len = state_len_of(c->cfg);
  return HIPIPM_OK;
}

// v-index -> (bounded lower?, compact index) helpers on the host
static void zfull_from(const Cfg& g, const double* rec, int o_lu, int o_uu, int o_ls, double* zl, double* zu) {
  for (int i = 0; i < g.n; ++i) { zl[i] = 0.0; zu[i] = 0.0; }
  for (int k = 0; k < g.N; ++k)
    for (int i = 0; i < NU; ++i) {
      zl[k * NZ + NX + i] = rec[o_lu + k * NU + i];
      zu[k * NZ + NX + i] = rec[o_uu + k * NU + i];
    }
  for (int q = 0; q < g.n_s; ++q) zl[g.n_w + q] = rec[o_ls + q];
}
static void zfull_to(const Cfg& g, double* rec, int o_lu, int o_uu, int o_ls, const double* zl, const double* zu) {
  for (int k = 0; k < g.N; ++k)
    for (int i = 0; i < NU; ++i) {
      rec[o_lu + k * NU + i] = zl[k * NZ + NX + i];
      rec[o_uu + k * NU + i] = zu[k * NZ + NX + i];
    }
  for (int q = 0; q < g.n_s; ++q) rec[o_ls + q] = zl[g.n_w + q];
}

int hipipm_state_export(hipipm_ctx* c, int32_t count, double* out, void* stream) {
  if (!c || !out || count < 0 || count > c->slots) return HIPIPM_ERR_INVALID_ARG;
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  const Cfg& g = c->cfg;
  const int n = g.n, m = g.m, L = state_len_of(g), NR = n + 2 * m;
  std::vector<double> rec((size_t)g.stride);
  for (int s = 0; s < count; ++s) {
    HIPCHK(c, hipMemcpyAsync(rec.data(), c->ws + (size_t)s * g.stride, g.stride * sizeof(double),
                             hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    double* o = out + (size_t)s * L;
    memset(o, 0, L * sizeof(double));
    const double* sc = rec.data() + g.o_sc;
    int ph = (int)sc[SC_PHASE];
    o[0] = ph >= PH_FINISH ? 3 : ph;
    o[1] = sc[SC_ITER]; o[2] = sc[SC_STATUS]; o[3] = sc[SC_INITF]; o[4] = sc[SC_THR];
    o[5] = sc[SC_WARM]; o[6] = sc[SC_WSTAGE];
    const bool resto = ph == PH_RESTO;
    double* p = o + 16;
    // main
    p[0] = sc[SC_MU]; p[1] = sc[SC_TAU]; p[2] = sc[SC_DXL]; p[3] = sc[SC_THMAX]; p[4] = sc[SC_THMIN];
    p[5] = sc[SC_TINY]; p[6] = sc[SC_NF];
    p += 8;
    memcpy(p, rec.data() + (resto ? g.o_xr : g.o_v), n * sizeof(double)); p += n;
    memcpy(p, rec.data() + g.o_y, m * sizeof(double)); p += m;
    zfull_from(g, rec.data(), g.o_zlu, g.o_zuu, g.o_zls, p, p + n); p += 2 * n;
    for (int i = 0; i < g.fc; ++i) { p[i] = rec[g.o_fm + i]; p[g.fc + i] = rec[g.o_fm + g.fc + i]; }
    for (int i = (int)sc[SC_NF]; i < g.fc; ++i) { p[i] = 0.0; p[g.fc + i] = 0.0; }
    p += 2 * g.fc;
    // restoration
    p[0] = sc[SC_RMU]; p[1] = sc[SC_RTAU]; p[2] = sc[SC_RDXL]; p[3] = sc[SC_RTHMAX]; p[4] = sc[SC_RTHMIN];
    p[5] = sc[SC_RTINY]; p[6] = sc[SC_RNF];
    p += 8;
    if (resto) {
      memcpy(p, rec.data() + g.o_v, n * sizeof(double));
      memcpy(p + n, rec.data() + g.o_p, m * sizeof(double));
      memcpy(p + n + m, rec.data() + g.o_nn, m * sizeof(double));
    }
    p += NR;
    memcpy(p, rec.data() + g.o_yr, m * sizeof(double)); p += m;
    {
      std::vector<double> zl(n), zu(n);
      zfull_from(g, rec.data(), g.o_rzlu, g.o_rzuu, g.o_rzls, zl.data(), zu.data());
      memcpy(p, zl.data(), n * sizeof(double));
      memcpy(p + n, rec.data() + g.o_zp, m * sizeof(double));
      memcpy(p + n + m, rec.data() + g.o_zn, m * sizeof(double));
      memcpy(p + NR, zu.data(), n * sizeof(double));
    }
    p += 2 * NR;
    for (int i = 0; i < g.fc; ++i) { p[i] = rec[g.o_fr + i]; p[g.fc + i] = rec[g.o_fr + g.fc + i]; }
    for (int i = (int)sc[SC_RNF]; i < g.fc; ++i) { p[i] = 0.0; p[g.fc + i] = 0.0; }
    p += 2 * g.fc;
    memcpy(p, rec.data() + g.o_xr, n * sizeof(double)); p += n;
    for (int i = 0; i < n; ++i) {
      double d = std::fmin(1.0, 1.0 / std::fabs(rec[g.o_xr + i]));
      p[i] = d * d;
    }
    p += n;
    // watchdog block
    for (int q = 0; q < 8; ++q) p[q] = sc[SC_WD_SHORT + q];
    p += 8;
    memcpy(p, rec.data() + g.o_wdv, n * sizeof(double)); p += n;
    memcpy(p, rec.data() + g.o_wdy, m * sizeof(double)); p += m;
    zfull_from(g, rec.data(), g.o_wdzlu, g.o_wdzuu, g.o_wdzls, p, p + n);
    p += 2 * n;
    for (int q = 0; q < 4; ++q) p[q] = sc[SC_SOFT + q];
    p += 4;
    for (int q = 0; q < 7; ++q) p[q] = sc[SC_MUFREE + q];   // free flag, references held, refs[4], mu_max
  }
  return HIPIPM_OK;
}

int hipipm_state_import(hipipm_ctx* c, int32_t count, const double* in, const double* theta_dev, void* stream) {
  if (!c || !in || !theta_dev || count < 0 || count > c->slots) return HIPIPM_ERR_INVALID_ARG;
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  const Cfg& g = c->cfg;
  const int n = g.n, m = g.m, L = state_len_of(g), NR = n + 2 * m;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> rec((size_t)g.stride), th((size_t)count * g.n_theta);
  HIPCHK(c, hipMemcpyAsync(th.data(), theta_dev, th.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  for (int s = 0; s < count; ++s) {
    std::fill(rec.begin(), rec.end(), 0.0);
    const double* o = in + (size_t)s * L;
    double* sc = rec.data() + g.o_sc;
    int ph = (int)o[0];
    sc[SC_PHASE] = ph == 3 ? PH_FINISH : ph;
    sc[SC_ITER] = o[1]; sc[SC_STATUS] = o[2]; sc[SC_INITF] = o[3]; sc[SC_THR] = o[4];
    sc[SC_WARM] = o[5]; sc[SC_WSTAGE] = o[6];
    sc[SC_INST] = s;
    const bool resto = ph == PH_RESTO;
    const double* p = o + 16;
    sc[SC_MU] = p[0]; sc[SC_TAU] = p[1]; sc[SC_DXL] = p[2]; sc[SC_THMAX] = p[3]; sc[SC_THMIN] = p[4];
    sc[SC_TINY] = p[5]; sc[SC_NF] = p[6];
    p += 8;
    const double* main_x = p;
    p += n;
    memcpy(rec.data() + g.o_y, p, m * sizeof(double)); p += m;
    zfull_to(g, rec.data(), g.o_zlu, g.o_zuu, g.o_zls, p, p + n); p += 2 * n;
    for (int i = 0; i < 2 * g.fc; ++i) rec[g.o_fm + i] = p[i];
    p += 2 * g.fc;
    sc[SC_RMU] = p[0]; sc[SC_RTAU] = p[1]; sc[SC_RDXL] = p[2]; sc[SC_RTHMAX] = p[3]; sc[SC_RTHMIN] = p[4];
    sc[SC_RTINY] = p[5]; sc[SC_RNF] = p[6];
    p += 8;
    const double* rx = p;
    p += NR;
    memcpy(rec.data() + g.o_yr, p, m * sizeof(double)); p += m;
    zfull_to(g, rec.data(), g.o_rzlu, g.o_rzuu, g.o_rzls, p, p + NR);
    memcpy(rec.data() + g.o_zp, p + n, m * sizeof(double));
    memcpy(rec.data() + g.o_zn, p + n + m, m * sizeof(double));
    p += 2 * NR;
    for (int i = 0; i < 2 * g.fc; ++i) rec[g.o_fr + i] = p[i];
    p += 2 * g.fc;
    memcpy(rec.data() + g.o_xr, p, n * sizeof(double));
    p += 2 * n;
    for (int q = 0; q < 8; ++q) sc[SC_WD_SHORT + q] = p[q];
    p += 8;
    memcpy(rec.data() + g.o_wdv, p, n * sizeof(double)); p += n;
    memcpy(rec.data() + g.o_wdy, p, m * sizeof(double)); p += m;
    zfull_to(g, rec.data(), g.o_wdzlu, g.o_wdzuu, g.o_wdzls, p, p + n);
    p += 2 * n;
    for (int q = 0; q < 4; ++q) sc[SC_SOFT + q] = p[q];
    p += 4;
    for (int q = 0; q < 7; ++q) sc[SC_MUFREE + q] = p[q];
    if (resto) {
      memcpy(rec.data() + g.o_v, rx, n * sizeof(double));
      memcpy(rec.data() + g.o_p, rx + n, m * sizeof(double));
      memcpy(rec.data() + g.o_nn, rx + n + m, m * sizeof(double));
    } else {
      memcpy(rec.data() + g.o_v, main_x, n * sizeof(double));
    }
    memcpy(rec.data() + g.o_th, th.data() + (size_t)s * g.n_theta, g.n_theta * sizeof(double));
    HIPCHK(c, hipMemcpyAsync(c->ws + (size_t)s * g.stride, rec.data(), g.stride * sizeof(double),
                             hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
  }
  launch_prepare(g, c->ws, count, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return HIPIPM_OK;
}

int hipipm_start(hipipm_ctx* c, int32_t count, const double* theta, const double* warm, void* stream) {
  if (!c || count < 0 || count > c->slots || (count > 0 && !theta)) return HIPIPM_ERR_INVALID_ARG;
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  if (count == 0) return HIPIPM_OK;
  hipStream_t st = (hipStream_t)stream;
  launch_setup(c->cfg, c->ws, count, count, theta, warm, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return HIPIPM_OK;
}

int hipipm_step(hipipm_ctx* c, int32_t count, int32_t passes, const double* theta, const double* warm,
                void* stream) {
  if (!c || count < 0 || count > c->slots || passes < 0 || (count > 0 && !theta)) return HIPIPM_ERR_INVALID_ARG;
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  if (count == 0) return HIPIPM_OK;
  hipStream_t st = (hipStream_t)stream;
  Outs none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // the same kernels as a solve: the fused pass kernel (precision 1, or fuse_below > 0), else
  // the per-phase kernels; no refill (no counter block)
  const bool fused = c->opts.precision == 1 || c->opts.fuse_below > 0;
  for (int p = 0; p < passes; ++p) {
    launch_eval(c->cfg, c->ws, count, st);
    if (fused) {
      launch_iter(c->cfg, c->ws, count, theta, warm, none, nullptr, 0, st);
    } else {
      launch_pre(c->cfg, c->ws, count, theta, warm, none, nullptr, 0, st);
      launch_fac(c->cfg, c->ws, count, st);
      launch_sol(c->cfg, c->ws, count, warm, st);
      launch_ls(c->cfg, c->ws, count, st);
    }
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return HIPIPM_OK;
}

int hipipm_kkt_factor_solve(hipipm_ctx* c, int32_t count, const double* theta, const double* v, const double* y,
                            const double* zl, const double* zu, double mu, double delta_x, double delta_c,
                            const double* rhs, double* sol, int32_t* inertia_ok, void* stream) {
  if (!c || count < 0 || count > c->slots || !theta || !v || !y || !zl || !zu || !rhs || !sol || !inertia_ok)
    return HIPIPM_ERR_INVALID_ARG;
  if (!c->ws) return fail(c, HIPIPM_ERR_WORKSPACE, "no workspace bound");
  if (count == 0) return HIPIPM_OK;
  const Cfg& g = c->cfg;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> hv((size_t)count * g.n), hy((size_t)count * g.m), hzl((size_t)count * g.n),
      hzu((size_t)count * g.n), th((size_t)count * g.n_theta), rec((size_t)g.stride);
  HIPCHK(c, hipMemcpyAsync(hv.data(), v, hv.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(hy.data(), y, hy.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(hzl.data(), zl, hzl.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(hzu.data(), zu, hzu.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(th.data(), theta, th.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  for (int s = 0; s < count; ++s) {
    std::fill(rec.begin(), rec.end(), 0.0);
    double* sc = rec.data() + g.o_sc;
    sc[SC_PHASE] = PH_REGULAR;
    sc[SC_MU] = mu;
    memcpy(rec.data() + g.o_v, hv.data() + (size_t)s * g.n, g.n * 8);
    memcpy(rec.data() + g.o_y, hy.data() + (size_t)s * g.m, g.m * 8);
    zfull_to(g, rec.data(), g.o_zlu, g.o_zuu, g.o_zls, hzl.data() + (size_t)s * g.n, hzu.data() + (size_t)s * g.n);
    memcpy(rec.data() + g.o_th, th.data() + (size_t)s * g.n_theta, g.n_theta * 8);
    HIPCHK(c, hipMemcpyAsync(c->ws + (size_t)s * g.stride, rec.data(), g.stride * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
  }
  launch_prepare(g, c->ws, count, st);
  launch_eval(g, c->ws, count, st);
  launch_kkt_test(g, c->ws, count, delta_x, delta_c, rhs, sol, inertia_ok, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return HIPIPM_OK;
}

int hipipm_stage_derivs(hipipm_ctx* c, int32_t count, const double* x, const double* u, const double* lam,
                        double* F, double* G, double* H, void* stream) {
  if (!c || count < 0 || !x || !u || !lam || !F || !G || !H) return HIPIPM_ERR_INVALID_ARG;
  if (count == 0) return HIPIPM_OK;
  hipStream_t st = (hipStream_t)stream;
  launch_stage_derivs(c->cfg, count, x, u, lam, F, G, H, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return HIPIPM_OK;
}

const char* hipipm_last_error(const hipipm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void hipipm_destroy(hipipm_ctx* c) {
  if (!c) return;
  if (c->hcnt) (void)hipHostFree(c->hcnt);
  for (auto e : c->cev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
