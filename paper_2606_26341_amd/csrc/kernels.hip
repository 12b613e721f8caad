// gfx950 kernels of one batched interior-point iteration (Sec. V) launched one per phase, the
// derivative kernel, slot setup and the kernel-parity hooks, and the host launch wrappers.  One
// pass is
//
//   k_eval   RK4 dynamics, Jacobian and Lagrangian-Hessian contraction per (slot, stage,
//            direction) -- eq. (4) W and A = grad c
//   k_pre, k_fac, k_sol, k_ls   the per-slot phases of slot.h, one launch each, or
//   k_iter   all four phases of a slot back to back (iter_fp64.hip, iter_mixed.hip)
//
// The factor and solve live in kernels of their own so that each gets the register budget of
// its own working set; the fused k_iter is the default for every pass.
#include "slot.h"

namespace hipipm {

// ============================================================================ derivatives
__global__ __launch_bounds__(256) void k_eval(Cfg c, double* ws, int slots) {
  const long long per = (long long)c.N * NZ;
  const long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= (long long)slots * per) return;
  const int slot = (int)(item / per);
  const int rem = (int)(item % per);
  const int k = rem / NZ, j = rem % NZ;
  Slot s = make_slot(c, ws, slot);
  const int ph = (int)s.sc[SC_PHASE];
  if (ph == PH_EMPTY) return;
  const double* yv = (ph == PH_RESTO) ? s.yr : s.y;
  double x[NX], u[NU], lam[NX], Fv[NX], Gc[NX], Hc[NZ];
#pragma unroll
  for (int i = 0; i < NX; ++i) x[i] = s.v[xo(k) + i];
#pragma unroll
  for (int i = 0; i < NU; ++i) u[i] = s.v[uo(k) + i];
  // the rows x_{k+1} - F(x_k, u_k) contribute -sum_r y_r Hess F_r to W
#pragma unroll
  for (int i = 0; i < NX; ++i) lam[i] = -yv[(k + 1) * NX + i];
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

// the counter block of a solve: queue head = first instance not yet in a slot, nothing done
__global__ __launch_bounds__(64) void k_counters_init(Counters* cnt, int head, int n_inst) {
  const int t = threadIdx.x;
  if (t == 0) { cnt->head = head; cnt->done = 0; cnt->n_inst = n_inst; cnt->pad = 0; }
  if (t < N_STATS) cnt->st[t] = 0ull;
}

__global__ __launch_bounds__(64) void k_prepare(Cfg c, double* ws) {
  Slot s = make_slot(c, ws, blockIdx.x);
  fill_ref(c, s, threadIdx.x);
}

__global__ __launch_bounds__(64) void k_setup(Cfg c, double* ws, int slots, int n_active, const double* theta,
                                              const double* warm) {
  const int slot = blockIdx.x, lane = threadIdx.x;
  Slot s = make_slot(c, ws, slot);
  if (slot < n_active) {
    init_instance(c, s, slot, theta, warm, lane);
  } else {
    for (int q = lane; q < SC_LEN; q += WAVE) s.sc[q] = 0.0;
    __syncthreads();
    if (lane == 0) s.sc[SC_PHASE] = PH_EMPTY;
  }
}

// ============================================================================ pass kernels
__global__ __launch_bounds__(64) void k_pre(Cfg c, double* ws, const double* theta, const double* warm, Outs out,
                                            Counters* cnt, int refill) {
  pre_body(c, make_slot(c, ws, blockIdx.x), theta, warm, out, cnt, refill, threadIdx.x);
}
__global__ __launch_bounds__(64) void k_fac(Cfg c, double* ws) {
  __shared__ FacLds L;
  fac_body(c, make_slot(c, ws, blockIdx.x), L, false, false, threadIdx.x);
}
__global__ __launch_bounds__(64) void k_sol(Cfg c, double* ws, const double* warm) {
  HIP_DYNAMIC_SHARED(double, sol_dyn)
  sol_body(c, make_slot(c, ws, blockIdx.x), warm, sol_dyn, nullptr, false, false, threadIdx.x);
}
__global__ __launch_bounds__(64) void k_ls(Cfg c, double* ws) {
  HIP_DYNAMIC_SHARED(double, sol_dyn)
  ls_body(c, make_slot(c, ws, blockIdx.x), sol_dyn, false, false, threadIdx.x);
}
// ============================================================================ parity hooks
__global__ __launch_bounds__(64) void k_stage_derivs(Cfg c, int count, const double* x, const double* u,
                                                     const double* lam, double* F, double* G, double* H) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= count * NZ) return;
  const int k = item / NZ, j = item % NZ;
  double xx[NX], uu[NU], ll[NX], Fv[NX], Gc[NX], Hc[NZ];
  for (int i = 0; i < NX; ++i) { xx[i] = x[k * NX + i]; ll[i] = lam[k * NX + i]; }
  for (int i = 0; i < NU; ++i) uu[i] = u[k * NU + i];
  rk4_deriv_dir(c, xx, uu, ll, j, j == 0 ? Fv : nullptr, Gc, Hc);
  for (int i = 0; i < NX; ++i) G[(long long)k * NX * NZ + i * NZ + j] = Gc[i];
  for (int i = 0; i < NZ; ++i) H[(long long)k * NZ * NZ + i * NZ + j] = Hc[i];
  if (j == 0)
    for (int i = 0; i < NX; ++i) F[k * NX + i] = Fv[i];
}

// factor + solve the regular-phase system of slot `blockIdx.x` (derivatives already evaluated)
__global__ __launch_bounds__(64) void k_kkt_test(Cfg c, double* ws, double dxp, double dcp, const double* rhs,
                                                 double* sol, int* inertia_ok) {
  __shared__ FacLds L;
  HIP_DYNAMIC_SHARED(double, sol_dyn)
  const int slot = blockIdx.x, lane = threadIdx.x;
  Slot s = make_slot(c, ws, slot);
  Iter it = cur_iter(s, false);
  Elim e{false, false, 0.0, 0.0, 0.0};
  kkt_stage_data(c, s, it, e, lane);
  e.dxp = dxp;
  e.dcp = dcp;
  // precision 1: FP32 factor and FP32 solve with FP64 refinement; as in the solver, an FP32
  // inertia verdict other than "correct" is taken again in FP64 (then the FP64 factor solves; no
  // refinement-failure fallback here: the caller sees the refined FP32 result).  inertia_ok = 1
  // inertia correct, 2 also the FP32 factor was used and its refinement converged, 0 wrong
  bool f32 = c.prec == 1;
  int st = factor_any(c, s, e, L, f32, lane);
  if (f32 && st != 0) {
    f32 = false;
    st = factor_any(c, s, e, L, false, lane);
  }
  if (lane == 0) { inertia_ok[slot] = (st == 0) ? 1 : 0; s.sc[SC_FPREC] = f32 ? 1.0 : 0.0; }
  if (st != 0) return;
  const double* b = rhs + (long long)slot * (c.n + c.m);
  for (int i = lane; i < c.n; i += WAVE) s.rv[i] = b[i];
  for (int r = lane; r < c.m; r += WAVE) s.rc[r] = b[c.n + r];
  __syncthreads();
  const bool conv = solve_refined(c, s, e, s.rv, s.rc, nullptr, nullptr, s.dv, s.dy, nullptr, nullptr, sol_dyn, f32, lane);
  if (lane == 0 && f32 && conv) inertia_ok[slot] = 2;
  double* o = sol + (long long)slot * (c.n + c.m);
  for (int i = lane; i < c.n; i += WAVE) o[i] = s.dv[i];
  for (int r = lane; r < c.m; r += WAVE) o[c.n + r] = s.dy[r];
}

}  // namespace hipipm

// ============================================================================ launch wrappers
namespace hipipm {
void launch_eval(const Cfg& c, double* ws, int slots, hipStream_t st) {
  long long items = (long long)slots * c.N * NZ;
  int blocks = (int)((items + 255) / 256);
  if (blocks > 0) hipLaunchKernelGGL(k_eval, dim3(blocks), dim3(256), 0, st, c, ws, slots);
}
int sd_len_host(int NI) { return sd_len_of(NI); }
void launch_pre(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                Counters* cnt, int refill, hipStream_t st) {
  hipLaunchKernelGGL(k_pre, dim3(slots), dim3(WAVE), 0, st, c, ws, theta, warm, out, cnt, refill);
}
void launch_fac(const Cfg& c, double* ws, int slots, hipStream_t st) {
  hipLaunchKernelGGL(k_fac, dim3(slots), dim3(WAVE), 0, st, c, ws);
}
void launch_sol(const Cfg& c, double* ws, int slots, const double* warm, hipStream_t st) {
  hipLaunchKernelGGL(k_sol, dim3(slots), dim3(WAVE), sol_bytes(c), st, c, ws, warm);
}
void launch_ls(const Cfg& c, double* ws, int slots, hipStream_t st) {
  hipLaunchKernelGGL(k_ls, dim3(slots), dim3(WAVE), sol_bytes(c), st, c, ws);
}
void launch_iter_fp64(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                      Counters* cnt, int refill, hipStream_t st);
void launch_iter_mixed(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                       Counters* cnt, int refill, hipStream_t st);
void launch_iter(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                 Counters* cnt, int refill, hipStream_t st) {
  if (c.prec == 1)
    launch_iter_mixed(c, ws, slots, theta, warm, out, cnt, refill, st);
  else
    launch_iter_fp64(c, ws, slots, theta, warm, out, cnt, refill, st);
}
void launch_setup(const Cfg& c, double* ws, int slots, int n_active, const double* theta, const double* warm,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(slots), dim3(WAVE), 0, st, c, ws, slots, n_active, theta, warm);
}
void launch_stage_derivs(const Cfg& c, int count, const double* x, const double* u, const double* lam, double* F,
                         double* G, double* H, hipStream_t st) {
  int blocks = (count * NZ + 63) / 64;
  if (blocks > 0) hipLaunchKernelGGL(k_stage_derivs, dim3(blocks), dim3(64), 0, st, c, count, x, u, lam, F, G, H);
}
void launch_counters_init(Counters* cnt, int head, int n_inst, hipStream_t st) {
  hipLaunchKernelGGL(k_counters_init, dim3(1), dim3(WAVE), 0, st, cnt, head, n_inst);
}
void launch_prepare(const Cfg& c, double* ws, int count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_prepare, dim3(count), dim3(WAVE), 0, st, c, ws);
}
void launch_kkt_test(const Cfg& c, double* ws, int count, double dxp, double dcp, const double* rhs, double* sol,
                     int* inertia_ok, hipStream_t st) {
  hipLaunchKernelGGL(k_kkt_test, dim3(count), dim3(WAVE), sol_bytes(c), st, c, ws, dxp, dcp, rhs, sol, inertia_ok);
}
}  // namespace hipipm

