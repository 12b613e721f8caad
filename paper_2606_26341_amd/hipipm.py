"""Thin ctypes binding of libhipipm.so (include/hipipm.h).

Argument marshalling only: device memory comes from torch (cuda tensors on ROCm), every
step of the solver runs in the library's HIP kernels.  Importing this module loads the
library and raises if it has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipipm.so")

STATUS = {0: "RUNNING", 1: "CONVERGED", 2: "MAX_ITER", 3: "RESTO_FAILED", 4: "INFEASIBLE", 5: "NUMERICAL"}
ST_CONVERGED = 1
KERNELS = ("eval", "pre", "factor", "solve", "linesearch", "fused", "setup", "async")


class ProblemDesc(C.Structure):
    _fields_ = [("family", C.c_int32), ("N", C.c_int32), ("n_agents", C.c_int32), ("n_obs", C.c_int32),
                ("dt", C.c_double), ("mass", C.c_double), ("jxx", C.c_double), ("jyy", C.c_double),
                ("jzz", C.c_double), ("arm", C.c_double), ("ctau", C.c_double), ("grav", C.c_double),
                ("q_weight", C.c_double), ("r_weight", C.c_double), ("d_min", C.c_double)]


class Options(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_iter", C.c_int32), ("mu_init", C.c_double), ("kappa_eps", C.c_double),
        ("kappa_mu", C.c_double), ("theta_mu", C.c_double), ("tau_min", C.c_double),
        ("kappa1", C.c_double), ("kappa2", C.c_double), ("lam_max", C.c_double), ("s_max", C.c_double),
        ("delta_min", C.c_double), ("delta_0", C.c_double), ("delta_max", C.c_double),
        ("delta_c_bar", C.c_double), ("kappa_c", C.c_double),
        ("kappa_minus", C.c_double), ("kappa_plus", C.c_double), ("kappa_plus_bar", C.c_double),
        ("gamma_theta", C.c_double), ("gamma_phi", C.c_double), ("delta_sw", C.c_double),
        ("s_theta", C.c_double), ("s_phi", C.c_double), ("eta_phi", C.c_double), ("gamma_alpha", C.c_double),
        ("max_soc", C.c_int32), ("kappa_soc", C.c_double), ("kappa_sigma", C.c_double),
        ("rho_resto", C.c_double), ("kappa_resto", C.c_double), ("bound_mult_reset", C.c_double),
        ("poll_every", C.c_int32), ("timing", C.c_int32),
        ("fuse_below", C.c_int32), ("precision", C.c_int32), ("refine_max", C.c_int32),
        ("refine_tol", C.c_double), ("warm_mu0", C.c_double), ("warm_push", C.c_double),
        ("warm_iter_cap", C.c_int32), ("warm_gate", C.c_int32), ("watchdog_trigger", C.c_int32),
        ("watchdog_max", C.c_int32), ("soft_resto_max", C.c_int32), ("soft_resto_factor", C.c_double),
        ("mu_strategy", C.c_int32), ("async_passes", C.c_int32), ("nested_resto", C.c_int32),
        ("resto_ls_max", C.c_int32),
    ]


class Dims(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("n", "m", "n_w", "n_s", "n_theta", "n_lower", "n_upper", "N", "nx", "nu",
                                         "n_ineq")]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("iterations", "resto_iterations", "soc_tried", "soc_accepted",
                                         "factorizations", "resto_entries", "tiny_steps", "passes",
                                         "instances_done", "solves", "fused_factorizations",
                                         "fused_solves", "refine_sweeps", "fp64_fallbacks", "warm_started",
                                         "warm_rejected", "warm_restarts", "fp32_retakes", "watchdog_starts",
                                         "watchdog_reverts", "soft_resto_steps", "soft_resto_fails",
                                         "mu_fallbacks", "nested_restorations", "cycles_eval", "cycles_pre", "cycles_factor",
                                         "cycles_solve", "cycles_linesearch")]


_lib = None
EXPORTS = ("hipipm_default_options", "hipipm_create", "hipipm_get_dims", "hipipm_resident_slots", "hipipm_workspace_bytes",
           "hipipm_bind_workspace", "hipipm_solve", "hipipm_solve_noalloc", "hipipm_stats_get", "hipipm_reset_stats",
           "hipipm_kernel_times", "hipipm_state_len", "hipipm_state_import", "hipipm_start", "hipipm_step",
           "hipipm_state_export", "hipipm_kkt_factor_solve", "hipipm_stage_derivs", "hipipm_last_error",
           "hipipm_destroy")


def load(path: str = LIB_PATH):
    """Load libhipipm.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    L = C.CDLL(path)
    vp, i32, dp = C.c_void_p, C.c_int32, C.c_double
    L.hipipm_default_options.argtypes = [vp]
    L.hipipm_create.argtypes = [vp, vp, i32, C.POINTER(vp)]
    L.hipipm_get_dims.argtypes = [vp, vp]
    L.hipipm_resident_slots.argtypes = [vp, C.POINTER(i32)]
    L.hipipm_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.hipipm_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.hipipm_solve.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.hipipm_solve_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.hipipm_stats_get.argtypes = [vp, vp]
    L.hipipm_reset_stats.argtypes = [vp]
    L.hipipm_kernel_times.argtypes = [vp, C.POINTER(i32), vp, vp]
    L.hipipm_state_len.argtypes = [vp, C.POINTER(i32)]
    L.hipipm_state_import.argtypes = [vp, i32, vp, vp, vp]
    L.hipipm_start.argtypes = [vp, i32, vp, vp, vp]
    L.hipipm_step.argtypes = [vp, i32, i32, vp, vp, vp]
    L.hipipm_state_export.argtypes = [vp, i32, vp, vp]
    L.hipipm_kkt_factor_solve.argtypes = [vp, i32, vp, vp, vp, vp, vp, dp, dp, dp, vp, vp, vp, vp]
    L.hipipm_stage_derivs.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.hipipm_last_error.argtypes = [vp]
    L.hipipm_last_error.restype = C.c_char_p
    L.hipipm_destroy.argtypes = [vp]
    L.hipipm_destroy.restype = None
    _lib = L
    return L


def default_options(**kw) -> Options:
    o = Options()
    load().hipipm_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def desc_from(w) -> ProblemDesc:
    m = w.model
    return ProblemDesc(int(w.family), int(w.N), int(w.n_agents), int(w.n_obs), float(w.dt), float(m.mass),
                       float(m.jxx), float(m.jyy), float(m.jzz), float(m.arm), float(m.ctau), float(m.grav),
                       float(w.q_weight), float(w.r_weight), float(w.d_min))


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class HipipmError(RuntimeError):
    pass


def resident_slots(workload, options: Options | None = None, device=None) -> int:
    """Slots the GPU runs at once in the asynchronous-slot kernel for this workload and options
    (hipipm_resident_slots): with that many slots and a large async_passes a solve is one launch
    with every slot resident."""
    if not torch.cuda.is_available():
        raise HipipmError("hipipm needs a ROCm GPU (torch.cuda.is_available() is False)")
    L = load()
    torch.cuda.set_device(torch.device(device if device is not None else "cuda:0"))
    desc = desc_from(workload)
    opts = options if options is not None else default_options()
    h = C.c_void_p()
    rc = L.hipipm_create(C.byref(desc), C.byref(opts), 1, C.byref(h))
    if rc != 0:
        raise HipipmError(f"hipipm_create failed with {rc}")
    n = C.c_int32()
    try:
        rc = L.hipipm_resident_slots(h, C.byref(n))
        if rc != 0:
            raise HipipmError(f"hipipm_resident_slots failed with {rc}: {L.hipipm_last_error(h).decode()}")
    finally:
        L.hipipm_destroy(h)
    return int(n.value)


class Solver:
    """A solver context with `slots` concurrently iterating instances and its workspace."""

    def __init__(self, workload, slots: int, options: Options | None = None, device=None):
        if not torch.cuda.is_available():
            raise HipipmError("hipipm needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.L = load()
        self.device = torch.device(device if device is not None else "cuda:0")
        torch.cuda.set_device(self.device)
        self.desc = desc_from(workload)
        self.opts = options if options is not None else default_options()
        self.slots = int(slots)
        h = C.c_void_p()
        self._check(self.L.hipipm_create(C.byref(self.desc), C.byref(self.opts), self.slots, C.byref(h)), None)
        self.h = h
        d = Dims()
        self._check(self.L.hipipm_get_dims(self.h, C.byref(d)))
        self.dims = d
        nb = C.c_size_t()
        self._check(self.L.hipipm_workspace_bytes(self.h, C.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self._check(self.L.hipipm_bind_workspace(self.h, _ptr(self.workspace), nb.value))

    def _check(self, rc, h="self"):
        if rc != 0:
            msg = self.L.hipipm_last_error(self.h).decode() if (h == "self" and getattr(self, "h", None)) else ""
            raise HipipmError(f"hipipm call failed with {rc}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.L.hipipm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ solve
    def alloc_outputs(self, n_inst: int) -> dict:
        d, dev = self.dims, self.device
        f64 = dict(dtype=torch.float64, device=dev)
        return dict(x=torch.empty((n_inst, d.n), **f64), y=torch.empty((n_inst, d.m), **f64),
                    zl=torch.empty((n_inst, d.n), **f64), zu=torch.empty((n_inst, d.n), **f64),
                    obj=torch.empty(n_inst, **f64), kkt=torch.empty(n_inst, **f64),
                    status=torch.empty(n_inst, dtype=torch.int32, device=dev),
                    iters=torch.empty(n_inst, dtype=torch.int32, device=dev))

    def solve(self, theta: torch.Tensor, warm: torch.Tensor | None = None, out: dict | None = None,
              stream=None) -> dict:
        assert theta.dtype == torch.float64 and theta.dim() == 2 and theta.shape[1] == self.dims.n_theta
        theta = theta.contiguous()
        n_inst = theta.shape[0]
        if warm is not None:
            assert warm.shape == (n_inst, self.dims.n_w + self.dims.m) and warm.dtype == torch.float64
            warm = warm.contiguous()
        o = out if out is not None else self.alloc_outputs(n_inst)
        self._check(self.L.hipipm_solve(self.h, n_inst, _ptr(theta), _ptr(warm), _ptr(o["x"]), _ptr(o["y"]),
                                        _ptr(o["zl"]), _ptr(o["zu"]), _ptr(o["obj"]), _ptr(o["kkt"]),
                                        _ptr(o["status"]), _ptr(o["iters"]), _stream(stream)))
        return o

    def solve_noalloc(self, theta: torch.Tensor, warm: torch.Tensor | None = None, out: dict | None = None,
                      stream=None) -> dict:
        """solve() through hipipm_solve_noalloc: the library's static device workspace instead of the
        bound one, no allocation inside the call (pass `out` to allocate nothing here either)."""
        assert theta.dtype == torch.float64 and theta.dim() == 2 and theta.shape[1] == self.dims.n_theta
        theta = theta.contiguous()
        n_inst = theta.shape[0]
        if warm is not None:
            assert warm.shape == (n_inst, self.dims.n_w + self.dims.m) and warm.dtype == torch.float64
            warm = warm.contiguous()
        o = out if out is not None else self.alloc_outputs(n_inst)
        self._check(self.L.hipipm_solve_noalloc(self.h, n_inst, _ptr(theta), _ptr(warm), _ptr(o["x"]), _ptr(o["y"]),
                                                _ptr(o["zl"]), _ptr(o["zu"]), _ptr(o["obj"]), _ptr(o["kkt"]),
                                                _ptr(o["status"]), _ptr(o["iters"]), _stream(stream)))
        return o

    def stats(self) -> dict:
        s = Stats()
        self._check(self.L.hipipm_stats_get(self.h, C.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in Stats._fields_}

    def reset_stats(self):
        self._check(self.L.hipipm_reset_stats(self.h))

    def kernel_times(self) -> dict:
        k = len(KERNELS)
        n = C.c_int32(k)
        ms = (C.c_double * k)()
        cnt = (C.c_int64 * k)()
        self._check(self.L.hipipm_kernel_times(self.h, C.byref(n), ms, cnt))
        return {KERNELS[i]: (float(ms[i]), int(cnt[i])) for i in range(min(k, n.value))}

    # ------------------------------------------------------------------ test hooks
    def state_len(self) -> int:
        n = C.c_int32()
        self._check(self.L.hipipm_state_len(self.h, C.byref(n)))
        return int(n.value)

    def state_import(self, states, theta: torch.Tensor, stream=None):
        import numpy as np
        states = np.ascontiguousarray(states, dtype=np.float64)
        assert states.ndim == 2 and states.shape[1] == self.state_len(), "state rows of another length"
        count = states.shape[0]
        assert count <= self.slots and theta.shape == (count, self.dims.n_theta)
        self._check(self.L.hipipm_state_import(self.h, count, states.ctypes.data_as(C.c_void_p),
                                               _ptr(theta.contiguous()), _stream(stream)))

    def start(self, theta: torch.Tensor, warm: torch.Tensor | None = None, stream=None):
        """Start the instances of theta (and warm rows) in slots 0..count-1 without solving."""
        assert theta.shape[0] <= self.slots and theta.shape[1] == self.dims.n_theta
        assert warm is None or warm.shape == (theta.shape[0], self.dims.n_w + self.dims.m)
        theta = theta.contiguous()
        warm = None if warm is None else warm.contiguous()
        self._check(self.L.hipipm_start(self.h, theta.shape[0], _ptr(theta), _ptr(warm), _stream(stream)))

    def step(self, count: int, passes: int, theta: torch.Tensor, warm: torch.Tensor | None = None, stream=None):
        """`passes` passes over slots 0..count-1 (theta / warm: the rows of those slots' instances)."""
        assert 0 <= count <= self.slots and theta.shape[0] >= count and theta.shape[1] == self.dims.n_theta
        assert warm is None or warm.shape == (theta.shape[0], self.dims.n_w + self.dims.m)
        theta = theta.contiguous()
        warm = None if warm is None else warm.contiguous()
        self._check(self.L.hipipm_step(self.h, int(count), int(passes), _ptr(theta), _ptr(warm), _stream(stream)))

    def state_export(self, count: int, stream=None):
        import numpy as np
        out = np.zeros((count, self.state_len()))
        self._check(self.L.hipipm_state_export(self.h, int(count), out.ctypes.data_as(C.c_void_p), _stream(stream)))
        return out

    def kkt_factor_solve(self, theta, v, y, zl, zu, mu, delta_x, delta_c, rhs, stream=None):
        count = theta.shape[0]
        d = self.dims
        sol = torch.empty((count, d.n + d.m), dtype=torch.float64, device=self.device)
        ok = torch.empty(count, dtype=torch.int32, device=self.device)
        self._check(self.L.hipipm_kkt_factor_solve(self.h, count, _ptr(theta), _ptr(v), _ptr(y), _ptr(zl), _ptr(zu),
                                                   float(mu), float(delta_x), float(delta_c), _ptr(rhs), _ptr(sol),
                                                   _ptr(ok), _stream(stream)))
        return sol, ok

    def stage_derivs(self, x, u, lam, stream=None):
        count = x.shape[0]
        dev = self.device
        F = torch.empty((count, 13), dtype=torch.float64, device=dev)
        G = torch.empty((count, 13, 17), dtype=torch.float64, device=dev)
        H = torch.empty((count, 17, 17), dtype=torch.float64, device=dev)
        self._check(self.L.hipipm_stage_derivs(self.h, count, _ptr(x.contiguous()), _ptr(u.contiguous()),
                                               _ptr(lam.contiguous()), _ptr(F), _ptr(G), _ptr(H), _stream(stream)))
        return F, G, H
