"""CPU FP64 oracle -- test infrastructure only.

A plain, slow, dense re-statement of the paper's interior-point method
(Sec. IV, Table I) used to check the HIP solver.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does.  The C sources in this directory share no code with the HIP
library.  ``build()`` compiles them with gcc into ``liboracle.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["bk.c", "quad.c", "ipm.c"]

PH_INIT_Y, PH_REGULAR, PH_RESTO, PH_DONE = 0, 1, 2, 3
ST_RUNNING, ST_CONVERGED, ST_MAX_ITER, ST_RESTO_FAILED, ST_INFEASIBLE, ST_NUMERICAL = range(6)
NSTAT = 17   # per-instance counters of solve_quad (see ipmo_solve_quad)


def build() -> str:
    cmd = ["gcc", "-O2", "-march=x86-64-v2", "-fPIC", "-shared", "-Wall", "-o", _SO]
    cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-lm", "-lpthread"]
    subprocess.check_call(cmd)
    return _SO


class Opts(C.Structure):
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
        ("warm_mu0", C.c_double), ("warm_push", C.c_double), ("warm_iter_cap", C.c_int32),
        ("warm_gate", C.c_int32), ("watchdog_trigger", C.c_int32), ("watchdog_max", C.c_int32),
        ("soft_resto_max", C.c_int32), ("soft_resto_factor", C.c_double), ("mu_strategy", C.c_int32),
        ("nested_resto", C.c_int32), ("resto_ls_max", C.c_int32),
    ]


class QuadDesc(C.Structure):
    _fields_ = [
        ("family", C.c_int32), ("N", C.c_int32), ("n_agents", C.c_int32), ("n_obs", C.c_int32),
        ("dt", C.c_double), ("mass", C.c_double), ("jxx", C.c_double), ("jyy", C.c_double),
        ("jzz", C.c_double), ("arm", C.c_double), ("ctau", C.c_double), ("grav", C.c_double),
        ("q_weight", C.c_double), ("r_weight", C.c_double), ("d_min", C.c_double),
    ]


_lib = None
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
CB_F = C.CFUNCTYPE(None, C.c_void_p, _DP, _DP)
CB_H = C.CFUNCTYPE(None, C.c_void_p, _DP, C.c_double, _DP, _DP)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        L = C.CDLL(_SO)
        L.ipmo_create_quad.restype = C.c_void_p
        L.ipmo_create_quad.argtypes = [C.c_void_p, C.c_void_p, _DP, _DP]
        L.ipmo_create_generic.restype = C.c_void_p
        L.ipmo_create_generic.argtypes = [C.c_int, C.c_int, _DP, _DP, CB_F, CB_F, CB_F, CB_F, CB_H,
                                          C.c_void_p, _DP]
        for nm in ("ipmo_destroy",):
            getattr(L, nm).argtypes = [C.c_void_p]
        for nm in ("ipmo_pass", "ipmo_run", "ipmo_phase", "ipmo_status", "ipmo_iter", "ipmo_state_len"):
            getattr(L, nm).argtypes = [C.c_void_p]
            getattr(L, nm).restype = C.c_int
        L.ipmo_state_get.argtypes = [C.c_void_p, _DP]
        L.ipmo_state_set.argtypes = [C.c_void_p, _DP]
        L.ipmo_last_info.argtypes = [C.c_void_p, _DP]
        L.ipmo_last_step.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP]
        L.ipmo_outputs.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP, _DP, _IP, _IP, _IP]
        L.ipmo_solve_quad.argtypes = [C.c_void_p, C.c_void_p, C.c_int, _DP, _DP, C.c_int,
                                      _DP, _DP, _DP, _DP, _DP, _DP, _IP, _IP, _IP]
        L.ipmo_bk_factor.argtypes = [C.c_int, _DP, _IP, _IP, _IP]
        L.ipmo_bk_solve.argtypes = [C.c_int, _DP, _IP, _IP, _DP]
        L.quad_stage_derivs.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP, _DP]
        L.quad_xdot.argtypes = [C.c_void_p, _DP, _DP, _DP]
        L.quad_cold_start.argtypes = [C.c_void_p, _DP, _DP]
        L.ipmo_quad_kkt_error.argtypes = [C.c_void_p, C.c_void_p, _DP, _DP, _DP, _DP, _DP, C.c_double]
        L.ipmo_quad_kkt_error.restype = C.c_double
        L.ipmo_quad_eval.argtypes = [C.c_void_p, _DP, _DP, _DP, C.c_double, _DP, _DP, _DP, _DP, _DP]
        L.ipmo_ftb_primal.argtypes = [C.c_int, _DP, _DP, _DP, _DP, C.c_double]
        L.ipmo_ftb_primal.restype = C.c_double
        L.ipmo_ftb_dual.argtypes = [C.c_int, _DP, _DP, _DP, _DP, _DP, _DP, C.c_double]
        L.ipmo_ftb_dual.restype = C.c_double
        L.ipmo_acceptable.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _DP, _DP, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _IP]
        L.ipmo_alpha_min.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.ipmo_alpha_min.restype = C.c_double
        L.ipmo_kkt_dense.argtypes = [C.c_void_p, _DP]
        L.ipmo_kkt_dense.restype = C.c_int
        L.ipmo_handle_kkt_error.argtypes = [C.c_void_p, C.c_double]
        L.ipmo_handle_kkt_error.restype = C.c_double
        L.ipmo_last_soc.argtypes = [C.c_void_p, _DP, _DP, _DP]
        L.ipmo_last_soc.restype = C.c_int
        assert L.ipmo_sizeof_opts() == C.sizeof(Opts)
        assert L.ipmo_sizeof_desc() == C.sizeof(QuadDesc)
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_DP)


def _ip(a):
    if a is None:
        return None
    return a.ctypes.data_as(_IP)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().ipmo_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def desc_from(w) -> QuadDesc:
    """Problem descriptor from a workload object (duck-typed: family, N, n_agents, ...)."""
    m = w.model
    return QuadDesc(int(w.family), int(w.N), int(w.n_agents), int(w.n_obs), float(w.dt), float(m.mass),
                    float(m.jxx), float(m.jyy), float(m.jzz), float(m.arm), float(m.ctau), float(m.grav),
                    float(w.q_weight), float(w.r_weight), float(w.d_min))


# ----------------------------------------------------------------------------- dense LDL^T
def bk_factor(A: np.ndarray):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    perm = np.zeros(n, np.int32)
    blk = np.zeros(n, np.int32)
    inertia = np.zeros(3, np.int32)
    lib().ipmo_bk_factor(n, _p(A), _ip(perm), _ip(blk), _ip(inertia))
    return A, perm, blk, tuple(int(v) for v in inertia)


def bk_solve(fact, b: np.ndarray) -> np.ndarray:
    F, perm, blk, _ = fact
    x = np.array(b, dtype=np.float64, copy=True)
    lib().ipmo_bk_solve(F.shape[0], _p(F), _ip(perm), _ip(blk), _p(x))
    return x


def bk_unpack(fact):
    """Return (P, L, D) with P A P^T = L D L^T (dense, for tests)."""
    F, perm, blk, _ = fact
    n = F.shape[0]
    L = np.eye(n)
    D = np.zeros((n, n))
    k = 0
    while k < n:
        if blk[k] == 2:
            D[k, k] = F[k, k]
            D[k + 1, k] = D[k, k + 1] = F[k + 1, k]
            D[k + 1, k + 1] = F[k + 1, k + 1]
            L[k + 2:, k] = F[k + 2:, k]
            L[k + 2:, k + 1] = F[k + 2:, k + 1]
            k += 2
        else:
            D[k, k] = F[k, k]
            L[k + 1:, k] = F[k + 1:, k]
            k += 1
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    return P, L, D


# ----------------------------------------------------------------------------- model
def stage_derivs(w, x, u, lam=None):
    """F (13), G = dF/d(x,u) (13x17), sum_r lam_r Hess F_r (17x17) for one quadrotor stage."""
    d = desc_from(w)
    x = np.ascontiguousarray(x, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    lam = np.zeros(13) if lam is None else np.ascontiguousarray(lam, np.float64)
    F = np.zeros(13)
    G = np.zeros((13, 17))
    HL = np.zeros((17, 17))
    lib().quad_stage_derivs(C.byref(d), _p(x), _p(u), _p(lam), _p(F), _p(G), _p(HL))
    return F, G, HL


def xdot(w, x, u):
    d = desc_from(w)
    out = np.zeros(13)
    lib().quad_xdot(C.byref(d), _p(np.ascontiguousarray(x, np.float64)), _p(np.ascontiguousarray(u, np.float64)),
                    _p(out))
    return out


def cold_start(w, theta):
    d = desc_from(w)
    v = np.zeros(w.n)
    lib().quad_cold_start(C.byref(d), _p(np.ascontiguousarray(theta, np.float64)), _p(v))
    return v


def quad_eval(w, theta, v, y=None, objf=1.0):
    """(f, grad f, c, Jacobian, Hessian of objf f + y^T c) of the NMPC transcription at v."""
    d = desc_from(w)
    th = np.ascontiguousarray(theta, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    y = np.zeros(w.m) if y is None else np.ascontiguousarray(y, np.float64)
    f = np.zeros(1); g = np.zeros(w.n); c = np.zeros(w.m); J = np.zeros((w.m, w.n)); H = np.zeros((w.n, w.n))
    lib().ipmo_quad_eval(C.byref(d), _p(th), _p(v), _p(y), float(objf), _p(f), _p(g), _p(c), _p(J), _p(H))
    return f[0], g, c, J, H


def kkt_error(w, theta, x, y, zl, zu, mu=0.0, opts=None):
    d = desc_from(w)
    o = opts or default_opts()
    f = lambda a: _p(np.ascontiguousarray(a, np.float64))
    return lib().ipmo_quad_kkt_error(C.byref(d), C.byref(o), f(theta), f(x), f(y), f(zl), f(zu), float(mu))


# ----------------------------------------------------------------------------- solves
def solve_quad(w, thetas: np.ndarray, threads: int = 1, warm=None, opts=None) -> dict:
    """Solve the instances `thetas` of workload w; cold start, or warm from the rows of `warm`
    ([k][n_w + m] = primal w without slacks, then the equality multipliers y)."""
    thetas = np.ascontiguousarray(thetas, np.float64)
    k = thetas.shape[0]
    d = desc_from(w)
    o = opts or default_opts()
    out = dict(x=np.zeros((k, w.n)), y=np.zeros((k, w.m)), zl=np.zeros((k, w.n)), zu=np.zeros((k, w.n)),
               obj=np.zeros(k), kkt=np.zeros(k), status=np.zeros(k, np.int32), iters=np.zeros(k, np.int32),
               stats=np.zeros((k, NSTAT), np.int32))
    wr = None
    if warm is not None:
        wr = np.ascontiguousarray(warm, np.float64)
        assert wr.shape == (k, w.n_w + w.m)
    lib().ipmo_solve_quad(C.byref(d), C.byref(o), k, _p(thetas), _p(wr), int(threads),
                          _p(out["x"]), _p(out["y"]), _p(out["zl"]), _p(out["zu"]), _p(out["obj"]),
                          _p(out["kkt"]), _ip(out["status"]), _ip(out["iters"]), _ip(out["stats"]))
    return out


# ----------------------------------------------------------------------------- method pieces
def ftb_primal(x, dx, xl, xu, tau):
    f = lambda a: _p(np.ascontiguousarray(a, np.float64))
    return lib().ipmo_ftb_primal(len(x), f(x), f(dx), f(xl), f(xu), float(tau))


def ftb_dual(zl, zu, dzl, dzu, xl, xu, tau):
    f = lambda a: _p(np.ascontiguousarray(a, np.float64))
    return lib().ipmo_ftb_dual(len(zl), f(zl), f(zu), f(dzl), f(dzu), f(xl), f(xu), float(tau))


def acceptable(theta_max, theta_min, filt, thk, phk, gphi, alpha, tht, pht, opts=None):
    """(accepted, switching condition, Armijo condition) of a trial point; filt: list of (theta, phi)."""
    o = opts or default_opts()
    fth = np.array([a for a, _ in filt] + [0.0], np.float64)
    fph = np.array([b for _, b in filt] + [0.0], np.float64)
    out = np.zeros(3, np.int32)
    lib().ipmo_acceptable(C.byref(o), float(theta_max), float(theta_min), len(filt), _p(fth), _p(fph), float(thk),
                          float(phk), float(gphi), float(alpha), float(tht), float(pht), _ip(out))
    return bool(out[0]), int(out[1]), int(out[2])


def alpha_min(thk, gphi, theta_min, opts=None):
    o = opts or default_opts()
    return lib().ipmo_alpha_min(C.byref(o), float(thk), float(gphi), float(theta_min))


class Handle:
    """One oracle solve, stepped pass by pass (INIT_Y / REGULAR / RESTO)."""

    def __init__(self, h, n, m, keep=()):
        self.h = h
        self.n, self.m = n, m
        self._keep = keep

    @classmethod
    def quad(cls, w, theta, warm_row=None, opts=None):
        d = desc_from(w)
        o = opts or default_opts()
        th = np.ascontiguousarray(theta, np.float64)
        wr = None if warm_row is None else np.ascontiguousarray(warm_row, np.float64)
        h = lib().ipmo_create_quad(C.byref(d), C.byref(o), _p(th), _p(wr))
        return cls(h, w.n, w.m, keep=(d, o, th, wr))

    @classmethod
    def generic(cls, n, m, xl, xu, f, grad, c, jac, hess, x0, opts=None):
        """Problem from numpy callables: f(x)->float, grad(x)->(n,), c(x)->(m,),
        jac(x)->(m,n), hess(x, objf, y)->(n,n)."""
        o = opts or default_opts()

        def wrap_vec(fn, size):
            def cb(_ud, xp, outp):
                x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
                r = np.asarray(fn(x), dtype=np.float64).ravel()
                if size:
                    np.ctypeslib.as_array(outp, shape=(size,))[:] = r
            return CB_F(cb)

        def cb_f(_ud, xp, outp):
            x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            outp[0] = float(f(x))

        def cb_h(_ud, xp, objf, yp, outp):
            x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            y = np.ctypeslib.as_array(yp, shape=(max(m, 1),))[:m].copy()
            np.ctypeslib.as_array(outp, shape=(n * n,))[:] = np.asarray(hess(x, objf, y), np.float64).ravel()

        cbs = (CB_F(cb_f), wrap_vec(grad, n), wrap_vec(c, m), wrap_vec(jac, m * n), CB_H(cb_h))
        xl = np.ascontiguousarray(xl, np.float64)
        xu = np.ascontiguousarray(xu, np.float64)
        x0 = np.ascontiguousarray(x0, np.float64)
        h = lib().ipmo_create_generic(n, m, _p(xl), _p(xu), *cbs, C.byref(o), _p(x0))
        return cls(h, n, m, keep=(cbs, o, xl, xu, x0))

    def __del__(self):
        if getattr(self, "h", None):
            lib().ipmo_destroy(self.h)
            self.h = None

    def step(self) -> int:
        return lib().ipmo_pass(self.h)

    def run(self) -> int:
        return lib().ipmo_run(self.h)

    @property
    def phase(self):
        return lib().ipmo_phase(self.h)

    @property
    def status(self):
        return lib().ipmo_status(self.h)

    @property
    def iter(self):
        return lib().ipmo_iter(self.h)

    def state(self) -> np.ndarray:
        s = np.zeros(lib().ipmo_state_len(self.h))
        lib().ipmo_state_get(self.h, _p(s))
        return s

    def set_state(self, s: np.ndarray):
        s = np.ascontiguousarray(s, np.float64)
        assert s.size == lib().ipmo_state_len(self.h)
        lib().ipmo_state_set(self.h, _p(s))

    def last_info(self) -> dict:
        a = np.zeros(8)
        lib().ipmo_last_info(self.h, _p(a))
        return dict(delta_x=a[0], delta_c=a[1], alpha=a[2], alpha_z=a[3], soc=bool(a[4]), mu=a[5], tau=a[6],
                    nf=int(a[7]))

    def last_step(self):
        dx, dy, dzl, dzu = np.zeros(self.n), np.zeros(max(self.m, 1)), np.zeros(self.n), np.zeros(self.n)
        lib().ipmo_last_step(self.h, _p(dx), _p(dy), _p(dzl), _p(dzu))
        return dx, dy[:self.m], dzl, dzu

    def kkt_matrix(self):
        """The unperturbed matrix of eq. (7) of the current phase's sub-problem at the current
        iterate (full symmetric), or None outside the regular and restoration phases."""
        N = self.n + 3 * self.m + self.m
        K = np.zeros(N * N)
        nn = lib().ipmo_kkt_dense(self.h, _p(K))
        return K[:nn * nn].reshape(nn, nn) if nn else None

    def kkt_error(self, mu=0.0) -> float:
        """E_mu of the current original-problem iterate."""
        return lib().ipmo_handle_kkt_error(self.h, float(mu))

    def last_soc(self):
        """Second-order corrections of the last pass: list of (c_soc [m], step [n_v], theta of the trial)."""
        k = self.m if self.m > 0 else 1
        nv = self.n + 2 * self.m
        cs = np.zeros((8, k)); ds = np.zeros((8, nv)); th = np.zeros(8)
        cnt = lib().ipmo_last_soc(self.h, _p(cs), _p(ds), _p(th))
        return [(cs[i, :self.m].copy(), ds[i].copy(), th[i]) for i in range(cnt)]

    def outputs(self) -> dict:
        n, m = self.n, self.m
        out = dict(x=np.zeros(n), y=np.zeros(max(m, 1)), zl=np.zeros(n), zu=np.zeros(n), obj=np.zeros(1),
                   kkt=np.zeros(1), status=np.zeros(1, np.int32), iters=np.zeros(1, np.int32),
                   stats=np.zeros(NSTAT, np.int32))
        lib().ipmo_outputs(self.h, _p(out["x"]), _p(out["y"]), _p(out["zl"]), _p(out["zu"]), _p(out["obj"]),
                           _p(out["kkt"]), _ip(out["status"]), _ip(out["iters"]), _ip(out["stats"]))
        out["y"] = out["y"][:m]
        return out


def unpack_state(s: np.ndarray, n: int, m: int) -> dict:
    """Split a flat oracle state into named fields (same order as ipmo_state_get); the filter
    capacity F of the format follows from the length."""
    rest = len(s) - 16 - (8 + 3 * n + m) - (8 + 3 * (n + 2 * m) + m) - 2 * n - (8 + 3 * n + m) - 4 - 8
    assert rest > 0 and rest % 4 == 0, "not a flat state of this problem size"
    fcap = rest // 4
    hdr = s[:16]
    p = 16

    def sub(p, nv):
        d = dict(mu=s[p], tau=s[p + 1], dx_last=s[p + 2], theta_max=s[p + 3], theta_min=s[p + 4],
                 tiny=int(s[p + 5]), nf=int(s[p + 6]))
        p += 8
        d["x"] = s[p:p + nv]; p += nv
        d["y"] = s[p:p + m]; p += m
        d["zl"] = s[p:p + nv]; p += nv
        d["zu"] = s[p:p + nv]; p += nv
        d["fth"] = s[p:p + fcap][:d["nf"]]; p += fcap
        d["fph"] = s[p:p + fcap][:d["nf"]]; p += fcap
        return d, p

    main, p = sub(p, n)
    rs, p = sub(p, n + 2 * m)
    xR, DR2 = s[p:p + n], s[p + n:p + 2 * n]
    p += 2 * n
    wd = dict(short=int(s[p]), active=int(s[p + 1]), iter=int(s[p + 2]), theta=s[p + 3], phi=s[p + 4],
              gphi=s[p + 5], alpha_max=s[p + 6], mu=s[p + 7])
    p += 8
    wd["x"] = s[p:p + n]; p += n
    wd["y"] = s[p:p + m]; p += m
    wd["zl"] = s[p:p + n]; p += n
    wd["zu"] = s[p:p + n]
    p += n
    soft = dict(active=int(s[p]), iter=int(s[p + 1]), theta=s[p + 2], phi=s[p + 3])
    p += 4
    adapt = dict(free=int(s[p]), n_refs=int(s[p + 1]), refs=s[p + 2:p + 2 + int(s[p + 1])], mu_max=s[p + 6])
    return dict(phase=int(hdr[0]), iter=int(hdr[1]), status=int(hdr[2]), init_filter=int(hdr[3]),
                theta_R=hdr[4], warm=int(hdr[5]), wstage=int(hdr[6]), main=main, resto=rs, xR=xR, DR2=DR2,
                watchdog=wd, soft=soft, adaptive=adapt)
