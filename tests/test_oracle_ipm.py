"""Pins for the oracle's interior-point method (Sec. IV, Table I) against closed forms,
brute force and optimality invariants, independent of the oracle's own arithmetic."""
import numpy as np
import pytest

import oracle
from paper_2606_26341_amd import workloads as W

INF = np.inf


def solve_generic(n, m, xl, xu, f, g, c, J, H, x0, **opts):
    h = oracle.Handle.generic(n, m, np.asarray(xl, float), np.asarray(xu, float), f, g, c, J, H,
                              np.asarray(x0, float), oracle.default_opts(**opts))
    h.run()
    return h, h.outputs()


# ------------------------------------------------------------------- convex closed forms
@pytest.mark.parametrize("seed", range(4))
def test_equality_qp_matches_closed_form_kkt_solve(seed):
    rng = np.random.default_rng([31, seed])
    n, m = 7, 3
    Mq = rng.normal(size=(n, n))
    Hq = Mq @ Mq.T + 0.5 * np.eye(n)
    gq = rng.normal(size=n)
    A = rng.normal(size=(m, n))
    b = rng.normal(size=m)
    h, out = solve_generic(n, m, np.full(n, -INF), np.full(n, INF),
                           lambda x: 0.5 * x @ Hq @ x + gq @ x, lambda x: Hq @ x + gq,
                           lambda x: A @ x - b, lambda x: A, lambda x, of, y: of * Hq, np.zeros(n))
    K = np.block([[Hq, A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-gq, b]))
    assert h.status == oracle.ST_CONVERGED
    assert np.allclose(out["x"], sol[:n], atol=1e-9)
    assert np.allclose(out["y"], sol[n:], atol=1e-8)


@pytest.mark.parametrize("seed", range(4))
def test_separable_box_qp_is_clipped_minimizer(seed):
    rng = np.random.default_rng([32, seed])
    n = 9
    hq = rng.uniform(0.5, 3.0, n)
    gq = rng.normal(scale=3.0, size=n)
    lo = rng.uniform(-2.0, -0.5, n)
    hi = rng.uniform(0.5, 2.0, n)
    h, out = solve_generic(n, 0, lo, hi, lambda x: 0.5 * hq @ (x * x) + gq @ x, lambda x: hq * x + gq,
                           lambda x: np.zeros(0), lambda x: np.zeros((0, n)), lambda x, of, y: of * np.diag(hq),
                           np.zeros(n))
    xs = np.clip(-gq / hq, lo, hi)
    assert h.status == oracle.ST_CONVERGED
    # on an active bound the iterate stays mu/z inside it; E_0 <= 1e-8 bounds that by ~1e-8/z*
    r = hq * xs + gq
    zstar = np.where(np.abs(r) > 0, np.abs(r), 1.0)
    assert np.all(np.abs(out["x"] - xs) <= 1e-7 + 1e-7 / zstar)
    # multipliers: z_L - z_U = h x* + g with the active side carrying the multiplier
    assert np.allclose(out["zl"] - out["zu"], r, atol=1e-6)


def test_lqr_matches_discrete_riccati_recursion():
    rng = np.random.default_rng(33)
    nx, nu, N = 3, 2, 6
    A = np.eye(nx) + 0.1 * rng.normal(size=(nx, nx))
    B = 0.3 * rng.normal(size=(nx, nu))
    Q = np.diag([1.0, 2.0, 0.5])
    R = np.diag([0.3, 0.7])
    Qf = 3.0 * np.eye(nx)
    x0 = np.array([1.0, -2.0, 0.5])
    # textbook backward Riccati recursion
    P = Qf
    Ks = []
    for _ in range(N):
        K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        P = Q + A.T @ P @ (A - B @ K)
        Ks.append(K)
    Ks = Ks[::-1]
    xs, us = [x0], []
    for k in range(N):
        us.append(-Ks[k] @ xs[-1])
        xs.append(A @ xs[-1] + B @ us[-1])
    # NLP over v = (x0, u0, x1, u1, ..., xN) with x0 - xbar0 = 0 and x_{k+1} - A x_k - B u_k = 0
    s = nx + nu
    n = N * s + nx
    m = (N + 1) * nx
    Hm = np.zeros((n, n))
    for k in range(N + 1):
        Hm[k * s:k * s + nx, k * s:k * s + nx] = Qf if k == N else Q
        if k < N:
            Hm[k * s + nx:(k + 1) * s, k * s + nx:(k + 1) * s] = R
    Jc = np.zeros((m, n))
    Jc[:nx, :nx] = np.eye(nx)
    for k in range(N):
        r = (k + 1) * nx
        Jc[r:r + nx, (k + 1) * s:(k + 1) * s + nx] = np.eye(nx)
        Jc[r:r + nx, k * s:k * s + nx] = -A
        Jc[r:r + nx, k * s + nx:(k + 1) * s] = -B
    rhs = np.zeros(m)
    rhs[:nx] = x0
    h, out = solve_generic(n, m, np.full(n, -INF), np.full(n, INF), lambda v: 0.5 * v @ Hm @ v, lambda v: Hm @ v,
                           lambda v: Jc @ v - rhs, lambda v: Jc, lambda v, of, y: of * Hm, np.zeros(n))
    v = out["x"]
    assert h.status == oracle.ST_CONVERGED
    for k in range(N):
        assert np.allclose(v[k * s:k * s + nx], xs[k], atol=1e-9)
        assert np.allclose(v[k * s + nx:(k + 1) * s], us[k], atol=1e-9)
    assert np.allclose(v[N * s:], xs[N], atol=1e-9)


# ------------------------------------------------------------------- nonconvex, brute force
def test_1d_nonconvex_matches_grid():
    f = lambda x: x[0] ** 4 - 3 * x[0] ** 3 + 2
    h, out = solve_generic(1, 0, [-1.0], [4.0], f, lambda x: np.array([4 * x[0] ** 3 - 9 * x[0] ** 2]),
                           lambda x: np.zeros(0), lambda x: np.zeros((0, 1)),
                           lambda x, of, y: np.array([[of * (12 * x[0] ** 2 - 18 * x[0])]]), [1.0])
    grid = np.linspace(-1.0, 4.0, 2_000_001)
    fg = grid ** 4 - 3 * grid ** 3 + 2
    assert h.status == oracle.ST_CONVERGED
    assert abs(out["obj"][0] - fg.min()) <= 1e-6
    assert abs(out["x"][0] - grid[fg.argmin()]) <= 1e-5


def test_2d_inequalities_via_slacks_match_grid():
    # min (x-2)^2 + (y-1)^2  s.t. x^2 - y <= 0, x + y <= 2  (slacks s1, s2 >= 0)
    f = lambda v: (v[0] - 2) ** 2 + (v[1] - 1) ** 2
    g = lambda v: np.array([2 * (v[0] - 2), 2 * (v[1] - 1), 0, 0])
    c = lambda v: np.array([v[0] ** 2 - v[1] + v[2], v[0] + v[1] + v[3] - 2])
    J = lambda v: np.array([[2 * v[0], -1, 1, 0], [1, 1, 0, 1.0]])

    def H(v, of, y):
        M = np.zeros((4, 4))
        M[0, 0] = 2 * of + 2 * y[0]
        M[1, 1] = 2 * of
        return M

    h, out = solve_generic(4, 2, [-INF, -INF, 0, 0], [INF] * 4, f, g, c, J, H, [0.0, 0.0, 1.0, 1.0])
    X, Y = np.meshgrid(np.linspace(-2, 3, 1501), np.linspace(-2, 3, 1501))
    feas = (X ** 2 - Y <= 0) & (X + Y <= 2)
    fg = np.where(feas, (X - 2) ** 2 + (Y - 1) ** 2, np.inf)
    assert h.status == oracle.ST_CONVERGED
    assert out["obj"][0] <= fg.min() + 1e-7           # no feasible grid point is better (up to mu-interiority)
    assert fg.min() - out["obj"][0] <= 1e-2           # and the grid resolution bounds the gap
    assert np.allclose(out["x"][:2], [1.0, 1.0], atol=1e-7)


def test_equality_circle_reaches_minimum():
    # min x + y s.t. x^2 + y^2 = 2: minimum (-1, -1), f = -2 (the other stationary point is a maximum)
    h, out = solve_generic(2, 1, [-INF, -INF], [INF, INF], lambda v: v[0] + v[1], lambda v: np.ones(2),
                           lambda v: np.array([v @ v - 2]), lambda v: 2 * v[None, :],
                           lambda v, of, y: 2 * y[0] * np.eye(2), [0.3, -0.8])
    th = np.linspace(0, 2 * np.pi, 2_000_001)
    fg = np.sqrt(2) * (np.cos(th) + np.sin(th))
    assert h.status == oracle.ST_CONVERGED
    assert abs(out["obj"][0] - fg.min()) <= 1e-6
    assert np.allclose(out["x"], [-1, -1], atol=1e-7)


# ------------------------------------------------------------------- algorithm pieces
def test_inertia_correction_sequence_on_negative_curvature():
    # W = -I with far bounds: delta_x goes 0 -> 1e-4 -> 1e-2 -> 1 (x100 steps from delta_0 while no
    # earlier value exists) and the next iteration restarts from 1/3 and grows by 8
    n = 2
    h = oracle.Handle.generic(n, 0, np.full(n, -1e4), np.full(n, 1e4), lambda x: -0.5 * x @ x, lambda x: -x,
                              lambda x: np.zeros(0), lambda x: np.zeros((0, n)), lambda x, of, y: -of * np.eye(n),
                              np.array([0.5, -0.25]))
    h.step()           # least-squares multipliers
    h.step()
    d1 = h.last_info()["delta_x"]
    assert d1 == pytest.approx(1.0, rel=0, abs=0)
    h.step()
    d2 = h.last_info()["delta_x"]
    k = np.log(d2 / (1.0 / 3.0)) / np.log(8.0)
    assert abs(k - round(k)) < 1e-12 and round(k) >= 0


def test_newton_step_solves_full_system_6():
    # after a regular pass without perturbation, (dx, dy, dz_L, dz_U) solves eq. (6) at the old point
    rng = np.random.default_rng(34)
    n, m = 5, 2
    Mq = rng.normal(size=(n, n))
    Hq = Mq @ Mq.T + np.eye(n)
    gq = rng.normal(size=n)
    A = rng.normal(size=(m, n))
    b = rng.normal(size=m) * 0.1
    lo = np.array([-1.0, -INF, -2.0, -INF, -0.5])
    hi = np.array([1.0, 2.0, INF, INF, 0.5])
    f = lambda x: 0.5 * x @ Hq @ x + gq @ x + 0.1 * np.sum(x ** 4)
    g = lambda x: Hq @ x + gq + 0.4 * x ** 3
    Hf = lambda x, of, y: of * (Hq + np.diag(1.2 * x ** 2))
    h = oracle.Handle.generic(n, m, lo, hi, f, g, lambda x: A @ x - b, lambda x: A, Hf, np.zeros(n))
    h.step()
    for _ in range(3):
        st = oracle.unpack_state(h.state(), n, m)["main"]
        x, y, zl, zu = st["x"].copy(), st["y"].copy(), st["zl"].copy(), st["zu"].copy()
        h.step()
        info = h.last_info()
        assert info["delta_x"] == 0.0 and info["delta_c"] == 0.0
        mu = info["mu"]
        dx, dy, dzl, dzu = h.last_step()
        L = np.isfinite(lo)
        U = np.isfinite(hi)
        r1 = Hf(x, 1.0, y) @ dx + A.T @ dy - dzl + dzu + (g(x) + A.T @ y - zl + zu)
        r2 = A @ dx + (A @ x - b)
        r3 = (zl * dx + (x - lo) * dzl + ((x - lo) * zl - mu))[L]
        r4 = (-zu * dx + (hi - x) * dzu + ((hi - x) * zu - mu))[U]
        for r in (r1, r2, r3, r4):
            assert np.abs(r).max() <= 1e-10


def test_restoration_initial_point_closed_form():
    # infeasible c(x) = x^2 + 1: the line search fails and restoration starts with p - n = c(x_R),
    # z_p p = z_n n = mu_R and the first-order condition 2 rho = mu_R / p + mu_R / n of the elastic terms
    h = oracle.Handle.generic(1, 1, np.array([-INF]), np.array([INF]), lambda x: x[0] ** 2, lambda x: 2 * x,
                              lambda x: np.array([x[0] ** 2 + 1]), lambda x: np.array([[2 * x[0]]]),
                              lambda x, of, y: np.array([[2 * of + 2 * y[0]]]), np.array([1.0]))
    seen = False
    for _ in range(60):
        ph = h.phase
        h.step()
        if ph == oracle.PH_REGULAR and h.phase == oracle.PH_RESTO:
            st = oracle.unpack_state(h.state(), 1, 1)
            xr = st["resto"]["x"]
            x, p, nn = xr[0], xr[1], xr[2]
            cR = x ** 2 + 1
            muR = st["resto"]["mu"]
            rho = oracle.default_opts().rho_resto
            assert abs((p - nn) - cR) <= 1e-12 * max(1, cR)
            assert abs(st["resto"]["zl"][1] * p - muR) <= 1e-12 * muR
            assert abs(st["resto"]["zl"][2] * nn - muR) <= 1e-12 * muR
            assert abs(muR / p + muR / nn - 2 * rho) <= 1e-9 * rho
            assert muR == pytest.approx(max(st["main"]["mu"], cR), rel=1e-15)
            seen = True
            break
    assert seen
    h.run()
    assert h.status == oracle.ST_INFEASIBLE
    assert abs(h.outputs()["x"][0]) <= 1e-6


def test_state_save_load_replays_bitwise():
    w = W.get("C1")
    th = w.theta(3)
    h = oracle.Handle.quad(w, th)
    for _ in range(4):
        h.step()
    s = h.state()
    h.step()
    s_next = h.state()
    h2 = oracle.Handle.quad(w, th)
    h2.set_state(s)
    h2.step()
    assert np.array_equal(h2.state(), s_next)


# ------------------------------------------------------------------- quadrotor NMPC invariants
def _reduced_kkt_inertia(w, th, out):
    f, g, c, J, H = oracle.quad_eval(w, th, out["x"], out["y"])
    n, m = w.n, w.m
    lo = np.full(n, -INF)
    hi = np.full(n, INF)
    uh = w.model.u_hover
    for k in range(w.N):
        lo[k * (w.nx + w.nu) + w.nx:(k + 1) * (w.nx + w.nu)] = 0.0
        hi[k * (w.nx + w.nu) + w.nx:(k + 1) * (w.nx + w.nu)] = 2 * uh
    lo[w.n_w:] = 0.0
    sig = np.zeros(n)
    L, U = np.isfinite(lo), np.isfinite(hi)
    sig[L] += out["zl"][L] / (out["x"][L] - lo[L])
    sig[U] += out["zu"][U] / (hi[U] - out["x"][U])
    K = np.block([[H + np.diag(sig), J.T], [J, np.zeros((m, m))]])
    ev = np.linalg.eigvalsh(K)
    return int((ev > 0).sum()), int((ev < 0).sum()), lo, hi


@pytest.mark.parametrize("i", range(6))
def test_c1_solution_satisfies_kkt_invariants(i):
    w = W.get("C1")
    th = w.theta(i)
    out = oracle.solve_quad(w, th[None, :])
    out = {k: v[0] for k, v in out.items()}
    assert out["status"] == oracle.ST_CONVERGED
    assert out["kkt"] <= 1e-8
    npos, nneg, lo, hi = _reduced_kkt_inertia(w, th, out)
    assert (npos, nneg) == (w.n, w.m)
    L, U = np.isfinite(lo), np.isfinite(hi)
    assert np.all(out["x"][L] > lo[L]) and np.all(out["x"][U] < hi[U])
    assert np.all(out["zl"][L] > 0) and np.all(out["zu"][U] > 0)
    # the recomputed error agrees with the reported one
    assert oracle.kkt_error(w, th, out["x"], out["y"], out["zl"], out["zu"]) == pytest.approx(out["kkt"], rel=1e-12)


def test_start_inside_obstacle_is_reported_infeasible():
    w = W.get("C1")
    th = w.theta(0).copy()
    th[16:19] = th[0:3]          # obstacle 0 centred on the start, radius 0.5: x_1 cannot leave it
    th[19] = 0.5
    out = oracle.solve_quad(w, th[None, :])
    assert out["status"][0] in (oracle.ST_INFEASIBLE, oracle.ST_RESTO_FAILED)
