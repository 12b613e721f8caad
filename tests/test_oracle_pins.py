"""Hand-computed pins of the oracle's method pieces (Sec. IV, Table I; constants and sub-rules as
the IPOPT paper publishes them): the scaled KKT error, fraction to the boundary, filter /
switching / Armijo acceptance, the smallest step size, the monotone barrier sequence, the bound
push and least-squares multipliers of the initialisation, the kappa_Sigma safeguard, the
second-order correction and the restoration exit.  Every expected value below is written out
from a hand computation (shown in the comments) or from a library routine (numpy's least
squares / dense solve), never from the oracle itself."""
import numpy as np
import pytest

import oracle
from paper_2606_26341_amd import workloads as W

from helpers import hover_at_target_workload

INF = np.inf


def _generic(n, m, xl, xu, f, g, c, J, H, x0, **opts):
    return oracle.Handle.generic(n, m, np.asarray(xl, float), np.asarray(xu, float), f, g, c, J, H,
                                 np.asarray(x0, float), oracle.default_opts(**opts))


def _set_main(h, x, y, zl, zu):
    """Put (x, y, z_L, z_U) into the handle's original-problem iterate."""
    s = h.state()
    n, m = h.n, h.m
    p = 16 + 8
    s[p:p + n] = x; p += n
    s[p:p + m] = y; p += m
    s[p:p + n] = zl; p += n
    s[p:p + n] = zu
    h.set_state(s)


# ------------------------------------------------------------------------ scaled KKT error
# n = 3, m = 2: f = 3 x0 - 2 x1 + x2, c = (x0 + x1 + x2 - 5, x0 - x1), bounds 0 <= x0 <= 4,
# x1 >= 1, x2 free: n_L = 2, n_U = 1, s_max = 100.
_F = lambda x: 3 * x[0] - 2 * x[1] + x[2]
_G = lambda x: np.array([3.0, -2.0, 1.0])
_C = lambda x: np.array([x[0] + x[1] + x[2] - 5, x[0] - x[1]])
_J = lambda x: np.array([[1.0, 1.0, 1.0], [1.0, -1.0, 0.0]])
_H = lambda x, of, y: np.zeros((3, 3))


def _kkt_handle():
    return _generic(3, 2, [0.0, 1.0, -INF], [4.0, INF, INF], _F, _G, _C, _J, _H, [1.0, 3.0, 2.0])


def test_scaled_kkt_error_hand_computed_dual_and_complementarity_scaling():
    # point A: x = (1, 3, 2), y = (850, 0), z_L = (300, 150, 0), z_U = (100, 0, 0)
    #   c = (1, -2)                                 -> |c|_inf = 2
    #   grad f + J^T y - z_L + z_U = (3 + 850 - 300 + 100, -2 + 850 - 150, 1 + 850) = (653, 698, 851)
    #   s_d = max(100, (|y|_1 + |z|_1) / (m + n_L + n_U)) / 100 = max(100, (850 + 550) / 5) / 100 = 2.8
    #   s_c = max(100, |z|_1 / (n_L + n_U)) / 100 = max(100, 550 / 3) / 100 = 1.8333...
    #   complementarity products: (1 - 0) 300 = 300, (4 - 1) 100 = 300, (3 - 1) 150 = 300
    h = _kkt_handle()
    _set_main(h, [1.0, 3.0, 2.0], [850.0, 0.0], [300.0, 150.0, 0.0], [100.0, 0.0, 0.0])
    # mu = 300: complementarity 0, E = 851 / 2.8
    assert h.kkt_error(300.0) == pytest.approx(303.92857142857144, rel=1e-14)
    # mu = 0: max(851 / 2.8, 2, 300 / 1.8333) = 303.93 (dual term)
    assert h.kkt_error(0.0) == pytest.approx(303.92857142857144, rel=1e-14)
    # mu = 1000: complementarity |300 - 1000| / 1.8333 = 381.81... dominates
    assert h.kkt_error(1000.0) == pytest.approx(381.8181818181818, rel=1e-14)


def test_scaled_kkt_error_hand_computed_primal_term_and_unit_scaling():
    # point C: x = (1, 3, 8), y = 0, z_L = (1, 0.5, 0), z_U = (1/3, 0, 0)
    #   c = (7, -2): |c|_inf = 7 (|c|_1 would be 9)
    #   dual residual (3 - 1 + 1/3, -2 - 0.5, 1) -> 2.5; s_d = s_c = 1 (the means are below s_max)
    #   complementarity products 1, 1, 1
    h = _kkt_handle()
    _set_main(h, [1.0, 3.0, 8.0], [0.0, 0.0], [1.0, 0.5, 0.0], [1.0 / 3.0, 0.0, 0.0])
    assert h.kkt_error(0.0) == pytest.approx(7.0, rel=1e-15)
    # mu = 9: |1 - 9| = 8 > 7
    assert h.kkt_error(9.0) == pytest.approx(8.0, rel=1e-15)


# ------------------------------------------------------------------------ fraction to the boundary
def test_fraction_to_boundary_primal_hand_computed():
    xl = [0.0, 1.0, -INF, -INF]
    xu = [1.0, INF, 3.0, INF]
    x = [0.5, 2.0, 1.0, 0.0]
    dx = [-1.0, -4.0, 4.0, -1e9]          # the free last component never limits the step
    # candidates: 0.99 * 0.5 / 1 = 0.495, 0.99 * (2 - 1) / 4 = 0.2475, 0.99 * (3 - 1) / 4 = 0.495
    assert oracle.ftb_primal(x, dx, xl, xu, 0.99) == pytest.approx(0.2475, rel=1e-15)
    # moving away from every bound: the full step
    assert oracle.ftb_primal(x, [1e-3, 5.0, -7.0, 1e9], xl, xu, 0.99) == 1.0
    # the upper bound of the first component: 0.9 * (1 - 0.5) / 2 = 0.225
    assert oracle.ftb_primal(x, [2.0, 0.0, 0.0, 0.0], xl, xu, 0.9) == pytest.approx(0.225, rel=1e-15)


def test_fraction_to_boundary_dual_hand_computed():
    xl = [0.0, 1.0, -INF]
    xu = [1.0, INF, 3.0]
    zl, zu = [2.0, 1.0, 0.0], [1.0, 0.0, 1.0]
    dzl = [-4.0, 1.0, -100.0]              # component 2 has no lower bound: ignored
    dzu = [-0.5, -9.0, -0.25]              # component 1 has no upper bound: ignored
    # candidates: 0.99 * 2 / 4 = 0.495, 0.99 * 1 / 0.5 = 1.98, 0.99 * 1 / 0.25 = 3.96 -> 0.495
    assert oracle.ftb_dual(zl, zu, dzl, dzu, xl, xu, 0.99) == pytest.approx(0.495, rel=1e-15)


# ------------------------------------------------------------------------ filter line search tests
# round constants so that the powers can be taken by hand: s_theta = 2, s_phi = 3, delta = 1,
# eta_phi = 0.1, gamma_theta = 0.1, gamma_phi = 0.2, gamma_alpha = 0.5
_LS = dict(delta_sw=1.0, s_theta=2.0, s_phi=3.0, eta_phi=0.1, gamma_theta=0.1, gamma_phi=0.2, gamma_alpha=0.5)


def _acc(thk, phk, gphi, alpha, tht, pht, filt=(), thmax=100.0, thmin=0.5):
    return oracle.acceptable(thmax, thmin, list(filt), thk, phk, gphi, alpha, tht, pht,
                             opts=oracle.default_opts(**_LS))


def test_switching_condition_and_armijo_hand_table():
    # theta_k = 0.4 <= theta_min, grad phi^T d = -2, alpha = 1:
    #   switching: 1 * 2^3 = 8 > 1 * 0.4^2 = 0.16 -> holds, so only Armijo decides:
    #   phi <= 10 + 0.1 * 1 * (-2) = 9.8
    assert _acc(0.4, 10.0, -2.0, 1.0, 0.3, 9.79) == (True, 1, 1)
    assert _acc(0.4, 10.0, -2.0, 1.0, 0.0, 9.81)[0] is False     # theta decrease does not help
    # theta_k = 0.6 > theta_min: sufficient decrease in theta or phi
    #   theta <= 0.9 * 0.6 = 0.54  or  phi <= 10 - 0.2 * 0.6 = 9.88
    assert _acc(0.6, 10.0, -2.0, 1.0, 0.55, 9.89)[0] is False
    assert _acc(0.6, 10.0, -2.0, 1.0, 0.53, 11.0)[0] is True
    ok, sw, arm = _acc(0.6, 10.0, -2.0, 1.0, 0.7, 9.87)
    assert ok and sw == 1 and arm == 0
    # switching fails: alpha = 0.5, grad phi^T d = -0.5: 0.5 * 0.125 = 0.0625 > 0.16 is false
    #   -> theta <= 0.36 or phi <= 10 - 0.08 = 9.92 (with s_theta and s_phi swapped it would hold:
    #   0.5 * 0.25 = 0.125 > 0.064, and the Armijo test would reject (0.35, 50))
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.35, 50.0) == (True, 0, 0)
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.37, 9.93)[0] is False
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.37, 9.91)[0] is True
    # an ascent direction never switches
    assert _acc(0.4, 10.0, 0.0, 1.0, 0.35, 50.0)[1] == 0


def test_filter_and_theta_max_hand_table():
    # theta_max: a trial above it is rejected whatever its phi
    assert _acc(0.6, 10.0, -2.0, 1.0, 150.0, -1e6)[0] is False
    # filter entry (0.3, 9.0): (0.35, 9.5) is dominated (0.35 >= 0.3, 9.5 >= 9.0), (0.29, 9.5) is not,
    # and (0.35, 8.9) is not
    f = [(0.3, 9.0)]
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.35, 9.5, filt=f)[0] is False
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.29, 9.5, filt=f)[0] is True
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.35, 8.9, filt=f)[0] is True
    # two entries: rejected if either dominates
    assert _acc(0.4, 10.0, -0.5, 0.5, 0.2, 9.5, filt=[(0.3, 9.0), (0.1, 9.4)])[0] is False


def test_alpha_min_hand_table():
    o = oracle.default_opts(**_LS)
    # descent, theta_k > theta_min: 0.5 * min(0.1, 0.2 * 0.6 / 2) = 0.5 * 0.06 = 0.03
    assert oracle.alpha_min(0.6, -2.0, 0.5, o) == pytest.approx(0.03, rel=1e-15)
    # descent, theta_k <= theta_min: 0.5 * min(0.1, 0.2 * 0.4 / 2, 0.4^2 / 2^3) = 0.5 * 0.02 = 0.01
    assert oracle.alpha_min(0.4, -2.0, 0.5, o) == pytest.approx(0.01, rel=1e-15)
    # gamma_theta is the least term: 0.5 * min(0.1, 0.2 * 0.6 / 0.5 = 0.24) = 0.05
    assert oracle.alpha_min(0.6, -0.5, 0.5, o) == pytest.approx(0.05, rel=1e-15)
    # no descent: gamma_alpha * gamma_theta = 0.05
    assert oracle.alpha_min(0.6, 0.3, 0.5, o) == pytest.approx(0.05, rel=1e-15)


# ------------------------------------------------------------------------ monotone barrier update
def test_monotone_barrier_sequence():
    # min 1/2 |x|^2 on the box [-1, 1]^2 from x = 0: the barrier problem is nearly solved at once,
    # so mu runs through mu <- max(tol / 10, min(0.2 mu, mu^1.5)):
    #   0.1 -> min(0.02, 0.0316) = 0.02 -> min(0.004, 0.02^1.5 = 0.0028284) -> min(5.66e-4, 1.5042e-4)
    #   -> min(3.01e-5, 1.8449e-6) -> min(3.69e-7, 2.5059e-9) -> max(1e-9, ...) = 1e-9
    want = [0.1, 0.02, 0.002828427124746191, 0.00015042412372345582, 1.8449144625279508e-06,
            2.5059035596800618e-09, 1e-09]
    h = _generic(2, 0, [-1.0, -1.0], [1.0, 1.0], lambda x: 0.5 * x @ x, lambda x: x.copy(),
                 lambda x: np.zeros(0), lambda x: np.zeros((0, 2)), lambda x, of, y: of * np.eye(2), [0.0, 0.0])
    seen = [oracle.unpack_state(h.state(), 2, 0)["main"]["mu"]]
    while h.phase != oracle.PH_DONE:
        h.step()
        st = oracle.unpack_state(h.state(), 2, 0)["main"]
        if st["mu"] != seen[-1]:
            seen.append(st["mu"])
        assert st["tau"] == pytest.approx(max(0.99, 1.0 - st["mu"]), rel=1e-15)
    assert h.status == oracle.ST_CONVERGED
    # several decreases may happen in one pass: the values seen between passes are an ordered
    # subsequence of the chain
    j = 0
    for mu in seen:
        while j < len(want) and abs(mu - want[j]) > 1e-13 * want[j]:
            j += 1
        assert j < len(want), (mu, seen)
    assert len(seen) >= 4 and seen[-1] <= want[4]


def test_tau_follows_mu_when_mu_is_small():
    # mu_0 = 1e-3: tau = max(0.99, 1 - 1e-3) = 0.999 at the start
    h = _generic(1, 0, [-1.0], [1.0], lambda x: 0.5 * x @ x, lambda x: x.copy(), lambda x: np.zeros(0),
                 lambda x: np.zeros((0, 1)), lambda x, of, y: of * np.eye(1), [0.3], mu_init=1e-3)
    assert oracle.unpack_state(h.state(), 1, 0)["main"]["tau"] == 0.999


# ------------------------------------------------------------------------ initialisation
def test_bound_push_closed_forms():
    # kappa_1 = kappa_2 = 1e-2:
    #   [0, 1],   x0 = -5    -> 0 + min(0.01 * 1, 0.01 * 1)        = 0.01
    #   [0, 0.5], x0 = -5    -> 0 + min(0.01, 0.01 * 0.5)           = 0.005
    #   [0, 0.5], x0 = 7     -> 0.5 - min(0.01 * 1, 0.005)          = 0.495
    #   [100, inf), x0 = 0   -> 100 + 0.01 * 100                    = 101
    #   (-inf, -200], x0 = 0 -> -200 - 0.01 * 200                   = -202
    #   [-3, 3],  x0 = 1     -> unchanged                            = 1
    #   [2, 1000], x0 = 2.001 -> 2 + min(0.01 * 2, 0.01 * 998)      = 2.02
    #   free,      x0 = -7   -> -7
    xl = [0.0, 0.0, 0.0, 100.0, -INF, -3.0, 2.0, -INF]
    xu = [1.0, 0.5, 0.5, INF, -200.0, 3.0, 1000.0, INF]
    x0 = [-5.0, -5.0, 7.0, 0.0, 0.0, 1.0, 2.001, -7.0]
    n = 8
    h = _generic(n, 0, xl, xu, lambda x: 0.0, lambda x: np.zeros(n), lambda x: np.zeros(0),
                 lambda x: np.zeros((0, n)), lambda x, of, y: np.zeros((n, n)), x0)
    st = oracle.unpack_state(h.state(), n, 0)["main"]
    assert st["x"] == pytest.approx([0.01, 0.005, 0.495, 101.0, -202.0, 1.0, 2.02, -7.0], rel=1e-15)
    assert list(st["zl"]) == [1, 1, 1, 1, 0, 1, 1, 0] and list(st["zu"]) == [1, 1, 1, 0, 1, 1, 1, 0]
    assert st["mu"] == 0.1 and st["tau"] == 0.99


def test_least_squares_multipliers_and_filter_bounds():
    # [[I, A^T], [A, 0]] [d; y] = -[grad f - z_L + z_U; 0]  <=>  y = argmin |grad f - z_L + z_U + A^T y|
    rng = np.random.default_rng(7)
    n, m = 6, 2
    A = rng.normal(size=(m, n))
    b = rng.normal(size=m)
    gq = rng.normal(size=n)
    xl = [0.0, -INF, -INF, -1.0, -INF, -INF]
    xu = [INF, INF, 2.0, 1.0, INF, INF]
    x0 = np.array([0.5, 0.3, 0.1, 0.2, -0.4, 0.9])
    h = _generic(n, m, xl, xu, lambda x: gq @ x, lambda x: gq.copy(), lambda x: A @ x - b, lambda x: A,
                 lambda x, of, y: np.zeros((n, n)), x0)
    st0 = oracle.unpack_state(h.state(), n, m)["main"]
    h.step()
    st = oracle.unpack_state(h.state(), n, m)
    r = gq - st0["zl"] + st0["zu"]
    y_ls = np.linalg.lstsq(A.T, -r, rcond=None)[0]
    assert np.abs(st["main"]["y"] - y_ls).max() <= 1e-12 * max(1.0, np.abs(y_ls).max())
    # theta_0 = |A x0 - b|_1; theta_max = 1e4 max(1, theta_0), theta_min = 1e-4 max(1, theta_0)
    th0 = np.abs(A @ st0["x"] - b).sum()
    assert st["main"]["theta_max"] == pytest.approx(1e4 * max(1.0, th0), rel=1e-14)
    assert st["main"]["theta_min"] == pytest.approx(1e-4 * max(1.0, th0), rel=1e-14)
    assert st["phase"] == oracle.PH_REGULAR


def test_least_squares_multipliers_discarded_above_lambda_max():
    # grad f = (1e5, 0) with one row x0 + x1 = 1: y = -1e5 > lambda_max = 1e3 -> y = 0
    h = _generic(2, 1, [-INF, -INF], [INF, INF], lambda x: 1e5 * x[0], lambda x: np.array([1e5, 0.0]),
                 lambda x: np.array([x[0] + x[1] - 1]), lambda x: np.array([[1.0, 1.0]]),
                 lambda x, of, y: np.zeros((2, 2)), [0.0, 0.0])
    h.step()
    assert oracle.unpack_state(h.state(), 2, 1)["main"]["y"][0] == 0.0


# ------------------------------------------------------------------------ kappa_Sigma safeguard
def test_kappa_sigma_keeps_multipliers_near_the_central_path():
    # with kappa_Sigma = 1.5 every accepted z lies in [mu / (1.5 s), 1.5 mu / s]; the safeguard must
    # actually bind on some component for the test to mean anything
    rng = np.random.default_rng(3)
    n = 5
    hq = rng.uniform(0.5, 2.0, n)
    gq = rng.normal(scale=4.0, size=n)
    lo, hi = -np.ones(n), np.ones(n)
    h = _generic(n, 0, lo, hi, lambda x: 0.5 * hq @ (x * x) + gq @ x, lambda x: hq * x + gq, lambda x: np.zeros(0),
                 lambda x: np.zeros((0, n)), lambda x, of, y: of * np.diag(hq), np.zeros(n), kappa_sigma=1.5)
    h.step()
    bound = 0
    while h.phase != oracle.PH_DONE:
        before = oracle.unpack_state(h.state(), n, 0)["main"]
        h.step()
        if h.phase == oracle.PH_DONE:
            break
        info = h.last_info()
        st = oracle.unpack_state(h.state(), n, 0)["main"]
        mu = info["mu"]
        _, _, dzl, dzu = h.last_step()
        for z, z0, dz, s in ((st["zl"], before["zl"], dzl, st["x"] - lo), (st["zu"], before["zu"], dzu, hi - st["x"])):
            assert np.all(z >= mu / (1.5 * s) * (1 - 1e-14)) and np.all(z <= 1.5 * mu / s * (1 + 1e-14))
            raw = z0 + info["alpha_z"] * dz
            bound += int(np.sum(np.abs(raw - z) > 1e-12 * np.abs(z)))
    assert h.status == oracle.ST_CONVERGED
    assert bound > 0


# ------------------------------------------------------------------------ second-order correction
def _maratos(th0):
    # min 2 (x^2 + y^2 - 1) - x  s.t.  x^2 + y^2 - 1 = 0 (the Maratos example): full Newton steps from
    # points of the circle increase the infeasibility, so the first trial is rejected
    f = lambda v: 2 * (v @ v - 1) - v[0]
    g = lambda v: 4 * v - np.array([1.0, 0.0])
    c = lambda v: np.array([v @ v - 1])
    J = lambda v: 2 * v[None, :]
    H = lambda v, of, y: (4 * of + 2 * y[0]) * np.eye(2)
    h = _generic(2, 1, [-INF, -INF], [INF, INF], f, g, c, J, H, [np.cos(th0), np.sin(th0)])
    return h, g, c, J, H


@pytest.mark.parametrize("th0,passes", [(0.5, 1), (1.0, 2)])
def test_second_order_correction_steps(th0, passes):
    h, g, c, J, H = _maratos(th0)
    h.step()                                   # least-squares multipliers
    for _ in range(passes):
        st = oracle.unpack_state(h.state(), 2, 1)["main"]
        x, y = st["x"].copy(), st["y"].copy()
        h.step()
    socs = h.last_soc()
    info = h.last_info()
    dx, dy, _, _ = h.last_step()
    assert socs, "the first trial must be rejected and corrected"
    assert info["delta_x"] == 0.0 and info["delta_c"] == 0.0
    # the KKT matrix of the step, written out: [[W, J^T], [J, 0]], W = (4 + 2 y) I
    K = np.block([[H(x, 1.0, y), J(x).T], [J(x), np.zeros((1, 1))]])
    r = g(x) + J(x).T @ y
    assert np.abs(np.linalg.solve(K, -np.concatenate([r, c(x)]))[:2] - dx).max() <= 1e-12
    # first correction: c_soc = alpha_0 c(x) + c(x + alpha_0 dx) with alpha_0 = 1 (no bounds)
    csoc = c(x) + c(x + dx)
    th_prev = abs(c(x + dx)[0])
    for k, (cs, d, th) in enumerate(socs):
        assert cs == pytest.approx(csoc, rel=1e-13)
        dsoc = np.linalg.solve(K, -np.concatenate([r, csoc]))[:2]
        assert np.abs(d[:2] - dsoc).max() <= 1e-12 * max(1.0, np.abs(dsoc).max())
        assert th == pytest.approx(abs(c(x + dsoc)[0]), rel=1e-12)
        if k > 0:
            assert socs[k - 1][2] <= 0.99 * th_prev      # the correction went on only after a 1 % decrease
        th_prev = socs[k - 1][2] if k > 0 else th_prev
        csoc = 1.0 * csoc + c(x + dsoc)                  # alpha_soc = 1 (no bounds)
    last_th = socs[-1][2]
    if len(socs) < 4 and not info["soc"]:
        # the loop stopped because theta did not fall by kappa_soc = 0.99
        prev = socs[-2][2] if len(socs) > 1 else abs(c(x + dx)[0])
        assert last_th > 0.99 * prev


def test_second_order_correction_stops_at_four():
    h, *_ = _maratos(1.0)
    for _ in range(3):
        h.step()
    assert len(h.last_soc()) == 4


# ------------------------------------------------------------------------ restoration exit
def test_restoration_exit_rule_and_multiplier_reset():
    # c(x) = x^3 - 2 x + 2 from x = 0.8 (near the local minimum of |c|): the line search fails,
    # restoration runs until theta <= 0.9 theta(x_R) at a point the original filter accepts
    f = lambda x: 0.0 * x[0]
    c = lambda x: np.array([x[0] ** 3 - 2 * x[0] + 2])
    h = _generic(1, 1, [-INF], [INF], f, lambda x: np.zeros(1), c, lambda x: np.array([[3 * x[0] ** 2 - 2]]),
                 lambda x, of, y: np.array([[6 * x[0] * y[0]]]), [0.8])
    exits = 0
    for _ in range(200):
        ph = h.phase
        if ph == oracle.PH_DONE:
            break
        before = oracle.unpack_state(h.state(), 1, 1)
        h.step()
        after = oracle.unpack_state(h.state(), 1, 1)
        if ph == oracle.PH_RESTO and after["phase"] == oracle.PH_INIT_Y:
            exits += 1
            x = after["main"]["x"][0]
            th = abs(c([x])[0])
            assert th <= 0.9 * before["theta_R"]
            # acceptable to the original filter: no entry dominates (theta, phi) (f = 0, no bounds)
            for fth, fph in zip(after["main"]["fth"], after["main"]["fph"]):
                assert not (th >= fth and 0.0 >= fph)
            # the restoration's bound multipliers are kept (none here) and the main iterate is its x
            assert x == after["resto"]["x"][0]
        elif ph == oracle.PH_RESTO and after["phase"] == oracle.PH_RESTO:
            x = after["resto"]["x"][0]
            th = abs(c([x])[0])
            dominated = any(th >= a and 0.0 >= b for a, b in zip(after["main"]["fth"], after["main"]["fph"]))
            assert th > 0.9 * after["theta_R"] or dominated
    assert exits == 1
    assert h.status == oracle.ST_CONVERGED


def _resto_exit_problem():
    # c(x1) = x1^3 - 2 x1 + 2 drives the line search into restoration from x1 = 0.7; x2 in [0, 10]
    # is decoupled (objective 1e-3 (x2 - 3)^2) and carries the bound multipliers
    c = lambda x: np.array([x[0] ** 3 - 2 * x[0] + 2])
    return _generic(2, 1, [-INF, 0.0], [INF, 10.0], lambda x: 1e-3 * (x[1] - 3) ** 2,
                    lambda x: np.array([0.0, 2e-3 * (x[1] - 3)]), c, lambda x: np.array([[3 * x[0] ** 2 - 2, 0.0]]),
                    lambda x, of, y: np.array([[6 * x[0] * y[0], 0.0], [0.0, of * 2e-3]]), [0.7, 1.0])


@pytest.mark.parametrize("z_set", [5e4, 5e5])
def test_restoration_exit_keeps_or_resets_bound_multipliers(z_set):
    # on return from restoration the bound multipliers are the restoration's, unless one of them
    # exceeds 1e3, in which case all are reset to 1
    h = _resto_exit_problem()
    k = 0
    while True:
        ph = h.phase
        h.step()
        k += 1
        if ph == oracle.PH_RESTO and h.phase == oracle.PH_INIT_Y:
            break
        assert h.phase != oracle.PH_DONE and k < 200
    h = _resto_exit_problem()
    for _ in range(k - 1):
        h.step()
    assert h.phase == oracle.PH_RESTO
    # raise z_L of x2 in the restoration iterate before the exit pass (the pass divides it by ~100)
    s = h.state()
    n, m = 2, 1
    F = (len(s) - 16 - (8 + 3 * n + m) - (8 + 3 * (n + 2 * m) + m) - 2 * n - (8 + 3 * n + m) - 4 - 8) // 4
    p_rs = 16 + (8 + 3 * n + m + 2 * F) + 8          # the restoration iterate's x
    s[p_rs + (n + 2 * m) + m + 1] = z_set              # its z_L of x2
    h.set_state(s)
    h.step()
    st = oracle.unpack_state(h.state(), 2, 1)
    assert st["phase"] == oracle.PH_INIT_Y
    zr_l, zr_u = st["resto"]["zl"][:2], st["resto"]["zu"][:2]
    if max(zr_l.max(), zr_u.max()) > 1e3:
        assert list(st["main"]["zl"]) == [0.0, 1.0] and list(st["main"]["zu"]) == [0.0, 1.0]
        assert z_set == 5e5
    else:
        assert np.array_equal(st["main"]["zl"], zr_l) and np.array_equal(st["main"]["zu"], zr_u)
        assert z_set == 5e4


# ------------------------------------------------------------------------ warm start (step 14)
def _c1_solution(i=3):
    w = W.get("C1")
    th = w.theta(i)
    o = oracle.solve_quad(w, th[None, :])
    assert o["status"][0] == oracle.ST_CONVERGED
    return w, th, o


def test_warm_start_at_the_solution_converges_at_once():
    # special case: from the method's own solution with mu_0 = 1e-6 it finishes within 3 iterations
    # at the same point
    w, th, o = _c1_solution()
    row = np.concatenate([o["x"][0, :w.n_w], o["y"][0]])
    g = oracle.solve_quad(w, th[None, :], warm=row[None, :], opts=oracle.default_opts(warm_mu0=1e-6))
    assert g["status"][0] == oracle.ST_CONVERGED and g["iters"][0] <= 3
    assert abs(g["obj"][0] - o["obj"][0]) <= 1e-6 * max(1.0, abs(o["obj"][0]))
    assert np.abs(g["x"][0] - o["x"][0]).max() <= 1e-5
    assert g["stats"][0, 8] == 1 and g["stats"][0, 9] == 0


def test_warm_initialisation_push_slacks_and_stationary_multipliers():
    # warm point pushed by warm_push = 1e-3: thrusts into [1e-3, 2 u_h - 1e-3], slacks s = max(g(w), 1e-3);
    # after the INIT_Y pass the bound multipliers satisfy z_L >= mu0 / s_L, z_U >= mu0 / s_U and the
    # stationarity residual grad f + A^T y - z_L + z_U is at most mu0 / s on each bounded component
    w, th, o = _c1_solution()
    row = np.concatenate([o["x"][0, :w.n_w], o["y"][0]])
    row[w.nx: w.nx + 2] = [-1.0, 99.0]               # u_0 outside its bounds
    mu0 = 1e-3
    h = oracle.Handle.quad(w, th, warm_row=row, opts=oracle.default_opts(warm_gate=0, warm_mu0=mu0))
    st = oracle.unpack_state(h.state(), w.n, w.m)
    uh = w.model.u_hover
    x = st["main"]["x"]
    # lower: 0 + min(1e-3 max(1, 0), 1e-3 (2 u_h - 0)) = 1e-3; upper: 2 u_h - min(1e-3 max(1, 2 u_h),
    # 1e-3 (2 u_h)) = 4.905 - 0.004905 = 4.900095
    assert x[w.nx] == 1e-3 and x[w.nx + 1] == pytest.approx(4.900095, rel=1e-15)
    f, g, c, J, _ = oracle.quad_eval(w, th, np.concatenate([row[:w.n_w], np.zeros(w.n_s)]))
    gw = c[(w.N + 1) * w.nx:] + 0.0                   # g(w) - 0 on the slack rows
    assert np.allclose(x[w.n_w:], np.maximum(gw, 1e-3), rtol=0, atol=1e-15)
    assert st["main"]["mu"] == mu0 and np.array_equal(st["main"]["y"], row[w.n_w:])
    h.step()
    st = oracle.unpack_state(h.state(), w.n, w.m)
    assert st["phase"] == oracle.PH_REGULAR
    z_l, z_u = st["main"]["zl"], st["main"]["zu"]
    _, g, _, J, _ = oracle.quad_eval(w, th, x, st["main"]["y"])
    r = g + J.T @ st["main"]["y"]
    lo = np.full(w.n, -INF)
    hi = np.full(w.n, INF)
    for k in range(w.N):
        lo[k * 17 + 13:k * 17 + 17] = 0.0
        hi[k * 17 + 13:k * 17 + 17] = 2 * uh
    lo[w.n_w:] = 0.0
    L, U = np.isfinite(lo), np.isfinite(hi)
    assert np.all(z_l[L] >= mu0 / (x[L] - lo[L]) * (1 - 1e-15))
    assert np.all(z_u[U] >= mu0 / (hi[U] - x[U]) * (1 - 1e-15))
    floor = np.where(L, mu0 / np.where(L, x - lo, 1.0), 0.0) + np.where(U, mu0 / np.where(U, hi - x, 1.0), 0.0)
    res = np.abs(r - z_l + z_u)
    assert np.all(res[L | U] <= floor[L | U] * (1 + 1e-12))


def test_warm_gate_rejects_a_worse_point_and_keeps_the_cold_start():
    # a warm point far worse than the cold start (E_mu0 larger) is rejected: after its two INIT_Y passes
    # the iterate is bit for bit the cold start after its single INIT_Y pass
    w, th, o = _c1_solution()
    bad = np.concatenate([o["x"][0, :w.n_w], o["y"][0]]) + 40.0
    hc = oracle.Handle.quad(w, th)
    hc.step()
    hw = oracle.Handle.quad(w, th, warm_row=bad)
    hw.step()
    assert hw.phase == oracle.PH_INIT_Y
    hw.step()
    sc = oracle.unpack_state(hc.state(), w.n, w.m)
    sw = oracle.unpack_state(hw.state(), w.n, w.m)
    assert sw["phase"] == oracle.PH_REGULAR and sw["warm"] == 0
    for k in ("x", "y", "zl", "zu", "mu", "tau", "theta_max", "theta_min"):
        assert np.array_equal(np.asarray(sc["main"][k]), np.asarray(sw["main"][k])), k
    # and the good one is kept
    good = np.concatenate([o["x"][0, :w.n_w], o["y"][0]])
    hg = oracle.Handle.quad(w, th, warm_row=good)
    hg.step()
    hg.step()
    sg = oracle.unpack_state(hg.state(), w.n, w.m)
    assert sg["warm"] == 1 and sg["main"]["mu"] == oracle.default_opts().warm_mu0


def test_warm_divergence_restarts_cold_and_keeps_counting():
    # a warm start still running after warm_iter_cap = 2 iterations restarts from the cold start: the
    # result is the cold solve's, bit for bit, after two more iterations
    w = W.get("C1")
    th = w.theta(5)
    cold = oracle.solve_quad(w, th[None, :])
    w3, th3, o3 = _c1_solution(6)                      # another instance's solution as a poor warm point
    row = np.concatenate([o3["x"][0, :w.n_w], o3["y"][0]])
    opts = oracle.default_opts(warm_gate=0, warm_iter_cap=2)
    g = oracle.solve_quad(w, th[None, :], warm=row[None, :], opts=opts)
    assert g["stats"][0, 10] == 1
    assert g["iters"][0] == cold["iters"][0] + 2
    assert np.array_equal(g["x"], cold["x"]) and g["status"][0] == cold["status"][0]


def test_tiny_step_fires_at_the_barrier_minimiser():
    # Table I row 4: at the barrier minimiser the Newton step is zero up to rounding, so the step
    # is taken without a line search and the next iteration must lower mu; here every iteration
    # is such a step (the multipliers move, x stays), so the solve is five tiny steps
    w, th = hover_at_target_workload()
    h = oracle.Handle.quad(w, th)
    h.step()                                             # least-squares multipliers
    s0 = oracle.unpack_state(h.state(), w.n, w.m)
    h.step()                                             # first iteration
    s1 = oracle.unpack_state(h.state(), w.n, w.m)
    assert s1["iter"] == 1 and s1["main"]["tiny"] == 1
    assert np.abs(s1["main"]["x"] - s0["main"]["x"]).max() <= 1e-14
    assert s1["main"]["mu"] == s0["main"]["mu"] == 0.1   # mu is lowered at the start of the next one
    h.step()
    s2 = oracle.unpack_state(h.state(), w.n, w.m)
    assert s2["main"]["mu"] < 0.1 and s2["main"]["nf"] == 0
    o = oracle.solve_quad(w, th[None, :])
    assert o["status"][0] == oracle.ST_CONVERGED and o["stats"][0, 6] == o["iters"][0] >= 3


def _moving_from_static(th_static, n_obs, vel):
    """tracking-family theta with the spheres of a fixed-sphere row and the given velocities"""
    head = th_static[:15]
    obs = th_static[15:].reshape(n_obs, 4)
    return np.concatenate([head, np.concatenate([obs, vel], axis=1).ravel()])


def test_moving_spheres_at_rest_reduce_to_the_fixed_family():
    # centre c + t_k * 0 = c exactly, so a sphere at rest gives the fixed-sphere tracking problem:
    # the same solve, bit for bit
    w1 = W.get("C2")
    wm = W.Workload("C2m-rest", W.FAMILY_QUAD_TRACK_MOVING, 2, N=w1.N, n_obs=w1.n_obs)
    th1 = w1.thetas(0, 2)
    thm = np.stack([_moving_from_static(t, w1.n_obs, np.zeros((w1.n_obs, 3))) for t in th1])
    a = oracle.solve_quad(w1, th1, threads=2)
    b = oracle.solve_quad(wm, thm, threads=2)
    for k in ("x", "y", "zl", "zu", "obj", "kkt", "status", "iters"):
        assert np.array_equal(a[k], b[k]), k


def test_moving_sphere_rows_closed_form():
    # inequality row of sphere j at stage k: |p_k - (c_j + k dt v_j)|^2 - r_j^2 - s_kj, gradient
    # 2 (p_k - c_j(t_k)) on p_k and -1 on s_kj, Hessian 2 y_kj I on p_k
    w = W.get("C2m")
    th = w.theta(3)
    rng = np.random.default_rng(5)
    v = oracle.cold_start(w, th) + 0.1 * rng.normal(size=w.n)
    y = rng.normal(size=w.m)
    f, g, c, J, H = oracle.quad_eval(w, th, v, y)
    obs = th[15:].reshape(w.n_obs, 7)
    nx, nz = 13, 17
    for k in (1, 7, w.N):
        p = v[k * nz:k * nz + 3]
        for j in range(w.n_obs):
            ck = obs[j, 0:3] + k * w.dt * obs[j, 4:7]
            row = (w.N + 1) * nx + (k - 1) * w.n_obs + j
            si = w.n_w + (k - 1) * w.n_obs + j
            assert abs(c[row] - (np.sum((p - ck) ** 2) - obs[j, 3] ** 2 - v[si])) <= 1e-12
            assert np.allclose(J[row, k * nz:k * nz + 3], 2.0 * (p - ck), rtol=0, atol=1e-14)
            assert J[row, si] == -1.0
    # the sphere rows' Hessian contribution: remove the objective and dynamics parts by comparing
    # with the multipliers of the sphere rows set to zero
    y0 = y.copy()
    y0[(w.N + 1) * nx:] = 0.0
    H0 = oracle.quad_eval(w, th, v, y0)[4]
    for k in (1, w.N):
        yk = y[(w.N + 1) * nx + (k - 1) * w.n_obs:(w.N + 1) * nx + k * w.n_obs].sum()
        D = (H - H0)[k * nz:k * nz + 3, k * nz:k * nz + 3]
        assert np.allclose(D, 2.0 * yk * np.eye(3), atol=1e-12)


def test_moving_sphere_solves_reach_kkt_points():
    w = W.get("C2m")
    TH = w.thetas(0, 8)
    o = oracle.solve_quad(w, TH, threads=8)
    assert (o["status"] == oracle.ST_CONVERGED).sum() >= 7
    for i in np.flatnonzero(o["status"] == oracle.ST_CONVERGED):
        assert o["kkt"][i] <= 1e-8
        x = o["x"][i]
        s = x[w.n_w:]
        assert (s >= 0).all() and (o["zl"][i] >= 0).all()


# ------------------------------------------------------------------------ watchdog (Table I row 3)
def _maratos_no_soc(ang, **opts):
    # min 2 (x1^2 + x2^2 - 1) - x1  s.t.  x1^2 + x2^2 = 1: the solution is (1, 0) (on the circle the
    # objective is -x1); started on the circle at angle `ang`, the filter test rejects full Newton
    # steps near the circle (the Maratos effect) when second-order corrections are off
    f = lambda x: 2 * (x[0] ** 2 + x[1] ** 2 - 1) - x[0]
    g = lambda x: np.array([4 * x[0] - 1, 4 * x[1]])
    c = lambda x: np.array([x[0] ** 2 + x[1] ** 2 - 1])
    J = lambda x: np.array([[2 * x[0], 2 * x[1]]])
    H = lambda x, of, y: (of * 4 + 2 * y[0]) * np.eye(2)
    return _generic(2, 1, [-INF, -INF], [INF, INF], f, g, c, J, H, [np.cos(ang), np.sin(ang)], max_soc=0, **opts)


def test_watchdog_full_steps_revert_and_solution():
    h = _maratos_no_soc(1.5, watchdog_trigger=1, watchdog_max=3)
    prev = oracle.unpack_state(h.state(), 2, 1)
    n_full = n_revert = 0
    while h.phase != oracle.PH_DONE:
        h.step()
        st = oracle.unpack_state(h.state(), 2, 1)
        wd = st["watchdog"]
        info = h.last_info()
        if prev["phase"] == oracle.PH_REGULAR and (prev["watchdog"]["active"] or prev["watchdog"]["short"] >= 1):
            ref = wd if wd["active"] else None
            if st["iter"] == prev["iter"]:
                # a revert: the iterate is the reference stored when the watchdog started, bit for bit,
                # and no iteration is counted
                n_revert += 1
                assert wd["active"] == 0 and wd["short"] == 0 and wd["iter"] == 3
                assert np.array_equal(st["main"]["x"], prev["watchdog"]["x"] if prev["watchdog"]["active"]
                                      else prev["main"]["x"])
                assert np.array_equal(st["main"]["y"], prev["watchdog"]["y"] if prev["watchdog"]["active"]
                                      else prev["main"]["y"])
            else:
                # a watchdog step: the full step (no bounds, so alpha_max = 1)
                n_full += 1
                dx = h.last_step()[0]
                assert info["alpha"] == 1.0
                assert np.array_equal(st["main"]["x"], prev["main"]["x"] + dx)
                if ref is not None:
                    assert ref["alpha_max"] == 1.0
        prev = st
    o = h.outputs()
    assert n_full >= 6 and n_revert >= 2
    assert o["status"][0] == oracle.ST_CONVERGED
    assert np.abs(o["x"] - [1.0, 0.0]).max() <= 1e-8
    assert o["stats"][12] == n_revert and o["stats"][11] >= n_revert + 1   # activations, reverts


def test_watchdog_off_takes_the_ordinary_line_search():
    # watchdog_trigger = 0: the counters stay zero and the solve is the one without the options
    h0 = _maratos_no_soc(1.5)
    h1 = _maratos_no_soc(1.5, watchdog_trigger=0, watchdog_max=7)
    h0.run(); h1.run()
    o0, o1 = h0.outputs(), h1.outputs()
    assert o1["stats"][11] == o1["stats"][12] == 0
    for k in ("x", "y", "iters"):
        assert np.array_equal(o0[k], o1[k]), k


# ------------------------------------------------------------------------ soft restoration (Table I row 5)
def _soft_problem(**opts):
    # min (x1 - 1)^2 + (x2 - 2)^2  s.t.  x1 + x2^2 = 1,  0 <= x <= 10, from (3, 3)
    f = lambda x: (x[0] - 1) ** 2 + (x[1] - 2) ** 2
    g = lambda x: np.array([2 * (x[0] - 1), 2 * (x[1] - 2)])
    c = lambda x: np.array([x[0] + x[1] ** 2 - 1])
    J = lambda x: np.array([[1.0, 2 * x[1]]])
    H = lambda x, of, y: np.diag([2 * of, 2 * of + 2 * y[0]])
    h = _generic(2, 1, [0.0, 0.0], [10.0, 10.0], f, g, c, J, H, [3.0, 3.0], **opts)
    return h, (f, g, c, J, H)


def _pd_error_np(fns, x, y, zl, zu, mu, xl, xu):
    f, g, c, J, H = fns
    d = g(x) + J(x).T @ y - zl + zu
    return (np.abs(d).sum() + np.abs(c(x)).sum() + np.abs((x - xl) * zl - mu).sum()
            + np.abs((xu - x) * zu - mu).sum())


def test_soft_restoration_steps_and_hand_over_to_hard_restoration():
    # with theta_max forced to ~0 every line-search trial is rejected, so each iteration fails its
    # line search: soft restoration takes the primal-dual step with alpha = min(alpha_max primal,
    # alpha_max dual) (checked here in numpy), which must lower the primal-dual error by the factor
    # 0.9999; after soft_resto_max soft steps the method moves on to hard restoration
    h, fns = _soft_problem(soft_resto_max=3)
    xl, xu = np.zeros(2), np.full(2, 10.0)
    h.step()                                            # least-squares multipliers
    s = h.state()
    s[16 + 3] = 1e-300                                  # theta_max of the original problem
    h.set_state(s)
    ks = oracle.default_opts().kappa_sigma
    for it in range(1, 4):
        a = oracle.unpack_state(h.state(), 2, 1)["main"]
        h.step()
        st = oracle.unpack_state(h.state(), 2, 1)
        b = st["main"]
        dx, dy, dzl, dzu = h.last_step()
        tau, mu = a["tau"], a["mu"]
        assert b["mu"] == mu
        ap = min(1.0, min((-tau * (a["x"][i] - xl[i]) / dx[i]) if dx[i] < 0 else (tau * (xu[i] - a["x"][i]) / dx[i])
                          for i in range(2) if dx[i] != 0))
        ad = min([1.0] + [-tau * a["zl"][i] / dzl[i] for i in range(2) if dzl[i] < 0]
                 + [-tau * a["zu"][i] / dzu[i] for i in range(2) if dzu[i] < 0])
        al = min(ap, ad)
        assert st["soft"]["active"] == 1 and st["soft"]["iter"] == it and st["iter"] == it
        assert np.array_equal(b["x"], a["x"] + al * dx) and np.array_equal(b["y"], a["y"] + al * dy)
        zl = np.maximum(np.minimum(a["zl"] + al * dzl, ks * mu / (b["x"] - xl)), mu / (ks * (b["x"] - xl)))
        zu = np.maximum(np.minimum(a["zu"] + al * dzu, ks * mu / (xu - b["x"])), mu / (ks * (xu - b["x"])))
        assert np.allclose(b["zl"], zl, rtol=1e-15, atol=0) and np.allclose(b["zu"], zu, rtol=1e-15, atol=0)
        e0 = _pd_error_np(fns, a["x"], a["y"], a["zl"], a["zu"], mu, xl, xu)
        e1 = _pd_error_np(fns, b["x"], b["y"], a["zl"] + al * dzl, a["zu"] + al * dzu, mu, xl, xu)
        assert e1 <= 0.9999 * e0
    h.step()                                            # soft steps used up: hard restoration
    st = oracle.unpack_state(h.state(), 2, 1)
    assert st["phase"] == oracle.PH_RESTO and st["soft"]["active"] == 0
    o = h.outputs()
    assert o["stats"][13] == 3 and o["stats"][14] == 1


def test_soft_restoration_returns_when_the_filter_accepts():
    # with the ordinary theta_max back after the first soft step, the next soft step's point is
    # acceptable to the filter with a decrease over the soft-restoration start: back to the ordinary
    # iteration, and that start point enters the filter
    h, fns = _soft_problem(soft_resto_max=5)
    h.step()
    s = h.state()
    thmax = s[16 + 3]
    s[16 + 3] = 1e-300
    h.set_state(s)
    h.step()
    st = oracle.unpack_state(h.state(), 2, 1)
    assert st["soft"]["active"] == 1
    s = h.state()
    s[16 + 3] = thmax
    h.set_state(s)
    nf0 = st["main"]["nf"]
    h.step()
    st = oracle.unpack_state(h.state(), 2, 1)
    assert st["soft"]["active"] == 0 and st["soft"]["iter"] == 2 and st["phase"] == oracle.PH_REGULAR
    assert st["main"]["nf"] == nf0 + 1
    th0, ph0 = st["soft"]["theta"], st["soft"]["phi"]
    o = oracle.default_opts()
    assert np.isclose(st["main"]["fth"][-1], (1 - o.gamma_theta) * th0, rtol=1e-15)
    assert np.isclose(st["main"]["fph"][-1], ph0 - o.gamma_phi * th0, rtol=1e-15)
    h.run()
    out = h.outputs()
    assert out["status"][0] == oracle.ST_CONVERGED


def test_kkt_matrix_export_is_the_assembled_eq7_matrix():
    # the conditioning hook: at a regular-phase state the exported matrix is
    # [[W + Sigma, A^T], [A, 0]] assembled here from the problem's own derivatives
    w = W.get("C1")
    th = w.theta(4)
    h = oracle.Handle.quad(w, th)
    for _ in range(3):
        h.step()
    st = oracle.unpack_state(h.state(), w.n, w.m)
    assert st["phase"] == oracle.PH_REGULAR
    x, y, zl, zu = (st["main"][k] for k in ("x", "y", "zl", "zu"))
    f, g, c, J, H = oracle.quad_eval(w, th, x, y)
    lo = np.full(w.n, -INF)
    hi = np.full(w.n, INF)
    for k in range(w.N):
        lo[k * 17 + 13:k * 17 + 17] = 0.0
        hi[k * 17 + 13:k * 17 + 17] = 2 * w.model.u_hover
    lo[w.n_w:] = 0.0
    sig = np.zeros(w.n)
    L, U = np.isfinite(lo), np.isfinite(hi)
    sig[L] += zl[L] / (x[L] - lo[L])
    sig[U] += zu[U] / (hi[U] - x[U])
    K = np.block([[H + np.diag(sig), J.T], [J, np.zeros((w.m, w.m))]])
    Ko = h.kkt_matrix()
    assert Ko.shape == K.shape and np.allclose(Ko, K, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------------ adaptive barrier update (Table I row 7)
def test_adaptive_mu_free_mode_loqo_rule():
    # free mode: mu = 0.1 min(0.05 (1 - xi) / xi, 2)^3 avg, avg the mean complementarity product over
    # the bounded components and xi = min / avg, computed here in numpy from the iterate
    w = W.get("C1")
    th = w.theta(2)
    h = oracle.Handle.quad(w, th, opts=oracle.default_opts(mu_strategy=1))
    h.step()                                           # least-squares multipliers
    for it in range(3):
        a = oracle.unpack_state(h.state(), w.n, w.m)
        x, zl, zu = a["main"]["x"], a["main"]["zl"], a["main"]["zu"]
        prods = []
        for k in range(w.N):
            u = x[k * 17 + 13:k * 17 + 17]
            prods += list(u * zl[k * 17 + 13:k * 17 + 17]) + list((2 * w.model.u_hover - u) * zu[k * 17 + 13:k * 17 + 17])
        prods += list(x[w.n_w:] * zl[w.n_w:])
        prods = np.array(prods)
        avg, xi = prods.mean(), prods.min() / prods.mean()
        want = 0.1 * min(0.05 * (1 - xi) / xi, 2.0) ** 3 * avg
        want = max(1e-9, want)
        h.step()
        b = oracle.unpack_state(h.state(), w.n, w.m)
        assert b["adaptive"]["free"] == 1
        mu_max = b["adaptive"]["mu_max"]
        assert np.isclose(b["main"]["mu"], min(want, mu_max), rtol=1e-12), (it, b["main"]["mu"], want)
        assert b["adaptive"]["n_refs"] == min(it + 1, 4)


def test_adaptive_mu_falls_back_to_monotone_without_progress():
    # with a reference E_0 far below the current one, the free mode gives up: monotone mode from
    # mu = 0.8 avg (numpy), filter reset, fallback counted; references far above: free mode kept
    w = W.get("C1")
    th = w.theta(2)
    h = oracle.Handle.quad(w, th, opts=oracle.default_opts(mu_strategy=1))
    h.step()
    h.step()
    s = h.state()
    n, m = w.n, w.m
    F = (len(s) - 16 - (8 + 3 * n + m) - (8 + 3 * (n + 2 * m) + m) - 2 * n - (8 + 3 * n + m) - 4 - 8) // 4
    pa = len(s) - 8                                    # adaptive block: free, n_refs, refs[4], mu_max, 0
    assert s[pa] == 1 and s[pa + 1] == 1
    s2 = s.copy()
    s2[pa + 2] = 1e-30                                 # a reference E_0 that cannot be improved on
    h.set_state(s2)
    a = oracle.unpack_state(s2, n, m)
    x, zl, zu = a["main"]["x"], a["main"]["zl"], a["main"]["zu"]
    prods = []
    for k in range(w.N):
        u = x[k * 17 + 13:k * 17 + 17]
        prods += list(u * zl[k * 17 + 13:k * 17 + 17]) + list((2 * w.model.u_hover - u) * zu[k * 17 + 13:k * 17 + 17])
    prods += list(x[w.n_w:] * zl[w.n_w:])
    h.step()
    b = oracle.unpack_state(h.state(), n, m)
    assert b["adaptive"]["free"] == 0
    assert np.isclose(b["main"]["mu"], max(1e-9, 0.8 * np.mean(prods)), rtol=1e-12)
    assert h.outputs()["stats"][15] == 1
    s3 = s.copy()
    s3[pa + 2] = 1e30
    h3 = oracle.Handle.quad(w, th, opts=oracle.default_opts(mu_strategy=1))
    h3.set_state(s3)
    h3.step()
    assert oracle.unpack_state(h3.state(), n, m)["adaptive"]["free"] == 1


# ------------------------------------------------------------------------ nested restoration
def _cubic_resto(**opts):
    # c(x) = x^3 - 2 x + 2 from x = 0.8 (near the local minimum of |c|): the line search fails and
    # the solve enters feasibility restoration
    c = lambda x: np.array([x[0] ** 3 - 2 * x[0] + 2])
    h = _generic(1, 1, [-INF], [INF], lambda x: 0.0 * x[0], lambda x: np.zeros(1), c,
                 lambda x: np.array([[3 * x[0] ** 2 - 2]]), lambda x, of, y: np.array([[6 * x[0] * y[0]]]), [0.8],
                 **opts)
    return h, c


def _restoration_state(p_scale):
    """State of the cubic problem in its first restoration iterate, with the elastic p scaled by
    p_scale (so that c(x) - p + n = 0 no longer holds when p_scale != 1)."""
    h, c = _cubic_resto()
    for _ in range(100):
        if h.phase == oracle.PH_RESTO:
            break
        h.step()
    assert h.phase == oracle.PH_RESTO
    s = h.state()
    n, m = 1, 1
    F = (len(s) - 16 - (8 + 3 * n + m) - (8 + 3 * (n + 2 * m) + m) - 2 * n - (8 + 3 * n + m) - 4 - 8) // 4
    p_rs = 16 + (8 + 3 * n + m + 2 * F) + 8          # the restoration iterate: x, p, n
    s[p_rs + n] *= p_scale
    return s, c


def test_nested_restoration_restores_the_elastic_rows():
    # The restoration pass cannot move (resto_ls_max = 0: its line search takes no trial point) at
    # a point where c(x) - p + n != 0.  The nested restoration keeps x and y and re-solves the
    # elastic pair in closed form: p - n = c(x), and (p, n) minimises rho (p + n) - mu (ln p + ln n)
    # on that line (2 rho = mu / p + mu / n), z_p = mu / p, z_n = mu / n; the failing point's
    # (theta, phi) enters the restoration filter with the usual margins; one restoration
    # iteration is counted and the phase continues.
    s, c = _restoration_state(1.5)
    before = oracle.unpack_state(s, 1, 1)
    h, _ = _cubic_resto(resto_ls_max=0)
    h.set_state(s)
    h.step()
    after = oracle.unpack_state(h.state(), 1, 1)
    assert after["phase"] == oracle.PH_RESTO and after["status"] == oracle.ST_RUNNING
    assert after["iter"] == before["iter"] + 1
    xb, pb, nb = before["resto"]["x"]
    x, p, nn = after["resto"]["x"]
    assert x == xb and np.array_equal(after["resto"]["y"], before["resto"]["y"])
    cx = c([x])[0]
    assert p > 0 and nn > 0
    assert abs((p - nn) - cx) <= 1e-13 * max(1.0, abs(cx))
    mu, rho = after["resto"]["mu"], 1000.0
    assert abs(mu / p + mu / nn - 2 * rho) <= 1e-10 * 2 * rho
    assert abs(after["resto"]["zl"][1] - mu / p) <= 1e-15 * mu / p
    assert abs(after["resto"]["zl"][2] - mu / nn) <= 1e-15 * mu / nn
    th = abs(cx - pb + nb)
    assert th > 1e-8
    gth = (1.0 - 1e-5) * th
    assert any(abs(t - gth) <= 1e-12 * gth for t in after["resto"]["fth"])
    assert h.outputs()["stats"][16] == 1


def test_nested_restoration_needs_a_violation_and_can_be_off():
    # at the restoration's own starting point c(x) - p + n = 0 holds, so a restoration that cannot
    # move there fails (RESTO_FAILED); with nested restoration off it fails at a violated point too
    s, _ = _restoration_state(1.0)
    h, _ = _cubic_resto(resto_ls_max=0)
    h.set_state(s)
    h.step()
    assert h.status == oracle.ST_RESTO_FAILED and h.outputs()["stats"][16] == 0
    s, _ = _restoration_state(1.5)
    h, _ = _cubic_resto(resto_ls_max=0, nested_resto=0)
    h.set_state(s)
    h.step()
    assert h.status == oracle.ST_RESTO_FAILED and h.outputs()["stats"][16] == 0
