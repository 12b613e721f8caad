"""Pins for the oracle's quadrotor model (Sec. VI: 13-state rigid body, position / attitude
quaternion / linear velocity / body rates) and for its hyper-dual derivatives.  The dynamics are
pinned by closed-form physics (hover equilibrium, free fall, torque-free rotation, Euler's
equations); the derivatives by finite differences of the oracle's own function values."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_26341_amd import workloads as W

w1 = W.get("C1")
M = w1.model
UH = M.u_hover


def hover(p=(0.3, -0.2, 1.0)):
    x = np.zeros(13)
    x[0:3] = p
    x[3] = 1.0
    return x


def qmul(a, b):
    w1_, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1_ * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1_ * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1_ * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1_ * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_hover_is_equilibrium():
    x = hover()
    F, _, _ = oracle.stage_derivs(w1, x, np.full(4, UH))
    assert np.abs(F - x).max() <= 1e-14


def test_free_fall_is_exact_under_rk4():
    # zero thrust, level attitude: p(t) = p0 + v0 t - g t^2/2 e_z is quadratic, RK4 integrates it exactly
    x = hover()
    x[7:10] = [0.4, -1.0, 2.0]
    F, _, _ = oracle.stage_derivs(w1, x, np.zeros(4))
    dt, g = w1.dt, M.grav
    p = x[0:3] + x[7:10] * dt - 0.5 * g * dt * dt * np.array([0, 0, 1.0])
    v = x[7:10] - g * dt * np.array([0, 0, 1.0])
    assert np.allclose(F[0:3], p, atol=1e-14)
    assert np.allclose(F[7:10], v, atol=1e-14)
    assert np.allclose(F[3:7], x[3:7], atol=1e-15)


@pytest.mark.parametrize("axis", [0, 2])
def test_torque_free_rotation_about_principal_axis(axis):
    # with tau = 0 and omega on a principal axis, omega is constant and q(t) = q0 (x) exp(omega t / 2)
    # (body-frame rates); a world-frame (left) product would differ at first order
    q0 = np.array([0.9, 0.1, -0.3, 0.2])
    q0 /= np.linalg.norm(q0)
    x = hover()
    x[3:7] = q0
    om = np.zeros(3)
    om[axis] = 2.0
    x[10:13] = om
    # zero thrust: no torque
    F, _, _ = oracle.stage_derivs(w1, x, np.zeros(4))
    ang = 2.0 * w1.dt
    e = np.zeros(4)
    e[0] = math.cos(ang / 2)
    e[1 + axis] = math.sin(ang / 2)
    assert np.abs(F[3:7] - qmul(q0, e)).max() <= 1e-7
    assert np.allclose(F[10:13], om, atol=1e-15)


def test_thrust_direction_for_roll():
    phi = 0.3
    x = hover()
    x[3:7] = [math.cos(phi / 2), math.sin(phi / 2), 0.0, 0.0]
    T = 4 * UH
    xd = oracle.xdot(w1, x, np.full(4, UH))
    expect = T / M.mass * np.array([0.0, -math.sin(phi), math.cos(phi)]) - np.array([0, 0, M.grav])
    assert np.allclose(xd[7:10], expect, atol=1e-14)


def test_rotor_torques_and_euler_equations():
    a = 0.7
    x = hover()
    xd = oracle.xdot(w1, x, np.array([0.0, a, 0.0, 0.0]))
    assert np.allclose(xd[10:13], [M.arm * a / M.jxx, 0.0, -M.ctau * a / M.jzz], atol=1e-13)
    x[10:13] = [1.0, 0.0, 3.0]
    xd = oracle.xdot(w1, x, np.zeros(4))
    # Euler: Jyy wdot_y = -(Jxx - Jzz) w_z w_x
    assert np.allclose(xd[10:13], [0.0, -(M.jxx - M.jzz) * 3.0 * 1.0 / M.jyy, 0.0], atol=1e-12)


def _random_state(rng):
    x = np.zeros(13)
    x[0:3] = rng.normal(size=3)
    q = rng.normal(size=4)
    x[3:7] = q / np.linalg.norm(q)
    x[7:10] = rng.normal(size=3)
    x[10:13] = rng.normal(size=3)
    return x


@pytest.mark.parametrize("seed", range(4))
def test_stage_jacobian_and_hessian_match_finite_differences(seed):
    rng = np.random.default_rng([21, seed])
    x = _random_state(rng)
    u = rng.uniform(0.5, 4.0, 4)
    lam = rng.normal(size=13)
    F, G, HL = oracle.stage_derivs(w1, x, u, lam)
    z = np.concatenate([x, u])
    h = 1e-6
    Gfd = np.zeros((13, 17))
    Hfd = np.zeros((17, 17))
    for j in range(17):
        zp, zm = z.copy(), z.copy()
        zp[j] += h
        zm[j] -= h
        Fp, Gp, _ = oracle.stage_derivs(w1, zp[:13], zp[13:])
        Fm, Gm, _ = oracle.stage_derivs(w1, zm[:13], zm[13:])
        Gfd[:, j] = (Fp - Fm) / (2 * h)
        Hfd[:, j] = lam @ (Gp - Gm) / (2 * h)
    assert np.abs(G - Gfd).max() <= 1e-6 * max(1.0, np.abs(G).max())
    assert np.abs(HL - Hfd).max() <= 1e-5 * max(1.0, np.abs(HL).max())
    assert np.allclose(HL, HL.T, atol=0)


@pytest.mark.parametrize("name", ["C1", "C2", "C3"])
def test_nlp_derivatives_match_finite_differences(name):
    w = W.get(name)
    if name == "C3":
        w = W.Workload("C3s", W.FAMILY_MULTI_QUAD, 1, N=3, n_agents=4)
    elif name == "C2":
        w = W.Workload("C2s", W.FAMILY_QUAD_TRACK, 1, N=4, n_obs=8, seed_tag=2)
    else:
        w = W.Workload("C1s", W.FAMILY_QUAD_OBS, 1, N=4, n_obs=3, seed_tag=1)
    th = w.theta(0)
    rng = np.random.default_rng(5)
    v = oracle.cold_start(w, th) + 0.05 * rng.normal(size=w.n)
    y = rng.normal(size=w.m)
    f, g, c, J, H = oracle.quad_eval(w, th, v, y)
    h = 1e-6
    gfd = np.zeros(w.n)
    Jfd = np.zeros((w.m, w.n))
    Hfd = np.zeros((w.n, w.n))
    for j in range(w.n):
        vp, vm = v.copy(), v.copy()
        vp[j] += h
        vm[j] -= h
        fp, gp, cp, Jp, _ = oracle.quad_eval(w, th, vp, y)
        fm, gm, cm, Jm, _ = oracle.quad_eval(w, th, vm, y)
        gfd[j] = (fp - fm) / (2 * h)
        Jfd[:, j] = (cp - cm) / (2 * h)
        Hfd[:, j] = ((gp + Jp.T @ y) - (gm + Jm.T @ y)) / (2 * h)
    assert np.abs(g - gfd).max() <= 1e-6 * max(1, np.abs(g).max())
    assert np.abs(J - Jfd).max() <= 1e-6 * max(1, np.abs(J).max())
    assert np.abs(H - Hfd).max() <= 1e-5 * max(1, np.abs(H).max())
    # constraint structure: the initial-state rows are x_0 - xbar0
    assert np.allclose(c[:13], v[:13] - th[:13])
