"""Seeded synthetic quadrotor NMPC workloads (input data only).

This module draws the parameter vectors theta of the batched parametric NLP
(Sec. III, eq. (1)-(2): instances share f, c and the bounds and differ only in
theta).  It holds the problem definition constants and the random instance
recipes and nothing of the solver's arithmetic, so both the HIP solver and the
CPU oracle are fed from it.

Instance ``i`` of workload ``c`` is drawn from ``numpy.random.default_rng([c, i])``
so that an instance is the same whatever the batch size or slot count.

theta layouts (float64, one row per instance):
  quad_obs          : [xbar0 (13), target position (3), n_obs x (cx, cy, cz, r)]
  quad_track        : [xbar0 (13), A, omega, n_obs x (cx, cy, cz, r)]
  multi_quad        : n_agents x [xbar0 (13), goal position (3)]
  quad_track_moving : [xbar0 (13), A, omega, n_obs x (cx, cy, cz, r, vx, vy, vz)], sphere centre
                      (cx, cy, cz) + t (vx, vy, vz) at time t = k dt of stage k
State order of xbar0: position (3), unit quaternion (w, x, y, z), world-frame
linear velocity (3), body rates (3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

FAMILY_QUAD_OBS = 0
FAMILY_QUAD_TRACK = 1
FAMILY_MULTI_QUAD = 2
FAMILY_QUAD_TRACK_MOVING = 3

NX1 = 13  # states per quadrotor
NU1 = 4   # rotor thrusts per quadrotor


@dataclass
class QuadModel:
    """Rigid-body quadrotor constants (mass 1 kg, inertia diag(0.01, 0.01, 0.02))."""
    mass: float = 1.0
    jxx: float = 0.01
    jyy: float = 0.01
    jzz: float = 0.02
    arm: float = 0.15      # rotor arm length [m] ("+" configuration)
    ctau: float = 0.01     # yaw torque per unit thrust [m]
    grav: float = 9.81

    @property
    def u_hover(self) -> float:
        return self.mass * self.grav / 4.0


@dataclass
class Workload:
    name: str
    family: int
    n_inst: int
    N: int
    n_obs: int = 0
    n_agents: int = 1
    dt: float = 0.05
    q_weight: float = 1.0
    r_weight: float = 0.1
    d_min: float = 0.5            # multi-quad pairwise separation [m]
    precision: str = "fp64"       # "fp64" or "fp32ir" (factor in fp32, fp64 refinement)
    seed_tag: int = 1
    model: QuadModel = field(default_factory=QuadModel)

    # ---- derived sizes -------------------------------------------------
    @property
    def nx(self) -> int:
        return NX1 * self.n_agents

    @property
    def nu(self) -> int:
        return NU1 * self.n_agents

    @property
    def n_ineq(self) -> int:
        """Inequality rows per stage k = 1..N."""
        if self.family == FAMILY_MULTI_QUAD:
            return self.n_agents * (self.n_agents - 1) // 2
        return self.n_obs

    @property
    def n_w(self) -> int:
        return (self.N + 1) * self.nx + self.N * self.nu

    @property
    def n_s(self) -> int:
        return self.N * self.n_ineq

    @property
    def n(self) -> int:
        return self.n_w + self.n_s

    @property
    def m(self) -> int:
        return (self.N + 1) * self.nx + self.n_s

    @property
    def n_theta(self) -> int:
        if self.family == FAMILY_QUAD_OBS:
            return NX1 + 3 + 4 * self.n_obs
        if self.family == FAMILY_QUAD_TRACK:
            return NX1 + 2 + 4 * self.n_obs
        if self.family == FAMILY_QUAD_TRACK_MOVING:
            return NX1 + 2 + 7 * self.n_obs
        return self.n_agents * (NX1 + 3)

    def as_dict(self) -> dict:
        d = asdict(self)
        d.update(nx=self.nx, nu=self.nu, n=self.n, m=self.m, n_theta=self.n_theta)
        return d

    # ---- instance generation -------------------------------------------
    def theta(self, i: int) -> np.ndarray:
        rng = np.random.default_rng([self.seed_tag, int(i)])
        if self.family == FAMILY_QUAD_OBS:
            return _draw_quad_obs(self, rng)
        if self.family == FAMILY_QUAD_TRACK:
            return _draw_quad_track(self, rng)
        if self.family == FAMILY_QUAD_TRACK_MOVING:
            return _draw_quad_track_moving(self, rng)
        return _draw_multi(self, rng)

    def thetas(self, start: int, count: int) -> np.ndarray:
        return np.stack([self.theta(i) for i in range(start, start + count)])


def _hover_state(p) -> np.ndarray:
    x = np.zeros(NX1)
    x[0:3] = p
    x[3] = 1.0
    return x


def _draw_obstacles(rng, n, keep_free, centre_fn, r_lo, r_hi, margin):
    """Draw n spheres; resample one whose surface comes within `margin` of a keep-free point."""
    obs = np.zeros((n, 4))
    for j in range(n):
        while True:
            c = centre_fn(rng)
            r = rng.uniform(r_lo, r_hi)
            if all(np.linalg.norm(c - p) >= r + margin for p in keep_free):
                break
        obs[j, 0:3] = c
        obs[j, 3] = r
    return obs


def _draw_quad_obs(w: Workload, rng) -> np.ndarray:
    if w.name.startswith("C4"):
        # cluttered: start/goal in a 6 m cube, at least 3 m apart; obstacles kept
        # 0.5 m clear of the start and goal (free corridors at the ends)
        while True:
            p0 = rng.uniform(-3.0, 3.0, 3)
            pt = rng.uniform(-3.0, 3.0, 3)
            if np.linalg.norm(pt - p0) >= 3.0:
                break
        obs = _draw_obstacles(rng, w.n_obs, [p0, pt],
                              lambda g: g.uniform(-3.0, 3.0, 3), 0.1, 0.4, 0.5)
    else:
        p0 = rng.uniform(-3.0, 3.0, 3)
        pt = rng.uniform(-3.0, 3.0, 3)
        obs = _draw_obstacles(rng, w.n_obs, [p0, pt],
                              lambda g: g.uniform(-2.0, 2.0, 3), 0.2, 0.5, 0.1)
    return np.concatenate([_hover_state(p0), pt, obs.ravel()])


def _fig8_pos(A, om, t):
    return np.array([A * math.sin(om * t), 0.5 * A * math.sin(2.0 * om * t), 0.0])


def _draw_quad_track(w: Workload, rng) -> np.ndarray:
    A = rng.uniform(1.0, 3.0)
    T = rng.uniform(2.0, 6.0)
    om = 2.0 * math.pi / T
    x0 = np.zeros(NX1)
    x0[3] = 1.0
    x0[0:3] = rng.normal(0.0, 0.3, 3)                       # ref start p = 0
    x0[7:10] = np.array([A * om, A * om, 0.0]) + rng.normal(0.0, 0.3, 3)
    horizon = w.N * w.dt

    def centre(g):
        tj = g.uniform(0.0, horizon)
        return _fig8_pos(A, om, tj) + g.normal(0.0, 0.5, 3)

    # keep the first 0.5 s of the reference (the braking distance at these speeds) clear by
    # 0.3 m and the start by 0.1 m, so that the drawn instances are mostly feasible
    start_seg = [_fig8_pos(A, om, t) for t in np.arange(0.0, 0.5 + 1e-9, w.dt)]
    obs = np.zeros((w.n_obs, 4))
    for j in range(w.n_obs):
        while True:
            c = centre(rng)
            r = rng.uniform(0.2, 0.5)
            if np.linalg.norm(c - x0[0:3]) >= r + 0.1 and all(np.linalg.norm(c - p) >= r + 0.3 for p in start_seg):
                break
        obs[j, 0:3] = c
        obs[j, 3] = r
    return np.concatenate([x0, [A, om], obs.ravel()])


def _draw_quad_track_moving(w: Workload, rng) -> np.ndarray:
    """Figure-eight tracking with spheres that cross the reference path at constant velocity: sphere
    j is near the reference position p_ref(t_j) (N(0, 0.3^2 I)) at a time t_j ~ U(0, N dt) and moves
    at v_j ~ N(0, 0.5^2 I) m/s; resampled if it comes within r + 0.1 m of the start at t = 0 or
    within r + 0.3 m of the reference during its first 0.5 s."""
    A = rng.uniform(1.0, 3.0)
    T = rng.uniform(2.0, 6.0)
    om = 2.0 * math.pi / T
    x0 = np.zeros(NX1)
    x0[3] = 1.0
    x0[0:3] = rng.normal(0.0, 0.3, 3)
    x0[7:10] = np.array([A * om, A * om, 0.0]) + rng.normal(0.0, 0.3, 3)
    horizon = w.N * w.dt
    ts = np.arange(0.0, 0.5 + 1e-9, w.dt)
    obs = np.zeros((w.n_obs, 7))
    for j in range(w.n_obs):
        while True:
            tj = rng.uniform(0.0, horizon)
            v = rng.normal(0.0, 0.5, 3)
            c0 = _fig8_pos(A, om, tj) + rng.normal(0.0, 0.3, 3) - tj * v
            r = rng.uniform(0.2, 0.5)
            if np.linalg.norm(c0 - x0[0:3]) >= r + 0.1 and \
                    all(np.linalg.norm(c0 + t * v - _fig8_pos(A, om, t)) >= r + 0.3 for t in ts):
                break
        obs[j, 0:3] = c0
        obs[j, 3] = r
        obs[j, 4:7] = v
    return np.concatenate([x0, [A, om], obs.ravel()])


def _draw_multi(w: Workload, rng) -> np.ndarray:
    out = []
    for a in range(w.n_agents):
        ang = a * 2.0 * math.pi / w.n_agents
        ring = np.array([2.0 * math.cos(ang), 2.0 * math.sin(ang), 0.0])
        p0 = ring + rng.normal(0.0, 0.2, 3)
        goal = -ring + rng.normal(0.0, 0.2, 3)
        out.append(np.concatenate([_hover_state(p0), goal]))
    return np.concatenate(out)


# The five workloads: plain FP64 point-to-point (C1), figure-eight tracking (C2),
# four-quadrotor swaps (C3), cluttered FP32+refinement (C4), learned warm start (C5); and the
# tracking task with three moving spheres (C2m).
WORKLOADS = {
    "C1": Workload("C1", FAMILY_QUAD_OBS, 64, N=10, n_obs=3, seed_tag=1),
    "C2": Workload("C2", FAMILY_QUAD_TRACK, 4096, N=30, n_obs=8, seed_tag=2),
    "C3": Workload("C3", FAMILY_MULTI_QUAD, 1024, N=20, n_agents=4, seed_tag=3),
    "C4": Workload("C4", FAMILY_QUAD_OBS, 8192, N=40, n_obs=32, precision="fp32ir", seed_tag=4),
    "C5": Workload("C5", FAMILY_QUAD_OBS, 16384, N=10, n_obs=3, precision="fp32ir", seed_tag=5),
    "C2m": Workload("C2m", FAMILY_QUAD_TRACK_MOVING, 4096, N=30, n_obs=3, seed_tag=6),
    # reduced cluttered case the oracle solves in seconds (parity of the FP32 + refinement path)
    "C4s": Workload("C4s", FAMILY_QUAD_OBS, 32, N=12, n_obs=8, precision="fp32ir", seed_tag=41),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]
