"""Shared helpers for the parity tests (comparison metrics only; no solver arithmetic)."""
import numpy as np

import oracle
from paper_2606_26341_amd import workloads as W

def e_v(a, b):
    """Largest scaled elementwise deviation max_i |a_i - b_i| / (1 + |b_i|) (Sec. VI, eq. (8))."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / (1.0 + np.abs(b))))


def state_fields(s, n, m):
    """Named fields of a flat state (oracle order), for comparisons."""
    return oracle.unpack_state(np.asarray(s), n, m)


def compare_states(sg, so, n, m):
    """Return (discrete mismatches, e_v over the continuous fields of the active sub-problem)."""
    g = state_fields(sg, n, m)
    o = state_fields(so, n, m)
    bad = []
    for k in ("phase", "iter", "status"):
        if g[k] != o[k]:
            bad.append((k, g[k], o[k]))
    ev = 0.0
    subs = ["main"] + (["resto"] if o["phase"] == oracle.PH_RESTO else [])
    for sub in subs:
        for k in ("nf", "tiny"):
            if g[sub][k] != o[sub][k]:
                bad.append((sub + "." + k, g[sub][k], o[sub][k]))
        for k in ("x", "y", "zl", "zu"):
            ev = max(ev, e_v(g[sub][k], o[sub][k]))
        for k in ("mu", "tau", "dx_last", "theta_max", "theta_min"):
            ev = max(ev, e_v([g[sub][k]], [o[sub][k]]))
        nf = min(g[sub]["nf"], o[sub]["nf"])
        if nf:
            ev = max(ev, e_v(g[sub]["fth"][:nf], o[sub]["fth"][:nf]))
            ev = max(ev, e_v(g[sub]["fph"][:nf], o[sub]["fph"][:nf]))
    return bad, ev


def hover_at_target_workload(N=10):
    """Point-to-point family with no spheres, started hovering at its own target: the start is the
    minimiser of every barrier sub-problem (the two log terms of a rotor bound balance at
    u = u_hover, the middle of [0, 2 u_hover]; the state cost is zero and hover is an equilibrium),
    so every Newton step is zero up to rounding and the tiny-step rule (Table I row 4) fires."""
    w = W.Workload("hover", W.FAMILY_QUAD_OBS, 1, N=N, n_obs=0)
    p = np.array([0.5, -1.0, 2.0])
    x0 = np.zeros(13)
    x0[:3] = p
    x0[3] = 1.0
    return w, np.concatenate([x0, p])
