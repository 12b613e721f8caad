"""Shared helpers for the parity tests (comparison metrics only; no solver arithmetic)."""
import numpy as np

import oracle

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
