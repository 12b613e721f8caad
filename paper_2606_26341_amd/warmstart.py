"""Learned warm start: a network from instance parameters to (w, y), trained on solutions the
solver itself produces and used as `warm` starting points of `Solver.solve`.

Every numeric step runs in the library's kernels (solver, network forward/backward, Adam,
normalisation statistics); this module only sequences the calls and selects the converged
training rows.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hipipm
from .mlp import Mlp


def solve_targets(w, thetas: np.ndarray, slots: int = 8192, device="cuda:0", **opts):
    """Cold FP64 solves of `thetas`; returns (theta, target) device tensors of the converged rows,
    target = [w* (n_w), y* (m)], and the iteration counts of all rows."""
    TH = torch.tensor(thetas, dtype=torch.float64, device=device)
    s = hipipm.Solver(w, min(slots, TH.shape[0]), hipipm.default_options(**opts))
    out = s.solve(TH)
    torch.cuda.synchronize()
    ok = out["status"] == hipipm.ST_CONVERGED
    target = torch.cat([out["x"][:, :w.n_w], out["y"]], dim=1)
    return TH[ok].contiguous(), target[ok].contiguous(), out["iters"]


class WarmStart:
    def __init__(self, w, hidden: int = 256, max_batch: int = 16384, device="cuda:0", seed: int = 0):
        assert w.family == 0, "the warm start is built for the point-to-point obstacle family"
        self.w = w
        self.net = Mlp(w.n_theta, w.n_w + w.m, hidden=hidden, max_batch=max_batch, device=device, seed=seed)

    def fit(self, theta: torch.Tensor, target: torch.Tensor, epochs: int = 30, batch: int = 1024,
            lr: float = 2e-3, lr_final: float = 1e-4, seed: int = 0, log=None):
        self.net.set_normalizer(theta, target)
        return self.net.train(theta, target, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, seed=seed,
                              log=log)

    def predict(self, theta: torch.Tensor) -> torch.Tensor:
        """Warm points [B][n_w + m] for `Solver.solve(theta, warm=...)` (batched to the workspace)."""
        outs = []
        for a in range(0, theta.shape[0], self.net.max_batch):
            outs.append(self.net.forward(theta[a:a + self.net.max_batch].contiguous()))
        return torch.cat(outs, dim=0)


def split(w, n: int, seed_tag: int):
    """`n` instances of w's distribution drawn under another seed tag (a split disjoint from w's own
    instances: the generator seed is (tag, index))."""
    from .workloads import Workload
    return Workload(f"{w.name}-split{seed_tag}", w.family, n, N=w.N, n_obs=w.n_obs, seed_tag=seed_tag).thetas(0, n)


def train_for(w, n_train: int, seed_tag: int, epochs: int = 30, batch: int = 1024, log=None, thetas=None, **opts):
    """Solve `n_train` instances of w's distribution (seed tag `seed_tag`, or the given `thetas`) cold
    and fit the network on the converged ones."""
    TH, T, _ = solve_targets(w, split(w, n_train, seed_tag) if thetas is None else thetas, **opts)
    ws = WarmStart(w, max_batch=max(batch, 16384))
    losses = ws.fit(TH, T, epochs=epochs, batch=batch, log=log)
    return ws, losses, int(TH.shape[0])


def select_options(ws: WarmStart, w, thetas: np.ndarray, mu0s=(1e-2, 1e-3, 1e-4), qs=(95.0, 99.0, 100.0),
                   device="cuda:0", **opts):
    """Choose the warm barrier parameter and the divergence cap on a validation split.

    mu0: the candidate with the fewest mean iterations per converged solve (ties: more converged),
    judged with the cap at the largest cold iteration count.  Cap: a percentile (qs) of the cold
    iteration counts on the same split (0 = no cap), the one whose batched warm solve of the split
    takes the least wall time (a warm solve that is cut off restarts cold and lengthens the batch;
    one that diverges without a cap does too).  Returns (warm_mu0, warm_iter_cap, table)."""
    import time
    TH = torch.tensor(thetas, dtype=torch.float64, device=device)
    n = TH.shape[0]
    s = hipipm.Solver(w, n, hipipm.default_options(**opts))
    cold = s.solve(TH)
    it_cold = cold["iters"].cpu().numpy()
    pts = ws.predict(TH)
    table = {"mu0": {}, "cap": {}}
    cap_max = int(it_cold.max())
    for mu in mu0s:
        s = hipipm.Solver(w, n, hipipm.default_options(warm_mu0=mu, warm_iter_cap=cap_max, **opts))
        out = s.solve(TH, warm=pts)
        ok = (out["status"] == hipipm.ST_CONVERGED).cpu().numpy()
        it = out["iters"].cpu().numpy()
        table["mu0"][mu] = (float(it[ok].mean()) if ok.any() else float("inf"), float(ok.mean()))
    best = min(mu0s, key=lambda m: (table["mu0"][m][0], -table["mu0"][m][1]))
    caps = sorted({int(np.ceil(np.percentile(it_cold, q))) for q in qs} | {0})
    for cap in caps:
        s = hipipm.Solver(w, n, hipipm.default_options(warm_mu0=best, warm_iter_cap=cap, **opts))
        out = s.alloc_outputs(n)
        s.solve(TH, warm=pts, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            s.solve(TH, warm=pts, out=out)
        torch.cuda.synchronize()
        ok = (out["status"] == hipipm.ST_CONVERGED).cpu().numpy()
        table["cap"][cap] = ((time.perf_counter() - t0) / 3 * 1e3, float(ok.mean()), int(out["iters"].max().item()))
    cap = min(caps, key=lambda k: (-table["cap"][k][1], table["cap"][k][0]))
    return best, cap, table
