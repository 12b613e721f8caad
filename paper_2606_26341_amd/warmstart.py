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


def train_for(w, n_train: int, seed_tag: int, epochs: int = 30, batch: int = 1024, log=None, **opts):
    """Generate `n_train` instances of w's distribution (seed tag `seed_tag`), solve them cold and fit
    the network on the converged ones."""
    from .workloads import Workload
    wt = Workload(w.name + "-train", w.family, n_train, N=w.N, n_obs=w.n_obs, seed_tag=seed_tag)
    TH, T, _ = solve_targets(w, wt.thetas(0, n_train), **opts)
    ws = WarmStart(w, max_batch=max(batch, 16384))
    losses = ws.fit(TH, T, epochs=epochs, batch=batch, log=log)
    return ws, losses, int(TH.shape[0])
