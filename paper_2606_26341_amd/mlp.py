"""Thin ctypes binding of the warm-start network entry points (include/hipipm_mlp.h).

Device buffers come from torch; the forward pass, the loss, the gradient and the Adam update
run in the library's HIP kernels.  `Mlp.train` is a host loop over those calls (minibatch order
from a seeded permutation).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import hipipm

EXPORTS = ("hipipm_mlp_sizes", "hipipm_mlp_weights_bf16", "hipipm_mlp_normalizer", "hipipm_mlp_forward",
           "hipipm_mlp_backward", "hipipm_mlp_adam")

i32, i64, vp, f32 = C.c_int32, C.c_int64, C.c_void_p, C.c_float


def _lib():
    L = hipipm.load()
    if not getattr(L, "_mlp_bound", False):
        L.hipipm_mlp_sizes.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp]
        L.hipipm_mlp_weights_bf16.argtypes = [i32, i32, i32, vp, vp, vp]
        L.hipipm_mlp_normalizer.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp]
        L.hipipm_mlp_forward.argtypes = [i32, i32, i32, vp, vp, vp, vp, i32, vp, vp]
        L.hipipm_mlp_backward.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
        L.hipipm_mlp_adam.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
        for n in EXPORTS:
            getattr(L, n).restype = C.c_int
        L._mlp_bound = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _s(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Mlp:
    def __init__(self, d_in: int, d_out: int, hidden: int = 256, max_batch: int = 16384, device="cuda:0", seed=0):
        self.L = _lib()
        self.d_in, self.h, self.d_out, self.device = d_in, hidden, d_out, torch.device(device)
        ml, npar, nw, ab = i64(), i64(), i64(), i64()
        self._check(self.L.hipipm_mlp_sizes(d_in, hidden, d_out, max_batch, C.byref(ml), C.byref(npar), C.byref(nw),
                                            C.byref(ab)))
        self.model_len, self.n_params, self.n_weights = ml.value, npar.value, nw.value
        self.max_batch = max_batch
        self.model = torch.zeros(self.model_len, dtype=torch.float32, device=self.device)
        self.wb = torch.zeros(self.n_weights, dtype=torch.int16, device=self.device)
        self.act = torch.empty(ab.value, dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.m = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.step = 0
        self.init_params(seed)

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise RuntimeError(f"hipipm_mlp call failed ({rc})")

    def layout(self):
        io = [self.d_in, self.h, self.h, self.h, self.d_out]
        return [(io[l], io[l + 1]) for l in range(4)]

    def init_params(self, seed=0):
        """He-uniform weights and zero biases from a seeded generator (host random numbers);
        identity normalisation."""
        rng = np.random.default_rng(seed)
        parts = []
        for i, o in self.layout():
            lim = np.sqrt(6.0 / i)
            parts += [rng.uniform(-lim, lim, size=o * i), np.zeros(o)]
        parts += [np.zeros(self.d_in), np.ones(self.d_in), np.zeros(self.d_out), np.ones(self.d_out)]
        self.set_model(np.concatenate(parts))

    def set_model(self, model_np):
        self.model.copy_(torch.tensor(np.asarray(model_np, dtype=np.float32), device=self.device))
        self._check(self.L.hipipm_mlp_weights_bf16(self.d_in, self.h, self.d_out, _p(self.model), _p(self.wb), _s()))
        self.m.zero_(); self.v.zero_(); self.step = 0

    def set_normalizer(self, inputs: torch.Tensor, targets: torch.Tensor):
        self._check(self.L.hipipm_mlp_normalizer(self.d_in, self.h, self.d_out, inputs.shape[0], _p(inputs),
                                                 _p(targets), _p(self.model), _s()))

    def forward(self, inputs: torch.Tensor) -> torch.Tensor:
        B = inputs.shape[0]
        assert inputs.dtype == torch.float64 and inputs.shape[1] == self.d_in and B <= self.max_batch
        out = torch.empty((B, self.d_out), dtype=torch.float64, device=self.device)
        self._check(self.L.hipipm_mlp_forward(self.d_in, self.h, self.d_out, _p(self.model), _p(self.wb),
                                              _p(inputs.contiguous()), _p(out), B, _p(self.act), _s()))
        return out

    def backward(self, inputs, targets, rows=None, batch=None):
        """Loss (host float) and gradient (self.grad) over `rows` (int32 device tensor) or all rows."""
        B = int(batch if batch is not None else (rows.shape[0] if rows is not None else inputs.shape[0]))
        assert B <= self.max_batch
        nparts = (B * self.d_out + 255) // 256
        parts = torch.empty(nparts, dtype=torch.float32, device=self.device)
        self._check(self.L.hipipm_mlp_backward(self.d_in, self.h, self.d_out, _p(self.model), _p(self.wb),
                                               _p(inputs), _p(targets), _p(rows), B, _p(self.act), _p(self.grad),
                                               _p(parts), _s()))
        return parts, B

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        self._check(self.L.hipipm_mlp_adam(self.d_in, self.h, self.d_out, _p(self.model), _p(self.wb), _p(self.grad),
                                           _p(self.m), _p(self.v), self.step, lr, beta1, beta2, eps, _s()))

    def train(self, inputs, targets, epochs=20, batch=1024, lr=1e-3, lr_final=1e-4, seed=0, log=None):
        """Minibatch Adam on (inputs, targets) (FP64 device tensors); returns per-epoch mean losses."""
        n = inputs.shape[0]
        rng = np.random.default_rng(seed)
        steps_per_epoch = n // batch
        total = epochs * steps_per_epoch
        losses = []
        for ep in range(epochs):
            perm = torch.tensor(rng.permutation(n).astype(np.int32), device=self.device)
            acc = []
            for b in range(steps_per_epoch):
                rows = perm[b * batch:(b + 1) * batch]
                parts, B = self.backward(inputs, targets, rows)
                t = (ep * steps_per_epoch + b) / max(1, total - 1)
                self.adam(lr=float(lr * (lr_final / lr) ** t))
                acc.append(parts)
            loss = float(torch.stack([p.sum() for p in acc]).sum().item()) / (steps_per_epoch * batch * self.d_out)
            losses.append(loss)
            if log:
                log(f"epoch {ep} loss {loss:.4e}")
        return losses
