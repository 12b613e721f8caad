"""Reference of the warm-start network -- test infrastructure only (see oracle/__init__.py).

A plain numpy statement of the multilayer perceptron d_in -> H -> H -> H -> d_out with GELU after
each hidden layer, normalised inputs and outputs, mean-squared-error loss and its gradient by
the chain rule.  ``bf16=False`` is the exact FP64 network; ``bf16=True`` additionally rounds to
BF16 (nearest even) wherever the GPU kernels hand a value to a matrix product: the normalised
input, the weights, the hidden activations, the output error and the back-propagated
pre-activation gradients.  Parameter layout: per layer the weight [out][in] (row major) then the
bias, then in_mu, in_sd, out_mu, out_sd.
"""
from __future__ import annotations

import math

import numpy as np

NL = 4


def layer_dims(d_in: int, h: int, d_out: int):
    io = [d_in, h, h, h, d_out]
    return [(io[l], io[l + 1]) for l in range(NL)]


def sizes(d_in: int, h: int, d_out: int):
    n = sum(i * o + o for i, o in layer_dims(d_in, h, d_out))
    return n, n + 2 * d_in + 2 * d_out


def unpack(model: np.ndarray, d_in: int, h: int, d_out: int):
    Ws, bs, o = [], [], 0
    for i, out in layer_dims(d_in, h, d_out):
        Ws.append(model[o:o + i * out].reshape(out, i)); o += i * out
        bs.append(model[o:o + out]); o += out
    in_mu, in_sd = model[o:o + d_in], model[o + d_in:o + 2 * d_in]
    o += 2 * d_in
    out_mu, out_sd = model[o:o + d_out], model[o + d_out:o + 2 * d_out]
    return Ws, bs, in_mu, in_sd, out_mu, out_sd


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_d(x):
    return 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(model, x, d_in, h, d_out, bf=False):
    """Network output (de-normalised) and the intermediate values."""
    Ws, bs, in_mu, in_sd, out_mu, out_sd = unpack(np.asarray(model, dtype=np.float64), d_in, h, d_out)
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    a = r((x - in_mu) / in_sd)
    acts, zs = [a], []
    for l in range(NL):
        z = a @ r(Ws[l]).T + bs[l]
        if l < NL - 1:
            zs.append(z)
            a = r(gelu(z))
            acts.append(a)
        else:
            y = z
    return y * out_sd + out_mu, dict(acts=acts, zs=zs, y=y)


def loss_grad(model, x, t, d_in, h, d_out, bf=False):
    """Mean squared error of the normalised outputs and its gradient (parameter layout)."""
    Ws, bs, in_mu, in_sd, out_mu, out_sd = unpack(np.asarray(model, dtype=np.float64), d_in, h, d_out)
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    _, c = forward(model, x, d_in, h, d_out, bf)
    B = x.shape[0]
    tn = (t - out_mu) / out_sd
    e = c["y"] - tn
    loss = float((e * e).sum() / (B * d_out))
    dz = r(2.0 * e / (B * d_out))
    gW, gb = [None] * NL, [None] * NL
    for l in range(NL - 1, -1, -1):
        gW[l] = dz.T @ c["acts"][l]
        gb[l] = dz.sum(axis=0)
        if l == 0:
            break
        da = dz @ r(Ws[l])
        dz = r(da * gelu_d(c["zs"][l - 1]))
    g = np.concatenate([np.concatenate([gW[l].ravel(), gb[l]]) for l in range(NL)])
    return loss, g
