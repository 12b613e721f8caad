"""Pins of the warm-start network reference (oracle/mlp_ref.py): closed forms of GELU, the BF16
rounding rule, and the chain-rule gradient against central finite differences."""
import math

import numpy as np

from oracle import mlp_ref as M


def test_gelu_closed_forms():
    # GELU(x) = x Phi(x): Phi(0) = 1/2, Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert abs(M.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(np.array([-1.0]))[0] + (1.0 - 0.8413447460685429)) < 1e-15
    assert abs(M.gelu_d(np.array([0.0]))[0] - 0.5) < 1e-15
    x = np.linspace(-4, 4, 33)
    fd = (M.gelu(x + 1e-6) - M.gelu(x - 1e-6)) / 2e-6
    assert np.abs(fd - M.gelu_d(x)).max() < 1e-8


def test_bf16_rounding_rule():
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie and rounds to even (1.0), 1 + 3 2^-9
    # rounds up to 1 + 2^-7, 1 + 2^-7 is exact; large and negative values keep their exponent
    v = M.bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7, -3.0, 2.0 ** 100, 1 + 2 ** -8 + 2 ** -20]))
    assert list(v) == [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -7, -3.0, 2.0 ** 100, 1 + 2 ** -7]


def test_gradient_matches_finite_differences():
    d_in, h, d_out, B = 3, 5, 2, 7
    rng = np.random.default_rng(3)
    npar, nmod = M.sizes(d_in, h, d_out)
    model = np.concatenate([rng.normal(0, 0.7, npar), rng.normal(0, 1, d_in), rng.uniform(0.5, 2, d_in),
                            rng.normal(0, 1, d_out), rng.uniform(0.5, 2, d_out)])
    x = rng.normal(size=(B, d_in))
    t = rng.normal(size=(B, d_out))
    loss, g = M.loss_grad(model, x, t, d_in, h, d_out)
    fd = np.zeros(npar)
    for k in range(npar):
        mp, mm = model.copy(), model.copy()
        mp[k] += 1e-6
        mm[k] -= 1e-6
        fd[k] = (M.loss_grad(mp, x, t, d_in, h, d_out)[0] - M.loss_grad(mm, x, t, d_in, h, d_out)[0]) / 2e-6
    assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())
    # the loss is the mean squared normalised error, by definition
    y, _ = M.forward(model, x, d_in, h, d_out)
    Ws, bs, _, _, mu, sd = M.unpack(model, d_in, h, d_out)
    assert abs(loss - np.mean(((y - t) / sd) ** 2)) < 1e-12
