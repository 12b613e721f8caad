"""GPU warm-start network kernels (BF16 matrix-core products, FP32 accumulation) against the
numpy reference: forward values, gradients and a training run."""
import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def _random_model(d_in, h, d_out, seed):
    rng = np.random.default_rng(seed)
    npar, _ = M.sizes(d_in, h, d_out)
    parts = []
    for i, o in M.layer_dims(d_in, h, d_out):
        parts += [rng.uniform(-1, 1, o * i) * np.sqrt(3.0 / i), rng.normal(0, 0.1, o)]
    parts += [rng.normal(0, 1, d_in), rng.uniform(0.5, 2, d_in), rng.normal(0, 1, d_out), rng.uniform(0.5, 2, d_out)]
    return np.concatenate(parts)


@pytest.mark.parametrize("d_in,h,d_out,B", [(28, 256, 356, 300), (5, 40, 7, 65)])
def test_forward_matches_reference(torch_cuda, d_in, h, d_out, B):
    torch = torch_cuda
    from paper_2606_26341_amd.mlp import Mlp
    model = _random_model(d_in, h, d_out, 5)
    net = Mlp(d_in, d_out, hidden=h, max_batch=B)
    net.set_model(model)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(B, d_in))
    y = net.forward(torch.tensor(x, dtype=torch.float64, device="cuda")).cpu().numpy()
    yb, _ = M.forward(model.astype(np.float32).astype(np.float64), x, d_in, h, d_out, bf=True)
    y64, _ = M.forward(model, x, d_in, h, d_out, bf=False)
    scale = np.abs(yb).max()
    eb = np.abs(y - yb).max() / scale
    e64 = np.abs(y - y64).max() / scale
    print("forward rel err vs bf16 reference", eb, "vs fp64", e64, flush=True)
    assert eb <= 5e-3 and e64 <= 5e-2


def test_gradient_matches_reference(torch_cuda):
    torch = torch_cuda
    from paper_2606_26341_amd.mlp import Mlp
    d_in, h, d_out, B = 28, 256, 356, 256
    model = _random_model(d_in, h, d_out, 7)
    net = Mlp(d_in, d_out, hidden=h, max_batch=B)
    net.set_model(model)
    rng = np.random.default_rng(8)
    x, t = rng.normal(size=(B, d_in)), rng.normal(size=(B, d_out))
    X = torch.tensor(x, dtype=torch.float64, device="cuda")
    T = torch.tensor(t, dtype=torch.float64, device="cuda")
    parts, _ = net.backward(X, T)
    g = net.grad.cpu().numpy().astype(np.float64)
    loss = float(parts.sum().item()) / (B * d_out)
    m32 = model.astype(np.float32).astype(np.float64)
    lb, gb = M.loss_grad(m32, x, t, d_in, h, d_out, bf=True)
    l64, g64 = M.loss_grad(m32, x, t, d_in, h, d_out, bf=False)
    cos = g @ gb / (np.linalg.norm(g) * np.linalg.norm(gb))
    rel = np.linalg.norm(g - gb) / np.linalg.norm(gb)
    rel64 = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    print("loss", loss, lb, l64, "grad cos", cos, "rel", rel, "rel fp64", rel64, flush=True)
    assert abs(loss - lb) <= 1e-3 * lb
    assert cos >= 0.9999 and rel <= 1e-2 and rel64 <= 5e-2


def test_training_fits_a_teacher_network(torch_cuda):
    torch = torch_cuda
    from paper_2606_26341_amd.mlp import Mlp
    d_in, h, d_out, n = 28, 256, 356, 8192
    teacher = _random_model(d_in, 64, d_out, 9)
    rng = np.random.default_rng(10)
    x = rng.normal(size=(n, d_in))
    t, _ = M.forward(teacher, x, d_in, 64, d_out)
    X = torch.tensor(x, dtype=torch.float64, device="cuda")
    T = torch.tensor(t, dtype=torch.float64, device="cuda")
    net = Mlp(d_in, d_out, hidden=h, max_batch=512)
    net.set_normalizer(X, T)
    losses = net.train(X, T, epochs=30, batch=512, lr=2e-3, lr_final=2e-4, seed=1)
    print("losses", losses, flush=True)
    assert losses[-1] < 0.25 * losses[0] and all(b < a * 1.05 for a, b in zip(losses, losses[1:]))


def test_normalizer_matches_column_statistics(torch_cuda):
    """Column means and standard deviations of the training arrays (ragged column counts, a
    constant column floored at 1e-6) against numpy."""
    torch = torch_cuda
    from paper_2606_26341_amd.mlp import Mlp
    rng = np.random.default_rng(12)
    rows, d_in, d_out = 10007, 28, 71
    x = rng.normal(3.0, 2.0, size=(rows, d_in))
    t = rng.uniform(-5, 5, size=(rows, d_out))
    x[:, 4] = 1.25
    net = Mlp(d_in, d_out, hidden=32, max_batch=64)
    net.set_normalizer(torch.tensor(x, dtype=torch.float64, device="cuda"),
                       torch.tensor(t, dtype=torch.float64, device="cuda"))
    model = net.model.cpu().numpy().astype(np.float64)
    _, _, in_mu, in_sd, out_mu, out_sd = M.unpack(model, d_in, 32, d_out)
    sd_x = np.maximum(x.std(axis=0), 1e-6)
    assert np.allclose(in_mu, x.mean(axis=0), rtol=1e-6, atol=1e-6)
    assert np.allclose(in_sd, sd_x, rtol=1e-5, atol=1e-7) and in_sd[4] == np.float32(1e-6)
    assert np.allclose(out_mu, t.mean(axis=0), rtol=1e-6, atol=1e-6)
    assert np.allclose(out_sd, t.std(axis=0), rtol=1e-5)
