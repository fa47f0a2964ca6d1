"""Pins of the learned-correction oracle: bfloat16 rounding against torch's
conversion, gradients against central finite differences and against
torch.autograd (CPU, float64), Adam against its closed form after one step."""
import numpy as np
import pytest


def test_bf16_round_matches_torch(oracle):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-5, 5, 2000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -7.5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.bf16_round(x), ref)


@pytest.mark.parametrize("rounding", [False, True])
def test_gradients_vs_autograd(oracle, rounding):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    dims = (6, 8, 8, 8, 1)
    p = rng.normal(size=oracle.mlp_n_params(dims)) * 0.4
    x = rng.normal(size=(13, 6))
    base = rng.normal(size=13)
    t = rng.normal(size=13)
    loss, g = oracle.mlp_loss_grad(p, x, base, t, dims, rounding=rounding)
    # torch reference with the same straight-through roundings
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)

    def rnd(v):
        if not rounding:
            return v
        r = v.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return v + (r - v).detach()

    a = torch.tensor(x, dtype=torch.float64)
    k = 0
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        W = pt[k:k + n_in * n_out].reshape(n_out, n_in)
        k += n_in * n_out
        b = pt[k:k + n_out]
        k += n_out
        z = rnd(a) @ rnd(W).T + b
        a = torch.relu(z) if i < len(dims) - 2 else z
    y = torch.tensor(base) + a[:, 0]
    L = ((y - torch.tensor(t)) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    assert np.allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_gradients_vs_finite_differences(oracle):
    rng = np.random.default_rng(2)
    dims = (5, 7, 7, 7, 1)
    p = rng.normal(size=oracle.mlp_n_params(dims)) * 0.5
    x = rng.normal(size=(9, 5))
    base = rng.normal(size=9)
    t = rng.normal(size=9)
    _, g = oracle.mlp_loss_grad(p, x, base, t, dims, rounding=False)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = oracle.mlp_loss_grad(p + e, x, base, t, dims, rounding=False)
        lm, _ = oracle.mlp_loss_grad(p - e, x, base, t, dims, rounding=False)
        fd[i] = (lp - lm) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_zero_output_layer_returns_base(oracle):
    p = oracle.mlp_init(3)
    x = np.random.default_rng(4).normal(size=(10, 20))
    base = np.linspace(0, 5, 10)
    y, _ = oracle.mlp_forward(p, x, base)
    assert np.array_equal(y, base)


def test_adam_first_step_closed_form(oracle):
    # after one step from m = v = 0, the update is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = oracle.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
