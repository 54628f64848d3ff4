"""Pins of the surrogate-MLP oracle: bfloat16 rounding, GELU, gradients and
the input Jacobian against PyTorch's CPU autograd in float64 (library
routines) and central differences; Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2311_13337_amd import inputs


def _torch_net(p):
    w = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(p).items()}

    def f(X):
        h1 = torch.nn.functional.gelu(X @ w["W1"].T + w["b1"])
        h2 = torch.nn.functional.gelu(h1 @ w["W2"].T + w["b2"])
        return h2 @ w["W3"].T + w["b3"]
    return w, f


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_gelu_and_derivative():
    x = np.linspace(-8, 8, 2001)
    t = torch.tensor(x, requires_grad=True)
    y = torch.nn.functional.gelu(t)
    y.sum().backward()
    np.testing.assert_allclose(mlp.gelu(x), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mlp.gelu_grad(x), t.grad.numpy(), rtol=1e-13, atol=1e-15)


def test_parameter_count():
    assert mlp.N_PARAMS == 17926 == inputs.mlp_init_params().size


def test_gradient_matches_autograd_and_differences():
    rng = np.random.default_rng(1)
    p = inputs.mlp_init_params(3).astype(np.float64)
    X = rng.uniform(-1, 1, (37, 4))
    T = rng.standard_normal((37, 6))
    loss, g = mlp.loss_and_grad(p, X, T, bf16_ops=False)
    w, f = _torch_net(p)
    L = ((f(torch.tensor(X)) - torch.tensor(T)) ** 2).mean()
    L.backward()
    gt = mlp.pack({k: v.grad.numpy() for k, v in w.items()})
    np.testing.assert_allclose(loss, L.item(), rtol=1e-13)
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-15)
    for i in rng.choice(mlp.N_PARAMS, 25, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, X, T, False)[0] - mlp.loss_and_grad(pm, X, T, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-9   # FD roundoff ~ eps L / h


def test_bf16_gradient_close_to_exact():
    rng = np.random.default_rng(2)
    p = inputs.mlp_init_params(4).astype(np.float64)
    X = rng.uniform(-1, 1, (64, 4))
    T = rng.standard_normal((64, 6))
    _, g = mlp.loss_and_grad(p, X, T, bf16_ops=False)
    _, gb = mlp.loss_and_grad(p, X, T, bf16_ops=True)
    assert np.linalg.norm(gb - g) <= 0.02 * np.linalg.norm(g)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    t_p = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t_p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        opt.zero_grad()
        t_p.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, t)
        np.testing.assert_allclose(p, t_p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_input_jacobian_matches_autograd():
    rng = np.random.default_rng(6)
    p = inputs.mlp_init_params(7).astype(np.float64)
    X = rng.uniform(-1, 1, (9, 4))
    J = mlp.input_jacobian(p, X, bf16_ops=False)
    _, f = _torch_net(p)
    for n in range(9):
        Jt = torch.autograd.functional.jacobian(f, torch.tensor(X[n:n + 1]))[0, :, 0, :]
        np.testing.assert_allclose(J[n], Jt.detach().numpy(), rtol=1e-11, atol=1e-14)
