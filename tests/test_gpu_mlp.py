"""Parity of the surrogate network's GPU kernels with the FP64 oracle.

The oracle (oracle/mlp.py) rounds every matrix-product operand to bfloat16 at
the same points as the kernels and evaluates the rest in FP64, so the only
differences left are FP32 evaluation of GELU/erf and summation order (and the
rare bfloat16 rounding flip that these cause). Tolerances below are derived
from that: FP32 sums of at most 128 terms (relative error ~1e-5 of the sum of
magnitudes) plus a few flips of one bfloat16 ulp (2^-8 relative) of a single
term, i.e. about 1e-3 of the largest entry of each parameter block.

Inputs are chosen so that the normalisation is exact in FP32 (x_lo = -1,
x_hi = 1 and bfloat16-representable inputs; target mean 0 and std 1): both
sides then see identical network inputs.
"""
import numpy as np
import pytest

from oracle import mlp as om
from paper_2311_13337_amd import inputs

pytestmark = pytest.mark.gpu

BLOCKS = (("W1", 0, 512), ("b1", 512, 640), ("W2", 640, 17024), ("b2", 17024, 17152),
          ("W3", 17152, 17920), ("b3", 17920, 17926))


def _bf16_inputs(rng, n):
    return om.bf16(rng.uniform(-1.0, 1.0, size=(n, 4))).astype(np.float32)


def _net(params, lr=1e-3, lo=(-1, -1, -1, -1), hi=(1, 1, 1, 1)):
    from paper_2311_13337_amd import vadx
    return vadx.Mlp(params, lo, hi, lr=lr)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _block_close(got, want, rel, what):
    for name, a, b in BLOCKS:
        g, w = got[a:b], want[a:b]
        scale = np.abs(w).max()
        err = np.abs(g - w).max()
        assert err <= rel * scale + 1e-7, f"{what} {name}: max err {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("n", [32, 100, 257])
def test_gradient_matches_oracle(n):
    rng = np.random.default_rng(11 + n)
    p = inputs.mlp_init_params(seed=5)
    X = _bf16_inputs(rng, n)
    Y = rng.normal(size=(n, 6)).astype(np.float32)
    net = _net(p)
    loss, g = net.grad(_dev(X), _dev(Y))
    lo, go = om.loss_and_grad(p.astype(np.float64), X, Y, bf16_ops=True)
    assert abs(loss - lo) <= 1e-5 * lo
    _block_close(g, go, 2e-3, "gradient")
    # the matched bfloat16 rounding matters: plain FP64 is further away than the
    # kernel is from the rounded oracle (for the blocks fed by products)
    _, g64 = om.loss_and_grad(p.astype(np.float64), X, Y, bf16_ops=False)
    e_k = np.abs(g[640:17024] - go[640:17024]).max()
    e_64 = np.abs(g64[640:17024] - go[640:17024]).max()
    assert e_k < e_64


@pytest.mark.parametrize("n", [1, 77, 1000])
def test_predict_and_jacobian_match_oracle(n):
    import torch
    rng = np.random.default_rng(3 + n)
    p = inputs.mlp_init_params(seed=9)
    # make the network less trivial than its initialisation
    p = (p * rng.uniform(1.0, 3.0, size=p.shape)).astype(np.float32)
    X = _bf16_inputs(rng, n)
    net = _net(p)
    Y, J, sc = net.predict(_dev(X), jacobian=True, score_outputs=(0, 5))
    torch.cuda.synchronize()
    Y, J, sc = Y.cpu().numpy(), J.cpu().numpy(), sc.cpu().numpy()
    f = om.forward(p.astype(np.float64), X, bf16_ops=True)
    Jo = om.input_jacobian(p.astype(np.float64), X, bf16_ops=True)
    assert np.abs(Y - f["Y"]).max() <= 2e-3 * np.abs(f["Y"]).max() + 1e-6
    assert np.abs(J - Jo).max() <= 2e-3 * np.abs(Jo).max() + 1e-6
    so = np.sqrt((Jo[:, 0, :] ** 2).sum(-1) + (Jo[:, 5, :] ** 2).sum(-1))
    assert np.abs(sc - so).max() <= 2e-3 * so.max() + 1e-6
    # the Jacobian is that of the network: central differences of the FP64
    # network agree with the FP64 Jacobian (pins the tangent propagation)
    J64 = om.input_jacobian(p.astype(np.float64), X[:4], bf16_ops=False)
    h = 1e-6
    for c in range(4):
        d = np.zeros(4)
        d[c] = h
        fd = (om.forward(p, X[:4] + d, False)["Y"] - om.forward(p, X[:4] - d, False)["Y"]) / (2 * h)
        assert np.allclose(fd, J64[:, :, c], rtol=1e-6, atol=1e-8)


def test_predict_units_and_ragged_edges():
    """Physical-unit inputs and outputs: x is min-max scaled to [-1, 1] inside,
    outputs are de-normalised with the target mean/std."""
    import torch
    rng = np.random.default_rng(21)
    p = inputs.mlp_init_params(seed=2)
    lo, hi = (0.0, 0.0, 0.0, 1.0), (0.5, 120.0, 20.0, 10.0)
    net = _net(p, lo=lo, hi=hi)
    mean = np.array([0.1, 0.2, -0.3, 5.0, 1.0, 0.05], np.float32)
    std = np.array([0.05, 0.1, 0.2, 3.0, 0.5, 0.02], np.float32)
    net.set_target_norm(mean, std)
    m2, s2 = net.target_norm()
    assert np.array_equal(m2, mean) and np.array_equal(s2, std)
    n = 45
    Xp = rng.uniform(lo, hi, size=(n, 4)).astype(np.float32)
    Y, _, _ = net.predict(_dev(Xp))
    torch.cuda.synchronize()
    xl, xs = np.float32(lo), np.float32(2.0) / (np.float32(hi) - np.float32(lo))
    Xn = (Xp - xl) * xs - np.float32(1.0)
    f = om.forward(p.astype(np.float64), Xn.astype(np.float64), bf16_ops=True)
    Yo = f["Y"] * std + mean
    tol = (5e-3 * np.abs(f["Y"]).max() + 1e-6) * std + 1e-6 * np.abs(mean)
    assert (np.abs(Y.cpu().numpy() - Yo) <= tol).all()
    # empty batch is a no-op
    Y0, _, _ = net.predict(torch.empty((0, 4), device="cuda"))
    assert Y0.shape == (0, 6)


def test_fit_target_norm():
    import torch
    rng = np.random.default_rng(8)
    Y = (rng.normal(size=(1000, 6)) * [1, 2, 3, 4, 5, 6] + [0, 1, 2, 3, 4, 5]).astype(np.float32)
    net = _net(inputs.mlp_init_params(seed=1))
    net.fit_target_norm(_dev(Y))
    torch.cuda.synchronize()
    m, s = net.target_norm()
    assert np.allclose(m, Y.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
    assert np.allclose(s, Y.astype(np.float64).std(0), rtol=1e-6)


def test_adam_training_matches_oracle():
    """One epoch of three minibatches (40, 40, 16 samples): every Adam step of
    the kernels against the oracle's gradient + Adam (Kingma & Ba, Alg. 1).
    Where a gradient entry is within the gradient tolerance of zero its sign,
    hence its first Adam update (~lr * sign), is not determined by the
    arithmetic: those entries are only bounded by the step size."""
    rng = np.random.default_rng(31)
    p0 = inputs.mlp_init_params(seed=7).astype(np.float64)
    n, batch, lr = 96, 40, 1e-3
    X = _bf16_inputs(rng, n)
    Y = rng.normal(size=(n, 6)).astype(np.float32)
    net = _net(p0.astype(np.float32), lr=lr)
    hist = net.train(_dev(X), _dev(Y), epochs=1, batch=batch)
    pg = net.params().astype(np.float64)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    sure = np.ones(p0.size, bool)
    loss_sum = 0.0
    t = 0
    for b0 in range(0, n, batch):
        xb, yb = X[b0:b0 + batch], Y[b0:b0 + batch]
        # the oracle's parameters are carried in FP32 like the kernel's
        lo, g = om.loss_and_grad(p, xb, yb, bf16_ops=True)
        loss_sum += lo * len(xb)
        for _, a, b in BLOCKS:
            sure[a:b] &= np.abs(g[a:b]) > 2e-2 * np.abs(g[a:b]).max()
        t += 1
        p, m, v = om.adam_step(p, g, m, v, t, lr=lr)
        p = p.astype(np.float32).astype(np.float64)
    assert abs(hist[0] - loss_sum / n) <= 1e-5 * loss_sum / n
    d = np.abs(pg - p)
    assert sure.mean() > 0.4
    assert d[sure].max() <= 5e-2 * lr, d[sure].max()
    assert d.max() <= 2 * lr * t + 1e-6


def test_training_is_deterministic_and_learns():
    """A smooth 4 -> 6 map is learnt (loss falls by 10x); two trainings from the
    same start give bit-identical parameters (fixed-order gradient sums)."""
    rng = np.random.default_rng(4)
    n = 4096
    X = rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    Y = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.cos(X[:, 1] + X[:, 2]), X[:, 3] ** 2,
                  X[:, 0] * X[:, 3], np.tanh(3 * X[:, 2]), X.sum(1) / 4], axis=1).astype(np.float32)
    p0 = inputs.mlp_init_params(seed=3)
    outs = []
    for _ in range(2):
        net = _net(p0, lr=3e-3)
        Yd = _dev(Y)
        net.fit_target_norm(Yd)
        hist = net.train(_dev(X), Yd, epochs=30, batch=256)
        outs.append((hist, net.params()))
    hist, pa = outs[0]
    assert hist[-1] < 0.1 * hist[0], hist
    assert np.array_equal(pa, outs[1][1])
    assert np.array_equal(hist, outs[1][0])


def test_invalid_arguments():
    import torch

    from paper_2311_13337_amd import vadx
    p = inputs.mlp_init_params(seed=1)
    with pytest.raises(vadx.VadxError):
        vadx.Mlp(p, (0, 0, 0, 0), (1, 1, 0, 1))          # empty input range
    bad = p.copy()
    bad[3] = np.nan
    with pytest.raises(vadx.VadxError):
        vadx.Mlp(bad, (0, 0, 0, 0), (1, 1, 1, 1))
    net = _net(p)
    X = torch.zeros((8, 4), device="cuda")
    with pytest.raises(vadx.VadxError):
        net.predict(X, score_outputs=(0, 6))
    with pytest.raises(vadx.VadxError):
        net.set_target_norm(np.zeros(6), np.zeros(6))
    with pytest.raises(vadx.VadxError):
        net.train(X, torch.zeros((8, 6), device="cuda"), epochs=1, batch=0)
