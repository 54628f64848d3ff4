"""Plain FP64 reference of the surrogate MLP (4 -> 128 -> 128 -> 6, GELU).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg). Shares no
code with the GPU library.

The surrogate maps a sweep point (S, b_e, a_e, v), min-max scaled to [-1, 1],
to z-scored FC and rate statistics. Every matrix-product operand is rounded to
bfloat16 (round to nearest even) at the same points as the GPU kernels, and the
products and everything else are evaluated in FP64 here; with ``bf16=False``
the network is exact FP64 (used to pin this code against torch.autograd and
finite differences).

Parameter vector layout (17926 floats): W1 [128, 4], b1 [128], W2 [128, 128],
b2 [128], W3 [6, 128], b3 [6], each row-major, concatenated in that order.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

DIMS = (4, 128, 128, 6)
SHAPES = (("W1", (128, 4)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
          ("W3", (6, 128)), ("b3", (6,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.ascontiguousarray(x, np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, np.float64)


def forward(p, X, bf16_ops=True):
    """Returns dict with Z1, H1, Z2, H2, Y for inputs X [n, 4]."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    Z1 = _r(X, bf16_ops) @ _r(w["W1"], bf16_ops).T + w["b1"]
    H1 = gelu(Z1)
    Z2 = _r(H1, bf16_ops) @ _r(w["W2"], bf16_ops).T + w["b2"]
    H2 = gelu(Z2)
    Y = _r(H2, bf16_ops) @ _r(w["W3"], bf16_ops).T + w["b3"]
    return {"X": X, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2, "Y": Y}


def loss_and_grad(p, X, T, bf16_ops=True, n_total=None):
    """MSE over the batch and the 6 outputs (normalised by n_total x 6, n_total
    defaulting to the batch size) and its gradient with respect to p."""
    w = unpack(p)
    f = forward(p, X, bf16_ops)
    n = X.shape[0] if n_total is None else n_total
    D = f["Y"] - np.asarray(T, np.float64)
    loss = float((D * D).sum() / (n * DIMS[3]))
    dY = 2.0 * D / (n * DIMS[3])
    g = {}
    g["W3"] = _r(dY, bf16_ops).T @ _r(f["H2"], bf16_ops)
    g["b3"] = dY.sum(0)
    dH2 = _r(dY, bf16_ops) @ _r(w["W3"], bf16_ops)
    dZ2 = dH2 * gelu_grad(f["Z2"])
    g["W2"] = _r(dZ2, bf16_ops).T @ _r(f["H1"], bf16_ops)
    g["b2"] = dZ2.sum(0)
    dH1 = _r(dZ2, bf16_ops) @ _r(w["W2"], bf16_ops)
    dZ1 = dH1 * gelu_grad(f["Z1"])
    g["W1"] = _r(dZ1, bf16_ops).T @ _r(f["X"], bf16_ops)
    g["b1"] = dZ1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def input_jacobian(p, X, bf16_ops=True):
    """dY/dX [n, 6, 4] by forward-mode tangents: T1 = g1' * W1, T2 = g2' * (W2 T1),
    J = W3 T2, with the matrix-product operands rounded like the kernels."""
    w = unpack(p)
    f = forward(p, X, bf16_ops)
    W1 = _r(w["W1"], bf16_ops)
    T1 = gelu_grad(f["Z1"])[:, :, None] * W1[None, :, :]              # [n, 128, 4]
    T2 = gelu_grad(f["Z2"])[:, :, None] * np.einsum(
        "ij,njk->nik", _r(w["W2"], bf16_ops), _r(T1, bf16_ops))         # [n, 128, 4]
    return np.einsum("ij,njk->nik", _r(w["W3"], bf16_ops), _r(T2, bf16_ops))
