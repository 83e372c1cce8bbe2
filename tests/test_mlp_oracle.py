"""Pins of the FP64 reference of the learned-correction network: bfloat16
rounding against its definition and torch's own conversion, GELU against the
normal CDF, the hand-written backward pass against central finite
differences, and the first Adam step against its closed form."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
import workloads as W


def test_bf16_round_ties_to_even_and_matches_torch():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, math.pi, -2.5e-3, 65504.0, 0.0], dtype=np.float32)
    r = M.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # halfway, ties to the even mantissa
    assert r[2] == 1 + 2 ** -6         # halfway, the odd neighbour loses
    assert r[3] == 3.140625
    assert r[6] == 0.0
    import torch
    u = (W.uniform(7, np.arange(4096)) * 2 - 1) * 10.0 ** (W.uniform(8, np.arange(4096)) * 8 - 4)
    u = u.astype(np.float32)
    ref = torch.from_numpy(u).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(u), ref)


def test_gelu_is_x_times_normal_cdf():
    from scipy.stats import norm
    x = np.linspace(-6, 6, 241)
    assert np.allclose(M.gelu(x), x * norm.cdf(x), rtol=0, atol=1e-15)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_d(x), fd, rtol=0, atol=1e-8)


def _net(seed, dims):
    shapes = [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]
    parts = []
    k = 0
    for (o, i) in shapes:
        u = W.uniform(seed, k + np.arange(o * i + o))
        k += o * i + o
        parts.append((2 * u - 1) * np.sqrt(3.0 / i))
    p = np.concatenate(parts)
    return M.bf16_round(p.astype(np.float32)), shapes   # bf16-representable: rounding is the identity


@pytest.mark.parametrize("dims", [(5, 7, 3), (9, 6, 6, 2)])
def test_backward_matches_central_differences(dims):
    p, shapes = _net(3, dims)
    B = 11
    X = W.uniform(4, np.arange(B * dims[0])).reshape(B, dims[0]) * 2 - 1
    T = W.uniform(5, np.arange(B * dims[-1])).reshape(B, dims[-1])
    loss, g = M.loss_and_grad(p, shapes, X, T)
    assert loss == pytest.approx(M.loss_only(p, shapes, X, T))
    h = 1e-6
    fd = np.empty_like(g)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (M.loss_only(p + e, shapes, X, T) - M.loss_only(p - e, shapes, X, T)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_forward_uses_rounded_weights():
    p, shapes = _net(9, (4, 5, 2))
    q = p * (1 + 2.0 ** -10)     # within half a bf16 step of p (the step is >= 2^-8 relative)
    X = W.uniform(10, np.arange(12)).reshape(3, 4)
    # weights of q round back to those of p; biases are not rounded
    mixed = q.copy()
    k = 0
    for (o, i) in shapes:
        mixed[k:k + o * i] = p[k:k + o * i]
        k += o * i + o
    y1, _ = M.forward(q, shapes, X)
    y2, _ = M.forward(mixed, shapes, X, round_weights=False)
    assert np.array_equal(y1, y2)
    y3, _ = M.forward(q, shapes, X, round_weights=False)
    assert not np.array_equal(y1, y3)


def test_first_adam_step_is_lr_times_sign():
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    p0 = np.zeros(4)
    p1, m, v = M.adam(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    # m_hat = g, v_hat = g^2: the update is lr * g / (|g| + eps)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    assert p1[3] == 0.0
    # constant gradient: m_hat = g and v_hat = g^2 at every step
    p, m, v = p0, np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        p, m, v = M.adam(p, g, m, v, t, lr=0.01, eps=0.0 + 1e-30)
    assert np.allclose(p[:3], -0.05 * np.sign(g[:3]), rtol=1e-12)
