"""FP64 reference of the learned correction network (test infrastructure:
only the tests, the smoke check and the benchmark's CPU leg use it).

The network is not part of the paper; it is the learned form's correction of
the non-equilibrium stress (Sec. 2, Landau decomposition of T^munu) of a
coarse-angle run.  Parameters are one flat vector
[W1 (h x in), b1, ..., Wout (out x h), bout]; hidden layers use
GELU(x) = x Phi(x) with the exact normal CDF; the forward pass uses weights
rounded to bfloat16 (round to nearest even) and accumulates in FP64; the loss
is 0.5/B sum (y - t)^2 and its gradient is taken with respect to the rounded
weights (straight-through).  Adam follows Kingma and Ba (2015), Algorithm 1.
"""
import math

import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _erf(x):
    return np.vectorize(math.erf)(x)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_d(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def unpack(p, shapes):
    out, k = [], 0
    for (o, i) in shapes:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    return out


def forward(p, shapes, X, round_weights=True):
    """Returns outputs and the per-layer (input, pre-activation) lists."""
    layers = unpack(np.asarray(p, dtype=np.float64), shapes)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        Wr = bf16_round(W.astype(np.float32)) if round_weights else W
        z = a @ Wr.T + b
        cache.append((a, z, Wr))
        a = z if li == len(layers) - 1 else gelu(z)
    return a, cache


def loss_and_grad(p, shapes, X, T):
    """0.5/B sum (y - t)^2 and its gradient w.r.t. the flat parameters."""
    y, cache = forward(p, shapes, X)
    B = y.shape[0]
    d = (y - T) / B
    loss = 0.5 * np.sum((y - T) ** 2) / B
    grads = []
    for li in range(len(cache) - 1, -1, -1):
        a, z, Wr = cache[li]
        if li != len(cache) - 1:
            d = d * gelu_d(z)
        grads.append((d.T @ a, d.sum(axis=0)))
        d = d @ Wr
    g = []
    for (gW, gb) in reversed(grads):
        g.append(gW.ravel())
        g.append(gb)
    return loss, np.concatenate(g)


def loss_only(p, shapes, X, T, round_weights=False):
    y, _ = forward(p, shapes, X, round_weights=round_weights)
    return 0.5 * np.sum((y - T) ** 2) / y.shape[0]


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns the new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
