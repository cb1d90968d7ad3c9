"""FP64 reference of the scatter-surrogate network (test infrastructure).

Network 8 -> 128 -> 128 -> 128 -> 1 with GELU in its tanh form
    gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
(Hendrycks and Gimpel, "Gaussian Error Linear Units", 2016), linear output,
mean-squared-error loss, and Adam with bias correction (Kingma and Ba,
"Adam: a method for stochastic optimization", ICLR 2015).

With ``bf16_round=True`` the passes round to bfloat16 (round to nearest
even) exactly where the GPU kernels do: the inputs and weights of every
matrix product, the activations fed to the next product and, backward, the
layer deltas.
"""
from __future__ import annotations

import numpy as np

C_GELU = np.sqrt(2.0 / np.pi)
A_GELU = 0.044715
LAYERS = 4


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returns float64."""
    f = np.ascontiguousarray(x, np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return (b.astype(np.uint32)).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(C_GELU * (x + A_GELU * x ** 3)))


def gelu_grad(x):
    u = C_GELU * (x + A_GELU * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * C_GELU * (1.0 + 3.0 * A_GELU * x * x)


def _w(p, k, rnd):
    w = np.asarray(p[k], np.float64)
    return bf16(w) if rnd else w


def forward(p: dict, X: np.ndarray, bf16_round: bool = False):
    """y = W4^T gelu(W3^T gelu(W2^T gelu(W1^T x + b1) + b2) + b3) + b4 per row of X.
    Returns (y, cache)."""
    h = np.asarray(X, np.float64)
    if bf16_round:
        h = bf16(h)
    cache = {"h0": h}
    for i in range(1, LAYERS):
        z = h @ _w(p, f"W{i}", bf16_round) + np.asarray(p[f"b{i}"], np.float64)
        h = gelu(z)
        if bf16_round:
            h = bf16(h)
        cache[f"z{i}"] = z
        cache[f"h{i}"] = h
    y = h @ _w(p, "W4", bf16_round)[:, 0] + float(p["b4"][0])
    return y, cache


def backward(p: dict, cache: dict, dy: np.ndarray, bf16_round: bool = False) -> dict:
    """Gradients of sum_b dy_b y_b with respect to every parameter."""
    dy = np.asarray(dy, np.float64)
    g = {}
    h3 = cache["h3"]
    g["W4"] = (h3.T @ dy)[:, None]
    g["b4"] = np.array([dy.sum()])
    dh = np.outer(dy, _w(p, "W4", bf16_round)[:, 0])
    for i in range(LAYERS - 1, 0, -1):
        d = dh * gelu_grad(cache[f"z{i}"])
        if bf16_round:
            d = bf16(d)
        g[f"W{i}"] = cache[f"h{i - 1}"].T @ d
        g[f"b{i}"] = d.sum(axis=0)
        if i > 1:
            dh = d @ _w(p, f"W{i}", bf16_round).T
    return g


def mse(y: np.ndarray, t: np.ndarray):
    """loss = mean((y - t)^2) and its gradient with respect to y."""
    r = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float, b1=0.9, b2=0.999,
              eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    p2, m2, v2 = {}, {}, {}
    for k in p:
        m2[k] = b1 * m[k] + (1 - b1) * g[k]
        v2[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m2[k] / (1 - b1 ** step)
        vh = v2[k] / (1 - b2 ** step)
        p2[k] = np.asarray(p[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p2, m2, v2
