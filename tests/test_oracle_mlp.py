"""Pins of the FP64 surrogate-network reference: central finite differences,
GELU limits and closeness to the exact erf form, Adam's first step in closed
form, and bfloat16 rounding on exactly representable and tie values."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import mlp as M
import synth


def test_gelu_limits_and_erf_form():
    x = np.linspace(-6, 6, 2001)
    exact = 0.5 * x * (1 + special.erf(x / math.sqrt(2)))
    assert np.max(np.abs(M.gelu(x) - exact)) < 5e-4          # tanh form approximates x Phi(x)
    assert M.gelu(0.0) == 0.0
    assert M.gelu(12.0) == pytest.approx(12.0, rel=1e-12)
    assert abs(M.gelu(-12.0)) < 1e-12
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), fd, rtol=1e-6, atol=1e-8)


def test_gradients_match_central_differences():
    p = {k: v.astype(np.float64) for k, v in synth.mlp_init_params(3).items()}
    rng = np.random.default_rng(0)
    for k in p:
        p[k] = p[k] + rng.normal(scale=0.05, size=p[k].shape)     # non-zero biases too
    X = rng.normal(size=(5, 8))
    t = rng.normal(size=5)

    def loss(pp):
        y, _ = M.forward(pp, X)
        return M.mse(y, t)[0]

    y, cache = M.forward(p, X)
    _, dy = M.mse(y, t)
    g = M.backward(p, cache, dy)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].ravel()[idx] += h
            up = loss(q)
            q[k].ravel()[idx] -= 2 * h
            dn = loss(q)
            fd = (up - dn) / (2 * h)
            assert g[k].ravel()[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), (k, idx)


def test_adam_first_step_is_signed_learning_rate():
    # after one step with zero moments, m_hat = g and v_hat = g^2, so the
    # update is -lr g / (|g| + eps) = -lr sign(g) up to eps
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 2.0])}
    z = {"w": np.zeros(3)}
    p2, m2, v2 = M.adam_step(p, g, z, z, 1, lr=1e-2)
    np.testing.assert_allclose(p2["w"] - p["w"], -1e-2 * np.sign(g["w"]), rtol=1e-4)


def test_adam_minimises_a_quadratic():
    p = {"w": np.array([3.0, -4.0])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    for s in range(1, 2001):
        g = {"w": 2 * p["w"]}
        p, m, v = M.adam_step(p, g, m, v, s, lr=5e-2)
    assert np.all(np.abs(p["w"]) < 1e-2)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -7 + 2 ** -9], np.float32)
    out = M.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even gives 1;
    # 1 + 3 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: to even gives 1 + 2^-6
    np.testing.assert_array_equal(out, [1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0 + 2 ** -7])
