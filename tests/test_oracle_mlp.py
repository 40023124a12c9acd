"""Pins of the learned-flag network's reference.

- bfloat16 rounding: exact values and ties to even;
- the fp64 gradient against central finite differences;
- closed forms: a network with zero weights outputs sigmoid(b3); the loss
  gradient of a single positive example is (p - 1) pos_weight;
- the first Adam step moves every parameter with a non-zero gradient by lr
  against the gradient's sign;
- features of a uniform block are the transformed state itself.
"""
import math

import numpy as np

from oracle import boundary, mlp


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -9, 3.140625, 0.0])
    out = mlp.bf16(vals)
    assert list(out) == [1.0, 1.0, 1.0 + 4 * 2 ** -8, -2.5, 1.0, 3.140625, 0.0]


def _data(n=64, seed=0):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, mlp.IN))
    y = (g.uniform(size=n) < 0.3).astype(np.uint8)
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_W1:mlp.OFF_B1] = g.uniform(-0.1, 0.1, mlp.IN * mlp.HID)
    p[mlp.OFF_B1:mlp.OFF_W2] = g.uniform(-0.05, 0.05, mlp.HID)
    p[mlp.OFF_W2:mlp.OFF_B2] = g.uniform(-0.2, 0.2, mlp.HID * mlp.HID)
    p[mlp.OFF_B2:mlp.OFF_W3] = g.uniform(-0.05, 0.05, mlp.HID)
    p[mlp.OFF_W3:mlp.OFF_B3] = g.uniform(-0.3, 0.3, mlp.HID)
    p[mlp.OFF_B3] = 0.1
    return x, y, p


def test_gradient_matches_finite_differences():
    x, y, p = _data()
    _, g = mlp.loss_and_grad(x, y, p, 2.5, bf16_round=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.integers(mlp.OFF_W1, mlp.OFF_B1, 20), rng.integers(mlp.OFF_B1, mlp.OFF_W2, 5),
                          rng.integers(mlp.OFF_W2, mlp.OFF_B2, 20), rng.integers(mlp.OFF_B2, mlp.OFF_W3, 5),
                          rng.integers(mlp.OFF_W3, mlp.OFF_B3, 10), [mlp.OFF_B3]])
    h = 1e-6
    for q in idx:
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (mlp.loss_and_grad(x, y, pp, 2.5, False)[0] - mlp.loss_and_grad(x, y, pm, 2.5, False)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(abs(g).max(), 1e-12), (q, fd, g[q])


def test_closed_forms():
    p = np.zeros(mlp.NPARAM)
    p[mlp.OFF_B3] = 0.7
    x = np.random.default_rng(2).standard_normal((5, mlp.IN))
    z, prob, _ = mlp.forward(x, p)
    assert np.allclose(prob, 1.0 / (1.0 + math.exp(-0.7)))
    loss, g = mlp.loss_and_grad(x[:1], [1], p, 3.0)
    pr = 1.0 / (1.0 + math.exp(-0.7))
    assert abs(g[mlp.OFF_B3] - (pr - 1.0) * 3.0) < 1e-15
    assert abs(loss - 3.0 * math.log1p(math.exp(-0.7))) < 1e-15


def test_first_adam_step():
    g = np.array([0.3, -2.0, 0.0, 1e-5])
    p = np.zeros(4)
    mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=1e-3, eps=1e-8)
    assert np.allclose(p[[0, 1]], [-1e-3, 1e-3], rtol=1e-6) and p[2] == 0.0


def test_features_of_a_uniform_block():
    W = np.zeros((8, 12, 12, 12))
    vals = [3.0, 0.4, -0.01, -0.2, 0.05, 0.3, 0.0, -0.1]
    for v in range(8):
        W[v] = vals[v]
    f = mlp.features(boundary.prims_to_cons(W, 1.5), 1.5).reshape(8, 64)
    expect = list(vals)
    expect[0], expect[4] = math.log10(3.0), math.log10(0.05)
    for v in range(8):
        assert np.allclose(f[v], np.float32(expect[v]), rtol=1e-6, atol=1e-7)
