"""The element-wise gradient bound of the learned-flag network (mlp_bounds)
holds for an fp32 computation of the gradient in shuffled summation orders
(the GPU path's arithmetic, emulated on the CPU), is tight where no bf16
rounding is ambiguous, and fails a gradient computed with a transposed
operand or a dropped ReLU mask."""
import numpy as np
import pytest

import mlp_bounds as mb
from oracle import mlp


@pytest.mark.parametrize("n", [1, 37, 120])
def test_fp32_gradient_within_the_bound(n):
    x, y, p = mb.exact_problem(n, seed=n)
    g, bound, amb, _ = mb.gradient_bound(x, y, p, 2.5)
    got = mb.fp32_emulation(x, y, p, 2.5, seed=3)
    err = np.abs(got.astype(np.float64) - g)
    assert np.all(err <= bound), (np.argmax(err - bound), amb)
    # the bound is a small fraction of each group's scale
    for a, b in ((mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_W2, mlp.OFF_B2), (mlp.OFF_W3, mlp.OFF_B3)):
        assert np.median(bound[a:b]) <= 1e-3 * np.abs(g[a:b]).max()


def test_bound_catches_planted_mistakes():
    n = 37
    x, y, p = mb.exact_problem(n, seed=5)
    g, bound, _, _ = mb.gradient_bound(x, y, p, 2.5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    # a transposed W2 in the backward pass (dH1 = dZ2 W2 instead of dZ2 W2^T)
    p_t = p.copy()
    p_t[mlp.OFF_W2:mlp.OFF_B2] = W2.T.ravel()
    got = mb.fp32_emulation(x, y, p, 2.5, seed=3)
    bad = got.copy()
    bad_W1 = mb.fp32_emulation(x, y, p_t, 2.5, seed=3)[mlp.OFF_W1:mlp.OFF_B1]
    bad[mlp.OFF_W1:mlp.OFF_B1] = bad_W1
    assert np.any(np.abs(bad - g) > bound)
    # one row of the W1 gradient off by 1 %
    bad = got.copy().astype(np.float64)
    row = slice(mlp.OFF_W1 + 7 * mlp.HID, mlp.OFF_W1 + 8 * mlp.HID)
    bad[row] *= 1.01
    assert np.any(np.abs(bad - g) > bound)
