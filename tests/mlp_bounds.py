"""Element-wise error bounds of the learned-flag network's gradient between a
bf16/fp32 implementation and the oracle's fp64 network with the same bf16
rounding points (test helper).

The forward inputs are built so that every forward sum is exact in fp32 (all
operands on coarse binary grids, sums of absolute values below the fp32
exactness limit): both sides then hold the same Z1, H1, Z2, H2 and logits.
The backward differs: the output-layer error dz comes from an fp32 sigmoid
against fp64, and the GEMMs accumulate in fp32 in an order of their own.
With u = 2^-24 and gamma_n = n u / (1 - n u) (the bound of any order of an
fp32 sum of n terms relative to the sum of their absolute values), the
propagated bounds are:

  dz:     |d dz| <= 16 u (pw + 1) / n + 16 u |dz|              (fp32 sigmoid)
  dZ2 = dz w3 [H2 > 0] before rounding: |d| <= |w3| |d dz| + u |dZ2|
  dZ2r = bf16(dZ2): either side may round to either neighbour when the
          interval dZ2 +- bound straddles a rounding boundary; the difference
          is then at most the distance between the two candidates
  dH1 = dZ2r W2^T:   |d| <= sum_j |d dZ2r| |W2| + gamma_128 sum_j |dZ2r W2|
  dZ1r = bf16(dH1 [H1 > 0]) likewise
  grad = A^T B:      |d| <= sum_b |A| |d B| + gamma_n sum_b |A B|   (A exact)
  bias = sum_b B:    |d| <= sum_b |d B| + gamma_n sum_b |B|
"""
import numpy as np

from oracle import mlp

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def exact_problem(n, seed):
    """Inputs x [n, 512] (fp32), labels y, fp32 parameters with every forward
    sum exact in fp32 (asserted)."""
    g = np.random.default_rng(seed)
    x = (g.integers(-16, 17, (n, mlp.IN)) / 16.0).astype(np.float32)
    p = np.zeros(mlp.NPARAM, dtype=np.float32)
    p[mlp.OFF_W1:mlp.OFF_B1] = g.integers(-16, 17, mlp.IN * mlp.HID) / 128.0
    p[mlp.OFF_B1:mlp.OFF_W2] = g.integers(-200, 201, mlp.HID) / 2048.0
    p[mlp.OFF_W2:mlp.OFF_B2] = g.integers(-4, 5, mlp.HID * mlp.HID) / 16.0
    p[mlp.OFF_B2:mlp.OFF_W3] = g.integers(-3000, 3001, mlp.HID) / 32768.0
    p[mlp.OFF_W3:mlp.OFF_B3] = g.integers(-2, 3, mlp.HID) / 64.0
    p[mlp.OFF_B3] = 37.0 / 2.0 ** 19
    y = (g.uniform(size=n) < 0.4).astype(np.uint8)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    X = x.astype(np.float64)
    # exactness: operand grids 2^-4 * 2^-7 = 2^-11 (layer 1), 2^-11 * 2^-4 =
    # 2^-15 (layer 2), 2^-15 * 2^-6 = 2^-21 (head); partial sums stay exact while
    # the sum of absolute values is below 2^(24 - grid exponent)
    assert (np.abs(X) @ np.abs(W1) + np.abs(b1)).max() < 2.0 ** (24 - 11)
    H1 = mlp.bf16(np.maximum(X @ W1 + b1, 0.0))
    assert np.all(H1 * 2.0 ** 11 == np.round(H1 * 2.0 ** 11))
    assert (H1 @ np.abs(W2) + np.abs(b2)).max() < 2.0 ** (24 - 15)
    H2 = mlp.bf16(np.maximum(H1 @ W2 + b2, 0.0))
    assert np.all(H2 * 2.0 ** 15 == np.round(H2 * 2.0 ** 15))
    assert (H2 @ np.abs(w3) + abs(b3)).max() < 2.0 ** (24 - 21)
    assert H1.any() and H2.any()
    return x, y, p


def _bf16_interval_err(P, d, R):
    """Largest |candidate - R| over the bf16 roundings of values in [P - d, P + d]."""
    lo, hi = mlp.bf16(P - d), mlp.bf16(P + d)
    return np.maximum(np.abs(lo - R), np.abs(hi - R))


def gradient_bound(x, y, p, pw):
    """(oracle gradient, element-wise bound of |gpu - oracle|, ambiguous counts)."""
    n = len(y)
    loss, g = mlp.loss_and_grad(x.astype(np.float64), y, p.astype(np.float64), pw)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    z, prob, (X, H1, H2) = mlp.forward(x.astype(np.float64), p.astype(np.float64))
    yy = np.asarray(y, dtype=np.float64)
    dz = (prob * (pw * yy + 1.0 - yy) - pw * yy) / n
    d_dz = 16.0 * U32 * (pw + 1.0) / n + 16.0 * U32 * np.abs(dz)
    w3r, W2r = mlp.bf16(w3), mlp.bf16(W2)
    m2 = H2 > 0.0
    P2 = np.outer(dz, w3r) * m2
    d_P2 = (np.outer(d_dz, np.abs(w3r)) + U32 * np.abs(P2)) * m2
    R2 = mlp.bf16(P2)
    e_R2 = _bf16_interval_err(P2, d_P2, R2)
    P1 = (R2 @ W2r.T) * (H1 > 0.0)
    d_P1 = (e_R2 @ np.abs(W2r).T + gamma(mlp.HID) * (np.abs(R2) @ np.abs(W2r).T)) * (H1 > 0.0)
    R1 = mlp.bf16(P1)
    e_R1 = _bf16_interval_err(P1, d_P1, R1)
    gn = gamma(n)
    b = np.zeros(mlp.NPARAM)
    b[mlp.OFF_W3:mlp.OFF_B3] = H2.T @ d_dz + gn * (H2.T @ np.abs(dz))
    b[mlp.OFF_B3] = d_dz.sum() + gn * np.abs(dz).sum()
    b[mlp.OFF_B2:mlp.OFF_W3] = d_P2.sum(axis=0) + gn * np.abs(P2).sum(axis=0)
    b[mlp.OFF_W2:mlp.OFF_B2] = (H1.T @ e_R2 + gn * (H1.T @ np.abs(R2))).ravel()
    b[mlp.OFF_B1:mlp.OFF_W2] = d_P1.sum(axis=0) + gn * np.abs(P1).sum(axis=0)
    b[mlp.OFF_W1:mlp.OFF_B1] = (np.abs(X).T @ e_R1 + gn * (np.abs(X).T @ np.abs(R1))).ravel()
    amb = dict(dZ2=int((e_R2 > 0).sum()), dZ1=int((e_R1 > 0).sum()))
    return g, b, amb, loss


def fp32_emulation(x, y, p, pw, seed):
    """The gradient computed the way the GPU path computes it, in float32 with
    shuffled summation orders (a stand-in for MFMA accumulation; CPU check of
    the bound)."""
    f = np.float32
    rng = np.random.default_rng(seed)
    n = len(y)
    W1, b1, W2, b2, w3, b3 = [np.asarray(a, dtype=np.float64) for a in mlp.unpack(p)]
    bf = lambda a: mlp.bf16(np.asarray(a, dtype=np.float32)).astype(np.float32)
    X = bf(x)
    H1 = bf(np.maximum((X.astype(np.float64) @ bf(W1) + b1).astype(np.float32), 0))
    H2 = bf(np.maximum((H1.astype(np.float64) @ bf(W2) + b2).astype(np.float32), 0))
    z = (H2.astype(np.float64) @ bf(w3) + b3).astype(np.float32)
    prob = (f(1) / (f(1) + np.exp(-z))).astype(np.float32)
    yy = y.astype(np.float32)
    dz = ((prob * (f(pw) * yy + f(1) - yy) - f(pw) * yy) / f(n)).astype(np.float32)

    def sum32(terms, axis):
        terms = np.moveaxis(np.asarray(terms, dtype=np.float32), axis, 0)
        order = rng.permutation(terms.shape[0])
        acc = np.zeros(terms.shape[1:], dtype=np.float32)
        for q in order:
            acc = (acc + terms[q]).astype(np.float32)
        return acc

    g = np.zeros(mlp.NPARAM, dtype=np.float32)
    g[mlp.OFF_W3:mlp.OFF_B3] = sum32(H2 * dz[:, None], 0)
    g[mlp.OFF_B3] = sum32(dz[:, None], 0)[0]
    dZ2 = (dz[:, None] * bf(w3)[None, :] * (H2 > 0)).astype(np.float32)
    g[mlp.OFF_B2:mlp.OFF_W3] = sum32(dZ2, 0)
    dZ2b = bf(dZ2)
    g[mlp.OFF_W2:mlp.OFF_B2] = sum32(H1[:, :, None] * dZ2b[:, None, :], 0).ravel()
    dH1 = sum32(dZ2b[:, None, :] * bf(W2)[None, :, :], 2)
    dZ1 = (dH1 * (H1 > 0)).astype(np.float32)
    g[mlp.OFF_B1:mlp.OFF_W2] = sum32(dZ1, 0)
    dZ1b = bf(dZ1)
    g[mlp.OFF_W1:mlp.OFF_B1] = sum32(X[:, :, None] * dZ1b[:, None, :], 0).ravel()
    return g
