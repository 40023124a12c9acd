"""Reference of the learned refinement-flag network (test infrastructure only).

A per-block network predicts whether the plain criterion will ask for
refinement.  Inputs: the 8 primitive variables (log10 rho, v_r, v_theta,
v_phi, log10 p, B_r, B_theta, B_phi; code units) averaged over each of the
4 x 4 x 4 sub-cubes of the block, order [primitive][k][j][i], z-scored per
input.  Layers 512 -> 128 (ReLU) -> 128 (ReLU) -> 1 (sigmoid); loss: mean
binary cross-entropy with the positive class weighted by pos_weight; Adam.

With ``bf16=True`` the reference rounds to bfloat16 (nearest even, via
float32) exactly where the GPU path does: inputs, W1, W2, w3, the hidden
activations, and dZ2, dZ1 where they enter products; everything else is
fp64.  With ``bf16=False`` it is the plain fp64 network (finite-difference
pins).  Parameter vector layout: W1[512][128] (input-major), b1, W2[128][128],
b2, w3[128], b3.
"""
import numpy as np

from .boundary import cons_to_prims

IN, HID = 512, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + IN * HID
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + HID
NPARAM = OFF_B3 + 1


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return ((u << 16).astype(np.uint32)).view(np.float32).astype(np.float64)


def features(U, gamma):
    """Un-normalised inputs of one block U[8, bk, bj, bi] -> float32[512]."""
    W = cons_to_prims(U, gamma)
    nk, nj, ni = U.shape[1:]
    pk, pj, pi = nk // 4, nj // 4, ni // 4
    out = np.zeros(IN, dtype=np.float32)
    for v in range(8):
        for k in range(4):
            for j in range(4):
                for i in range(4):
                    m = W[v, k * pk:(k + 1) * pk, j * pj:(j + 1) * pj, i * pi:(i + 1) * pi].mean()
                    if v in (0, 4):
                        m = np.log10(m)
                    out[v * 64 + k * 16 + j * 4 + i] = np.float32(m)
    return out


def normalise(raw, mean, std):
    """(raw - mean) / std in float32 arithmetic, as the GPU does it."""
    raw = np.asarray(raw, dtype=np.float32)
    istd = np.float32(1.0) / np.asarray(std, dtype=np.float32)
    return (raw - np.asarray(mean, dtype=np.float32)) * istd


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(IN, HID), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(HID, HID),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def forward(x, p, bf16_round=True):
    """Logits, probabilities and the activations of rows x (normalised, [n, 512])."""
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = r(x)
    Z1 = X @ r(W1) + b1
    H1 = r(np.maximum(Z1, 0.0))
    Z2 = H1 @ r(W2) + b2
    H2 = r(np.maximum(Z2, 0.0))
    z = H2 @ r(w3) + b3
    prob = 1.0 / (1.0 + np.exp(-z))
    return z, prob, (X, H1, H2)


def loss_and_grad(x, y, p, pos_weight, bf16_round=True):
    """Mean weighted BCE and its gradient (parameter layout)."""
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(p)
    n = len(y)
    y = np.asarray(y, dtype=np.float64)
    z, prob, (X, H1, H2) = forward(x, p, bf16_round)
    log_p = -np.logaddexp(0.0, -z)
    log_q = -np.logaddexp(0.0, z)
    loss = float(np.mean(-(pos_weight * y * log_p + (1.0 - y) * log_q)))
    dz = (prob * (pos_weight * y + 1.0 - y) - pos_weight * y) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = H2.T @ dz
    g[OFF_B3] = dz.sum()
    dZ2 = np.outer(dz, r(w3)) * (H2 > 0.0)
    g[OFF_B2:OFF_W3] = dZ2.sum(axis=0)
    dZ2r = r(dZ2)
    g[OFF_W2:OFF_B2] = (H1.T @ dZ2r).ravel()
    dH1 = dZ2r @ r(W2).T
    dZ1 = dH1 * (H1 > 0.0)
    g[OFF_B1:OFF_W2] = dZ1.sum(axis=0)
    g[OFF_W1:OFF_B1] = (X.T @ r(dZ1)).ravel()
    return loss, g


def adam_step(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on p, m1, m2); t counts from 1."""
    m1[:] = b1 * m1 + (1.0 - b1) * g
    m2[:] = b2 * m2 + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return p
