"""Inputs for the MLP checks (test helper).

exact_case(N, seed): parameters, features and targets on which every value
the BF16/FP32 network forms is exact -- BF16 operands with a few bits, hidden
units with two nonzero inputs each, targets set so that out - y is a small
dyadic multiple of N's odd part -- so the products, every FP32 sum and every
BF16 rounding are exact, whatever the summation order.  On these inputs the
rounded network equals the real-valued one bit for bit, and a GPU evaluation
must equal the FP64 reference bit for bit.
"""
import numpy as np

from oracle import mlp_oracle as M


def _odd_part(N):
    while N % 2 == 0:
        N //= 2
    return N


def exact_case(N, seed):
    rng = np.random.default_rng(seed)
    IN, H = M.IN, M.H
    P = np.zeros(M.NPARAM)
    W1 = np.zeros((IN, H))
    for h in range(H):
        a, b = rng.choice(IN, size=2, replace=False)
        W1[a, h], W1[b, h] = rng.choice([-1.0, -0.5, -0.25, 0.25, 0.5, 1.0], size=2)
    W2 = np.zeros((H, H))
    p1, p2 = rng.permutation(H), rng.permutation(H)
    for o in range(H):
        i1, i2 = p1[o], p2[o]
        if i2 == i1:
            i2 = (i2 + 1) % H
        W2[i1, o], W2[i2, o] = rng.choice([-1.0, -0.5, 0.5, 1.0], size=2)
    P[M.OFF_W1:M.OFF_B1] = W1.ravel()
    P[M.OFF_B1:M.OFF_W2] = rng.choice([-0.125, 0.0, 0.125, 0.25], size=H)
    P[M.OFF_W2:M.OFF_B2] = W2.ravel()
    P[M.OFF_B2:M.OFF_W3] = rng.choice([-0.25, -0.0625, 0.0, 0.0625, 0.25], size=H)
    P[M.OFF_W3:M.OFF_B3] = rng.choice([-0.5, -0.25, 0.25, 0.5], size=H)
    P[M.OFF_B3] = 0.25
    F = rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], size=(N, IN))
    out, _ = M.forward(P, F, bf=False)
    e = _odd_part(N) * rng.choice([-2.0, -1.0, 1.0, 2.0], size=N) * 2.0 ** -6
    y = out - e
    return P.astype(np.float32), F.astype(np.float32), y.astype(np.float32)


def fp32_eval(P, F, y):
    """The rounded network evaluated in numpy FP32 (BLAS accumulation order):
    an evaluation independent of the FP64 reference, for checking its
    intervals.  Returns (out, grad, loss)."""
    f32 = np.float32
    b = lambda a: M.bf16(a).astype(f32)                  # noqa: E731
    W1, b1, W2, b2, W3, b3 = (np.asarray(x, dtype=f32) for x in M.unpack(P))
    Fr, W1r, W2r, W3r = b(F), b(W1), b(W2), b(W3)
    y = np.asarray(y, dtype=f32)
    N = len(y)
    h1 = b(np.maximum(Fr @ W1r + b1, 0))
    h2 = b(np.maximum(h1 @ W2r + b2, 0))
    out = h2 @ W3r + b3
    d = (f32(2) * (out - y)) / f32(N)
    g = np.zeros(M.NPARAM, dtype=f32)
    g[M.OFF_W3:M.OFF_B3] = h2.T @ d
    g[M.OFF_B3] = d.sum()
    dh2 = b(np.where(h2 > 0, d[:, None] * W3r[None, :], f32(0)))
    g[M.OFF_W2:M.OFF_B2] = (h1.T @ dh2).ravel()
    g[M.OFF_B2:M.OFF_W3] = dh2.sum(0)
    dh1 = b(np.where(h1 > 0, dh2 @ W2r.T, f32(0)))
    g[M.OFF_B1:M.OFF_W2] = dh1.sum(0)
    g[M.OFF_W1:M.OFF_B1] = (Fr.T @ dh1).ravel()
    loss = ((out - y) ** 2).sum() / f32(N)
    return out, g, loss
