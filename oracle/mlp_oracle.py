"""FP64 reference of the candidate ranker's MLP (32 -> 128 -> 128 -> 1).

TEST INFRASTRUCTURE: only tests/ import this module.  It mirrors the
rounding points of the library's BF16 matrix products (inputs to each
product rounded to nearest-even BF16, products and sums exact in FP64);
with bf16=False it is the plain real-valued network, whose gradient the
tests pin with central finite differences.

Parameter layout (flat vector): W1[32][128], b1[128], W2[128][128], b2[128],
W3[128], b3.  Loss = mean_r (out_r - y_r)^2.
"""
import numpy as np

IN, H = 32, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + IN * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1


def bf16(x):
    """Round to FP32, then to BF16 (round to nearest, ties to even)."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[OFF_W1:OFF_B1].reshape(IN, H), P[OFF_B1:OFF_W2], P[OFF_W2:OFF_B2].reshape(H, H),
            P[OFF_B2:OFF_W3], P[OFF_W3:OFF_B3], P[OFF_B3])


def forward(P, F, bf=True):
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    F = np.asarray(F, dtype=np.float64)
    a1 = r(F) @ r(W1) + b1
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ r(W2) + b2
    h2 = r(np.maximum(a2, 0.0))
    out = h2 @ r(W3) + b3
    return out, (F, a1, h1, a2, h2)


def loss_and_grad(P, F, y, bf=True):
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    out, (F, a1, h1, a2, h2) = forward(P, F, bf)
    y = np.asarray(y, dtype=np.float64)
    N = len(y)
    d = 2.0 * (out - y) / N
    loss = float(np.sum((out - y) ** 2) / N)
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ d
    g[OFF_B3] = d.sum()
    mask2 = (h2 > 0) if bf else (a2 > 0)
    dh2 = r(d[:, None] * r(W3)[None, :] * mask2)
    g[OFF_W2:OFF_B2] = (h1.T @ dh2).reshape(-1)
    g[OFF_B2:OFF_W3] = dh2.sum(0)
    mask1 = (h1 > 0) if bf else (a1 > 0)
    dh1 = r((dh2 @ r(W2).T) * mask1)
    g[OFF_B1:OFF_W2] = dh1.sum(0)
    g[OFF_W1:OFF_B1] = (r(F).T @ dh1).reshape(-1)
    return loss, g


def adam(P, m1, m2, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mh = m1 / (1 - beta1 ** step)
    vh = m2 / (1 - beta2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m1, m2
