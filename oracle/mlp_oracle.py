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


# ------------------------------------------------------------------ intervals
# Bounds on what a BF16/FP32 evaluation of the same network can return.  The
# evaluation keeps the rounding points of forward() / loss_and_grad() (BF16
# operands of every matrix product, BF16 hidden activations and hidden
# gradients) but accumulates its sums in FP32, in any order and with any
# rounding mode: one FP32 rounding is at most U32 relative, and a sum of n
# terms (products exact or rounded once) is within gamma(n + 1) sum |terms| of
# the exact sum (the standard bound for recursive summation, Higham, Accuracy
# and Stability of Numerical Algorithms, Sec. 4.2).  A BF16 rounding of a
# value known only to lie in [lo, hi] lies in [bf16(lo), bf16(hi)] because
# rounding to nearest is monotone; it flips to the neighbouring BF16 value
# only when [lo, hi] holds a rounding boundary, so the bounds stay tight
# elsewhere.  ReLU masks decided by a value whose interval holds 0 take the
# hull with 0.
U32 = 2.0 ** -23


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def _pos(a):
    return np.maximum(a, 0.0)


def _neg(a):
    return np.minimum(a, 0.0)


def _widen(lo, hi, slack):
    # slack also covers the FP64 rounding of these bound computations
    s = slack * (1.0 + 2.0 ** -20) + 1e-300
    return lo - s, hi + s


def _bf_iv(lo, hi):
    return bf16(lo), bf16(hi)


def _relu_iv(lo, hi):
    return np.maximum(lo, 0.0), np.maximum(hi, 0.0)


def _mask_iv(lo, hi, act_lo, act_hi):
    """Multiply [lo, hi] by the ReLU derivative of an activation in
    [act_lo, act_hi] (act >= 0): 1 when act_lo > 0, 0 when act_hi == 0, either
    otherwise (hull with 0)."""
    one = act_lo > 0.0
    zero = act_hi <= 0.0
    lo2 = np.where(one, lo, np.where(zero, 0.0, np.minimum(lo, 0.0)))
    hi2 = np.where(one, hi, np.where(zero, 0.0, np.maximum(hi, 0.0)))
    return lo2, hi2


def _matmul_iv(Alo, Ahi, B):
    """[Alo, Ahi] @ B for a fixed matrix B: entrywise min / max of the sums."""
    Bp, Bn = _pos(B), _neg(B)
    return Alo @ Bp + Ahi @ Bn, Ahi @ Bp + Alo @ Bn


def _tmatmul_nonneg_iv(Hlo, Hhi, Dlo, Dhi):
    """[Hlo, Hhi]^T @ [Dlo, Dhi] for H >= 0: min over h of h x is h_lo x for
    x >= 0 and h_hi x for x < 0, taken at x = D_lo (and the max at D_hi)."""
    return Hlo.T @ _pos(Dlo) + Hhi.T @ _neg(Dlo), Hhi.T @ _pos(Dhi) + Hlo.T @ _neg(Dhi)


def forward_interval(P, F):
    """Per row, [lo, hi] holding the output of any FP32-accumulating
    evaluation of forward(P, F, bf=True); also the intervals of the hidden
    activations (h1lo, h1hi, h2lo, h2hi)."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    Fr, W1r, W2r, W3r = bf16(F), bf16(W1), bf16(W2), bf16(W3)
    # layer 1: 32 exact products and the bias, summed in FP32
    a1 = Fr @ W1r + b1
    lo, hi = _widen(a1, a1, _gamma(IN + 1) * (np.abs(Fr) @ np.abs(W1r) + np.abs(b1)))
    h1lo, h1hi = _bf_iv(*_relu_iv(lo, hi))
    # layer 2
    lo, hi = _matmul_iv(h1lo, h1hi, W2r)
    lo, hi = _widen(lo + b2, hi + b2, _gamma(H + 1) * (h1hi @ np.abs(W2r) + np.abs(b2)))
    h2lo, h2hi = _bf_iv(*_relu_iv(lo, hi))
    # output: 128 products (exact in FP32) and the bias, summed in FP32
    lo, hi = _matmul_iv(h2lo, h2hi, W3r)
    olo, ohi = _widen(lo + b3, hi + b3, _gamma(H + 2) * (h2hi @ np.abs(W3r) + abs(b3)))
    return olo, ohi, (h1lo, h1hi, h2lo, h2hi)


def grad_interval(P, F, y):
    """Entrywise [lo, hi] holding the gradient of mean_r (out_r - y_r)^2 that
    any FP32-accumulating evaluation of loss_and_grad(P, F, y, bf=True)
    returns, and [lo, hi] of the loss.  Sums over the rows may be split into
    tiles whose partials are added afterwards (at most N + 64 terms in any
    chain)."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    Fr, W2r, W3r = bf16(F), bf16(W2), bf16(W3)
    y = np.asarray(y, dtype=np.float64)
    N = len(y)
    gR = _gamma(N + 65)
    olo, ohi, (h1lo, h1hi, h2lo, h2hi) = forward_interval(P, F)
    # d = 2 (out - y) / N: the difference and the quotient rounded once each
    dlo, dhi = 2.0 * (olo - y) / N, 2.0 * (ohi - y) / N
    dlo, dhi = _widen(dlo, dhi, 2 * U32 * np.maximum(np.abs(dlo), np.abs(dhi)))
    dmax = np.maximum(np.abs(dlo), np.abs(dhi))
    glo, ghi = np.zeros(NPARAM), np.zeros(NPARAM)

    def put(off, lo, hi, slack):
        lo, hi = _widen(np.ravel(lo), np.ravel(hi), np.ravel(slack))
        glo[off:off + lo.size], ghi[off:off + hi.size] = lo, hi

    # dW3[h] = sum_r h2[r, h] d[r], db3 = sum_r d[r]
    lo, hi = _tmatmul_nonneg_iv(h2lo, h2hi, dlo[:, None], dhi[:, None])
    put(OFF_W3, lo, hi, gR * (h2hi.T @ dmax))
    put(OFF_B3, dlo.sum(), dhi.sum(), gR * dmax.sum())
    # dH2 = bf16(mask2 * fl32(d w3))
    p1, p2 = dlo[:, None] * W3r[None, :], dhi[:, None] * W3r[None, :]
    plo, phi = _widen(np.minimum(p1, p2), np.maximum(p1, p2), U32 * np.maximum(np.abs(p1), np.abs(p2)))
    dh2lo, dh2hi = _mask_iv(*_bf_iv(plo, phi), h2lo, h2hi)
    dh2max = np.maximum(np.abs(dh2lo), np.abs(dh2hi))
    # dW2[i][o] = sum_r h1[r, i] dH2[r, o], db2 = sum_r dH2[r]
    lo, hi = _tmatmul_nonneg_iv(h1lo, h1hi, dh2lo, dh2hi)
    put(OFF_W2, lo, hi, gR * (h1hi.T @ dh2max))
    put(OFF_B2, dh2lo.sum(0), dh2hi.sum(0), gR * dh2max.sum(0))
    # dH1 = bf16(mask1 * (dH2 W2^T))
    lo, hi = _matmul_iv(dh2lo, dh2hi, W2r.T)
    lo, hi = _widen(lo, hi, _gamma(H + 1) * (dh2max @ np.abs(W2r).T))
    dh1lo, dh1hi = _mask_iv(*_bf_iv(lo, hi), h1lo, h1hi)
    dh1max = np.maximum(np.abs(dh1lo), np.abs(dh1hi))
    # dW1[k][i] = sum_r F[r, k] dH1[r, i], db1 = sum_r dH1[r]
    put(OFF_B1, dh1lo.sum(0), dh1hi.sum(0), gR * dh1max.sum(0))
    Fp, Fn = _pos(Fr), _neg(Fr)
    lo = Fp.T @ dh1lo + Fn.T @ dh1hi
    hi = Fp.T @ dh1hi + Fn.T @ dh1lo
    put(OFF_W1, lo, hi, gR * (np.abs(Fr).T @ dh1max))
    # loss = sum_r (out_r - y_r)^2 / N
    elo, ehi = olo - y, ohi - y
    sqlo = np.where((elo <= 0) & (ehi >= 0), 0.0, np.minimum(elo * elo, ehi * ehi))
    sqhi = np.maximum(elo * elo, ehi * ehi)
    llo, lhi = _widen(sqlo.sum() / N, sqhi.sum() / N, 2 * gR * sqhi.sum() / N)
    return glo, ghi, (llo, lhi)
