"""The MLP reference is pinned by central finite differences (real-valued
mode) and its BF16 rounding by bit-level checks."""
import numpy as np

from oracle import mlp_oracle as M


def _params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(M.NPARAM) * scale


def test_bf16_rounding():
    assert M.bf16(1.0) == 1.0
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0                 # tie -> even
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (up)
    assert M.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7     # representable
    assert M.bf16(-3.0) == -3.0
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(M.bf16(x) - x) <= np.abs(x) * 2.0 ** -8 * 1.0001)


def test_gradient_finite_differences():
    rng = np.random.default_rng(1)
    P = _params(2)
    F = rng.standard_normal((23, M.IN))
    y = rng.standard_normal(23)
    loss, g = M.loss_and_grad(P, F, y, bf=False)
    idx = list(rng.choice(M.NPARAM, size=60, replace=False)) + [M.OFF_B3, M.OFF_W3, M.OFF_B1, M.OFF_W1]
    for i in idx:
        h = 1e-6
        Pp = P.copy(); Pp[i] += h
        Pm = P.copy(); Pm[i] -= h
        lp, _ = M.loss_and_grad(Pp, F, y, bf=False)
        lm, _ = M.loss_and_grad(Pm, F, y, bf=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_linear_special_case():
    # all-positive pre-activations: the network is linear; out = F W1 W2 W3 + ...
    rng = np.random.default_rng(3)
    P = np.abs(_params(4)) * 0.1
    F = np.abs(rng.standard_normal((5, M.IN)))
    W1, b1, W2, b2, W3, b3 = M.unpack(P)
    want = ((F @ W1 + b1) @ W2 + b2) @ W3 + b3
    out, _ = M.forward(P, F, bf=False)
    np.testing.assert_allclose(out, want, rtol=1e-12)


def test_adam_first_step_is_sign_step():
    g = np.array([3.0, -2.0, 0.5])
    P, m1, m2 = M.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01)
    np.testing.assert_allclose(P, -0.01 * np.sign(g), rtol=1e-6)


# ---------------------------------------------------------------- BF16 mode
# Pins of the rounded (bf=True) reference that do not restate its formula.

def test_bf16_mode_equals_real_network_on_exact_inputs():
    from tests.mlp_cases import exact_case
    for N, seed in ((48, 0), (64, 1), (7, 2), (130, 3)):
        P, F, y = exact_case(N, seed)
        o1, _ = M.forward(P, F, bf=True)
        o0, _ = M.forward(P, F, bf=False)
        assert o1.tobytes() == o0.tobytes()
        l1, g1 = M.loss_and_grad(P, F, y, bf=True)
        l0, g0 = M.loss_and_grad(P, F, y, bf=False)
        assert l1 == l0 and g1.tobytes() == g0.tobytes()
        assert np.count_nonzero(g1) > 1000          # the case exercises the gradient


def test_bf16_mode_rounds_operands_not_biases():
    # a perturbation far below half a BF16 ulp of a product operand leaves the
    # rounded network unchanged; the output bias is not rounded
    from tests.mlp_cases import exact_case
    P, F, y = exact_case(64, 5)
    P = P.astype(np.float64)
    F = F.astype(np.float64)
    base, _ = M.forward(P, F, bf=True)
    _, gbase = M.loss_and_grad(P, F, y, bf=True)
    tiny = 1.0 + 2.0 ** -14
    out, _ = M.forward(P, F * tiny, bf=True)
    assert out.tobytes() == base.tobytes()
    for lo, hi in ((M.OFF_W1, M.OFF_B1), (M.OFF_W2, M.OFF_B2), (M.OFF_W3, M.OFF_B3)):
        Q = P.copy()
        Q[lo:hi] *= tiny
        out, _ = M.forward(Q, F, bf=True)
        assert out.tobytes() == base.tobytes(), (lo, hi)
        _, g = M.loss_and_grad(Q, F, y, bf=True)
        assert g.tobytes() == gbase.tobytes(), (lo, hi)
        out0, _ = M.forward(Q, F, bf=False)          # the real network does move
        assert out0.tobytes() != base.tobytes()
    Q = P.copy()
    Q[M.OFF_B3] *= tiny
    out, _ = M.forward(Q, F, bf=True)
    assert np.all(out != base)


def test_bf16_mode_rounds_hidden_activations():
    # one hidden unit fed a value just off a BF16 grid point: the rounded
    # network sees the grid point, the real one the value itself
    P = np.zeros(M.NPARAM)
    P[M.OFF_W1 + 0 * M.H + 0] = 1.0               # a1[0] = F[0]
    P[M.OFF_B1 + 0] = 2.0 ** -12                  # + a bias below half an ulp of 1
    P[M.OFF_W2 + 0 * M.H + 0] = 1.0
    P[M.OFF_W3 + 0] = 1.0
    F = np.zeros((1, M.IN))
    F[0, 0] = 1.0
    o1, _ = M.forward(P, F, bf=True)
    o0, _ = M.forward(P, F, bf=False)
    assert o1[0] == 1.0 and o0[0] == 1.0 + 2.0 ** -12


# ---------------------------------------------------------------- intervals

def _random_case(N, seed):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal(M.NPARAM) * 0.15
    F = rng.standard_normal((N, M.IN))
    y = rng.standard_normal(N)
    return P.astype(np.float32), F.astype(np.float32), y.astype(np.float32)


def test_intervals_hold_the_reference_and_an_fp32_evaluation():
    from tests.mlp_cases import exact_case, fp32_eval
    cases = [_random_case(N, s) for N, s in ((200, 0), (33, 1), (1000, 2))] + [exact_case(96, 4)]
    for q, (P, F, y) in enumerate(cases):
        olo, ohi, _ = M.forward_interval(P, F)
        glo, ghi, (llo, lhi) = M.grad_interval(P, F, y)
        ref, _ = M.forward(P, F, bf=True)
        lref, gref = M.loss_and_grad(P, F, y, bf=True)
        assert np.all((olo <= ref) & (ref <= ohi))
        assert np.all((glo <= gref) & (gref <= ghi))
        assert llo <= lref <= lhi
        o32, g32, l32 = fp32_eval(P, F, y)
        assert np.all((olo <= o32) & (o32 <= ohi))
        assert np.all((glo <= g32) & (g32 <= ghi))
        assert llo <= l32 <= lhi
        if q == 3:
            continue
        # the bounds stay narrow on random inputs (a few BF16 flips per row
        # widen them beyond the FP32 accumulation error)
        wid = (ohi - olo) / (np.abs(ref) + 1.0)
        assert np.median(wid) < 4e-3, np.median(wid)
        gw = (ghi - glo) / (np.abs(gref) + 1e-3 * np.max(np.abs(gref)))
        assert np.median(gw) < 3e-2, np.median(gw)


def test_intervals_catch_a_misplaced_rounding():
    # an evaluation that skips the BF16 rounding of the hidden activations
    # (h1 in FP32) leaves the output interval on random inputs
    P, F, y = _random_case(400, 7)
    olo, ohi, _ = M.forward_interval(P, F)
    f32 = np.float32
    W1, b1, W2, b2, W3, b3 = (np.asarray(x, dtype=f32) for x in M.unpack(P))
    b = lambda a: M.bf16(a).astype(f32)                  # noqa: E731
    h1 = np.maximum(b(F) @ b(W1) + b1, 0)                # not rounded
    h2 = b(np.maximum(b(h1) @ b(W2) + b2, 0))
    h2_bad = b(np.maximum(h1 @ b(W2) + b2, 0))
    good = h2 @ b(W3) + b3
    bad = h2_bad @ b(W3) + b3
    assert np.all((olo <= good) & (good <= ohi))
    assert np.mean((bad < olo) | (bad > ohi)) > 0.5
