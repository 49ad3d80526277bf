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
