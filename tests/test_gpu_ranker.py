"""GPU parity of the candidate ranker: MLP forward / gradient / Adam against
the FP64 reference that mirrors the BF16 rounding points, features against
their FP64 definition, and the ranked fit against the exhaustive oracle."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import oracle as O
from paper_2402_16712_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_16712_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _params(seed):
    from paper_2402_16712_amd import ranker
    P = ranker.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    # nonzero biases so every term of the gradient is exercised
    P[M.OFF_B1:M.OFF_W2] = rng.standard_normal(M.H) * 0.1
    P[M.OFF_B2:M.OFF_W3] = rng.standard_normal(M.H) * 0.1
    P[M.OFF_B3] = 0.3
    return P.astype(np.float32)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


# FP32 accumulation against the exact FP64 sums: an FP32 sum of <= 128 BF16
# products is within ~1e-6 relative of the exact one, which can flip the BF16
# rounding of a hidden activation (one ulp = 2^-8 relative) in rare cases.
# The bound below admits a few such flips, no structural error.
def _close(got, want, rel, what):
    got = np.asarray(got, dtype=np.float64)
    err = np.linalg.norm(got - want)
    scale = np.linalg.norm(want) + 1e-30
    assert err <= rel * scale, (what, err / scale)


@pytest.mark.parametrize("N", [1, 15, 16, 17, 333, 4096 + 5])
def test_mlp_forward(ctx, N):
    _say(f"mlp_forward N={N}")
    P = _params(1)
    F = np.random.default_rng(N).standard_normal((N, M.IN)).astype(np.float32)
    out = ctx.mlp_forward(_dev(P), _dev(F)).cpu().numpy()
    want, _ = M.forward(P, F, bf=True)
    _close(out, want, 2e-3, "out")
    # elementwise: most rows agree to FP32 accumulation accuracy
    d = np.abs(out - want) / (np.abs(want) + 1e-3)
    assert np.mean(d < 1e-4) > 0.95, np.mean(d < 1e-4)


@pytest.mark.parametrize("N", [1, 31, 32, 33, 500, 2048 + 7])
def test_mlp_grad(ctx, N):
    _say(f"mlp_grad N={N}")
    P = _params(2)
    rng = np.random.default_rng(N + 7)
    F = rng.standard_normal((N, M.IN)).astype(np.float32)
    y = rng.standard_normal(N).astype(np.float32)
    g, loss = ctx.mlp_grad(_dev(P), _dev(F), _dev(y))
    g = g.cpu().numpy()
    want_loss, want = M.loss_and_grad(P, F, y, bf=True)
    assert abs(float(loss.item()) - want_loss) <= 1e-4 * abs(want_loss), (float(loss.item()), want_loss)
    for name, lo, hi in (("W1", M.OFF_W1, M.OFF_B1), ("b1", M.OFF_B1, M.OFF_W2), ("W2", M.OFF_W2, M.OFF_B2),
                         ("b2", M.OFF_B2, M.OFF_W3), ("W3", M.OFF_W3, M.OFF_B3), ("b3", M.OFF_B3, M.NPARAM)):
        _close(g[lo:hi], want[lo:hi], 1e-2, name)


@pytest.mark.parametrize("N", [1, 17, 333, 4096 + 5])
def test_mlp_forward_elementwise_bound(ctx, N):
    # every row inside the interval any FP32-accumulating evaluation with
    # the reference's BF16 rounding points must reach (oracle.mlp_oracle:
    # forward_interval)
    _say(f"mlp_forward interval N={N}")
    P = _params(1)
    F = np.random.default_rng(N + 50).standard_normal((N, M.IN)).astype(np.float32)
    out = ctx.mlp_forward(_dev(P), _dev(F)).cpu().numpy().astype(np.float64)
    lo, hi, _ = M.forward_interval(P, F)
    bad = np.nonzero((out < lo) | (out > hi))[0]
    assert bad.size == 0, (bad[:5], out[bad[:5]], lo[bad[:5]], hi[bad[:5]])


@pytest.mark.parametrize("N", [1, 31, 33, 500, 2048 + 7])
def test_mlp_grad_elementwise_bound(ctx, N):
    _say(f"mlp_grad interval N={N}")
    P = _params(2)
    rng = np.random.default_rng(N + 70)
    F = rng.standard_normal((N, M.IN)).astype(np.float32)
    y = rng.standard_normal(N).astype(np.float32)
    g, loss = ctx.mlp_grad(_dev(P), _dev(F), _dev(y))
    g = g.cpu().numpy().astype(np.float64)
    lo, hi, (llo, lhi) = M.grad_interval(P, F, y)
    bad = np.nonzero((g < lo) | (g > hi))[0]
    assert bad.size == 0, (bad[:5], g[bad[:5]], lo[bad[:5]], hi[bad[:5]])
    assert llo <= float(loss.item()) <= lhi


@pytest.mark.parametrize("N,seed", [(48, 0), (64, 1), (7, 2), (130, 3), (96, 4)])
def test_mlp_exact_inputs_bitwise(ctx, N, seed):
    # inputs on which every product, FP32 sum and BF16 rounding is exact: the
    # kernels must return the reference's values bit for bit, every entry
    from tests.mlp_cases import exact_case
    _say(f"mlp exact inputs N={N}")
    P, F, y = exact_case(N, seed)
    out = ctx.mlp_forward(_dev(P), _dev(F)).cpu().numpy()
    want, _ = M.forward(P, F, bf=True)
    assert out.tobytes() == want.astype(np.float32).tobytes()
    g, loss = ctx.mlp_grad(_dev(P), _dev(F), _dev(y))
    wl_, wg = M.loss_and_grad(P, F, y, bf=True)
    g = g.cpu().numpy()
    bad = np.nonzero(g != wg.astype(np.float32))[0]
    assert bad.size == 0, (bad[:8], g[bad[:8]], wg[bad[:8]])
    assert float(loss.item()) == np.float32(wl_)


def test_mlp_grad_deterministic(ctx):
    P = _params(3)
    rng = np.random.default_rng(5)
    F = _dev(rng.standard_normal((1000, M.IN)))
    y = _dev(rng.standard_normal(1000))
    g1, l1 = ctx.mlp_grad(_dev(P), F, y)
    g2, l2 = ctx.mlp_grad(_dev(P), F, y)
    assert g1.cpu().numpy().tobytes() == g2.cpu().numpy().tobytes()
    assert l1.cpu().numpy().tobytes() == l2.cpu().numpy().tobytes()


def test_mlp_adam(ctx):
    rng = np.random.default_rng(11)
    P = rng.standard_normal(M.NPARAM).astype(np.float32)
    m1 = (rng.standard_normal(M.NPARAM) * 0.01).astype(np.float32)
    m2 = (rng.random(M.NPARAM) * 1e-4).astype(np.float32)
    g = rng.standard_normal(M.NPARAM).astype(np.float32)
    dP, dm1, dm2 = _dev(P), _dev(m1), _dev(m2)
    ctx.mlp_adam(dP, dm1, dm2, _dev(g), 7, 1e-3)
    # the kernel's constants are the FP32 roundings of 0.9, 0.999, 1e-8 and
    # the learning rate (1 - beta is then exact); the reference takes them
    f = lambda x: float(np.float32(x))
    wP, wm1, wm2 = M.adam(P.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64),
                          g.astype(np.float64), 7, f(1e-3), beta1=f(0.9), beta2=f(0.999), eps=f(1e-8))
    u = 2.0 ** -24
    g64, m164, m264 = g.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64)
    # FP32 rounding: a few units in the last place of the terms summed
    assert np.all(np.abs(dm1.cpu().numpy() - wm1) <= 4 * u * (0.9 * np.abs(m164) + 0.1 * np.abs(g64)))
    assert np.all(np.abs(dm2.cpu().numpy() - wm2) <= 4 * u * (0.999 * m264 + 0.001 * g64 * g64))
    # the step carries powf's rounding amplified by 1/(1 - beta2^7) ~ 140
    step = np.abs(P.astype(np.float64) - wP)
    assert np.all(np.abs(dP.cpu().numpy() - wP) <= 2 * u * np.abs(wP) + 400 * u * step)


def _features_from(W, zeros, D, Zr, lam, n):
    """The 32 features in FP64 from their definition, given the column
    masses, zero counts and the sign sums D, Zr."""
    m = len(W)
    S = np.abs(D) - Zr - lam
    np.fill_diagonal(S, -1.0)
    pos = S > 0
    Wk = W[None, :]
    okw = pos & (Wk > 0)
    Wsafe = np.where(Wk > 0, Wk, 1.0)
    A = np.stack([np.where(pos, S, 0.0).sum(1), np.where(okw, S * S / Wsafe, 0.0).sum(1),
                  np.where(okw, S / Wsafe, 0.0).sum(1), pos.sum(1).astype(np.float64)], axis=1)
    f = np.zeros((m, 32))

    def stand(v):
        mean, mx = v.mean(), v.max()
        sd = np.sqrt(max(np.mean(v * v) - mean * mean, 0.0))
        return ((v - mean) / sd, (v - mx) / sd) if sd > 0 else (np.zeros(m), np.zeros(m))

    f[:, 0], f[:, 1] = stand(W)
    with np.errstate(divide="ignore", invalid="ignore"):
        f[:, 2] = np.where(W > 0, np.log(np.where(W > 0, W, 1.0) / W.mean()), -30.0)
        f[:, 3] = zeros / n
        f[:, 4] = np.where(W > 0, np.minimum(lam / np.where(W > 0, W, 1.0), 10.0), 10.0)
        f[:, 5] = A[:, 3] / max(m - 1, 1)
        for q in range(4):
            f[:, 6 + 2 * q], f[:, 7 + 2 * q] = stand(A[:, q])
        f[:, 14] = np.where(W > 0, np.log1p(A[:, 0] / np.where(W > 0, W, 1.0)), 0.0)
    f[:, 15] = 1.0
    return f


def _signsums_fp64(X):
    """D[j, k] = sum_i x_ij sgn(x_ik), Zr[j, k] = sum_i |x_ij| [x_ik = 0] by
    numpy FP64 matrix products."""
    return X.T @ np.sign(X), np.abs(X).T @ (X == 0).astype(np.float64)


FEATURE_CASES = [(300, 40, 0), (50, 25, 1), (1000, 60, 2), (64, 9, 3), (2500, 130, 4)]


@pytest.mark.parametrize("n,m,seed", FEATURE_CASES)
def test_feature_signsums_within_their_bound(ctx, n, m, seed):
    """The BF16 sign sums against FP64 products, inside the bounds the header
    states: |dD| <= (2^-15 + 2 n u) W_j, |dZr| <= (2^-8 + 2 n u) Zr, u = 2^-24
    (plus 1e-12 W_j for the FP64 reference's own rounding)."""
    from paper_2402_16712_amd import binding as B
    _say(f"feature sign sums {n}x{m} seed {seed}")
    X = wl.rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (20, seed))
    DZ = ctx.feature_signsums(B.device_matrix(X)).cpu().numpy()
    D, Zr = _signsums_fp64(X)
    W = np.abs(X).sum(0)[:, None]
    u = 2.0 ** -24
    assert np.all(np.abs(DZ[:, :, 0] - D) <= (2.0 ** -15 + 2 * n * u) * W + 1e-12 * W)
    assert np.all(np.abs(DZ[:, :, 1] - Zr) <= (2.0 ** -8 + 2 * n * u) * Zr + 1e-12 * W)
    # not trivially loose: the high and low parts carry D far below the bound
    assert np.max(np.abs(DZ[:, :, 0] - D) / W) < 2.0 ** -15


def test_feature_signsums_scaled_columns(ctx):
    """Columns of very different magnitudes (each scaled by its own power of
    two before the BF16 split) and exact zeros, signs and ties."""
    from paper_2402_16712_amd import binding as B
    rng = np.random.default_rng(5)
    n, m = 700, 23
    X = rng.standard_normal((n, m)) * np.exp2(rng.integers(-200, 200, m))[None, :]
    X[rng.random((n, m)) < 0.05] = 0.0
    X[:, 3] = np.where(np.arange(n) % 3 == 0, 0.0, 2.0 ** 300)
    X[:, 5] = 0.0                                    # an all-zero column
    X[::2, 6] = 2.0 ** -1060                         # subnormal magnitudes
    X = np.asfortranarray(X)
    _say("feature sign sums, scaled columns")
    DZ = ctx.feature_signsums(B.device_matrix(X)).cpu().numpy()
    D, Zr = _signsums_fp64(X)
    W = np.abs(X).sum(0)[:, None]
    u = 2.0 ** -24
    assert np.all(np.abs(DZ[:, :, 0] - D) <= (2.0 ** -15 + 2 * n * u) * W)
    assert np.all(np.abs(DZ[:, :, 1] - Zr) <= (2.0 ** -8 + 2 * n * u) * Zr + 1e-12 * W)


@pytest.mark.parametrize("n,m,seed", FEATURE_CASES)
def test_features(ctx, n, m, seed):
    """The features from their definition on the device's own sign sums, and
    close to the features of the FP64 sign sums."""
    from paper_2402_16712_amd import binding as B
    _say(f"features {n}x{m} seed {seed}")
    X = wl.rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (20, seed))
    lam = 0.05 * wl.max_column_mass(X)
    Xd = B.device_matrix(X)
    F = ctx.features(Xd, lam).cpu().numpy()
    DZ = ctx.feature_signsums(Xd).cpu().numpy()
    W, zeros = O.column_stats(X)
    want = _features_from(W, zeros, DZ[:, :, 0], DZ[:, :, 1], lam, n)
    # FP32 roundings of FP64 arithmetic (aggregates and statistics summed in
    # different orders)
    np.testing.assert_allclose(F, want, rtol=1e-5, atol=2e-6)
    D, Zr = _signsums_fp64(X)
    exact = _features_from(W, zeros, D, Zr, lam, n)
    # the ranking signal is the same: every feature within 1e-3 of its value
    # on the FP64 sign sums, except where a slope sits at 0 and flips a count
    assert np.mean(np.abs(F - exact) <= 1e-3 + 1e-3 * np.abs(exact)) > 0.99


def _topk_ref(scores, K):
    s = np.where(np.isnan(scores), np.inf, scores.astype(np.float64))
    order = np.lexsort((np.arange(len(s)), s))
    return order[:K], (s[order[K]] - s[order[0]]) if K < len(s) else 0.0


# (the last two: candidate sign sums cut into 5 and 9 row parts)
@pytest.mark.parametrize("n,m,K,seed", [(400, 50, 8, 0), (120, 17, 1, 1), (900, 64, 63, 2), (3000, 200, 16, 3),
                                        (5000, 70, 32, 4)])
def test_fit_ranked_candidates(ctx, n, m, K, seed):
    """Threshold 0: never falls back unless K = m; the answer is the exact
    optimum over the K best-scored columns."""
    from paper_2402_16712_amd import binding as B
    _say(f"fit_ranked {n}x{m} K={K}")
    X = wl.rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (21, seed))
    lam = 0.05 * wl.max_column_mass(X)
    ctx.ranker_set_params(_dev(_params(seed)))
    r = ctx.fit_ranked(B.device_matrix(X), lam, K, 0.0)
    assert int(r["status"].item()) == 0
    assert int(r["used_fallback"].item()) == 0
    scores = r["scores"].cpu().numpy()
    cand, _ = _topk_ref(scores, K)
    ref = O.fit(X, lam)
    z = ref["z_all"][cand]
    jbest = int(cand[np.lexsort((cand, z))[0]])
    assert int(r["j"].item()) == jbest
    assert np.float64(r["obj"].item()).tobytes() == np.float64(ref["z_all"][jbest]).tobytes()
    one = O.fit_j(X, jbest, [lam])
    assert r["v"].cpu().numpy().tobytes() == one["V"][0].tobytes()
    assert np.array_equal(r["row"].cpu().numpy(), one["ROW"][0])


@pytest.mark.parametrize("m,K", [(8200, 32), (300, 7)])
def test_fit_ranked_candidate_selection(ctx, m, K):
    """The K best scores for m above (per-round reductions) and below (one
    LDS sort) 8192 columns, with trained-like and with all-zero weights
    (every score tied: the K lowest indices).  The answer must be the best
    exact z over those candidates, judged by the exhaustive GPU fit (itself
    bit-exact against the oracle in test_gpu_fit)."""
    from paper_2402_16712_amd import binding as B
    n = 40
    _say(f"fit_ranked candidate selection m={m} K={K}")
    X = wl.rank_one_matrix(n, m, max(1, m // 10), 4, 20.0, 0.01, (22, m))
    lam = 0.05 * wl.max_column_mass(X)
    Xd = B.device_matrix(X)
    z = ctx.fit(Xd, lam)["z_all"].cpu().numpy()
    for params in (_params(5), np.zeros_like(_params(5))):
        ctx.ranker_set_params(_dev(params))
        r = ctx.fit_ranked(Xd, lam, K, 0.0)
        assert int(r["status"].item()) == 0 and int(r["used_fallback"].item()) == 0
        cand, _ = _topk_ref(r["scores"].cpu().numpy(), K)
        if not params.any():
            assert np.array_equal(np.sort(cand), np.arange(K))
        jbest = int(cand[np.lexsort((cand, z[cand]))[0]])
        assert int(r["j"].item()) == jbest
        assert np.float64(r["obj"].item()).tobytes() == np.float64(z[jbest]).tobytes()


@pytest.mark.parametrize("K", [5, 30])
def test_fit_ranked_fallback(ctx, K):
    """A threshold no margin reaches (or K = m) runs the exhaustive search:
    the result is the oracle's, bit for bit."""
    from paper_2402_16712_amd import binding as B
    X = wl.rank_one_matrix(500, 30, 3, 50, 20.0, 0.01, (22, K))
    lam = 0.05 * wl.max_column_mass(X)
    ctx.ranker_set_params(_dev(_params(9)))
    r = ctx.fit_ranked(B.device_matrix(X), lam, K, 1e30)
    ref = O.fit(X, lam)
    assert int(r["status"].item()) == 0
    assert int(r["used_fallback"].item()) == 1
    assert int(r["j"].item()) == ref["j"]
    assert np.float64(r["obj"].item()).tobytes() == np.float64(ref["obj"]).tobytes()
    assert r["v"].cpu().numpy().tobytes() == ref["v"].tobytes()
    assert np.array_equal(r["row"].cpu().numpy(), ref["row"])


@pytest.mark.parametrize("bias", [float("nan"), float("inf")])
def test_fit_ranked_nonfinite_scores_fall_back(ctx, bias):
    """Weights whose output bias is NaN (or +inf) give every column a
    non-finite score: nothing separates the candidates, so the exhaustive
    search runs even at threshold 0 and the result is the oracle's."""
    from paper_2402_16712_amd import binding as B
    X = wl.rank_one_matrix(300, 24, 3, 30, 20.0, 0.01, (24, 0))
    lam = 0.05 * wl.max_column_mass(X)
    P = _params(10)
    P[M.OFF_B3] = bias
    ctx.ranker_set_params(_dev(P))
    r = ctx.fit_ranked(B.device_matrix(X), lam, 4, 0.0)
    ref = O.fit(X, lam)
    assert not np.any(np.isfinite(r["scores"].cpu().numpy()))
    assert int(r["status"].item()) == 0
    assert int(r["used_fallback"].item()) == 1
    assert int(r["j"].item()) == ref["j"]
    assert r["v"].cpu().numpy().tobytes() == ref["v"].tobytes()


def test_fit_ranked_bad_args(ctx):
    from paper_2402_16712_amd import binding as B
    X = B.device_matrix(wl.random_small(1, 20, 5))
    ctx.ranker_set_params(_dev(_params(0)))
    ctx.last_error()                           # clear
    for K, thr in ((0, 0.1), (6, 0.1), (2, -1.0), (2, float("nan")), (2, float("inf"))):
        with pytest.raises(B.L1LineError):
            ctx.fit_ranked(X, 1.0, K, thr)
    assert ctx.last_error() == B.EINVAL        # the first rejected call, then cleared
    assert ctx.last_error() == B.OK


def test_fit_ranked_needs_weights():
    from paper_2402_16712_amd import binding as B
    c = B.Context(0)
    try:
        with pytest.raises(B.L1LineError) as e:
            c.fit_ranked(B.device_matrix(wl.random_small(2, 30, 6)), 1.0, 2, 0.1)
        assert e.value.code == B.ENOMODEL
    finally:
        c.close()


def test_ranker_save_load_roundtrip(ctx, tmp_path):
    from paper_2402_16712_amd import binding as B
    P = _dev(_params(5))
    ctx.ranker_set_params(P)
    path = str(tmp_path / "w.l1rk")
    ctx.ranker_save(path)
    w, state, head = B.read_ranker_file(path)
    assert w.tobytes() == P.cpu().numpy().tobytes() and state is None
    c = B.Context(0)
    try:
        c.ranker_load(path)
        assert c.ranker_get_params().cpu().numpy().tobytes() == w.tobytes()
        bad = tmp_path / "bad.l1rk"
        bad.write_bytes(open(path, "rb").read()[:64])
        with pytest.raises(B.L1LineError) as e:
            c.ranker_load(str(bad))
        assert e.value.code == B.EIO
    finally:
        c.close()


def test_shipped_weights_rank_exactly():
    """The shipped weights through l1line_ranker_load: the ranked fit is the
    oracle's exact optimum over the candidates it chose."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import ranker
    c = B.Context(0)
    try:
        c.ranker_load(ranker.WEIGHTS)
        X = wl.rank_one_matrix(600, 70, 7, 60, 20.0, 0.01, (23, 0))
        lam = 0.05 * wl.max_column_mass(X)
        r = c.fit_ranked(B.device_matrix(X), lam, 8, 0.0)
        cand, _ = _topk_ref(r["scores"].cpu().numpy(), 8)
        ref = O.fit(X, lam)
        z = ref["z_all"][cand]
        jbest = int(cand[np.lexsort((cand, z))[0]])
        assert int(r["j"].item()) == jbest
        assert np.float64(r["obj"].item()).tobytes() == np.float64(ref["z_all"][jbest]).tobytes()
    finally:
        c.close()


def test_native_train_resume(tmp_path):
    """l1line_ranker_train: 6 steps in one run equal 3 steps, a checkpoint
    and 3 more in a fresh context, bit for bit."""
    from paper_2402_16712_amd import binding as B
    a, b = str(tmp_path / "a.l1rk"), str(tmp_path / "b.l1rk")
    c1 = B.Context(0)
    try:
        c1.ranker_train(6, seed=3, ckpt_path=a)
    finally:
        c1.close()
    c2 = B.Context(0)
    try:
        c2.ranker_train(3, seed=3, ckpt_path=b)
    finally:
        c2.close()
    c3 = B.Context(0)
    try:
        c3.ranker_train(6, seed=99, ckpt_path=b)     # resumes: the file's seed wins
    finally:
        c3.close()
    wa, sa, ha = B.read_ranker_file(a)
    wb, sb, hb = B.read_ranker_file(b)
    assert ha == hb == dict(step=6, seed=3, cursor=6)
    assert sa is not None and np.all(np.isfinite(wa))
    assert wa.tobytes() == wb.tobytes()
    assert sa[0].tobytes() == sb[0].tobytes() and sa[1].tobytes() == sb[1].tobytes()


def test_trainer_resume(ctx, tmp_path):
    """A checkpointed trainer resumed in a fresh object continues bit for bit."""
    from paper_2402_16712_amd import ranker
    kw = dict(n_range=(100, 300), m_range=(20, 40))
    a = ranker.Trainer(ctx, seed=4, lr=1e-3)
    a.train(3, **kw)
    path = str(tmp_path / "ck.npz")
    a.save(path)
    a.train(2, **kw)
    b = ranker.Trainer(ctx, seed=99, lr=5.0)
    b.load(path)
    b.train(2, **kw)
    assert a.step == b.step == 5 and a.cursor == b.cursor
    assert a.params.cpu().numpy().tobytes() == b.params.cpu().numpy().tobytes()
    assert a.m2.cpu().numpy().tobytes() == b.m2.cpu().numpy().tobytes()


def test_trained_network_gains_over_the_method_without_it():
    """What the trained network adds, on the first 12 evaluation matrices
    (10000 x 4000, the ranked fit's workload; exact z_j of every column from
    the exhaustive fit): the optimal column is among the network's 32 best
    on all of them and ranked near the top, while untrained weights and the
    column mass miss it and the slope aggregate alone ranks it lower."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import ranker
    import torch
    c = B.Context(0)
    try:
        trained = ranker.load_params(ranker.WEIGHTS)
        untrained = torch.from_numpy(ranker.init_params(1)).to("cuda:0")
        _say("ranker ablation 12 x 10000x4000")
        rows = ranker.ablation(c, [ranker.EVAL_BASE + q for q in range(12)], trained, untrained, K=32,
                                  n=10000, m=4000)
        summ = ranker.ablation_summary(rows)
    finally:
        c.close()
    t, u, cm, sa = (summ[k] for k in ("trained", "untrained", "column_mass", "slope_aggregate"))
    assert t["hit_rate"] == 1.0 and t["within_rate"] == 1.0 and t["fallback_rate"] == 0.0
    assert t["top_k_rate"]["8"] == 1.0
    assert u["hit_rate"] <= 0.5 and cm["hit_rate"] <= 0.75
    assert t["mean_rank"] < sa["mean_rank"] and t["top_k_rate"]["1"] > sa["top_k_rate"]["1"]
