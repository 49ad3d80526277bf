"""GPU parity of the uneven batch (one persistent launch sequence, optional
captured graph) and of the lambda path at full size, against the oracle."""
import sys

import numpy as np
import pytest

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


def _np(outs):
    import torch
    torch.cuda.synchronize()
    res = []
    for o in outs:
        r = {k: (v.cpu().numpy() if v is not None else None) for k, v in o.items()}
        r["status"] = int(r["status"][0])
        res.append(r)
    return res


def _eq(g, r, tag):
    assert g["status"] == 0, (tag, g["status"])
    assert np.array_equal(g["J"], r["J"]), (tag, g["J"], r["J"])
    assert g["V"].tobytes() == r["V"].tobytes(), tag
    assert np.array_equal(g["ROW"], r["ROW"]), tag
    assert g["ZALL"].tobytes() == r["ZALL"].tobytes(), tag
    assert g["OBJ"].tobytes() == r["OBJ"].tobytes(), tag


def _small_batch(seed):
    rng = np.random.default_rng(seed)
    probs = []
    for q in range(14):
        n = int(rng.integers(1, 700))
        m = int(rng.integers(1, 40))
        X = wl.random_small(5000 + 31 * seed + q, n, m, integer=(q % 4 == 3), zero_frac=0.05, span=3)
        L = int(rng.integers(1, 17))
        mass = float(np.abs(X).sum(0).max())
        lams = wl.log_lambdas(mass, L) if L > 1 else np.array([0.1 * mass])
        probs.append((X, lams))
    return probs


@pytest.mark.parametrize("seed", [0, 1])
def test_uneven_batch_matches_oracle(ctx, seed):
    from paper_2402_16712_amd import binding as B
    probs = _small_batch(seed)
    dev = [(B.device_matrix(X), lam) for X, lam in probs]
    _say(f"case batch seed={seed} B={len(probs)}")
    outs = _np(ctx.fit_batch(dev))
    for q, ((X, lam), g) in enumerate(zip(probs, outs)):
        _eq(g, O.fit_path(X, lam), f"problem {q} {X.shape} L={len(lam)}")


def test_batch_graph_capture_and_replay(ctx):
    from paper_2402_16712_amd import binding as B
    probs = _small_batch(2)
    dev = [(B.device_matrix(X), lam) for X, lam in probs]
    _say("case batch graph")
    plain = _np(ctx.fit_batch(dev))
    arr, outs, keep = ctx._batch_args(dev, True, True)
    for rep in range(3):                      # capture, then two replays
        ctx.fit_batch_prepared(arr, len(dev), graph=True)
        got = _np(outs)
        for q, (g, p) in enumerate(zip(got, plain)):
            _eq(g, p, f"graph rep {rep} problem {q}")
    other = _small_batch(3)                    # a different layout in between
    ctx.fit_batch([(B.device_matrix(X), lam) for X, lam in other], graph=True)
    ctx.fit_batch_prepared(arr, len(dev), graph=True)
    for q, (g, p) in enumerate(zip(_np(outs), plain)):
        _eq(g, p, f"graph after switch problem {q}")


def test_batch_with_long_columns(ctx):
    # one problem longer than the LDS copy of column j: the whole launch
    # reads columns j from global memory
    from paper_2402_16712_amd import binding as B
    probs = [(wl.random_small(900 + q, n, m, zero_frac=0.02), None) for q, (n, m) in
             enumerate([(5000, 4), (300, 9), (37, 5), (1200, 6)])]
    probs = [(X, np.array([0.0, 0.02, 0.3]) * float(np.abs(X).sum(0).max())) for X, _ in probs]
    dev = [(B.device_matrix(X), lam) for X, lam in probs]
    _say("case batch long columns")
    outs = _np(ctx.fit_batch(dev))
    for q, ((X, lam), g) in enumerate(zip(probs, outs)):
        _eq(g, O.fit_path(X, lam), f"long-column problem {q} {X.shape}")


def test_batch_equals_path_per_problem(ctx):
    from paper_2402_16712_amd import binding as B
    probs = wl.uneven_batch(12345, B=6, L=16, n_range=(50, 900), m_range=(10, 60))
    dev = [(B.device_matrix(p.X), p.lambdas) for p in probs]
    _say("case batch vs path")
    outs = _np(ctx.fit_batch(dev))
    for q, (p, g) in enumerate(zip(probs, outs)):
        import torch
        r = ctx.fit_path(B.device_matrix(p.X), p.lambdas)
        torch.cuda.synchronize()
        r = {k: (v.cpu().numpy() if v is not None else None) for k, v in r.items()}
        r["status"] = int(r["status"][0])
        _eq(g, r, f"batch-vs-path {q}")
        if p.n * p.m * p.m <= 2e6:
            _eq(g, O.fit_path(p.X, p.lambdas), f"batch-vs-oracle {q}")


def test_autotune_keeps_results(ctx):
    from paper_2402_16712_amd import binding as B
    probs = _small_batch(4)
    dev = [(B.device_matrix(X), lam) for X, lam in probs]
    _say("case autotune batch")
    before = _np(ctx.fit_batch(dev))
    default = ctx.tune_get()
    params = ctx.autotune(dev)
    assert params[0] in (2, 3, 4) and params[1] in (8, 32, 128) and params[2] in (12, 24, 48)
    # the batch's size class launches with the tuned entry, the default stays
    assert ctx.tune_lookup(dev) == (tuple(params), True)
    assert ctx.tune_get() == default
    after = _np(ctx.fit_batch(dev))
    for q, (a, b) in enumerate(zip(after, before)):
        _eq(a, b, f"after tune {q}")
    # another size class (one problem) keeps the default
    one = [dev[0]]
    assert ctx.tune_lookup(one) == (tuple(default), False)


def test_autotune_one_problem_class(tmp_path):
    """One problem tunes its own class (the grid of implicit items); the
    entry is read back from the cache file by a new context and leaves the
    results bit for bit unchanged."""
    import torch
    from paper_2402_16712_amd import binding as B
    path = str(tmp_path / "tune.txt")
    p = wl.large_fit(3, n=900, m=120)
    c = B.Context(0, tune_cache_path=path)
    try:
        X = B.device_matrix(p.X)
        _say("case autotune one problem")
        ref = {k: v.cpu().numpy() for k, v in c.fit(X, float(p.lambdas[0])).items()}
        params = c.autotune([(X, p.lambdas)])
        assert params[0] in (2, 3, 4) and params[1] in (64, 256, 512) and params[2] == 24
        got = {k: v.cpu().numpy() for k, v in c.fit(X, float(p.lambdas[0])).items()}
        torch.cuda.synchronize()
        for k in ("v", "j", "obj", "row", "z_all"):
            assert got[k].tobytes() == ref[k].tobytes(), k
        lines = open(path).read().splitlines()
        assert lines[0].startswith("l1line-tune ") and any(l.startswith("l1line-tune-class ") for l in lines)
    finally:
        c.close()
    c2 = B.Context(0, tune_cache_path=path)
    try:
        X = B.device_matrix(p.X)
        assert c2.tune_lookup([(X, p.lambdas)]) == (tuple(params), True)
    finally:
        c2.close()


def test_path_full_size_sampled(ctx):
    """The 64-penalty path on 2000 x 2000 at full size: every z_j(lambda_t)
    from the GPU; the oracle recomputes sampled columns for all 64 lambdas."""
    import torch
    from paper_2402_16712_amd import binding as B
    p = wl.lambda_path(0)
    _say("case path 2000x2000x64")
    out = ctx.fit_path(B.device_matrix(p.X), p.lambdas)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    assert int(g["status"][0]) == 0
    Z = g["ZALL"]
    assert np.array_equal(g["J"], np.argmin(Z, axis=1))
    for j in sorted({int(g["J"][0]), int(g["J"][-1]), 5, 1234}):
        _say(f"  oracle column j={j}")
        r = O.fit_j(p.X, j, p.lambdas)
        assert r["ZJ"].tobytes() == Z[:, j].tobytes(), j
        for t in np.nonzero(g["J"] == j)[0]:
            assert r["V"][t].tobytes() == g["V"][t].tobytes()
