"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: v, j*, the median rows and every z_j bit for bit (both sides use exact
weight sums and the same fixed R64 order for the reported sums), which is
stronger than the 1e-12 relative objective tolerance.
"""
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


def gpu_path(ctx, X, lambdas, ld=None):
    import torch
    from paper_2402_16712_amd import binding as B
    if ld is None:
        Xd = B.device_matrix(X)
    else:
        n, m = X.shape
        buf = torch.zeros(ld * m, dtype=torch.float64, device="cuda:0")
        buf.view(m, ld)[:, :n] = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")
        Xd = buf.as_strided((n, m), (1, ld))
    out = ctx.fit_path(Xd, lambdas)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["status"] = int(res["status"][0])
    return res


def gpu_fit(ctx, X, lam):
    import torch
    from paper_2402_16712_amd import binding as B
    out = ctx.fit(B.device_matrix(X), lam)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["status"] = int(res["status"][0])
    return res


def assert_path_equal(g, r, tag):
    assert g["status"] == 0, (tag, g["status"])
    assert np.array_equal(g["J"], r["J"]), (tag, g["J"], r["J"])
    assert g["V"].tobytes() == r["V"].tobytes(), (tag, np.argwhere(g["V"] != r["V"])[:5])
    assert np.array_equal(g["ROW"], r["ROW"]), (tag, np.argwhere(g["ROW"] != r["ROW"])[:5])
    assert g["ZALL"].tobytes() == r["ZALL"].tobytes(), (tag, np.max(np.abs(g["ZALL"] - r["ZALL"])))
    assert g["OBJ"].tobytes() == r["OBJ"].tobytes(), tag


@pytest.mark.parametrize("seed", range(6))
def test_small_fit_workload(ctx, seed):
    p = wl.small_fit(seed)
    lam = float(p.lambdas[0])
    _say(f"case small_fit seed={seed}")
    g = gpu_fit(ctx, p.X, lam)
    r = O.fit(p.X, lam)
    assert g["status"] == 0
    assert int(g["j"][0]) == r["j"]
    assert g["v"].tobytes() == r["v"].tobytes()
    assert np.array_equal(g["row"], r["row"])
    assert g["z_all"].tobytes() == r["z_all"].tobytes()
    assert g["obj"].tobytes() == np.float64(r["obj"]).tobytes()
    # the objective bar of the method, stated explicitly
    assert abs(g["obj"][0] - r["obj"]) <= 1e-12 * abs(r["obj"])


SHAPES = [(1, 1), (1, 5), (5, 1), (7, 3), (63, 4), (64, 5), (65, 6), (127, 9), (128, 3), (129, 17),
          (200, 20), (333, 33), (640, 7), (1000, 12), (2049, 5), (4096, 3), (4097, 3), (10000, 4),
          (16384, 3)]


@pytest.mark.parametrize("n,m", SHAPES)
def test_random_shapes_path(ctx, n, m):
    X = wl.random_small(1000 + n, n, m, zero_frac=0.03)
    mass = float(np.abs(X).sum(0).max())
    lams = np.array([0.0, 1e-3 * mass, 0.02 * mass, 0.1 * mass, 0.5 * mass, mass, 2 * mass])
    _say(f"case random n={n} m={m}")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), f"{n}x{m}")


@pytest.mark.parametrize("n,m,seed", [(20000, 6, 0), (50000, 4, 1), (65535, 3, 2)])
def test_rows_beyond_16384(ctx, n, m, seed):
    # more rows than the LDS copy of column j, up to the 16-bit row ids' limit
    X = wl.random_small(3000 + seed, n, m, zero_frac=0.02)
    mass = float(np.abs(X).sum(0).max())
    lams = np.array([0.0, 1e-3 * mass, 0.05 * mass, 0.3 * mass, mass])
    _say(f"case rows n={n} m={m}")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), f"{n}x{m}")
    g = gpu_fit(ctx, X, float(lams[2]))
    r = O.fit(X, float(lams[2]))
    assert g["status"] == 0 and int(g["j"][0]) == r["j"] and g["z_all"].tobytes() == r["z_all"].tobytes()


def test_rows_beyond_16384_structured_and_ties(ctx):
    # the rank-one workload recipe with outlier rows at 30000 rows, and
    # integer data at 40000 rows (thousands of tied ratios across the lists)
    X = wl.rank_one_matrix(30000, 7, 2, 3000, 20.0, 0.01, (34, 30000))
    lam = 0.05 * wl.max_column_mass(X)
    _say("case rows 30000x7 rank one")
    assert_path_equal(gpu_path(ctx, X, np.array([lam, 0.0])), O.fit_path(X, np.array([lam, 0.0])), "r1-30000")
    Y = wl.random_small(77, 40000, 4, integer=True, zero_frac=0.1, span=3)
    lams = np.array([0.0, 10.0, 1000.0, 20000.0])
    _say("case rows 40000x4 integer")
    assert_path_equal(gpu_path(ctx, Y, lams), O.fit_path(Y, lams), "int-40000")


@pytest.mark.parametrize("kind,n,m", [("rank1", 10000, 8), ("rank1", 30000, 6), ("int", 40000, 4),
                                      ("int", 12000, 5), ("cauchy", 15000, 7), ("mix", 25000, 6)])
def test_one_penalty_windows_too_full_for_the_list(ctx, kind, n, m):
    # one penalty at many rows: the sampled key window around the median
    # holds more elements than the list, so it is bisected before the exact
    # listing.  Clustered ratios (rank one, outlier rows) and thousands of
    # tied ratios (small integers), where a bisection can stall on one key.
    if kind == "rank1":
        X = wl.rank_one_matrix(n, m, max(2, m // 2), n // 10, 20.0, 0.01, (35, n, m))
        mass = wl.max_column_mass(X)
        lams = [0.0, 0.01 * mass, 0.05 * mass]
    elif kind == "int":
        # a rounded rank-one matrix: 42 distinct integers, medians on ties
        X = np.asfortranarray(np.rint(3.0 * wl.rank_one_matrix(n, m, m, n // 10, 2.0, 0.05, (36, n, m),
                                                             laplace_b=0.2)))
        lams = [0.0, 10.0, 0.05 * wl.max_column_mass(X)]
    else:
        # heavy-tailed noise (Cauchy), or a fifth of the rows replaced by
        # large outliers: ratio clusters with far tails
        rng = np.random.default_rng(n + m)
        X = np.outer(rng.standard_normal(n), rng.uniform(-1.0, 1.0, m))
        if kind == "cauchy":
            X = X + 0.05 * rng.standard_cauchy((n, m))
        else:
            X = X + 0.1 * rng.laplace(size=(n, m))
            rows = rng.choice(n, n // 5, replace=False)
            X[rows] = 50.0 * rng.standard_normal((n // 5, m))
        X = np.asfortranarray(X)
        mass = wl.max_column_mass(X)
        lams = [0.0, 0.02 * mass, 0.08 * mass]
    for lam in lams:
        _say(f"case one penalty {kind} {n}x{m} lambda={lam!r}")
        g = gpu_fit(ctx, X, float(lam))
        r = O.fit(X, float(lam))
        assert g["status"] == 0, g["status"]
        assert int(g["j"][0]) == r["j"], (int(g["j"][0]), r["j"])
        assert g["v"].tobytes() == r["v"].tobytes(), np.argwhere(g["v"] != r["v"])[:5]
        assert np.array_equal(g["row"], r["row"]), np.argwhere(g["row"] != r["row"])[:5]
        assert g["z_all"].tobytes() == r["z_all"].tobytes()


@pytest.mark.parametrize("seed,span", [(0, 1), (1, 2), (2, 2), (3, 3), (4, 5)])
def test_integer_ties(ctx, seed, span):
    # integer data: many equal ratios and exact ties of the weighted median
    X = wl.random_small(2000 + seed, 150 + 37 * seed, 8, integer=True, zero_frac=0.1, span=span)
    lams = np.arange(0.0, 40.0, 1.0)
    _say(f"case integer seed={seed} span={span}")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), f"int{seed}")


def test_ties_above_64_in_one_key(ctx):
    # hundreds of identical ratios: the selection must fall back to row order
    n = 700
    X = np.ones((n, 3))
    X[:, 1] = 2.0
    X[::7, 1] = 3.0
    X[::5, 2] = -1.0
    X = np.asfortranarray(X)
    lams = np.array([0.0, 0.5, 3.0, 100.0, 1000.0])
    _say("case ties>64")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), "ties")


def test_zero_rows_and_columns(ctx):
    X = wl.random_small(7, 300, 9, zero_frac=0.2)
    X[:40, :] = 0.0          # zero rows
    X[:, 4] = 0.0            # an all-zero column
    X[100:160, 6] = 0.0
    X = np.asfortranarray(X)
    lams = np.array([0.0, 0.3, 3.0])
    _say("case zeros")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), "zeros")


@pytest.mark.parametrize("scale_exp", [-1060, -600, 600, 1000])
def test_extreme_magnitudes(ctx, scale_exp):
    # subnormal and huge data (power-of-two scaling keeps every column's range)
    X = np.asfortranarray(wl.random_small(8, 200, 6) * 2.0 ** scale_exp)
    mass = float(np.abs(X).sum(0).max())
    lams = np.array([0.0, 0.05 * mass, 0.4 * mass])
    _say(f"case scale 2^{scale_exp}")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), f"2^{scale_exp}")


def test_underflowing_ratios(ctx):
    # column 2 sits near the bottom of the subnormal range, column 5 just
    # above it: many of x_i2 / x_ij underflow to 0 (they join the zero block),
    # so the sign sums of those pairs must be overruled by the exact pass
    X = wl.random_small(11, 300, 8)
    X[:, 2] *= 2.0 ** -1072
    X[:, 5] *= 2.0 ** -1000
    X = np.asfortranarray(X)
    mass = float(np.abs(X).sum(0).max())
    # lambda > 0 keeps the tiny preserved columns at v = 0 (their ratios overflow)
    lams = np.array([0.05 * mass, 0.4 * mass])
    _say("case underflowing ratios")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), "underflow")


def test_padded_leading_dimension(ctx):
    X = wl.random_small(9, 150, 11, zero_frac=0.05)
    lams = np.array([0.0, 2.0, 20.0])
    _say("case ld>n")
    assert_path_equal(gpu_path(ctx, X, lams, ld=192), O.fit_path(X, lams), "ld")


def test_status_nonfinite_and_wide(ctx):
    X = wl.random_small(10, 100, 5)
    Y = X.copy(order="F")
    Y[3, 2] = np.nan
    _say("case nonfinite")
    assert gpu_fit(ctx, Y, 0.5)["status"] == -3
    Z = X.copy(order="F")
    Z[0, 1] = 1e-200
    Z[1, 1] = 1e100
    _say("case wide")
    assert gpu_fit(ctx, Z, 0.5)["status"] == -6
    # a wide column that is never the preserved one is fine: scale a column
    # uniformly by 2^-900 (its own range stays narrow)
    W = X.copy(order="F")
    W[:, 3] *= 2.0 ** -900
    _say("case scaled column")
    g = gpu_fit(ctx, W, 0.5)
    r = O.fit(W, 0.5)
    assert g["status"] == 0 and int(g["j"][0]) == r["j"] and g["v"].tobytes() == r["v"].tobytes()


def test_overflowing_ratio_reports_erange(ctx):
    Z = np.asfortranarray(np.array([[1e-300, 1e300, 1.0], [2e-300, 3e300, 2.0], [1e-300, 2e300, 1.5]]))
    _say("case erange")
    g = gpu_path(ctx, Z, np.array([0.0]))
    assert g["status"] == -4


def test_path_many_unsorted_penalties(ctx):
    # 100 penalties (two groups of 64 targets) in random order, with repeats
    X = wl.random_small(12, 700, 12, zero_frac=0.02)
    mass = float(np.abs(X).sum(0).max())
    rng = np.random.default_rng(5)
    lams = np.concatenate([rng.uniform(0.0, 0.6 * mass, 90), [0.0, 0.0, mass, 0.3 * mass],
                           np.full(6, 0.05 * mass)])
    rng.shuffle(lams)
    _say("case 100 unsorted penalties")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), "L100")


@pytest.mark.parametrize("n", [1500, 3000, 6000])
def test_path_wide_windows(ctx, n):
    # strongly correlated columns spread the penalties' targets over much of
    # a segment: the shared window overflows the list and the penalties are
    # retried one by one (or go to the rounds when even that overflows)
    X = wl.rank_one_matrix(n, 6, 6, 0, 20.0, 0.0, (30, n), laplace_b=0.02)
    mass = float(np.abs(X).sum(0).max())
    lams = wl.log_lambdas(mass, 16)
    _say(f"case wide windows n={n}")
    assert_path_equal(gpu_path(ctx, X, lams), O.fit_path(X, lams), f"wide{n}")


def test_fit_matches_path_and_is_deterministic(ctx):
    p = wl.lambda_path(0, n=600, m=150, L=8)
    _say("case fit-vs-path 600x150")
    g = gpu_path(ctx, p.X, p.lambdas)
    g2 = gpu_path(ctx, p.X, p.lambdas)
    assert g["V"].tobytes() == g2["V"].tobytes() and g["ZALL"].tobytes() == g2["ZALL"].tobytes()
    for t in (0, 3, 7):
        f = gpu_fit(ctx, p.X, float(p.lambdas[t]))
        assert int(f["j"][0]) == int(g["J"][t])
        assert f["v"].tobytes() == g["V"][t].tobytes()
        assert f["z_all"].tobytes() == g["ZALL"][t].tobytes()
    r = O.fit_path(p.X, p.lambdas)
    assert_path_equal(g, r, "path600")


def test_path_workload_reduced(ctx):
    # the lambda-path workload recipe (64 log-spaced penalties) at a size the
    # oracle finishes in seconds
    p = wl.lambda_path(1, n=400, m=64, L=64)
    _say("case path 400x64x64")
    assert_path_equal(gpu_path(ctx, p.X, p.lambdas), O.fit_path(p.X, p.lambdas), "path64")


def test_large_fit_full_size_sampled(ctx):
    """2000 x 2000 at the benchmark's launch configuration: every z_j from
    the GPU, the oracle recomputes j*, the runner-up and sampled columns."""
    p = wl.large_fit(0)
    lam = float(p.lambdas[0])
    _say("case large_fit 2000x2000")
    g = gpu_fit(ctx, p.X, lam)
    assert g["status"] == 0
    z = g["z_all"]
    js = int(g["j"][0])
    assert js == int(np.argmin(z)) and z[js] == g["obj"][0]
    order = np.argsort(z, kind="stable")
    sample = sorted({js, int(order[1]), int(order[2]), 0, 777, 1999})
    for j in sample:
        _say(f"  oracle column j={j}")
        r = O.fit_j(p.X, j, [lam])
        assert r["ZJ"][0].tobytes() == z[j].tobytes(), (j, r["ZJ"][0], z[j])
        if j == js:
            assert r["V"][0].tobytes() == g["v"].tobytes()
            assert np.array_equal(r["ROW"][0], g["row"])


def test_sticky_error_and_tune_cache(tmp_path):
    import torch
    from paper_2402_16712_amd import binding as B
    path = str(tmp_path / "tune.txt")
    c = B.Context(0, tune_cache_path=path)
    try:
        Y = wl.random_small(10, 100, 5)
        Y[3, 2] = np.nan
        c.fit(B.device_matrix(np.asfortranarray(Y)), 0.5)
        torch.cuda.synchronize()
        assert c.last_error() == B.ENONFINITE
        assert c.last_error() == B.OK
        probs = [(B.device_matrix(wl.random_small(40 + q, 60, 5)), np.array([0.1, 1.0])) for q in range(3)]
        best = c.autotune(probs)
        cls = [l.split() for l in open(path).read().splitlines() if l.startswith("l1line-tune-class ")]
        assert len(cls) == 1 and cls[0][-3:] == [str(x) for x in best]
    finally:
        c.close()
    c2 = B.Context(0, tune_cache_path=path)
    try:
        assert c2.tune_lookup(probs) == (tuple(best), True)
    finally:
        c2.close()
