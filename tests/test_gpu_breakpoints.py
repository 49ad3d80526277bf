"""GPU parity of Algorithm 2 (every segment's breakpoints and lambda_max)
against the oracle, bit for bit."""
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


def _gpu(ctx, X, ld=None):
    import torch
    from paper_2402_16712_amd import binding as B
    if ld is None:
        Xd = B.device_matrix(X)
    else:
        n, m = X.shape
        buf = torch.zeros(ld * m, dtype=torch.float64, device="cuda:0")
        buf.view(m, ld)[:, :n] = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")
        Xd = buf.as_strided((n, m), (1, ld))
    out = ctx.breakpoints(Xd)
    torch.cuda.synchronize()
    r = {k: t.cpu().numpy() for k, t in out.items()}
    r["status"] = int(r["status"][0])
    return r


def _eq(g, r, tag):
    assert g["status"] == 0, (tag, g["status"])
    assert np.array_equal(g["offsets"], r["offsets"]), (tag, np.argwhere(g["offsets"] != r["offsets"])[:5])
    assert g["lambda_max"].tobytes() == r["lambda_max"].tobytes(), tag
    assert g["lam"].tobytes() == r["lam"].tobytes(), (tag, np.argwhere(g["lam"] != r["lam"])[:5])
    assert g["v"].tobytes() == r["v"].tobytes(), tag
    assert np.array_equal(g["row"], r["row"]), tag


def test_toy(ctx, toy):
    X = np.asfortranarray(np.array(toy["points"], dtype=float))
    _eq(_gpu(ctx, X), O.breakpoints(X), "toy")


@pytest.mark.parametrize("n,m,integer,seed", [(1, 3, False, 0), (7, 4, False, 1), (63, 5, False, 2),
                                              (64, 6, False, 3), (65, 5, True, 4), (300, 9, False, 5),
                                              (300, 9, True, 6), (1000, 7, False, 7), (2100, 4, False, 8)])
def test_random(ctx, n, m, integer, seed):
    X = wl.random_small(3000 + seed, n, m, integer=integer, zero_frac=0.05, span=3)
    _say(f"case bp n={n} m={m} integer={integer}")
    _eq(_gpu(ctx, X), O.breakpoints(X), f"{n}x{m}")


@pytest.mark.parametrize("n", [1500, 4000, 9000, 16384])
def test_many_breakpoints_per_segment(ctx, n):
    # strongly correlated columns: most points lie between the lambda = 0
    # minimiser and 0, more than one window list holds
    X = wl.rank_one_matrix(n, 5, 5, 0, 20.0, 0.0, (32, n), laplace_b=0.02)
    _say(f"case bp correlated n={n}")
    _eq(_gpu(ctx, X), O.breakpoints(X), f"corr{n}")


def test_integer_ties_long_columns(ctx):
    # integer data, 12000 rows: thousands of equal breakpoints across the
    # segments, several window passes per segment
    X = wl.rank_one_matrix(12000, 4, 4, 0, 20.0, 0.0, (62, 12000), laplace_b=0.02)
    X = np.asfortranarray(np.round(X * 32.0))
    _say("case bp integer ties 12000x4")
    _eq(_gpu(ctx, X), O.breakpoints(X), "int12000")


def test_one_key_with_many_rows(ctx):
    # 1500 identical ratios in one segment: streamed in row order
    rng = np.random.default_rng(4)
    n = 2000
    X = np.empty((n, 3))
    X[:, 0] = rng.uniform(0.5, 1.5, n)
    X[:, 1] = -2.0 * X[:, 0]
    X[1500:, 1] = rng.standard_normal(500)
    X[:, 2] = rng.standard_normal(n)
    X = np.asfortranarray(X)
    _say("case bp ties")
    _eq(_gpu(ctx, X), O.breakpoints(X), "ties")


def test_zero_columns_padding_and_status(ctx):
    X = wl.random_small(77, 200, 6, zero_frac=0.2)
    X[:, 2] = 0.0
    X[:50, :] = 0.0
    X = np.asfortranarray(X)
    _eq(_gpu(ctx, X, ld=256), O.breakpoints(X), "zeros+ld")
    Y = X.copy(order="F")
    Y[5, 4] = np.inf
    from paper_2402_16712_amd import binding as B
    assert _gpu(ctx, Y)["status"] == B.ENONFINITE


def test_capacity_too_small_reports_esize(ctx):
    import torch
    from paper_2402_16712_amd import binding as B
    X = B.device_matrix(wl.random_small(5, 100, 4))
    n, m = 100, 4
    offs = torch.empty(m * m + 1, dtype=torch.int64, device="cuda:0")
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    lam = torch.empty(1, dtype=torch.float64, device="cuda:0")
    v = torch.empty(1, dtype=torch.float64, device="cuda:0")
    row = torch.empty(1, dtype=torch.int32, device="cuda:0")
    rc = B.lib().l1line_breakpoints(ctx._h, B._ptr(X), n, m, n, B._ptr(offs), None, B._ptr(lam), B._ptr(v),
                                    B._ptr(row), 1, B._ptr(st), ctx._stream())
    torch.cuda.synchronize()
    assert rc == 0 and int(offs[-1].item()) > 1 and int(st.item()) == B.ESIZE
    ctx.last_error()


def test_full_size_sampled(ctx):
    """2000 x 2000 (the benchmark's matrix): sampled segments against the
    oracle, every segment's count consistent with its entries."""
    import torch
    from paper_2402_16712_amd import binding as B
    p = wl.large_fit(0)
    _say("case bp 2000x2000")
    out = ctx.breakpoints(B.device_matrix(p.X))
    torch.cuda.synchronize()
    g = {k: t.cpu().numpy() for k, t in out.items()}
    assert int(g["status"][0]) == 0
    off, m = g["offsets"], p.X.shape[1]
    cnt = np.diff(off)
    assert np.all(cnt[np.arange(m) * m + np.arange(m)] == 0)
    term = off[1:][cnt > 0] - 1                  # every segment ends in (lambda_max, 0, -1)
    assert np.all(g["row"][term] == -1) and np.all(g["v"][term] == 0.0)
    assert np.array_equal(g["lam"][term], g["lambda_max"][cnt > 0])
    rng = np.random.default_rng(9)
    for _ in range(40):
        j, k = (int(x) for x in rng.choice(m, 2, replace=False))
        gs = j * m + k
        lam, v, row, lm = O.breakpoints_segment(p.X, j, k)
        a, b = off[gs], off[gs + 1]
        assert g["lam"][a:b].tobytes() == lam.tobytes(), (j, k)
        assert g["v"][a:b].tobytes() == v.tobytes() and np.array_equal(g["row"][a:b], row), (j, k)
        assert g["lambda_max"][gs] == lm
