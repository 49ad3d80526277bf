"""GPU parity of the successive components against the oracle, bit for bit
(components, preserved columns, objectives and the projected data)."""
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


def _gpu(ctx, X, lam, p, ld=None):
    import torch
    from paper_2402_16712_amd import binding as B
    if ld is None:
        Xd = B.device_matrix(X)
    else:
        n, m = X.shape
        buf = torch.zeros(ld * m, dtype=torch.float64, device="cuda:0")
        buf.view(m, ld)[:, :n] = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")
        Xd = buf.as_strided((n, m), (1, ld))
    out = ctx.components(Xd, lam, p)
    torch.cuda.synchronize()
    r = {k: t.cpu().numpy() for k, t in out.items()}
    r["status"] = int(r["status"][0])
    return r


def _eq(g, r, tag):
    assert g["status"] == 0, (tag, g["status"])
    assert np.array_equal(g["J"], r["J"]), (tag, g["J"], r["J"])
    assert g["V"].tobytes() == r["V"].tobytes(), (tag, np.argwhere(g["V"] != r["V"])[:5])
    assert g["OBJ"].tobytes() == r["OBJ"].tobytes(), tag
    assert np.asfortranarray(g["work"]).tobytes() == np.asfortranarray(r["Xlast"]).tobytes(), tag


def _planted(seed, n=300, m=10):
    rng = np.random.default_rng(seed)
    u1, u2 = rng.standard_normal(n), rng.standard_normal(n)
    l1 = np.zeros(m)
    l1[:5] = rng.uniform(0.5, 1.0, 5) * np.sign(rng.standard_normal(5))
    l2 = np.zeros(m)
    l2[5:] = rng.uniform(0.5, 1.0, 5) * np.sign(rng.standard_normal(5))
    X = np.outer(u1, l1) + 0.7 * np.outer(u2, l2) + 0.01 * rng.laplace(size=(n, m))
    return np.asfortranarray(X)


@pytest.mark.parametrize("seed", range(3))
def test_planted(ctx, seed):
    X = _planted(seed)
    lam = 0.1 * wl.max_column_mass(X)
    print(f"case components planted seed {seed}", flush=True)
    _eq(_gpu(ctx, X, lam, 3), O.components(X, lam, 3), f"planted{seed}")


@pytest.mark.parametrize("n,m,p,integer", [(1, 3, 2, False), (70, 5, 5, False), (200, 9, 4, False),
                                           (150, 12, 3, True), (1100, 8, 3, False)])
def test_random(ctx, n, m, p, integer):
    X = wl.random_small(4100 + n, n, m, integer=integer, zero_frac=0.05, span=4)
    lam = 0.03 * wl.max_column_mass(X)
    print(f"case components {n}x{m} p={p}", flush=True)
    r = O.components(X, lam, p)
    if r["status"] != 0:
        pytest.skip(f"oracle status {r['status']}")
    _eq(_gpu(ctx, X, lam, p), r, f"{n}x{m}")


def test_padded_and_first_equals_fit(ctx):
    X = wl.random_small(4200, 160, 7, zero_frac=0.1)
    lam = 0.05 * wl.max_column_mass(X)
    g = _gpu(ctx, X, lam, 2, ld=192)
    _eq(g, O.components(X, lam, 2), "ld")
    f = O.fit(X, lam)
    assert g["V"][0].tobytes() == f["v"].tobytes() and int(g["J"][0]) == f["j"]


def test_workload_size_rank(ctx):
    """The 2000 x 2000 benchmark matrix, three components: the GPU's first
    component is the plain fit, each later projected matrix is orthogonal to
    the earlier directions."""
    import torch
    from paper_2402_16712_amd import binding as B
    p = wl.large_fit(0)
    lam = float(p.lambdas[0])
    out = ctx.components(B.device_matrix(p.X), lam, 3)
    f = ctx.fit(B.device_matrix(p.X), lam)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == 0
    assert out["V"][0].cpu().numpy().tobytes() == f["v"].cpu().numpy().tobytes()
    V = out["V"].cpu().numpy()
    W = []
    for c in range(2):
        w = V[c].copy()
        for q in W:
            w -= (q @ V[c]) / (q @ q) * q
        W.append(w)
    Y = out["work"].cpu().numpy()
    for w in W:
        assert np.linalg.norm(Y @ w) <= 1e-9 * np.linalg.norm(p.X) * np.linalg.norm(w)
