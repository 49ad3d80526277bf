"""Pins of the oracle's successive components (Algorithm 1 on the data
projected onto the null space of the components found so far)."""
import numpy as np

from oracle import oracle as O
from paper_2402_16712_amd import workloads as wl


def _planted(seed=0, n=300, m=10):
    rng = np.random.default_rng(seed)
    u1, u2 = rng.standard_normal(n), rng.standard_normal(n)
    l1 = np.zeros(m)
    l1[:5] = rng.uniform(0.5, 1.0, 5) * np.sign(rng.standard_normal(5))
    l2 = np.zeros(m)
    l2[5:] = rng.uniform(0.5, 1.0, 5) * np.sign(rng.standard_normal(5))
    X = np.outer(u1, l1) + 0.7 * np.outer(u2, l2) + 0.01 * rng.laplace(size=(n, m))
    return np.asfortranarray(X)


def test_first_component_is_the_fit():
    X = wl.random_small(40, 120, 8, zero_frac=0.05)
    lam = 0.05 * wl.max_column_mass(X)
    r = O.components(X, lam, 1)
    f = O.fit(X, lam)
    assert r["V"][0].tobytes() == f["v"].tobytes() and r["J"][0] == f["j"]
    assert r["OBJ"][0] == f["obj"]


def test_planted_supports_are_recovered():
    # two rank-one parts on disjoint coordinate blocks: the first component
    # is supported on one block, the second (after projecting it away) on
    # the other
    for seed in range(3):
        X = _planted(seed)
        r = O.components(X, 0.1 * wl.max_column_mass(X), 2)
        s1 = set(np.nonzero(r["V"][0])[0].tolist())
        s2 = set(np.nonzero(r["V"][1])[0].tolist())
        blocks = [set(range(5)), set(range(5, 10))]
        assert s1 in blocks and s2 in blocks and s1 != s2, (seed, s1, s2)


def test_projected_data_is_orthogonal_to_earlier_components():
    X = wl.random_small(41, 200, 9)
    lam = 0.02 * wl.max_column_mass(X)
    p = 4
    r = O.components(X, lam, p)
    # Gram-Schmidt of the components in plain floating point
    W = []
    for c in range(p - 1):
        w = r["V"][c].copy()
        for q in W:
            w -= (q @ r["V"][c]) / (q @ q) * q
        W.append(w)
    scale = np.linalg.norm(X)
    for w in W:
        assert np.linalg.norm(r["Xlast"] @ w) <= 1e-10 * scale * np.linalg.norm(w)
    # and the objectives drop as the structure is projected away
    assert r["OBJ"][0] > r["OBJ"][-1]
