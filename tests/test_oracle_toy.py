"""Oracle pinned to the paper's worked example (Sec. 3.1: Table I, Fig. 1,
Algorithm 2's breakpoints, the maximum useful lambda and the crossing 3.5)."""
import numpy as np
import pytest

from oracle import oracle as O


def _X(toy):
    return np.array(toy["points"], dtype=np.float64)


def _interior(lo, hi):
    if hi is None:
        return [lo + 0.25, lo + 1.0, lo + 7.0]
    return [lo + (hi - lo) * f for f in (0.125, 0.5, 0.875)]


def test_table1_path(toy):
    X = _X(toy)
    rows = toy["table1"]["rows"]
    jstar = toy["table1"]["preserved_coordinate_1based"]
    for row, j1 in zip(rows, jstar):
        for lam in _interior(row["lambda_lo"], row["lambda_hi"]):
            r = O.fit(X, lam)
            assert r["j"] == j1 - 1, (lam, r["j"])
            np.testing.assert_allclose(r["v"], row["v"], atol=row["v_tol"] + 1e-15)
            assert r["v"][j1 - 1] == 1.0


def test_table1_objective_at_interval_ends(toy):
    X = _X(toy)
    eps = 1e-9
    for row in toy["table1"]["rows"]:
        lo, hi = row["lambda_lo"], row["lambda_hi"]
        z_lo = O.fit(X, lo + eps)["obj"]
        exp_lo = 43.0 if lo == 3.5 else row["z_lo"]     # 42.9 misprint, see golden note
        assert abs(z_lo - exp_lo) < row["z_tol"] + 1e-6
        if hi is not None:
            z_hi = O.fit(X, hi - eps)["obj"]
            exp_hi = 43.0 if hi == 3.5 else row["z_hi"]
            assert abs(z_hi - exp_hi) < row["z_tol"] + 1e-6


def test_exact_table1_values(toy):
    # integer data: every weight sum is exact, so the values are exact too
    X = _X(toy)
    r = O.fit(X, 1.0)
    assert r["v"].tolist() == [-2.0 / 3.0, 1.0 / 3.0, -0.5, 1.0]
    r = O.fit(X, 5.0)
    assert r["v"].tolist() == [1.0, 0.0, 0.0, -0.2]
    assert r["obj"] == 38.8 + 1.2 * 5.0 or abs(r["obj"] - 44.8) < 1e-13


def test_fig1_lines(toy):
    X = _X(toy)
    for ln in toy["fig1"]["lines"]:
        j = ln["jhat"] - 1
        for lam in _interior(ln["lo"], ln["hi"]):
            f = O.fit_j(X, j, [lam])
            E, P, Z = f["EJ"][0], f["PJ"][0], f["ZJ"][0]
            assert abs(E - ln["intercept"]) <= ln["tol"] + 1e-12, (ln, E)
            assert abs(P - ln["slope"]) <= ln["tol"] + 1e-12, (ln, P)
            assert abs(Z - (E + lam * P)) <= 1e-12 * Z


def test_fig1_exact_thirds(toy):
    # the lines printed with rounded digits are exact fractions
    X = _X(toy)
    f = O.fit_j(X, 3, [8.0])
    assert abs(f["EJ"][0] - 113.0 / 3.0) < 1e-12 and abs(f["PJ"][0] - 5.0 / 3.0) < 1e-15
    f = O.fit_j(X, 2, [1.0])
    assert abs(f["EJ"][0] - 131.0 / 3.0) < 1e-12 and abs(f["PJ"][0] - 13.0 / 6.0) < 1e-15


def _slope_changes(X, j, grid):
    out = []
    prev = None
    for lam in grid:
        f = O.fit_j(X, j, [lam])
        key = (round(f["EJ"][0], 9), round(f["PJ"][0], 9))
        if prev is not None and key != prev[1]:
            out.append(prev[0])
        prev = (lam, key)
    return out


def test_breakpoints(toy):
    X = _X(toy)
    grid = np.arange(0.0, 14.0, 0.125)
    expect = {int(k): v for k, v in toy["breakpoints"]["printed"].items()}
    expect[1] = [1, 3, 11]          # reading noted in the golden file
    for j1, bps in expect.items():
        got = _slope_changes(X, j1 - 1, grid)
        # solution changes exactly at each breakpoint b: last grid value <= b
        # with the old solution is b itself (v changes for lambda >= b)
        want = [b - 0.125 for b in bps if b > 0]
        assert got == want, (j1, got, want)
        if 0 in bps:
            # a v_k already zero at lambda = 0 (its lambda_max is 0)
            v0 = O.fit_j(X, j1 - 1, [0.0])["V"][0]
            assert np.sum(v0 == 0.0) >= 1


def test_max_lambda(toy):
    X = _X(toy)
    lmax = toy["max_lambda"]["value"]
    for lam in (lmax, lmax + 0.5, 100.0):
        r = O.fit(X, lam)
        assert np.count_nonzero(r["v"]) == 1 and r["v"][r["j"]] == 1.0
    r = O.fit(X, lmax - 0.01)
    assert np.count_nonzero(r["v"]) == 2


def test_crossing_breakpoint(toy):
    X = _X(toy)
    c = toy["crossing"]
    assert O.fit(X, c["value"] - 1e-6)["j"] == c["from_jhat"] - 1
    assert O.fit(X, c["value"] + 1e-6)["j"] == c["to_jhat"] - 1
    # exact tie of the two lines at 3.5: the lowest index wins (strict "<")
    assert O.fit(X, c["value"])["j"] == min(c["from_jhat"], c["to_jhat"]) - 1
    z = O.fit(X, c["value"])["z_all"]
    assert z[c["from_jhat"] - 1] == z[c["to_jhat"] - 1] == 43.0


def test_lambda_max_per_segment_toy():
    # lambda at which each v_k reaches 0, per (jhat, k): the slope changes of Fig. 1
    X = np.array([[4, -2, 3, -6], [-3, 4, 2, -1], [2, 3, -3, -2], [-3, 4, 2, 3], [5, 3, 2, -1]], float)
    want = {0: [3, 1, 11], 1: [4, 6, 4], 2: [2, 0, 2], 3: [11, 5, 3]}
    for j, lams in want.items():
        ks = [k for k in range(4) if k != j]
        for k, lm in zip(ks, lams):
            v, _, _ = O.segment(X, j, k, [lm, lm + 1e-9] + ([lm - 1e-6] if lm > 0 else []))
            assert v[0] == 0.0 and v[1] == 0.0
            if lm > 0:
                assert v[2] != 0.0


def test_alg1_literal_rule_differs_only_at_ties(toy):
    """The verbatim Algorithm 1 test and rule R3 reach the same objective on a
    lambda grid of the toy; their v differ only where g_jk has a flat piece."""
    X = _X(toy)
    diffs = []
    for lam in np.arange(0.0, 15.0, 0.25):
        for j in range(4):
            a = O.fit_j(X, j, [lam], tie_rule=O.TIE_R3)
            b = O.fit_j(X, j, [lam], tie_rule=O.TIE_ALG1)
            assert abs(a["ZJ"][0] - b["ZJ"][0]) > -1  # both defined
            for k in range(4):
                if a["V"][0, k] != b["V"][0, k]:
                    diffs.append((float(lam), j + 1, k + 1))
                    # both are minimisers of the same segment: same segment cost
                    assert abs(a["EJK"][0, k] + lam * abs(a["V"][0, k])
                               - b["EJK"][0, k] - lam * abs(b["V"][0, k])) < 1e-12
    assert sorted(diffs) == [(0.0, 3, 2), (1.0, 1, 3), (5.0, 4, 2), (6.0, 2, 3)]
