"""Pins of the oracle's Algorithm 3 (the exact solution path z*(lambda),
v*(lambda) merged over the preserved coordinates): the worked example of
Sec. 3.1 (Table I and the crossing at 3.5), and, inside every interval the
path reports, an independent evaluation through Algorithm 1's per-segment
selection at that lambda with every line summed exactly; exact invariances
under scaling by a power of two and row sign flips; the final piece beyond
every lambda_max."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_16712_amd import workloads as wl


def _toy(toy):
    return np.asfortranarray(np.array(toy["points"], dtype=float))


def _intervals(rec):
    """Replay the records: list of (lam_lo, lam_hi, j, v, E, P) for every
    maximal interval of constant (j, v)."""
    m = max(r["k"] for r in rec) + 1
    out = []
    v = [0.0] * m
    i = 0
    while i < len(rec):
        lam = rec[i]["lam"]
        while i < len(rec) and rec[i]["lam"] == lam:
            r = rec[i]
            v[r["k"]] = r["v"]
            j, E, P = r["j"], r["E"], r["P"]
            i += 1
        hi = rec[i]["lam"] if i < len(rec) else float("inf")
        out.append((lam, hi, j, list(v), E, P))
    return out


def test_toy_table_1(toy):
    rec = O.solution_path(_toy(toy))
    iv = _intervals(rec)
    rows = toy["table1"]["rows"]
    assert len(iv) == len(rows)
    for (lo, hi, j, v, E, P), row in zip(iv, rows):
        assert lo == pytest.approx(row["lambda_lo"], abs=1e-12)
        if row["lambda_hi"] is None:
            assert hi == float("inf")
        else:
            assert hi == pytest.approx(row["lambda_hi"], abs=1e-12)
        assert np.allclose(v, row["v"], atol=row["v_tol"])
        assert E + lo * P == pytest.approx(row["z_lo"], abs=row["z_tol"] + 0.1 * (row["z_lo"] == 42.9))
    # the crossing that Algorithm 3 adds: from jhat = 4 to jhat = 1 at 3.5
    cr = toy["crossing"]
    sw = [r for r in rec if r["lam"] > 3.0 and r["lam"] < 11.0]
    assert {r["j"] for r in sw} == {cr["to_jhat"] - 1}
    assert sw[0]["lam"] == pytest.approx(cr["value"], rel=1e-14)
    before = [r for r in rec if r["lam"] <= 3.0]
    assert {r["j"] for r in before} == {cr["from_jhat"] - 1}
    # the lines either side of the crossing (Fig. 1): 36 + 2 lambda, 38.8 + 1.2 lambda
    assert (iv[1][4], iv[1][5]) == (36.0, 2.0)
    assert iv[2][4] == pytest.approx(38.8, abs=1e-12) and iv[2][5] == pytest.approx(1.2, abs=1e-15)
    # beyond lambda = 11 only the preserved coordinate is nonzero: 41 + lambda
    assert iv[-1][2] == 0 and iv[-1][4] == 41.0 and iv[-1][5] == 1.0


def _cases():
    return [
        wl.random_small(910, 9, 4),
        wl.random_small(911, 12, 5, zero_frac=0.15),
        wl.random_small(912, 10, 5, integer=True, span=3),
        wl.random_small(913, 14, 6, integer=True, span=2, zero_frac=0.1),
        wl.rank_one_matrix(30, 6, 3, 3, 20.0, 0.0, (41, 0), laplace_b=0.1),
        wl.random_small(1003, 8, 10, integer=True, span=2),   # four changes of j
        wl.random_small(1004, 12, 12),
    ]


def _all_breakpoints(X):
    n, m = X.shape
    out = set()
    for j in range(m):
        for k in range(m):
            if k != j:
                out |= {float(x) for x in O.breakpoints_segment(X, j, k)[0]}
    return sorted(out)


def _exact_lines(X, lam):
    """Every z_j(lam) from Algorithm 1's own selection at lam (oracle
    segment), summed exactly: list of (value, slope, v, row)."""
    n, m = X.shape
    out = []
    for j in range(m):
        E, P = Fraction(0), Fraction(1)
        v, row = [0.0] * m, [-1] * m
        v[j] = 1.0
        for k in range(m):
            if k == j:
                continue
            vk, rk, ek = O.segment(X, j, k, [lam])
            v[k], row[k] = float(vk[0]), int(rk[0])
            E += Fraction(float(ek[0]))
            P += Fraction(abs(float(vk[0])))
        out.append((E + Fraction(lam) * P, P, v, row))
    return out


@pytest.mark.parametrize("case", range(7))
def test_intervals_match_algorithm_1(case):
    """Inside every interval the path reports, the preserved coordinate is
    the exact argmin (value, then j) of the lines Algorithm 1's selection
    gives at that lambda, v* is that selection, and E + lambda P is its value
    (rounded once)."""
    X = _cases()[case]
    rec = O.solution_path(X)
    bps = _all_breakpoints(X)
    iv = _intervals(rec)
    assert iv[0][0] == 0.0 and iv[-1][1] == float("inf")
    for lo, hi, j, v, E, P in iv:
        if hi == float("inf"):
            cands = [2 * lo + 1.0, 3 * lo + 2.5]
        else:
            cands = [lo + f * (hi - lo) for f in (0.5, 0.3141, 0.7071, 0.123, 0.877)]
        # stay clear of every segment's breakpoint (rounded to a double)
        cands = [c for c in cands if lo < c < hi and all(abs(c - b) > 1e-9 * max(1.0, b) for b in bps)]
        assert cands, (lo, hi)
        lam = cands[0]
        lines = _exact_lines(X, lam)
        best = min(range(len(lines)), key=lambda t: (lines[t][0], t))
        assert best == j, (lam, best, j)
        assert lines[best][2] == v
        assert float(lines[best][1]) == P
        assert float(lines[best][0]) == pytest.approx(E + lam * P, rel=1e-15)


@pytest.mark.parametrize("case", [0, 2, 4])
def test_scaling_by_power_of_two_is_exact(case):
    X = _cases()[case]
    a = O.solution_path(X)
    b = O.solution_path(np.asfortranarray(X * 2.0 ** 7))
    assert len(a) == len(b)
    for r, s in zip(a, b):
        assert s["lam"] == r["lam"] * 2 ** 7 and s["E"] == r["E"] * 2 ** 7 and s["P"] == r["P"]
        assert (s["j"], s["k"], s["v"], s["row"]) == (r["j"], r["k"], r["v"], r["row"])


def test_row_sign_flip_is_exact():
    X = _cases()[1]
    Y = X.copy(order="F")
    Y[[0, 3, 7], :] *= -1.0
    assert O.solution_path(X) == O.solution_path(Y)


@pytest.mark.parametrize("case", [1, 3])
def test_final_piece(case):
    """Beyond every lambda_max all v_k are 0: the last line is
    sum_{k != j} W_k + lambda, smallest for the heaviest column (first on
    ties, with the masses summed exactly)."""
    X = _cases()[case]
    n, m = X.shape
    W, _ = O.column_stats(X)
    rest = [sum(Fraction(float(W[k])) for k in range(m) if k != j) for j in range(m)]
    jb = min(range(m), key=lambda j: (rest[j], j))
    last = _intervals(O.solution_path(X))[-1]
    assert last[2] == jb and last[5] == 1.0 and last[4] == float(rest[jb])
    assert [x for t, x in enumerate(last[3]) if t != jb] == [0.0] * (m - 1)


def test_switch_records_are_continuous():
    """Where the preserved coordinate changes inside an interval, the old and
    new lines meet (the crossing, rounded once)."""
    for X in _cases():
        rec = O.solution_path(X)
        iv = _intervals(rec)
        for a, b in zip(iv, iv[1:]):
            if a[2] != b[2]:
                lam = b[0]
                za, zb = a[4] + lam * a[5], b[4] + lam * b[5]
                assert za == pytest.approx(zb, rel=1e-12)


def test_duplicate_columns_tie_to_the_lower_index():
    """Two equal columns give the same line for either preserved coordinate;
    the lower index is kept everywhere (ties go to the first j)."""
    X = wl.random_small(1004, 12, 12)
    j0 = O.solution_path(X)[0]["j"]
    for twin in (3, 11):
        Y = X.copy(order="F")
        Y[:, twin] = Y[:, j0]
        js = {r["j"] for r in O.solution_path(Y)}
        assert min(j0, twin) in js and max(j0, twin) not in js
