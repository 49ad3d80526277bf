"""Pins of the oracle's Algorithm 2 (breakpoints of every segment):
the worked example of Sec. 3.1, the solution of Algorithm 1 (itself pinned by
brute force and LP) inside every interval the breakpoints delimit, and
Lemma 1's exact threshold for lambda_max."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_16712_amd import workloads as wl


def test_toy_breakpoint_sets(toy):
    # per preserved coordinate: the positive breakpoints and the lambda_max of
    # every other column (Sec. 3.1 prints them; 11 for jhat = 1 is read from
    # Fig. 1, see the fixture's note)
    X = np.asfortranarray(np.array(toy["points"], dtype=float))
    printed = {int(k): set(v) for k, v in toy["breakpoints"]["printed"].items()}
    printed[1] = printed[1] | {11}
    for j in range(4):
        got = set()
        for k in range(4):
            if k == j:
                continue
            lam, v, row, lmax = O.breakpoints_segment(X, j, k)
            got |= {float(x) for x in lam[:-1] if x > 0} | {lmax}
            assert lam[-1] == lmax and v[-1] == 0.0 and row[-1] == -1
            assert lam[0] == 0.0 and np.all(np.diff(lam) >= 0)
        assert got == printed[j + 1], (j + 1, got)


def _cases():
    out = []
    for seed in range(4):
        out.append(wl.random_small(600 + seed, 9 + seed, 5, zero_frac=0.1))
        out.append(wl.random_small(700 + seed, 12, 4, integer=True, zero_frac=0.1, span=3))
    out.append(wl.rank_one_matrix(40, 5, 5, 0, 20.0, 0.0, (31, 0), laplace_b=0.05))
    return out


@pytest.mark.parametrize("case", range(9))
def test_intervals_reproduce_algorithm_1(case):
    """Inside every interval [lam_t, lam_t+1) the fit of Algorithm 1 (rule
    R3) selects exactly (v_t, row_t); beyond lambda_max it gives 0."""
    X = _cases()[case]
    n, m = X.shape
    for j in range(m):
        for k in range(m):
            if k == j:
                continue
            lam, v, row, lmax = O.breakpoints_segment(X, j, k)
            probes, want = [], []
            for t in range(len(lam) - 1):
                if lam[t + 1] > lam[t]:
                    probes.append(0.5 * (lam[t] + lam[t + 1]))
                    want.append((v[t], row[t]))
            probes.append(2.0 * lmax + 1.0)
            want.append((0.0, -1))
            probes.append(0.0)
            want.append((v[0], row[0]))
            gv, gr, _ = O.segment(X, j, k, np.array(probes))
            for (wv, wr), a, b, lp in zip(want, gv, gr, probes):
                assert (a, b) == (wv, wr), (case, j, k, lp)


def test_lambda_max_is_lemma_1_threshold():
    """lambda_max = max(0, |D| - Zr) with D the signed weight of the ratios
    and Zr the weight of the zero ratios, in exact rationals."""
    for X in _cases():
        n, m = X.shape
        for j in range(m):
            for k in range(m):
                if k == j:
                    continue
                D, Zr = Fraction(0), Fraction(0)
                for i in range(n):
                    a, b = X[i, j], X[i, k]
                    if a == 0.0:
                        continue
                    r = b / a + 0.0
                    w = Fraction(abs(a))
                    if r > 0:
                        D += w
                    elif r < 0:
                        D -= w
                    else:
                        Zr += w
                want = max(Fraction(0), abs(D) - Zr)
                _, _, _, lmax = O.breakpoints_segment(X, j, k)
                assert lmax == float(want), (j, k)


def test_layout_of_all_segments():
    X = _cases()[0]
    n, m = X.shape
    r = O.breakpoints(X)
    off = r["offsets"]
    assert off[0] == 0 and len(off) == m * m + 1 and np.all(np.diff(off) >= 0)
    for j in range(m):
        assert off[j * m + j + 1] == off[j * m + j]        # no segment on the diagonal
    assert len(r["lam"]) == off[-1] == len(r["v"]) == len(r["row"])
