"""The pins are not vacuous: plant a plausible mistake in a copy of the
oracle (on the CPU), rebuild it, and check that at least one pin fails."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from tests import test_oracle_exact as TE
from tests import test_oracle_toy as TT
import json

SRC = os.path.join(os.path.dirname(O.__file__), "l1line_oracle.c")

MUTANTS = {
    "tie_gt_to_ge": ("if (big_cmp(&twoS, &WpL) > 0) return p;",
                     "if (big_cmp(&twoS, &WpL) >= 0) return p;"),
    "zero_test_strict": ("big_cmp(&W, &twoBpL) <= 0)", "big_cmp(&W, &twoBpL) < 0)"),
    "residual_sign": ("double diff = XAT(X, ld, i, k) - prod;",
                      "double diff = XAT(X, ld, i, k) + prod;"),
    "drop_own_penalty": ("vv[t * m + k] = 1.0;", "vv[t * m + k] = 0.0;"),
    "signed_weight": ("pts[np].w = fabs(xj);", "pts[np].w = xj > 0 ? xj : 0.5 * -xj;"),
    "argmin_last_tie": ("if (Z[j * L + t] < Z[best * L + t]) best = j;",
                        "if (Z[j * L + t] <= Z[best * L + t]) best = j;"),
    "row_order_reversed": ("if (a->row < b->row) return -1;\n    if (a->row > b->row) return 1;",
                           "if (a->row > b->row) return -1;\n    if (a->row < b->row) return 1;"),
    "positive_side_off_by_one": ("for (int64_t p = N + Z; p < np; ++p) {",
                                 "for (int64_t p = N + Z + (Z > 0); p < np; ++p) {"),
}


def _battery(toy):
    """A quick subset of the pins; raises AssertionError on the first failure."""
    TT.test_table1_path(toy)
    TT.test_fig1_lines(toy)
    TT.test_crossing_breakpoint(toy)
    TT.test_lambda_max_per_segment_toy()
    for case in TE.CASES[:16] + TE.CASES[-8:]:
        TE.test_bruteforce_segments(*case)
    for seed in range(4):
        TE.test_lambda_max_closed_form(seed)
        TE.test_dual_certificate(seed)


@pytest.fixture(scope="module")
def toy_data():
    with open(os.path.join(os.path.dirname(__file__), "golden", "toy.json")) as f:
        return json.load(f)


def test_unmutated_passes_battery(toy_data):
    _battery(toy_data)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, toy_data):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared",
                    "-fPIC", "-o", str(so), str(mut), "-lm"], check=True)
    real = O._load()
    lib = ctypes.CDLL(str(so))
    for fn in ("oracle_column_stats", "oracle_segment", "oracle_fit_j", "oracle_fit_path"):
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
        getattr(lib, fn).restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    O._lib = lib
    try:
        with pytest.raises((AssertionError, O.OracleError)):
            _battery(toy_data)
    finally:
        O._lib = real
