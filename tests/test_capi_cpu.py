"""C ABI checks that need no GPU: the built library loads, exports every
symbol the header declares, and rejects bad arguments on the host before
any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2402_16712_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^(?:int|const char \*)\s*(l1line_\w+)\s*\(", text, re.M)
    return names


def test_library_loads_and_exports_header_symbols():
    lib = B.lib()
    names = _declared()
    assert len(names) >= 6
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(B.EXPORTS) <= set(names)


def test_strerror_names_every_code():
    for c in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10):
        assert B.strerror(c) != "unknown status"
    assert B.strerror(-99) == "unknown status"


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "l1line.h")).read()
    consts = dict(re.findall(r"#define (L1LINE_\w+) \(?(-?\d+)\)?", text))
    assert int(consts["L1LINE_MAX_N"]) == B.MAX_N
    assert int(consts["L1LINE_BP_MAX_N"]) == B.BP_MAX_N
    assert int(consts["L1LINE_MAX_LAMBDAS"]) == B.MAX_LAMBDAS
    assert int(consts["L1LINE_NOALLOC_MAX_M"]) == B.NOALLOC_MAX_M
    assert int(consts["L1LINE_EWIDE"]) == B.EWIDE and int(consts["L1LINE_ERANGE"]) == B.ERANGE


class _Fake:
    """A non-null context pointer: argument checks run before it is used."""

    def __init__(self):
        # zeroed and larger than the context structure: a rejected call
        # records its code in the context's sticky error field
        self.buf = ctypes.create_string_buffer(4096)
        self.h = ctypes.cast(self.buf, ctypes.c_void_p)


def _fit(h, X, n, m, ld, lam, v=1, j=1, obj=1):
    P = ctypes.c_void_p
    return B.lib().l1line_fit(h, P(X), n, m, ld, lam, P(v) if v else None, P(j) if j else None,
                              P(obj) if obj else None, None, None, None, None)


def test_fit_host_argument_checks():
    f = _Fake()
    assert _fit(None, 1, 10, 4, 10, 0.5) == B.EINVAL
    assert _fit(f.h, 0, 10, 4, 10, 0.5) == B.EINVAL          # null X
    assert _fit(f.h, 1, 0, 4, 10, 0.5) == B.EINVAL           # n < 1
    assert _fit(f.h, 1, 10, 0, 10, 0.5) == B.EINVAL          # m < 1
    assert _fit(f.h, 1, 10, 4, 9, 0.5) == B.EINVAL           # ld < n
    assert _fit(f.h, 1, 10, 4, 10, -1.0) == B.EINVAL         # lambda < 0
    assert _fit(f.h, 1, 10, 4, 10, float("nan")) == B.EINVAL
    assert _fit(f.h, 1, 10, 4, 10, float("inf")) == B.EINVAL
    assert _fit(f.h, 1, 10, 4, 10, 0.5, v=0) == B.EINVAL     # null output
    assert _fit(f.h, 1, B.MAX_N + 1, 4, B.MAX_N + 1, 0.5) == B.ESIZE


def test_fit_noalloc_host_argument_checks():
    f = _Fake()
    P = ctypes.c_void_p

    def call(h, X, n, m, ld, lam, v=1):
        return B.lib().l1line_fit_noalloc(h, P(X), n, m, ld, lam, P(v) if v else None, P(1), P(1), None, None,
                                          None, None)
    assert call(None, 1, 10, 4, 10, 0.5) == B.EINVAL
    assert call(f.h, 0, 10, 4, 10, 0.5) == B.EINVAL
    assert call(f.h, 1, 10, 4, 9, 0.5) == B.EINVAL
    assert call(f.h, 1, 10, 4, 10, float("nan")) == B.EINVAL
    assert call(f.h, 1, 10, 4, 10, 0.5, v=0) == B.EINVAL
    assert call(f.h, 1, B.MAX_N + 1, 4, B.MAX_N + 1, 0.5) == B.ESIZE
    assert call(f.h, 1, 10, B.NOALLOC_MAX_M + 1, 10, 0.5) == B.ESIZE


def test_path_host_argument_checks():
    f = _Fake()
    P = ctypes.c_void_p
    lib = B.lib()
    lam = np.array([0.1, 0.2, -0.3])

    def call(lams, L):
        return lib.l1line_fit_path(f.h, P(1), 10, 4, 10, lams.ctypes.data_as(P), L, P(1), P(1), P(1),
                                   None, None, None, None)
    assert call(lam, 3) == B.EINVAL                          # negative lambda
    assert call(lam, 0) == B.EINVAL                          # L < 1
    big = np.full(B.MAX_LAMBDAS + 1, 0.5)
    assert call(big, B.MAX_LAMBDAS + 1) == B.EINVAL          # too many lambdas
    assert lib.l1line_fit_path(f.h, P(1), 10, 4, 10, None, 2, P(1), P(1), P(1),
                               None, None, None, None) == B.EINVAL


def test_stats_and_create_checks():
    lib = B.lib()
    P = ctypes.c_void_p
    assert lib.l1line_column_stats(None, P(1), 5, 5, 5, None, None, None, None) == B.EINVAL
    f = _Fake()
    assert lib.l1line_column_stats(f.h, P(1), 5, 5, 4, None, None, None, None) == B.EINVAL
    assert lib.l1line_create(None, 0, None) == B.EINVAL
    assert lib.l1line_destroy(None) == B.EINVAL
    assert lib.l1line_last_error(None) == B.EINVAL


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        B.lib()


def test_batch_host_argument_checks():
    lib = B.lib()
    f = _Fake()
    P = ctypes.c_void_p
    lam = np.array([0.5, 1.0])
    good = B.Problem(1, 10, 4, 10, lam.ctypes.data, 2, 1, 1, 1, None, None, None)
    arr = (B.Problem * 2)(good, good)
    cast = ctypes.cast(arr, P)
    assert lib.l1line_fit_batch(f.h, cast, 0, 0, None) == B.EINVAL        # B < 1
    assert lib.l1line_fit_batch(f.h, None, 2, 0, None) == B.EINVAL        # null array
    assert lib.l1line_fit_batch(f.h, cast, 2, 4, None) == B.EINVAL        # unknown flag
    assert lib.l1line_fit_batch(None, cast, 2, 0, None) == B.EINVAL
    bad = (B.Problem * 2)(good, B.Problem(1, 0, 4, 10, lam.ctypes.data, 2, 1, 1, 1, None, None, None))
    assert lib.l1line_fit_batch(f.h, ctypes.cast(bad, P), 2, 0, None) == B.EINVAL   # n < 1
    neg = np.array([0.5, -1.0])
    bad2 = (B.Problem * 1)(B.Problem(1, 10, 4, 10, neg.ctypes.data, 2, 1, 1, 1, None, None, None))
    assert lib.l1line_fit_batch(f.h, ctypes.cast(bad2, P), 1, 0, None) == B.EINVAL
    big = (B.Problem * 1)(B.Problem(1, B.MAX_N + 1, 4, B.MAX_N + 1, lam.ctypes.data, 2, 1, 1, 1, None, None, None))
    assert lib.l1line_fit_batch(f.h, ctypes.cast(big, P), 1, 0, None) == B.ESIZE
    assert lib.l1line_autotune(f.h, cast, 0, None, None) == B.EINVAL
    assert lib.l1line_tune_get(None, None) == B.EINVAL
    assert lib.l1line_tune_set(None, None) == B.EINVAL


def test_ranker_host_checks():
    lib = B.lib()
    f = _Fake()
    P = ctypes.c_void_p
    assert lib.l1line_ranker_load(None, b"x") == B.EINVAL
    assert lib.l1line_ranker_load(f.h, None) == B.EINVAL
    assert lib.l1line_ranker_save(f.h, None) == B.EINVAL
    assert lib.l1line_ranker_save(f.h, b"/nonexistent/x") == B.ENOMODEL      # no weights yet
    assert lib.l1line_ranker_get_params(f.h, P(1), None) == B.ENOMODEL
    assert lib.l1line_ranker_set_params(f.h, None, None) == B.EINVAL
    assert lib.l1line_ranker_train(None, None, 10, 0) == B.EINVAL
    assert lib.l1line_ranker_train(f.h, None, -1, 0) == B.EINVAL
    out = [P(1)] * 3
    # K outside [1, m], a bad threshold, then no weights
    assert lib.l1line_fit_ranked(f.h, P(1), 10, 4, 10, 0.5, 0, 0.1, *out, None, None, None, None, None) == B.EINVAL
    assert lib.l1line_fit_ranked(f.h, P(1), 10, 4, 10, 0.5, 5, 0.1, *out, None, None, None, None, None) == B.EINVAL
    assert lib.l1line_fit_ranked(f.h, P(1), 10, 4, 10, 0.5, 2, -1.0, *out, None, None, None, None, None) == B.EINVAL
    assert lib.l1line_fit_ranked(f.h, P(1), 10, 70000, 10, 0.5, 2, 0.1, *out, None, None, None, None,
                                 None) == B.ESIZE
    assert lib.l1line_fit_ranked(f.h, P(1), 10, 4, 10, 0.5, 2, 0.1, *out, None, None, None, None,
                                 None) == B.ENOMODEL


def test_ranker_file_roundtrip(tmp_path):
    w = np.random.default_rng(0).standard_normal(B.MLP_PARAMS).astype(np.float32)
    path = tmp_path / "w.l1rk"
    B.write_ranker_file(path, w)
    assert path.stat().st_size == 40 + 4 * B.MLP_PARAMS
    r, state, head = B.read_ranker_file(path)
    assert r.tobytes() == w.tobytes() and state is None and head == dict(step=0, seed=0, cursor=0)
    bad = tmp_path / "bad.l1rk"
    bad.write_bytes(path.read_bytes()[:100])
    with pytest.raises(ValueError):
        B.read_ranker_file(bad)


def test_shipped_ranker_weights_readable():
    from paper_2402_16712_amd import ranker
    w, _, _ = B.read_ranker_file(ranker.WEIGHTS)
    assert w.shape == (B.MLP_PARAMS,) and np.all(np.isfinite(w))


def test_components_and_breakpoints_host_checks():
    lib = B.lib()
    f = _Fake()
    P = ctypes.c_void_p
    o = [P(1)] * 3
    assert lib.l1line_components(f.h, P(1), 10, 4, 10, 0.5, 0, P(1), *o, None, None) == B.EINVAL     # p < 1
    assert lib.l1line_components(f.h, P(1), 10, 4, 10, 0.5, 5, P(1), *o, None, None) == B.EINVAL     # p > m
    assert lib.l1line_components(f.h, P(1), 10, 4, 10, 0.5, 2, None, *o, None, None) == B.EINVAL     # no work
    assert lib.l1line_components(f.h, P(1), 10, 4, 10, -0.5, 2, P(1), *o, None, None) == B.EINVAL   # lambda
    assert lib.l1line_breakpoints(f.h, P(1), 10, 4, 10, None, None, None, None, None, 0, None, None) == B.EINVAL
    assert lib.l1line_breakpoints(f.h, P(1), 10, 4, 10, P(1), None, None, None, None, 5, None, None) == B.EINVAL
    assert lib.l1line_breakpoints(f.h, P(1), 10, 9000, 10, P(1), None, None, None, None, 0, None,
                                  None) == B.ESIZE
    big = B.BP_MAX_N + 1                                   # Algorithms 2 and 3 keep the smaller row limit
    assert lib.l1line_breakpoints(f.h, P(1), big, 4, big, P(1), None, None, None, None, 0, None,
                                  None) == B.ESIZE


def test_solution_path_host_checks():
    lib = B.lib()
    f = _Fake()
    P = ctypes.c_void_p
    cnt = ctypes.c_int64(0)
    o = [P(1)] * 7
    assert lib.l1line_solution_path(None, P(1), 10, 4, 10, 0, ctypes.byref(cnt), *([None] * 7), None,
                                    None) == B.EINVAL
    assert lib.l1line_solution_path(f.h, P(1), 10, 4, 10, 0, None, *([None] * 7), None, None) == B.EINVAL
    assert lib.l1line_solution_path(f.h, P(1), 10, 4, 10, -1, ctypes.byref(cnt), *o, None, None) == B.EINVAL
    assert lib.l1line_solution_path(f.h, P(1), 10, 4, 10, 5, ctypes.byref(cnt), *([None] * 7), None,
                                    None) == B.EINVAL                                     # outputs missing
    assert lib.l1line_solution_path(f.h, None, 10, 4, 10, 0, ctypes.byref(cnt), *([None] * 7), None,
                                    None) == B.EINVAL                                     # null X
    assert lib.l1line_solution_path(f.h, P(1), 10, 9000, 10, 0, ctypes.byref(cnt), *([None] * 7), None,
                                    None) == B.ESIZE
    big = B.BP_MAX_N + 1
    assert lib.l1line_solution_path(f.h, P(1), big, 4, big, 0, ctypes.byref(cnt), *([None] * 7), None,
                                    None) == B.ESIZE
