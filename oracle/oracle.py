"""ctypes front end of the exact CPU oracle (l1line_oracle.c).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU
baseline leg import this module.  It never touches the GPU library.

All arrays are numpy; X is n x m FP64 and may be C- or F-ordered (it is
copied to column-major).  Indices are 0-based.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "l1line_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

OK, EINVAL, ENONFINITE, ERANGE, ENOMEM = 0, -1, -3, -4, -5

TIE_R3 = 0     # zero if zero minimises, else the minimiser closest to zero
TIE_ALG1 = 1   # Algorithm 1's interval test verbatim (last match wins)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                        "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.oracle_column_stats.argtypes = [P, I64, I64, I64, P, P]
        lib.oracle_segment.argtypes = [P, I64, I64, I64, I64, I64, P, I64, I, P, P, P]
        lib.oracle_fit_j.argtypes = [P, I64, I64, I64, I64, P, I64, I, P, P, P, P, P, P]
        lib.oracle_fit_path.argtypes = [P, I64, I64, I64, P, I64, I, I, P, P, P, P, P]
        lib.oracle_breakpoints.argtypes = [P, I64, I64, I64, I64, I64, I64, P, P, P, P, P]
        lib.oracle_components.argtypes = [P, I64, I64, I64, ctypes.c_double, I64, P, P, P, P]
        lib.oracle_residual.argtypes = [P, I64, I64, I64, I64, I64, ctypes.c_double, P]
        for f in (lib.oracle_column_stats, lib.oracle_segment, lib.oracle_fit_j,
                  lib.oracle_fit_path):
            f.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(X):
    X = np.asfortranarray(np.asarray(X, dtype=np.float64))
    if X.ndim != 2:
        raise ValueError("X must be 2-D")
    return X, X.shape[0], X.shape[1]


def _lams(lambdas):
    return np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))


def _check(code, what, allow_erange=False):
    if code != OK and not (allow_erange and code == ERANGE):
        raise OracleError(code, what)
    return code


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def column_stats(X):
    """(W, zeros): W_j = R64-ordered sum_i |x_ij|, zeros_j = #{x_ij == 0}."""
    X, n, m = _prep(X)
    W = np.empty(m)
    Z = np.empty(m, dtype=np.int64)
    _check(_load().oracle_column_stats(_ptr(X), n, m, n, _ptr(W), _ptr(Z)), "column_stats")
    return W, Z


def segment(X, j, k, lambdas, tie_rule=TIE_R3):
    """Per lambda: (v_k, row, e_jk) of the single problem (j, k)."""
    X, n, m = _prep(X)
    lam = _lams(lambdas)
    L = lam.size
    v = np.empty(L)
    row = np.empty(L, dtype=np.int32)
    e = np.empty(L)
    code = _load().oracle_segment(_ptr(X), n, m, n, int(j), int(k), _ptr(lam), L,
                                  int(tie_rule), _ptr(v), _ptr(row), _ptr(e))
    _check(code, "segment", allow_erange=True)
    return v, row, e


def fit_j(X, j, lambdas, tie_rule=TIE_R3):
    """Everything for one preserved coordinate j: dict of V, ROW, EJK (L x m)
    and EJ, PJ, ZJ (L)."""
    X, n, m = _prep(X)
    lam = _lams(lambdas)
    L = lam.size
    out = dict(V=np.empty((L, m)), ROW=np.empty((L, m), dtype=np.int32),
               EJK=np.empty((L, m)), EJ=np.empty(L), PJ=np.empty(L), ZJ=np.empty(L))
    code = _load().oracle_fit_j(_ptr(X), n, m, n, int(j), _ptr(lam), L, int(tie_rule),
                                _ptr(out["V"]), _ptr(out["ROW"]), _ptr(out["EJK"]),
                                _ptr(out["EJ"]), _ptr(out["PJ"]), _ptr(out["ZJ"]))
    out["status"] = _check(code, "fit_j", allow_erange=True)
    return out


def fit_path(X, lambdas, tie_rule=TIE_R3, nthreads=0):
    """Algorithm 1 for each lambda: dict V (L x m), J (L), OBJ (L),
    ROW (L x m), ZALL (L x m)."""
    X, n, m = _prep(X)
    lam = _lams(lambdas)
    L = lam.size
    out = dict(V=np.empty((L, m)), J=np.empty(L, dtype=np.int64), OBJ=np.empty(L),
               ROW=np.empty((L, m), dtype=np.int32), ZALL=np.empty((L, m)))
    code = _load().oracle_fit_path(_ptr(X), n, m, n, _ptr(lam), L, int(tie_rule), int(nthreads),
                                   _ptr(out["V"]), _ptr(out["J"]), _ptr(out["OBJ"]),
                                   _ptr(out["ROW"]), _ptr(out["ZALL"]))
    out["status"] = _check(code, "fit_path", allow_erange=True)
    return out


def fit(X, lam, tie_rule=TIE_R3, nthreads=0):
    """Algorithm 1 for one lambda: dict v (m), j, obj, row (m), z_all (m)."""
    r = fit_path(X, [lam], tie_rule, nthreads)
    return dict(v=r["V"][0], j=int(r["J"][0]), obj=float(r["OBJ"][0]), row=r["ROW"][0],
                z_all=r["ZALL"][0], status=r["status"])


def breakpoints_segment(X, j, k):
    """Algorithm 2 for one segment: (lam, v, row) entries in increasing lambda
    (the terminal entry (lambda_max, 0, -1) last) and lambda_max."""
    X, n, m = _prep(X)
    cnt = ctypes.c_int64()
    lmax = ctypes.c_double()
    _check(_load().oracle_breakpoints(_ptr(X), n, m, n, int(j), int(k), 0, None, None, None,
                                      ctypes.byref(cnt), ctypes.byref(lmax)), "breakpoints")
    c = cnt.value
    lam, v, row = np.empty(c), np.empty(c), np.empty(c, dtype=np.int32)
    _check(_load().oracle_breakpoints(_ptr(X), n, m, n, int(j), int(k), c, _ptr(lam), _ptr(v), _ptr(row),
                                      ctypes.byref(cnt), ctypes.byref(lmax)), "breakpoints")
    return lam, v, row, lmax.value


def breakpoints(X):
    """Algorithm 2 for every segment, as the GPU lays it out: offsets[m*m+1]
    (segment g = j*m + k; the diagonal has no entries), lambda_max[m*m] (0 on
    the diagonal), and the concatenated lam, v, row."""
    X, n, m = _prep(X)
    offs = [0]
    lmax = np.zeros(m * m)
    lams, vs, rows = [], [], []
    for j in range(m):
        for k in range(m):
            if k == j:
                offs.append(offs[-1])
                continue
            la, v, r, lm = breakpoints_segment(X, j, k)
            lmax[j * m + k] = lm
            lams.append(la)
            vs.append(v)
            rows.append(r)
            offs.append(offs[-1] + len(la))
    cat = (lambda a, dt: np.concatenate(a) if a else np.empty(0, dtype=dt))
    return dict(offsets=np.array(offs, dtype=np.int64), lambda_max=lmax, lam=cat(lams, np.float64),
                v=cat(vs, np.float64), row=cat(rows, np.int32))


def components(X, lam, p):
    """p successive components: dict V (p x m), J (p), OBJ (p), Xlast (the
    projected data the last component was fitted on, n x m)."""
    X, n, m = _prep(X)
    V, J, OBJ = np.empty((p, m)), np.empty(p, dtype=np.int64), np.empty(p)
    Xl = np.empty((n, m), order="F")
    code = _load().oracle_components(_ptr(X), n, m, n, float(lam), int(p), _ptr(V), _ptr(J), _ptr(OBJ), _ptr(Xl))
    st = _check(code, "components", allow_erange=True)
    return dict(V=V, J=J, OBJ=OBJ, Xlast=Xl, status=st)


def residual(X, j, k, v):
    """e_jk at a given v, R64 over the rows of |x_ik - fl(v x_ij)| (the score
    Algorithm 1 gives a selection)."""
    X, n, m = _prep(X)
    e = ctypes.c_double()
    _check(_load().oracle_residual(_ptr(X), n, m, n, int(j), int(k), float(v), ctypes.byref(e)), "residual")
    return e.value


def solution_path(X):
    """Algorithm 3 (Sec. 2): the exact solution path z*(lambda), v*(lambda)
    over every lambda >= 0, merged from the per-coordinate paths that
    Algorithm 2 gives.  Pure Python with exact rationals; small inputs only.

    Reading taken.  For a preserved coordinate j the path of Algorithm 2 fixes,
    on each interval of lambda, every v_k and so a line
        z_j(lambda) = E_j + lambda P_j,
        E_j = sum_k e_jk(v_k)  (e_jk as Algorithm 1 scores it, e_jj = 0),
        P_j = 1 + sum_{k != j} |v_k|.
    Entry t of segment (j, k) (Algorithm 2's list, lambda_t rounded once to a
    double) holds for lambda >= lambda_t until the next entry; entries that
    share a lambda apply in (k, t) order.  E_j and P_j are EXACT sums of the
    doubles e_jk and |v_k| (rationals here).  Algorithm 3 compares the lines
    of all j between consecutive breakpoints; its beta_L/beta_U are the
    crossings of the best line with the others.  Here the same merge is a
    sweep over lambda: between two consecutive breakpoints the best line at
    the left end (smallest value, then smallest slope, then smallest j) is
    followed through its crossings with lines of smaller slope; the preserved
    coordinate changes at the first crossing, to the smallest slope (then j)
    among the lines that meet there.

    Returns the records of the path in lambda order, each a dict with
      lam  where the change happens (a breakpoint, or a crossing rounded
           once to the nearest double),
      j    the preserved coordinate from there on,
      k, v, row  the coordinate of v* that takes value v (row: the median
           row, -1 when v is 0 or k = j),
      E, P the line z* = E + lambda P from there on (each rounded once).
    A change of the preserved coordinate (and the start at lambda = 0) lists
    all m coordinates k = 0..m-1 at that lambda; otherwise one record per
    breakpoint entry of the current j."""
    from fractions import Fraction as Fr

    X, n, m = _prep(X)
    one = Fr(1)
    # per j: events (lam, k, t, dE, dP, v, row) sorted by (lam, k, t)
    events = []
    for j in range(m):
        ev = []
        for k in range(m):
            if k == j:
                continue
            lam, v, row, _ = breakpoints_segment(X, j, k)
            pe, pp = Fr(0), Fr(0)
            for t in range(len(lam)):
                e = Fr(residual(X, j, k, v[t]))
                a = Fr(abs(float(v[t])))
                ev.append((float(lam[t]), k, t, e - pe, a - pp, float(v[t]), int(row[t])))
                pe, pp = e, a
        ev.sort(key=lambda x: (x[0], x[1], x[2]))
        events.append(ev)
    points = sorted({0.0} | {e[0] for ev in events for e in ev})
    E = [Fr(0)] * m
    P = [one] * m
    vcur = [[(1.0 if k == j else 0.0, -1) for k in range(m)] for j in range(m)]
    ptr = [0] * m
    out = []

    def batch(lam, j):
        for k in range(m):
            vv, rr = vcur[j][k]
            out.append(dict(lam=lam, j=j, k=k, v=vv, row=rr, E=float(E[j]), P=float(P[j])))

    cur = None
    for idx, p in enumerate(points):
        q = points[idx + 1] if idx + 1 < len(points) else None
        fp = Fr(p)
        applied = {}
        for j in range(m):
            ev = events[j]
            while ptr[j] < len(ev) and ev[ptr[j]][0] == p:
                lam, k, t, dE, dP, v, row = ev[ptr[j]]
                E[j] += dE
                P[j] += dP
                vcur[j][k] = (v, row)
                applied.setdefault(j, []).append((k, v, row, float(E[j]), float(P[j])))
                ptr[j] += 1
        new = min(range(m), key=lambda j: (E[j] + fp * P[j], P[j], j))
        if cur is None or new != cur:
            batch(p, new)
        else:
            for k, v, row, e, pp in applied.get(cur, []):
                out.append(dict(lam=p, j=cur, k=k, v=v, row=row, E=e, P=pp))
        cur = new
        # crossings strictly inside (p, q)
        while True:
            best, tied = None, []
            for s in range(m):
                if P[s] < P[cur]:
                    x = (E[s] - E[cur]) / (P[cur] - P[s])
                    if best is None or x < best:
                        best, tied = x, [s]
                    elif x == best:
                        tied.append(s)
            if best is None or (q is not None and best >= Fr(q)):
                break
            cur = min(tied, key=lambda s: (P[s], s))
            batch(float(best), cur)
    return out
