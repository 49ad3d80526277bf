"""Writes tests/golden/fullsize.json: the oracle's results on the full-size
workloads, which the oracle takes too long to recompute inside a GPU test.

    python tests/golden/make_fullsize.py [--only fit,path,batch]

Calls only the CPU oracle (oracle/) on inputs from the seeded generators
(paper_2402_16712_amd/workloads.py); nothing here touches the GPU library.
Records:
  fit    2000 x 2000, seed 0, lambda = 0.05 x max column mass (the benchmark's
         main workload): every z_j (hex), j*, z*, and SHA-256 of v* and of the
         median rows (Algorithm 1, Sec. 2).
  path   the same matrix with 64 penalties log-spaced from 1e-3 to 1 x the
         max column mass: j*(lambda_t), z*(lambda_t) (hex), and SHA-256 of
         V, ROW and ZALL (L x m, C order).
  batch  six problems of the 512-matrix uneven batch (batch seed 12345, 16
         penalties each) with 2000 <= n <= 4000 and 200 <= m <= 500: the three
         of largest n m^2 and the three of lowest index among the rest; per
         problem the same fields as path.
Cost: about 20 core-minutes (fit), 2 core-hours (path), 25 core-minutes
(batch) with the oracle on every host thread.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from paper_2402_16712_amd import workloads as wl     # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def hexes(a):
    return [float(x).hex() for x in np.asarray(a, dtype=np.float64).ravel()]


def batch_subset(probs):
    """Indices of the six config-size problems the GPU test compares."""
    elig = [b for b, p in enumerate(probs) if 2000 <= p.n <= 4000 and 200 <= p.m <= 500]
    big = sorted(elig, key=lambda b: (-probs[b].n * probs[b].m ** 2, b))[:3]
    rest = [b for b in elig if b not in big][:3]
    return sorted(big + rest)


def path_record(X, lambdas):
    r = O.fit_path(X, lambdas)
    assert r["status"] == 0
    return dict(n=int(X.shape[0]), m=int(X.shape[1]), L=int(len(lambdas)), J=[int(x) for x in r["J"]],
                OBJ=hexes(r["OBJ"]), V_sha=sha(r["V"]), ROW_sha=sha(r["ROW"].astype(np.int32)),
                ZALL_sha=sha(r["ZALL"]), lambdas=hexes(lambdas))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="fit,path,batch")
    a = ap.parse_args()
    which = set(a.only.split(","))
    rec = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            rec = json.load(f)
    rec["threads"] = O.max_threads()
    if "fit" in which:
        t = time.time()
        p = wl.large_fit(0)
        lam = float(p.lambdas[0])
        r = O.fit(p.X, lam)
        assert r["status"] == 0
        rec["fit_2000x2000_seed0"] = dict(lam=lam.hex(), j=int(r["j"]), obj=float(r["obj"]).hex(),
                                          z_all=hexes(r["z_all"]), v_sha=sha(r["v"]),
                                          row_sha=sha(r["row"].astype(np.int32)))
        print(f"fit done in {time.time() - t:.0f} s", flush=True)
    if "path" in which:
        t = time.time()
        p = wl.lambda_path(0)
        rec["path_2000x2000x64_seed0"] = path_record(p.X, p.lambdas)
        print(f"path done in {time.time() - t:.0f} s", flush=True)
    if "batch" in which:
        t = time.time()
        probs = wl.uneven_batch()
        sub = batch_subset(probs)
        rec["batch12345_subset"] = {str(b): path_record(probs[b].X, probs[b].lambdas) for b in sub}
        print(f"batch subset {sub} done in {time.time() - t:.0f} s", flush=True)
    with open(OUT + ".tmp", "w") as f:
        json.dump(rec, f, indent=0)
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
