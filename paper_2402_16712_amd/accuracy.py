"""Error and sparsity of Algorithm 1 as the penalty varies (Sec. 3, "Effect
of Varying m and n on Error and Sparsity"; the curves of its Fig. 3).

For each size (n fixed at 3000 with m = 1000, 2000, 3000; m fixed at 1000
with n = 1000, 2000, 3000) and five seeds, a matrix from
workloads.accuracy_matrix is fitted by the library over a grid of penalties
in one l1line_fit_path call, and each v*(lambda) is compared with the true
direction v:
  discordance(v, v*) = 1 - |<v, v*>| / (||v|| ||v*||)  (0: the same line,
                        1: orthogonal; the sign of a line's direction is
                        immaterial)
  sparsity          = ||v*||_0 / m  (share of nonzero coordinates)
averaged over the seeds, per penalty.  The paper names the error measure
"discordance" without defining it; this is the reading taken.

    python -m paper_2402_16712_amd.accuracy [--seeds 5] [--L 64]
"""
from __future__ import annotations

import json

import numpy as np

from . import binding as B
from . import workloads as wl

# (n, m) settings and the penalty range of each panel of the figure
PANEL_A = {"sizes": [(3000, 1000), (3000, 2000), (3000, 3000)], "lam_max": 8500.0}
PANEL_B = {"sizes": [(1000, 1000), (2000, 1000), (3000, 1000)], "lam_max": 5500.0}


def discordance(v, w) -> float:
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    nv, nw = np.linalg.norm(v), np.linalg.norm(w)
    if nv == 0.0 or nw == 0.0:
        return 1.0
    return float(1.0 - abs(np.dot(v, w)) / (nv * nw))


def sparsity(w) -> float:
    w = np.asarray(w)
    return float(np.count_nonzero(w)) / w.size


def run(ctx: B.Context, sizes, lambdas, seeds):
    """Mean discordance and sparsity per penalty for each size: dict
    "n x m" -> {"discordance": [L], "sparsity": [L], "j": [[L] per seed]}."""
    import torch
    out = {}
    for n, m in sizes:
        disc = np.zeros(len(lambdas))
        spars = np.zeros(len(lambdas))
        js = []
        for seed in seeds:
            X, v = wl.accuracy_matrix(n, m, seed)
            r = ctx.fit_path(B.device_matrix(X), lambdas, rows=False, z_all=False)
            torch.cuda.synchronize()
            if int(r["status"].item()) != 0:
                raise RuntimeError(f"fit status {int(r['status'].item())} for {n}x{m} seed {seed}")
            V = r["V"].cpu().numpy()
            disc += np.array([discordance(v, V[t]) for t in range(len(lambdas))])
            spars += np.array([sparsity(V[t]) for t in range(len(lambdas))])
            js.append([int(x) for x in r["J"].cpu().numpy()])
        out[f"{n}x{m}"] = {"discordance": (disc / len(seeds)).tolist(), "sparsity": (spars / len(seeds)).tolist(),
                           "j": js}
    return out


def _main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--seeds", type=int, default=5)
    ap.add_argument("--L", type=int, default=64)
    a = ap.parse_args(argv)
    ctx = B.Context(0)
    seeds = list(range(a.seeds))
    for name, panel in (("a", PANEL_A), ("b", PANEL_B)):
        lam = np.linspace(0.0, panel["lam_max"], a.L)
        res = run(ctx, panel["sizes"], lam, seeds)
        print(json.dumps({"panel": name, "lambdas": lam.tolist(), "results": res}), flush=True)
    ctx.close()


if __name__ == "__main__":
    _main()
