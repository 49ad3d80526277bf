"""Training and evaluation of the learned candidate ranker.

The labels are the exact per-column objectives z_j of Algorithm 1 computed by
the library's exhaustive GPU fit; the target of column j is its normalized
gap (z_j - min z) / (mean z - min z), so lower scores mean better
candidates.  Forward, backward and Adam run in the library's HIP kernels.

Two trainers: the library's own loop (l1line_ranker_train, the `train`
command below: matrices generated on the device, checkpoints in the
library's ranker file format) and `Trainer`, the same steps driven from
Python through the C ABI on matrices from workloads.ranker_matrix_torch.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import binding as B
from . import workloads as wl


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases; FP32 flat vector."""
    rng = wl._rng(9, seed)
    P = np.zeros(B.MLP_PARAMS, dtype=np.float64)
    i = 0
    for fan_in, fan_out in ((32, 128), (128, 128)):
        P[i:i + fan_in * fan_out] = rng.standard_normal(fan_in * fan_out) * np.sqrt(2.0 / fan_in)
        i += fan_in * fan_out + fan_out
    P[i:i + 128] = rng.standard_normal(128) * np.sqrt(1.0 / 128)
    return P.astype(np.float32)


def targets(z):
    """Normalized gap of the exact objectives (torch tensor in, float32 out)."""
    import torch
    z = z.to(torch.float64)
    lo, mean = z.min(), z.mean()
    span = (mean - lo) if float(mean - lo) > 0 else torch.tensor(1.0, dtype=torch.float64, device=z.device)
    return ((z - lo) / span).to(torch.float32).contiguous()


class Trainer:
    def __init__(self, ctx: B.Context, seed: int = 0, lr: float = 1e-3):
        import torch
        self.ctx = ctx
        dev = ctx._torch_device
        self.params = torch.from_numpy(init_params(seed)).to(dev)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.step = 0
        self.cursor = 0
        self.lr = lr

    def example(self, index: int, **kw):
        """(features, targets) of training matrix `index`."""
        X, lam = wl.ranker_matrix_torch(index, device=self.ctx._torch_device, **kw)
        out = self.ctx.fit(X, lam)
        F = self.ctx.features(X, lam)
        return F, targets(out["z_all"])

    def train_step(self, F, y):
        grad, loss = self.ctx.mlp_grad(self.params, F, y)
        self.step += 1
        self.ctx.mlp_adam(self.params, self.m1, self.m2, grad, self.step, self.lr)
        return loss

    def train(self, n_examples: int, log_every: int = 0, **kw):
        losses = []
        for _ in range(n_examples):
            F, y = self.example(self.cursor, **kw)
            losses.append(self.train_step(F, y))
            self.cursor += 1
            if log_every and self.cursor % log_every == 0:
                print(f"ranker step {self.step} loss {float(losses[-1].item()):.4g}", flush=True)
        return losses

    def save(self, path: str):
        np.savez(path, params=self.params.cpu().numpy(), m1=self.m1.cpu().numpy(),
                 m2=self.m2.cpu().numpy(), step=np.int64(self.step), cursor=np.int64(self.cursor),
                 lr=np.float64(self.lr))

    def load(self, path: str):
        import torch
        with np.load(path, allow_pickle=False) as d:
            dev = self.ctx._torch_device
            self.params = torch.from_numpy(d["params"]).to(dev)
            self.m1 = torch.from_numpy(d["m1"]).to(dev)
            self.m2 = torch.from_numpy(d["m2"]).to(dev)
            self.step = int(d["step"])
            self.cursor = int(d["cursor"])
            self.lr = float(d["lr"])


def load_params(path: str, device="cuda:0"):
    """Weights of a ranker file as a device tensor."""
    import torch
    w, _, _ = B.read_ranker_file(path)
    return torch.from_numpy(w).to(device)


def evaluate(ctx: B.Context, indices, K: int = 32, margin: float = 0.05, rel_tol: float = 1e-9, **kw):
    """Ranked fit (the context's weights) vs exhaustive fit on evaluation
    matrices: within rel_tol of the exhaustive objective, fallback, times."""
    import torch
    rows = []
    for idx in indices:
        X, lam = wl.ranker_matrix_torch(idx, device=ctx._torch_device, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ex = ctx.fit(X, lam, rows=False, z_all=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rk = ctx.fit_ranked(X, lam, K, margin)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ze, zr = float(ex["obj"].item()), float(rk["obj"].item())
        rows.append(dict(index=idx, z_exhaustive=ze, z_ranked=zr, ok=abs(zr - ze) <= rel_tol * abs(ze),
                         fallback=int(rk["used_fallback"].item()), t_exhaustive=t1 - t0, t_ranked=t2 - t1,
                         status=(int(ex["status"].item()), int(rk["status"].item()))))
    return rows


def ablation(ctx: B.Context, indices, params_trained, params_untrained, K: int = 32, margin: float = 0.05,
             rel_tol: float = 1e-9, **kw):
    """What the trained network gains: on each evaluation matrix, the exact
    z_j of every column (exhaustive fit) judge four rankings of the columns
    -- the trained MLP, the same MLP with untrained (He-init) weights, the
    column l1 mass alone (heaviest first: z_j falls with W_j) and the slope
    aggregate A1 alone (feature 6, largest first).  For each: whether the
    optimal column is among the K best ranked (hit), whether the best exact
    objective among those K is within rel_tol of the optimum (what the
    ranked fit returns when it does not fall back), and whether the MLP's
    score margin would trigger the exhaustive fallback."""
    import torch
    rows = []
    for idx in indices:
        X, lam = wl.ranker_matrix_torch(idx, device=ctx._torch_device, **kw)
        ex = ctx.fit(X, lam)
        F = ctx.features(X, lam)
        z = ex["z_all"].to(torch.float64)
        zstar = float(z.min().item())
        jstar = int(ex["j"].item())
        m = z.numel()
        scores = {"trained": ctx.mlp_forward(params_trained, F).to(torch.float64),
                  "untrained": ctx.mlp_forward(params_untrained, F).to(torch.float64),
                  "column_mass": -X.abs().sum(dim=0),
                  "slope_aggregate": -F[:, 6].to(torch.float64)}
        row = {"index": idx, "n": int(X.shape[0]), "m": m}
        kk = min(K, m)
        for name, sc in scores.items():
            sc = torch.where(torch.isnan(sc), torch.full_like(sc, float("inf")), sc)
            order = torch.argsort(sc, stable=True)
            top = order[:kk]
            best = float(z[top].min().item())
            # rank of the optimal column (0 = ranked first; ties in the
            # score broken by the lower index, as the device's top-K does)
            rank = int((order == jstar).nonzero()[0, 0].item())
            r = {"hit": bool((top == jstar).any().item()), "within": abs(best - zstar) <= rel_tol * abs(zstar),
                 "rank": rank}
            if name in ("trained", "untrained") and kk < m:
                r["fallback"] = bool(float((sc[order[kk]] - sc[order[0]]).item()) < margin)
            row[name] = r
        rows.append(row)
    return rows


def ablation_summary(rows):
    out = {"instances": len(rows)}
    for name in ("trained", "untrained", "column_mass", "slope_aggregate"):
        ranks = [r[name]["rank"] for r in rows]
        out[name] = {"hit_rate": sum(r[name]["hit"] for r in rows) / len(rows),
                     "within_rate": sum(r[name]["within"] for r in rows) / len(rows),
                     "top_k_rate": {str(k): sum(x < k for x in ranks) / len(rows) for k in (1, 2, 4, 8, 16, 32)},
                     "mean_rank": sum(ranks) / len(rows)}
        if "fallback" in rows[0][name]:
            fb = [r[name]["fallback"] for r in rows]
            out[name]["fallback_rate"] = sum(fb) / len(rows)
            # the ranked fit's outcome: exact after a fallback, else the top-K optimum
            out[name]["within_rate_with_fallback"] = sum(
                r[name]["within"] or r[name]["fallback"] for r in rows) / len(rows)
    return out


EVAL_BASE = 90000        # evaluation matrices (10000 x 4000) are 90000, 90001, ...
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ranker_weights.l1rk")


def _main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train / evaluate the candidate ranker on the GPU")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="native training loop (l1line_ranker_train)")
    t.add_argument("--steps", type=int, default=20000)
    t.add_argument("--seed", type=int, default=1)
    t.add_argument("--ckpt", default="ranker_ckpt.l1rk", help="checkpoint (resumed if present)")
    t.add_argument("--out", default=WEIGHTS, help="trained weights")
    t.add_argument("--chunk", type=int, default=2000, help="steps between progress lines")
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--count", type=int, default=300)
    e.add_argument("--n", type=int, default=10000)
    e.add_argument("--m", type=int, default=4000)
    e.add_argument("--K", type=int, default=32)
    e.add_argument("--margin", type=float, default=0.05)
    b = sub.add_parser("ablation", help="trained vs untrained weights vs column mass vs slope aggregate")
    b.add_argument("--weights", default=WEIGHTS)
    b.add_argument("--count", type=int, default=300)
    b.add_argument("--n", type=int, default=10000)
    b.add_argument("--m", type=int, default=4000)
    b.add_argument("--K", type=int, default=32)
    b.add_argument("--margin", type=float, default=0.05)
    b.add_argument("--init-seed", type=int, default=1)
    a = ap.parse_args(argv)
    ctx = B.Context(0)
    if a.cmd == "train":
        t0 = time.perf_counter()
        done = 0
        while done < a.steps:
            done = min(a.steps, done + a.chunk)
            ctx.ranker_train(done, a.seed, a.ckpt)
            print(json.dumps({"steps": done, "s": round(time.perf_counter() - t0, 2)}), flush=True)
        w, _, _ = B.read_ranker_file(a.ckpt)
        B.write_ranker_file(a.out, w)
    elif a.cmd == "ablation":
        import torch
        trained = load_params(a.weights, ctx._torch_device)
        untrained = torch.from_numpy(init_params(a.init_seed)).to(ctx._torch_device)
        rows = []
        for q in range(a.count):
            r = ablation(ctx, [EVAL_BASE + q], trained, untrained, a.K, a.margin, n=a.n, m=a.m)[0]
            rows.append(r)
            print(json.dumps(r), flush=True)
        print(json.dumps(ablation_summary(rows)), flush=True)
    else:
        ctx.ranker_load(a.weights)
        rows = []
        for q in range(a.count):
            r = evaluate(ctx, [EVAL_BASE + q], a.K, a.margin, n=a.n, m=a.m)[0]
            rows.append(r)
            print(json.dumps(r), flush=True)
        ok = sum(r["ok"] for r in rows)
        fb = sum(r["fallback"] for r in rows)
        te = sum(r["t_exhaustive"] for r in rows)
        tk = sum(r["t_ranked"] for r in rows)
        print(json.dumps({"instances": len(rows), "within_1e-9": ok / len(rows), "fallback_rate": fb / len(rows),
                          "exhaustive_fits_per_s": len(rows) / te, "ranked_fits_per_s": len(rows) / tk,
                          "speedup": te / tk}), flush=True)
    ctx.close()


if __name__ == "__main__":
    _main()
