"""Benchmark: exhaustive fits of the sparse robust l1 line on one GPU.

One step = one call of the whole hot path (column prep, every (j, k)
weighted median with its residual, the per-j objectives, the argmin) on a
2000 x 2000 FP64 matrix resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--legs path,batch,ranked]

Besides the main line it reports, as extra fields, the 64-penalty path on
the same matrix, the 512-matrix uneven batch, the learned top-K fit,
Algorithm 2 (every segment's breakpoints), three successive components of
the same matrix and Algorithm 3 (the exact solution path over every lambda).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (the roofline denominators; the measured ceilings
# of l1line_measure_peaks are reported beside them)
PEAK_FP64_TFLOPS = 78.6        # FP64 vector (an FMA counts 2)
PEAK_FP64_MFMA_TFLOPS = 78.6   # FP64 matrix
PEAK_HBM_GBPS = 8000.0
CLOCK_HZ = 2.4e9
SIMDS = 256 * 4


def algorithmic_work(X):
    """FP64 operations the method performs on one exhaustive fit, by the
    plain algorithm: every ratio element (x_ij != 0, k != j) one IEEE divide
    and one prefix-sum add; every residual term (all n rows of every (j, k),
    k != j) one multiply, one subtract and one add (the absolute value is a
    sign bit).  Elements skipped by the sign-sum test still count: the
    figure measures the method's work per second."""
    n, m = X.shape
    elements = float(np.count_nonzero(X, axis=0).sum()) * (m - 1)
    residual_terms = float(n) * m * (m - 1)
    return {"ratio_elements": elements, "residual_terms": residual_terms,
            "flops": 2.0 * elements + 3.0 * residual_terms}


SS_ROWS = 16   # rows per LDS stage of k_signsum_batch


def signsum_mfma_issued(X):
    """FP64 MFMAs k_signsum_batch issues on X (column-major n x m): the
    matrix is staged in SS_ROWS-row steps and 64-column tiles (zero padded);
    per 64 x 64 output tile, every block of 4 rows x 16 columns k costs one
    16x16x4 MFMA per wave (4 waves) for D, and one more for Zr only when the
    block holds an exact zero (padding included)."""
    n, m = X.shape
    n_pad, m_pad = -(-n // SS_ROWS) * SS_ROWS, -(-m // 64) * 64
    Z = np.ones((n_pad, m_pad), dtype=bool)
    Z[:n, :m] = (X == 0.0)
    blocks_zero = int(Z.reshape(n_pad // 4, 4, m_pad // 16, 16).any(axis=(1, 3)).sum())
    blocks = (n_pad // 4) * (m_pad // 16)
    jtiles = m_pad // 64
    return {"mfma_D": blocks * jtiles * 4, "mfma_Zr": blocks_zero * jtiles * 4, "flops_per_mfma": 2 * 16 * 16 * 4}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-columns", type=int, default=0, help="oracle sample size (columns j)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 512 MiB device buffer 3 times (scale for HBM byte counters)")
    ap.add_argument("--legs", default="path,batch,ranked,breakpoints,components,solution_path",
                    help="extra workloads reported beside the main line (comma list; '' for none)")
    ap.add_argument("--ranked-instances", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="time with the default launch parameters only")
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV [SQ_CSV]: turn rocprofv3 counter files "
                         "(bench run and --calibrate-copy run) into profiles/traffic.json and exit")
    return ap.parse_args()


def calibrate_copy():
    """Three device-to-device copies of exactly 512 MiB: the FETCH_SIZE /
    WRITE_SIZE counters of these dispatches give the counters' scale."""
    import torch
    nbytes = 512 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}))


def _source_hash():
    """Hash of the sources that define the segment kernels (the counters in
    profiles/traffic.json are only used while these are unchanged)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_16712_amd", "csrc")
    for f in ("device_common.h", "fit_kernels.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _counters(kernel_key):
    """The committed counter record of the dominant kernel (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE, SQ instruction counts), if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != _source_hash():
        return None
    return rec


def _pmc_per_dispatch(path, counter):
    """Mean counter value (KiB) per dispatch of each kernel in a rocprofv3
    counter_collection.csv."""
    import csv
    import collections
    tot, disp = collections.defaultdict(float), collections.defaultdict(set)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            # kernel name without "void ", template arguments and parameters
            k = r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").strip()
            tot[k] += float(r["Counter_Value"])
            disp[k].add(r["Dispatch_Id"])
    return {k: tot[k] / len(disp[k]) for k in tot}


def pmc_summary(fetch_csv, write_csv, copyf_csv, copyw_csv, sq_csv=None, lds_csv=None):
    """The dominant kernel's counter record: HBM bytes per launch of
    k_seg_batch from the FETCH_SIZE and WRITE_SIZE counters, each scaled by
    what the counter reads for a copy of exactly 512 MiB (bench.py
    --calibrate-copy), (optional) SQ_INSTS_VALU / SQ_INSTS_LDS per launch
    and (optional) SQ_LDS_IDX_ACTIVE / GRBM_GUI_ACTIVE per launch."""
    nbytes = 512 << 20
    cf = _pmc_per_dispatch(copyf_csv, "FETCH_SIZE")["__amd_rocclr_copyBuffer"] * 1024
    cw = _pmc_per_dispatch(copyw_csv, "WRITE_SIZE")["__amd_rocclr_copyBuffer"] * 1024
    fs, ws = nbytes / cf, nbytes / cw
    f = _pmc_per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _pmc_per_dispatch(write_csv, "WRITE_SIZE")
    kern = "k_seg_batch"
    fetch = f[kern] * 1024 * fs
    write = w[kern] * 1024 * ws
    rec = {"kernel": kern, "bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
           "fetch_scale": fs, "write_scale": ws,
           "raw_kib": {"FETCH_SIZE": f[kern], "WRITE_SIZE": w[kern]}, "source_hash": _source_hash()}
    if sq_csv:
        rec["sq_insts_valu"] = _pmc_per_dispatch(sq_csv, "SQ_INSTS_VALU")[kern]
        rec["sq_insts_lds"] = _pmc_per_dispatch(sq_csv, "SQ_INSTS_LDS")[kern]
    if lds_csv:
        rec["sq_lds_idx_active"] = _pmc_per_dispatch(lds_csv, "SQ_LDS_IDX_ACTIVE")[kern]
        rec["grbm_gui_active"] = _pmc_per_dispatch(lds_csv, "GRBM_GUI_ACTIVE")[kern]
    out = {"seg_2000x2000": rec}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, lam, z_gpu, columns):
    """The oracle timed on the host: a bounded sample of candidate columns j
    (all k for each) of the timed workload on every host thread (a thread
    pool over j) and on one thread, one warm-up then three timed runs each
    (fits/s from the best run); every sampled z_j compared with the GPU's bit
    for bit.  Also the 200 x 20 workload in full, both ways."""
    from oracle import oracle as O
    from paper_2402_16712_amd import workloads as wl
    O.build()
    cores = max(1, min(os.cpu_count() or 1, 32))
    m = p.X.shape[1]
    if columns <= 0:
        columns = 2 * cores
    rng = np.random.default_rng(1)
    js = sorted(rng.choice(m, size=min(columns, m), replace=False).tolist())
    X = np.asfortranarray(p.X)

    def one(j):
        return j, O.fit_j(X, j, [lam])["ZJ"][0]

    def timed(fn, runs=3):
        fn()                                              # warm-up
        best = float("inf")
        for _ in range(runs):
            t0 = time.perf_counter()
            out = fn()
            best = min(best, time.perf_counter() - t0)
        return out, best

    def pool():
        with ThreadPoolExecutor(max_workers=cores) as ex:
            return list(ex.map(one, js))

    res, dt = timed(pool)
    mism = [j for j, z in res if np.float64(z).tobytes() != np.float64(z_gpu[j]).tobytes()]
    js1 = js[:max(1, len(js) // cores)]
    _, dt1 = timed(lambda: [one(j) for j in js1])
    small = wl.small_fit(0)
    slam = float(small.lambdas[0])
    _, ds_all = timed(lambda: O.fit(small.X, slam, nthreads=cores))
    _, ds_one = timed(lambda: O.fit(small.X, slam, nthreads=1))
    return dict(value=(len(js) / m) / dt, unit="fits/s", cores=cores, kind="oracle",
                sample=f"{len(js)} of {m} candidate columns j (all k each) of the timed workload on "
                       f"{cores} threads, best of 3 runs after a warm-up ({dt:.2f} s); fits/s = (columns/m)/s",
                single_thread=(len(js1) / m) / dt1,
                single_thread_sample=f"{len(js1)} columns on 1 thread, best of 3 ({dt1:.2f} s)",
                cpu_model=_cpu_model(),
                small_fit_200x20={"fits_per_s_all_threads": 1.0 / ds_all, "fits_per_s_one_thread": 1.0 / ds_one},
                z_mismatches=len(mism))


def _timed(fn, steps, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / steps


def leg_path(ctx, seed, steps, stream):
    """Lambda path: 2000 x 2000, 64 penalties, one call."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl
    p = wl.lambda_path(seed)
    X = B.device_matrix(p.X)
    ctx.fit_path(X, p.lambdas)
    out, ms = _timed(lambda: ctx.fit_path(X, p.lambdas, rows=False, z_all=False), steps, stream)
    st = int(out["status"].item())
    n, m = p.X.shape
    L = len(p.lambdas)
    return {"workload": f"lambda path {n}x{m} FP64, {L} penalties log-spaced 1e-3..1 x max column mass",
            "ms_per_call": ms, "fits_per_s": L * 1000.0 / ms, "medians_per_s": m * (m - 1) * L * 1000.0 / ms,
            "status": st}


def leg_batch(ctx, steps, stream):
    """512 uneven problems (n 50..4000, m 10..500, 16 penalties each), one
    batch call replayed from a captured graph: with the default launch
    parameters, then with the autotuned entry of the batch's size class."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl
    probs = wl.uneven_batch()
    dev = [(B.device_matrix(p.X), p.lambdas) for p in probs]
    arr, outs, keep = ctx._batch_args(dev, False, False)

    def timed():
        ctx.fit_batch_prepared(arr, len(dev), graph=True)       # capture
        ctx.fit_batch_prepared(arr, len(dev), graph=True)       # replay
        return _timed(lambda: ctx.fit_batch_prepared(arr, len(dev), graph=True), steps, stream)[1]

    default_params, _ = ctx.tune_lookup(dev)
    default_ms = timed()
    tuned = ctx.autotune(dev)
    ms = timed()
    bad = sum(int(o["status"].item()) != 0 for o in outs)
    medians = sum(p.m * (p.m - 1) * len(p.lambdas) for p in probs)
    del keep
    return {"workload": "512 uneven matrices n~U{50..4000} m~U{10..500}, 16 penalties each, graph replay",
            "ms_per_batch": ms, "problems_per_s": len(probs) * 1000.0 / ms,
            "medians_per_s": medians * 1000.0 / ms, "nonzero_status": bad,
            "launch_params": {"tuned": tuned, "default": list(default_params), "default_ms_per_batch": default_ms}}


def leg_breakpoints(ctx, seed, steps, stream):
    """Algorithm 2 on the main workload's 2000 x 2000 matrix: every
    segment's breakpoints and lambda_max (count pass, offsets, entries)."""
    import torch
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl
    p = wl.large_fit(seed)
    X = B.device_matrix(p.X)
    n, m = p.X.shape
    out = ctx.breakpoints(X)                      # sizes the outputs
    total = int(out["offsets"][-1].item())
    lib, ptr = B.lib(), B._ptr

    def call():
        return lib.l1line_breakpoints(ctx._h, ptr(X), n, m, n, ptr(out["offsets"]), ptr(out["lambda_max"]),
                                      ptr(out["lam"]), ptr(out["v"]), ptr(out["row"]), total, ptr(out["status"]),
                                      ctx._stream())
    call()
    _, ms = _timed(call, steps, stream)
    torch.cuda.synchronize()
    return {"workload": f"Algorithm 2, all {m * (m - 1)} segments of the {n}x{m} matrix",
            "ms_per_call": ms, "entries": total, "entries_per_s": total * 1000.0 / ms,
            "segments_per_s": m * (m - 1) * 1000.0 / ms, "status": int(out["status"].item())}


def leg_components(ctx, seed, steps, stream):
    """Three successive components of the main workload's matrix (fit,
    projection, fit, projection, fit)."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl
    p = wl.large_fit(seed)
    X = B.device_matrix(p.X)
    lam = float(p.lambdas[0])
    ctx.components(X, lam, 3)
    out, ms = _timed(lambda: ctx.components(X, lam, 3), steps, stream)
    n, m = p.X.shape
    return {"workload": f"3 successive components of the {n}x{m} matrix, lambda = 0.05 x max column mass",
            "ms_per_call": ms, "components_per_s": 3000.0 / ms, "status": int(out["status"].item())}


def leg_solution_path(ctx, seed, steps, stream):
    """Algorithm 3 on the main workload's 2000 x 2000 matrix: the exact
    solution path over every lambda (Algorithm 2's entries, their residuals,
    per-coordinate sort into exact lines, tile pruning, the sweep), with the
    time of each stage."""
    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl
    p = wl.large_fit(seed)
    X = B.device_matrix(p.X)
    n, m = p.X.shape
    first = ctx.solution_path(X)                  # sizes the outputs
    cap = first["count"]
    out, ms = _timed(lambda: ctx.solution_path(X, capacity=cap), steps, stream)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    ctx.solution_path(X, capacity=cap)
    stages = {name: ctx.profile_read(name)[0] for name in ("bp_count", "bp_emit", "sp_resid", "sp_delta", "sp_sort",
                                                           "sp_bounds", "sp_sweep")}
    ctx.profile_read(reset=True)
    ctx.profile(False)
    lam = out["lam"].cpu().numpy()
    jj = out["j"].cpu().numpy()
    switches = int(np.count_nonzero(jj[1:] != jj[:-1]))
    return {"workload": f"Algorithm 3, the exact solution path of the {n}x{m} matrix over every lambda >= 0",
            "ms_per_call": ms, "records": int(out["count"]), "preserved_coordinate_changes": switches,
            "lambda_top": float(lam[-1]) if lam.size else 0.0, "stage_ms": stages,
            "status": int(out["status"].item())}


def leg_ranked(ctx, count):
    """Learned top-K (K = 32) vs exhaustive on 10000 x 4000 matrices."""
    import os
    from paper_2402_16712_amd import ranker
    if not os.path.exists(ranker.WEIGHTS):
        return {"skipped": "no trained ranker weights in the package"}
    ctx.ranker_load(ranker.WEIGHTS)
    # one warm-up instance outside the statistics (allocations, first launches)
    ranker.evaluate(ctx, [ranker.EVAL_BASE + 10 ** 6], n=2000, m=500)
    rows = ranker.evaluate(ctx, [ranker.EVAL_BASE + q for q in range(count)], n=10000, m=4000)
    te = sum(r["t_exhaustive"] for r in rows)
    tk = sum(r["t_ranked"] for r in rows)
    return {"workload": f"ranked fit, {count} matrices 10000x4000 FP64, K=32, margin 0.05, lambda 0.05 x mass",
            "exhaustive_fits_per_s": len(rows) / te, "ranked_fits_per_s": len(rows) / tk,
            "speedup": te / tk, "within_1e-9": sum(r["ok"] for r in rows) / len(rows),
            "fallback_rate": sum(r["fallback"] for r in rows) / len(rows),
            "statuses_nonzero": sum(1 for r in rows if r["status"] != (0, 0))}


def main():
    a = _args()
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.pmc_summary:
        pmc_summary(*a.pmc_summary)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2402_16712_amd import binding as B
    from paper_2402_16712_amd import workloads as wl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    p = wl.large_fit(a.seed)
    n, m = p.X.shape
    lam = float(p.lambdas[0])
    ctx = B.Context(0)
    X = B.device_matrix(p.X)
    stream = torch.cuda.current_stream()

    # the default launch parameters, then the autotuned ones of this size
    # class (tuning runs before the timed region)
    out = ctx.fit(X, lam)
    torch.cuda.synchronize()
    _, default_ms = _timed(lambda: ctx.fit(X, lam, rows=False, z_all=False), max(3, a.steps // 2), stream)
    default_params = ctx.tune_get()
    tuned_params = ctx.autotune([(X, [lam])]) if not a.no_tune else default_params
    for _ in range(a.warmup):
        out = ctx.fit(X, lam)
    torch.cuda.synchronize()

    ctx.profile(True)
    ctx.profile_read(reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(a.steps):
        out = ctx.fit(X, lam)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern = {}
    for name in ("colprep", "signsum", "zero_seg", "fit_seg", "reduce", "argmin"):
        ms, cnt = ctx.profile_read(name)
        kern[name] = ms / max(cnt, 1)
    ctx.profile_read(reset=True)
    ctx.profile(False)

    st = int(out["status"].item())
    if st != 0:
        raise SystemExit(f"fit status {st}: {B.strerror(st)}")
    ms_per_step = total_ms / a.steps
    fits_per_s = 1000.0 / ms_per_step
    medians = m * (m - 1)
    z_gpu = out["z_all"].cpu().numpy()
    j_star = int(out["j"].item())

    # roofline of the dominant kernel, k_seg_batch (one launch = the m(m-1)
    # segments of one fit), against the method's algorithmic FP64 work
    work = algorithmic_work(p.X)
    seg_s = kern["fit_seg"] / 1000.0
    achieved = work["flops"] / seg_s / 1e12
    peaks = ctx.measure_peaks()
    rec = _counters("seg_2000x2000")
    roof = {"bound": "alu", "kernel": "k_seg_batch", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": rec.get("bytes_per_launch") if rec else None,
            "work": dict(work, basis="per fit: 2 flops per ratio element (IEEE divide, prefix-sum add), "
                                     "3 per residual term (mul, sub, add)"),
            "avg_launch_ms": kern["fit_seg"],
            "peak_measured": peaks["fp64_valu_TFLOPs"], "frac_measured": achieved / peaks["fp64_valu_TFLOPs"]}
    if rec and rec.get("sq_insts_valu"):
        # VALU issue: every wave64 instruction occupies a SIMD for 4 cycles
        busy = rec["sq_insts_valu"] * 4.0 / (SIMDS * CLOCK_HZ * seg_s)
        roof["issue"] = {"valu_instructions_per_launch": rec["sq_insts_valu"],
                         "lds_instructions_per_launch": rec.get("sq_insts_lds"),
                         "valu_busy": busy,
                         "basis": "SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz x launch time)"}
    if rec and rec.get("sq_insts_lds") and rec.get("sq_lds_idx_active") and rec.get("grbm_gui_active"):
        # the window lists' sort and scan run through the LDS: its index
        # unit's busy share of the launch (GRBM_GUI_ACTIVE sums the 8 XCDs'
        # cycles, SQ_LDS_IDX_ACTIVE the 256 CUs'), and the bytes moved if
        # every LDS instruction moves 8 bytes per lane, against the measured
        # LDS read peak
        lds_bytes = rec["sq_insts_lds"] * 64 * 8
        roof["lds"] = {"instructions_per_launch": rec["sq_insts_lds"],
                       "busy": rec["sq_lds_idx_active"] / (256 * rec["grbm_gui_active"] / 8),
                       "bytes_est": lds_bytes, "achieved_GBps_est": lds_bytes / seg_s / 1e9,
                       "peak_measured_GBps": peaks["lds_GBps"],
                       "frac_est": lds_bytes / seg_s / 1e9 / peaks["lds_GBps"],
                       "basis": "busy = SQ_LDS_IDX_ACTIVE / (256 CUs x GRBM_GUI_ACTIVE / 8 XCDs); bytes = "
                                "SQ_INSTS_LDS x 64 lanes x 8 B (the list keys and column j are 8-byte entries)"}

    # the sign-sum contraction on the FP64 matrix units: the MFMAs the
    # kernel issues (the Zr product only for 4 x 16 blocks holding a zero)
    mf = signsum_mfma_issued(p.X)
    ss_flops = (mf["mfma_D"] + mf["mfma_Zr"]) * mf["flops_per_mfma"]
    ss_s = kern["signsum"] / 1000.0
    roof_ss = {"bound": "mfma", "kernel": "k_signsum_batch", "achieved": ss_flops / ss_s / 1e12,
               "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s (FP64 matrix)",
               "frac": ss_flops / ss_s / 1e12 / PEAK_FP64_MFMA_TFLOPS, "flops_per_launch": ss_flops,
               "mfma_issued": mf, "avg_launch_ms": kern["signsum"],
               "peak_measured": peaks["fp64_mfma_TFLOPs"],
               "frac_measured": ss_flops / ss_s / 1e12 / peaks["fp64_mfma_TFLOPs"]}

    line = {
        "metric": "fits/s & weighted-medians/s, 2000x2000 FP64; learned top-K vs exhaustive",
        "value": fits_per_s,
        "unit": "fits/s",
        "medians_per_s": fits_per_s * medians,
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"exhaustive fit {n}x{m} FP64 (rank-one signal, Laplace noise, "
                               f"10% outlier rows, 1% zeros), lambda = 0.05 * max column mass, "
                               f"all {m} candidate j", "n": n, "m": m, "L": 1, "seed": a.seed,
                   "launch_params": {"tuned": tuned_params, "default": default_params,
                                     "default_ms_per_step": default_ms}},
        "kernels_ms": kern,
        "roofline": roof,
        "roofline_signsum": roof_ss,
        "peaks_measured": peaks,
        "j_star": j_star,
    }
    legs = [x for x in a.legs.split(",") if x]
    if "path" in legs:
        line["path"] = leg_path(ctx, a.seed, 3, stream)
    if "batch" in legs:
        line["batch"] = leg_batch(ctx, 3, stream)
    if "ranked" in legs:
        line["ranked"] = leg_ranked(ctx, a.ranked_instances)
    if "breakpoints" in legs:
        line["breakpoints"] = leg_breakpoints(ctx, a.seed, 3, stream)
    if "components" in legs:
        line["components"] = leg_components(ctx, a.seed, 3, stream)
    if "solution_path" in legs:
        line["solution_path"] = leg_solution_path(ctx, a.seed, 3, stream)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, lam, z_gpu, a.cpu_columns)
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
