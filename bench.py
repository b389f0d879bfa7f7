"""Benchmark: Tucker-compressed Matern grids per second at n = 256^3, eps = 1e-6 (one MI355X).

One step = the whole path over one batch: the 9 Matern covariances (nu in {1/2, 3/2, 5/2} x
ell in {0.1, 0.3, 1.0}, sigma2 = 1) sampled on the 256^3 offset grid of [-1, 1]^3 (h = 2/255)
are compressed by one tk_compress_batch call (per grid: grid evaluation, three Gram
contractions, eigensolves, 2 HOOI sweeps, core, error norm, eps truncation; three groups of three
grids, each group sharing every launch, run concurrently on the context's worker streams); then
one tk_quadratic_form_batch call, per grid the quadratic form with a seeded N(0,1) FP32 vector
(the Kronecker-Toeplitz covariance matvec y = C z and z^T y; the five FFT passes of the grids run
back to back, their small preambles on a worker stream), and per grid tk_trace.  Inputs (the z
vectors, made on the device by tk_normal_fill: Philox4x32-10 keyed by the master seed and the
grid) are resident in HBM before the timed region.  Inside it only the roofline kernel (the
axis-0 FFT pass) is bracketed by HIP events.  After it, one more quadratic-form batch times the
other FFT passes, and each grid is compressed alone, --alone-reps passes over the nine grids
(single-request latency p50/p99 over 27 compressions by default; per-class kernel times without
the overlap of the batch).  The compression-only rate is also reported against its algorithmic
bound, and the FP64 oracle is timed on all host cores and on one.

Prints one JSON line (see the keys below).  --gpus N with N > 1 exits: the benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp32_mfma_TFs": 157.3, "fp64_mfma_TFs": 78.6, "bf16_mfma_TFs": 2516.6}


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def kernel_source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1711_06874_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(n, rows_sample, seed_stream, threads=None):
    """Time the FP64 oracle on a bounded sample of the same workload: one 256^3 compress
    (Matern 1/2, ell = 0.1, eps = 1e-6, 2 HOOI sweeps) plus `rows_sample` rows of the plain
    covariance product; the matvec time is extrapolated to all n^3 rows.  threads: the oracle's
    OpenMP thread count (None: all host cores)."""
    import numpy as np
    from oracle import oracle as o
    import synth
    o.build()
    all_threads = o.num_threads()
    if threads:
        o.set_num_threads(threads)
    try:
        k = o.Kernel(o.MATERN, nu=0.5, ell=0.1)
        g = o.Grid(n=(n, n, n), layout=o.OFFSET)
        t0 = time.perf_counter()
        t = o.compress(k, g, eps=1e-6, sweeps=2)
        t1 = time.perf_counter()
        z = o.normal_philox(n ** 3, synth.MASTER_SEED, seed_stream).astype(np.float64)
        rows = (np.arange(rows_sample, dtype=np.int64) * 1000003) % (n ** 3)
        t2 = time.perf_counter()
        o.cov_matvec_rows(t, g, z, rows)
        t3 = time.perf_counter()
        cores = o.num_threads()
    finally:
        o.set_num_threads(all_threads)
    per_row = (t3 - t2) / rows_sample
    grid_s = (t1 - t0) + per_row * n ** 3
    return {
        "value": 1.0 / grid_s, "unit": "grids/s", "cores": cores, "kind": "oracle",
        "sample": (f"one {n}^3 Matern nu=1/2 ell=0.1 compress (eps 1e-6, 2 HOOI sweeps) = {t1 - t0:.2f} s, "
                   f"plus {rows_sample} rows of the plain covariance product ({per_row * 1e3:.1f} ms/row) "
                   f"extrapolated to all {n ** 3} rows"),
        "compress_s": t1 - t0, "matvec_row_s": per_row,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--alone-reps", type=int, default=3,
                    help="passes over the nine grids compressed one at a time after the timed region")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1711_06874_amd import tk

    torch.cuda.set_device(0)
    n = args.n
    prec = tk.TK_FP32 if args.prec == "fp32" else tk.TK_BF16X3
    ctx = tk.Context(0)
    kernels = synth.c2_kernels(include_slater=False)
    tkernels = [tk.make_kernel(k.family, nu=k.nu, ell=k.ell, sigma2=k.sigma2) for k in kernels]
    grid = tk.make_grid(n, 1.0, tk.TK_OFFSET)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    # seeded N(0,1) vectors made on the device (Philox4x32-10 keyed by the master seed and the grid)
    zs = [torch.empty((n, n, n), dtype=torch.float32, device="cuda") for _ in kernels]
    for i, z in enumerate(zs):
        tk.tk_normal_fill(ctx.handle, synth.MASTER_SEED, i + 1, z)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # tile shapes: the Gram split count of each mode, tuned for this grid and precision (untimed)
    tuned = ctx.autotune(grid, prec, stream)
    grids = [grid] * len(tkernels)
    lat = {"compress_batch": [], "quadform_batch": [], "trace": []}
    ranks_seen = []

    def step(record):
        t0 = time.perf_counter()
        ts = ctx.compress_batch(tkernels, grids, opts, stream)
        t1 = time.perf_counter()
        ta = time.perf_counter()
        ctx.quadratic_form_batch(ts, zs, io=tk.TK_FP32, stream=stream)
        tb = time.perf_counter()
        if record:
            lat["quadform_batch"].append((tb - ta) * 1e3)
        for i, t in enumerate(ts):
            tb = time.perf_counter()
            ctx.trace(t, stream)
            tc = time.perf_counter()
            if record:
                lat["trace"].append((tc - tb) * 1e3)
                ranks_seen.append((t.ranks, t.rel_err))
        if record:
            lat["compress_batch"].append((t1 - t0) * 1e3)
        for t in ts:
            t.free()

    for _ in range(args.warmup):
        step(False)
    tk.tk_profile_reset()
    # inside the timed region only the roofline kernel's launches are bracketed by events (each
    # event pair costs its stream a few microseconds); the other classes are timed afterwards
    tk.tk_profile_select(["fft_axis0"])
    tk.tk_profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    tk.tk_profile_enable(False)
    elapsed = t_end - t_start
    n_grids = len(tkernels) * args.steps
    value = n_grids / elapsed
    timed = {}
    for name, cls in tk.PROF_CLASSES.items():
        launches, ms = tk.tk_profile_read(cls)
        timed[name] = {"launches": launches, "ms": ms}
    tk.tk_profile_reset()

    # ---- untimed: one quadratic-form batch with every class bracketed (the FFT passes other
    # than the roofline kernel)
    tk.tk_profile_select(None)
    ts = ctx.compress_batch(tkernels, grids, opts, stream)
    torch.cuda.synchronize()
    tk.tk_profile_enable(True)
    ctx.quadratic_form_batch(ts, zs, io=tk.TK_FP32, stream=stream)
    torch.cuda.synchronize()
    tk.tk_profile_enable(False)
    qf = {}
    for name, cls in tk.PROF_CLASSES.items():
        launches, ms = tk.tk_profile_read(cls)
        qf[name] = {"launches": launches, "ms": ms}
    tk.tk_profile_reset()
    for t in ts:
        t.free()

    # ---- untimed: each grid compressed alone on the caller's stream (single-request latency, and
    # per-class kernel times free of the overlap inside the batch)
    alone_ms = []
    tk.tk_profile_enable(True)
    for _ in range(args.alone_reps):
        for k in tkernels:
            t0 = time.perf_counter()
            t = ctx.compress(k, grid, opts, stream)
            alone_ms.append((time.perf_counter() - t0) * 1e3)
            t.free()
    torch.cuda.synchronize()
    tk.tk_profile_enable(False)
    alone = {}
    for name, cls in tk.PROF_CLASSES.items():
        launches, ms = tk.tk_profile_read(cls)
        alone[name] = {"launches": launches, "ms": ms}
    tk.tk_profile_reset()

    # ---- algorithmic work per class
    N = n ** 3
    m = n                                   # offset layout: the operator acts on all n^3 points
    L = 1
    while L < 2 * m - 1:
        L *= 2
    H2 = L // 2 + 1
    fft_bytes = (4.0 * N + 8.0 * m * m * H2) + (8.0 * m * m * H2 + 8.0 * m * L * H2) \
        + (8.0 * m * L * H2 + 8.0 * m * m * H2) + (8.0 * m * m * H2 + 4.0 * N)
    axis0_bytes = 16.0 * m * L * H2
    n_alone = len(tkernels) * args.alone_reps
    work_alone = {
        "grid": 4.0 * N * n_alone,                                  # bytes written (FP32)
        "gram": 3 * float(n) ** 3 * (n + 1) * n_alone,              # unique Gram entries x 2 flops
        "ttm": 4.0 * N * alone["ttm"]["launches"],                  # each launch streams the tensor once
        "norm": 4.0 * N * alone["norm"]["launches"],
    }
    work_timed = {"fft_axis0": axis0_bytes * n_grids}
    work_qf = {"fft": fft_bytes * len(tkernels)}
    bound = {"grid": ("hbm", "GB/s", PEAK["hbm_GBs"]), "gram": ("mfma", "TFLOP/s", PEAK["fp32_mfma_TFs"]),
             "ttm": ("hbm", "GB/s", PEAK["hbm_GBs"]), "norm": ("hbm", "GB/s", PEAK["hbm_GBs"]),
             "fft": ("hbm", "GB/s", PEAK["hbm_GBs"]), "fft_axis0": ("hbm", "GB/s", PEAK["hbm_GBs"])}
    if prec == tk.TK_BF16X3:
        bound["gram"] = ("mfma", "TFLOP/s", PEAK["bf16_mfma_TFs"] / 3.0)
    kernels_out = {}
    for name, (b, unit, peak) in bound.items():
        if name in work_timed:
            src, w, where = timed, work_timed, "timed region"
        elif name in work_qf:
            src, w, where = qf, work_qf, "one quadratic-form batch after the timed region"
        else:
            src, w, where = alone, work_alone, "grids compressed alone"
        ms = src[name]["ms"]
        if ms <= 0:
            continue
        scale = 1e-9 if unit == "GB/s" else 1e-12
        achieved = w[name] * scale / (ms * 1e-3)
        kernels_out[name] = {"bound": b, "unit": unit, "ms_total": ms, "launches": src[name]["launches"],
                             "achieved": achieved, "peak": peak, "frac": achieved / peak, "measured": where}
    for name in ("eig", "small"):
        kernels_out[name] = {"bound": "latency", "ms_total": alone[name]["ms"], "launches": alone[name]["launches"],
                             "measured": "grids compressed alone"}
    # the roofline kernel: the largest single bandwidth-bound kernel of the timed region, the
    # axis-0 pass of the FFT matvec (the other FFT class spans four kernels; the eigensolver
    # kernels are latency-bound single work-groups that overlap across the grids of a batch)
    dom = "fft_axis0"
    d = kernels_out[dom]

    # HBM traffic from rocprofv3 counters, valid only for the kernel source it was taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            ent = tj.get(dom)
            if ent and ent.get("source_hash") == kernel_source_hash(ent["sources"]):
                traffic = ent["bytes_per_launch"]
        except Exception:
            traffic = None

    roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                "frac": d["frac"], "traffic": traffic,
                "ms_per_launch": d["ms_total"] / max(1, d["launches"])}

    # compression alone against its algorithmic bound: HBM traffic (20 + 8 s) n^3 bytes (grid
    # write, three Gram reads, two A-streaming products per sweep, the error norm; s = 2 sweeps)
    # at peak bandwidth plus the unique Gram flops 3 n^3 (n + 1) at the MFMA peak of the precision
    sweeps = 2
    gram_peak = PEAK["fp32_mfma_TFs"] if prec == tk.TK_FP32 else PEAK["bf16_mfma_TFs"] / 3.0
    bound_s = (20 + 8 * sweeps) * float(N) / (PEAK["hbm_GBs"] * 1e9) + 3 * float(n) ** 3 * (n + 1) / (gram_peak * 1e12)
    cb_p50 = percentile(lat["compress_batch"], 50)
    compress_rate = len(tkernels) / (cb_p50 * 1e-3)
    compress_out = {"grids_per_s": compress_rate, "bound_grids_per_s": 1.0 / bound_s,
                    "frac": compress_rate * bound_s,
                    "measured": "p50 of the timed steps' compress_batch calls (nine grids each)"}

    out = {
        "metric": "Tucker-compressed Matern grids/sec at n=256^3, eps=1e-6",
        "value": value, "unit": "grids/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == tk.TK_FP32 else "bf16x3+f32", "data": "synthetic",
        "config": {"workload": f"9 Matern covariances (nu 1/2,3/2,5/2 x ell 0.1,0.3,1.0) on the {n}^3 offset grid "
                               f"of [-1,1]^3: compress at eps 1e-6 with 2 HOOI sweeps, covariance matvec + "
                               f"quadratic form with a seeded N(0,1) vector, trace",
                   "n": n, "grids_per_step": len(tkernels), "eps": 1e-6, "hooi_sweeps": 2,
                   "precision": args.prec},
        "latency_ms": dict({k: {"p50": percentile(v, 50), "p99": percentile(v, 99)} for k, v in lat.items()},
                           compress_alone={"p50": percentile(alone_ms, 50), "p99": percentile(alone_ms, 99)}),
        "ranks": sorted(set(r for r, _ in ranks_seen)),
        "max_rel_err": max(e for _, e in ranks_seen),
        "roofline": roofline,
        "compress": compress_out,
        "kernels": kernels_out,
        "gram_autotune": {"tile_per_mode": [128 if c >= (1 << 20) else 64 for c in tuned["nsplit"]],
                          "nsplit_per_mode": [c % (1 << 20) for c in tuned["nsplit"]],
                          "ms_per_mode": list(tuned["ms"])},
    }
    ctx.destroy()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_rows, 1)
        # the same oracle on one host core (a smaller row sample: about a second per 1000 rows)
        out["cpu_baseline_1core"] = cpu_baseline(n, max(64, args.cpu_rows // 16), 1, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
