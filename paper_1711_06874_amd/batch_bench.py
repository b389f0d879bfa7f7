"""Uneven batch workload: 256 independent Matern tensors of different sizes compressed to
eps = 1e-6, as one batch call and as 256 sequential single calls, one JSON line per form.

    python -m paper_1711_06874_amd.batch_bench [--count 256] [--workers 4 8] [--prec fp32]
                                               [--no-seq] [--profile] [--autotune] [--graphs]

Per tensor (seeded, in order): n uniform over {32, 48, 64, 96, 128, 192, 256}, nu uniform over
{1/2, 3/2, 5/2}, ell log-uniform on [0.05, 1], sigma2 = 1, centred grid on [-1, 1]^3; HOSVD,
2 HOOI sweeps, eps truncation.  Reported: wall time of the whole batch (results complete),
tensors/s, input elements/s, p50/p99 of the single-call latency per size, the algorithmic
bound of the batch (HBM bytes and Gram FLOPs of the method at FP32), and with --profile the
summed kernel time per class.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_GBS = 8000.0
FP32_TFS = 157.3


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def algorithmic_bound(sizes, sweeps=2):
    """Per tensor at FP32: grid write 4n^3, Gram reads 3*4n^3, 2 A-streaming TTMs per HOOI sweep
    (2*4n^3 each sweep), error norm 4n^3 bytes; symmetric Gram n^3(n+1) FLOPs per mode."""
    byts = sum((4 + 12 + 8 * sweeps + 4) * n ** 3 for n in sizes)
    flops = sum(3 * n ** 3 * (n + 1) for n in sizes)
    return byts, flops, 1e3 * (byts / (HBM_GBS * 1e9) + flops / (FP32_TFS * 1e12))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--workers", type=int, nargs="+", default=[4, 8])
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--reps", type=int, default=3, help="timed batch calls per worker count")
    ap.add_argument("--no-seq", action="store_true", help="skip the 256 sequential calls")
    ap.add_argument("--profile", action="store_true", help="per-class kernel times of one batch call")
    ap.add_argument("--autotune", action="store_true", help="tune the Gram kernel and split of every size first")
    ap.add_argument("--graphs", action="store_true", help="replay the captured compression pipeline of every "
                    "shape (tk_ctx_set_graphs)")
    ap.add_argument("--qr", choices=["cholesky", "householder"], default="cholesky",
                    help="orthonormalisation of the span-only steps (tk_ctx_set_cholqr)")
    args = ap.parse_args()

    import torch
    import synth
    from paper_1711_06874_amd import tk

    torch.cuda.set_device(0)
    items = synth.uneven_batch(args.count)
    prec = tk.TK_FP32 if args.prec == "fp32" else tk.TK_BF16X3
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    kernels = [tk.make_kernel(tk.TK_MATERN, nu=k.nu, ell=k.ell) for k, _ in items]
    grids = [tk.make_grid(g.n, g.b, g.layout) for _, g in items]
    sizes = [g.n[0] for _, g in items]
    byts, flops, bound_ms = algorithmic_bound(sizes)
    elems = sum(n ** 3 for n in sizes)
    common = {"count": args.count, "precision": args.prec, "eps": 1e-6, "hooi_sweeps": 2,
              "input_elements": elems, "algorithmic_GB": byts / 1e9, "gram_TFLOP": flops / 1e12,
              "bound_ms": bound_ms,
              "workload": "256 Matern tensors, n uniform over {32,...,256}, centred grids, eps 1e-6"}
    ctx = tk.Context(0)
    common["graphs"] = bool(args.graphs)
    common["qr"] = args.qr
    try:
        if args.graphs:
            ctx.set_graphs(True)
        if args.qr == "householder":
            ctx.set_cholqr(0.0)
        if args.autotune:
            common["gram_autotune"] = {str(n): ctx.autotune(tk.make_grid(n, 1.0, 0), prec)["nsplit"]
                                       for n in sorted(set(sizes))}
        # warm-up: one batch call (kernels loaded, workspaces pooled)
        for t in ctx.compress_batch(kernels, grids, opts):
            t.free()
        torch.cuda.synchronize()
        print("warm-up batch done", file=sys.stderr, flush=True)

        if not args.no_seq:
            lat = {}
            ranks, errs = [], []
            t0 = time.perf_counter()
            for k, g, n in zip(kernels, grids, sizes):
                a = time.perf_counter()
                t = ctx.compress(k, g, opts)
                lat.setdefault(n, []).append((time.perf_counter() - a) * 1e3)
                ranks.append(t.ranks)
                errs.append(t.rel_err)
                t.free()
            wall = time.perf_counter() - t0
            out = dict(common, form="sequential", workers=1, wall_ms=wall * 1e3,
                       tensors_per_s=args.count / wall, elements_per_s=elems / wall,
                       frac_of_bound=bound_ms / (wall * 1e3), eps_met=sum(e <= 1e-6 for e in errs),
                       max_rank=max(max(r) for r in ranks),
                       latency_ms_by_n={str(n): {"count": len(v), "p50": pct(v, 50), "p99": pct(v, 99)}
                                        for n, v in sorted(lat.items())})
            print(json.dumps(out), flush=True)

        for w in args.workers:
            ctx.set_workers(w)
            walls = []
            for rep in range(args.reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.compress_batch(kernels, grids, opts)
                wall = time.perf_counter() - t0
                walls.append(wall)
                errs = [t.rel_err for t in res]
                ranks = [t.ranks for t in res]
                for t in res:
                    t.free()
            wall = min(walls)
            out = dict(common, form="batch", workers=w, wall_ms=wall * 1e3, wall_ms_all=[x * 1e3 for x in walls],
                       tensors_per_s=args.count / wall, elements_per_s=elems / wall,
                       frac_of_bound=bound_ms / (wall * 1e3), eps_met=sum(e <= 1e-6 for e in errs),
                       max_rank=max(max(r) for r in ranks))
            if args.profile:
                tk.tk_profile_reset()
                tk.tk_profile_enable(True)
                for t in ctx.compress_batch(kernels, grids, opts):
                    t.free()
                tk.tk_profile_enable(False)
                prof = {}
                for name, cls in tk.PROF_CLASSES.items():
                    cnt, ms = tk.tk_profile_read(cls)
                    if cnt:
                        prof[name] = {"launches": cnt, "ms": ms}
                out["kernel_ms_by_class"] = prof
            print(json.dumps(out), flush=True)
    finally:
        ctx.destroy()


if __name__ == "__main__":
    main()
