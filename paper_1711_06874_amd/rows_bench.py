"""Timings of the widened rows on one GPU, each against the bound that its dominant work sets.

  python -m paper_1711_06874_amd.rows_bench [--only multigrid,families,sinc,kron1] [--reps 5]

Rows (one JSON line each, medians over --reps synchronised calls after one warm-up call):
- multigrid: Tucker of the Slater p = 1 covariance (Fig. 7) on the centred 1024^3 grid (the
  largest the library takes), three coarser levels (128, 256, 512), fixed ranks 16, two ALS sweeps per level, FP32 storage,
  against the direct compression of the same grid.  Bound: the finest level's HBM traffic (grid
  write, two A-streaming TTMs per sweep, the error norm: 4 n^3 bytes each) at 8 TB/s.
- families: FP32 grid evaluation of the closed-form Matern 3/2, a general-order Matern (nu = 0.3,
  K_nu by series and continued fraction in FP64), the spectral density and an anisotropic
  Matern at 256^3, in values per second and GB/s written.
- sinc: canonical-to-Tucker of the sinc-quadrature canonical tensor (M = 64, rank 129) at
  n = 256 and 1024 per axis, ranks 16, two ALS sweeps; the n^3 tensor is never formed.
- kron1: the separable covariance at the size of the example of Sec. 4 (n = 6000 per axis):
  forming the three 1-D factors and their Cholesky factors (n^3 / 3 flops each, FP64 MFMA
  bound), and the log-likelihood of a 512^3 vector (three dense mode products with the factor
  inverses, 2 n^4 flops each).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_GBS = 8000.0
FP64_MFMA_TFS = 78.6


def _timed(fn, reps):
    import torch
    fn()                      # warm-up (workspaces, tables)
    torch.cuda.synchronize()
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), ts, out


def row_multigrid(tk, ctx, reps):
    n, levels, r = 1024, 3, 16
    kern = tk.make_kernel(tk.TK_SLATER, alpha=1.0, p=1.0, ell=1.0)
    grid = tk.make_grid(n, 1.0, tk.TK_CENTERED)
    opts = tk.make_opts(ranks=r, hooi_sweeps=2, prec=tk.TK_FP32)
    held = []

    def mg():
        t = ctx.compress_multigrid(kern, grid, levels, opts)
        held.append(t)
        return t

    def direct():
        t = ctx.compress(kern, grid, opts)
        held.append(t)
        return t

    ms_mg, ts_mg, t_mg = _timed(mg, reps)
    e_mg = t_mg.rel_err
    for t in held:
        t.free()
    held.clear()
    ms_d, ts_d, t_d = _timed(direct, reps)
    e_d = t_d.rel_err
    for t in held:
        t.free()
    bytes_fine = 4.0 * n ** 3 * (1 + 2 * 2 + 1)
    return {"row": "multigrid", "n": n, "levels": levels, "ranks": r, "sweeps": 2, "prec": "fp32",
            "kernel": "slater p=1 ell=1", "ms": ms_mg, "ms_all": ts_mg, "rel_err": e_mg,
            "direct_ms": ms_d, "direct_rel_err": e_d, "speedup_vs_direct": ms_d / ms_mg,
            "bound_ms": bytes_fine / (HBM_GBS * 1e9) * 1e3,
            "frac_of_bound": bytes_fine / (HBM_GBS * 1e9) * 1e3 / ms_mg}


def row_families(tk, ctx, reps):
    import torch
    n = 256
    grid = tk.make_grid(n, 1.0, tk.TK_OFFSET)
    out = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    cases = [("matern15", tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.3)),
             ("matern_nu03", tk.make_kernel(tk.TK_MATERN, nu=0.3, ell=0.2)),
             ("spectral_nu04_a01", tk.make_kernel(tk.TK_SPECTRAL, nu=0.4, alpha=0.1)),
             ("matern15_aniso", tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.3, metric=(4.0, 1.0, 0.25)))]
    res = []
    for name, kern in cases:
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tk.tk_grid_eval(ctx.handle, kern, grid, tk.TK_FP32, out)
        torch.cuda.synchronize()
        inner = 20
        ts = []
        for _ in range(reps):
            start.record()
            for _ in range(inner):
                tk.tk_grid_eval(ctx.handle, kern, grid, tk.TK_FP32, out)
            end.record()
            end.synchronize()
            ts.append(start.elapsed_time(end) / inner)
        ms = float(np.median(ts))
        res.append({"kernel": name, "us": ms * 1e3, "gvalues_per_s": n ** 3 / ms / 1e6,
                    "GBs_written": 4.0 * n ** 3 / ms / 1e6,
                    "frac_hbm": 4.0 * n ** 3 / ms / 1e6 / HBM_GBS})
    return {"row": "families", "n": n, "prec": "fp32", "cases": res}


def row_sinc(tk, ctx, reps):
    res = []
    for n in (256, 1024):
        kern = tk.make_kernel(tk.TK_MATERN, nu=0.5, ell=0.3)
        grid = tk.make_grid(n, 1.0, tk.TK_CENTERED)
        held = []

        def run():
            t = ctx.compress_sinc(kern, grid, 64, 1.0, (16, 16, 16), 2)
            held.append(t)
            return t

        ms, ts, t = _timed(run, reps)
        e = t.rel_err
        for x in held:
            x.free()
        res.append({"n": n, "M": 64, "cp_rank": 129, "ranks": 16, "sweeps": 2, "ms": ms, "ms_all": ts,
                    "rel_err_vs_cp": e})
    return {"row": "sinc", "kernel": "matern nu=1/2 ell=0.3", "cases": res}


def row_kron1(tk, ctx, reps):
    import torch
    out = {"row": "kron1"}
    n = 6000
    kern = tk.make_kernel(tk.TK_GAUSS, ell=0.3)
    grid = tk.make_grid(n, 1.0)
    held = []

    def create():
        k = tk.Kron1(ctx, [kern] * 3, grid, (1e-4, 1e-4, 1e-4))
        held.append(k)
        return k

    ms, ts, k = _timed(create, reps)
    ld, per = k.logdet()
    for x in held:
        x.free()
    flops = 3 * n ** 3 / 3.0
    out["create_n6000"] = {"ms": ms, "ms_all": ts, "logdet": ld, "cholesky_flops": flops,
                           "TFs_if_all_cholesky": flops / ms / 1e9,
                           "frac_fp64_mfma": flops / ms / 1e9 / FP64_MFMA_TFS}
    n2 = 512
    kern2 = tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.3)
    k2 = tk.Kron1(ctx, [kern2] * 3, tk.make_grid(n2, 1.0), (1e-2, 1e-2, 1e-2))
    z32 = torch.empty((n2, n2, n2), dtype=torch.float32, device="cuda")
    tk.tk_normal_fill(ctx.handle, 1711, 1, z32)
    z = z32.double()
    del z32
    k2.loglik(z)                 # factor inverses formed once
    torch.cuda.synchronize()
    ms2, ts2, val = _timed(lambda: k2.loglik(z), reps)
    flops2 = 3 * 2.0 * n2 ** 4
    out["loglik_n512"] = {"ms": ms2, "ms_all": ts2, "loglik": val[0], "flops": flops2,
                          "TFs": flops2 / ms2 / 1e9, "frac_fp64_mfma": flops2 / ms2 / 1e9 / FP64_MFMA_TFS}
    k2.free()
    return out


ROWS = {"multigrid": row_multigrid, "families": row_families, "sinc": row_sinc, "kron1": row_kron1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=",".join(ROWS))
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch
    from paper_1711_06874_amd import tk
    if not torch.cuda.is_available():
        raise SystemExit("rows_bench needs a GPU")
    ctx = tk.Context(0)
    for name in a.only.split(","):
        print("row %s ..." % name, file=sys.stderr, flush=True)
        print(json.dumps(ROWS[name](tk, ctx, a.reps)), flush=True)
    ctx.destroy()


if __name__ == "__main__":
    main()
