"""Small fixed workloads for hardware-counter runs (rocprofv3 --pmc), one per subcommand:

    python -m paper_1711_06874_amd.profile_driver copy --bytes 1073741824
        five plain device-to-device copies of that many bytes (the scale of FETCH_SIZE and
        WRITE_SIZE per byte moved)
    python -m paper_1711_06874_amd.profile_driver fill --bytes 67108864
        plain fills of a float buffer of that many bytes (the write-only rate of the device)
    python -m paper_1711_06874_amd.profile_driver gram --n 512 --prec fp32
        the three mode Grams (tk_gram) of the Matern 3/2 (ell = 0.2) tensor on the centred n^3
        grid, --reps times each
    python -m paper_1711_06874_amd.profile_driver grid --n 256
        FP32 grid evaluation of the 256^3 offset Matern grid (tk_grid_eval), --reps times
    python -m paper_1711_06874_amd.profile_driver compress --n 256 --prec fp32
        single compressions (tk_compress, Matern 3/2, ell = 0.3, eps 1e-6, two sweeps) of the
        offset n^3 grid, --reps times, each timed on the host

Every kernel runs in the library; the driver only allocates device memory and prints one line
per step.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["copy", "fill", "gram", "grid", "compress"])
    ap.add_argument("--bytes", type=int, default=1 << 30)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16x3"], default="fp32")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)

    import torch
    from paper_1711_06874_amd import tk
    torch.cuda.set_device(0)
    if args.what == "copy":
        x = torch.ones(args.bytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.reps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.bytes, "reps": args.reps}), flush=True)
        return 0
    if args.what == "fill":
        x = torch.empty(args.bytes // 4, dtype=torch.float32, device="cuda")
        for i in range(args.reps):
            x.fill_(float(i))
        torch.cuda.synchronize()
        print(json.dumps({"fill_bytes": args.bytes, "reps": args.reps}), flush=True)
        return 0
    prec = {"fp64": tk.TK_FP64, "fp32": tk.TK_FP32, "bf16x3": tk.TK_BF16X3}[args.prec]
    ctx = tk.Context(0)
    n = args.n
    if args.what == "compress":
        kern = tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.3)
        grid = tk.make_grid(n, 1.0, tk.TK_OFFSET)
        opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
        ms = []
        for _ in range(args.reps):
            t0 = time.perf_counter()
            t = ctx.compress(kern, grid, opts)
            ms.append((time.perf_counter() - t0) * 1e3)
            t.free()
        ms.sort()
        print(json.dumps({"compress": n, "prec": args.prec, "reps": args.reps, "ms_p50": ms[len(ms) // 2],
                          "ms_min": ms[0]}), flush=True)
        ctx.destroy()
        return 0
    if args.what == "grid":
        kern = tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.3)
        grid = tk.make_grid(n, 1.0, tk.TK_OFFSET)
        A = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        for _ in range(args.reps):
            tk.tk_grid_eval(ctx.handle, kern, grid, tk.TK_FP32, A)
        torch.cuda.synchronize()
        print(json.dumps({"grid_eval": n, "reps": args.reps, "s": time.perf_counter() - t0}), flush=True)
        ctx.destroy()
        return 0
    # gram: the tensor in the storage type of the precision (float for FP32 and BF16x3)
    kern = tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.2)
    grid = tk.make_grid(n, 1.0, tk.TK_CENTERED)
    store = tk.TK_FP64 if prec == tk.TK_FP64 else tk.TK_FP32
    A = torch.empty((n, n, n), dtype=torch.float64 if store == tk.TK_FP64 else torch.float32, device="cuda")
    tk.tk_grid_eval(ctx.handle, kern, grid, store, A)
    G = torch.empty((n, n), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for mode in range(3):
        t0 = time.perf_counter()
        for _ in range(args.reps):
            tk.tk_gram(ctx.handle, A, (n, n, n), mode, prec, G)
        torch.cuda.synchronize()
        print(json.dumps({"gram_mode": mode, "n": n, "prec": args.prec, "reps": args.reps,
                          "s": time.perf_counter() - t0}), flush=True)
    ctx.destroy()
    return 0


if __name__ == "__main__":
    sys.exit(main())
