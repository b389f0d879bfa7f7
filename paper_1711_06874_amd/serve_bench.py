"""Serving workload: a Poisson stream of mixed requests replayed in real time against the
request loop (tk_server_*), one JSON line per arrival rate.

    python -m paper_1711_06874_amd.serve_bench [--rates 50 200 500] [--count 300]
                                              [--workers 4] [--budget-gib 64]

70% compress requests (Matern nu in {1/2, 3/2, 5/2}, ell log-uniform on [0.05, 1], eps 1e-6,
FP32, offset grid n in {64, 128, 256, 384}), 30% follow-ups split evenly among the covariance
matvec, the trace and the quadratic form on an earlier compress (seeded N(0,1) vectors drawn on
the device).  Admission is capped by the HBM budget.  Reported per request type: p50 / p99 of
the latency (finish - arrival, queueing included) and of the service time (finish - start),
and the throughput over the whole stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def run_rate(tk, ctx, rate, count, workers, prec):
    import torch
    import synth
    reqs = synth.serving_stream(rate, count)
    sv = tk.Server(ctx, workers)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    tickets = {}          # rid -> ticket
    sizes = {}            # compress rid -> n
    keep = {}             # ticket -> device vectors kept alive until the request finished
    order = []            # (ticket, kind, rid)
    results = {}
    lock = threading.Lock()
    submitted = threading.Semaphore(0)

    def collector():
        for _ in range(len(reqs)):
            submitted.acquire()
            with lock:
                t, kind, rid = order[len(results)]
            r = sv.wait(t)
            with lock:
                results[t] = (kind, rid, r)
                keep.pop(t, None)

    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    try:
        for q in reqs:
            now = time.perf_counter() - t0
            if q.t_arrive > now:
                time.sleep(q.t_arrive - now)
            if q.kind == "compress":
                k = tk.make_kernel(q.kernel.family, nu=q.kernel.nu, ell=q.kernel.ell)
                g = tk.make_grid(q.grid.n, q.grid.b, q.grid.layout)
                t = sv.submit_compress(k, g, opts)
                sizes[q.rid] = q.grid.n[0]
            else:
                target = tickets[q.target]
                n = sizes[q.target]
                if q.kind == "trace":
                    t = sv.submit_trace(target)
                else:
                    z = synth.normal_vector_device((n, n, n), q.rid)
                    y = torch.empty_like(z)
                    t = (sv.submit_matvec(target, z, y) if q.kind == "matvec"
                         else sv.submit_quadform(target, z, y=y))
                    with lock:
                        keep[t] = (z, y)
            tickets[q.rid] = t
            with lock:
                order.append((t, q.kind, q.rid))
            submitted.release()
        th.join()
    finally:
        sv.destroy()
    by = {}
    t_first, t_last, failures, eps_miss = None, None, [], 0
    for t, (kind, rid, r) in results.items():
        if r["status"] != tk.TK_OK:
            failures.append({"rid": rid, "kind": kind, "status": r["status"], "error": r["error"]})
            continue
        if kind == "compress" and r["rel_err"] > 1e-6:
            eps_miss += 1
        d = by.setdefault(kind, {"latency": [], "service": []})
        d["latency"].append((r["t_end"] - r["t_submit"]) * 1e3)
        d["service"].append((r["t_end"] - r["t_start"]) * 1e3)
        t_first = r["t_submit"] if t_first is None else min(t_first, r["t_submit"])
        t_last = r["t_end"] if t_last is None else max(t_last, r["t_end"])
    done = sum(len(d["latency"]) for d in by.values())
    span = (t_last - t_first) if done else 0.0
    return {
        "rate_req_s": rate, "requests": len(reqs), "completed": done, "failed": len(failures),
        "failures": failures,
        "compress_eps_missed": eps_miss,
        "throughput_req_s": done / span if span > 0 else None,
        "per_type": {k: {"count": len(d["latency"]),
                         "latency_ms": {"p50": pct(d["latency"], 50), "p99": pct(d["latency"], 99)},
                         "service_ms": {"p50": pct(d["service"], 50), "p99": pct(d["service"], 99)}}
                     for k, d in sorted(by.items())},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", type=float, nargs="+", default=[50.0, 200.0, 500.0])
    ap.add_argument("--count", type=int, default=300)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    args = ap.parse_args()
    import torch
    from paper_1711_06874_amd import tk
    torch.cuda.set_device(0)
    ctx = tk.Context(0, hbm_budget_bytes=int(args.budget_gib * (1 << 30)))
    prec = tk.TK_FP32 if args.prec == "fp32" else tk.TK_BF16X3
    try:
        for rate in args.rates:
            out = run_rate(tk, ctx, rate, args.count, args.workers, prec)
            out.update({"workers": args.workers, "budget_gib": args.budget_gib, "precision": args.prec,
                        "workload": "Poisson stream: 70% compress (Matern, offset grid n in {64,128,256,384}, "
                                    "eps 1e-6), 30% matvec / trace / quadratic form on earlier results"})
            print(json.dumps(out), flush=True)
    finally:
        ctx.destroy()


if __name__ == "__main__":
    main()
