"""Serving workload: a Poisson stream of mixed requests replayed in real time against the
request loop (tk_server_*), one JSON line per arrival rate.

    python -m paper_1711_06874_amd.serve_bench [--rates 10 20 50 100 200 500] [--count 2000]
                                              [--workers 4] [--budget-gib 64]

70% compress requests (Matern nu in {1/2, 3/2, 5/2}, ell log-uniform on [0.05, 1], eps 1e-6,
FP32, offset grid n in {64, 128, 256, 384}), 30% follow-ups split evenly among the covariance
matvec, the trace and the quadratic form on an earlier compress (seeded N(0,1) vectors drawn on
the device before the replay).  Admission is capped by the HBM budget.  Reported per request type: p50 / p99 of
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


ZPOOL = 4   # distinct seeded input vectors per grid size
YPOOL = 12  # matvec outputs per grid size allocated before the replay


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def run_rate(tk, ctx, rate, count, workers, prec, trace=None, batching=32):
    import torch
    import synth
    reqs = synth.serving_stream(rate, count)
    sv = tk.Server(ctx, workers)
    sv.set_batching(batching)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    tickets = {}          # rid -> ticket
    sizes = {}            # compress rid -> n
    keep = {}             # ticket -> output vector in use until the request finished
    spare = {}            # n -> free output vectors (reused, not reallocated per request)
    # seeded N(0,1) inputs, drawn before the replay (ZPOOL per size, read-only, shared by the
    # requests), so the client does no device work while the server is measured
    zpool = {}
    for n in synth.STREAM_SIZES:
        zpool[n] = []
        for j in range(ZPOOL):
            z = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
            tk.tk_normal_fill(ctx.handle, synth.MASTER_SEED, 1_000_000 * n + j, z)
            zpool[n].append(z)
    # matvec outputs, allocated before the replay as well (more only if all are in use)
    for n in synth.STREAM_SIZES:
        spare[n] = [torch.empty((n, n, n), dtype=torch.float32, device="cuda") for _ in range(YPOOL)]
    extra = [0]
    torch.cuda.synchronize()
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
                y = keep.pop(t, None)
                if y is not None:
                    spare.setdefault(y.shape[0], []).append(y)
                if len(results) % 250 == 0:
                    print("rate %g: %d of %d finished" % (rate, len(results), len(reqs)), file=sys.stderr, flush=True)

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
                elif q.kind == "quadform":
                    t = sv.submit_quadform(target, zpool[n][q.rid % ZPOOL], stream=tk.STREAM_READY)
                else:
                    with lock:
                        free = spare.get(n)
                        y = free.pop() if free else None
                    if y is None:
                        extra[0] += 1
                        y = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
                    t = sv.submit_matvec(target, zpool[n][q.rid % ZPOOL], y, stream=tk.STREAM_READY)
                    with lock:
                        keep[t] = y
            tickets[q.rid] = t
            with lock:
                order.append((t, q.kind, q.rid))
            submitted.release()
        th.join()
    finally:
        sv.destroy()
    if trace:
        n_of = {rid: n for rid, n in sizes.items()}
        with open(trace, "a") as f:
            for t, (kind, rid, r) in sorted(results.items(), key=lambda kv: kv[1][2]["t_submit"]):
                q = reqs[rid]
                n = n_of.get(rid if kind == "compress" else q.target, 0)
                f.write("%g,%d,%s,%d,%.6f,%.6f,%.6f,%d\n" % (rate, rid, kind, n, r["t_submit"], r["t_start"],
                                                             r["t_end"], r["status"]))
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
        "outputs_allocated_during_replay": extra[0],
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
    ap.add_argument("--rates", type=float, nargs="+", default=[10.0, 20.0, 50.0, 100.0, 200.0, 500.0])
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--batching", type=int, default=32, help="compress requests one pass may take (1: off)")
    ap.add_argument("--trace", default=None, help="append one CSV row per request: rate, id, kind, n, "
                                                  "t_submit, t_start, t_end, status")
    args = ap.parse_args()
    import torch
    from paper_1711_06874_amd import tk
    torch.cuda.set_device(0)
    ctx = tk.Context(0, hbm_budget_bytes=int(args.budget_gib * (1 << 30)))
    prec = tk.TK_FP32 if args.prec == "fp32" else tk.TK_BF16X3
    try:
        for rate in args.rates:
            out = run_rate(tk, ctx, rate, args.count, args.workers, prec, args.trace, args.batching)
            out.update({"workers": args.workers, "budget_gib": args.budget_gib, "precision": args.prec,
                        "batching": args.batching,
                        "workload": "Poisson stream: 70% compress (Matern, offset grid n in {64,128,256,384}, "
                                    "eps 1e-6), 30% matvec / trace / quadratic form on earlier results"})
            print(json.dumps(out), flush=True)
    finally:
        ctx.destroy()


if __name__ == "__main__":
    main()
