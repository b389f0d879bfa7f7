"""Rank caps, budget accounting and error paths of the C ABI on the GPU.

- a float-path compression whose working rank exceeds the register tiles of its kernels is
  refused (TK_EUNSUPPORTED) instead of running with columns missing; up to that cap the full
  rank r = n recovers the tensor (the exact-recovery property of the Tucker format at full
  rank, Sec. 3.1), and the FP64 path recovers it up to its own cap;
- a result of a higher third rank than the FFT matvec's register tile takes the dense form,
  checked against the oracle's plain covariance product;
- an eps miss raised as an error holds no budget afterwards;
- the device memory a context holds stays within its budget plus the stated rounding while a
  request loop of mixed sizes runs.
"""
import threading
import time

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, require_gpu, say, to_oracle_tucker, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


@pytest.fixture(scope="module")
def ctx(tk):
    require_gpu()
    c = tk.Context(0)
    yield c
    c.destroy()


def _recon(U, core):
    X = np.einsum("ia,abc->ibc", U[0], core)
    X = np.einsum("jb,ibc->ijc", U[1], X)
    return np.einsum("kc,ijc->ijk", U[2], X)


def test_float_rank_above_register_tiles_is_refused(ctx, tk):
    say("fp32 n=50 ranks=50")
    for prec in (tk.TK_FP32, tk.TK_BF16X3):
        with pytest.raises(tk.TkError) as ei:
            ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.3), tk.make_grid(50),
                         tk.make_opts(ranks=50, hooi_sweeps=1, prec=prec))
        assert "TK_EUNSUPPORTED" in str(ei.value)
    assert ctx.budget()[1] == 0


@pytest.mark.parametrize("prec,n,tol", [("TK_FP32", 48, 3e-6), ("TK_FP64", 50, 1e-13)])
def test_full_rank_recovers_the_tensor(ctx, tk, oracle, prec, n, tol):
    """r = n: the Tucker format is exact (orthonormal square factors)."""
    say("full rank", prec, n)
    kern = tk.make_kernel(0, nu=1.5, ell=0.3)
    t = ctx.compress(kern, tk.make_grid(n), tk.make_opts(ranks=n, hooi_sweeps=1, prec=getattr(tk, prec)))
    assert t.ranks == (n, n, n)
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.3), oracle.Grid(n=(n, n, n)))
    U, core = t.factors()
    d = _recon(U, core) - A
    err = np.sqrt(np.sum(d * d) / np.sum(A * A))
    say("  recon err %.3e, reported %.3e" % (err, t.rel_err))
    assert err <= tol and t.rel_err <= tol
    for k in range(3):
        assert np.abs(U[k].T @ U[k] - np.eye(n)).max() <= (1e-12 if prec == "TK_FP64" else 1e-5)
    t.free()


def test_high_rank_result_takes_the_dense_matvec(ctx, tk, oracle):
    """FP64 result of third rank 52 > 48: the FP32 matvec falls back to the dense form; sampled
    rows against the oracle's plain product with the same generator."""
    n, r = 52, 52
    say("rank-52 result, fp32 matvec")
    kern = tk.make_kernel(0, nu=0.5, ell=0.4)
    g = tk.make_grid(n, 1.0, tk.TK_OFFSET)
    t = ctx.compress(kern, g, tk.make_opts(ranks=(6, 6, r), hooi_sweeps=1, prec=tk.TK_FP64))
    assert t.ranks == (6, 6, r)
    U, core = t.factors()
    z = synth.normal_vector((n, n, n), 7)
    y = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    ctx.kron_matvec(t, dev(z, np.float32), y, io=tk.TK_FP32)
    got = host(y)
    og = oracle.Grid(n=(n, n, n), layout=oracle.OFFSET)
    rows = np.random.default_rng(3).choice(n ** 3, 300, replace=False)
    want = oracle.cov_matvec_rows(to_oracle_tucker(oracle, U, core), og, z.astype(np.float32).astype(np.float64),
                                  rows)
    Q = _recon(U, core)
    # each row within 2e-5 of sum_j |C_ij||z_j| (FP32 products, FP32 accumulation)
    absrow = oracle.cov_rows_from_generator(np.abs(Q), og, np.abs(z.astype(np.float64)), rows)
    assert np.all(np.abs(got[rows] - want) <= 2e-5 * absrow + 1e-30)
    # the quadratic form takes the same route
    qf = ctx.quadratic_form(t, dev(z, np.float32), io=tk.TK_FP32)
    assert np.isfinite(qf)
    t.free()


def test_eps_miss_holds_no_budget(ctx, tk):
    before = ctx.budget()[1]
    for _ in range(3):
        with pytest.raises(tk.TkError) as ei:
            ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.05), tk.make_grid(64), tk.make_opts(eps=1e-9, r_max=3))
        assert "TK_ENOCONV" in str(ei.value)
    assert ctx.budget()[1] == before


def test_device_memory_stays_within_budget(tk):
    """A request loop of mixed sizes under a budget that admits about one large request at a
    time: the device memory the context holds (sampled from another thread while the loop
    runs) never exceeds the budget plus the rounding of the busy workspace blocks."""
    require_gpu()
    torch.cuda.synchronize()
    budget = 1536 << 20
    zs = {n: dev(synth.normal_vector((n, n, n), n), np.float32) for n in (64, 128, 192)}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    c = tk.Context(0, hbm_budget_bytes=budget)
    sv = tk.Server(c, workers=4)
    peak = [0]
    stop = threading.Event()

    def sampler():
        while not stop.is_set():
            used = free0 - torch.cuda.mem_get_info()[0]
            peak[0] = max(peak[0], used)
            time.sleep(0.002)

    th = threading.Thread(target=sampler)
    th.start()
    try:
        rng = np.random.default_rng(5)
        tickets = []
        comp = []
        for i in range(24):
            n = int(rng.choice([64, 128, 192]))
            g = tk.make_grid(n, 1.0, tk.TK_OFFSET)
            kern = tk.make_kernel(0, nu=float(rng.choice([0.5, 1.5, 2.5])), ell=float(rng.uniform(0.1, 1.0)))
            tck = sv.submit_compress(kern, g, tk.make_opts(eps=1e-6, prec=tk.TK_FP32))
            comp.append((tck, n))
            tickets.append(tck)
            if i % 3 == 2:
                tgt, tn = comp[int(rng.integers(len(comp)))]
                tickets.append(sv.submit_quadform(tgt, zs[tn], stream=tk.STREAM_READY))
        for tck in tickets:
            r = sv.wait(tck)
            assert r["status"] in (tk.TK_OK, tk.TK_ENOMEM), r
    finally:
        stop.set()
        th.join()
        sv.destroy()
    held = free0 - torch.cuda.mem_get_info()[0]
    c.destroy()
    slack = 8 * (16 << 20) + (64 << 20)   # 16 MiB per worker stream slot, context staging, pool granularity
    say("peak held %.1f MiB, after the loop %.1f MiB, budget %.1f MiB" % (peak[0] / 2 ** 20, held / 2 ** 20,
                                                                          budget / 2 ** 20))
    assert peak[0] <= budget + slack
