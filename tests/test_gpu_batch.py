"""tk_compress_batch: problems of uneven sizes run concurrently on the context's worker
streams; every result must be identical to what tk_compress returns for the problem alone,
also when a small HBM budget makes the problems wait for admission."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


# (n, nu, ell, layout): uneven sizes, all three Matern orders, both layouts
_ITEMS = [(48, 0.5, 0.1, 1), (33, 1.5, 0.3, 0), (64, 2.5, 1.0, 1), (40, 0.5, 0.3, 1),
          (57, 1.5, 0.1, 0), (32, 2.5, 0.3, 1), (64, 0.5, 1.0, 0)]


def _problems(tk):
    ks = [tk.make_kernel(0, nu=nu, ell=ell) for (_, nu, ell, _) in _ITEMS]
    gs = [tk.make_grid(n, 1.0, lay) for (n, _, _, lay) in _ITEMS]
    return ks, gs


def _same(a, b):
    (Ua, Ca), (Ub, Cb) = a.factors(), b.factors()
    return (a.ranks == b.ranks and a.rel_err == b.rel_err and np.array_equal(Ca, Cb)
            and all(np.array_equal(x, y) for x, y in zip(Ua, Ub)))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_matches_single(tk, prec):
    require_gpu()
    ctx = tk.Context(0)
    try:
        ks, gs = _problems(tk)
        opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
        alone = [ctx.compress(k, g, opts) for k, g in zip(ks, gs)]
        for workers in (4, 2):
            ctx.set_workers(workers)
            say("batch prec", prec, "workers", workers)
            mix = ctx.compress_batch(ks, gs, opts)
            for i, (a, b) in enumerate(zip(alone, mix)):
                assert _same(a, b), f"item {i} differs in the batch"
            for t in mix:
                t.free()
        for t in alone:
            t.free()
    finally:
        ctx.destroy()


def test_batch_under_tight_budget(tk):
    """A budget that holds about one problem at a time: the others wait, nothing fails."""
    require_gpu()
    ks, gs = _problems(tk)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    big = tk.tk_estimate_bytes(gs[2], opts)
    ctx = tk.Context(0, hbm_budget_bytes=int(1.5 * big))
    try:
        alone = [ctx.compress(k, g, opts) for k, g in zip(ks, gs)]
        ref = [(t.ranks, t.rel_err, t.factors()) for t in alone]
        for t in alone:
            t.free()
        mix = ctx.compress_batch(ks, gs, opts)
        for i, (t, (r, e, (U, C))) in enumerate(zip(mix, ref)):
            Ub, Cb = t.factors()
            assert t.ranks == r and t.rel_err == e and np.array_equal(Cb, C), f"item {i}"
            assert all(np.array_equal(x, y) for x, y in zip(U, Ub)), f"item {i}"
        for t in mix:
            t.free()
    finally:
        ctx.destroy()


def test_batch_empty_and_errors(tk):
    require_gpu()
    ctx = tk.Context(0)
    try:
        assert ctx.compress_batch([], [], tk.make_opts(eps=1e-6)) == []
        ks, gs = _problems(tk)
        bad = list(ks)
        bad[3] = tk.make_kernel(0, nu=0.7, ell=0.3)        # unsupported order
        with pytest.raises(tk.TkError) as ei:
            ctx.compress_batch(bad, gs, tk.make_opts(eps=1e-6))
        assert ei.value.status == tk.TK_EUNSUPPORTED
        with pytest.raises(tk.TkError):
            ctx.set_workers(0)
    finally:
        ctx.destroy()
