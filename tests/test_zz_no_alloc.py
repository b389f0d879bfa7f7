"""The allocation-free covariance matvec (tk_kron_matvec_noalloc) against tk_kron_matvec.

Both run the FFT form of y = C z (Sec. 3.6 circulant embedding, Sec. 4 eq. (4.1)) with the same
kernels and launch shapes; the allocation-free one takes its workspace from the device's fixed
scratch array.  Its y must equal tk_kron_matvec's bit for bit, on two calls in a row (the second
on a smaller operator, so the scratch holds the first call's leftovers), device memory must not
change across the calls, and an operator larger than the scratch is refused before anything runs.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, require_gpu, say, torch

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


def _result(ctx, tk, n, nu, ell):
    return ctx.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, tk.TK_OFFSET),
                        tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=tk.TK_FP32))


def test_noalloc_matvec_equals_the_allocating_one(ctx, tk):
    ctx.set_matvec_method(tk.TK_MV_FFT)
    cases = [(64, 0.5, 0.3, 11), (40, 2.5, 0.6, 12)]     # second call on a smaller operator
    results = [_result(ctx, tk, n, nu, ell) for n, nu, ell, _ in cases]
    zs = [dev(synth.normal_vector((n, n, n), seed)) for n, _, _, seed in cases]
    refs = []
    for t, z in zip(results, zs):
        y = torch.empty_like(z)
        ctx.kron_matvec(t, z, y, io=tk.TK_FP32)
        refs.append(host(y))
    outs = [torch.full_like(z, float("nan")) for z in zs]
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    in_use0 = tk.tk_ctx_budget(ctx.handle)[1]
    for (n, nu, ell, _), t, z, y in zip(cases, results, zs, outs):
        say("noalloc matvec n=%d nu=%g ell=%g ranks %s" % (n, nu, ell, t.ranks))
        ctx.kron_matvec_noalloc(t, z, y)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert tk.tk_ctx_budget(ctx.handle)[1] == in_use0
    for (n, _, _, _), ref, y in zip(cases, refs, outs):
        got = host(y)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), (n, float(np.abs(got - ref).max()))
    # again in the opposite order: the larger operator after the smaller one's leftovers
    for t, z, y in reversed(list(zip(results, zs, outs))):
        y.fill_(float("nan"))
        ctx.kron_matvec_noalloc(t, z, y)
    for ref, y in zip(refs, outs):
        assert np.array_equal(host(y), ref)
    for t in results:
        t.free()
    ctx.set_matvec_method(tk.TK_MV_AUTO)


def test_noalloc_matvec_refuses_what_the_scratch_cannot_hold(ctx, tk):
    t = _result(ctx, tk, 80, 1.5, 0.5)      # 80 points per axis: circulant length 256
    z = dev(synth.normal_vector((80, 80, 80), 13))
    y = torch.zeros_like(z)
    with pytest.raises(tk.TkError) as ei:
        ctx.kron_matvec_noalloc(t, z, y)
    assert "TK_ENOMEM" in str(ei.value) and "scratch" in str(ei.value)
    assert float(host(y).max()) == 0.0 and float(host(y).min()) == 0.0
    with pytest.raises(tk.TkError) as ei:
        ctx.kron_matvec_noalloc(t, z, z)
    assert "TK_EINVAL" in str(ei.value)
    t.free()
