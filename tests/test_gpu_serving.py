"""The request loop (tk_server_*): mixed compress / matvec / trace / quadratic-form requests
submitted at once run concurrently on the server's workers; every result must be identical to
the same request run alone through the plain entry points, also when a small HBM budget makes
requests wait for admission.  Error paths finish with a status instead of failing the loop."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


# compress requests: (n, nu, ell, layout); follow-ups: (kind, index of the compress)
_COMPRESS = [(48, 0.5, 0.1, 1), (33, 1.5, 0.3, 0), (64, 2.5, 1.0, 1), (40, 0.5, 0.3, 1), (57, 1.5, 0.1, 0),
             (64, 0.5, 1.0, 1)]
_FOLLOW = [("matvec", 0), ("trace", 1), ("quadform", 2), ("matvec", 3), ("quadform", 0), ("trace", 5),
           ("matvec", 4), ("quadform", 5), ("trace", 2)]


def _dims(tucker_or_n, layout):
    n = tucker_or_n
    return (n,) * 3 if layout == 1 else (((n + 1) // 2),) * 3


def _run_mix(tk, ctx, workers, prec):
    sv = tk.Server(ctx, workers)
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    try:
        tickets = [sv.submit_compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, lay), opts)
                   for (n, nu, ell, lay) in _COMPRESS]
        vecs, fol = [], []
        for j, (kind, ci) in enumerate(_FOLLOW):
            n, _, _, lay = _COMPRESS[ci]
            z = dev(synth.normal_vector(_dims(n, lay), 100 + j))
            y = torch.empty_like(z)
            vecs.append((z, y))
            if kind == "matvec":
                fol.append(sv.submit_matvec(tickets[ci], z, y))
            elif kind == "trace":
                fol.append(sv.submit_trace(tickets[ci]))
            else:
                fol.append(sv.submit_quadform(tickets[ci], z, y=y))
        comp = [sv.wait(t) for t in tickets]
        res = [sv.wait(t) for t in fol]
        facs = [sv.tucker(t).factors() for t in tickets]
        ys = [host(y) for (_, y) in vecs]
        return comp, res, facs, ys
    finally:
        sv.destroy()


def _run_alone(tk, ctx, prec):
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=prec)
    ts = [ctx.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, lay), opts)
          for (n, nu, ell, lay) in _COMPRESS]
    res, ys = [], []
    for j, (kind, ci) in enumerate(_FOLLOW):
        n, _, _, lay = _COMPRESS[ci]
        z = dev(synth.normal_vector(_dims(n, lay), 100 + j))
        y = torch.empty_like(z)
        if kind == "matvec":
            ctx.kron_matvec(ts[ci], z, y)
            res.append(None)
        elif kind == "trace":
            res.append(ctx.trace(ts[ci]))
        else:
            res.append(ctx.quadratic_form(ts[ci], z, y=y))
        ys.append(host(y))
    out = [(t.ranks, t.rel_err, t.factors()) for t in ts]
    for t in ts:
        t.free()
    return out, res, ys


def _check_same(tk, comp, res, facs, ys, alone):
    a_comp, a_res, a_ys = alone
    for i, (c, f, (rk, e, (U, G))) in enumerate(zip(comp, facs, a_comp)):
        assert c["status"] == tk.TK_OK, f"compress {i}"
        assert c["ranks"] == tuple(rk) and c["rel_err"] == e, f"compress {i}"
        assert np.array_equal(f[1], G) and all(np.array_equal(x, u) for x, u in zip(f[0], U)), f"compress {i}"
    for j, ((kind, _), r, y, ar, ay) in enumerate(zip(_FOLLOW, res, ys, a_res, a_ys)):
        assert r["status"] == tk.TK_OK, f"follow-up {j}"
        if kind in ("matvec", "quadform"):
            assert np.array_equal(y, ay), f"follow-up {j} ({kind}): y differs"
        if kind in ("trace", "quadform"):
            assert r["value"] == ar, f"follow-up {j} ({kind})"


@pytest.mark.parametrize("prec", [1, 0])
def test_serving_mix_equals_alone(tk, prec):
    require_gpu()
    ctx = tk.Context(0)
    try:
        alone = _run_alone(tk, ctx, prec)
        for workers in (4, 2):
            say("serving mix, prec", prec, "workers", workers)
            comp, res, facs, ys = _run_mix(tk, ctx, workers, prec)
            _check_same(tk, comp, res, facs, ys, alone)
            # timestamps are ordered per request
            for r in comp + res:
                assert r["t_submit"] <= r["t_start"] <= r["t_end"]
    finally:
        ctx.destroy()


def test_serving_tight_budget(tk):
    """A budget of about one request at a time: requests queue for admission, nothing fails."""
    require_gpu()
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    need = max(tk.tk_estimate_bytes(tk.make_grid(n, 1.0, lay), opts) for (n, _, _, lay) in _COMPRESS)
    probe = tk.Context(0)
    try:
        for (n, nu, ell, lay) in _COMPRESS:
            t = probe.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, lay), opts)
            need = max(need, tk.tk_estimate_matvec_bytes(probe.handle, t.handle))
            t.free()
    finally:
        probe.destroy()
    ctx = tk.Context(0, hbm_budget_bytes=int(1.6 * need))
    try:
        alone = _run_alone(tk, ctx, 1)
        comp, res, facs, ys = _run_mix(tk, ctx, 4, 1)
        _check_same(tk, comp, res, facs, ys, alone)
    finally:
        ctx.destroy()


def test_serving_errors(tk):
    require_gpu()
    ctx = tk.Context(0)
    sv = tk.Server(ctx, 2)
    try:
        bad = sv.submit_compress(tk.make_kernel(0, nu=0.7, ell=0.3), tk.make_grid(32, 1.0, 1), tk.make_opts(eps=1e-6))
        assert sv.wait(bad)["status"] == tk.TK_EUNSUPPORTED
        assert sv.wait(sv.submit_trace(bad))["status"] == tk.TK_EINVAL          # on a failed compress
        assert sv.wait(sv.submit_trace(12345))["status"] == tk.TK_EINVAL        # unknown target
        good = sv.submit_compress(tk.make_kernel(0, nu=1.5, ell=0.3), tk.make_grid(32, 1.0, 1), tk.make_opts(eps=1e-6))
        assert sv.wait(good)["status"] == tk.TK_OK
        assert sv.wait(sv.submit_trace(good))["status"] == tk.TK_OK
        sv.release(good)
        assert sv.wait(sv.submit_trace(good))["status"] == tk.TK_EINVAL         # released
        with pytest.raises(tk.TkError):
            sv.wait(good)                                                        # collected already
    finally:
        sv.destroy()
        ctx.destroy()
