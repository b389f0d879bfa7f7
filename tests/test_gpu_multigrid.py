"""Multigrid Tucker on the GPU (Sec. 3.2, last paragraph; Sec. 3.7 Fig. 7) against the oracle.

The GPU runs the HOSVD on the coarsest grid only and starts Tucker-ALS on every finer grid from
the interpolated, orthonormalised factors of the level below, as the oracle's
multigrid_compress does.  FP64 with fixed sweeps: the same iterates up to rounding, so the
error matches to the FP64 HOOI tolerance; converged: the paper's Table 4.2 through the multigrid
route; FP32 at 256^3: the error of the direct compression at the same ranks."""
import json
import os

import numpy as np
import pytest

from tests.gpu_util import require_gpu, say, sign_align

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


@pytest.mark.parametrize("n,levels,layout,ranks,sweeps", [
    ((65, 65, 65), 2, 0, (5, 5, 5), 2),
    ((64, 50, 72), 1, 1, (4, 6, 5), 1),
    ((129, 129, 129), 3, 0, (8, 8, 8), 2),
])
def test_multigrid_fp64_matches_oracle(ctx, tk, oracle, n, levels, layout, ranks, sweeps):
    kw = dict(nu=1.5, ell=0.3)
    say("multigrid fp64", n, levels, ranks, sweeps)
    og = oracle.Grid(n=n, b=(1.0, 1.0, 1.0), layout=layout)
    ref = oracle.multigrid_compress(oracle.Kernel(oracle.MATERN, **kw), og, ranks, levels, sweeps=sweeps)
    t = ctx.compress_multigrid(tk.make_kernel(0, **kw), tk.make_grid(n, 1.0, layout), levels,
                               tk.make_opts(ranks=ranks, hooi_sweeps=sweeps, prec=tk.TK_FP64))
    say("  E gpu %.10e oracle %.10e" % (t.rel_err, ref.rel_err))
    assert t.ranks == tuple(ranks)
    assert t.rel_err == pytest.approx(ref.rel_err, rel=1e-9)
    U, core = t.factors()
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, **kw), og)
    d = _recon(U, core) - oracle.reconstruct(ref.core, ref.U)
    assert np.sqrt(np.sum(d * d) / np.sum(A * A)) <= 1e-9
    t.free()


def test_multigrid_table_4_2_n257(ctx, tk):
    """Table 4.2 (Sec. 4) at n = 257 through 65 -> 129 -> 257 with converged Tucker-ALS."""
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table_4_2.json")))
    b = tab["box_half_width"]
    printed = tab["printed"]["257"]
    excluded = set(tab["excluded"].get("257", []))
    kern = tk.make_kernel(tk.TK_SLATER, alpha=1.0, p=1.0, ell=1.0)
    grid = tk.make_grid(257, b, tk.TK_CENTERED)
    for r in range(1, 11):
        t = ctx.compress_multigrid(kern, grid, 2, tk.make_opts(ranks=r, hooi_sweeps=tk.TK_HOOI_CONVERGE,
                                                               prec=tk.TK_FP64))
        err = 1.0 - ctx.trace(t) / 129 ** 3
        say("r=%d 1 - A_r(x0) = %.4g (printed %.3g)" % (r, err, printed[r - 1]))
        t.free()
        if r not in excluded:
            assert err == pytest.approx(printed[r - 1], rel=tab["rel_tol"])


@pytest.mark.parametrize("prec", ["TK_FP32", "TK_BF16X3"])
def test_multigrid_float_256_matches_direct(ctx, tk, prec):
    """256^3 (levels 128 -> 256), rank 10, two sweeps per level: the multigrid error is that of
    the direct compression at the same ranks, to the float paths' 1e-5 relative tolerance of
    the reconstruction (the two starts lead the sweeps to the same subspaces)."""
    kern = tk.make_kernel(0, nu=1.5, ell=0.2)
    grid = tk.make_grid(256, 1.0, tk.TK_OFFSET)
    opts = tk.make_opts(ranks=10, hooi_sweeps=2, prec=getattr(tk, prec))
    mg = ctx.compress_multigrid(kern, grid, 1, opts)
    d = ctx.compress(kern, grid, opts)
    say(prec, "E multigrid %.6e direct %.6e" % (mg.rel_err, d.rel_err))
    assert abs(mg.rel_err - d.rel_err) <= 1e-5 * max(d.rel_err, 1e-3) + 2e-7
    mg.free()
    d.free()


def test_multigrid_levels_too_deep(ctx, tk):
    with pytest.raises(tk.TkError) as ei:
        ctx.compress_multigrid(tk.make_kernel(0, nu=0.5, ell=0.3), tk.make_grid(16), 5, tk.make_opts(ranks=2))
    assert "TK_EINVAL" in str(ei.value)
