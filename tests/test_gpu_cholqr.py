"""The float eps path's Cholesky QR (tk_ctx_set_cholqr) through the C ABI: every register size of
the orthonormalisation kernel (p = 8, 16, 24, 32 over 256 threads, p = 24 over 512), blocks it
hands to the Householder QR (p = 32 over 512 rows, more than 512 rows), a rank-one tensor whose
trailing columns are rounding noise (the random completion), and each route (the default
thresholds, two passes always, the in-kernel Householder fallback always) against the
Householder-only route and against the FP64 oracle.  The routes agree to the float path's bar,
not bitwise: the trailing factor columns carry the FP32 rounding of the tensor, which any change
of rounding order moves."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say

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


# (kernel, shape, nu/ell, layout, eps, r_max): the working rank is r_max (default 24) per mode
# below n
CASES = [
    ("matern", (72, 72, 72), 1.5, 0.2, 1, 1e-6, 0),      # p 24, 256 threads, three modes in one launch
    ("matern", (72, 72, 72), 0.5, 0.1, 1, 1e-3, 16),     # p 16
    ("matern", (64, 64, 64), 2.5, 1.0, 1, 1e-3, 8),      # p 8
    ("matern", (300, 40, 36), 0.5, 0.3, 1, 1e-6, 32),    # p 32: Householder (mode 0), 256 threads (1, 2)
    ("matern", (300, 40, 36), 1.5, 0.3, 0, 1e-6, 24),    # p 24, 512 threads (mode 0)
    ("matern", (700, 48, 40), 1.5, 0.3, 0, 1e-6, 24),    # Householder above 512 rows (mode 0)
    ("gauss", (96, 80, 72), 0.0, 0.5, 1, 1e-6, 0),       # rank one: 23 noise columns per block
]

# (floor, one_pass, accept2): default, always two passes, always the fallback (a second pass
# that never passes), Householder only
ROUTES = {"default": (1e-12, 1e-4, 0.25), "two_pass": (1e-12, 2.0, 0.25), "fallback": (1e-12, 2.0, 2.0),
          "householder": (0.0, 1e-4, 0.25)}


@pytest.mark.parametrize("family,shape,nu,ell,layout,eps,rmax", CASES)
def test_cholqr_routes_match_householder_and_oracle(ctx, tk, oracle, family, shape, nu, ell, layout, eps, rmax):
    say("cholqr", family, shape, nu, ell, eps, rmax)
    if family == "gauss":
        kern = tk.make_kernel(tk.TK_GAUSS, ell=ell)
        ok = oracle.Kernel(oracle.GAUSS, ell=ell)
    else:
        kern = tk.make_kernel(tk.TK_MATERN, nu=nu, ell=ell)
        ok = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell)
    grid = tk.make_grid(shape, 1.0, layout)
    opts = tk.make_opts(eps=eps, r_max=rmax, hooi_sweeps=2, prec=tk.TK_FP32)
    out = {}
    try:
        for name, args in ROUTES.items():
            ctx.set_cholqr(*args)
            t = ctx.compress(kern, grid, opts)
            U, core = t.factors()
            out[name] = (t.ranks, t.rel_err, U, core)
            t.free()
            say("  %-11s ranks %s E %.4e" % (name, out[name][0], out[name][1]))
    finally:
        ctx.set_cholqr()
    og = oracle.Grid(n=shape, layout=layout)
    A = oracle.grid_eval(ok, og)
    ref = oracle.compress(ok, og, eps=eps, sweeps=2)
    nA = np.sqrt(np.sum(A * A))
    say("  oracle ranks %s E %.4e" % (ref.ranks, ref.rel_err))
    R_ref = oracle.reconstruct(ref.core, ref.U)
    R_hh = _recon(out["householder"][2], out["householder"][3])
    for name, (ranks, E, U, core) in out.items():
        assert E <= eps, (name, E)
        assert all(a <= b + 1 for a, b in zip(ranks, ref.ranks)), (name, ranks, ref.ranks)
        for k in range(3):
            Uk = U[k]
            assert np.abs(Uk.T @ Uk - np.eye(Uk.shape[1])).max() <= 1e-9, (name, k)
        R = _recon(U, core)
        # the reported error is the measured one, and the result is the oracle's within the
        # float path's bar (the same as for the Householder route)
        e_true = np.sqrt(np.sum((R - A) ** 2)) / nA
        assert e_true == pytest.approx(E, rel=2e-2, abs=2e-8), (name, e_true, E)
        assert np.sqrt(np.sum((R - R_ref) ** 2)) / nA <= 1e-5, name
        assert np.sqrt(np.sum((R - R_hh) ** 2)) / nA <= 1e-5, name


def test_cholqr_setter_rejects_nan(ctx, tk):
    nan = float("nan")
    for args in ((nan, 1e-4, 0.25), (1e-12, nan, 0.25), (1e-12, 1e-4, nan)):
        with pytest.raises(tk.TkError):
            ctx.set_cholqr(*args)
    ctx.set_cholqr()
