"""Per-kernel parity of the HIP path against the FP64 oracle (grid, Gram, eigensolver).

Called through the C ABI.  Sizes span several 64-wide tiles with ragged tails."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_1711_06874_amd import tk
    c = tk.Context(0)
    yield c
    c.destroy()


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


KERNELS = [
    ("matern05", dict(family=0, nu=0.5, ell=0.3)),
    ("matern15", dict(family=0, nu=1.5, ell=0.1, sigma2=2.0)),
    ("matern25", dict(family=0, nu=2.5, ell=1.0)),
    ("slater_p1", dict(family=1, alpha=1.0, p=1.0, ell=0.3)),
    ("slater_p19", dict(family=1, alpha=0.7, p=1.9, ell=0.5)),
    ("gauss", dict(family=2, ell=0.6)),
    # short lengths: values down through the float subnormals to zero (s up to ~150 and ~370)
    ("matern05_short", dict(family=0, nu=0.5, ell=0.012)),
    ("slater_short", dict(family=1, alpha=2.0, p=1.0, ell=0.01)),
]


@pytest.mark.parametrize("name,kw", KERNELS)
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n,b", [((37, 70, 67), (1.0, 0.8, 1.3)),     # every row evaluated
                                 ((66, 66, 45), (0.9, 0.9, 1.2))])    # rows (i0,i1), (i1,i0) shared
def test_grid_eval(ctx, tk, oracle, name, kw, layout, n, b):
    say("grid_eval", name, layout, n)
    A = oracle.grid_eval(oracle.Kernel(**kw), oracle.Grid(n=n, b=b, layout=layout))
    k = tk.make_kernel(**kw)
    g = tk.make_grid(n, b, layout)
    d64 = torch.empty(n, dtype=torch.float64, device="cuda")
    tk.tk_grid_eval(ctx.handle, k, g, tk.TK_FP64, d64)
    got = host(d64)
    # e^{-s} turns an absolute error in s into the same relative error.  Coordinates, radius,
    # 1/ell and the products each round (fused or not) on either side, up to a few u s, so
    # the bound adds 8 u s to the exponential's own error (s = -ln(A / sigma2)).
    sigma2 = kw.get("sigma2", 1.0)
    s_exp = -np.log(np.maximum(np.abs(A) / sigma2, 1e-300))
    rtol = 2e-14 + 8 * 2.220446049250313e-16 * s_exp
    assert np.all(np.abs(got - A) <= rtol * np.abs(A) + 1e-300)
    _check_f32(ctx, tk, k, g, n, A)


def _check_f32(ctx, tk, k, g, n, A):
    """Float storage against the oracle rounded to float.  The closed forms take exp(-s) as
    2^k 2^f with 2^f (in [0.70, 1.42]) from the hardware FP32 exp2 of f: its 1 ulp is at most
    2^-23 relative; rounding f (|f| <= 1/2) to float moves 2^f by at most ln2 2^-26 relative; the
    final rounding to float adds at most 2^-24 relative.  So the value is within 3.2 * 2^-24 of the
    exact one, and the oracle rounded to float within 2^-24.  Bound: 4.25 * 2^-24 |A|, plus two
    subnormal spacings where the values leave the normal range."""
    d32 = torch.empty(n, dtype=torch.float32, device="cuda")
    tk.tk_grid_eval(ctx.handle, k, g, tk.TK_FP32, d32)
    g32 = host(d32).astype(np.float64)
    ref32 = A.astype(np.float32).astype(np.float64)
    err = np.abs(g32 - ref32)
    bound = 4.25 * 2.0 ** -24 * np.abs(ref32) + 2.0 ** -148
    say("  FP32 max err / bound %.3f, %.4f of the values equal" % (float(np.max(err / bound)), float(np.mean(err == 0))))
    assert np.all(err <= bound)


FAMILIES = [
    # Matern orders without a closed form (Temme's series below argument 2, Steed's fraction
    # above, upward recurrence); arguments from 0 to ~120
    ("matern_nu03", dict(family=0, nu=0.3, ell=0.2)),
    ("matern_nu075_short", dict(family=0, nu=0.75, ell=0.02)),
    ("matern_nu12", dict(family=0, nu=1.2, ell=0.35, sigma2=1.3)),
    ("matern_nu37", dict(family=0, nu=3.7, ell=0.5)),
    ("matern_nu11", dict(family=0, nu=11.0, ell=0.9)),
    # the Matern spectral density of Sec. 3.7 (Fig. 8: nu = 0.4, alpha = 0.1 and 100)
    ("spectral_a01", dict(family=3, nu=0.4, alpha=0.1)),
    ("spectral_a100", dict(family=3, nu=0.4, alpha=100.0)),
    ("spectral_nu15", dict(family=3, nu=1.5, alpha=2.0, sigma2=3.0)),
    # anisotropic diagonal metric (Sec. 2.2)
    ("matern15_aniso", dict(family=0, nu=1.5, ell=0.3, metric=(4.0, 1.0, 0.25))),
    ("slater_aniso", dict(family=1, alpha=0.7, p=1.9, ell=0.5, metric=(0.5, 2.0, 1.0))),
    ("matern_nu12_aniso", dict(family=0, nu=1.2, ell=0.3, metric=(1.0, 3.0, 0.7))),
]


@pytest.mark.parametrize("name,kw", FAMILIES)
@pytest.mark.parametrize("layout", [0, 1])
def test_grid_eval_families(ctx, tk, oracle, name, kw, layout):
    """General Matern orders, the spectral density and the anisotropic metric against the
    oracle (which takes K_nu from its integral representation, a different algorithm).  FP64:
    both sides evaluate exp(log constant + nu log s) K_nu(s) or (alpha^2 + rho^2)^-(nu+3/2)
    through exponents of size up to ~200, each rounded once: 2e-13, plus the 8 u s of the
    radius rounding as in test_grid_eval.  FP32 as in _check_f32."""
    n = (37, 70, 67)
    b = (1.0, 0.8, 1.3)
    say("grid_eval family", name, layout, n)
    okw = dict(kw)
    if "metric" in okw:
        okw["metric"] = tuple(okw["metric"])
    A = oracle.grid_eval(oracle.Kernel(**okw), oracle.Grid(n=n, b=b, layout=layout))
    k = tk.make_kernel(**kw)
    g = tk.make_grid(n, b, layout)
    d64 = torch.empty(n, dtype=torch.float64, device="cuda")
    tk.tk_grid_eval(ctx.handle, k, g, tk.TK_FP64, d64)
    got = host(d64)
    sigma2 = kw.get("sigma2", 1.0)
    s_exp = np.abs(np.log(np.maximum(np.abs(A) / sigma2, 1e-300)))
    rtol = 2e-13 + 8 * 2.220446049250313e-16 * s_exp
    err = np.abs(got - A) / np.maximum(np.abs(A), 1e-300)
    say("  max rel err / tol %.3e" % np.max(err / rtol))
    assert np.all(np.abs(got - A) <= rtol * np.abs(A) + 1e-300)
    _check_f32(ctx, tk, k, g, n, A)


# Grids of one spacing h with first nodes in (h/2) Z: the Matern orders above without a closed
# form take the radial-table route (one evaluation per squared radius, all parities of the
# index compression: all even, all odd, mixed); the other families and the anisotropic metric
# still take the direct route.
RADIAL_GRIDS = [
    ((40, 40, 40), (1.0, 1.0, 1.0), 1),          # offset: 2 x0 / h = 0 on every axis
    ((40, 40, 40), (1.0, 1.0, 1.0), 0),          # centred, n even: odd c_k
    ((33, 17, 25), (1.0, 0.5, 0.75), 0),         # centred, n odd, h = 1/16 on every axis
    ((33, 18, 25), (1.0, 0.53125, 0.75), 0),     # centred, mixed parities
]


@pytest.mark.parametrize("name,kw", FAMILIES)
@pytest.mark.parametrize("n,b,layout", RADIAL_GRIDS)
def test_grid_eval_families_radial(ctx, tk, oracle, name, kw, n, b, layout):
    """The radial-table route against the oracle (same bounds as test_grid_eval_families)."""
    say("grid_eval radial", name, n, b, layout)
    okw = dict(kw)
    if "metric" in okw:
        okw["metric"] = tuple(okw["metric"])
    A = oracle.grid_eval(oracle.Kernel(**okw), oracle.Grid(n=n, b=b, layout=layout))
    k = tk.make_kernel(**kw)
    g = tk.make_grid(n, b, layout)
    d64 = torch.empty(n, dtype=torch.float64, device="cuda")
    tk.tk_grid_eval(ctx.handle, k, g, tk.TK_FP64, d64)
    got = host(d64)
    sigma2 = kw.get("sigma2", 1.0)
    s_exp = np.abs(np.log(np.maximum(np.abs(A) / sigma2, 1e-300)))
    rtol = 2e-13 + 8 * 2.220446049250313e-16 * s_exp
    assert np.all(np.abs(got - A) <= rtol * np.abs(A) + 1e-300)
    _check_f32(ctx, tk, k, g, n, A)


@pytest.mark.parametrize("name,kw", [f for f in FAMILIES if "metric" not in f[1]][:3])
def test_compress_radial_route_matches_direct(ctx, tk, oracle, name, kw):
    """A compression whose grid takes the radial-table route against the same compression of the
    oracle's tensor handed in (tk_compress_tensor, no grid evaluation on the GPU)."""
    n = (48, 48, 48)
    kern = tk.make_kernel(**kw)
    grid = tk.make_grid(n, 1.0, 1)
    A = oracle.grid_eval(oracle.Kernel(**kw), oracle.Grid(n=n, b=(1.0, 1.0, 1.0), layout=1))
    opts = tk.make_opts(ranks=6, hooi_sweeps=2, prec=tk.TK_FP64)
    t1 = ctx.compress(kern, grid, opts)
    t2 = ctx.compress_tensor(dev(A), grid, opts)
    say("  rel_err route %.6e tensor %.6e" % (t1.rel_err, t2.rel_err))
    assert abs(t1.rel_err - t2.rel_err) <= 1e-9 * max(t2.rel_err, 1e-12) + 1e-14
    t1.free()
    t2.free()


# (256, 288, 32) and (64, 32, 320): FP32 modes with n_mode >= 256 take the large-tile kernel
# (128 x 128 tiles; 288 and 320 leave a ragged last tile)
@pytest.mark.parametrize("shape", [(64, 64, 64), (70, 33, 129), (5, 7, 200), (256, 288, 32), (64, 32, 320)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_gram(ctx, tk, oracle, shape, prec):
    say("gram", shape, prec)
    X = synth.random_tensor(shape, 21) + 0.5
    if prec != 0:
        X = X.astype(np.float32).astype(np.float64)   # the GPU sees exactly these floats
    Xd = dev(X, np.float64 if prec == 0 else np.float32)
    for mode in range(3):
        G = torch.empty((shape[mode], shape[mode]), dtype=torch.float64, device="cuda")
        tk.tk_gram(ctx.handle, Xd, shape, mode, prec, G)
        got = host(G)
        ref = oracle.gram(X, mode)
        scale = np.abs(ref).max()
        tol = {0: 1e-13, 1: 1e-5, 2: 6e-5}[prec]
        err = np.abs(got - ref).max() / scale
        say("  mode", mode, "rel err %.2e" % err)
        assert err <= tol
        assert np.array_equal(got, got.T)          # mirrored exactly


@pytest.mark.parametrize("shape,mode", [((96, 80, 72), 1), ((32, 256, 64), 1), ((256, 32, 256), 2)])
def test_gram_deterministic(ctx, tk, shape, mode):
    X = dev(synth.random_tensor(shape, 5), np.float32)
    outs = []
    for _ in range(2):
        G = torch.empty((shape[mode], shape[mode]), dtype=torch.float64, device="cuda")
        tk.tk_gram(ctx.handle, X, shape, mode, tk.TK_FP32, G)
        outs.append(host(G))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("n,r", [(40, 6), (64, 16), (100, 12), (256, 24), (300, 48)])
def test_eig_topr(ctx, tk, oracle, n, r):
    say("eig", n, r)
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.2),
                         oracle.Grid(n=(n, 24, 20), layout=oracle.OFFSET))
    G = oracle.gram(A, 0)
    lam_o, V_o, _ = oracle.jacobi_eig(G)
    Gd = dev(G)
    lam = torch.empty(r, dtype=torch.float64, device="cuda")
    U = torch.empty((n, r), dtype=torch.float64, device="cuda")
    tk.tk_eig_topr(ctx.handle, 1, n, r, Gd, lam, U)
    lam_g, U_g = host(lam), host(U)
    l1 = lam_o[0]
    np.testing.assert_allclose(lam_g, lam_o[:r], rtol=0, atol=1e-13 * l1)
    assert np.abs(U_g.T @ U_g - np.eye(r)).max() < 1e-12
    assert np.abs(G @ U_g - U_g * lam_g).max() <= 1e-12 * l1
    # eigenvectors that the FP64 Gram determines (gap >> u * lambda_1) match the oracle's
    for j in range(r):
        gap = min(abs(lam_o[j] - lam_o[j - 1]) if j > 0 else np.inf, abs(lam_o[j] - lam_o[j + 1]))
        bound = 1e-14 * l1 / gap * 50 + 1e-13
        if bound < 1e-4:
            assert np.abs(U_g[:, j] - V_o[:, j]).max() <= bound, (j, gap / l1)


@pytest.mark.parametrize("n,r", [(640, 24), (1000, 12), (1024, 20)])
def test_eig_topr_large(ctx, tk, oracle, n, r):
    """Blocks of 513-1024 rows: the register QR holds two rows per thread.  Reference: LAPACK's
    symmetric eigensolver (numpy.linalg.eigh) on the oracle's Gram."""
    say("eig large", n, r)
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.3),
                         oracle.Grid(n=(n, 16, 12), layout=oracle.CENTERED))
    G = oracle.gram(A, 0)
    w, V = np.linalg.eigh(G)
    lam_o, V_o = w[::-1], V[:, ::-1]
    lam = torch.empty(r, dtype=torch.float64, device="cuda")
    U = torch.empty((n, r), dtype=torch.float64, device="cuda")
    tk.tk_eig_topr(ctx.handle, 1, n, r, dev(G), lam, U)
    lam_g, U_g = host(lam), host(U)
    l1 = lam_o[0]
    np.testing.assert_allclose(lam_g, lam_o[:r], rtol=0, atol=1e-12 * l1)
    assert np.abs(U_g.T @ U_g - np.eye(r)).max() < 1e-12
    assert np.abs(G @ U_g - U_g * lam_g).max() <= 1e-11 * l1


def test_eig_batched_matches_single(ctx, tk, oracle):
    n, r = 96, 10
    Gs = []
    for i, ell in enumerate((0.1, 0.3, 1.0)):
        A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=1.5, ell=ell), oracle.Grid(n=(n, 20, 20)))
        Gs.append(oracle.gram(A, 0))
    Gd = dev(np.stack(Gs))
    lam = torch.empty((3, r), dtype=torch.float64, device="cuda")
    U = torch.empty((3, n, r), dtype=torch.float64, device="cuda")
    tk.tk_eig_topr(ctx.handle, 3, n, r, Gd, lam, U)
    lb, Ub = host(lam), host(U)
    for i in range(3):
        lam1 = torch.empty(r, dtype=torch.float64, device="cuda")
        U1 = torch.empty((n, r), dtype=torch.float64, device="cuda")
        tk.tk_eig_topr(ctx.handle, 1, n, r, dev(Gs[i]), lam1, U1)
        np.testing.assert_allclose(lb[i], host(lam1), rtol=0, atol=1e-13 * lb[i][0])
