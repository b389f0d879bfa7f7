"""Separable covariance C = C_1 (x) C_2 (x) C_3 on the GPU (Sec. 4, "Separable covariance
matrices") against the oracle's plain Cholesky, substitution solves and log-determinant lemma.

Tolerances: a backward-stable Cholesky has ||L L^T - C|| <= c n u ||C||; factors, solves and
log-likelihoods are then compared to the oracle within the forward error the conditioning of
the factors allows (cond(C_k) u, summed over the three modes)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


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


def _setup(tk, oracle, n, layout=0):
    okern = [oracle.Kernel(oracle.GAUSS, ell=0.5, sigma2=1.7), oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.4),
             oracle.Kernel(oracle.GAUSS, ell=0.8)]
    kerns = [tk.make_kernel(tk.TK_GAUSS, ell=0.5, sigma2=1.7), tk.make_kernel(tk.TK_MATERN, nu=1.5, ell=0.4),
             tk.make_kernel(tk.TK_GAUSS, ell=0.8)]
    nug = (1e-3, 1e-4, 1e-3)
    b = (1.0, 1.3, 0.8)
    Cs = [oracle.cov_factor_1d(okern[a], n[a], b[a], layout, nug[a]) for a in range(3)]
    return kerns, tk.make_grid(n, b, layout), nug, Cs


@pytest.mark.parametrize("n,layout", [((40, 64, 33), 0), ((97, 130, 70), 1), ((2, 17, 5), 0)])
def test_kron1_factors_and_logdet(ctx, tk, oracle, n, layout):
    kerns, grid, nug, Cs = _setup(tk, oracle, n, layout)
    say("kron1 factors", n, layout)
    k = tk.Kron1(ctx, kerns, grid, nug)
    Ls = [oracle.cholesky(C) for C in Cs]
    for a in range(3):
        L = k.factor(a)
        C = Cs[a]
        bwd = np.abs(L @ L.T - C).max() / np.abs(C).max()
        fwd = np.abs(L - Ls[a]).max() / np.abs(Ls[a]).max()
        cond = np.linalg.cond(C)
        say("  axis %d: n=%d backward %.2e forward %.2e cond %.1e" % (a, n[a], bwd, fwd, cond))
        assert bwd <= 4 * n[a] * U64
        assert fwd <= 10 * cond * U64 + 1e-15
        assert np.all(np.triu(L, 1) == 0)
    ld, per = k.logdet()
    want = oracle.kron1_logdet(Ls)
    assert ld == pytest.approx(want, rel=1e-10, abs=1e-9)
    k.free()


def test_kron1_solve_cholesky_loglik(ctx, tk, oracle):
    n = (24, 30, 20)
    kerns, grid, nug, Cs = _setup(tk, oracle, n)
    k = tk.Kron1(ctx, kerns, grid, nug)
    Ls = [oracle.cholesky(C) for C in Cs]
    z = synth.random_tensor(n, 17)
    zd = dev(z.reshape(-1))
    w = torch.empty_like(zd)
    k.solve(zd, w)
    want = oracle.kron1_solve(Ls, z).reshape(-1)
    cond = sum(np.linalg.cond(C) for C in Cs)
    err = np.abs(host(w) - want).max() / np.abs(want).max()
    say("solve rel err %.2e (cond sum %.1e)" % (err, cond))
    assert err <= 10 * cond * U64
    y = torch.empty_like(zd)
    k.chol_apply(zd, y)
    want = oracle.kron1_chol_apply(Ls, z).reshape(-1)
    assert np.abs(host(y) - want).max() <= 1e-12 * np.abs(want).max()
    ll, q = k.loglik(zd)
    want_ll = oracle.kron1_loglik(Ls, z)
    say("loglik gpu %.12e oracle %.12e" % (ll, want_ll))
    assert ll == pytest.approx(want_ll, rel=10 * cond * U64)
    k.free()


def test_kron1_sampling_covariance(ctx, tk, oracle):
    """y = L z with z ~ N(0, I) has covariance L L^T = C, and its quadratic form is
    y^T C^-1 y = z^T L^T L^-T L^-1 L z = z^T z (up to rounding)."""
    n = (16, 20, 12)
    kerns, grid, nug, Cs = _setup(tk, oracle, n)
    k = tk.Kron1(ctx, kerns, grid, nug)
    z = synth.normal_vector(n, 3).astype(np.float64)
    zd = dev(z.reshape(-1))
    y = torch.empty_like(zd)
    k.chol_apply(zd, y)
    _, q = k.loglik(y)
    assert q == pytest.approx(float(np.dot(z.reshape(-1), z.reshape(-1))), rel=1e-9)
    k.free()


def test_kron1_not_positive_definite(ctx, tk):
    kern = tk.make_kernel(tk.TK_GAUSS, ell=2.0)
    with pytest.raises(tk.TkError) as ei:
        tk.Kron1(ctx, [kern] * 3, tk.make_grid(200, 1.0), None)
    assert "TK_EINVAL" in str(ei.value) and "nugget" in str(ei.value)


def test_kron1_paper_size_6000(ctx, tk):
    """The size of the example in Sec. 4 (n = 6000 per axis, d = 3, N = 6000^3): only the three
    factors and their Cholesky factors are formed, never C or L.  Backward error on sampled rows."""
    n = 6000
    kern = tk.make_kernel(tk.TK_GAUSS, ell=0.3)
    grid = tk.make_grid(n, 1.0)
    k = tk.Kron1(ctx, [kern] * 3, grid, (1e-4, 1e-4, 1e-4))
    ld, per = k.logdet()
    L = k.factor(0)
    x = np.linspace(-1.0, 1.0, n)
    rows = np.random.default_rng(0).choice(n, 40, replace=False)
    for i in rows:
        c = np.exp(-((x[i] - x) / 0.3) ** 2)
        c[i] += 1e-4
        assert np.abs(L[i] @ L.T - c).max() <= 8 * n * U64
    assert np.isfinite(ld) and ld == pytest.approx(3 * n * n * per[0], rel=1e-12)
    k.free()
