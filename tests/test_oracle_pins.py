"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compare the oracle with itself: each checks it against a library routine used
only here (scipy / numpy), a closed form, an invariant, a special case with a textbook answer,
brute force on tiny inputs, or the values the paper prints (Table 4.2).
"""
import json
import os

import numpy as np
import pytest
from scipy import special

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- covariance functions ----

@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("ell", [0.05, 0.3, 1.0])
def test_matern_matches_scipy_bessel(oracle, nu, ell):
    """Sec. 2.2 eq. (2.3) evaluated with scipy's K_nu and Gamma."""
    for r in [1e-6, 0.01, 0.1, 0.5, 1.0, 1.7]:
        s = np.sqrt(2 * nu) * r / ell
        if s > 600:
            continue
        ref = 2.0 ** (1 - nu) / special.gamma(nu) * s ** nu * special.kv(nu, s)
        got = oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=nu, ell=ell, sigma2=2.0), r)
        assert got == pytest.approx(2.0 * ref, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_closed_forms(oracle, nu):
    """The half-integer closed forms: e^{-s}, (1+s)e^{-s}, (1+s+s^2/3)e^{-s}."""
    ell = 0.37
    for r in np.linspace(0.0, 2.0, 23):
        s = np.sqrt(2 * nu) * r / ell
        poly = {0.5: 1.0, 1.5: 1.0 + s, 2.5: 1.0 + s + s * s / 3.0}[nu]
        assert oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=nu, ell=ell), r) == \
            pytest.approx(poly * np.exp(-s), rel=1e-13, abs=1e-300)


def test_kernel_at_zero_is_variance(oracle):
    for fam, kw in [(oracle.MATERN, dict(nu=0.5)), (oracle.MATERN, dict(nu=1.5)),
                    (oracle.MATERN, dict(nu=2.5)), (oracle.SLATER, dict(p=0.1)),
                    (oracle.GAUSS, {})]:
        assert oracle.kernel_value(oracle.Kernel(fam, ell=0.2, sigma2=3.5, **kw), 0.0) == 3.5


def test_nonpositive_nu_is_nan(oracle):
    assert np.isnan(oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=0.0), 0.3))
    assert np.isnan(oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=-1.0), 0.3))


def test_slater_p1_equals_exponential_matern(oracle):
    for ell in (0.1, 0.3, 1.0):
        for r in np.linspace(0.0, 1.8, 19):
            a = oracle.kernel_value(oracle.Kernel(oracle.SLATER, alpha=1.0, p=1.0, ell=ell), r)
            b = oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=0.5, ell=ell), r)
            assert a == pytest.approx(b, rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("p", [0.1, 0.5, 1.9, 2.0])
@pytest.mark.parametrize("alpha", [0.7, 2.0])
@pytest.mark.parametrize("ell", [0.05, 0.5])
def test_slater_special_points(oracle, p, alpha, ell):
    """p-Slater sigma2 exp(-alpha (r/ell)^p) (Sec. 3.7 eq. (3.27) with rate and length) at points
    where the exponent is a plain number: r = ell gives exp(-alpha) for every p, r = 2 ell gives
    exp(-alpha 2^p), r = ell/4 gives exp(-alpha 4^-p).  A length applied after the power
    (r^p / ell) or a rate applied inside it fails these for p != 1."""
    k = oracle.Kernel(oracle.SLATER, alpha=alpha, p=p, ell=ell, sigma2=1.3)
    for r, expo in [(ell, 1.0), (2 * ell, 2.0 ** p), (ell / 4, 0.25 ** p)]:
        assert oracle.kernel_value(k, r) == pytest.approx(1.3 * np.exp(-alpha * expo), rel=1e-14)


@pytest.mark.parametrize("p", [0.1, 0.5, 1.9])
def test_slater_scaling_laws(oracle, p):
    """C(r; alpha, p, ell) = C(c r; alpha, p, c ell) (a length scale), and
    C(r; alpha, p, ell) = C(r; alpha c^p, p, c ell) (rate and length trade through the power)."""
    base = oracle.Kernel(oracle.SLATER, alpha=0.9, p=p, ell=0.3)
    for c in (0.37, 4.1):
        stretched = oracle.Kernel(oracle.SLATER, alpha=0.9, p=p, ell=0.3 * c)
        traded = oracle.Kernel(oracle.SLATER, alpha=0.9 * c ** p, p=p, ell=0.3 * c)
        for r in np.linspace(0.01, 1.7, 12):
            v = oracle.kernel_value(base, r)
            assert oracle.kernel_value(stretched, c * r) == pytest.approx(v, rel=1e-13, abs=1e-300)
            assert oracle.kernel_value(traded, r) == pytest.approx(v, rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("alpha", [0.7, 2.0])
def test_slater_p2_is_gaussian(oracle, alpha):
    """p = 2: exp(-alpha (r/ell)^2) is the Gaussian of length ell / sqrt(alpha)."""
    for ell in (0.05, 0.5):
        s = oracle.Kernel(oracle.SLATER, alpha=alpha, p=2.0, ell=ell, sigma2=0.8)
        g = oracle.Kernel(oracle.GAUSS, ell=ell / np.sqrt(alpha), sigma2=0.8)
        for r in np.linspace(0.0, 3 * ell, 13):
            assert oracle.kernel_value(s, r) == pytest.approx(oracle.kernel_value(g, r), rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("a", [0.3, 1.0, 2.5])
def test_slater_p1_laplace_representation(oracle, a):
    """Sec. 3.5: exp(-2 sqrt(a q)) = sqrt(a/pi) int_0^inf t^(-3/2) exp(-a/t - q t) dt with
    q = ||x||^2, i.e. the Slater function of rate 2 sqrt(a) (p = 1) -- evaluated by quadrature."""
    from scipy import integrate
    k = oracle.Kernel(oracle.SLATER, alpha=2 * np.sqrt(a), p=1.0, ell=1.0)
    for r in (0.05, 0.4, 1.3):
        q = r * r
        f = lambda t: t ** -1.5 * np.exp(-a / t - q * t)
        val = np.sqrt(a / np.pi) * (integrate.quad(f, 0, 1, limit=200, epsabs=0, epsrel=1e-13)[0] +
                                    integrate.quad(f, 1, np.inf, limit=200, epsabs=0, epsrel=1e-13)[0])
        assert oracle.kernel_value(k, r) == pytest.approx(val, rel=1e-9)


# ------------------------------------------------------- general Matern order, spectral density ----

@pytest.mark.parametrize("nu", [0.05, 0.3, 0.8, 1.2, 2.0, 3.7, 7.3, 15.0])
def test_bessel_k_integral_matches_mpmath(oracle, nu):
    """K_nu by the trapezoidal rule on its integral representation against mpmath's
    arbitrary-precision K_nu (test-only library).  Each term exp(nu t - x cosh t) is rounded
    once in its exponent, whose size reaches ~200 at small x and large nu: 1e-13 relative."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for x in [1e-4, 1e-3, 0.01, 0.3, 1.0, 2.0, 2.5, 10.0, 50.0, 200.0, 600.0]:
        ref = float(mpmath.besselk(nu, x))
        assert oracle.bessel_k(nu, x) == pytest.approx(ref, rel=1e-13), (nu, x)


@pytest.mark.parametrize("nu", [0.4, 0.75, 1.0, 2.2, 4.0])
def test_matern_general_order(oracle, nu):
    """Sec. 2.2 eq. (2.3) at orders that are not half-integers, against mpmath; r = 0 gives
    sigma2; the value is continuous in nu across a half-integer (the series branch)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    ell, s2 = 0.35, 1.7
    k = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell, sigma2=s2)
    assert oracle.kernel_value(k, 0.0) == s2
    for r in [1e-5, 0.01, 0.2, 0.7, 1.5, 3.0]:
        sv = mpmath.sqrt(2 * mpmath.mpf(nu)) * r / ell
        ref = s2 * float(2 ** (1 - mpmath.mpf(nu)) / mpmath.gamma(nu) * sv ** nu * mpmath.besselk(nu, sv))
        assert oracle.kernel_value(k, r) == pytest.approx(ref, rel=5e-14), (nu, r)
    a = oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=1.5 + 1e-9, ell=ell), 0.4)
    b = oracle.kernel_value(oracle.Kernel(oracle.MATERN, nu=1.5, ell=ell), 0.4)
    assert a == pytest.approx(b, rel=1e-8)


@pytest.mark.parametrize("nu,alpha", [(0.4, 0.1), (0.4, 100.0), (1.5, 2.0), (2.7, 0.5)])
def test_spectral_density_is_a_probability_density(oracle, nu, alpha):
    """The constant of the spectral density in Diagram 1 (Sec. 2.2) makes it integrate to one
    over R^3: 4 pi int_0^inf rho^2 f(rho) d rho = 1 (quadrature)."""
    from scipy import integrate
    k = oracle.Kernel(oracle.SPECTRAL, nu=nu, alpha=alpha)
    f = lambda rho: 4 * np.pi * rho * rho * oracle.kernel_value(k, rho)
    tot = sum(integrate.quad(f, a, b, limit=400, epsabs=0, epsrel=1e-12)[0]
              for a, b in [(0, alpha), (alpha, 10 * alpha), (10 * alpha, np.inf)])
    assert tot == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("nu,ell", [(0.5, 0.3), (1.5, 0.5), (2.3, 0.4)])
def test_spectral_density_transforms_to_matern(oracle, nu, ell):
    """Diagram 1 (Sec. 2.2): the 3-D Fourier transform of the spectral density with
    alpha = sqrt(2 nu)/ell is the Matern covariance, C(r) = (4 pi / r) int rho sin(rho r) f(rho).
    Pins the spectral family against the Matern family (two independent code paths)."""
    from scipy import integrate
    alpha = np.sqrt(2 * nu) / ell
    ks = oracle.Kernel(oracle.SPECTRAL, nu=nu, alpha=alpha)
    km = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell)
    for r in (0.1, 0.4, 1.0):
        g = lambda rho: rho * oracle.kernel_value(ks, rho)
        val = 4 * np.pi / r * integrate.quad(g, 0, np.inf, weight="sin", wvar=r, limlst=200)[0]
        assert val == pytest.approx(oracle.kernel_value(km, r), rel=1e-6), (nu, r)


def test_anisotropic_metric(oracle):
    """r^2 = sum_k a_k x_k^2 with a positive diagonal metric (Sec. 2.2): the identity metric is
    the isotropic tensor, and metric a on the box b equals the isotropic tensor on the box
    sqrt(a) b (coordinates scaled per axis)."""
    n = (7, 9, 8)
    for layout in (oracle.CENTERED, oracle.OFFSET):
        g = oracle.Grid(n=n, b=(1.0, 0.8, 1.3), layout=layout)
        iso = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.4)
        same = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.4, metric=(1.0, 1.0, 1.0))
        assert np.array_equal(oracle.grid_eval(iso, g), oracle.grid_eval(same, g))
        a = (4.0, 1.0, 0.25)
        an = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.4, metric=a)
        g2 = oracle.Grid(n=n, b=tuple(np.sqrt(a) * np.asarray(g.b)), layout=layout)
        np.testing.assert_allclose(oracle.grid_eval(an, g), oracle.grid_eval(iso, g2), rtol=1e-14, atol=0)


# ------------------------------------------------------------------------------- grid ----

def test_grid_coordinates(oracle):
    x = oracle.grid_coords(9, 2.0, oracle.CENTERED)
    np.testing.assert_allclose(x, np.linspace(-2.0, 2.0, 9), rtol=0, atol=1e-15)
    y = oracle.grid_coords(9, 2.0, oracle.OFFSET)
    np.testing.assert_allclose(y, np.linspace(0.0, 4.0, 9), rtol=0, atol=1e-15)


def test_grid_values_direct(oracle):
    """Entries against a direct numpy evaluation of the closed form on explicit coordinates."""
    k = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.3, sigma2=1.7)
    g = oracle.Grid(n=(5, 6, 7), b=(1.0, 0.5, 2.0), layout=oracle.CENTERED)
    A = oracle.grid_eval(k, g)
    xs = [np.linspace(-b, b, n) for n, b in zip(g.n, g.b)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    s = np.sqrt(3.0) * np.sqrt(X ** 2 + Y ** 2 + Z ** 2) / 0.3
    np.testing.assert_allclose(A, 1.7 * (1 + s) * np.exp(-s), rtol=1e-13, atol=0)


def test_grid_symmetries(oracle):
    k = oracle.Kernel(oracle.MATERN, nu=2.5, ell=0.4)
    A = oracle.grid_eval(k, oracle.Grid(n=(11, 11, 11)))
    np.testing.assert_allclose(A, A[::-1, :, :], rtol=1e-14)
    np.testing.assert_allclose(A, A[:, ::-1, ::-1], rtol=1e-14)
    np.testing.assert_allclose(A, A.transpose(1, 0, 2), rtol=1e-14)
    np.testing.assert_allclose(A, A.transpose(2, 1, 0), rtol=1e-14)


# ------------------------------------------------------------------------------- Gram ----

@pytest.mark.parametrize("shape", [(3, 4, 5), (8, 8, 8), (7, 2, 6)])
def test_gram_bruteforce(oracle, shape):
    X = synth.random_tensor(shape, 1)
    subs = ["ajk,bjk->ab", "iaj,ibj->ab", "ija,ijb->ab"]
    for k in range(3):
        G = oracle.gram(X, k)
        np.testing.assert_allclose(G, np.einsum(subs[k], X, X), rtol=1e-13, atol=1e-13)
        assert np.trace(G) == pytest.approx(np.sum(X * X), rel=1e-13)
        np.testing.assert_array_equal(G, G.T)
        assert np.linalg.eigvalsh(G).min() > -1e-12 * np.trace(G)


def test_gram_equal_modes_on_symmetric_tensor(oracle):
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3), oracle.Grid(n=(9, 9, 9)))
    G = [oracle.gram(A, k) for k in range(3)]
    np.testing.assert_allclose(G[0], G[1], rtol=1e-13)
    np.testing.assert_allclose(G[0], G[2], rtol=1e-13)


# ------------------------------------------------------------------------------ eigen ----

def _sign_fix(V):
    V = V.copy()
    for j in range(V.shape[1]):
        a = np.abs(V[:, j])
        lead = int(np.nonzero(a >= a.max() * (1 - 1e-10))[0][0])
        if V[lead, j] < 0:
            V[:, j] = -V[:, j]
    return V


@pytest.mark.parametrize("n", [1, 2, 7, 20, 33])
def test_jacobi_matches_eigh(oracle, n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    S = B + B.T
    lam, V, sweeps = oracle.jacobi_eig(S)
    assert sweeps >= 0
    ref_l, ref_v = np.linalg.eigh(S)
    order = np.argsort(-ref_l, kind="stable")
    np.testing.assert_allclose(lam, ref_l[order], rtol=0, atol=1e-13 * np.linalg.norm(S))
    np.testing.assert_allclose(V, _sign_fix(ref_v[:, order]), rtol=0, atol=1e-11)
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-14 * max(n, 1) ** 0.5 * 10)
    resid = S @ V - V * lam[None, :]
    assert np.abs(resid).max() <= 1e-13 * np.linalg.norm(S)
    assert np.all(np.diff(lam) <= 0)


def test_jacobi_gram_spectrum_and_trace(oracle):
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3), oracle.Grid(n=(24, 20, 16)))
    for k in range(3):
        G = oracle.gram(A, k)
        lam, V, _ = oracle.jacobi_eig(G)
        assert np.sum(lam) == pytest.approx(np.trace(G), rel=1e-13)
        assert np.abs(G @ V - V * lam).max() <= 1e-13 * np.linalg.norm(G)
        np.testing.assert_allclose(lam[:6], np.linalg.eigvalsh(G)[::-1][:6], rtol=0,
                                   atol=1e-13 * np.linalg.norm(G))


def test_jacobi_repeated_eigenvalues(oracle):
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    d = np.array([5.0, 5.0, 5.0, 2.0, 2.0, 1.0, 0.0, 0.0, -1.0, -1.0])
    S = (Q * d) @ Q.T
    lam, V, _ = oracle.jacobi_eig(S)
    np.testing.assert_allclose(lam, np.sort(d)[::-1], atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(10), atol=1e-13)
    assert np.abs(S @ V - V * lam).max() <= 1e-13 * 10


# -------------------------------------------------------------------- mode products ----

def test_mode_product_bruteforce(oracle):
    X = synth.random_tensor((4, 5, 6), 2)
    rng = np.random.default_rng(5)
    subs = ["ja,abc->jbc", "jb,abc->ajc", "jc,abc->abj"]
    for k in range(3):
        M = rng.standard_normal((3, X.shape[k]))
        np.testing.assert_allclose(oracle.mode_product(X, k, M), np.einsum(subs[k], M, X),
                                   rtol=1e-13, atol=1e-13)


# -------------------------------------------------------------------------- HOSVD ----

def test_full_rank_is_exact(oracle):
    """Full rank gives an exact representation (Sec. 1 list of properties)."""
    X = synth.random_tensor((5, 6, 7), 3)
    t = oracle.hosvd(X, X.shape)
    assert t.rel_err <= 1e-13
    np.testing.assert_allclose(oracle.reconstruct(t.core, t.U), X, atol=1e-13)
    for u in t.U:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)


def test_gaussian_is_rank_one(oracle):
    """Separable covariance (Sec. 4.4): the Gaussian kernel is a rank-1 tensor."""
    A = oracle.grid_eval(oracle.Kernel(oracle.GAUSS, ell=0.6), oracle.Grid(n=(12, 10, 14)))
    t = oracle.hosvd(A, (1, 1, 1))
    assert t.rel_err <= 1e-13
    # eps^2 must stay above the Gram route's FP64 noise (~1e-16 relative eigenvalues)
    assert oracle.eps_ranks(t.lambdas, t.norm_a2, 1e-6) == (1, 1, 1)


def test_separable_exponential_is_rank_one(oracle):
    """Sec. 3.1: exp(x1 + x2 + x3) discretised on a tensor grid is canonical rank 1."""
    xs = [np.linspace(-1, 1, n) for n in (9, 11, 13)]
    A = np.exp(xs[0][:, None, None] + xs[1][None, :, None] + xs[2][None, None, :])
    t = oracle.hosvd(A, (1, 1, 1))
    assert t.rel_err <= 1e-13


def test_two_dimensional_case_is_svd(oracle):
    """Sec. 3.1: for d = 2 the orthogonal Tucker decomposition is the SVD."""
    A3 = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3),
                          oracle.Grid(n=(30, 24, 5)))
    A = np.ascontiguousarray(A3[:, :, 1:2])        # a 30 x 24 x 1 tensor (d = 2)
    M = A[:, :, 0]
    s = np.linalg.svd(M, compute_uv=False)
    Usvd, _, _ = np.linalg.svd(M)
    for r in (1, 2, 3, 4):
        t = oracle.hosvd(A, (r, r, 1))
        expect = np.sqrt(np.sum(s[r:] ** 2)) / np.sqrt(np.sum(s ** 2))
        assert expect > 1e-6          # above the Gram route's FP64 floor (~sqrt(u))
        assert t.rel_err == pytest.approx(expect, rel=1e-6)
        # same leading left singular subspace
        P = t.U[0] @ t.U[0].T
        Ps = Usvd[:, :r] @ Usvd[:, :r].T
        assert np.abs(P - Ps).max() < 1e-8


def _c1_tensor(oracle, n=32):
    return oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3), oracle.Grid(n=(n, n, n)))


def test_hosvd_sandwich_bound(oracle):
    """HOSVD error bound: max_k tau_k <= E^2 <= sum_k tau_k (De Lathauwer et al.)."""
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.25),
                         oracle.Grid(n=(20, 16, 12)))
    f = oracle.hosvd_factors(A)
    na2 = oracle.sumsq(A)
    for r in (1, 2, 4, 6):
        t = oracle.hosvd(A, (r, r, r), f)
        tau = [np.sum(f[k][0][r:]) / na2 for k in range(3)]
        e2 = t.rel_err ** 2
        assert max(tau) * (1 - 1e-9) <= e2 <= sum(tau) * (1 + 1e-9) + 1e-28


def test_hosvd_error_decays_exponentially(oracle):
    """Sec. 3.7: E_FN decays exponentially in the Tucker rank (above the FP64 floor of the
    Gram route) and never increases with r (nested subspaces)."""
    A = _c1_tensor(oracle, 40)
    f = oracle.hosvd_factors(A)
    errs = [oracle.hosvd(A, (r, r, r), f).rel_err for r in range(1, 13)]
    assert all(b <= a * (1 + 1e-9) for a, b in zip(errs, errs[1:]))
    pre = [e for e in errs if e > 1e-7]
    slope = np.polyfit(np.arange(len(pre)), np.log(pre), 1)[0]
    assert slope < -0.8          # at least a factor e^0.8 per rank
    assert pre[-1] < 1e-5


def test_eps_rule_meets_tolerance(oracle):
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=2.5, ell=0.3), oracle.Grid(n=(28, 28, 28)))
    for eps in (1e-2, 1e-4, 1e-6):
        t = oracle.compress(oracle.Kernel(), oracle.Grid(), eps=eps, sweeps=0, A=A)
        assert t.rel_err <= eps
        smaller = [max(1, r - 1) for r in t.ranks]
        if smaller != list(t.ranks):
            worse = oracle.hosvd(A, smaller)
            assert worse.rel_err > t.rel_err


def test_pythagoras(oracle):
    """Orthogonal projection: ||A||^2 = ||G||^2 + ||A - A_r||^2."""
    A = _c1_tensor(oracle, 24)
    for r in (1, 3, 5):
        t = oracle.hosvd(A, (r, r, r))
        na2 = oracle.sumsq(A)
        assert oracle.sumsq(t.core) + t.rel_err ** 2 * na2 == pytest.approx(na2, rel=1e-13)


# --------------------------------------------------------------------------- HOOI ----

def test_hooi_improves_and_is_monotone(oracle):
    A = oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.2),
                         oracle.Grid(n=(22, 18, 26)))
    for r in (2, 4):
        h0 = oracle.hosvd(A, (r, r + 1, r))
        h = oracle.hooi(A, h0, sweeps=None)
        assert h.rel_err <= h0.rel_err * (1 + 1e-12)
        hist = np.asarray(h.history)
        assert np.all(np.diff(hist) >= -1e-12 * hist[0])
        na2 = oracle.sumsq(A)
        assert oracle.sumsq(h.core) + h.rel_err ** 2 * na2 == pytest.approx(na2, rel=1e-12)


def _table_case(oracle, n, ranks_to_check):
    tab = json.load(open(os.path.join(GOLDEN, "table_4_2.json")))
    b = tab["box_half_width"]
    printed = tab["printed"][str(n)]
    excluded = set(tab["excluded"].get(str(n), []))
    A = oracle.grid_eval(oracle.Kernel(oracle.SLATER, alpha=1.0, p=1.0, ell=1.0),
                         oracle.Grid(n=(n, n, n), b=(b, b, b)))
    f = oracle.hosvd_factors(A)
    c = (n - 1) // 2
    for r in ranks_to_check:
        if r in excluded:
            continue
        h = oracle.hooi(A, oracle.hosvd(A, (r, r, r), f), sweeps=None)
        err = 1.0 - oracle.reconstruct(h.core, h.U)[c, c, c]
        want = printed[r - 1]
        assert err == pytest.approx(want, rel=tab["rel_tol"]), (n, r, err, want)
        # the origin value is also the relative trace error of the covariance (odd grid)
        g = oracle.Grid(n=(n, n, n), b=(b, b, b))
        m = (n + 1) // 2
        assert oracle.cov_trace(h, g) == pytest.approx((1.0 - err) * m ** 3, rel=1e-12)


def test_table_4_2_n129(oracle):
    _table_case(oracle, 129, range(1, 11))


def test_table_4_2_n257(oracle):
    _table_case(oracle, 257, range(1, 11))


def test_table_4_2_n513(oracle):
    _table_case(oracle, 513, range(1, 11))


# ------------------------------------------------------------ covariance operator ----

def _dense_cov_from_generator(Q, off, m):
    """Dense matrix C[(i),(j)] = Q[off + |i - j|] built by plain index arithmetic."""
    idx = np.array(np.unravel_index(np.arange(m[0] * m[1] * m[2]), m)).T
    N = idx.shape[0]
    C = np.empty((N, N))
    for a in range(N):
        d = np.abs(idx - idx[a]) + np.asarray(off)
        C[a] = Q[d[:, 0], d[:, 1], d[:, 2]]
    return C


@pytest.mark.parametrize("layout,n", [(1, (6, 5, 7)), (0, (7, 5, 9))])
def test_cov_matvec_bruteforce(oracle, layout, n):
    k = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.5)
    g = oracle.Grid(n=n, b=(1.0, 0.7, 1.3), layout=layout)
    A = oracle.grid_eval(k, g)
    t = oracle.hosvd(A, (3, 2, 4))
    off, m = oracle.cov_offsets(g)
    z = synth.normal_vector(m, 1).astype(np.float64)
    y = oracle.cov_matvec(t, g, z)
    C = _dense_cov_from_generator(oracle.reconstruct(t.core, t.U), off, m)
    np.testing.assert_allclose(y.reshape(-1), C @ z.reshape(-1), rtol=1e-12, atol=1e-12)
    # symmetry <y, C z> = <C y, z>
    w = synth.normal_vector(m, 2).astype(np.float64)
    assert np.dot(w.reshape(-1), y.reshape(-1)) == pytest.approx(
        np.dot(oracle.cov_matvec(t, g, w).reshape(-1), z.reshape(-1)), rel=1e-12)


def test_cov_full_rank_is_exact_covariance(oracle):
    """At full rank the operator is the covariance matrix C_ij = c(||x_i - x_j||) (Sec. 3.6)."""
    k = oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.4, sigma2=1.3)
    g = oracle.Grid(n=(5, 6, 4), b=(1.0, 1.0, 1.0), layout=oracle.OFFSET)
    A = oracle.grid_eval(k, g)
    t = oracle.hosvd(A, A.shape)
    xs = [np.linspace(-1, 1, n) for n in g.n]
    P = np.stack(np.meshgrid(*xs, indexing="ij"), -1).reshape(-1, 3)
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    C = 1.3 * np.exp(-D / 0.4)
    z = synth.normal_vector(g.n, 3).astype(np.float64)
    np.testing.assert_allclose(oracle.cov_matvec(t, g, z).reshape(-1), C @ z.reshape(-1),
                               rtol=1e-12, atol=1e-12)
    assert oracle.cov_trace(t, g) == pytest.approx(1.3 * np.prod(g.n), rel=1e-12)


def test_cov_separable_vector_lemma(oracle):
    """Sec. 4 eq. (4.1) / Lemma 4.1: for separable z the product is a sum of Kronecker terms
    sum_abc G_abc (T1a z1) (x) (T2b z2) (x) (T3c z3)."""
    k = oracle.Kernel(oracle.MATERN, nu=2.5, ell=0.6)
    g = oracle.Grid(n=(6, 7, 5), layout=oracle.OFFSET)
    t = oracle.hosvd(oracle.grid_eval(k, g), (3, 3, 2))
    rng = np.random.default_rng(9)
    zs = [rng.standard_normal(n) for n in g.n]
    z = np.einsum("i,j,k->ijk", *zs)
    y = oracle.cov_matvec(t, g, z)

    def toep(u):
        n = u.shape[0]
        return u[np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])]

    r = t.core.shape
    ref = np.zeros(g.n)
    for a in range(r[0]):
        for b in range(r[1]):
            for c in range(r[2]):
                f = [toep(t.U[0][:, a]) @ zs[0], toep(t.U[1][:, b]) @ zs[1],
                     toep(t.U[2][:, c]) @ zs[2]]
                ref += t.core[a, b, c] * np.einsum("i,j,k->ijk", *f)
    np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-12)


def test_trace_formulas_agree(oracle):
    for layout, n in ((1, (8, 6, 7)), (0, (9, 7, 11))):
        g = oracle.Grid(n=n, layout=layout)
        t = oracle.hosvd(oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3), g), (4, 3, 5))
        assert oracle.cov_trace(t, g) == pytest.approx(oracle.cov_trace_kron(t, g), rel=1e-12)


def test_even_centred_grid_has_no_covariance(oracle):
    assert oracle.cov_offsets(oracle.Grid(n=(8, 8, 8))) is None


def test_quadratic_form_is_dot(oracle):
    g = oracle.Grid(n=(5, 6, 4), layout=oracle.OFFSET)
    t = oracle.hosvd(oracle.grid_eval(oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.5), g), (2, 2, 2))
    z = synth.normal_vector(g.n, 4).astype(np.float64)
    C = _dense_cov_from_generator(oracle.reconstruct(t.core, t.U), (0, 0, 0), g.n)
    assert oracle.quadratic_form(t, g, z) == pytest.approx(z.reshape(-1) @ C @ z.reshape(-1),
                                                           rel=1e-12)


# ------------------------------------------------------------------- multigrid Tucker ----

def test_multigrid_sizes(oracle):
    assert oracle.multigrid_sizes(513, 3) == [65, 129, 257, 513]
    assert oracle.multigrid_sizes(1024, 3) == [128, 256, 512, 1024]
    assert oracle.multigrid_sizes(100, 1) == [50, 100]


def test_multigrid_interpolation_is_exact_on_linear_columns(oracle):
    """Linear interpolation reproduces affine functions exactly, nested (2^k+1 grids) or not."""
    for (nc, nf, layout) in [(9, 17, oracle.CENTERED), (16, 32, oracle.OFFSET), (7, 20, oracle.CENTERED)]:
        xc = oracle.grid_coords(nc, 1.3, layout)
        xf = oracle.grid_coords(nf, 1.3, layout)
        U = np.stack([1.0 + 2.0 * xc, 3.0 - 0.5 * xc], axis=1)
        want = np.stack([1.0 + 2.0 * xf, 3.0 - 0.5 * xf], axis=1)
        np.testing.assert_allclose(oracle.interpolate_factor(U, xc, xf), want, rtol=0, atol=1e-14)


def test_orthonormalize_keeps_the_span(oracle):
    U = synth.random_tensor((40, 6, 1), 3)[:, :, 0]
    Q = oracle.orthonormalize(U)
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), rtol=0, atol=1e-14)
    # U = Q (Q^T U): the columns of U lie in the span of Q
    np.testing.assert_allclose(Q @ (Q.T @ U), U, rtol=0, atol=1e-13)


def test_multigrid_reaches_the_direct_optimum(oracle):
    """Sec. 3.2: the multigrid start (coarse HOSVD, interpolated factors) and the direct start
    (HOSVD on the fine grid) lead converged Tucker-ALS to the same approximation."""
    k = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.3)
    g = oracle.Grid(n=(65, 65, 65), b=(1.0, 1.0, 1.0))
    A = oracle.grid_eval(k, g)
    f = oracle.hosvd_factors(A)
    for r in (3, 5, 7):
        mg = oracle.multigrid_compress(k, g, (r, r, r), 2, sweeps=None)
        d = oracle.hooi(A, oracle.hosvd(A, (r, r, r), f), sweeps=None)
        assert mg.rel_err == pytest.approx(d.rel_err, rel=1e-6), r


def test_multigrid_table_4_2_n129(oracle):
    """Table 4.2 at n = 129 reproduced through the multigrid route 33 -> 65 -> 129."""
    tab = json.load(open(os.path.join(GOLDEN, "table_4_2.json")))
    b = tab["box_half_width"]
    printed = tab["printed"]["129"]
    k = oracle.Kernel(oracle.SLATER, alpha=1.0, p=1.0, ell=1.0)
    g = oracle.Grid(n=(129, 129, 129), b=(b, b, b))
    for r in (1, 3, 5, 7, 9):
        t = oracle.multigrid_compress(k, g, (r, r, r), 2, sweeps=None)
        err = 1.0 - oracle.reconstruct(t.core, t.U)[64, 64, 64]
        assert err == pytest.approx(printed[r - 1], rel=tab["rel_tol"]), (r, err)


# ------------------------------------------------- separable covariance (rank-1 Kronecker) ----

def _kron3(a, b, c):
    return np.kron(np.kron(a, b), c)


def test_kron1_cholesky_matches_numpy(oracle):
    """Backward error ||L L^T - C|| at the rounding level, and numpy's factor to within the
    forward error that the condition number allows (cond(C) u)."""
    for n, ell in [(7, 0.4), (30, 0.9), (64, 0.2)]:
        C = oracle.cov_factor_1d(oracle.Kernel(oracle.GAUSS, ell=ell), n, 1.0, nugget=1e-6)
        L = oracle.cholesky(C)
        assert np.abs(L @ L.T - C).max() <= 4 * n * 2.2e-16 * np.abs(C).max()
        tol = 10 * np.linalg.cond(C) * 2.2e-16
        np.testing.assert_allclose(L, np.linalg.cholesky(C), rtol=0, atol=tol)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(-np.eye(3))


def test_gaussian_covariance_is_a_kronecker_product(oracle):
    """Sec. 4: the Gaussian covariance exp(-|x - y|^2 / ell^2) of the 3-D grid is exactly
    C_1 (x) C_2 (x) C_3 of its 1-D factors (checked against the plain covariance product of the
    offset generator, a different route)."""
    n = (4, 5, 3)
    k = oracle.Kernel(oracle.GAUSS, ell=0.7)
    Cs = [oracle.cov_factor_1d(k, n[a], 1.0) for a in range(3)]
    g = oracle.Grid(n=n, layout=oracle.OFFSET)
    Q = oracle.grid_eval(k, g)
    N = int(np.prod(n))
    dense = np.stack([oracle.cov_rows_from_generator(Q, g, np.eye(N)[j], np.arange(N)) for j in range(N)], axis=1)
    np.testing.assert_allclose(_kron3(*Cs), dense, rtol=1e-14, atol=1e-15)


def test_kron1_lemmas_against_dense(oracle):
    """Cholesky, inverse, log-determinant and log-likelihood of C = C_1 (x) C_2 (x) C_3 (the
    lemmas of Sec. 4) against the dense N x N matrix: numpy's Cholesky, slogdet and solve and
    scipy's multivariate normal log-density (test-only libraries)."""
    from scipy.stats import multivariate_normal
    n = (4, 6, 5)
    ks = [oracle.Kernel(oracle.GAUSS, ell=0.6), oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.4),
          oracle.Kernel(oracle.GAUSS, ell=1.1)]
    Cs = [oracle.cov_factor_1d(ks[a], n[a], 1.0, nugget=1e-2) for a in range(3)]
    Ls = [oracle.cholesky(C) for C in Cs]
    C = _kron3(*Cs)
    L = _kron3(*Ls)
    np.testing.assert_allclose(L, np.linalg.cholesky(C), rtol=0, atol=1e-12)
    z = synth.random_tensor(n, 8)
    zf = z.reshape(-1)
    assert oracle.kron1_logdet(Ls) == pytest.approx(np.linalg.slogdet(C)[1], rel=1e-12)
    np.testing.assert_allclose(oracle.kron1_solve(Ls, z).reshape(-1), np.linalg.solve(C, zf), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(oracle.kron1_chol_apply(Ls, z).reshape(-1), L @ zf, rtol=1e-13, atol=1e-14)
    ref = multivariate_normal(mean=np.zeros(zf.size), cov=C).logpdf(zf)
    assert oracle.kron1_loglik(Ls, z) == pytest.approx(ref, rel=1e-11)


# --------------------------------------------- sinc-quadrature CP, canonical-to-Tucker ----

@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_laplace_weights_reproduce_matern(oracle, nu):
    """int_0^inf omega(t) exp(-r^2 t) dt equals the half-integer Matern (Sec. 3.5's Laplace
    representation and its derivatives in the rate), by adaptive quadrature (scipy)."""
    from scipy import integrate
    ell = 0.4
    k = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell)
    for r in (0.05, 0.3, 1.0):
        f = lambda t: oracle.laplace_weight(nu, ell, t) * np.exp(-r * r * t)
        c2 = 2 * nu / ell ** 2
        val = sum(integrate.quad(f, a, b, limit=400, epsabs=0, epsrel=1e-12)[0]
                  for a, b in [(0, c2 / 40), (c2 / 40, c2), (c2, 40 * c2 / max(r * r * c2, 1e-3)), (40 * c2 / max(r * r * c2, 1e-3), np.inf)])
        assert val == pytest.approx(oracle.kernel_value(k, r), rel=1e-9), (nu, r)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_sinc_cp_converges_exponentially(oracle, nu):
    """Sec. 3.4 eq. (3.11): the sinc rule with R = 2M+1 terms converges exponentially in M away
    from the origin; at M = 40, C0 = 2 it reproduces the tensor to ~1e-9 of sigma2."""
    k = oracle.Kernel(oracle.MATERN, nu=nu, ell=0.3)
    g = oracle.Grid(n=(17, 20, 15), layout=oracle.OFFSET)
    A = oracle.grid_eval(k, g)
    mask = np.ones(A.shape, bool)
    mask[0, 0, 0] = False                         # r = 0: the rule's tail decays only like e^{-u/2}
    errs = []
    for M in (10, 20, 40):
        Q, w, t = oracle.sinc_cp(k, g, M, 2.0)
        errs.append(np.abs(oracle.cp_full(Q) - A)[mask].max())
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 2e-9, errs


def test_c2t_full_rank_is_exact(oracle):
    k = oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.5)
    g = oracle.Grid(n=(9, 11, 10), layout=oracle.CENTERED)
    Q, w, t = oracle.sinc_cp(k, g, 6, 2.0)
    Ac = oracle.cp_full(Q)
    c = oracle.c2t(Q, (9, 11, 10), sweeps=0)
    T = oracle.reconstruct(c.core, c.U)
    assert np.abs(T - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_c2t_matches_tucker_als_of_the_full_cp_tensor(oracle):
    """Canonical-to-Tucker with ALS on the canonical data reaches what Tucker-ALS on the
    materialised canonical tensor reaches (converged both), without forming that tensor;
    ||G|| grows with every mode update."""
    k = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.3)
    g = oracle.Grid(n=(33, 30, 36), layout=oracle.OFFSET)
    Q, w, t = oracle.sinc_cp(k, g, 30, 2.0)
    Ac = oracle.cp_full(Q)
    for r in (3, 6):
        c = oracle.c2t(Q, (r, r, r), sweeps=12)
        e_c2t = np.sqrt(oracle.diff_sumsq(Ac, oracle.reconstruct(c.core, c.U)) / oracle.sumsq(Ac))
        d = oracle.hooi(Ac, oracle.hosvd(Ac, (r, r, r)), sweeps=None)
        assert e_c2t == pytest.approx(d.rel_err, rel=1e-6), r
        hist = np.asarray(c.history)
        assert np.all(np.diff(hist) >= -1e-12 * hist[0])


# ------------------------------------------------------------------ seeded N(0,1) inputs ----

def _kat():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox_kat.json")
    return json.load(open(path))["vectors"]


def test_philox_known_answer_vectors(oracle):
    """Philox4x32-10 reproduces the known-answer vectors published with the generator's
    reference implementation (tests/golden/philox_kat.json)."""
    for v in _kat():
        ctr = [[int(x, 16) for x in v["counter"]]]
        key = [int(x, 16) for x in v["key"]]
        out = oracle.philox4x32_10(ctr, key)[0]
        assert ["%08x" % int(x) for x in out] == v["output"]


def test_philox_blocks_counter_layout(oracle):
    """Block c is the counter (c mod 2^32, c / 2^32, 0, 0): blocks across the 2^32 boundary
    equal the generator applied to those counters one by one."""
    c0 = (1 << 32) - 2
    w = oracle.philox_blocks((5, 9), c0, 4)
    for i in range(4):
        c = c0 + i
        assert np.array_equal(w[i], oracle.philox4x32_10([[c & 0xFFFFFFFF, c >> 32, 0, 0]], (5, 9))[0])


def test_normal_philox_is_box_muller_of_the_words(oracle):
    """z[2c]^2 + z[2c+1]^2 = -2 log(1 - u_a) and atan2(z[2c+1], z[2c]) = 2 pi u_b (mod 2 pi)
    for the block's uniforms; the values are N(0,1) (Kolmogorov-Smirnov at 1e6 draws)."""
    from scipy import stats
    z = oracle.normal_philox(1_000_000, 1711, 4).astype(np.float64)
    w = oracle.philox_blocks((1711, 4), 0, 500_000).astype(np.uint64)
    ua = (((w[:, 1] << np.uint64(32)) | w[:, 0]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    ub = (((w[:, 3] << np.uint64(32)) | w[:, 2]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r2 = z[0::2] ** 2 + z[1::2] ** 2
    assert np.allclose(r2, -2.0 * np.log(1.0 - ua), rtol=1e-6, atol=1e-6)
    ang = np.mod(np.arctan2(z[1::2], z[0::2]), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * ub)
    d = np.minimum(d, 2 * np.pi - d)
    assert np.all(d[r2 > 1e-6] < 1e-5)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5e-3 and abs(z.var() - 1.0) < 5e-3
    # an odd count drops the last sine value only
    assert np.array_equal(oracle.normal_philox(7, 1711, 4), z[:7].astype(np.float32))
