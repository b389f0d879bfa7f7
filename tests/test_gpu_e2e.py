"""End-to-end parity of tk_compress / tk_kron_matvec / tk_trace / tk_quadratic_form against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, fp64_e_tolerance, host, require_gpu, say, to_oracle_tucker, torch

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


def _recon_host(U, core):
    X = core
    X = np.einsum("ia,abc->ibc", U[0], X)
    X = np.einsum("jb,ibc->ijc", U[1], X)
    X = np.einsum("kc,ijc->ijk", U[2], X)
    return X


# --------------------------------------------------------------- FP64: the plain method ----

def test_c1_hosvd_error_curve_fp64(ctx, tk, oracle):
    """Exponential kernel, 64^3 centred grid, HOSVD at ranks 1..16: the relative Frobenius
    error per rank matches the oracle to 1e-10, or to the Gram route's FP64 floor where that is
    larger (fp64_e_tolerance); where the floor reaches E itself both only lie below 3e-8."""
    k, g, ranks = synth.c1_small()
    ok = oracle.Kernel(k.family, nu=k.nu, ell=k.ell)
    og = oracle.Grid(n=g.n, b=g.b, layout=g.layout)
    A = oracle.grid_eval(ok, og)
    f = oracle.hosvd_factors(A)
    kern = tk.make_kernel(k.family, nu=k.nu, ell=k.ell)
    grid = tk.make_grid(g.n, g.b, g.layout)
    for r in ranks:
        say("rank", r)
        t = ctx.compress(kern, grid, tk.make_opts(ranks=r, hooi_sweeps=0, prec=tk.TK_FP64))
        ref = oracle.hosvd(A, (r, r, r), f)
        lam = f[0][0]
        gap = (lam[r - 1] - lam[r]) / lam[r - 1] if r < len(lam) else 1.0
        tol = fp64_e_tolerance(A, f, r, ref.rel_err)
        say("  E_gpu %.6e E_oracle %.6e tol %.2e" % (t.rel_err, ref.rel_err, tol))
        if tol <= 1e-2 * ref.rel_err:
            assert abs(t.rel_err - ref.rel_err) <= tol, (r, t.rel_err, ref.rel_err, tol)
            U, core = t.factors()
            d = _recon_host(U, core) - oracle.reconstruct(ref.core, ref.U)
            # the r-th factor column is fixed by the FP64 Gram only to u*lambda_1/gap; it enters
            # the reconstruction weighted by sigma_r, hence u * sqrt(lambda_1/lambda_r) / gap
            tol = max(1e-10, 100 * 2.2e-16 * np.sqrt(lam[0] / lam[r - 1]) / gap)
            assert np.sqrt(np.sum(d * d) / np.sum(A * A)) <= tol, (r, tol)
        else:
            assert 0 <= t.rel_err <= 3e-8 and ref.rel_err <= 3e-8
        t.free()


@pytest.mark.parametrize("shape,ranks,sweeps", [((40, 36, 44), (3, 4, 5), 2), ((33, 65, 70), (6, 5, 7), 1),
                                                 ((36, 36, 36), (3, 5, 7), 2), ((60, 60, 60), (4, 6, 5), 1)])
def test_hooi_fp64_matches_oracle(ctx, tk, oracle, shape, ranks, sweeps):
    ok = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.25)
    og = oracle.Grid(n=shape, b=(1.0, 1.2, 0.9), layout=oracle.CENTERED)
    ref = oracle.compress(ok, og, ranks=ranks, sweeps=sweeps)
    t = ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.25), tk.make_grid(shape, (1.0, 1.2, 0.9), 0),
                     tk.make_opts(ranks=ranks, hooi_sweeps=sweeps, prec=tk.TK_FP64))
    assert t.ranks == tuple(ranks)
    assert t.rel_err == pytest.approx(ref.rel_err, rel=1e-10)
    U, core = t.factors()
    A = oracle.grid_eval(ok, og)
    d = _recon_host(U, core) - oracle.reconstruct(ref.core, ref.U)
    # the r-th column of mode k is fixed by the FP64 Gram only to u lambda_1 / gap and enters the
    # reconstruction weighted by sigma_r: tolerance max(1e-10, 100 u sqrt(lambda_1/lambda_r) / gap)
    tol = 1e-10
    for k, r in enumerate(ranks):
        M = np.moveaxis(A, k, 0).reshape(shape[k], -1)
        lam = np.sort(np.linalg.eigvalsh(M @ M.T))[::-1]
        gap = (lam[r - 1] - lam[r]) / lam[r - 1]
        tol = max(tol, 100 * 2.2e-16 * np.sqrt(lam[0] / lam[r - 1]) / gap)
    assert np.sqrt(np.sum(d * d) / np.sum(A * A)) <= tol
    # orthonormal factors, core = projection
    for u in U:
        assert np.abs(u.T @ u - np.eye(u.shape[1])).max() < 1e-12
    np.testing.assert_allclose(core, oracle.project_core(A, U), rtol=0, atol=1e-12 * np.abs(core).max())


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("n,ranks", [(48, (4, 6, 8)), (64, (7, 5, 6))])
def test_fixed_unequal_ranks_float_matches_oracle(ctx, tk, oracle, prec, n, ranks):
    """Cubic grid, unequal fixed ranks on the float paths (each mode its own eigensolve)."""
    ok = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.25)
    og = oracle.Grid(n=(n, n, n), b=(1.0, 1.2, 0.9), layout=oracle.CENTERED)
    ref = oracle.compress(ok, og, ranks=ranks, sweeps=2)
    t = ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.25), tk.make_grid(n, (1.0, 1.2, 0.9), 0),
                     tk.make_opts(ranks=ranks, hooi_sweeps=2, prec=prec))
    assert t.ranks == tuple(ranks)
    U, core = t.factors()
    A = oracle.grid_eval(ok, og)
    d = _recon_host(U, core) - oracle.reconstruct(ref.core, ref.U)
    assert np.sqrt(np.sum(d * d) / np.sum(A * A)) <= 1e-5
    assert t.rel_err == pytest.approx(ref.rel_err, rel=1e-3, abs=1e-6)


def test_full_rank_is_exact_fp64(ctx, tk, oracle):
    X = synth.random_tensor((7, 9, 8), 3)
    t = ctx.compress_tensor(dev(X), tk.make_grid((7, 9, 8)), tk.make_opts(ranks=(7, 9, 8), hooi_sweeps=0,
                                                                           prec=tk.TK_FP64))
    assert t.rel_err <= 1e-13
    U, core = t.factors()
    np.testing.assert_allclose(_recon_host(U, core), X, atol=1e-12)


def test_rank_clamped_to_n(ctx, tk):
    X = synth.random_tensor((5, 6, 7), 4)
    t = ctx.compress_tensor(dev(X), tk.make_grid((5, 6, 7)), tk.make_opts(ranks=(9, 9, 9), hooi_sweeps=0,
                                                                           prec=tk.TK_FP64))
    assert t.ranks == (5, 6, 7)
    assert t.rel_err <= 1e-13


def test_separable_gaussian_rank_one(ctx, tk):
    for prec in (tk.TK_FP64, tk.TK_FP32):
        t = ctx.compress(tk.make_kernel(2, ell=0.5), tk.make_grid((40, 50, 60)),
                         tk.make_opts(ranks=1, hooi_sweeps=1, prec=prec))
        assert t.rel_err <= (1e-12 if prec == tk.TK_FP64 else 3e-7)


def test_fp64_eps_mode_ranks_match_oracle(ctx, tk, oracle):
    ok = oracle.Kernel(oracle.MATERN, nu=0.5, ell=0.3)
    og = oracle.Grid(n=(48, 48, 48))
    for eps in (1e-3, 1e-5):
        ref = oracle.compress(ok, og, eps=eps, sweeps=2)
        t = ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.3), tk.make_grid(48),
                         tk.make_opts(eps=eps, hooi_sweeps=2, prec=tk.TK_FP64))
        assert t.ranks == ref.ranks
        assert t.rel_err == pytest.approx(ref.rel_err, rel=1e-9)
        assert t.rel_err <= eps


# -------------------------------------------------------------- FP32 / split precision ----

@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("nu,ell,layout", [(0.5, 0.1, 1), (1.5, 0.2, 0), (2.5, 1.0, 1)])
def test_eps_compress_split_precision(ctx, tk, oracle, prec, nu, ell, layout):
    n = 72
    say("eps compress", prec, nu, ell, layout)
    ok = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell)
    og = oracle.Grid(n=(n, n, n), layout=layout)
    eps = 1e-6
    ref = oracle.compress(ok, og, eps=eps, sweeps=2)
    t = ctx.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, layout),
                     tk.make_opts(eps=eps, hooi_sweeps=2, prec=prec))
    say("  gpu ranks", t.ranks, "E %.3e" % t.rel_err, "oracle", ref.ranks, "E %.3e" % ref.rel_err)
    assert t.rel_err <= eps
    assert all(a <= b + 1 for a, b in zip(t.ranks, ref.ranks))
    U, core = t.factors()
    A = oracle.grid_eval(ok, og)
    # the reported error is the measured one
    d_true = _recon_host(U, core) - A
    assert np.sqrt(np.sum(d_true ** 2) / np.sum(A ** 2)) == pytest.approx(t.rel_err, rel=2e-2, abs=2e-8)
    d = _recon_host(U, core) - oracle.reconstruct(ref.core, ref.U)
    assert np.sqrt(np.sum(d * d) / np.sum(A * A)) <= 1e-5


def test_compress_deterministic(ctx, tk):
    outs = []
    for _ in range(2):
        t = ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.3), tk.make_grid(80, 1.0, 1), tk.make_opts(eps=1e-6))
        outs.append(t.factors())
    for k in range(3):
        assert np.array_equal(outs[0][0][k], outs[1][0][k])
    assert np.array_equal(outs[0][1], outs[1][1])


# ----------------------------------------------------------------- covariance operator ----

@pytest.mark.parametrize("layout,n", [(1, (6, 7, 5)), (0, (9, 7, 11)), (1, (20, 17, 24))])
def test_matvec_fp64_exact_small(ctx, tk, oracle, layout, n):
    ok = oracle.Kernel(oracle.MATERN, nu=1.5, ell=0.5)
    og = oracle.Grid(n=n, layout=layout)
    ranks = (3, 2, 4)
    t = ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.5), tk.make_grid(n, 1.0, layout),
                     tk.make_opts(ranks=ranks, hooi_sweeps=1, prec=tk.TK_FP64))
    U, core = t.factors()
    to = to_oracle_tucker(oracle, U, core)
    off, m = oracle.cov_offsets(og)
    assert t.cov_dims() == tuple(m)
    z = synth.normal_vector(m, 5).astype(np.float64)
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    ctx.kron_matvec(t, dev(z), y, io=tk.TK_FP64)
    want = oracle.cov_matvec(to, og, z)
    np.testing.assert_allclose(host(y), want, rtol=0, atol=1e-12 * np.abs(want).max())
    # trace and quadratic form
    assert ctx.trace(t) == pytest.approx(oracle.cov_trace(to, og), rel=1e-12)
    assert ctx.trace(t) == pytest.approx(oracle.cov_trace_kron(to, og), rel=1e-12)
    q = ctx.quadratic_form(t, dev(z), io=tk.TK_FP64)
    assert q == pytest.approx(float(np.dot(z.reshape(-1), want.reshape(-1))), rel=1e-11)


def test_matvec_fp32_sampled(ctx, tk, oracle):
    n = 96
    og = oracle.Grid(n=(n, n, n), layout=oracle.OFFSET)
    t = ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.1), tk.make_grid(n, 1.0, 1), tk.make_opts(eps=1e-6))
    U, core = t.factors()
    to = to_oracle_tucker(oracle, U, core)
    z = synth.normal_vector((n, n, n), 6)
    zd = dev(z)
    y = torch.empty_like(zd)
    ctx.kron_matvec(t, zd, y, io=tk.TK_FP32)
    got = host(y).reshape(-1)
    rows = np.random.default_rng(1).choice(n ** 3, 48, replace=False)
    want = oracle.cov_matvec_rows(to, og, z.astype(np.float64), rows)
    Q = np.abs(oracle.reconstruct(to.core, to.U))
    absz = np.abs(z.astype(np.float64))
    # error bound: a few FP32 roundings of sum_j |C_ij z_j| per output
    bound = oracle.cov_rows_from_generator(Q, og, absz, rows)
    err = np.abs(got[rows] - want)
    say("fp32 matvec max err/bound %.3e" % (err / bound).max())
    assert np.all(err <= 2e-5 * bound)


def test_covariance_errors(ctx, tk):
    t = ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.3), tk.make_grid(16), tk.make_opts(ranks=3, prec=tk.TK_FP64))
    z = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(z)
    with pytest.raises(tk.TkError) as ei:
        ctx.kron_matvec(t, z, y, io=tk.TK_FP64)
    assert "TK_ELAYOUT" in str(ei.value)
    with pytest.raises(tk.TkError):
        ctx.trace(t)
    with pytest.raises(tk.TkError):
        tk.tk_kron_matvec(ctx.handle, t.handle, z, z, tk.TK_FP64)


def test_argument_errors(ctx, tk):
    with pytest.raises(tk.TkError) as ei:
        ctx.compress(tk.make_kernel(0, nu=31.0, ell=0.3), tk.make_grid(16), tk.make_opts(eps=1e-6))
    assert "TK_EUNSUPPORTED" in str(ei.value)
    for bad in (dict(ell=-1.0), dict(ell=float("nan")), dict(sigma2=0.0), dict(nu=0.0),
                dict(metric=(1.0, -1.0, 1.0)), dict(metric=(1.0, 0.0, 1.0))):
        kw = dict(family=0, nu=0.5, ell=0.3)
        kw.update(bad)
        with pytest.raises(tk.TkError) as ei:
            ctx.compress(tk.make_kernel(**kw), tk.make_grid(16), tk.make_opts(eps=1e-6))
        assert "TK_EINVAL" in str(ei.value)


def test_budget_exhaustion_is_reported(ctx, tk):
    small = tk.Context(0, hbm_budget_bytes=1 << 20)
    with pytest.raises(tk.TkError) as ei:
        small.compress(tk.make_kernel(0, nu=0.5, ell=0.3), tk.make_grid(64), tk.make_opts(eps=1e-6))
    assert "TK_ENOMEM" in str(ei.value)
    assert small.budget()[1] == 0
    small.destroy()


def test_noconv_when_rmax_too_small(ctx, tk):
    with pytest.raises(tk.TkError) as ei:
        ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.05), tk.make_grid(64), tk.make_opts(eps=1e-9, r_max=3))
    assert "TK_ENOCONV" in str(ei.value)
    t = ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.05), tk.make_grid(64), tk.make_opts(eps=1e-9, r_max=3),
                     allow_noconv=True)
    assert t.ranks == (3, 3, 3) and t.rel_err > 1e-9


def test_save_load_roundtrip(ctx, tk, tmp_path):
    t = ctx.compress(tk.make_kernel(0, nu=1.5, ell=0.3), tk.make_grid(30, 1.0, 1), tk.make_opts(ranks=4))
    p = str(tmp_path / "t.tkt")
    tk.tk_tucker_save(t.handle, p)
    h = tk.tk_tucker_load(ctx.handle, p)
    t2 = tk.Tucker(h, ctx)
    a, b = t.factors(), t2.factors()
    for k in range(3):
        assert np.array_equal(a[0][k], b[0][k])
    assert np.array_equal(a[1], b[1])
    assert t2.rel_err == t.rel_err and t2.layout == 1


# ------------------------------------------------- full size, in the benchmark's launch setup ----

@pytest.mark.parametrize("nu,ell", [(nu, ell) for nu in (0.5, 1.5, 2.5) for ell in (0.1, 0.3, 1.0)])
def test_bench_configuration_256(ctx, tk, oracle, nu, ell):
    """256^3 offset grid, eps 1e-6, 2 HOOI sweeps, FP32 -- exactly what bench.py times, all nine of
    its kernels -- on sampled outputs: error <= eps, ranks within one of the oracle's,
    reconstruction and covariance matvec rows against the FP64 oracle."""
    n, eps = 256, 1e-6
    og = oracle.Grid(n=(n, n, n), layout=oracle.OFFSET)
    ok = oracle.Kernel(oracle.MATERN, nu=nu, ell=ell)
    say("full size", nu, ell)
    stream = torch.cuda.current_stream()
    t = ctx.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, tk.TK_OFFSET),
                     tk.make_opts(eps=eps, hooi_sweeps=2, prec=tk.TK_FP32), stream)
    ref = oracle.compress(ok, og, eps=eps, sweeps=2)
    say("  gpu", t.ranks, "%.3e" % t.rel_err, "oracle", ref.ranks, "%.3e" % ref.rel_err)
    assert t.rel_err <= eps
    assert all(a <= b + 1 for a, b in zip(t.ranks, ref.ranks))
    U, core = t.factors()
    rng = np.random.default_rng(7)
    idx = rng.integers(0, n, size=(4096, 3))
    def at(Uf, G):
        return np.einsum("sa,sb,sc,abc->s", Uf[0][idx[:, 0]], Uf[1][idx[:, 1]], Uf[2][idx[:, 2]], G)
    A_s = np.array([oracle.kernel_value(ok, np.sqrt(np.sum((2.0 / (n - 1) * i) ** 2))) for i in idx])
    d = at(U, core) - at(ref.U, ref.core)
    assert np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(A_s * A_s)) <= 1e-5
    # covariance matvec through the quadratic form (as timed), sampled rows
    z = synth.normal_vector((n, n, n), 1)
    zd = dev(z)
    y = torch.empty_like(zd)
    q = ctx.quadratic_form(t, zd, io=tk.TK_FP32, stream=stream, y=y)
    got = host(y).reshape(-1)
    rows = rng.choice(n ** 3, 24, replace=False)
    to = to_oracle_tucker(oracle, U, core)
    Q = oracle.reconstruct(to.core, to.U)
    want = oracle.cov_rows_from_generator(Q, og, z.astype(np.float64), rows)
    bound = oracle.cov_rows_from_generator(np.abs(Q), og, np.abs(z.astype(np.float64)), rows)
    say("  matvec max err/bound %.3e" % (np.abs(got[rows] - want) / bound).max())
    assert np.all(np.abs(got[rows] - want) <= 2e-5 * bound)
    assert q == pytest.approx(float(np.dot(z.reshape(-1).astype(np.float64), got.astype(np.float64))), rel=1e-6)
    tr = ctx.trace(t)
    assert tr == pytest.approx(oracle.cov_trace_kron(to, og), rel=1e-12)


@pytest.mark.parametrize("layout,n", [(1, (6, 7, 5)), (0, (9, 7, 11)), (1, (20, 17, 24)), (0, (3, 5, 7)),
                                      (1, (33, 40, 64)), (1, (2, 2, 3))])
def test_matvec_fft_matches_oracle_and_dense(ctx, tk, oracle, layout, n):
    """The FFT form (circulant embedding of every Toeplitz factor, Sec. 3.6) against the plain
    product of the oracle and against the dense Toeplitz mode products."""
    og = oracle.Grid(n=n, layout=layout)
    ranks = tuple(min(4, x) for x in n)
    t = ctx.compress(tk.make_kernel(0, nu=0.5, ell=0.4), tk.make_grid(n, 1.0, layout),
                     tk.make_opts(ranks=ranks, hooi_sweeps=1, prec=tk.TK_FP64))
    U, core = t.factors()
    to = to_oracle_tucker(oracle, U, core)
    off, m = oracle.cov_offsets(og)
    z = synth.normal_vector(m, 9)
    want = oracle.cov_matvec(to, og, z.astype(np.float64)).reshape(-1)
    Q = oracle.reconstruct(to.core, to.U)
    rows = np.arange(int(np.prod(m)))
    bound = oracle.cov_rows_from_generator(np.abs(Q), og, np.abs(z.astype(np.float64)), rows)
    outs = {}
    for name, method in (("fft", tk.TK_MV_FFT), ("dense", tk.TK_MV_DENSE)):
        ctx.set_matvec_method(method)
        y = torch.empty(m, dtype=torch.float32, device="cuda")
        ctx.kron_matvec(t, dev(z), y, io=tk.TK_FP32)
        outs[name] = host(y).reshape(-1).astype(np.float64)
        say(name, "max err/bound %.3e" % (np.abs(outs[name] - want) / bound).max())
    ctx.set_matvec_method(tk.TK_MV_AUTO)
    for name in outs:
        assert np.all(np.abs(outs[name] - want) <= 2e-5 * bound), name
    # the quadratic form z^T C z (FFT path: summed in FP64 as the last pass forms C z, without
    # storing it) against the oracle's quadratic form over the same generator; the bound is
    # 2e-5 of sum_i |z_i| (|C| |z|)_i, as for the rows
    zf = z.astype(np.float64).reshape(-1)
    q_want = oracle.quadratic_form(to, og, zf)
    q_bound = float(np.dot(np.abs(zf), bound))
    for name, method in (("fft", tk.TK_MV_FFT), ("dense", tk.TK_MV_DENSE)):
        ctx.set_matvec_method(method)
        q = ctx.quadratic_form(t, dev(z), io=tk.TK_FP32)
        say(name, "quadratic form rel err %.3e" % (abs(q - q_want) / q_bound))
        assert abs(q - q_want) <= 2e-5 * q_bound, name
    ctx.set_matvec_method(tk.TK_MV_AUTO)


def test_quadratic_form_batch_matches_single(ctx, tk):
    """FFT path: the batch runs the preambles on a worker stream and the passes of the items in
    turn with shared spectrum buffers; dense path: items concurrently on the worker streams.
    Every value (and y, when given) is bitwise the single call's, and a single call without y
    (C z never stored) gives the same value as with it."""
    opts = tk.make_opts(eps=1e-6, hooi_sweeps=2, prec=1)
    ts = [ctx.compress(tk.make_kernel(0, nu=nu, ell=ell), tk.make_grid(n, 1.0, lay), opts)
          for (n, nu, ell, lay) in [(64, 0.5, 0.2, 1), (96, 1.5, 0.3, 1), (65, 2.5, 0.5, 0), (64, 1.5, 1.0, 1)]]
    zs = [dev(synth.normal_vector(t.cov_dims(), 40 + i)) for i, t in enumerate(ts)]
    single, ys_single = [], []
    for t, z in zip(ts, zs):
        y = torch.empty_like(z)
        single.append(ctx.quadratic_form(t, z, y=y))
        ys_single.append(host(y))
    for workers in (4, 2):
        ctx.set_workers(workers)
        assert ctx.quadratic_form_batch(ts, zs) == single
        ys = [torch.empty_like(z) for z in zs]
        assert ctx.quadratic_form_batch(ts, zs, ys=ys) == single
        assert all(np.array_equal(host(y), ya) for y, ya in zip(ys, ys_single))
    ctx.set_workers(4)
    assert [ctx.quadratic_form(t, z) for t, z in zip(ts, zs)] == single
    # mixed shapes in a different order: the shared buffers are sized for the largest item
    order = [3, 1, 0, 2]
    assert ctx.quadratic_form_batch([ts[i] for i in order], [zs[i] for i in order]) == [single[i] for i in order]
    ctx.set_matvec_method(tk.TK_MV_DENSE)
    try:
        dense = [ctx.quadratic_form(t, z) for t, z in zip(ts[:2], zs[:2])]
        assert ctx.quadratic_form_batch(ts[:2], zs[:2]) == dense
    finally:
        ctx.set_matvec_method(tk.TK_MV_AUTO)
    for t in ts:
        t.free()
