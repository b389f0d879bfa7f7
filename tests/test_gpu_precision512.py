"""The precision study at full size: Matern nu = 3/2, ell = 0.2 on the 512^3 centred grid of
[-1, 1]^3, eps in {1e-4, 1e-6}, Gram contractions in FP64, FP32 and split BF16x3, each against
the FP64 oracle's compression of the same tensor (tests/golden/c3_512.npz, written by
tests/golden/make_c3_512.py: eps-rule HOSVD plus two Tucker-ALS sweeps, Sec. 3.2).  Checked:
E <= eps, orthonormal factors, ||A||^2 = ||G||^2 + ||A - A_r||^2, sampled tensor entries
(evaluated one by one by the oracle), ranks against the oracle's, and the reconstruction, core
and energy-weighted factor errors against the oracle's result."""
import numpy as np
import pytest

import synth
from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


@pytest.fixture(scope="module")
def study_results(tk, oracle):
    require_gpu()
    ks, gs, eps_list = synth.c3(512)
    n = gs.n[0]
    ctx = tk.Context(0)
    kernel = tk.make_kernel(ks.family, nu=ks.nu, ell=ks.ell)
    grid = tk.make_grid(n, 1.0, tk.TK_CENTERED)
    out = {}
    try:
        for eps in eps_list:
            for prec in (tk.TK_FP64, tk.TK_FP32, tk.TK_BF16X3):
                say("512^3 compress eps", eps, "prec", prec)
                t = ctx.compress(kernel, grid, tk.make_opts(eps=eps, hooi_sweeps=2, prec=prec))
                U, core = t.factors()
                out[(eps, prec)] = (t.ranks, t.rel_err, t.norm_a, U, core)
                say("  ranks", t.ranks, "E %.3e" % t.rel_err)
                t.free()
    finally:
        ctx.destroy()
    ok = oracle.Kernel(oracle.MATERN, nu=ks.nu, ell=ks.ell)
    rng = np.random.default_rng(512)
    idx = rng.integers(0, n, size=(4096, 3))
    x = oracle.grid_coords(n, 1.0, oracle.CENTERED)
    A_s = np.array([oracle.kernel_value(ok, float(np.sqrt(x[i] ** 2 + x[j] ** 2 + x[k] ** 2))) for i, j, k in idx])
    return out, idx, A_s, eps_list


def _hosvd_basis(U, G):
    """Rotate (U, G) to the HOSVD basis of G (eigenvectors of each core unfolding's Gram,
    descending) and sign every factor column so that its entry of largest magnitude is positive,
    negating the matching core slice."""
    U = [u.copy() for u in U]
    G = G.copy()
    for k in range(3):
        Gk = np.moveaxis(G, k, 0).reshape(G.shape[k], -1)
        lam, V = np.linalg.eigh(Gk @ Gk.T)
        V = V[:, ::-1]
        U[k] = U[k] @ V
        G = np.moveaxis(np.tensordot(V.T, np.moveaxis(G, k, 0), axes=1), 0, k)
        lead = np.argmax(np.abs(U[k]), axis=0)
        s = np.sign(U[k][lead, np.arange(U[k].shape[1])])
        s[s == 0] = 1.0
        U[k] = U[k] * s
        G = np.moveaxis(np.moveaxis(G, k, 0) * s[:, None, None], 0, k)
    return U, G


def _at(U, core, idx):
    return np.einsum("sa,sb,sc,abc->s", U[0][idx[:, 0]], U[1][idx[:, 1]], U[2][idx[:, 2]], core)


@pytest.mark.parametrize("eps_i", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_precision512_error_and_invariants(tk, study_results, eps_i, prec):
    out, idx, A_s, eps_list = study_results
    eps = eps_list[eps_i]
    ranks, E, norm_a, U, core = out[(eps, prec)]
    assert E <= eps
    for k in range(3):
        assert np.abs(U[k].T @ U[k] - np.eye(ranks[k])).max() <= 1e-12
    # Pythagoras for orthonormal factors: ||A||^2 = ||G||^2 + (E ||A||)^2
    g2 = float(np.sum(core ** 2))
    assert g2 + (E * norm_a) ** 2 == pytest.approx(norm_a ** 2, rel=1e-7)
    # sampled reconstruction against the tensor entries the oracle computes one by one: the
    # mean squared sample error estimates E^2 (factor 4 of slack for sampling)
    d = _at(U, core, idx) - A_s
    rms_rel = np.sqrt(np.mean(d * d) / np.mean(A_s * A_s))
    say("eps", eps, "prec", prec, "ranks", ranks, "E %.3e" % E, "sampled %.3e" % rms_rel)
    assert rms_rel <= 4.0 * max(E, 1e-12) + 1e-12


def _golden():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_512.npz")
    return np.load(path, allow_pickle=False)


def _recon_diff(U, G, Uo, Go):
    """||A_r - A_o|| for two Tucker tensors without forming either: with Q_k R_k the QR of
    [U_k, U_o,k], A_r - A_o = (G x_k R_k[:, :r_k] - G_o x_k R_k[:, r_k:]) x_k Q_k and Q_k has
    orthonormal columns, so the norm is that of the small (2r)^3 difference (no cancellation
    between ||A_r||^2 and ||A_o||^2)."""
    X, Y = G, Go
    for k in range(3):
        Q, R = np.linalg.qr(np.hstack([U[k], Uo[k]]))
        r = U[k].shape[1]
        X = np.moveaxis(np.tensordot(R[:, :r], np.moveaxis(X, k, 0), axes=([1], [0])), 0, k)
        Y = np.moveaxis(np.tensordot(R[:, r:], np.moveaxis(Y, k, 0), axes=([1], [0])), 0, k)
    return float(np.linalg.norm(X - Y))


@pytest.mark.parametrize("eps_i", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_precision512_against_oracle(tk, study_results, eps_i, prec):
    """Every precision against the FP64 oracle at 512^3: ranks equal (FP64: same eps rule on
    the same spectrum) or within one (float paths: the rule on the truncated core), the
    reconstruction within 1e-5 of the oracle's relative to ||A|| (FP64: 1e-8 on the sampled
    nodes; the float paths from the exact small-product form), and, where the ranks agree, the
    sign-aligned core and the energy-weighted factor errors in the basis of each core's HOSVD."""
    out, idx, A_s, eps_list = study_results
    gold = _golden()
    eps = eps_list[eps_i]
    assert float(gold["eps"][eps_i]) == eps
    ro = tuple(int(x) for x in gold["ranks%d" % eps_i])
    Eo = float(gold["rel_err%d" % eps_i])
    Go = gold["core%d" % eps_i]
    Uo = [gold["U%d_%d" % (eps_i, k)] for k in range(3)]
    na = float(np.sqrt(gold["norm_a2"]))
    r, E, norm_a, U, G = out[(eps, prec)]
    msg = ["eps %g prec %d: ranks %s (oracle %s), E %.4e (oracle %.4e)" % (eps, prec, r, ro, E, Eo)]
    assert norm_a == pytest.approx(na, rel=1e-6)
    if prec == 0:
        assert tuple(r) == ro
        d = _at(U, G, idx) - _at(Uo, Go, idx)
        rec = np.sqrt(np.mean(d * d) / np.mean(A_s * A_s))
        msg.append("reconstruction (sampled) %.2e" % rec)
        assert rec <= 1e-8
    else:
        assert all(a <= b + 1 for a, b in zip(r, ro))
        rec = _recon_diff(U, G, Uo, Go) / na
        msg.append("reconstruction %.2e (|E - E_o| %.2e)" % (rec, abs(E - Eo)))
        assert rec <= 1e-5
    if tuple(r) == ro:
        Ua, Ga = _hosvd_basis(U, G)
        Ub, Gb = _hosvd_basis(Uo, Go)
        core_err = float(np.linalg.norm(Ga - Gb) / np.linalg.norm(Gb))
        fac = []
        for k in range(3):
            w = np.sum(np.moveaxis(Gb, k, 0).reshape(r[k], -1) ** 2, axis=1)   # sigma_a^2
            fac.append(float(np.sum(w * np.sum((Ua[k] - Ub[k]) ** 2, axis=0)) / np.sum(w)))
        msg.append("core %.2e, factors (energy-weighted) %s" % (core_err, ["%.1e" % v for v in fac]))
        assert core_err <= (1e-8 if prec == 0 else 1e-3)
        assert max(fac) <= (1e-14 if prec == 0 else 1e-6)
    say(*msg)
