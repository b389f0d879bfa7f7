"""Shared helpers for the GPU parity tests (device buffers via torch, oracle conversions)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def dev(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_kernel(o, fam, **kw):
    return o.Kernel(family=fam, **kw)


def to_oracle_tucker(o, U, core, norm_a2=0.0):
    return o.Tucker(U=[np.asarray(u, dtype=np.float64) for u in U], core=np.asarray(core, dtype=np.float64),
                    norm_a2=norm_a2)


def sign_align(V, ref):
    """Flip columns of V to best match ref (for comparisons that must ignore the gauge)."""
    V = V.copy()
    for j in range(V.shape[1]):
        if np.dot(V[:, j], ref[:, j]) < 0:
            V[:, j] = -V[:, j]
    return V


def say(*args):
    print(*args, flush=True)


U64 = 2.0 ** -53


def _tucker_err(A, Us):
    """||A - A x_k U_k U_k^T|| / ||A|| by explicit reconstruction (orthonormal U_k)."""
    C = np.einsum("ijk,ia,jb,kc->abc", A, *Us, optimize=True)
    Ah = np.einsum("abc,ia,jb,kc->ijk", C, *Us, optimize=True)
    return float(np.sqrt(np.sum((A - Ah) ** 2) / np.sum(A * A)))


def fp64_e_tolerance(A, f, r, e):
    """Parity tolerance of an FP64 HOSVD error E against the oracle: 1e-10 E, or the Gram
    route's floor where that is larger.

    Two correct FP64 implementations form the mode Grams with different rounding; each
    eigenvector u_j of G_k is then fixed only up to a rotation toward u_i by about
    theta = 4 u lambda_1 / |lambda_j - lambda_i| (u the unit roundoff; a factor 4 for the two
    Grams and the two eigensolvers).  HOSVD factors are not a stationary point of E (the leading
    subspaces of A_(k) A_(k)^T are not those of the single-hole Grams that would make them one),
    so E moves at first order under such rotations.  The floor adds, over the kept columns j in
    [r-4, r) and the discarded directions i in [r, r+4) of every mode (the nearest pairs: theta
    falls like 1/gap), |dE/dtheta| theta (central differences on the oracle's own factors), or,
    for angles of 1e-4 and more, where the first-order term no longer describes the change, the
    larger change of E under the rotation by +theta or -theta itself (theta capped at pi/4).
    f holds the oracle's full eigendecompositions (lambda_k, V_k)."""
    if np.isscalar(r):
        r = (int(r),) * 3
    lams = [np.asarray(x[0]) for x in f]
    Vs = [np.asarray(x[1]) for x in f]
    base = [Vs[k][:, :r[k]] for k in range(3)]
    e0 = _tucker_err(A, base)
    floor = 0.0
    for k in range(3):
        n, lam = Vs[k].shape[0], lams[k]
        for j in range(max(0, r[k] - 4), r[k]):
            for i in range(r[k], min(r[k] + 4, n)):
                gap = lam[j] - lam[i]
                theta = 4.0 * U64 * lam[0] / gap if gap > 0 else np.inf
                step = 1e-6 if theta < 1e-4 else min(theta, np.pi / 4)
                es = []
                for sgn in (1.0, -1.0):
                    Us = [b.copy() for b in base]
                    Us[k][:, j] = np.cos(step) * Vs[k][:, j] + sgn * np.sin(step) * Vs[k][:, i]
                    es.append(_tucker_err(A, Us))
                if theta < 1e-4:
                    floor += abs(es[0] - es[1]) / (2 * step) * theta
                else:
                    floor += max(abs(es[0] - e0), abs(es[1] - e0))
    return max(1e-10 * e, floor)
