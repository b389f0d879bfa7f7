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


def fp64_e_tolerance(lams, r, e, na2, n):
    """Parity tolerance of an FP64 HOSVD/HOOI error E against the oracle: 1e-10 E, or the
    Gram route's floor if larger.  Both eigensolvers are backward stable (exact for a Gram
    perturbed by about n u ||G||); E is stationary in the factors at the exact eigenvectors, so
    the perturbation moves it at second order, by about
    (n u lambda_1)^2 / ((lambda_r - lambda_{r+1}) E ||A||^2) per mode."""
    floor = 0.0
    for lam in lams:
        gap = lam[r - 1] - lam[r] if r < len(lam) else lam[r - 1]
        floor += (n * U64 * lam[0]) ** 2 / (max(gap, 1e-300) * max(e, 1e-300) * na2)
    return max(1e-10 * e, floor)
