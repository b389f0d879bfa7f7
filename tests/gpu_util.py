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
