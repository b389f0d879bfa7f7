"""ctypes binding of libtk.so (the C ABI in include/tk.h).

Argument marshalling only: every step runs in the HIP library.  Device buffers are passed as
raw pointers (for example ``tensor.data_ptr()`` of a torch.cuda tensor) and streams as
``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``).  Importing this module
fails loudly when the library has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1711_06874_amd.build` "
                      "(the GPU path has no fallback)")

_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------------------- constants
TK_OK, TK_EINVAL, TK_EUNSUPPORTED, TK_ELAYOUT, TK_ENOMEM, TK_EHIP, TK_ENOCONV = 0, -1, -2, -3, -4, -5, -6
TK_MATERN, TK_SLATER, TK_GAUSS, TK_SPECTRAL = 0, 1, 2, 3
TK_CENTERED, TK_OFFSET = 0, 1
TK_FP64, TK_FP32, TK_BF16X3 = 0, 1, 2
TK_HOOI_CONVERGE = -2   # tk_opts.hooi_sweeps: Tucker-ALS until the core norm stops changing


class tk_kernel(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("nu", ctypes.c_double), ("ell", ctypes.c_double),
                ("sigma2", ctypes.c_double), ("alpha", ctypes.c_double), ("p", ctypes.c_double),
                ("metric", ctypes.c_double * 3)]


class tk_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("b", ctypes.c_double * 3), ("layout", ctypes.c_int)]


class tk_opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("ranks", ctypes.c_int * 3), ("r_max", ctypes.c_int),
                ("hooi_sweeps", ctypes.c_int), ("prec", ctypes.c_int)]


TK_REQ_COMPRESS, TK_REQ_MATVEC, TK_REQ_TRACE, TK_REQ_QUADFORM = 0, 1, 2, 3


class tk_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("kernel", tk_kernel), ("grid", tk_grid), ("opts", tk_opts),
                ("target", ctypes.c_longlong), ("z_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p),
                ("io", ctypes.c_int), ("stream", ctypes.c_void_p)]


class tk_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("kind", ctypes.c_int), ("ranks", ctypes.c_int * 3),
                ("rel_err", ctypes.c_double), ("value", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("error", ctypes.c_char * 192)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_st = ctypes.c_int

_SIGS = {
    "tk_ctx_create": (_st, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "tk_ctx_destroy": (None, [_vp]),
    "tk_ctx_budget": (_st, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "tk_estimate_bytes": (_st, [ctypes.POINTER(tk_grid), ctypes.POINTER(tk_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "tk_compress": (_st, [_vp, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid), ctypes.POINTER(tk_opts), _vp,
                          ctypes.POINTER(_vp)]),
    "tk_compress_tensor": (_st, [_vp, _vp, ctypes.POINTER(tk_grid), ctypes.POINTER(tk_opts), _vp,
                                 ctypes.POINTER(_vp)]),
    "tk_compress_multigrid": (_st, [_vp, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid), ctypes.c_int,
                                    ctypes.POINTER(tk_opts), _vp, ctypes.POINTER(_vp)]),
    "tk_compress_sinc": (_st, [_vp, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid), ctypes.c_int,
                               ctypes.c_double, _ip, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "tk_compress_group": (_st, [_vp, ctypes.c_int, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid),
                                ctypes.POINTER(tk_opts), _vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int)]),
    "tk_compress_batch": (_st, [_vp, ctypes.c_int, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid),
                                ctypes.POINTER(tk_opts), _vp, ctypes.POINTER(_vp)]),
    "tk_tucker_info": (_st, [_vp, _ip, _ip, _dp, _dp, _ip]),
    "tk_tucker_get": (_st, [_vp, ctypes.POINTER(_dp), _dp]),
    "tk_tucker_device": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "tk_reconstruct": (_st, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "tk_tucker_save": (_st, [_vp, ctypes.c_char_p]),
    "tk_tucker_load": (_st, [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "tk_tucker_free": (None, [_vp]),
    "tk_cov_dims": (_st, [_vp, _ip]),
    "tk_kron_matvec": (_st, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "tk_kron_matvec_noalloc": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "tk_trace": (_st, [_vp, _vp, _vp, _dp]),
    "tk_quadratic_form": (_st, [_vp, _vp, _vp, ctypes.c_int, _vp, _dp, _vp]),
    "tk_normal_fill": (_st, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, ctypes.c_size_t, _vp]),
    "tk_philox4x32": (_st, [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64, ctypes.c_size_t, _vp, _vp]),
    "tk_grid_eval": (_st, [_vp, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid), ctypes.c_int, _vp, _vp]),
    "tk_gram": (_st, [_vp, _vp, _ip, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "tk_eig_topr": (_st, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tk_set_matvec_method": (_st, [_vp, ctypes.c_int]),
    "tk_autotune": (_st, [_vp, ctypes.POINTER(tk_grid), ctypes.c_int, _vp, _ip, _dp]),
    "tk_autotune_save": (_st, [_vp, ctypes.c_char_p]),
    "tk_autotune_load": (_st, [_vp, ctypes.c_char_p]),
    "tk_ctx_release_stream": (_st, [_vp, _vp]),
    "tk_ctx_set_workers": (_st, [_vp, ctypes.c_int]),
    "tk_ctx_set_graphs": (_st, [_vp, ctypes.c_int]),
    "tk_ctx_set_cholqr": (_st, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "tk_quadratic_form_batch": (_st, [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, _vp,
                                      _dp, ctypes.POINTER(_vp)]),
    "tk_estimate_matvec_bytes": (_st, [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "tk_server_create": (_st, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    "tk_server_set_batching": (_st, [_vp, ctypes.c_int]),
    "tk_server_submit": (_st, [_vp, ctypes.POINTER(tk_request), ctypes.POINTER(ctypes.c_longlong)]),
    "tk_server_wait": (_st, [_vp, ctypes.c_longlong, ctypes.POINTER(tk_result)]),
    "tk_server_tucker": (_st, [_vp, ctypes.c_longlong, ctypes.POINTER(_vp)]),
    "tk_server_release": (_st, [_vp, ctypes.c_longlong]),
    "tk_server_destroy": (None, [_vp]),
    "tk_profile_enable": (_st, [ctypes.c_int]),
    "tk_profile_select": (_st, [ctypes.c_uint]),
    "tk_profile_reset": (_st, []),
    "tk_profile_read": (_st, [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), _dp]),
    "tk_kron1_create": (_st, [_vp, ctypes.POINTER(tk_kernel), ctypes.POINTER(tk_grid), _dp, _vp, ctypes.POINTER(_vp)]),
    "tk_kron1_logdet": (_st, [_vp, _dp, _dp]),
    "tk_kron1_factor": (_st, [_vp, ctypes.c_int, _vp]),
    "tk_kron1_apply": (_st, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp]),
    "tk_kron1_loglik": (_st, [_vp, _vp, _vp, _vp, _dp, _dp]),
    "tk_kron1_free": (None, [_vp]),
    "tk_last_error": (ctypes.c_char_p, []),
    "tk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tk_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class TkError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.tk_last_error().decode()
        super().__init__(f"{where}: {_lib.tk_strerror(status).decode()} ({msg})")


def _check(status: int, where: str, allow=()):
    if status != TK_OK and status not in allow:
        raise TkError(status, where)
    return status


def _check_result(status: int, out, where: str, allow_noconv: bool):
    """A call that returns TK_ENOCONV still hands over a live result through `out`: free it
    before raising, so an eps miss holds no device memory or budget."""
    if status == TK_ENOCONV and not allow_noconv and out.value:
        err = TkError(status, where)
        _lib.tk_tucker_free(out.value)
        out.value = None
        raise err
    _check(status, where, allow=(TK_ENOCONV,) if allow_noconv else ())


def make_kernel(family=TK_MATERN, nu=0.5, ell=1.0, sigma2=1.0, alpha=1.0, p=1.0, metric=None) -> tk_kernel:
    m = (ctypes.c_double * 3)(*([0.0, 0.0, 0.0] if metric is None else [float(a) for a in metric]))
    return tk_kernel(int(family), float(nu), float(ell), float(sigma2), float(alpha), float(p), m)


def make_grid(n, b=(1.0, 1.0, 1.0), layout=TK_CENTERED) -> tk_grid:
    if np.isscalar(n):
        n = (int(n),) * 3
    if np.isscalar(b):
        b = (float(b),) * 3
    return tk_grid((ctypes.c_int * 3)(*[int(x) for x in n]), (ctypes.c_double * 3)(*[float(x) for x in b]),
                   int(layout))


def make_opts(eps=0.0, ranks=(0, 0, 0), r_max=0, hooi_sweeps=-1, prec=TK_FP32) -> tk_opts:
    if np.isscalar(ranks):
        ranks = (int(ranks),) * 3
    return tk_opts(float(eps), (ctypes.c_int * 3)(*[int(x) for x in ranks]), int(r_max), int(hooi_sweeps),
                   int(prec))


def _stream(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


# ------------------------------------------------------------------------ raw entry points
def tk_version() -> str:
    return _lib.tk_version().decode()


def tk_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = _vp()
    _check(_lib.tk_ctx_create(int(device), int(hbm_budget_bytes), ctypes.byref(out)), "tk_ctx_create")
    return out.value


def tk_ctx_destroy(ctx: int) -> None:
    _lib.tk_ctx_destroy(ctx)


def tk_ctx_budget(ctx: int):
    b, u = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.tk_ctx_budget(ctx, ctypes.byref(b), ctypes.byref(u)), "tk_ctx_budget")
    return b.value, u.value


def tk_estimate_bytes(grid: tk_grid, opts: tk_opts) -> int:
    out = ctypes.c_size_t()
    _check(_lib.tk_estimate_bytes(ctypes.byref(grid), ctypes.byref(opts), ctypes.byref(out)), "tk_estimate_bytes")
    return out.value


def tk_compress(ctx: int, kernel: tk_kernel, grid: tk_grid, opts: tk_opts, stream=None, allow_noconv=False):
    out = _vp()
    st = _lib.tk_compress(ctx, ctypes.byref(kernel), ctypes.byref(grid), ctypes.byref(opts), _stream(stream),
                          ctypes.byref(out))
    _check_result(st, out, "tk_compress", allow_noconv)
    return out.value


def tk_compress_tensor(ctx: int, A, grid: tk_grid, opts: tk_opts, stream=None, allow_noconv=False):
    out = _vp()
    st = _lib.tk_compress_tensor(ctx, _ptr(A), ctypes.byref(grid), ctypes.byref(opts), _stream(stream),
                                 ctypes.byref(out))
    _check_result(st, out, "tk_compress_tensor", allow_noconv)
    return out.value


def tk_compress_sinc(ctx: int, kernel: tk_kernel, grid: tk_grid, M: int, C0: float, ranks, sweeps: int = 0,
                     stream=None, allow_noconv=False):
    out = _vp()
    rk = (ctypes.c_int * 3)(*([int(ranks)] * 3 if isinstance(ranks, int) else [int(x) for x in ranks]))
    st = _lib.tk_compress_sinc(ctx, ctypes.byref(kernel), ctypes.byref(grid), int(M), float(C0), rk, int(sweeps),
                               _stream(stream), ctypes.byref(out))
    _check_result(st, out, "tk_compress_sinc", allow_noconv)
    return out.value


def tk_compress_multigrid(ctx: int, kernel: tk_kernel, grid: tk_grid, levels: int, opts: tk_opts, stream=None,
                          allow_noconv=False):
    out = _vp()
    st = _lib.tk_compress_multigrid(ctx, ctypes.byref(kernel), ctypes.byref(grid), int(levels), ctypes.byref(opts),
                                    _stream(stream), ctypes.byref(out))
    _check_result(st, out, "tk_compress_multigrid", allow_noconv)
    return out.value


def tk_estimate_matvec_bytes(ctx: int, t: int, io: int = TK_FP32) -> int:
    out = ctypes.c_size_t()
    _check(_lib.tk_estimate_matvec_bytes(ctx, t, int(io), ctypes.byref(out)), "tk_estimate_matvec_bytes")
    return out.value


def tk_compress_batch(ctx: int, kernels, grids, opts: tk_opts, stream=None):
    n = len(kernels)
    ks = (tk_kernel * n)(*kernels)
    gs = (tk_grid * n)(*grids)
    outs = (_vp * n)()
    _check(_lib.tk_compress_batch(ctx, n, ks, gs, ctypes.byref(opts), _stream(stream), outs), "tk_compress_batch")
    return [o for o in outs]


def tk_compress_group(ctx: int, kernels, grid: tk_grid, opts: tk_opts, stream=None):
    """Returns [(handle, status)] for problems sharing `grid` (status TK_OK or TK_ENOCONV)."""
    n = len(kernels)
    ks = (tk_kernel * n)(*kernels)
    outs = (_vp * n)()
    sts = (ctypes.c_int * n)()
    _check(_lib.tk_compress_group(ctx, n, ks, ctypes.byref(grid), ctypes.byref(opts), _stream(stream), outs, sts),
           "tk_compress_group")
    return [(o, s) for o, s in zip(outs, sts)]


def tk_tucker_info(t: int):
    n = (ctypes.c_int * 3)()
    r = (ctypes.c_int * 3)()
    e, na = ctypes.c_double(), ctypes.c_double()
    lay = ctypes.c_int()
    _check(_lib.tk_tucker_info(t, n, r, ctypes.byref(e), ctypes.byref(na), ctypes.byref(lay)), "tk_tucker_info")
    return dict(n=tuple(n), ranks=tuple(r), rel_err=e.value, norm_a=na.value, layout=lay.value)


def tk_tucker_get(t: int):
    info = tk_tucker_info(t)
    n, r = info["n"], info["ranks"]
    U = [np.empty((n[k], r[k]), dtype=np.float64) for k in range(3)]
    core = np.empty(r, dtype=np.float64)
    ptrs = (_dp * 3)(*[u.ctypes.data_as(_dp) for u in U])
    _check(_lib.tk_tucker_get(t, ptrs, core.ctypes.data_as(_dp)), "tk_tucker_get")
    return U, core


def tk_tucker_device(t: int):
    U = (_vp * 3)()
    c = _vp()
    _check(_lib.tk_tucker_device(t, U, ctypes.byref(c)), "tk_tucker_device")
    return [u for u in U], c.value


def tk_reconstruct(ctx: int, t: int, A, io=TK_FP64, stream=None) -> None:
    _check(_lib.tk_reconstruct(ctx, t, _ptr(A), int(io), _stream(stream)), "tk_reconstruct")


def tk_tucker_save(t: int, path: str) -> None:
    _check(_lib.tk_tucker_save(t, path.encode()), "tk_tucker_save")


def tk_tucker_load(ctx: int, path: str) -> int:
    out = _vp()
    _check(_lib.tk_tucker_load(ctx, path.encode(), ctypes.byref(out)), "tk_tucker_load")
    return out.value


def tk_tucker_free(t: int) -> None:
    if t:
        _lib.tk_tucker_free(t)


def tk_cov_dims(t: int):
    m = (ctypes.c_int * 3)()
    _check(_lib.tk_cov_dims(t, m), "tk_cov_dims")
    return tuple(m)


def tk_kron_matvec(ctx: int, t: int, z, y, io=TK_FP32, stream=None) -> None:
    _check(_lib.tk_kron_matvec(ctx, t, _ptr(z), _ptr(y), int(io), _stream(stream)), "tk_kron_matvec")


def tk_kron_matvec_noalloc(ctx: int, t: int, z, y, stream=None) -> None:
    _check(_lib.tk_kron_matvec_noalloc(ctx, t, _ptr(z), _ptr(y), _stream(stream)), "tk_kron_matvec_noalloc")


def tk_trace(ctx: int, t: int, stream=None) -> float:
    out = ctypes.c_double()
    _check(_lib.tk_trace(ctx, t, _stream(stream), ctypes.byref(out)), "tk_trace")
    return out.value


def tk_quadratic_form(ctx: int, t: int, z, io=TK_FP32, stream=None, y=None) -> float:
    out = ctypes.c_double()
    _check(_lib.tk_quadratic_form(ctx, t, _ptr(z), int(io), _stream(stream), ctypes.byref(out), _ptr(y)),
           "tk_quadratic_form")
    return out.value


def tk_quadratic_form_batch(ctx: int, ts, zs, io=TK_FP32, stream=None, ys=None):
    n = len(ts)
    th = (_vp * n)(*[int(t) for t in ts])
    zp = (_vp * n)(*[_ptr(z) for z in zs])
    yp = (_vp * n)(*[_ptr(y) if y is not None else None for y in ys]) if ys is not None else None
    out = (ctypes.c_double * n)()
    _check(_lib.tk_quadratic_form_batch(ctx, n, th, zp, int(io), _stream(stream), out, yp), "tk_quadratic_form_batch")
    return list(out)


def tk_normal_fill(ctx: int, seed: int, stream_id: int, z, stream=None) -> None:
    """z (a float32 device tensor) <- seeded N(0,1) values (Philox4x32-10 + Box-Muller)."""
    _check(_lib.tk_normal_fill(ctx, int(seed) & 0xffffffff, int(stream_id) & 0xffffffff, _ptr(z), int(z.numel()),
                               _stream(stream)), "tk_normal_fill")


def tk_philox4x32(ctx: int, key, counter0: int, out, stream=None) -> None:
    """out (an int32/uint32 device tensor of 4 n words) <- Philox4x32-10 of counters
    counter0 .. counter0 + n - 1 under key (two 32-bit words)."""
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    _check(_lib.tk_philox4x32(ctx, k, int(counter0), int(out.numel()) // 4, _ptr(out), _stream(stream)),
           "tk_philox4x32")


def tk_grid_eval(ctx: int, kernel: tk_kernel, grid: tk_grid, prec: int, A, stream=None) -> None:
    _check(_lib.tk_grid_eval(ctx, ctypes.byref(kernel), ctypes.byref(grid), int(prec), _ptr(A), _stream(stream)),
           "tk_grid_eval")


def tk_gram(ctx: int, A, n, mode: int, prec: int, G, stream=None) -> None:
    nn = (ctypes.c_int * 3)(*[int(x) for x in n])
    _check(_lib.tk_gram(ctx, _ptr(A), nn, int(mode), int(prec), _ptr(G), _stream(stream)), "tk_gram")


def tk_eig_topr(ctx: int, count: int, n: int, r: int, G, lam, U, stream=None) -> None:
    _check(_lib.tk_eig_topr(ctx, int(count), int(n), int(r), _ptr(G), _ptr(lam), _ptr(U), _stream(stream)),
           "tk_eig_topr")


PROF_CLASSES = {"grid": 0, "gram": 1, "eig": 2, "ttm": 3, "norm": 4, "toep_right": 5, "toep_left": 6,
                "small": 7, "fft": 8, "fft_axis0": 9}
TK_MV_AUTO, TK_MV_FFT, TK_MV_DENSE = 0, 1, 2


def tk_set_matvec_method(ctx: int, method: int) -> None:
    _check(_lib.tk_set_matvec_method(ctx, int(method)), "tk_set_matvec_method")


def tk_profile_enable(on: bool = True) -> None:
    _check(_lib.tk_profile_enable(1 if on else 0), "tk_profile_enable")


def tk_profile_select(classes=None) -> None:
    """Bracket only the launches of the given classes (names of PROF_CLASSES); None: all."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << PROF_CLASSES[c] for c in classes)
    _check(_lib.tk_profile_select(mask), "tk_profile_select")


def tk_profile_reset() -> None:
    _check(_lib.tk_profile_reset(), "tk_profile_reset")


def tk_profile_read(cls: int):
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    _check(_lib.tk_profile_read(int(cls), ctypes.byref(n), ctypes.byref(ms)), "tk_profile_read")
    return n.value, ms.value


def tk_strerror(status: int) -> str:
    return _lib.tk_strerror(int(status)).decode()


def tk_last_error() -> str:
    return _lib.tk_last_error().decode()


# ------------------------------------------------------------------- convenience wrappers
class Tucker:
    """Owns one tk_tucker handle; frees it when garbage-collected."""

    def __init__(self, handle: int, ctx: "Context"):
        self.handle = handle
        self.ctx = ctx
        info = tk_tucker_info(handle)
        self.n, self.ranks, self.rel_err, self.norm_a, self.layout = (
            info["n"], info["ranks"], info["rel_err"], info["norm_a"], info["layout"])

    def factors(self):
        return tk_tucker_get(self.handle)

    def cov_dims(self):
        return tk_cov_dims(self.handle)

    def free(self):
        if self.handle:
            tk_tucker_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.handle = tk_ctx_create(device, hbm_budget_bytes)

    def compress(self, kernel, grid, opts, stream=None, allow_noconv=False) -> Tucker:
        return Tucker(tk_compress(self.handle, kernel, grid, opts, stream, allow_noconv), self)

    def compress_multigrid(self, kernel, grid, levels, opts, stream=None, allow_noconv=False) -> Tucker:
        return Tucker(tk_compress_multigrid(self.handle, kernel, grid, levels, opts, stream, allow_noconv), self)

    def compress_sinc(self, kernel, grid, M, C0, ranks, sweeps=0, stream=None, allow_noconv=False) -> Tucker:
        return Tucker(tk_compress_sinc(self.handle, kernel, grid, M, C0, ranks, sweeps, stream, allow_noconv), self)

    def compress_tensor(self, A, grid, opts, stream=None, allow_noconv=False) -> Tucker:
        return Tucker(tk_compress_tensor(self.handle, A, grid, opts, stream, allow_noconv), self)

    def compress_group(self, kernels, grid, opts, stream=None):
        return [Tucker(h, self) for h, _ in tk_compress_group(self.handle, kernels, grid, opts, stream)]

    def compress_batch(self, kernels, grids, opts, stream=None):
        return [Tucker(h, self) for h in tk_compress_batch(self.handle, kernels, grids, opts, stream)]

    def kron_matvec(self, t: Tucker, z, y, io=TK_FP32, stream=None):
        tk_kron_matvec(self.handle, t.handle, z, y, io, stream)

    def kron_matvec_noalloc(self, t: Tucker, z, y, stream=None):
        tk_kron_matvec_noalloc(self.handle, t.handle, z, y, stream)

    def trace(self, t: Tucker, stream=None) -> float:
        return tk_trace(self.handle, t.handle, stream)

    def quadratic_form(self, t: Tucker, z, io=TK_FP32, stream=None, y=None) -> float:
        return tk_quadratic_form(self.handle, t.handle, z, io, stream, y)

    def quadratic_form_batch(self, ts, zs, io=TK_FP32, stream=None, ys=None):
        return tk_quadratic_form_batch(self.handle, [t.handle for t in ts], zs, io, stream, ys)

    def budget(self):
        return tk_ctx_budget(self.handle)

    def set_matvec_method(self, method: int):
        tk_set_matvec_method(self.handle, method)

    def autotune(self, grid, prec, stream=None):
        """Tune the Gram split of each mode for this grid shape and precision; returns
        {"nsplit": (s0, s1, s2), "ms": (t0, t1, t2)}."""
        ns = (ctypes.c_int * 3)()
        ms = (ctypes.c_double * 3)()
        _check(_lib.tk_autotune(self.handle, ctypes.byref(grid), int(prec), _stream(stream), ns, ms), "tk_autotune")
        return {"nsplit": tuple(ns), "ms": tuple(ms)}

    def autotune_save(self, path: str):
        _check(_lib.tk_autotune_save(self.handle, str(path).encode()), "tk_autotune_save")

    def autotune_load(self, path: str):
        _check(_lib.tk_autotune_load(self.handle, str(path).encode()), "tk_autotune_load")

    def release_stream(self, stream):
        _check(_lib.tk_ctx_release_stream(self.handle, _stream(stream)), "tk_ctx_release_stream")

    def set_workers(self, workers: int):
        _check(_lib.tk_ctx_set_workers(self.handle, workers), "tk_ctx_set_workers")

    def set_graphs(self, on: bool):
        _check(_lib.tk_ctx_set_graphs(self.handle, 1 if on else 0), "tk_ctx_set_graphs")

    def set_cholqr(self, floor: float = 1e-12, one_pass: float = 1e-4, accept2: float = 0.25):
        _check(_lib.tk_ctx_set_cholqr(self.handle, float(floor), float(one_pass), float(accept2)),
               "tk_ctx_set_cholqr")

    def destroy(self):
        if self.handle:
            tk_ctx_destroy(self.handle)
            self.handle = 0


class TuckerView:
    """A result owned by someone else (a server); never freed from Python."""

    def __init__(self, handle: int):
        self.handle = handle
        info = tk_tucker_info(handle)
        self.n, self.ranks, self.rel_err, self.norm_a, self.layout = (
            info["n"], info["ranks"], info["rel_err"], info["norm_a"], info["layout"])

    def factors(self):
        return tk_tucker_get(self.handle)


STREAM_READY = object()   # submit stream marker: the request's vectors are complete already (TK_STREAM_READY)


TK_KRON1_SOLVE, TK_KRON1_CHOL = 0, 1


class Kron1:
    """Separable covariance C = C_1 (x) C_2 (x) C_3 (tk_kron1_*): Cholesky factors, log det,
    solves, Cholesky products and the Gaussian log-likelihood on the device."""

    def __init__(self, ctx: "Context", kernels, grid: tk_grid, nugget=None, stream=None):
        ks = (tk_kernel * 3)(*kernels)
        ng = (ctypes.c_double * 3)(*([0.0] * 3 if nugget is None else [float(x) for x in nugget]))
        h = _vp()
        _check(_lib.tk_kron1_create(ctx.handle, ks, ctypes.byref(grid), ng, _stream(stream), ctypes.byref(h)),
               "tk_kron1_create")
        self.handle = h.value
        self.ctx = ctx
        self.n = tuple(int(x) for x in grid.n)

    def logdet(self):
        out = ctypes.c_double()
        per = (ctypes.c_double * 3)()
        _check(_lib.tk_kron1_logdet(self.handle, ctypes.byref(out), per), "tk_kron1_logdet")
        return out.value, tuple(per)

    def factor(self, axis: int) -> np.ndarray:
        n = self.n[axis]
        L = np.empty((n, n), dtype=np.float64)
        _check(_lib.tk_kron1_factor(self.handle, int(axis), L.ctypes.data), "tk_kron1_factor")
        return L

    def solve(self, z, y, stream=None):
        _check(_lib.tk_kron1_apply(self.ctx.handle, self.handle, TK_KRON1_SOLVE, _ptr(z), _ptr(y), _stream(stream)),
               "tk_kron1_apply")

    def chol_apply(self, z, y, stream=None):
        _check(_lib.tk_kron1_apply(self.ctx.handle, self.handle, TK_KRON1_CHOL, _ptr(z), _ptr(y), _stream(stream)),
               "tk_kron1_apply")

    def loglik(self, z, stream=None):
        out, q = ctypes.c_double(), ctypes.c_double()
        _check(_lib.tk_kron1_loglik(self.ctx.handle, self.handle, _ptr(z), _stream(stream), ctypes.byref(out),
                                    ctypes.byref(q)), "tk_kron1_loglik")
        return out.value, q.value

    def free(self):
        if self.handle:
            _lib.tk_kron1_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Request loop over resident results (tk_server_*): submit returns a ticket, wait blocks
    until that request finished and returns its result as a dict.  Work queued on `stream`
    (default: torch's current stream) before a submit happens before that request; the vectors
    must stay alive until the request finished."""

    def __init__(self, ctx: "Context", workers: int = 4):
        h = _vp()
        _check(_lib.tk_server_create(ctx.handle, int(workers), ctypes.byref(h)), "tk_server_create")
        self.handle = h.value
        self.ctx = ctx

    @staticmethod
    def _order(stream):
        # default: the stream the caller's device work (torch's current stream) is queued on;
        # STREAM_READY: the vectors are complete, no ordering
        if stream is STREAM_READY:
            return (1 << 64) - 1
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    return int(torch.cuda.current_stream().cuda_stream)
            except ImportError:
                pass
            return 0
        return _stream(stream)

    def set_batching(self, max_group: int):
        _check(_lib.tk_server_set_batching(self.handle, int(max_group)), "tk_server_set_batching")

    def _submit(self, req: tk_request) -> int:
        t = ctypes.c_longlong()
        _check(_lib.tk_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "tk_server_submit")
        return t.value

    def submit_compress(self, kernel, grid, opts, stream=None) -> int:
        return self._submit(tk_request(kind=TK_REQ_COMPRESS, kernel=kernel, grid=grid, opts=opts,
                                       stream=self._order(stream)))

    def submit_matvec(self, target: int, z, y, io=TK_FP32, stream=None) -> int:
        return self._submit(tk_request(kind=TK_REQ_MATVEC, target=int(target), z_dev=_ptr(z), y_dev=_ptr(y), io=io,
                                       stream=self._order(stream)))

    def submit_trace(self, target: int, stream=None) -> int:
        return self._submit(tk_request(kind=TK_REQ_TRACE, target=int(target), stream=self._order(stream)))

    def submit_quadform(self, target: int, z, io=TK_FP32, y=None, stream=None) -> int:
        return self._submit(tk_request(kind=TK_REQ_QUADFORM, target=int(target), z_dev=_ptr(z),
                                       y_dev=_ptr(y) if y is not None else None, io=io, stream=self._order(stream)))

    def wait(self, ticket: int) -> dict:
        r = tk_result()
        _check(_lib.tk_server_wait(self.handle, int(ticket), ctypes.byref(r)), "tk_server_wait")
        return dict(status=r.status, kind=r.kind, ranks=tuple(r.ranks), rel_err=r.rel_err, value=r.value,
                    t_submit=r.t_submit, t_start=r.t_start, t_end=r.t_end,
                    error=r.error.decode(errors="replace"))

    def tucker(self, ticket: int) -> TuckerView:
        h = _vp()
        _check(_lib.tk_server_tucker(self.handle, int(ticket), ctypes.byref(h)), "tk_server_tucker")
        return TuckerView(h.value)

    def release(self, ticket: int):
        _check(_lib.tk_server_release(self.handle, int(ticket)), "tk_server_release")

    def destroy(self):
        if self.handle:
            _lib.tk_server_destroy(self.handle)
            self.handle = 0
