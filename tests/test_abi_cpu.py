"""The C-ABI library loads, exports every symbol include/tk.h declares, and validates
arguments on the host (calls that need no device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tk.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def tk():
    from paper_1711_06874_amd import tk as mod
    return mod


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("tk_compress", "tk_kron_matvec", "tk_trace", "tk_quadratic_form", "tk_compress_batch"):
        assert must in names


def test_library_exports_every_declared_symbol(tk):
    lib = ctypes.CDLL(tk.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) <= set(tk.EXPORTED)


def test_version_and_strerror(tk):
    assert "gfx950" in tk.tk_version()
    assert tk.tk_strerror(tk.TK_ELAYOUT) == "TK_ELAYOUT"
    assert tk.tk_strerror(tk.TK_ENOCONV) == "TK_ENOCONV"


def test_estimate_bytes_scales_with_grid(tk):
    o = tk.make_opts(eps=1e-6, prec=tk.TK_FP32)
    small = tk.tk_estimate_bytes(tk.make_grid(64), o)
    big = tk.tk_estimate_bytes(tk.make_grid(256), o)
    assert big > 4 * 256 ** 3          # at least the FP32 tensor
    assert big > 8 * small
    d = tk.tk_estimate_bytes(tk.make_grid(64), tk.make_opts(ranks=4, prec=tk.TK_FP64))
    assert d > 8 * 64 ** 3


@pytest.mark.parametrize("grid_kw,opts_kw,status", [
    (dict(n=(1, 8, 8)), dict(eps=1e-6), "TK_EINVAL"),          # n < 2
    (dict(n=(8, 8, 2000)), dict(eps=1e-6), "TK_EUNSUPPORTED"),  # n too large
    (dict(n=8, b=(-1.0, 1.0, 1.0)), dict(eps=1e-6), "TK_EINVAL"),
    (dict(n=8), dict(eps=0.0, ranks=(0, 2, 2)), "TK_EINVAL"),   # neither eps nor ranks
    (dict(n=8), dict(eps=-1.0), "TK_EINVAL"),
    (dict(n=8), dict(eps=1e-6, r_max=60), "TK_EUNSUPPORTED"),
    (dict(n=8), dict(eps=1e-6, prec=7), "TK_EINVAL"),
    (dict(n=8, layout=5), dict(eps=1e-6), "TK_EINVAL"),
])
def test_estimate_rejects_bad_arguments(tk, grid_kw, opts_kw, status):
    with pytest.raises(tk.TkError) as ei:
        tk.tk_estimate_bytes(tk.make_grid(**grid_kw), tk.make_opts(**opts_kw))
    assert status in str(ei.value)


def test_ctx_create_without_gpu_fails_cleanly(tk):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(tk.TkError) as ei:
        tk.tk_ctx_create(0, 0)
    assert "TK_EHIP" in str(ei.value) or "TK_EINVAL" in str(ei.value)
