"""The device's seeded N(0,1) inputs against the oracle's independent Philox4x32-10 and
Box-Muller: the 32-bit word stream bit for bit (several keys, counters across the 2^32
boundary), the normals within one float ulp (both round an FP64 Box-Muller value once; the FP64
log/cos/sin of the two sides may differ in the last bit, which moves the float only when the
value sits on a rounding boundary)."""
import numpy as np
import pytest

from tests.gpu_util import host, require_gpu, say, torch

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


@pytest.mark.parametrize("key,c0,nb", [((0, 0), 0, 1), ((1711, 1), 0, 100_003), ((0xFFFFFFFF, 7), (1 << 32) - 50, 4096),
                                       ((0xa4093822, 0x299f31d0), 123456789, 777)])
def test_philox_words_bitwise(ctx, tk, oracle, key, c0, nb):
    out = torch.empty(4 * nb, dtype=torch.int32, device="cuda")
    tk.tk_philox4x32(ctx.handle, key, c0, out)
    got = host(out).view(np.uint32).reshape(nb, 4)
    want = oracle.philox_blocks(key, c0, nb)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("count,seed,stream", [(1, 1711, 1), (1_000_001, 1711, 2), (256 ** 3, 1711, 9)])
def test_normal_fill_matches_oracle(ctx, tk, oracle, count, seed, stream):
    z = torch.empty(count, dtype=torch.float32, device="cuda")
    tk.tk_normal_fill(ctx.handle, seed, stream, z)
    got = host(z)
    want = oracle.normal_philox(count, seed, stream)
    ulp = np.spacing(np.abs(want).astype(np.float32))
    diff = np.abs(got.astype(np.float64) - want.astype(np.float64))
    exact = float(np.mean(got == want))
    say("count %d: %.6f of the values bit-equal, max diff %.2f ulp" % (count, exact, float((diff / ulp).max())))
    assert np.all(diff <= ulp)
    assert np.isfinite(got).all()
