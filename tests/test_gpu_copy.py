"""The streaming copy that serves as the measured bandwidth ceiling: exact
copies at sizes that leave ragged grid-stride tails, and the argument checks
(alignment, size, overlap) before any launch."""
import pytest

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


@pytest.mark.parametrize("nfloat", [4, 1028, 1 << 20, (64 << 20) + 12])
def test_stream_copy_is_exact(nfloat):
    torch = gh.torch_mod()
    L = gh.lib()
    g = torch.Generator(device="cuda").manual_seed(nfloat)
    a = torch.rand(nfloat, device="cuda", generator=g)
    b = torch.full_like(a, -1.0)
    L.lbrt_stream_copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_stream_copy_rejects_bad_arguments():
    torch = gh.torch_mod()
    L = gh.lib()
    a = torch.zeros(1024, device="cuda")
    lib = L.library()
    import ctypes
    base = a.data_ptr()
    cases = [
        (base, base + 2048, 1000),       # not a multiple of 16 bytes
        (base + 4, base + 2048, 1024),   # misaligned source
        (base, base + 512, 1024),        # overlap
    ]
    for src, dst, nbytes in cases:
        rc = lib.lbrt_stream_copy(ctypes.c_void_p(src), ctypes.c_void_p(dst),
                                  ctypes.c_int64(nbytes), ctypes.c_void_p(0))
        assert rc == L.LBRT_E_INVAL, (src - base, dst - base, nbytes)
