"""fph_hbm_copy, the copy the bandwidth ceilings are measured with: both
access patterns copy every byte and nothing beyond the end, for ragged sizes
and any workgroup count."""

import ctypes

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pattern", [0, 1])
@pytest.mark.parametrize("n16,nblocks", [(1, 0), (7, 3), (4097, 0), (123457, 7), (123457, 480),
                                         (1 << 20, 0), (1000, 2000)])
def test_copy_every_byte_and_nothing_more(pattern, n16, nblocks):
    from paper_2203_01291_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(n16 + nblocks)
    src = torch.randn(4 * n16, device=dev, generator=g)
    guard = 64
    dst = torch.full((4 * n16 + guard,), 7.0, device=dev)
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.fph_hbm_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                          16 * n16, nblocks, pattern, sp)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:4 * n16], src)
    assert torch.all(dst[4 * n16:] == 7.0)
