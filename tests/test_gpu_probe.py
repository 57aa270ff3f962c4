"""The bandwidth probes (lbm_stream_probe): the copy moves every byte, the
write kind zeroes exactly the requested range, the read kind leaves its
output alone, for launch shapes whose grid covers the buffer several times
over and for ones that need a remainder pass."""
import ctypes

import pytest

from paper_1611_02445_amd import _abi

pytestmark = pytest.mark.gpu


def _probe(kind, src, dst, nbytes, blocks, threads):
    import torch
    s = torch.cuda.current_stream()
    _abi.call("lbm_stream_probe", ctypes.c_void_p(s.cuda_stream), kind,
              None if src is None else ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
              blocks, threads)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n16,blocks,threads", [(1, 1, 64), (1000, 3, 64), (4096 * 5 + 7, 16, 256),
                                                (1 << 20, 1024, 1024), ((1 << 22) + 3, 8192, 256)])
def test_probe_kinds(n16, blocks, threads):
    import torch
    g = torch.Generator(device="cuda").manual_seed(n16)
    src = torch.randint(-2**31, 2**31 - 1, (4 * n16 + 8,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.full_like(src, -1)
    _probe(3, src, dst, 16 * n16, blocks, threads)
    assert torch.equal(dst[:4 * n16], src[:4 * n16])
    assert bool((dst[4 * n16:] == -1).all())  # nothing past the requested bytes
    _probe(2, None, dst, 16 * n16, blocks, threads)
    assert bool((dst[:4 * n16] == 0).all()) and bool((dst[4 * n16:] == -1).all())
    dst.fill_(7)
    _probe(1, src, dst, 16 * n16, blocks, threads)
    # the read kind writes one word only when the data hash to one fixed value
    assert int((dst != 7).sum()) <= 1
