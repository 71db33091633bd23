"""The streaming-bandwidth probe copies exactly (whole chunks and a ragged
tail) and reports a rate below the device's published peak."""
import ctypes as C

import pytest

from paper_2507_16087_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("nbytes", [16, 16 * 1000 + 16, 16 * 1024 * 3 + 48, 64 << 20])
def test_probe_copies_exactly(torch, nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    a = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    b = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    gbs = C.c_double(0.0)
    st = L.lib().cbs_stream_probe(a.data_ptr(), b.data_ptr(), nbytes, 2, C.byref(gbs), None)
    assert st == L.CBS_OK
    torch.cuda.synchronize()
    assert torch.equal(b[:nbytes], a)
    assert int(b[nbytes:].count_nonzero()) == 0   # nothing written past the end
    assert gbs.value > 0


def test_probe_rate_is_below_peak(torch):
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    gbs = C.c_double(0.0)
    st = L.lib().cbs_stream_probe(a.data_ptr(), b.data_ptr(), nbytes, 5, C.byref(gbs),
                                  torch.cuda.current_stream().cuda_stream)
    assert st == L.CBS_OK
    print(f"streaming copy of 1 GiB: {gbs.value:.0f} GB/s")
    assert 1000.0 < gbs.value < 8000.0
