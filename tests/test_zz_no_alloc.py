"""The allocation-free delta decoder (svb_delta_decode_noalloc), through the C ABI: its output must
equal svb_delta_decode's bit for bit (and the oracle's input), on two calls in a row whose second
is smaller, so that the shared static scratch is reused with stale contents from the first call;
sizes past SVB_NOALLOC_MAX_N are refused before anything runs."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u8, u32_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()


def both(stream, n, start):
    """(svb_delta_decode output, svb_delta_decode_noalloc output, noalloc err) on one stream."""
    d = to_dev_u8(stream)
    ref = torch.full((n + 4,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    got = torch.full((n + 4,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    svb.svb_delta_decode(n, d, stream.size, ref, start)
    rc = svb.lib().svb_delta_decode_noalloc(ctypes.c_uint64(n), ctypes.c_void_p(d.data_ptr()),
                                            ctypes.c_uint64(stream.size), ctypes.c_void_p(got.data_ptr()),
                                            ctypes.c_uint32(start), ctypes.c_void_p(err.data_ptr()),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    r, g = u32_host(ref), u32_host(got)
    assert np.all(g[n:] == 0x5A5A5A5A), "written past n"
    return r[:n].copy(), g[:n].copy(), int(err.item())


@pytest.mark.parametrize("sizes", [(5_000_003, 70_001), (300 * 4096 + 5, 4097), (70_001, 3)])
def test_noalloc_equals_delta_decode_twice_second_smaller(sizes):
    for i, n in enumerate(sizes):
        x, _ = inputs.docids(n, seed=40 + i, start=1000 * i)
        start = 77 * (i + 1)
        s = oracle.encode(x, delta=True, start=start)
        log_case("noalloc", "call=%d" % i, "n=%d" % n)
        ref, got, err = both(s, n, start)
        assert err == 0
        np.testing.assert_array_equal(got, ref, err_msg="call %d n=%d" % (i, n))
        np.testing.assert_array_equal(got, x)


def test_noalloc_every_length_then_small():
    """Values of every byte length (corrections on nearly every block, long group spans), then a
    small call."""
    for i, n in enumerate((1_000_003, 1025)):
        x = np.cumsum(inputs.stress_lengths(n, seed=60 + i), dtype=np.uint32)
        s = oracle.encode(x, delta=True, start=9)
        log_case("noalloc every length", "n=%d" % n)
        ref, got, err = both(s, n, 9)
        assert err == 0
        np.testing.assert_array_equal(got, ref)


def test_noalloc_refuses_n_past_its_maximum():
    cap = svb.SVB_NOALLOC_MAX_N
    # rejected on the host before any launch (the pointers are never read)
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    o = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(svb.SvbError):
        svb.svb_delta_decode_noalloc(cap + 1, d, (cap + 4) // 4 + 1, o)
    assert svb.svb_delta_decode_noalloc(0, None, 0, None) == 0
