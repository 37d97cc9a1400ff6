"""GPU parity of append without re-encoding (svb_append / svb_delta_append): the result equals,
byte for byte, the oracle's encoding of the concatenated integers, for every old length mod 4,
empty sides, random byte alignments, and nothing is written past the new stream's end."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u8_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

SENTINEL8 = 0xA7


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()


def values(n, rng):
    return (rng.integers(0, 1 << 32, size=n, dtype=np.uint64) >> rng.integers(0, 32, size=n).astype(np.uint64)
            ).astype(np.uint32)


def run_append(old, n, b, delta, prev, in_shift, out_shift):
    buf = np.full(old.size + in_shift + 32, 0x5C, dtype=np.uint8)
    buf[in_shift:in_shift + old.size] = old
    d_in = to_dev_u8(buf)
    cap = (n + b.size + 3) // 4 + (old.size - (n + 3) // 4) + 4 * b.size
    out = torch.full((cap + out_shift + 48,), SENTINEL8, dtype=torch.uint8, device="cuda")
    size = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    vals = to_dev_u32(b if b.size else np.zeros(1, np.uint32))
    base_in, base_out = d_in.data_ptr() + in_shift, out.data_ptr() + out_shift
    if delta:
        svb.svb_delta_append(n, base_in, old.size, b.size, vals, prev, base_out, size)
    else:
        svb.svb_append(n, base_in, old.size, b.size, vals, base_out, size)
    torch.cuda.synchronize()
    host = u8_host(out)
    sz = int(size.item())
    assert np.all(host[:out_shift] == SENTINEL8)
    assert np.all(host[out_shift + sz:] == SENTINEL8)
    return host[out_shift:out_shift + sz].copy()


@pytest.mark.parametrize("delta", [False, True])
def test_append_small_cases(delta):
    rng = np.random.default_rng(5 + delta)
    log_case("append small", "delta=%s" % delta)
    for n in [0, 1, 2, 3, 4, 5, 6, 7, 63, 64, 65, 1023, 1024, 1025, 4099]:
        for k in [0, 1, 2, 3, 4, 5, 17, 1024, 1025, 5000]:
            a, b = values(n, rng), values(k, rng)
            start = int(rng.integers(0, 1 << 32)) if delta else 0
            old = oracle.encode(a, delta=delta, start=start)
            prev = (int(a[-1]) if n else start) if delta else 0
            want = oracle.encode(np.concatenate([a, b]), delta=delta, start=start)
            got = run_append(old, n, b, delta, prev, int(rng.integers(0, 16)), int(rng.integers(0, 16)))
            np.testing.assert_array_equal(got, want, err_msg="n=%d k=%d" % (n, k))


def test_append_to_a_long_delta_stream():
    """Document ids (Section 5's setting): 2^20 stored, 300,001 appended, several alignments."""
    x, _ = inputs.docids((1 << 20) + 300_001, seed=12)
    a, b = x[:1 << 20], x[1 << 20:]
    old = oracle.encode(a, delta=True)
    want = oracle.encode(x, delta=True)
    log_case("append long")
    for in_shift, out_shift in [(0, 0), (3, 11), (15, 1)]:
        got = run_append(old, a.size, b, True, int(a[-1]), in_shift, out_shift)
        np.testing.assert_array_equal(got, want)


def test_append_argument_errors():
    d = torch.zeros(64, dtype=torch.uint8, device="cuda")
    v = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(svb.SvbError):
        svb.svb_append(100, d, 10, 1, v, d)  # in_bytes below the control stream
    with pytest.raises(svb.SvbError):
        svb.svb_append(0, d, 0, 2, v.data_ptr() + 2, d)  # misaligned values
