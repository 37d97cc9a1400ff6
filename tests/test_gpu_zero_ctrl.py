"""GPU parity of the zero-control decoder variant (rows of all-zero control bytes decoded by byte
widening): identical output to the oracle and to the general variant, on streams made only of
one-byte integers, on mixed streams and on random ones; the autotuner picks one of the two."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

SIZES = [1, 3, 4, 5, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097, 8193, 65_537, 250_001]


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()
    for delta in (False, True):
        svb.svb_set_decode_variant(delta, -1)


def small_deltas(n, seed):
    """Running sums of deltas below 2^8 (every control byte 0 under delta coding)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.integers(0, 256, size=n, dtype=np.uint64), dtype=np.uint64).astype(np.uint32)


def decode_gpu(stream, n, delta, start, shift):
    buf = np.zeros(stream.size + shift + 16, dtype=np.uint8)
    buf[shift:shift + stream.size] = stream
    d = to_dev_u8(buf)
    out = torch.full((n + 8,), 0x5EED, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    if delta:
        svb.svb_delta_decode(n, d.data_ptr() + shift, stream.size, out, start, err)
    else:
        svb.svb_decode(n, d.data_ptr() + shift, stream.size, out, err)
    torch.cuda.synchronize()
    host = u32_host(out)
    assert int(err.item()) == 0
    assert np.all(host[n:] == 0x5EED)
    return host[:n].copy()


@pytest.mark.parametrize("delta", [False, True])
def test_zero_control_variant_matches_oracle(delta):
    rng = np.random.default_rng(17 + delta)
    for n in SIZES:
        cases = [small_deltas(n, n) if delta else (rng.integers(0, 256, size=n)).astype(np.uint32),
                 inputs.docids(n, seed=n)[0],
                 (rng.integers(0, 1 << 32, size=n, dtype=np.uint64) >> rng.integers(0, 32, size=n).astype(np.uint64)
                  ).astype(np.uint32)]
        for ci, x in enumerate(cases):
            start = int(rng.integers(0, 1 << 32)) if delta else 0
            if delta and ci == 0:
                x = (x.astype(np.uint64) + start).astype(np.uint32)  # deltas below 2^8 from `start`
            s = oracle.encode(x, delta=delta, start=start)
            want, _ = oracle.decode(s, n, delta=delta, start=start)
            log_case("zero-control", "n=%d" % n, "case=%d" % ci, "delta=%s" % delta)
            shift = int(rng.integers(0, 16))
            svb.svb_set_decode_variant(delta, 1)
            got1 = decode_gpu(s, n, delta, start, shift)
            svb.svb_set_decode_variant(delta, 0)
            got0 = decode_gpu(s, n, delta, start, shift)
            np.testing.assert_array_equal(got1, want, err_msg="variant 1 n=%d case %d" % (n, ci))
            np.testing.assert_array_equal(got0, want, err_msg="variant 0 n=%d case %d" % (n, ci))


def test_autotune_decode_picks_a_variant():
    n = 1 << 22
    x = small_deltas(n, 3)
    s = oracle.encode(x, delta=True)
    d = to_dev_u8(s)
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    log_case("zero-control autotune")
    v = svb.svb_autotune_decode(n, d, s.size, out, 0, True)
    assert v in (0, 1, 2, 3)  # delta: zero-control bit, sums-by-decoding bit
    out.zero_()
    svb.svb_delta_decode(n, d, s.size, out, 0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32_host(out), x)
    svb.svb_set_decode_variant(True, -1)
