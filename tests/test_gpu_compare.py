"""GPU parity of the comparison formats (VByte and varint-GB, Table 1): encoders byte for byte
against the oracle's streams, decoders against the oracle's values, at sizes spanning several
segments, tiles and supertiles with ragged tails, at any input alignment, with bytes after the
stream, and on truncated or over-long input."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host, u8_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

SIZES = [1, 2, 3, 4, 5, 63, 64, 65, 255, 1023, 1024, 1025, 4097, 16_385, 65_537, 250_001]
FORMATS = {
    "vbyte": (oracle.vbyte_encode, oracle.vbyte_decode, "svb_vbyte_encode", "svb_vbyte_decode",
              "svb_vbyte_max_bytes"),
    "varintgb": (oracle.varintgb_encode, oracle.varintgb_decode, "svb_varintgb_encode", "svb_varintgb_decode",
                 "svb_varintgb_max_bytes"),
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()


def values(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "bits":  # every byte length of both formats
        return (rng.integers(0, 1 << 32, size=n, dtype=np.uint64) >> rng.integers(0, 32, size=n).astype(np.uint64)
                ).astype(np.uint32)
    if kind == "gaps":  # document-id gaps
        return inputs.docid_gaps(n, seed=seed)
    if kind == "zeros":
        return np.zeros(n, dtype=np.uint32)
    return np.full(n, 0xFFFFFFFF, dtype=np.uint32)


def encode_gpu(fmt, x):
    _, _, enc, _, maxb = FORMATS[fmt]
    n = x.size
    cap = getattr(svb, maxb)(n)
    out = torch.full((cap + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    getattr(svb, enc)(n, to_dev_u32(x), out, size)
    torch.cuda.synchronize()
    return u8_host(out), int(size.item())


def decode_gpu(fmt, stream, n, shift=0, extra=b""):
    dec = FORMATS[fmt][3]
    buf = np.zeros(stream.size + len(extra) + shift + 16, dtype=np.uint8)
    buf[shift:shift + stream.size] = stream
    buf[shift + stream.size:shift + stream.size + len(extra)] = np.frombuffer(extra, dtype=np.uint8)
    d = to_dev_u8(buf)
    out = torch.full((n + 8,), 0x5EED, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    getattr(svb, dec)(n, d.data_ptr() + shift, stream.size + len(extra), out, err)
    torch.cuda.synchronize()
    host = u32_host(out)
    assert np.all(host[n:] == 0x5EED), "wrote past the output"
    return host[:n].copy(), int(err.item())


@pytest.mark.parametrize("fmt", sorted(FORMATS))
@pytest.mark.parametrize("kind", ["bits", "gaps", "zeros", "max"])
def test_encode_matches_oracle(fmt, kind):
    for n in SIZES:
        x = values(kind, n, n)
        log_case("compare encode", fmt, kind, "n=%d" % n)
        want = FORMATS[fmt][0](x)
        got, size = encode_gpu(fmt, x)
        assert size == want.size, (n, size, want.size)
        np.testing.assert_array_equal(got[:size], want, err_msg="%s %s n=%d" % (fmt, kind, n))
        assert np.all(got[size:] == 0xA5), "wrote past the stream"


@pytest.mark.parametrize("fmt", sorted(FORMATS))
@pytest.mark.parametrize("kind", ["bits", "gaps", "zeros", "max"])
def test_decode_matches_oracle(fmt, kind):
    rng = np.random.default_rng(31)
    for n in SIZES:
        x = values(kind, n, n + 1)
        s = FORMATS[fmt][0](x)
        want, _ = FORMATS[fmt][1](s, n)
        shift = int(rng.integers(0, 16))
        extra = bytes(rng.integers(0, 256, size=int(rng.integers(0, 40)), dtype=np.uint8)) if n % 2 else b""
        log_case("compare decode", fmt, kind, "n=%d" % n, "shift=%d" % shift, "extra=%d" % len(extra))
        got, err = decode_gpu(fmt, s, n, shift, extra)
        assert err == 0, (fmt, kind, n)
        np.testing.assert_array_equal(got, want, err_msg="%s %s n=%d" % (fmt, kind, n))


@pytest.mark.parametrize("fmt", sorted(FORMATS))
def test_large_round_trip(fmt):
    """2^22 document-id gaps: device encode, stream equal to the oracle's, device decode."""
    n = 1 << 22
    x = inputs.docid_gaps(n, seed=12)
    log_case("compare round trip", fmt, "n=%d" % n)
    got, size = encode_gpu(fmt, x)
    want = FORMATS[fmt][0](x)
    assert size == want.size
    np.testing.assert_array_equal(got[:size], want)
    dec, err = decode_gpu(fmt, want, n, shift=3)
    assert err == 0
    np.testing.assert_array_equal(dec, x)


@pytest.mark.parametrize("fmt", sorted(FORMATS))
def test_truncated_stream_is_reported(fmt):
    for n in (5, 1025, 65_537):
        x = values("bits", n, 40 + n)
        s = FORMATS[fmt][0](x)
        lo = n if fmt == "vbyte" else n + (n + 3) // 4
        if s.size - 1 < lo:
            continue
        log_case("compare truncated", fmt, "n=%d" % n)
        with pytest.raises(ValueError):
            FORMATS[fmt][1](s[:-1], n)
        _, err = decode_gpu(fmt, s[:-1], n)
        assert err == svb.SVB_DECODE_CORRUPT


def test_vbyte_overlong_integer_is_reported():
    """An integer of six bytes among the first n is corrupt (the oracle refuses it too); one
    after the n-th integer is not read."""
    good = oracle.vbyte_encode(values("bits", 3000, 50))
    bad = np.concatenate([good[:700], np.array([0x81] * 5 + [0x01], dtype=np.uint8), good[700:]])
    n_before = int(np.sum(good[:700] < 0x80))
    n = n_before + 1 + 10
    with pytest.raises(ValueError):
        oracle.vbyte_decode(bad, n)
    log_case("compare vbyte overlong")
    _, err = decode_gpu("vbyte", bad, n)
    assert err == svb.SVB_DECODE_CORRUPT
    want, _ = oracle.vbyte_decode(bad, n_before)
    got, err = decode_gpu("vbyte", bad, n_before)
    assert err == 0
    np.testing.assert_array_equal(got, want)


def test_empty_input():
    for fmt in FORMATS:
        _, _, enc, dec, _ = FORMATS[fmt]
        size = torch.full((1,), 7, dtype=torch.int64, device="cuda")
        getattr(svb, enc)(0, None, None, size)
        getattr(svb, dec)(0, None, 0, None)
        torch.cuda.synchronize()
        assert int(size.item()) == 0


@pytest.mark.parametrize("fmt", sorted(FORMATS))
def test_streams_of_tens_of_megabytes(fmt):
    """2^25 document-id gaps: for varint-GB about 42 MB, 82 supertiles of 512 KiB, so the true
    chain is followed across more supertiles than one pass of the top-level wave holds (64); for
    VByte about 34 MB, whose 1 KiB tiles take the multi-workgroup scan."""
    n = 1 << 25
    x = inputs.docid_gaps(n, seed=15)
    s = FORMATS[fmt][0](x)
    assert s.size > 32 * 1024 * 1024
    log_case("compare tens of MB", fmt, "n=%d" % n, "bytes=%d" % s.size)
    got, err = decode_gpu(fmt, s, n, shift=5)
    assert err == 0
    np.testing.assert_array_equal(got, x)
