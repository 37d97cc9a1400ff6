"""GPU parity: the HIP library (through its C ABI) against the oracle, bit for bit.

Everything here is integer work, so the bar is exact equality: encoded bytes,
decoded values, stream sizes and the corruption flag.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host, u8_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

BOUNDS = [(0, 1 << 8), (1 << 8, 1 << 16), (1 << 16, 1 << 24), (1 << 24, 1 << 32)]
TILE = 4096    # integers per encoder tile
SEG = 1024     # integers per decoder segment (one wave)
GROUP = 4096   # integers per decoder group (segments walked by one wave)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()  # fails loudly if the library is missing
    yield
    torch.cuda.synchronize()


def gpu_encode(x, delta=False, start=0, out_pad=0, out_shift=0):
    """Encode with the library; returns (stream bytes, reported size)."""
    n = x.size
    d = to_dev_u32(x)
    cap = svb.svb_max_compressed_bytes(n) + out_pad + out_shift
    out = torch.full((max(1, cap),), 0xA5, dtype=torch.uint8, device="cuda")
    size = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    view = out[out_shift:]
    if delta:
        svb.svb_delta_encode(n, d, view, start, size)
    else:
        svb.svb_encode(n, d, view, size)
    torch.cuda.synchronize()
    sz = int(size.item())
    host = u8_host(out)
    # bytes past the stream are untouched
    assert np.all(host[out_shift + sz:] == 0xA5)
    assert np.all(host[:out_shift] == 0xA5)
    return host[out_shift:out_shift + sz], sz


def gpu_decode(stream, n, delta=False, start=0, in_shift=0, trailing=0):
    """Decode with the library; returns (values, err flag)."""
    buf = np.concatenate([np.full(in_shift, 0x5A, np.uint8), np.asarray(stream, np.uint8),
                          np.full(trailing, 0xFF, np.uint8)])
    d = to_dev_u8(buf)
    view = d[in_shift:]
    out = torch.full((max(1, n) + 1,), 0x7EADBEEF, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    if delta:
        svb.svb_delta_decode(n, view, view.numel(), out, start, err)
    else:
        svb.svb_decode(n, view, view.numel(), out, err)
    torch.cuda.synchronize()
    host = u32_host(out)
    assert host[max(1, n)] == 0x7EADBEEF  # nothing written past n
    return host[:n], int(err.item())


def check_round_trip(x, delta=False, start=0, tag=""):
    log_case("round_trip", tag, "n=%d" % x.size, "delta=%s" % delta, "start=%d" % start)
    ref = oracle.encode(x, delta=delta, start=start)
    got, sz = gpu_encode(x, delta=delta, start=start)
    assert sz == ref.size
    np.testing.assert_array_equal(got, ref)
    vals, err = gpu_decode(ref, x.size, delta=delta, start=start)
    assert err == 0
    np.testing.assert_array_equal(vals, x)


# ------------------------------------------------------------------ sizes spanning tiles

SIZES = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 63, 64, 65, 255, 256, 257, SEG - 1, SEG, SEG + 1, TILE - 1, TILE,
         TILE + 1, 3 * TILE + 5, GROUP - 1, GROUP, GROUP + 1, 3 * GROUP + SEG - 3, 8191, 8192, 8193, 65_537,
         250_001]


@pytest.mark.parametrize("n", SIZES)
def test_round_trip_random(n):
    rng = np.random.default_rng(n)
    x = (inputs.random_u32(n, seed=n) >> rng.integers(0, 32, size=n).astype(np.uint32)).astype(np.uint32)
    check_round_trip(x, tag="mixed")
    check_round_trip(x, delta=True, start=7, tag="mixed")


@pytest.mark.parametrize("n", [0, 1, 4, 4097])
def test_zero_and_max_values(n):
    check_round_trip(np.zeros(n, np.uint32), tag="zeros")
    check_round_trip(np.full(n, 0xFFFFFFFF, np.uint32), tag="max")
    check_round_trip(np.full(n, 0xFFFFFFFF, np.uint32), delta=True, start=0xFFFFFFFF, tag="max")


@pytest.mark.parametrize("start", [0, 1, 0x80000000, 0xFFFFFFFF])
def test_delta_starts(start):
    x, _ = inputs.docids(3 * TILE + 17, seed=5, start=start)
    check_round_trip(x, delta=True, start=start, tag="docids")


def test_uniform_lengths_config_full():
    """1,000,003 integers, lengths uniform in 1..4 (n mod 4 = 3): plain encode and decode."""
    x = inputs.uniform_lengths(1_000_003, seed=1)
    check_round_trip(x, tag="uniform_lengths")


# ------------------------------------------------------------------ brute force

def _pattern_values(pattern, variant):
    out = []
    for i, L in enumerate(pattern):
        lo, hi = BOUNDS[L - 1]
        out.append([lo, lo + 1, hi - 1][(i + variant) % 3])
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_brute_force_patterns(n):
    for pattern in itertools.product(range(1, 5), repeat=n):
        x = _pattern_values(pattern, 0)
        ref = oracle.encode(x)
        got, sz = gpu_encode(x)
        assert sz == ref.size and np.array_equal(got, ref), pattern
        vals, err = gpu_decode(ref, n)
        assert err == 0 and np.array_equal(vals, x), pattern


def test_brute_force_all_six_patterns_in_one_stream():
    """All 4^6 length patterns with boundary values, back to back in one stream, at every
    alignment they fall on; plain and delta."""
    parts = [_pattern_values(p, v) for v in range(3) for p in itertools.product(range(1, 5), repeat=6)]
    x = np.concatenate(parts)
    check_round_trip(x, tag="all_patterns")
    check_round_trip(x, delta=True, start=3, tag="all_patterns")


# ------------------------------------------------------------------ random streams

@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 1001, TILE + 3, 5 * TILE + 2])
def test_random_stream_decode(n):
    """Random control bytes (garbage in unused tail fields) and the data they describe."""
    k = (n + 3) // 4
    ctrl = inputs.random_bytes(k, seed=300 + n)
    need = sum(((int(ctrl[i // 4]) >> (2 * (i % 4))) & 3) + 1 for i in range(n))
    stream = np.concatenate([ctrl, inputs.random_bytes(need, seed=400 + n)])
    ref, used = oracle.decode(stream, n)
    assert used == stream.size
    log_case("random_stream", n)
    vals, err = gpu_decode(stream, n)
    assert err == 0
    np.testing.assert_array_equal(vals, ref)
    dref, _ = oracle.decode(stream, n, delta=True, start=11)
    dvals, err = gpu_decode(stream, n, delta=True, start=11)
    assert err == 0
    np.testing.assert_array_equal(dvals, dref)


@pytest.mark.slow
def test_encode_with_64bit_segment_offsets():
    """1.05e9 integers: the encoder's worst case (4.25 bytes per integer) passes 4 GiB, so its
    segment offsets are 64-bit
    (below that they are 32-bit).  Checked by what holds at any size: integer i is i mod 256, one
    byte each, so every control byte is 0, data byte i is i mod 256 and the size is ceil(n/4) + n;
    the stream then decodes back to the input."""
    n = 1_050_000_000
    log_case("encode with 64-bit segment offsets", "n=%d" % n)
    x = torch.arange(n, dtype=torch.int32, device="cuda").bitwise_and_(0xFF)
    cap = svb.svb_max_compressed_bytes(n)
    assert cap >= 1 << 32
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_encode(n, x, out, size)
    torch.cuda.synchronize()
    nc = (n + 3) // 4
    assert int(size.item()) == nc + n
    assert int(torch.count_nonzero(out[:nc]).item()) == 0
    assert bool(torch.equal(out[nc:nc + n], x.to(torch.uint8)))
    back = torch.empty(n, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    svb.svb_decode(n, out, nc + n, back, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and bool(torch.equal(back, x))
    del x, out, back


def test_buffer_of_4gib_takes_64bit_offsets():
    """A buffer declared 4 GiB or larger switches the group offsets to 64 bits (below that they
    are 32-bit); the stream at its start decodes the same, plain and delta, and the bytes after
    it are not read into any value."""
    x = inputs.docids(250_001, seed=14)[0]
    big = torch.empty((1 << 32) + 64, dtype=torch.uint8, device="cuda")
    for delta in (False, True):
        s = oracle.encode(x, delta=delta)
        want, _ = oracle.decode(s, x.size, delta=delta)
        big[:s.size].copy_(to_dev_u8(s))
        big[s.size:s.size + 4096].fill_(0xFF)
        log_case("4 GiB buffer", "delta=%s" % delta)
        out = torch.zeros(x.size, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        if delta:
            svb.svb_delta_decode(x.size, big, big.numel(), out, 0, err)
        else:
            svb.svb_decode(x.size, big, big.numel(), out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        np.testing.assert_array_equal(u32_host(out), want)
    del big


@pytest.mark.parametrize("shift", [1, 2, 3, 5, 13])
def test_misaligned_streams(shift):
    """Streams at any byte alignment, and trailing bytes after the stream."""
    x = inputs.stress_lengths(2 * TILE + 9, seed=shift)
    ref = oracle.encode(x)
    log_case("misaligned", shift)
    vals, err = gpu_decode(ref, x.size, in_shift=shift, trailing=shift * 3)
    assert err == 0
    np.testing.assert_array_equal(vals, x)
    got, sz = gpu_encode(x, out_shift=shift)
    assert sz == ref.size
    np.testing.assert_array_equal(got, ref)


# ------------------------------------------------------------------ corruption and arguments

@pytest.mark.parametrize("n", [1, 5, 4099, 3 * TILE])
def test_truncated_stream_flags_corrupt(n):
    x = inputs.uniform_lengths(n, seed=n)
    ref = oracle.encode(x)
    for cut in (1, 2, 17):
        if cut > ref.size - (n + 3) // 4:
            continue
        log_case("truncated", n, cut)
        _, err = gpu_decode(ref[:-cut], n)
        assert err == svb.SVB_DECODE_CORRUPT
        _, err = gpu_decode(ref[:-cut], n, delta=True)
        assert err == svb.SVB_DECODE_CORRUPT


def test_argument_errors():
    d8 = torch.zeros(64, dtype=torch.uint8, device="cuda")
    d32 = torch.zeros(64, dtype=torch.int32, device="cuda")
    L = svb.lib()
    # control stream longer than in_bytes
    assert L.svb_decode(9, d8.data_ptr(), 2, d32.data_ptr(), None, None) == -1
    # misaligned uint32 output / input
    assert L.svb_decode(4, d8.data_ptr(), 64, d32.data_ptr() + 2, None, None) == -1
    assert L.svb_encode(4, d32.data_ptr() + 1, d8.data_ptr(), None, None) == -1
    # null pointers with n > 0
    assert L.svb_decode(4, None, 64, d32.data_ptr(), None, None) == -1
    assert L.svb_encode(4, d32.data_ptr(), None, None, None) == -1
    # n = 0 is fine and reports an empty stream
    size = torch.full((1,), 99, dtype=torch.int64, device="cuda")
    assert L.svb_encode(0, None, None, size.data_ptr(), None) == 0
    torch.cuda.synchronize()
    assert int(size.item()) == 0


def test_repeated_calls_and_streams():
    """Many launches in a row (fresh epochs), two streams at once, growing sizes."""
    xs = [inputs.stress_lengths(n, seed=n) for n in (TILE * 40 + 3, TILE * 2, TILE * 300 + 1)]
    refs = [oracle.encode(x, delta=True, start=1) for x in xs]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        outs = []
        for i, (x, ref) in enumerate(zip(xs, refs)):
            st = s1 if (i + rep) % 2 == 0 else s2
            with torch.cuda.stream(st):
                d = to_dev_u8(ref)
                o = torch.empty(x.size, dtype=torch.int32, device="cuda")
                svb.svb_delta_decode(x.size, d, d.numel(), o, 1, None, st)
                outs.append((o, d))
        torch.cuda.synchronize()
        for (o, _), x in zip(outs, xs):
            np.testing.assert_array_equal(u32_host(o), x)


# ------------------------------------------------------------------ full-size workloads

@pytest.mark.slow
def test_docids_2pow26_delta_full():
    """2^26 sorted document ids, delta encode and delta decode, against the oracle in full."""
    x, g = inputs.docids(1 << 26, seed=2)
    check_round_trip(x, delta=True, start=0, tag="docids_2^26")


@pytest.mark.slow
def test_stress_2pow28_plain_decode_full():
    """2^28 integers with unpredictable lengths: plain decode in full, and delta decode of the
    same bytes read as gaps; encode too."""
    x = inputs.stress_lengths(1 << 28, seed=3)
    ref = oracle.encode(x)
    log_case("stress_2^28", "decode")
    vals, err = gpu_decode(ref, x.size)
    assert err == 0
    assert np.array_equal(vals, x)
    del vals
    log_case("stress_2^28", "delta decode")
    dvals, err = gpu_decode(ref, x.size, delta=True, start=0)
    assert err == 0
    assert np.array_equal(dvals, np.cumsum(x, dtype=np.uint32))
    del dvals
    log_case("stress_2^28", "encode")
    got, sz = gpu_encode(x)
    assert sz == ref.size and np.array_equal(got, ref)


@pytest.mark.slow
def test_docids_2pow28_delta_decode_full():
    x, _ = inputs.docids(1 << 28, seed=2)
    ref = oracle.encode(x, delta=True, start=0)
    log_case("docids_2^28", "delta decode")
    vals, err = gpu_decode(ref, x.size, delta=True, start=0)
    assert err == 0
    assert np.array_equal(vals, x)
