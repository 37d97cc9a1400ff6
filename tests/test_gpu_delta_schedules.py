"""GPU parity of the delta decoder's two ways of taking the value sums, through the C ABI, against
the oracle.

Delta decoding needs, for every group of integers, the sum of all differences stored before it.
Variant bit 1 clear: each group's sum from its plain byte sum plus a correction per block of
multi-byte integers, read from the span staged in LDS (or, past the staged part, from memory).
Bit 1 set: each group's sum by decoding it.  Bit 0 picks the zero-control decoder.  All four, and
the automatic choice, must equal the oracle exactly, on streams of every shape the byte sum treats
differently: one-byte differences (no corrections), every length (corrections on nearly every
block, spans past the staged part), partial last groups and blocks, byte misalignment, corrupt
streams, and calls of changing sizes in a row.
"""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u8, u32_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

GROUP = 4096
VARIANTS = [-1, 0, 1, 2, 3]  # -1: the automatic choice
SIZES = [1, 2, 3, 4, 5, 63, 64, 65, 1023, 1024, 1025, GROUP - 1, GROUP, GROUP + 1, 2 * GROUP + 3,
         5 * GROUP - 2, 64 * GROUP + 7, 257 * GROUP + 1, 250_001]


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()
    svb.svb_set_decode_variant(True, -1)


def kinds(n, seed):
    """Value arrays whose delta streams differ in what the byte sum does with them."""
    rng = np.random.default_rng(seed)
    docids, _ = inputs.docids(n, seed=seed, start=int(rng.integers(0, 1 << 32)))
    every_len = np.cumsum(inputs.stress_lengths(n, seed=seed), dtype=np.uint32)
    wide = inputs.random_u32(n, seed=seed)
    small = np.cumsum(rng.integers(0, 256, size=n, dtype=np.uint64), dtype=np.uint64).astype(np.uint32)
    return {"docids": docids, "every_length": every_len, "random": wide, "one_byte": small}


def decode(stream, n, start, variant, shift=0, trailing=0):
    svb.svb_set_decode_variant(True, variant)
    buf = np.concatenate([np.full(shift, 0x33, np.uint8), stream, np.full(trailing, 0xEE, np.uint8)])
    d = to_dev_u8(buf)
    out = torch.full((n + 4,), 0x7EADBEEF, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    svb.svb_delta_decode(n, d.data_ptr() + shift, stream.size + trailing, out, start, err)
    torch.cuda.synchronize()
    host = u32_host(out)
    assert np.all(host[n:] == 0x7EADBEEF), "written past n"
    return host[:n].copy(), int(err.item())


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", SIZES)
def test_schedules_match_oracle(n, variant):
    for name, x in kinds(n, seed=n).items():
        start = int(x[0]) ^ 0x5A5A5A5A
        ref = oracle.encode(x, delta=True, start=start)
        log_case("delta schedule", "variant=%d" % variant, "n=%d" % n, name)
        got, err = decode(ref, n, start, variant, shift=n % 7, trailing=n % 5)
        assert err == 0
        np.testing.assert_array_equal(got, x, err_msg="%s n=%d variant=%d" % (name, n, variant))


@pytest.mark.parametrize("variant", VARIANTS)
def test_random_streams_with_garbage_tail_codes(variant):
    """Random control bytes (garbage in the unused codes of the last block) and random data: the
    corrections see blocks of every length pattern, partial last blocks included."""
    for n in (1, 2, 3, 5, 6, 7, 4097, 4098, 4099, 3 * GROUP + 1, 40_003):
        k = (n + 3) // 4
        ctrl = inputs.random_bytes(k, seed=500 + n)
        codes = (ctrl[np.arange(n) // 4].astype(np.uint32) >> (2 * (np.arange(n) % 4)).astype(np.uint32)) & 3
        stream = np.concatenate([ctrl, inputs.random_bytes(int(codes.sum()) + n, seed=600 + n)])
        ref, used = oracle.decode(stream, n, delta=True, start=99)
        assert used == stream.size
        log_case("delta random stream", "variant=%d" % variant, "n=%d" % n)
        got, err = decode(stream, n, 99, variant)
        assert err == 0
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("variant", VARIANTS)
def test_truncated_streams_flag_corrupt(variant):
    for n in (5, 4099, 3 * GROUP, 70_001):
        x = inputs.stress_lengths(n, seed=n)
        ref = oracle.encode(x, delta=True)
        for cut in (1, 3, 40):
            if cut > ref.size - (n + 3) // 4:
                continue
            log_case("delta truncated", "variant=%d" % variant, "n=%d" % n, "cut=%d" % cut)
            _, err = decode(ref[:-cut], n, 0, variant)
            assert err == svb.SVB_DECODE_CORRUPT


@pytest.mark.parametrize("variant", [-1, 0, 2])
def test_calls_of_changing_size_in_a_row(variant):
    """The library's scratch lives across calls: large, small, large again, with different starts,
    on one stream and on a second one, each checked."""
    sizes = [300 * GROUP + 5, 3, GROUP + 1, 100 * GROUP, 1, 300 * GROUP + 5, 17 * GROUP - 1]
    xs = [inputs.docids(n, seed=70 + i, start=i * 1_000_003)[0] for i, n in enumerate(sizes)]
    refs = [oracle.encode(x, delta=True, start=i * 7) for i, x in enumerate(xs)]
    svb.svb_set_decode_variant(True, variant)
    s2 = torch.cuda.Stream()
    for rep in range(2):
        outs = []
        for i, (x, ref) in enumerate(zip(xs, refs)):
            st = s2 if (rep == 1 and i % 2) else torch.cuda.current_stream()
            with torch.cuda.stream(st):
                d = to_dev_u8(ref)
                o = torch.empty(x.size, dtype=torch.int32, device="cuda")
                svb.svb_delta_decode(x.size, d, d.numel(), o, i * 7, None, st)
                outs.append((o, d))
        torch.cuda.synchronize()
        for i, ((o, _), x) in enumerate(zip(outs, xs)):
            log_case("delta changing sizes", "variant=%d" % variant, "rep=%d" % rep, "call=%d" % i)
            np.testing.assert_array_equal(u32_host(o), x)


def test_many_calls_reuse_the_scratch():
    """200 calls in a row on one stream, sizes cycling, the last of each size checked."""
    xs = [inputs.docids(n, seed=90 + n, start=n)[0] for n in (GROUP * 9 + 1, 77, GROUP * 33)]
    refs = [to_dev_u8(oracle.encode(x, delta=True, start=5)) for x in xs]
    outs = [torch.empty(x.size, dtype=torch.int32, device="cuda") for x in xs]
    svb.svb_set_decode_variant(True, -1)
    log_case("delta many calls")
    for k in range(200):
        i = k % 3
        svb.svb_delta_decode(xs[i].size, refs[i], refs[i].numel(), outs[i], 5)
    torch.cuda.synchronize()
    for o, x in zip(outs, xs):
        np.testing.assert_array_equal(u32_host(o), x)


@pytest.mark.parametrize("variant", [-1, 0, 2])
def test_more_than_five_thousand_groups(variant):
    """More than 5,000 groups (multi-tile scans of the offsets and of the sums, with sums whose top
    bit is set); document ids and every-length values (spans past the staged part), compared in
    full."""
    n = 1300 * 4 * GROUP + 5
    for name, x in (("docids", inputs.docids(n, seed=31, start=12345)[0]),
                    ("every_length", np.cumsum(inputs.stress_lengths(n, seed=32), dtype=np.uint32))):
        ref = oracle.encode(x, delta=True, start=17)
        log_case("delta many groups", "variant=%d" % variant, name, "n=%d" % n)
        got, err = decode(ref, n, 17, variant)
        assert err == 0
        np.testing.assert_array_equal(got, x, err_msg=name)
