"""GPU parity of the batched calls (svb_encode_batch / svb_decode_batch) against the oracle applied to
each list on its own: streams byte for byte, sizes, decoded values, corruption flags."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host, u8_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

CHUNKS = [1, 2, 4, 8, 16]
EDGE_SIZES = [0, 1, 3, 4, 5, 63, 64, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095,
              4096, 4097, 8191, 8192, 8193, 16385, 40000, 100003]
SENTINEL32 = 0x5EEDF00D
SENTINEL8 = 0xA7


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()
    for kind in range(4):
        svb.svb_set_batch_chunk(kind, 4)


def dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


def make_lists(sizes, seed, delta):
    rng = np.random.default_rng(seed)
    lists = []
    for i, n in enumerate(sizes):
        if delta and i % 2 == 0:
            x, _ = inputs.docids(int(n), seed=seed * 1000 + i, start=int(rng.integers(0, 1 << 32)))
        else:
            x = (inputs.random_u32(int(n), seed=seed * 1000 + i)
                 >> rng.integers(0, 32, size=int(n)).astype(np.uint32)).astype(np.uint32)
        lists.append(np.asarray(x, dtype=np.uint32))
    starts = rng.integers(0, 1 << 32, size=len(sizes), dtype=np.uint64).astype(np.uint32) if delta else None
    return lists, starts


def layout(lengths, seed, unit_gap):
    """Offsets with random gaps between consecutive regions (unit_gap: max gap in units)."""
    rng = np.random.default_rng(seed)
    offs, pos = [], 0
    for n in lengths:
        pos += int(rng.integers(0, unit_gap + 1))
        offs.append(pos)
        pos += int(n)
    return np.array(offs, dtype=np.uint64), pos


def run_decode_batch(streams, counts, starts, seed, total_ints=None, in_bytes_override=None):
    m = len(counts)
    in_off, in_total = layout([s.size for s in streams], seed, 7)  # arbitrary byte alignment
    buf = np.full(max(1, in_total + 16), 0xEE, dtype=np.uint8)
    for o, s in zip(in_off, streams):
        buf[int(o):int(o) + s.size] = s
    in_bytes = np.array([s.size for s in streams], dtype=np.uint64)
    if in_bytes_override is not None:
        for i, v in in_bytes_override.items():
            in_bytes[i] = v
    out_off, out_total = layout(counts, seed + 1, 5)
    out = torch.full((max(1, out_total + 8),), SENTINEL32, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    total = int(np.sum(np.asarray(counts, dtype=np.uint64))) if total_ints is None else total_ints
    svb.svb_decode_batch(m, dev_u64(counts), dev_u64(in_off), dev_u64(in_bytes), to_dev_u8(buf), dev_u64(out_off),
                         out, None if starts is None else to_dev_u32(starts), total, err)
    torch.cuda.synchronize()
    host = u32_host(out)
    outs = [host[int(o):int(o) + int(n)] for o, n in zip(out_off, counts)]
    # nothing is written outside the lists' ranges
    mask = np.ones(host.size, dtype=bool)
    for o, n in zip(out_off, counts):
        mask[int(o):int(o) + int(n)] = False
    assert np.all(host[mask] == SENTINEL32)
    return outs, int(err.item())


def run_encode_batch(lists, starts, seed, total_ints=None):
    m = len(lists)
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    in_off, in_total = layout(counts, seed, 3)
    vals = np.zeros(max(1, in_total), dtype=np.uint32)
    for o, x in zip(in_off, lists):
        vals[int(o):int(o) + x.size] = x
    caps = [svb.svb_max_compressed_bytes(int(n)) for n in counts]
    out_off, out_total = layout(caps, seed + 2, 9)
    out = torch.full((max(1, out_total + 16),), SENTINEL8, dtype=torch.uint8, device="cuda")
    sizes = torch.full((m,), -1, dtype=torch.int64, device="cuda")
    total = int(counts.sum()) if total_ints is None else total_ints
    svb.svb_encode_batch(m, dev_u64(counts), dev_u64(in_off), to_dev_u32(vals), dev_u64(out_off), out, sizes,
                         None if starts is None else to_dev_u32(starts), total)
    torch.cuda.synchronize()
    host = u8_host(out)
    sz = sizes.cpu().numpy().view(np.uint64)
    return [host[int(o):int(o) + int(min(s, c))] for o, s, c in zip(out_off, sz, caps)], sz, host, out_off, caps


def check_batch(lists, starts, seed, tag):
    delta = starts is not None
    refs = oracle.encode_lists(lists, delta=delta, starts=starts)
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    log_case("batch encode", tag, "m=%d" % len(lists), "delta=%s" % delta)
    got, sizes, host, out_off, caps = run_encode_batch(lists, starts, seed)
    for i, r in enumerate(refs):
        assert int(sizes[i]) == r.size, (tag, i)
        np.testing.assert_array_equal(got[i], r, err_msg="%s list %d" % (tag, i))
        # bytes of the reserved region past the stream are untouched
        tail = host[int(out_off[i]) + r.size:int(out_off[i]) + caps[i]]
        assert np.all(tail == SENTINEL8), (tag, i)
    log_case("batch decode", tag, "m=%d" % len(lists), "delta=%s" % delta)
    outs, err = run_decode_batch(refs, counts, starts, seed)
    assert err == 0
    for i, x in enumerate(lists):
        np.testing.assert_array_equal(outs[i], x, err_msg="%s list %d" % (tag, i))


@pytest.mark.parametrize("delta", [False, True])
@pytest.mark.parametrize("chunk", CHUNKS)
def test_batch_edge_sizes(chunk, delta):
    for kind in range(4):
        svb.svb_set_batch_chunk(kind, chunk)
    lists, starts = make_lists(EDGE_SIZES, seed=11 + chunk, delta=delta)
    check_batch(lists, starts, seed=5 + chunk, tag="edges chunk=%d" % chunk)


SVB_BATCH_QUEUE = 0x100


@pytest.mark.parametrize("delta", [False, True])
@pytest.mark.parametrize("chunk", [1, 2, 4, 8])
def test_batch_work_queue_schedule(chunk, delta):
    """The decode walk's work-queue schedule (waves grab chunks of tasks from a device counter):
    the edge sizes, and 70,000 mostly tiny lists (more tasks than the grid's waves take in one
    grab each), against the oracle; the queue is refused for encoding."""
    for kind in (2, 3):
        with pytest.raises(svb.SvbError):
            svb.svb_set_batch_chunk(kind, SVB_BATCH_QUEUE | chunk)
        svb.svb_set_batch_chunk(kind, 4)
    for kind in (0, 1):
        svb.svb_set_batch_chunk(kind, SVB_BATCH_QUEUE | chunk)
    lists, starts = make_lists(EDGE_SIZES, seed=61 + chunk, delta=delta)
    check_batch(lists, starts, seed=62 + chunk, tag="queue edges chunk=%d" % chunk)
    rng = np.random.default_rng(63 + chunk)
    sizes = rng.integers(0, 300, size=70_000)
    lists, starts = make_lists(sizes, seed=64 + chunk, delta=delta)
    check_batch(lists, starts, seed=65 + chunk, tag="queue many chunk=%d" % chunk)
    for kind in (0, 1):
        svb.svb_set_batch_chunk(kind, 4)


@pytest.mark.parametrize("delta", [False, True])
def test_batch_many_small_lists(delta):
    """70,000 lists (more than 16384 lists and tasks), so the scans take the multi-workgroup path."""
    rng = np.random.default_rng(21)
    sizes = rng.integers(0, 48, size=70_000)
    sizes[::9_973] = rng.integers(9_000, 30_000, size=sizes[::9_973].size)
    lists, starts = make_lists(sizes, seed=22, delta=delta)
    for kind in range(4):
        svb.svb_set_batch_chunk(kind, 16)
    check_batch(lists, starts, seed=23, tag="many")


def test_batch_posting_lists_sample():
    """Posting-list shaped batch (rank-size Zipf lengths, sorted sets), delta-coded."""
    vals, offs = inputs.posting_lists(m=3_000, total=4_000_000, cap=1 << 17, seed=31)
    lists = [vals[offs[i]:offs[i + 1]] for i in range(offs.size - 1)]
    starts = np.zeros(len(lists), dtype=np.uint32)
    check_batch(lists, starts, seed=32, tag="posting")


def test_batch_corrupt_list_is_flagged_and_others_decode():
    lists, _ = make_lists([5000, 300, 12000, 7], seed=41, delta=False)
    refs = oracle.encode_lists(lists)
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    log_case("batch corrupt")
    # list 1: in_bytes below its control stream; list 2: truncated data
    outs, err = run_decode_batch(refs, counts, None, seed=42, in_bytes_override={1: 10, 2: refs[2].size - 3})
    assert err == svb.SVB_DECODE_CORRUPT
    for i in (0, 3):
        np.testing.assert_array_equal(outs[i], lists[i])


def test_batch_bound_overflow_does_nothing():
    lists, starts = make_lists([9000, 9000, 100], seed=51, delta=True)
    refs = oracle.encode_lists(lists, delta=True, starts=starts)
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    log_case("batch overflow")
    outs, err = run_decode_batch(refs, counts, starts, seed=52, total_ints=100)
    assert err == svb.SVB_BATCH_OVERFLOW
    for o in outs:
        assert np.all(o == SENTINEL32)
    _, sizes, _, _, _ = run_encode_batch(lists, starts, seed=53, total_ints=100)
    assert np.all(sizes == np.uint64(0xFFFFFFFFFFFFFFFF))


def test_batch_autotune_then_decode():
    vals, offs = inputs.posting_lists(m=1_000, total=2_000_000, cap=1 << 16, seed=61)
    lists = [vals[offs[i]:offs[i + 1]] for i in range(offs.size - 1)]
    starts = np.arange(len(lists), dtype=np.uint32)
    refs = oracle.encode_lists(lists, delta=True, starts=starts)
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    in_off, in_total = layout([s.size for s in refs], 62, 0)
    buf = np.zeros(in_total, dtype=np.uint8)
    for o, s in zip(in_off, refs):
        buf[int(o):int(o) + s.size] = s
    out_off, out_total = layout(counts, 63, 0)
    out = torch.zeros(out_total, dtype=torch.int32, device="cuda")
    d_args = (len(lists), dev_u64(counts), dev_u64(in_off), dev_u64([s.size for s in refs]), to_dev_u8(buf),
              dev_u64(out_off), out, to_dev_u32(starts), int(counts.sum()))
    log_case("batch autotune")
    g = svb.svb_autotune_decode_batch(*d_args)
    assert g in CHUNKS
    out.zero_()
    svb.svb_decode_batch(*d_args)
    torch.cuda.synchronize()
    host = u32_host(out)
    for i, x in enumerate(lists):
        np.testing.assert_array_equal(host[int(out_off[i]):int(out_off[i]) + x.size], x)
