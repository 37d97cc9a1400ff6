"""GPU parity of seek and select on resident compressed lists (svb_seek_batch / svb_select_batch)
against the oracle's walk over each list's own stream: positions and values exactly equal."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")

U64_MAX = 0xFFFFFFFFFFFFFFFF


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()


def dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


class Lists:
    """Lists encoded by the oracle, packed at arbitrary byte offsets, with a seek index."""

    def __init__(self, lists, delta, starts=None, seed=0, in_bytes_override=None):
        self.lists = [np.asarray(x, dtype=np.uint32) for x in lists]
        self.m = len(lists)
        self.delta = delta
        self.starts = (np.zeros(self.m, np.uint32) if starts is None else np.asarray(starts, np.uint32)) if delta \
            else None
        self.streams = [oracle.encode(x, delta=delta, start=0 if not delta else int(self.starts[i]))
                        for i, x in enumerate(self.lists)]
        rng = np.random.default_rng(seed)
        sizes = np.array([s.size for s in self.streams], dtype=np.uint64)
        gaps = rng.integers(0, 9, size=self.m).astype(np.uint64)
        in_off = np.zeros(self.m, dtype=np.uint64)
        if self.m > 1:
            np.cumsum(sizes[:-1] + gaps[:-1], out=in_off[1:])
        buf = np.zeros(int(in_off[-1] + sizes[-1] + 16) if self.m else 16, dtype=np.uint8)
        for o, s in zip(in_off, self.streams):
            buf[int(o):int(o) + s.size] = s
        in_bytes = sizes.copy()
        for i, v in (in_bytes_override or {}).items():
            in_bytes[i] = v
        self.counts = np.array([x.size for x in self.lists], dtype=np.uint64)
        self.dev = (dev_u64(self.counts), dev_u64(in_off), dev_u64(in_bytes), to_dev_u8(buf),
                    None if self.starts is None else to_dev_u32(self.starts))
        self.index = svb.svb_seek_index_create(self.m, *self.dev, int(self.counts.sum()) + 1)

    def close(self):
        if self.index:
            svb.svb_seek_index_destroy(self.index)
            self.index = None

    def start(self, i):
        return int(self.starts[i]) if self.delta else 0

    def seek(self, ids, targets):
        q = len(ids)
        pos = torch.full((max(1, q),), -7, dtype=torch.int64, device="cuda")
        val = torch.full((max(1, q),), -7, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        svb.svb_seek_batch(self.index, q, to_dev_u32(np.asarray(ids, np.uint32)),
                           to_dev_u32(np.asarray(targets, np.uint32)), pos, val, err)
        torch.cuda.synchronize()
        return pos.cpu().numpy().view(np.uint64)[:q], u32_host(val)[:q], int(err.item())

    def select(self, ids, idx):
        q = len(ids)
        val = torch.full((max(1, q),), -7, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        svb.svb_select_batch(self.index, q, to_dev_u32(np.asarray(ids, np.uint32)), dev_u64(idx), val, err)
        torch.cuda.synchronize()
        return u32_host(val)[:q], int(err.item())

    def check(self, ids, targets, idx, tag):
        log_case("seek", tag, "m=%d" % self.m, "q=%d" % len(ids), "delta=%s" % self.delta)
        pos, val, err = self.seek(ids, targets)
        assert err == 0, tag
        for k, (l, t) in enumerate(zip(ids, targets)):
            want = oracle.seek(self.streams[l], self.lists[l].size, int(t), self.delta, self.start(l))
            assert (int(pos[k]), int(val[k])) == want, (tag, k, int(l), int(t))
        log_case("select", tag, "m=%d" % self.m, "q=%d" % len(ids))
        keep = [k for k, l in enumerate(ids) if self.lists[l].size > 0]
        sids = [ids[k] for k in keep]
        sidx = np.array([idx[k] for k in keep], dtype=np.uint64)
        got, err = self.select(sids, sidx)
        assert err == 0, tag
        for k, (l, i) in enumerate(zip(sids, sidx)):
            want = oracle.select(self.streams[l], self.lists[l].size, int(i), self.delta, self.start(l))
            assert int(got[k]) == want, (tag, k, int(l), int(i))


def edge_queries(lists):
    """For every list: targets 0, each segment's first and last value, one past them, the list's
    first and last value and one past the last; positions 0, each segment boundary and the end."""
    ids, targets, idx = [], [], []
    for l, x in enumerate(lists):
        n = x.size
        pts = {0, n - 1} | {s for s in range(0, n, 1024)} | {min(n - 1, s + 1023) for s in range(0, n, 1024)}
        pts = sorted(p for p in pts if 0 <= p < n)
        ts = {0, 0xFFFFFFFF} | {int(x[p]) for p in pts} | {min(int(x[p]) + 1, 0xFFFFFFFF) for p in pts}
        for t in sorted(ts):
            ids.append(l)
            targets.append(t)
            idx.append(pts[len(ids) % len(pts)] if pts else 0)
    return ids, targets, idx


@pytest.mark.parametrize("bits", [1, 8, 9, 24])
def test_seek_select_paper_workload(bits):
    """Section 5's seek/select workload: lists of 256 running sums of deltas below 2^b."""
    vals, offs = inputs.seek_lists(3_000, bits, seed=200 + bits)
    lists = [vals[offs[i]:offs[i + 1]] for i in range(offs.size - 1)]
    L = Lists(lists, delta=True, seed=bits)
    ids, targets, idx = inputs.seek_queries(vals, offs, 4_000, seed=300 + bits)
    L.check(list(ids), list(targets), list(idx), "b=%d" % bits)
    e_ids, e_t, e_i = edge_queries(lists[:40])
    L.check(e_ids, e_t, e_i, "b=%d edges" % bits)
    L.close()


@pytest.mark.parametrize("delta", [True, False])
def test_seek_select_posting_lists(delta):
    """Long posting lists (up to 2^18 integers, so up to 256 segments: the search takes two steps),
    random and boundary queries."""
    vals, offs = inputs.posting_lists(m=400, total=3_000_000, cap=1 << 18, seed=41)
    lists = [vals[offs[i]:offs[i + 1]] for i in range(offs.size - 1)]
    starts = np.arange(len(lists), dtype=np.uint32) * 17 if delta else None
    # delta lists are the sets shifted by their start, so the values stay sorted
    if delta:
        lists = [(x.astype(np.uint64) + int(s)).astype(np.uint32) for x, s in zip(lists, starts)]
    L = Lists(lists, delta=delta, starts=starts, seed=42)
    ids, targets, idx = inputs.seek_queries(np.concatenate(lists), offs, 3_000, seed=43)
    L.check(list(ids), list(targets), list(idx), "posting")
    big = list(np.argsort([x.size for x in lists])[::-1][:6])
    e_ids, e_t, e_i = edge_queries([lists[b] for b in big])
    L.check([big[i] for i in e_ids], e_t, e_i, "posting edges")
    L.close()


@pytest.mark.parametrize("delta", [False, True])
def test_seek_unsorted_lists(delta):
    """Unsorted lists (plain random values; delta lists whose differences wrap modulo 2^32):
    seek still returns the first position at or above the target."""
    rng = np.random.default_rng(51 + delta)
    sizes = [1, 2, 3, 5, 255, 256, 1023, 1024, 1025, 3000, 9000, 70_000]
    lists = [(rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
              >> rng.integers(0, 32, size=n).astype(np.uint64)).astype(np.uint32) for n in sizes]
    starts = rng.integers(0, 1 << 32, size=len(sizes), dtype=np.uint64).astype(np.uint32) if delta else None
    L = Lists(lists, delta=delta, starts=starts, seed=53)
    ids, targets, idx = [], [], []
    for l, x in enumerate(lists):
        for t in list(rng.integers(0, 1 << 32, size=60, dtype=np.uint64)) + [int(v) for v in x[:: max(1, x.size // 20)]]:
            ids.append(l)
            targets.append(int(t))
            idx.append(int(rng.integers(0, x.size)))
    L.check(ids, targets, idx, "unsorted")
    L.close()


def test_empty_lists_and_refusals():
    lists = [np.zeros(0, np.uint32), np.arange(10, 5000, 3, dtype=np.uint32), np.zeros(0, np.uint32),
             np.array([7], np.uint32)]
    L = Lists(lists, delta=True, seed=61)
    log_case("seek empty and refusals")
    pos, val, err = L.seek([0, 1, 2, 3, 3], [0, 11, 5, 7, 8])
    assert err == 0
    assert [int(p) for p in pos] == [0, 1, 0, 0, 1] and [int(v) for v in val] == [0, 13, 0, 7, 0]
    # a list id past the index's last list
    pos, val, err = L.seek([1, 4, 1], [0, 0, 5000])
    assert err == svb.SVB_QUERY_OUT_OF_RANGE
    assert int(pos[1]) == U64_MAX and int(val[1]) == 0
    assert (int(pos[0]), int(val[0])) == (0, 10) and (int(pos[2]), int(val[2])) == (lists[1].size, 0)
    # select past a list's end (and on an empty list)
    got, err = L.select([1, 1, 0, 3], np.array([lists[1].size - 1, lists[1].size, 0, 0], np.uint64))
    assert err == svb.SVB_QUERY_OUT_OF_RANGE
    assert int(got[0]) == int(lists[1][-1]) and int(got[1]) == 0 and int(got[2]) == 0 and int(got[3]) == 7
    L.close()


def test_index_refuses_corrupt_list():
    lists = [np.arange(1, 3000, dtype=np.uint32) * 1000, np.arange(5, dtype=np.uint32)]
    log_case("seek index corrupt")
    with pytest.raises(svb.SvbError):
        Lists(lists, delta=True, seed=71, in_bytes_override={0: oracle.encode(lists[0], delta=True).size - 2})


def test_seek_select_full_size_sampled():
    """The measured configuration (2^20 lists of 256 integers, deltas below 2^8, 2^20 queries of
    each kind in one call), checked on a sample of the answers."""
    m, bits, q = 1 << 20, 8, 1 << 20
    vals, offs = inputs.seek_lists(m, bits, seed=81)
    log_case("seek full size", "m=%d" % m, "q=%d" % q)
    cap = svb.svb_max_compressed_bytes(256)  # each stream's reserved region
    comp = torch.empty(m * cap, dtype=torch.uint8, device="cuda")
    x_dev = torch.from_numpy(vals.view(np.int32)).cuda()
    counts = np.full(m, 256, dtype=np.uint64)
    byte_off = np.arange(m, dtype=np.uint64) * cap
    sizes = torch.empty(m, dtype=torch.int64, device="cuda")
    starts = torch.zeros(m, dtype=torch.int32, device="cuda")
    svb.svb_encode_batch(m, dev_u64(counts), dev_u64(offs[:-1]), x_dev, dev_u64(byte_off), comp, sizes, starts,
                         256 * m)
    torch.cuda.synchronize()
    # deltas below 2^8: 64 control bytes and 256 one-byte integers per list
    assert np.all(sizes.cpu().numpy() == 320)
    index = svb.svb_seek_index_create(m, dev_u64(counts), dev_u64(byte_off), sizes, comp, starts, 256 * m)
    ids, targets, idx = inputs.seek_queries(vals, offs, q, seed=82)
    pos = torch.empty(q, dtype=torch.int64, device="cuda")
    val = torch.empty(q, dtype=torch.int32, device="cuda")
    sval = torch.empty(q, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_ids = to_dev_u32(ids)
    svb.svb_seek_batch(index, q, d_ids, to_dev_u32(targets), pos, val, err)
    svb.svb_select_batch(index, q, d_ids, dev_u64(idx), sval, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    pos_h, val_h, sval_h = pos.cpu().numpy(), u32_host(val), u32_host(sval)
    comp_h = comp.cpu().numpy().view(np.uint8)
    for k in np.random.default_rng(83).integers(0, q, size=3_000):
        l = int(ids[k])
        s = comp_h[l * cap:l * cap + 320]
        assert (int(pos_h[k]), int(val_h[k])) == oracle.seek(s, 256, int(targets[k]), True, 0), k
        assert int(sval_h[k]) == oracle.select(s, 256, int(idx[k]), True, 0), k
    svb.svb_seek_index_destroy(index)
