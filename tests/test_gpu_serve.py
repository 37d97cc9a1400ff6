"""GPU tests of the serving runtime: continuous batching with admission by memory gives every query
exactly the result it gets alone, and both equal the oracle's decode of the query's lists."""
import numpy as np
import pytest

import oracle
from paper_1709_08990_amd import inputs
from tests.gpu_util import log_case, to_dev_u32, to_dev_u8, u32_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
svb = pytest.importorskip("paper_1709_08990_amd")
from paper_1709_08990_amd import serve  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    svb.lib()
    yield
    torch.cuda.synchronize()


def dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


def make_pool(m, total, cap, delta, seed):
    vals, offs = inputs.posting_lists(m=m, total=total, cap=cap, seed=seed)
    lists = [vals[offs[i]:offs[i + 1]] for i in range(m)]
    starts = (np.arange(m, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32) if delta else None
    streams = oracle.encode_lists(lists, delta=delta, starts=starts)
    sizes = np.array([s.size for s in streams], dtype=np.uint64)
    in_off = np.zeros(m, dtype=np.uint64)
    np.cumsum(sizes[:-1] + 3, out=in_off[1:])   # 3 bytes of gap: streams at any alignment
    buf = np.zeros(int(in_off[-1] + sizes[-1] + 8), dtype=np.uint8)
    for o, s in zip(in_off, streams):
        buf[int(o):int(o) + s.size] = s
    counts = np.array([x.size for x in lists], dtype=np.uint64)
    dev = dict(counts=dev_u64(counts), in_off=dev_u64(in_off), in_bytes=dev_u64(sizes), streams=to_dev_u8(buf),
               starts=None if starts is None else to_dev_u32(starts))
    return lists, starts, counts, dev


def expected(lists, starts, delta, pick):
    # the oracle decodes each list of the query from its own stream
    outs = []
    for l in pick:
        s = oracle.encode(lists[l], delta=delta, start=0 if starts is None else int(starts[l]))
        v, _ = oracle.decode(s, lists[l].size, delta=delta, start=0 if starts is None else int(starts[l]))
        outs.append(v)
    return np.concatenate(outs) if outs else np.zeros(0, np.uint32)


def read_result(server, off, n):
    out = torch.empty(max(1, n), dtype=torch.int32, device="cuda")
    if n:
        svb.svb_copy_u32(n, svb.svb_server_arena(server.handle) + 4 * off, out)
    torch.cuda.synchronize()
    return u32_host(out)[:n].copy()


def read_result_on(server, off, n, stream):
    """Reads a result on its own stream and waits for that stream only: the server's batches on
    its slot streams keep running meanwhile."""
    with torch.cuda.stream(stream):
        out = torch.empty(max(1, n), dtype=torch.int32, device="cuda")
        if n:
            svb.svb_copy_u32(n, svb.svb_server_arena(server.handle) + 4 * off, out, stream=stream)
        host = u32_host(out)[:n].copy()
    return host


@pytest.mark.parametrize("delta", [True, False])
def test_results_alone_equal_results_in_the_mix(delta):
    lists, starts, counts, dev = make_pool(3_000, 3_000_000, 1 << 16, delta, seed=71 if delta else 72)
    # arrivals faster than the batches finish, so that batches launched while others are still on
    # the device run alongside them
    times, picks = inputs.poisson_queries(300, qps=200_000.0, n_lists=len(lists), seed=73)
    # an arena of 2 MiB holds only a few dozen average queries at once: admission throttles
    arena = 2 << 20
    need = [int(counts[p].sum()) * 4 for p in picks]
    assert max(need) <= arena
    # small batches that leave as soon as a slot is free: a step launches several at once
    server = serve.Server(dev["counts"], dev["in_off"], dev["in_bytes"], dev["streams"], dev["starts"],
                          arena_bytes=arena, slots=4, max_batch_lists=8)
    server.set_batching(0, 0)
    mixed = {}
    log_case("serve mix", "delta=%s" % delta)
    cs = torch.cuda.Stream()
    lat, wall = serve.run_open_loop(server, times, picks,
                                    on_result=lambda q, off, n: mixed.__setitem__(q, read_result_on(server, off, n, cs)))
    st = server.stats()
    assert st["completed"] == len(picks) and st["admitted"] == len(picks)
    assert st["err"] == 0
    assert st["batches"] > 1
    assert st["peak_busy_slots"] >= 2, "no two batches were on the device together"
    assert st["arena_peak_ints"] * 4 <= arena
    assert np.all(lat > 0)
    # every result equals the oracle's decode of its lists
    for q, p in enumerate(picks):
        np.testing.assert_array_equal(mixed[q], expected(lists, starts, delta, p), err_msg="query %d" % q)
    # a sample of queries alone, one at a time on a fresh server: same bytes
    server.close()
    alone_server = serve.Server(dev["counts"], dev["in_off"], dev["in_bytes"], dev["streams"], dev["starts"],
                                arena_bytes=arena, slots=1, max_batch_lists=256)
    log_case("serve alone", "delta=%s" % delta)
    for q in range(0, len(picks), 7):
        alone_server.submit(10_000 + q, picks[q])
        got = []
        while not got:
            alone_server.step(block=True)
            got = alone_server.poll()
        (qid, off, n), = got
        assert qid == 10_000 + q
        np.testing.assert_array_equal(read_result(alone_server, off, n), mixed[q], err_msg="query %d alone" % q)
        alone_server.release(qid)
    assert alone_server.stats()["batches"] == len(range(0, len(picks), 7))
    alone_server.close()


def test_overlapping_batches_and_refusals():
    lists, starts, counts, dev = make_pool(500, 600_000, 1 << 14, True, seed=81)
    server = serve.Server(dev["counts"], dev["in_off"], dev["in_bytes"], dev["streams"], dev["starts"],
                          arena_bytes=1 << 20, slots=3, max_batch_lists=64)
    # a query larger than the arena, and one with more lists than a batch holds, are refused
    big = np.argsort(counts)[::-1][:200]
    if int(counts[big].sum()) * 4 > (1 << 20):
        with pytest.raises(svb.SvbError):
            server.submit(1, big[:64])
    with pytest.raises(svb.SvbError):
        server.submit(2, np.arange(65))
    _, picks = inputs.poisson_queries(200, qps=1.0, n_lists=len(lists), seed=82)
    log_case("serve closed loop")
    lat, wall = serve.run_closed_loop(server, picks, outstanding=32)
    st = server.stats()
    assert st["completed"] == 200 and st["err"] == 0
    assert st["waiting"] == 0 and st["admitted_not_launched"] == 0 and st["arena_in_use_ints"] == 0
    server.close()


def test_replay_open_and_closed_loop():
    lists, starts, counts, dev = make_pool(2_000, 1_500_000, 1 << 15, True, seed=91)
    server = serve.Server(dev["counts"], dev["in_off"], dev["in_bytes"], dev["streams"], dev["starts"],
                          arena_bytes=4 << 20, slots=4, max_batch_lists=512)
    times, qoff, ids = inputs.poisson_queries_flat(3_000, 20_000.0, len(lists), seed=92)
    # queries of the ordinary interface, queued before the replay, ride along in its batches
    mine = {100 + q: ids[qoff[q]:qoff[q + 1]] for q in range(5)}
    for qid, p in mine.items():
        server.submit(qid, p)
    log_case("serve replay open loop")
    lat, wall = server.replay((qoff, ids), arrivals=times)
    got = {}
    while len(got) < len(mine):
        server.step(block=True)
        for qid, off, n in server.poll():
            got[qid] = read_result(server, off, n)
            server.release(qid)
    for qid, p in mine.items():
        np.testing.assert_array_equal(got[qid], expected(lists, starts, True, p), err_msg="query %d" % qid)
    assert lat.size == 3_000 and np.all(lat > 0) and wall >= times[-1]
    log_case("serve replay closed loop")
    lat2, _ = server.replay((qoff, ids), outstanding=64)
    assert lat2.size == 3_000 and np.all(lat2 > 0)
    st = server.stats()
    assert st["peak_busy_slots"] >= 2
    assert st["completed"] == 6_005 and st["err"] == 0 and st["arena_in_use_ints"] == 0
    assert st["integers"] == 2 * int(counts[ids].sum()) + sum(int(counts[p].sum()) for p in mine.values())
    # the server still answers ordinary queries afterwards, correctly
    p = ids[qoff[5]:qoff[6]]
    server.submit(7, p)
    got = []
    while not got:
        server.step(block=True)
        got = server.poll()
    (_, off, n), = got
    np.testing.assert_array_equal(read_result(server, off, n), expected(lists, starts, True, p))
    server.release(7)
    server.close()


def test_replay_poisson_open_loop():
    """Arrivals drawn in the call over a trace used cyclically: the generated count is a Poisson
    draw around qps x seconds, every generated query completes, the figures are consistent, and
    ordinary queries queued before it and after it still get the oracle's results."""
    lists, starts, counts, dev = make_pool(2_000, 1_500_000, 1 << 15, True, seed=95)
    server = serve.Server(dev["counts"], dev["in_off"], dev["in_bytes"], dev["streams"], dev["starts"],
                          arena_bytes=4 << 20, slots=4, max_batch_lists=512)
    _, qoff, ids = inputs.poisson_queries_flat(700, 1.0, len(lists), seed=96)
    mine = {200 + q: ids[qoff[q]:qoff[q + 1]] for q in range(3)}
    for qid, p in mine.items():
        server.submit(qid, p)
    qps, seconds, warmup = 30_000.0, 1.0, 0.2
    log_case("serve replay poisson", "qps=%g" % qps, "seconds=%g" % seconds)
    r = server.replay_poisson((qoff, ids), qps, seconds, warmup_s=warmup, seed=7)
    got = {}
    while len(got) < len(mine):
        server.step(block=True)
        for qid, off, n in server.poll():
            got[qid] = read_result(server, off, n)
            server.release(qid)
    for qid, p in mine.items():
        np.testing.assert_array_equal(got[qid], expected(lists, starts, True, p), err_msg="query %d" % qid)
    gen = r["generated"]
    assert abs(gen - qps * seconds) < 6 * np.sqrt(qps * seconds)
    assert abs(r["queries"] - qps * (seconds - warmup)) < 6 * np.sqrt(qps * seconds)
    assert 0 < r["p50_s"] <= r["p99_s"] < 0.1 and r["mean_s"] > 0 and r["wall_s"] > 0 and r["batches"] >= 1
    st = server.stats()
    assert st["completed"] == gen + len(mine) and st["err"] == 0 and st["arena_in_use_ints"] == 0
    # the trace is used cyclically: query i asks for entry i mod 700
    per_entry = np.add.reduceat(counts[ids], qoff[:-1].astype(np.int64))
    n = int(gen)
    want = int(per_entry.sum()) * (n // 700) + int(per_entry[: n % 700].sum())
    assert st["integers"] == want + sum(int(counts[p].sum()) for p in mine.values())
    p = ids[qoff[9]:qoff[10]]
    server.submit(9, p)
    out = []
    while not out:
        server.step(block=True)
        out = server.poll()
    (_, off, n2), = out
    np.testing.assert_array_equal(read_result(server, off, n2), expected(lists, starts, True, p))
    server.release(9)
    server.close()
