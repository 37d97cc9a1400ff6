"""Seeded synthetic workloads (numpy PCG64).  No codec arithmetic lives here.

These generators feed both the GPU library's tests and benchmark and the
oracle's tests; they produce plain uint32 arrays and list layouts only.  The
shapes stand in for the paper's posting-list collection (Section 5: document
identifiers of the one million most frequent words of ClueWeb09, sorted and
delta-coded), which is not available here.

Workloads (sizes are defaults; every function takes ``n``/``m`` so tests can
run them small):

* ``uniform_lengths``  -- 1,000,003 values; byte length uniform in {1,2,3,4},
  value uniform within that length's range.
* ``docids``           -- 2^26 sorted document ids from gaps that are geometric
  (mean 8) with probability 0.99 and uniform in [2^8, 2^20) otherwise; the
  running sum wraps modulo 2^32.
* ``stress_lengths``   -- 2^28 values, byte length 1..4 with probabilities
  0.4/0.3/0.2/0.1, value uniform within the range.
* ``zipf_rank_lengths`` + ``sorted_sets`` -- posting lists: list lengths follow
  Zipf's law over list rank (exponent 1.1, clipped to [1, cap]) scaled to a
  total integer count; each list is a sorted set of distinct ids in [0, 2^31).
* ``poisson_queries``  -- arrival times of a Poisson process and, per query,
  2..8 distinct list ids.
* ``sorted_sets_device`` -- the posting-list sets drawn on a GPU with torch, for
  the serving pool (10^6 lists, about 1.6e9 integers).
"""
import numpy as np

MASK32 = 0xFFFFFFFF

# (lo, hi) of the values a given byte length covers: [lo, hi)
_RANGES = [(0, 1 << 8), (1 << 8, 1 << 16), (1 << 16, 1 << 24), (1 << 24, 1 << 32)]


def _values_for_lengths(rng, lens):
    lo = np.array([r[0] for r in _RANGES], dtype=np.uint64)[lens - 1]
    hi = np.array([r[1] for r in _RANGES], dtype=np.uint64)[lens - 1]
    u = rng.random(lens.size)
    v = lo + np.floor(u * (hi - lo).astype(np.float64)).astype(np.uint64)
    v = np.minimum(v, hi - np.uint64(1))
    return v.astype(np.uint32)


def uniform_lengths(n=1_000_003, seed=1):
    """Byte length uniform in {1,2,3,4}; value uniform in [2^(8(L-1)), 2^(8L)) ([0, 256) for L=1)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 5, size=n)
    return _values_for_lengths(rng, lens)


def stress_lengths(n=1 << 28, seed=3, chunk=1 << 24):
    """Byte lengths i.i.d. with P(1..4) = (.4, .3, .2, .1); values uniform within the length range."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = rng.random(e - s)
        lens = 1 + (u >= 0.4).astype(np.int64) + (u >= 0.7) + (u >= 0.9)
        out[s:e] = _values_for_lengths(rng, lens)
    return out


def docid_gaps(n=1 << 26, seed=2, chunk=1 << 24):
    """Gaps between sorted document ids: Geometric(p=1/8) on {1,2,...} with probability 0.99,
    uniform in [2^8, 2^20) with probability 0.01.  The geometric draw is the inverse CDF,
    ceil(log(U) / log(1 - p)) for U uniform in (0, 1]."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint32)
    scale = 1.0 / np.log1p(-1.0 / 8.0)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = 1.0 - rng.random(e - s)                  # (0, 1]
        g = np.ceil(np.log(u) * scale)
        g = np.maximum(g, 1.0).astype(np.uint32)
        big = rng.random(e - s) < 0.01
        nb = int(big.sum())
        g[big] = rng.integers(1 << 8, 1 << 20, size=nb, dtype=np.uint32)
        out[s:e] = g
    return out


def docids(n=1 << 26, seed=2, start=0):
    """Sorted document ids: start + running total of ``docid_gaps`` (wrapping modulo 2^32).
    Returns (ids, gaps)."""
    g = docid_gaps(n, seed)
    x = (np.cumsum(g, dtype=np.uint64) + np.uint64(start)) & np.uint64(MASK32)
    return x.astype(np.uint32), g


def zipf_rank_lengths(m, total, cap, s=1.1, seed=4):
    """List lengths by Zipf's law over rank: L_r = clip(round(c * r^-s), 1, cap), r = 1..m,
    with c found by bisection so the lengths sum to ``total`` (as close as integers allow);
    returned in a seeded random order (int64)."""
    r = np.arange(1, m + 1, dtype=np.float64)
    w = r ** (-s)

    def lens_for(c):
        return np.clip(np.rint(c * w), 1, cap).astype(np.int64)

    lo, hi = 0.0, float(total) * 2.0 + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lens_for(mid).sum() < total:
            lo = mid
        else:
            hi = mid
    lens = lens_for(hi)
    rng = np.random.default_rng(seed)
    rng.shuffle(lens)
    return lens


def sorted_sets(lengths, universe=1 << 31, seed=5, chunk=1 << 24):
    """For each length l, l distinct sorted ids in [0, universe).

    Uses exponential spacings: with S_k the running sum of l+1 Exp(1) draws,
    y_k = floor(S_k / S_{l+1} * (universe - l)) is a sorted uniform sample and
    x_k = y_k + k makes it strictly increasing.  Returns (values uint32,
    offsets int64 of size m+1)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths.size
    offsets = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    out = np.empty(int(offsets[-1]), dtype=np.uint32)
    rng = np.random.default_rng(seed)
    i = 0
    while i < m:
        # lists i..j-1 hold about ``chunk`` values (at least one list)
        j = int(np.searchsorted(offsets, offsets[i] + chunk, side="right")) - 1
        j = min(m, max(j, i + 1))
        ls = lengths[i:j]
        nvals = int(ls.sum())
        seg = ls + 1                                   # l+1 spacings per list
        cs = np.cumsum(rng.standard_exponential(int(seg.sum())))
        seg_end = np.cumsum(seg) - 1                   # position of S_{l+1}
        seg_begin = seg_end - ls                       # position of S_1
        base = np.where(seg_begin > 0, cs[np.maximum(seg_begin - 1, 0)], 0.0)
        tot = cs[seg_end] - base
        lid = np.repeat(np.arange(j - i), ls)
        k = np.arange(nvals) - np.repeat(np.cumsum(ls) - ls, ls)
        frac = (cs[seg_begin[lid] + k] - base[lid]) / tot[lid]
        span = np.float64(universe) - ls.astype(np.float64)[lid]
        y = np.minimum(np.floor(frac * span), span - 1.0)
        out[offsets[i]:offsets[j]] = (y + k).astype(np.uint64).astype(np.uint32)
        i = j
    return out, offsets


def posting_lists(m=200_000, total=300_000_000, cap=1 << 20, seed=4):
    """Posting-list workload: Zipf rank-size lengths, sorted distinct ids over [0, 2^31).
    Returns (values, offsets)."""
    lens = zipf_rank_lengths(m, total, cap, seed=seed)
    return sorted_sets(lens, seed=seed + 1)


def seek_lists(m, bits, n=256, seed=9):
    """Seek/select workload (Section 5's experiment, scaled to m lists): per list, n deltas drawn
    uniformly from [0, 2^bits), bits <= 24, and their running sum as the list (non-decreasing, equal
    neighbours wherever a delta is 0).  Returns (values uint32[m * n], offsets int64[m + 1])."""
    if not 1 <= bits <= 24:
        raise ValueError("bits must be in 1..24")
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 1 << bits, size=(m, n), dtype=np.uint64)
    vals = np.cumsum(d, axis=1, dtype=np.uint64).astype(np.uint32).reshape(-1)
    return vals, np.arange(m + 1, dtype=np.int64) * n


def seek_queries(values, offsets, q, seed=10):
    """q queries over the lists of (values, offsets): a uniform list id, a target uniform in
    [0, last value + 2) of that list (so some targets lie past every value), and a uniform index
    below the list's length.  Empty lists get index 0.  Returns (list ids uint32, targets uint32,
    indexes uint64)."""
    rng = np.random.default_rng(seed)
    m = offsets.size - 1
    ids = rng.integers(0, m, size=q).astype(np.int64)
    lens = (offsets[ids + 1] - offsets[ids]).astype(np.int64)
    last = np.where(lens > 0, values[np.maximum(offsets[ids + 1] - 1, 0)].astype(np.int64), 0)
    targets = np.minimum((rng.random(q) * (last + 2)).astype(np.int64), 0xFFFFFFFF).astype(np.uint32)
    idx = np.where(lens > 0, (rng.random(q) * lens).astype(np.int64), 0).astype(np.uint64)
    return ids.astype(np.uint32), targets, idx


def poisson_queries(n_queries, qps, n_lists, seed=6, kmin=2, kmax=8):
    """Arrival times (seconds, Poisson process at ``qps``) and, per query, kmin..kmax distinct
    list ids chosen uniformly.  Returns (times float64[n], list of int64 arrays)."""
    t, qoff, ids = poisson_queries_flat(n_queries, qps, n_lists, seed, kmin, kmax)
    return t, [ids[qoff[i]:qoff[i + 1]] for i in range(n_queries)]


def poisson_queries_flat(n_queries, qps, n_lists, seed=6, kmin=2, kmax=8, distinct=True):
    """``poisson_queries`` with the picks flattened: (times, qoff int64[n+1], ids int64).  With
    ``distinct`` False a query's lists are drawn with replacement (no redraw of repeated ids), and
    qoff and ids come as uint64 and uint32, the layout the replay reads: for traces of hundreds of
    millions of queries."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=n_queries))
    ks = rng.integers(kmin, kmax + 1, size=n_queries, dtype=np.int64 if distinct else np.uint8)
    if n_lists < kmax:
        ks = np.minimum(ks, n_lists)
    qoff = np.zeros(n_queries + 1, dtype=np.int64 if distinct else np.uint64)
    np.cumsum(ks, out=qoff[1:])
    if not distinct:
        return t, qoff, rng.integers(0, n_lists, size=int(qoff[-1]), dtype=np.uint32)
    ids = rng.integers(0, n_lists, size=int(qoff[-1]), dtype=np.int64)
    # a query holding a repeated id is drawn again without replacement (queries of equal k are
    # checked together, each id against the ones before it)
    for k in np.unique(ks):
        rows = np.nonzero(ks == k)[0]
        block = ids[qoff[rows][:, None] + np.arange(k)[None, :]]
        rep = np.zeros(rows.size, dtype=bool)
        for a in range(1, k):
            rep |= np.any(block[:, :a] == block[:, a:a + 1], axis=1)
        for q in rows[rep]:
            ids[qoff[q]:qoff[q + 1]] = rng.choice(n_lists, size=int(k), replace=False)
    return t, qoff, ids


def sorted_sets_device(lengths, universe=1 << 31, seed=5, chunk=1 << 26, device="cuda"):
    """``sorted_sets`` generated on a torch device (for pools too large for the host to build
    quickly): the same exponential-spacings construction, drawn with torch's generator, so the
    values differ from the host version's.  Within a list the values are non-decreasing and
    below ``universe``.  Returns (values as a device int32 tensor holding the uint32 bits,
    offsets int64 numpy of size m+1)."""
    import torch
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths.size
    offsets = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    out = torch.empty(max(1, int(offsets[-1])), dtype=torch.int32, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    i = 0
    while i < m:
        j = int(np.searchsorted(offsets, offsets[i] + chunk, side="right")) - 1
        j = min(m, max(j, i + 1))
        ls = torch.from_numpy(lengths[i:j]).to(device)
        nvals = int(offsets[j] - offsets[i])
        seg = ls + 1
        e = torch.empty(int(seg.sum().item()), dtype=torch.float64, device=device).exponential_(generator=g)
        cs = torch.cumsum(e, 0)
        del e
        seg_end = torch.cumsum(seg, 0) - 1
        seg_begin = seg_end - ls
        base = torch.where(seg_begin > 0, cs[torch.clamp(seg_begin - 1, min=0)], torch.zeros_like(cs[:1]))
        tot = cs[seg_end] - base
        lid = torch.repeat_interleave(torch.arange(j - i, device=device), ls)
        k = torch.arange(nvals, device=device) - torch.repeat_interleave(torch.cumsum(ls, 0) - ls, ls)
        frac = (cs[seg_begin[lid] + k] - base[lid]) / tot[lid]
        del cs
        span = float(universe) - ls.to(torch.float64)[lid]
        y = torch.minimum(torch.floor(frac * span), span - 1.0)
        vals = y.to(torch.int64) + k
        out[int(offsets[i]):int(offsets[j])] = (vals & 0xFFFFFFFF).to(torch.int32) if universe > (1 << 31) \
            else vals.to(torch.int32)
        del frac, span, y, vals, lid, k
        i = j
    return out, offsets


def random_bytes(n, seed=7):
    """Uniform random bytes (for streams with arbitrary control bytes and data)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=n, dtype=np.uint8)


def random_u32(n, seed=8):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)


def bounded_gaps(n, bits, seed=13):
    """Integers drawn uniformly from [0, 2^bits): a list whose deltas all fit in `bits` bits, the
    compressibility axis along which Section 5 compares the byte-oriented formats (VByte's bits per
    integer on the horizontal axis of its size and speed figures)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(np.uint32)
