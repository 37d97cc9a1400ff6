#!/usr/bin/env python3
"""Stream VByte on one MI355X: delta-decode throughput against the HBM roofline.

One step = one svb_delta_decode call (control-byte lengths -> group byte
offsets -> group value sums -> running-sum decode) of 2^26 sorted document ids
whose gaps are geometric with mean 8 (probability 0.99) or uniform in
[2^8, 2^20) (probability 0.01), start value 0.  The compressed input is made by
the library's delta encoder and is resident in HBM before timing starts.

Prints one JSON line.  Besides the headline it carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average duration (HIP events recorded by the library on the
                launch stream, over a second pass of the timed steps) against
                8 TB/s, and the HBM bytes per launch from committed rocprofv3
                counters;
  kernels       average duration of every kernel of the call;
  cpu_baseline  the scalar C oracle, single-threaded, on the host cores;
  encode        delta encode of the same array;
  protocol      the headline's timing: every call after a 1 GiB read that
                evicts the caches (the median of at least 21 calls);
  dirty_flush   the same with a 1 GiB write before each call instead (up to
                256 MB of its dirty lines are written back during the call);
  unflushed     the mean of back-to-back calls;
  copy          a plain copy kernel (the practical bandwidth ceiling);
  at_2p28       delta decode of the same generator at 2^28 integers, and plain
                decode of 2^28 integers with unpredictable lengths;
  batched       200,000 delta-coded posting lists (about 3e8 integers):
                autotuned batched decode and encode, against the single-array
                rate, against one array of the same integers (the lists back
                to back, one stream) and against one svb_delta_decode call
                per list;
  seek_select   seek and select over 2^20 lists of 256 running sums (deltas
                below 2^8 and 2^16), 2^22 queries per call, queries/s and
                algorithmic GB/s, the oracle's walk timed beside them;
  append        2^22 document ids appended to the 2^26-id delta stream
                without re-encoding it, GB/s against HBM, the oracle's
                append timed beside it;
  zero_control  delta decode of 2^28 running sums of deltas below 2^8 with
                the general decoder and with the zero-control variant;
  serving       a pool of 10^6 delta-coded lists (about 1.6e9 integers) kept
                in HBM, queries of 2..8 lists: closed-loop saturation rate,
                then Poisson arrivals at 0.5x and 0.8x of it (windows of
                --serve-seconds, 30 s by default, arrivals drawn in the
                replay), p50/p99 latency and
                integers/s, against the 2^28 single-array rate and against
                the pool's integers decoded as one array.

`python bench.py --summarize-counters FETCH.csv WRITE.csv OUT.md` turns two
rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE) into the
counter summary that later runs read back (no GPU needed for that step).
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "decoded uint32/s + achieved HBM GB/s (% of peak), delta decode, 1 GPU"
WORKLOAD = ("delta decode of 2^26 sorted uint32 document ids: gaps Geometric(1/8) on {1,2,...} "
            "w.p. 0.99, uniform in [2^8, 2^20) w.p. 0.01, running sum wrapping mod 2^32, start 0")
N_HEAD = 1 << 26
COPY_WORDS = 1 << 26                     # 256 MiB copied by the ceiling / counter-scaling copy
COUNTERS_FILE = "counters_delta_decode_docids_2p26.md"
DOMINANT_SYMBOL = "decode_kernel<1, false>"  # rocprofv3 name fragment of the delta decode pass (general variant)
COPY_SYMBOL = "copy_kernel"


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


# Sources the dominant kernel (the delta decode pass) is built from: a change
# to any of them voids the stored counter figures.
DIGEST_FILES = ("svb_decode.hip", "svb_delta.hip", "svb_scan.hip", "svb_segment.hpp", "svb_device.hpp",
                "svb_internal.hpp")


def source_digest():
    h = hashlib.sha256()
    for name in DIGEST_FILES:
        with open(os.path.join(ROOT, "paper_1709_08990_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", COUNTERS_FILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"^source_digest:\s*(\w+)", text, re.M)
    m_val = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m_src or not m_val or m_src.group(1) != source_digest():
        return None
    return float(m_val.group(1))


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


# ------------------------------------------------------------------ counters (offline)

def _counter_means(path, counter):
    """Mean value per dispatch of `counter` for every kernel name in a rocprofv3 counter CSV."""
    per = collections.defaultdict(list)
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in per.items()}


def _pick(means, fragment):
    hits = [(k, v) for k, v in means.items() if fragment in k]
    if not hits:
        raise SystemExit("no kernel matching %r in counter file" % fragment)
    return hits[0]


def summarize_counters(fetch_csv, write_csv, out_md, command):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the dominant kernel, each scaled by what
    the same counter reads for the copy kernel, which moves exactly COPY_WORDS * 4 bytes each way."""
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")
    copy_bytes = 4.0 * COPY_WORDS
    kf, f_dom = _pick(fetch, DOMINANT_SYMBOL)
    _, f_copy = _pick(fetch, COPY_SYMBOL)
    kw, w_dom = _pick(write, DOMINANT_SYMBOL)
    _, w_copy = _pick(write, COPY_SYMBOL)
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    fetched = f_dom * 1024.0 * f_scale
    written = w_dom * 1024.0 * w_scale
    lines = [
        "# HBM traffic of the delta decode pass, docids 2^26",
        "",
        "Two rocprofv3 counter passes over bench.py (one counter each):",
        "",
        "    " + command.replace("{COUNTER}", "FETCH_SIZE"),
        "    " + command.replace("{COUNTER}", "WRITE_SIZE"),
        "",
        "Counters are KiB per dispatch, averaged over dispatches.  Each is scaled by",
        "bytes / counter of the copy kernel in the same run, which reads and writes",
        "exactly %d bytes." % copy_bytes,
        "",
        "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |",
        "|---|---|---|",
        "| %s | %.1f | %.1f |" % (kf, f_dom, w_dom),
        "| copy (%d B each way) | %.1f | %.1f |" % (copy_bytes, f_copy, w_copy),
        "",
        "fetch_scale: %.4f" % f_scale,
        "write_scale: %.4f" % w_scale,
        "fetched_bytes_per_launch: %.0f" % fetched,
        "written_bytes_per_launch: %.0f" % written,
        "traffic_bytes_per_launch: %.0f" % (fetched + written),
        "source_digest: %s" % source_digest(),
        "",
    ]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4  # 1024 SIMDs, one wave64 instruction per 4 cycles each


def _pmc_rows(paths):
    """Per kernel: every counter's values (one per dispatch) and the dispatch durations, over the
    counter_collection CSVs of several rocprofv3 --pmc runs."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(list)
    for path in paths:
        seen = set()
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = r["Kernel_Name"]
                per[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
                key = (k, r.get("Dispatch_Id"), path)
                if key not in seen:
                    seen.add(key)
                    dur[k].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return per, dur


def _short(name, width=70):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
    return name if len(name) <= width else name[:width - 3] + "..."


def summarize_pmc(out_md, title, commands, paths, only=None):
    """Every kernel of one or more rocprofv3 --pmc runs (or those whose name holds one of the
    fragments in `only`): median dispatch duration, HBM bytes from FETCH_SIZE / WRITE_SIZE scaled
    by what the same counters read for the copy kernel (COPY_WORDS * 4 bytes each way), and SQ
    instruction counts per wave with the VALU issue share they imply."""
    per, dur = _pmc_rows(paths)
    copy = [k for k in per if COPY_SYMBOL in k]
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        if copy and per[copy[0]].get(c):
            v = per[copy[0]][c]
            scale[c] = 4.0 * COPY_WORDS / (1024.0 * sum(v) / len(v))
    mean = lambda k, c: (sum(per[k][c]) / len(per[k][c])) if per[k].get(c) else None
    med = lambda k: sorted(dur[k])[len(dur[k]) // 2] / 1e3 if dur[k] else float("nan")
    names = [k for k in per if "svb" in k and (not only or any(f in k for f in only))]
    names.sort(key=lambda k: -med(k))
    lines = ["# %s" % title, "", "rocprofv3 counter runs (one per line):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Durations are the median over dispatches of the counter runs (counters serialise",
              "dispatches, so they run somewhat longer than in a plain run)."]
    if scale:
        lines += ["", "HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over dispatches), each",
                  "scaled by bytes / counter of the copy kernel of the same run (%d bytes each way):"
                  % (4 * COPY_WORDS),
                  " ".join("%s scale %.4f;" % (c, v) for c, v in sorted(scale.items())), "",
                  "| kernel | dispatches | median us | fetched MB | written MB | GB/s |", "|---|---|---|---|---|---|"]
        for k in names:
            f, w = mean(k, "FETCH_SIZE"), mean(k, "WRITE_SIZE")
            fb = f * 1024 * scale.get("FETCH_SIZE", 1) if f is not None else None
            wb = w * 1024 * scale.get("WRITE_SIZE", 1) if w is not None else None
            gb = ((fb or 0) + (wb or 0)) / (med(k) * 1e3) if (fb is not None or wb is not None) else None
            fmt = lambda v: "%.2f" % (v / 1e6) if v is not None else "-"
            lines.append("| `%s` | %d | %.1f | %s | %s | %s |" % (_short(k), len(dur[k]), med(k), fmt(fb), fmt(wb),
                                                                 "%.0f" % gb if gb is not None else "-"))
        dom = [k for k in names if DOMINANT_SYMBOL in k and mean(k, "FETCH_SIZE") is not None
               and mean(k, "WRITE_SIZE") is not None]
        if dom:
            k = dom[0]
            lines += ["", "traffic_bytes_per_launch: %.0f" % (1024 * (mean(k, "FETCH_SIZE") * scale.get("FETCH_SIZE", 1)
                                                                      + mean(k, "WRITE_SIZE") * scale.get("WRITE_SIZE", 1))),
                      "(of `%s`, the bench line's dominant kernel: read by bench.py as roofline.traffic while the "
                      "source digest below matches)" % _short(k)]
    sq = [c for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
                      "SQ_WAIT_INST_ANY") if any(per[k].get(c) for k in names)]
    if sq and any(per[k].get("SQ_WAVES") for k in names):
        lines += ["", "Instructions per wave (SQ counters, summed over the device, over SQ_WAVES); VALU share =",
                  "SQ_INSTS_VALU / (%.1f G wave instructions/s x median duration): 1024 SIMDs issuing one"
                  % (VALU_WAVE_INSTR_PER_S / 1e9),
                  "wave64 VALU instruction per 4 cycles each at 2.4 GHz.", "",
                  "| kernel | waves | " + " | ".join(c.replace("SQ_INSTS_", "").replace("SQ_", "").lower() + "/wave"
                                                    for c in sq) + " | VALU share |",
                  "|---|---|" + "---|" * len(sq) + "---|"]
        for k in names:
            wv = mean(k, "SQ_WAVES")
            if not wv:
                continue
            cells = ["%.1f" % (mean(k, c) / wv) if mean(k, c) is not None else "-" for c in sq]
            valu = mean(k, "SQ_INSTS_VALU")
            share = valu / (VALU_WAVE_INSTR_PER_S * med(k) * 1e-6) if valu is not None else None
            lines.append("| `%s` | %.0f | %s | %s |" % (_short(k), wv, " | ".join(cells),
                                                        "%.2f" % share if share is not None else "-"))
    other = sorted({c for k in names for c in per[k]} - set(sq) - {"SQ_WAVES", "FETCH_SIZE", "WRITE_SIZE"})
    if other:
        lines += ["", "Other counters (mean per dispatch):", "", "| kernel | " + " | ".join(other) + " |",
                  "|---|" + "---|" * len(other)]
        for k in names:
            lines.append("| `%s` | %s |" % (_short(k), " | ".join("%.4g" % mean(k, c) if mean(k, c) is not None
                                                                  else "-" for c in other)))
    lines += ["", "source_digest: %s" % source_digest(), ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def summarize_trace(stats_csv, out_md, title, command, bench_json=None):
    """Turns a rocprofv3 --kernel-trace --stats kernel_stats.csv into a short table, and, given
    the bench line of the same command, puts the dominant kernel's HIP-event average beside
    rocprofv3's."""
    rows = []
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["MinNs"]), float(r["MaxNs"])))
    rows.sort(key=lambda r: -r[2])
    lines = ["# %s" % title, "", "rocprofv3 kernel-trace summary (kernel_stats.csv) of:", "", "    " + command, "",
             "| kernel | calls | total us | average us | min us | max us |", "|---|---|---|---|---|---|"]
    for name, calls, tot, avg, mn, mx in rows:
        short = name if len(name) <= 90 else name[:87] + "..."
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f | %.1f |" % (short, calls, tot / 1e3, avg / 1e3, mn / 1e3,
                                                                  mx / 1e3))
    if bench_json:
        with open(bench_json) as fh:
            line = json.loads(fh.read().strip().splitlines()[-1])
        rf = line["roofline"]
        dom = [r for r in rows if DOMINANT_SYMBOL in r[0]]
        lines += ["", "bench.py, same command: dominant kernel `%s` %.1f us per launch by the library's HIP events;"
                  % (rf["kernel"], 1e3 * rf["kernel_ms"]),
                  "rocprofv3 average for `%s`: %s us." % (DOMINANT_SYMBOL, "%.1f" % (dom[0][3] / 1e3) if dom else "n/a")]
    lines += ["", "source_digest: %s" % source_digest(), ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


# ------------------------------------------------------------------ GPU measurement

def event_loop(fn, steps, torch, before=None):
    """Runs fn() `steps` times with a torch event pair around each call on the current stream.
    Returns (wall seconds, mean per-call milliseconds)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        if before is not None:
            before()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, sum(a.elapsed_time(b) for a, b in ev) / steps


def kernel_means(svb):
    """Average milliseconds per kernel name from the library's event records."""
    per = collections.defaultdict(list)
    for name, ms in svb.svb_kernel_times():
        per[name].append(ms)
    return {k: sum(v) / len(v) for k, v in per.items()}


def timed_steps(svb, torch, fn, steps, warmup):
    """`warmup` untimed calls, then the timed region: `steps` calls between two device
    synchronisations (wall clock), then the same `steps` calls again with the library recording
    HIP events around each kernel on the launch stream (per-kernel durations; the event records
    add a few microseconds per kernel, which is why the wall-clock region runs without them).
    Back to back, no cache flush: inputs that fit the 256 MB MALL stay there.  Returns (wall
    seconds, per-kernel mean ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    svb.svb_kernel_times()  # drop stale records
    svb.svb_set_kernel_timing(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    svb.svb_set_kernel_timing(False)
    return wall, kernel_means(svb)


MIN_REPS = 21


class Flush:
    """Two ways of evicting the L2s and the 256 MB MALL before a timed call, over one 1 GiB buffer:
    clean() reads it (the caches end up holding clean lines of an unrelated buffer: the call's
    inputs come from HBM and nothing foreign is left to write back); dirty() writes it (the caches
    end up holding up to 256 MB of dirty lines, whose write-back then falls inside the timed call,
    as a previous call's output would in a stream of calls)."""

    def __init__(self, svb, torch):
        self.svb = svb
        self.buf = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")

    def clean(self):
        self.buf.sum()

    def dirty(self):
        self.svb.svb_fill_u32(self.buf.numel(), self.buf, 0)

    def __call__(self):
        self.clean()


def protocol_steps(svb, torch, fn, steps, warmup, flush):
    """The measurement protocol: `warmup` untimed calls, then the timed region of exactly `steps`
    calls between two device synchronisations, each call preceded by flush.clean() (a 1 GiB read
    that evicts the L2s and the 256 MB MALL) and bracketed by events on the current stream; more
    flushed calls until at least 21 have been timed.  The call time is the median of the event
    durations.  Then the same number of flushed calls with the library's per-kernel HIP events
    (median per kernel name), as many again after flush.dirty() (a 1 GiB write; median), and
    `steps` calls back to back without flushing (mean, for reference).  Returns a dict."""
    for _ in range(warmup):
        flush()
        fn()
    reps = max(steps, MIN_REPS)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (a, b) in enumerate(ev):
        flush()
        a.record()
        fn()
        b.record()
        if i + 1 == steps:
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    svb.svb_kernel_times()  # drop stale records
    svb.svb_set_kernel_timing(True)
    for _ in range(reps):
        flush()
        fn()
    torch.cuda.synchronize()
    svb.svb_set_kernel_timing(False)
    per = collections.defaultdict(list)
    for name, t in svb.svb_kernel_times(cap=1 << 16):
        per[name].append(t)
    kms = {k: sorted(v)[len(v) // 2] for k, v in per.items()}
    dev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in dev:
        flush.dirty()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    dms = sorted(a.elapsed_time(b) for a, b in dev)
    t1 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    unflushed = 1e3 * (time.perf_counter() - t1) / steps
    return {"median_ms": ms[len(ms) // 2], "reps": reps, "min_ms": ms[0], "max_ms": ms[-1],
            "timed_region_s": wall, "kernels_ms": kms, "dirty_flush_median_ms": dms[len(dms) // 2],
            "unflushed_mean_ms": unflushed}


def gbs(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def measure_delta(svb, torch, x_dev, steps, warmup, flush):
    """Delta decode and delta encode of one array under the protocol (flushed median)."""
    n = x_dev.numel()
    comp = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n, x_dev, comp, 0, size)
    torch.cuda.synchronize()
    nbytes = int(size.item())
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    alg = nbytes + 4 * n

    def dec():
        svb.svb_delta_decode(n, comp, nbytes, out, 0, err)

    pr = protocol_steps(svb, torch, dec, steps, warmup, flush)
    ok = bool(torch.equal(out, x_dev)) and int(err.item()) == 0
    call_ms = pr["median_ms"]
    res = {"n": n, "compressed_bytes": nbytes, "bits_per_int": 8.0 * nbytes / n, "alg_bytes_per_call": alg,
           "ms_per_call": call_ms, "round_trip_ok": ok, "protocol": pr,
           "uint32_per_s": n / (call_ms * 1e-3), "call_GBps": gbs(alg, call_ms),
           "call_frac_of_peak": gbs(alg, call_ms) / HBM_PEAK_GBS, "kernels_ms": pr["kernels_ms"],
           "dirty_flush": {"ms_per_call": pr["dirty_flush_median_ms"],
                           "frac_of_peak": gbs(alg, pr["dirty_flush_median_ms"]) / HBM_PEAK_GBS,
                           "note": "median, each call after a 1 GiB write (its dirty lines are written "
                                   "back during the call)"},
           "unflushed": {"ms_per_call": pr["unflushed_mean_ms"],
                         "frac_of_peak": gbs(alg, pr["unflushed_mean_ms"]) / HBM_PEAK_GBS,
                         "note": "mean of back-to-back calls, no cache flush"}}

    def enc():
        svb.svb_delta_encode(n, x_dev, comp, 0, size)

    ep = protocol_steps(svb, torch, enc, steps, max(1, warmup // 2), flush)
    ems = ep["median_ms"]
    res["encode"] = {"ms_per_call": ems, "uint32_per_s": n / (ems * 1e-3), "GBps": gbs(alg, ems),
                     "frac_of_peak": gbs(alg, ems) / HBM_PEAK_GBS, "kernels_ms": ep["kernels_ms"],
                     "dirty_flush_ms": ep["dirty_flush_median_ms"],
                     "dirty_flush_frac_of_peak": gbs(alg, ep["dirty_flush_median_ms"]) / HBM_PEAK_GBS,
                     "unflushed_ms": ep["unflushed_mean_ms"], "size_ok": int(size.item()) == nbytes}
    del comp, out
    return res


def measure_plain(svb, torch, x_dev, steps, warmup, flush):
    n = x_dev.numel()
    comp = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_encode(n, x_dev, comp, size)
    torch.cuda.synchronize()
    nbytes = int(size.item())
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    alg = nbytes + 4 * n
    pr = protocol_steps(svb, torch, lambda: svb.svb_decode(n, comp, nbytes, out), steps, warmup, flush)
    ok = bool(torch.equal(out, x_dev))
    call_ms = pr["median_ms"]
    del comp, out
    return {"n": n, "compressed_bytes": nbytes, "ms_per_call": call_ms, "uint32_per_s": n / (call_ms * 1e-3),
            "call_GBps": gbs(alg, call_ms), "call_frac_of_peak": gbs(alg, call_ms) / HBM_PEAK_GBS,
            "kernels_ms": pr["kernels_ms"], "dirty_flush_ms": pr["dirty_flush_median_ms"],
            "dirty_flush_frac_of_peak": gbs(alg, pr["dirty_flush_median_ms"]) / HBM_PEAK_GBS,
            "unflushed_ms": pr["unflushed_mean_ms"], "round_trip_ok": ok}


def measure_copy(svb, torch, steps):
    a = torch.empty(COPY_WORDS, dtype=torch.int32, device="cuda").fill_(7)
    b = torch.empty_like(a)
    svb.svb_copy_u32(COPY_WORDS, a, b)
    _, ms = event_loop(lambda: svb.svb_copy_u32(COPY_WORDS, a, b), steps, torch)
    ok = bool(torch.equal(a, b))
    del a, b
    return {"bytes_each_way": 4 * COPY_WORDS, "ms": ms, "GBps": gbs(8 * COPY_WORDS, ms),
            "frac_of_peak": gbs(8 * COPY_WORDS, ms) / HBM_PEAK_GBS, "ok": ok}


def measure_batched(svb, torch, np, inputs, steps, warmup, per_list=True):
    """C4: 200,000 posting lists (rank-size Zipf lengths in [1, 2^20], about 3e8 integers, sorted sets
    over [0, 2^31)), delta-coded from 0.  Batched encode, autotuned batched delta decode, and one
    svb_delta_decode call per list on the same streams."""
    import ctypes
    vals, offs = inputs.posting_lists()
    m = offs.size - 1
    counts = np.diff(offs).astype(np.uint64)
    total = int(counts.sum())
    x_dev = torch.from_numpy(vals.view(np.int32)).cuda()
    del vals
    caps = (counts + 3) // 4 + 4 * counts
    comp_off = np.zeros(m, dtype=np.uint64)
    np.cumsum(caps[:-1], out=comp_off[1:])
    u64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
    d_counts, d_in_off, d_comp_off = u64(counts), u64(offs[:-1]), u64(comp_off)
    comp = torch.empty(int(caps.sum()), dtype=torch.uint8, device="cuda")
    sizes = torch.empty(m, dtype=torch.int64, device="cuda")
    starts = torch.zeros(m, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    enc_args = (m, d_counts, d_in_off, x_dev, d_comp_off, comp, sizes, starts, total)
    g_enc = svb.svb_autotune_encode_batch(*enc_args)
    ewall, ekms = timed_steps(svb, torch, lambda: svb.svb_encode_batch(*enc_args), steps, warmup)
    nbytes = int(sizes.sum().item())
    dec_args = (m, d_counts, d_comp_off, sizes, comp, d_in_off, out, starts, total, err)
    g_dec = svb.svb_autotune_decode_batch(*dec_args)
    wall, kms = timed_steps(svb, torch, lambda: svb.svb_decode_batch(*dec_args), steps, warmup)
    ok = bool(torch.equal(out, x_dev)) and int(err.item()) == 0
    call_ms = 1e3 * wall / steps
    alg = nbytes + 4 * total
    res = {"lists": m, "integers": total, "compressed_bytes": nbytes, "chunk_decode": g_dec,
           "chunk_encode": g_enc, "ms_per_call": call_ms, "uint32_per_s": total / (call_ms * 1e-3),
           "call_GBps": gbs(alg, call_ms), "call_frac_of_peak": gbs(alg, call_ms) / HBM_PEAK_GBS,
           "kernels_ms": kms, "round_trip_ok": ok,
           "encode": {"ms_per_call": 1e3 * ewall / steps, "uint32_per_s": total / ewall * steps, "kernels_ms": ekms}}
    # the same integers as one array: the lists back to back, delta-coded as a single stream (so the
    # same byte lengths, bar one difference per list boundary), decoded by one svb_delta_decode call
    one = torch.empty(svb.svb_max_compressed_bytes(total), dtype=torch.uint8, device="cuda")
    one_size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(total, x_dev, one, 0, one_size)
    torch.cuda.synchronize()
    one_bytes = int(one_size.item())
    out.zero_()
    owall, okms = timed_steps(svb, torch, lambda: svb.svb_delta_decode(total, one, one_bytes, out, 0), steps, warmup)
    one_ms = 1e3 * owall / steps
    res["single_array_same_ints"] = {"ms_per_call": one_ms, "uint32_per_s": total / (one_ms * 1e-3),
                                     "compressed_bytes": one_bytes, "kernels_ms": okms,
                                     "round_trip_ok": bool(torch.equal(out, x_dev))}
    res["vs_single_array_same_ints"] = res["uint32_per_s"] / res["single_array_same_ints"]["uint32_per_s"]
    del one
    if not per_list:
        del x_dev, comp, out
        return res
    # one svb_delta_decode call per list, same streams, same output
    L = svb.lib()
    h_sizes = sizes.cpu().numpy().astype(np.uint64)
    stream = torch.cuda.current_stream().cuda_stream
    cbase, obase = comp.data_ptr(), out.data_ptr()
    out.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(m):
        st = L.svb_delta_decode(int(counts[i]), cbase + int(comp_off[i]), int(h_sizes[i]),
                                obase + 4 * int(offs[i]), 0, None, stream)
        if st != 0:
            raise RuntimeError("svb_delta_decode failed for list %d" % i)
    torch.cuda.synchronize()
    per_list_s = time.perf_counter() - t0
    res["one_call_per_list"] = {"seconds": per_list_s, "uint32_per_s": total / per_list_s,
                                "round_trip_ok": bool(torch.equal(out, x_dev))}
    del x_dev, comp, out
    return res


def measure_seek(svb, torch, np, inputs, steps, warmup, oracle_sample=20_000):
    """Seek and select (Section 5's operations on compressed lists) at GPU scale: the paper's
    workload of lists of 256 running sums of deltas below 2^b, 2^20 lists, one call answering 2^22
    random queries (a uniform list, a uniform target in [0, last + 2) or a uniform position).
    Algorithmic bytes of a query: its inputs and outputs, the index entries it reads (list bases,
    the running maximum, the segment's 64-byte descriptor) and the segment it decodes (control
    and data bytes).  The answers are checked on a sample against the input lists (sorted, so seek
    is numpy's lower bound); the oracle is only timed, as this section's CPU baseline."""
    import oracle
    out = {}
    m, q = 1 << 20, 1 << 22
    cap = svb.svb_max_compressed_bytes(256)
    u64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
    for bits in (8, 16):
        vals, offs = inputs.seek_lists(m, bits, seed=90 + bits)
        x_dev = torch.from_numpy(vals.view(np.int32)).cuda()
        counts = np.full(m, 256, dtype=np.uint64)
        byte_off = np.arange(m, dtype=np.uint64) * cap
        comp = torch.empty(m * cap, dtype=torch.uint8, device="cuda")
        sizes = torch.empty(m, dtype=torch.int64, device="cuda")
        starts = torch.zeros(m, dtype=torch.int32, device="cuda")
        d_counts, d_val_off = u64(counts), u64(offs[:-1])
        svb.svb_encode_batch(m, d_counts, d_val_off, x_dev, u64(byte_off), comp, sizes, starts, 256 * m)
        torch.cuda.synchronize()
        # the streams packed back to back, as an index over stored lists holds them (encoded again at
        # their final offsets)
        h_sizes = sizes.cpu().numpy().view(np.uint64).copy()
        byte_off = np.zeros(m, dtype=np.uint64)
        np.cumsum(h_sizes[:-1], out=byte_off[1:])
        del comp
        comp = torch.empty(int(h_sizes.sum()) + 64, dtype=torch.uint8, device="cuda")
        d_off = u64(byte_off)
        svb.svb_encode_batch(m, d_counts, d_val_off, x_dev, d_off, comp, sizes, starts, 256 * m)
        torch.cuda.synchronize()
        seg_bytes = float(h_sizes.mean())
        t0 = time.perf_counter()
        index = svb.svb_seek_index_create(m, d_counts, d_off, sizes, comp, starts, 256 * m)
        build_s = time.perf_counter() - t0
        ids, targets, idx = inputs.seek_queries(vals, offs, q, seed=95 + bits)
        d_ids, d_t, d_i = torch.from_numpy(ids.view(np.int32)).cuda(), torch.from_numpy(targets.view(np.int32)).cuda(), \
            u64(idx)
        pos = torch.empty(q, dtype=torch.int64, device="cuda")
        val = torch.empty(q, dtype=torch.int32, device="cuda")
        sval = torch.empty(q, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        swall, skms = timed_steps(svb, torch, lambda: svb.svb_seek_batch(index, q, d_ids, d_t, pos, val, err), steps,
                                  warmup)
        lwall, lkms = timed_steps(svb, torch, lambda: svb.svb_select_batch(index, q, d_ids, d_i, sval, err), steps,
                                  warmup)
        ok = int(err.item()) == 0
        pos_h, val_h, sval_h = pos.cpu().numpy(), val.cpu().numpy().view(np.uint32), sval.cpu().numpy().view(np.uint32)
        rng = np.random.default_rng(bits)
        sample = rng.integers(0, q, size=oracle_sample)
        for k in sample[:2_000]:
            x = vals[offs[ids[k]]:offs[ids[k] + 1]]
            p = int(np.searchsorted(x, targets[k], side="left"))
            ok &= (int(pos_h[k]), int(val_h[k])) == (p, int(x[p]) if p < x.size else 0)
            ok &= int(sval_h[k]) == int(x[idx[k]])
        # CPU baseline of this section: the oracle's walk over the sampled queries (one ctypes call each)
        host_streams = comp.cpu().numpy().view(np.uint8)
        t0 = time.perf_counter()
        for k in sample:
            l = int(ids[k])
            o = int(byte_off[l])
            oracle.seek(host_streams[o:o + int(h_sizes[l])], 256, int(targets[k]), True, 0)
        oracle_s = time.perf_counter() - t0
        svb.svb_seek_index_destroy(index)
        q_in_out = 4 + 4 + 8 + 4           # list id, target, position, value
        index_bytes = 8 + 4 + 64           # list bases, running maximum, descriptor
        per_query = q_in_out + index_bytes + seg_bytes
        seek_ms, sel_ms = 1e3 * swall / steps, 1e3 * lwall / steps
        out["b%d" % bits] = {
            "lists": m, "ints_per_list": 256, "queries_per_call": q, "stream_bytes_per_list": seg_bytes,
            "index_build_s": build_s,
            "seek": {"ms_per_call": seek_ms, "queries_per_s": q / (seek_ms * 1e-3),
                     "alg_bytes_per_query": per_query, "GBps": gbs(per_query * q, seek_ms),
                     "frac_of_peak": gbs(per_query * q, seek_ms) / HBM_PEAK_GBS, "kernels_ms": skms},
            "select": {"ms_per_call": sel_ms, "queries_per_s": q / (sel_ms * 1e-3),
                       "alg_bytes_per_query": per_query, "GBps": gbs(per_query * q, sel_ms),
                       "frac_of_peak": gbs(per_query * q, sel_ms) / HBM_PEAK_GBS, "kernels_ms": lkms},
            "cpu_oracle": {"queries_per_s": oracle_sample / oracle_s, "cores": 1, "kind": "oracle",
                           "sample": "%d seeks, one ctypes call each (call overhead included)" % oracle_sample},
            "sample_matches_input": bool(ok)}
        del x_dev, comp, host_streams
        torch.cuda.empty_cache()
    return out


def measure_zero_control(svb, torch, np, steps, warmup, n=1 << 28):
    """The zero-control decoder variant against the general one: delta decode of 2^28 running sums of
    deltas below 2^8 (every control byte 0).  Each variant is set explicitly; the general one is
    restored afterwards."""
    rng = np.random.default_rng(41)
    x = np.cumsum(rng.integers(0, 256, size=n, dtype=np.uint64), dtype=np.uint64).astype(np.uint32)
    x_dev = torch.from_numpy(x.view(np.int32)).cuda()
    del x
    comp = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n, x_dev, comp, 0, size)
    torch.cuda.synchronize()
    nb = int(size.item())
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {"n": n, "compressed_bytes": nb}
    for v in (0, 1):
        svb.svb_set_decode_variant(True, v)
        out.zero_()
        wall, kms = timed_steps(svb, torch, lambda: svb.svb_delta_decode(n, comp, nb, out, 0), steps, warmup)
        ms = 1e3 * wall / steps
        res["variant%d" % v] = {"ms_per_call": ms, "uint32_per_s": n / (ms * 1e-3),
                                "call_frac_of_peak": gbs(nb + 4 * n, ms) / HBM_PEAK_GBS, "kernels_ms": kms,
                                "round_trip_ok": bool(torch.equal(out, x_dev))}
    svb.svb_set_decode_variant(True, -1)
    res["speedup"] = res["variant0"]["ms_per_call"] / res["variant1"]["ms_per_call"]
    del x_dev, comp, out
    return res


def measure_append(svb, torch, np, inputs, steps, warmup, n=1 << 26, k=1 << 22):
    """Append without re-encoding: 2^22 document ids appended to the delta stream of the 2^26 before
    them (the same generator).  Algorithmic bytes of a call: the old stream read, the new values
    read, the new stream written.  The result is checked against one encode of all the ids; the
    oracle's append (one host core) is timed beside it, as this section's CPU baseline."""
    import oracle
    x, _ = inputs.docids(n + k, seed=21)
    x_dev = torch.from_numpy(x.view(np.int32)).cuda()
    old = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
    osz = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n, x_dev, old, 0, osz)
    want = torch.empty(svb.svb_max_compressed_bytes(n + k), dtype=torch.uint8, device="cuda")
    wsz = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n + k, x_dev, want, 0, wsz)
    torch.cuda.synchronize()
    old_bytes, new_bytes = int(osz.item()), int(wsz.item())
    out = torch.empty(svb.svb_max_compressed_bytes(n + k), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    vals = x_dev[n:]
    prev = int(x[n - 1])
    call = lambda: svb.svb_delta_append(n, old, old_bytes, k, vals, prev, out, size)
    wall, kms = timed_steps(svb, torch, call, steps, warmup)
    ok = int(size.item()) == new_bytes and bool(torch.equal(out[:new_bytes], want[:new_bytes]))
    ms = 1e3 * wall / steps
    alg = old_bytes + 4 * k + new_bytes
    host_old = old[:old_bytes].cpu().numpy().view(np.uint8)
    t0 = time.perf_counter()
    oracle.append(host_old, n, x[n:], delta=True, prev=prev)
    oracle_s = time.perf_counter() - t0
    del x_dev, old, want, out
    return {"stored": n, "appended": k, "old_bytes": old_bytes, "new_bytes": new_bytes, "ms_per_call": ms,
            "alg_bytes": alg, "GBps": gbs(alg, ms), "frac_of_peak": gbs(alg, ms) / HBM_PEAK_GBS, "kernels_ms": kms,
            "matches_full_encode": ok,
            "cpu_oracle": {"ms_per_call": 1e3 * oracle_s, "cores": 1, "kind": "oracle",
                           "sample": "one append of the same streams, host memory"}}


def measure_compare(svb, torch, np, inputs, steps, warmup, n=1 << 26, sweep_n=1 << 22):
    """Stream VByte against the comparison formats of Table 1 on the same integers: the 2^26
    document-id gaps of the headline workload, each format encoded and decoded on the device
    (plain, no differential step), checked against the input; then the storage comparison (bits
    per integer, and the extra over VByte) on 2^22 integers uniform below 2^b for a sweep of b."""
    x = inputs.docid_gaps(n, seed=2)
    x_dev = torch.from_numpy(x.view(np.int32)).cuda()
    fmts = {"stream_vbyte": (svb.svb_max_compressed_bytes, svb.svb_encode, svb.svb_decode),
            "vbyte": (svb.svb_vbyte_max_bytes, svb.svb_vbyte_encode, svb.svb_vbyte_decode),
            "varint_gb": (svb.svb_varintgb_max_bytes, svb.svb_varintgb_encode, svb.svb_varintgb_decode)}
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    res = {"n": n, "workload": "document-id gaps of the delta decode workload (plain decode)"}
    for name, (maxb, enc, dec) in fmts.items():
        comp = torch.empty(maxb(n), dtype=torch.uint8, device="cuda")
        ewall, ekms = timed_steps(svb, torch, lambda: enc(n, x_dev, comp, size), steps, warmup)
        torch.cuda.synchronize()
        nb = int(size.item())
        out.zero_()
        dwall, dkms = timed_steps(svb, torch, lambda: dec(n, comp, nb, out, err), steps, warmup)
        ok = bool(torch.equal(out, x_dev)) and int(err.item()) == 0
        dms, ems = 1e3 * dwall / steps, 1e3 * ewall / steps
        res[name] = {"bytes": nb, "bits_per_int": 8.0 * nb / n, "decode_ms": dms, "decode_uint32_per_s": n / (dms * 1e-3),
                     "decode_GBps": gbs(nb + 4 * n, dms), "decode_kernels_ms": dkms, "encode_ms": ems,
                     "encode_uint32_per_s": n / (ems * 1e-3), "encode_kernels_ms": ekms, "round_trip_ok": ok}
        del comp
    for name in ("vbyte", "varint_gb"):
        res[name]["stream_vbyte_decode_speedup"] = res[name]["decode_ms"] / res["stream_vbyte"]["decode_ms"]
    sweep = []
    comp = torch.empty(svb.svb_vbyte_max_bytes(sweep_n), dtype=torch.uint8, device="cuda")
    for b in (4, 7, 8, 12, 14, 16, 20, 21, 24, 28, 32):
        xs = torch.from_numpy(inputs.bounded_gaps(sweep_n, b, seed=100 + b).view(np.int32)).cuda()
        row = {"bits": b}
        for name, (_, enc, _) in fmts.items():
            enc(sweep_n, xs, comp, size)
            torch.cuda.synchronize()
            row[name] = 8.0 * int(size.item()) / sweep_n
        row["stream_vbyte_extra"] = row["stream_vbyte"] - row["vbyte"]
        row["varint_gb_extra"] = row["varint_gb"] - row["vbyte"]
        sweep.append(row)
    res["storage_bits_per_int"] = {"n": sweep_n, "values": "uniform in [0, 2^bits)", "rows": sweep}
    del x_dev, out, comp
    return res


def build_pool(svb, torch, np, inputs, m, total, cap, seed):
    """Serving pool: m delta-coded posting lists (rank-size Zipf lengths in [1, cap] summing to
    `total`, sorted sets over [0, 2^31) drawn on the GPU), encoded by the batched encoder and
    packed back to back.  Returns device tables plus the source values for checking."""
    lens = inputs.zipf_rank_lengths(m, total, cap, seed=seed)
    vals, offs = inputs.sorted_sets_device(lens, seed=seed + 1)
    counts = lens.astype(np.uint64)
    n = int(counts.sum())
    u64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
    caps = (counts + 3) // 4 + 4 * counts
    loose_off = np.zeros(m, dtype=np.uint64)
    np.cumsum(caps[:-1], out=loose_off[1:])
    d_counts, d_val_off = u64(counts), u64(offs[:-1])
    starts = torch.zeros(m, dtype=torch.int32, device="cuda")
    sizes = torch.empty(m, dtype=torch.int64, device="cuda")
    loose = torch.empty(int(caps.sum()), dtype=torch.uint8, device="cuda")
    svb.svb_encode_batch(m, d_counts, d_val_off, vals, u64(loose_off), loose, sizes, starts, n)
    h_sizes = sizes.cpu().numpy().view(np.uint64).copy()
    del loose
    tight_off = np.zeros(m, dtype=np.uint64)
    np.cumsum(h_sizes[:-1], out=tight_off[1:])
    nbytes = int(h_sizes.sum())
    tight = torch.empty(nbytes + 64, dtype=torch.uint8, device="cuda")
    sizes2 = torch.empty(m, dtype=torch.int64, device="cuda")
    d_tight_off = u64(tight_off)
    svb.svb_encode_batch(m, d_counts, d_val_off, vals, d_tight_off, tight, sizes2, starts, n)
    torch.cuda.synchronize()
    assert torch.equal(sizes, sizes2), "pool encode is not deterministic"
    return {"counts": d_counts, "in_off": d_tight_off, "in_bytes": sizes, "streams": tight, "starts": starts,
            "vals": vals, "val_off": offs, "h_counts": counts, "integers": n, "compressed_bytes": nbytes}


def latency_summary(lat, ints, wall):
    import numpy as np
    return {"queries": int(lat.size), "wall_s": wall, "qps": lat.size / wall,
            "uint32_per_s": float(ints) / wall, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean())}


SERVE_TRACE_QUERIES = 1 << 22  # queries of the open loops' trace, used cyclically


def measure_serving(svb, torch, np, inputs, seconds, lists=1_000_000, total=1_600_000_000, cap=1 << 22,
                    arena_bytes=1 << 30, slots=16, max_batch_lists=16384):
    """Serving loop over a device-resident pool of delta-coded posting lists: closed-loop saturation,
    then open-loop Poisson arrivals at 0.5x and 0.8x of the saturation rate for `seconds` each
    (arrivals drawn in the native replay); each query 2..8 lists chosen uniformly (with replacement
    in the open loops); latency from arrival to the host seeing the batch complete."""
    from paper_1709_08990_amd import serve
    t0 = time.perf_counter()
    pool = build_pool(svb, torch, np, inputs, lists, total, cap, seed=91)
    log("serving: pool of %d lists, %d integers, %.2f GB compressed (%.1f s)"
        % (lists, pool["integers"], pool["compressed_bytes"] / 1e9, time.perf_counter() - t0))
    server = serve.Server(pool["counts"], pool["in_off"], pool["in_bytes"], pool["streams"], pool["starts"],
                          arena_bytes=arena_bytes, slots=slots, max_batch_lists=max_batch_lists)
    h_counts = pool["h_counts"]
    # correctness: a few queries read back from the arena against the source values
    _, check = inputs.poisson_queries(64, 1.0, lists, seed=92)
    for q, p in enumerate(check):
        server.submit(q, p)
    seen, ok = 0, True
    while seen < len(check):
        server.step(block=True)
        for qid, off, n in server.poll():
            p = check[qid]
            want = torch.cat([pool["vals"][int(pool["val_off"][l]):int(pool["val_off"][l + 1])] for l in p])
            got = torch.empty(max(1, n), dtype=torch.int32, device="cuda")
            if n:
                svb.svb_copy_u32(n, svb.svb_server_arena(server.handle) + 4 * off, got)
            torch.cuda.synchronize()
            ok = ok and torch.equal(got[:n], want)
            server.release(qid)
            seen += 1
    assert ok, "served results differ from the pool's source values"
    # the same integers as one delta-coded array: the single-array rate for data of this density
    n_all = pool["vals"].numel()
    comp = torch.empty(svb.svb_max_compressed_bytes(n_all), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n_all, pool["vals"], comp, 0, size)
    torch.cuda.synchronize()
    nb = int(size.item())
    out = torch.empty(n_all, dtype=torch.int32, device="cuda")
    flush = Flush(svb, torch)
    pr = protocol_steps(svb, torch, lambda: svb.svb_delta_decode(n_all, comp, nb, out, 0), MIN_REPS, 2, flush)
    same_ok = bool(torch.equal(out, pool["vals"]))
    same = {"n": n_all, "compressed_bytes": nb, "ms_per_call": pr["median_ms"],
            "uint32_per_s": n_all / (pr["median_ms"] * 1e-3), "round_trip_ok": same_ok}
    del comp, out, flush, pool["vals"]
    assert same_ok, "the pool's integers as one array did not round-trip"
    log("serving: the pool's %d integers as one array decode at %.3g ints/s" % (n_all, same["uint32_per_s"]))

    def query_ints(qoff, ids):
        c = h_counts[ids]
        return np.add.reduceat(c, qoff[:-1]).astype(np.float64) if ids.size else np.zeros(0)

    # warm-up, then closed loop at a few depths to find the saturation rate
    _, qo, ids = inputs.poisson_queries_flat(5_000, 1.0, lists, seed=93)
    server.replay((qo, ids), outstanding=512)
    closed = []
    est_qps = None
    for depth in (256, 1024, 4096, 16384, 65536):
        nq = 20_000 if est_qps is None else int(min(4e6, max(20_000, 2.0 * est_qps)))
        _, qo, ids = inputs.poisson_queries_flat(nq, 1.0, lists, seed=94 + depth)
        lat, wall = server.replay((qo, ids), outstanding=depth)
        r = latency_summary(lat, query_ints(qo, ids).sum(), wall)
        r["outstanding"] = depth
        closed.append(r)
        est_qps = max(est_qps or 0.0, r["qps"])
        log("serving closed loop depth %d: %.0f queries/s, %.3g ints/s, p50 %.3f ms, p99 %.3f ms"
            % (depth, r["qps"], r["uint32_per_s"], r["p50_ms"], r["p99_ms"]))
    sat = max(closed, key=lambda r: r["qps"])
    opened = []
    warmup = 0.25  # seconds of arrivals replayed first and left out of the figures (GPU clocks ramp up)
    # open loop: Poisson arrivals drawn in the replay itself over a trace of SERVE_TRACE_QUERIES
    # queries used cyclically, so a window of any length needs no host trace
    _, bq, bi = inputs.poisson_queries_flat(SERVE_TRACE_QUERIES, 1.0, lists, seed=97, distinct=False)
    for load in (0.5, 0.8):
        rate = load * sat["qps"]
        log("serving open loop %.1fx: %.3g queries/s, %.1f s of arrivals" % (load, rate, seconds + warmup))
        f = server.replay_poisson((bq, bi), rate, seconds + warmup, warmup_s=warmup, seed=97 + int(10 * load))
        r = {"queries": int(f["queries"]), "wall_s": f["wall_s"], "qps": f["queries"] / f["wall_s"],
             "uint32_per_s": f["ints"] / f["wall_s"], "p50_ms": 1e3 * f["p50_s"], "p99_ms": 1e3 * f["p99_s"],
             "mean_ms": 1e3 * f["mean_s"], "generated": int(f["generated"]), "batches": int(f["batches"]),
             "load": load, "offered_qps": rate, "window_s": seconds, "warmup_s": warmup,
             "trace_queries": SERVE_TRACE_QUERIES}
        r["batching"] = {"min_lists": 1024, "max_wait_us": 20}  # the server's defaults
        opened.append(r)
        log("serving open loop %.1fx: offered %.0f q/s over %.1f s, %.3g ints/s, p50 %.3f ms, p99 %.3f ms"
            % (load, rate, seconds, r["uint32_per_s"], r["p50_ms"], r["p99_ms"]))
    st = server.stats()
    server.close()
    assert st["err"] == 0, "a served batch reported corrupt input"
    return {"pool": {"lists": lists, "integers": pool["integers"], "compressed_bytes": pool["compressed_bytes"],
                     "max_list": int(h_counts.max()), "median_list": float(np.median(h_counts))},
            "arena_bytes": arena_bytes, "slots": slots, "max_batch_lists": max_batch_lists,
            "results_checked": len(check), "closed_loop": closed, "saturation_qps": sat["qps"],
            "saturation_uint32_per_s": sat["uint32_per_s"], "open_loop": opened, "server_stats": st,
            "single_array_same_ints": same}


def run_cpu_baseline(x, min_seconds=10.0):
    """The oracle as it stands: single-threaded scalar C delta decode of the whole array, repeated."""
    import oracle
    stream = oracle.encode(x, delta=True, start=0)
    times = []
    t_end = time.perf_counter() + min_seconds
    while len(times) < 3 or time.perf_counter() < t_end:
        t0 = time.perf_counter()
        oracle.decode(stream, x.size, delta=True, start=0)
        times.append(time.perf_counter() - t0)
        if len(times) >= 200:
            break
    times.sort()
    med = times[len(times) // 2]
    model, ncpu = host_cpu()
    return {"value": x.size / med, "unit": "uint32/s", "cores": 1, "kind": "oracle",
            "sample": "full %d-integer delta decode (the bench workload), %d repetitions, median, host memory"
                      % (x.size, len(times)),
            "host_cpu": model, "host_threads_available": ncpu}


ONLY_KINDS = ("delta26", "delta28", "plain28", "encode28", "batched", "seek8", "serve")


def profile_serve(steps, depth=16384, queries=2_000_000, slots=16, max_batch_lists=16384):
    """The serving pool of measure_serving and `steps` closed-loop replays of `queries` queries at
    `depth` outstanding, for profiler runs.  Prints one JSON line with the median rate."""
    import numpy as np
    import torch

    import paper_1709_08990_amd as svb
    from paper_1709_08990_amd import inputs, serve
    svb.lib()
    lists, total, cap = 1_000_000, 1_600_000_000, 1 << 22
    pool = build_pool(svb, torch, np, inputs, lists, total, cap, seed=91)
    del pool["vals"]
    server = serve.Server(pool["counts"], pool["in_off"], pool["in_bytes"], pool["streams"], pool["starts"],
                          arena_bytes=1 << 30, slots=slots, max_batch_lists=max_batch_lists)
    _, qo, ids = inputs.poisson_queries_flat(queries, 1.0, lists, seed=94)
    ints = float(pool["h_counts"][ids].sum())
    rates = []
    for _ in range(max(1, steps)):
        lat, wall = server.replay((qo, ids), outstanding=depth)
        rates.append((queries / wall, ints / wall, float(np.percentile(lat, 99)) * 1e3))
    st = server.stats()
    server.close()
    rates.sort()
    q, i, p99 = rates[len(rates) // 2]
    print(json.dumps({"only": "serve", "depth": depth, "queries": queries, "slots": slots,
                      "max_batch_lists": max_batch_lists, "qps": q, "uint32_per_s": i, "p99_ms": p99,
                      "server_stats": st}))


def profile_only(kind, steps, warmup, variant=None, dirty=False):
    """Runs one kind of call only (`warmup` + `steps` calls, each after the 1 GiB cache-evicting
    read, or write with `dirty`), for rocprofv3 runs that should see nothing else: delta26 / delta28 (delta decode of the
    document ids at 2^26 / 2^28), plain28 (plain decode of 2^28 integers of unpredictable length),
    encode28 (delta encode of the 2^28 document ids), batched (delta decode of the 200,000 posting
    lists), seek8 (2^22 seeks over 2^20 lists of 256 running sums of deltas below 2^8).  Prints one
    JSON line with the median call time by torch events.  One plain copy of COPY_WORDS words runs
    after the timed calls: counter runs scale each counter by what it reads for that copy."""
    import numpy as np
    import torch

    import paper_1709_08990_amd as svb
    from paper_1709_08990_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    svb.lib()
    if variant is not None:
        svb.svb_set_decode_variant(kind != "plain28", variant)
    flush = Flush(svb, torch)
    fl = flush.dirty if dirty else flush.clean
    if kind == "seek8":
        m, q = 1 << 20, 1 << 22
        vals, offs = inputs.seek_lists(m, 8, seed=98)
        x_dev = torch.from_numpy(vals.view(np.int32)).cuda()
        counts = np.full(m, 256, dtype=np.uint64)
        u64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
        cap = svb.svb_max_compressed_bytes(256)
        d_counts, d_val_off = u64(counts), u64(offs[:-1])
        comp = torch.empty(m * cap, dtype=torch.uint8, device="cuda")
        sizes = torch.empty(m, dtype=torch.int64, device="cuda")
        starts = torch.zeros(m, dtype=torch.int32, device="cuda")
        svb.svb_encode_batch(m, d_counts, d_val_off, x_dev, u64(np.arange(m, dtype=np.uint64) * cap), comp, sizes,
                             starts, 256 * m)
        torch.cuda.synchronize()
        h_sizes = sizes.cpu().numpy().view(np.uint64).copy()
        byte_off = np.zeros(m, dtype=np.uint64)
        np.cumsum(h_sizes[:-1], out=byte_off[1:])
        comp = torch.empty(int(h_sizes.sum()) + 64, dtype=torch.uint8, device="cuda")
        d_off = u64(byte_off)
        svb.svb_encode_batch(m, d_counts, d_val_off, x_dev, d_off, comp, sizes, starts, 256 * m)
        index = svb.svb_seek_index_create(m, d_counts, d_off, sizes, comp, starts, 256 * m)
        ids, targets, _ = inputs.seek_queries(vals, offs, q, seed=99)
        d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
        d_t = torch.from_numpy(targets.view(np.int32)).cuda()
        pos = torch.empty(q, dtype=torch.int64, device="cuda")
        val = torch.empty(q, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        n = q
        fn = lambda: svb.svb_seek_batch(index, q, d_ids, d_t, pos, val, err)

        def check():
            ok = int(err.item()) == 0
            ph, vh = pos.cpu().numpy(), val.cpu().numpy().view(np.uint32)
            for k in range(0, q, q // 1000):
                x = vals[offs[ids[k]]:offs[ids[k] + 1]]
                p = int(np.searchsorted(x, targets[k], side="left"))
                ok &= (int(ph[k]), int(vh[k])) == (p, int(x[p]) if p < x.size else 0)
            return ok
    elif kind == "batched":
        vals, offs = inputs.posting_lists()
        m = offs.size - 1
        counts = np.diff(offs).astype(np.uint64)
        total = int(counts.sum())
        x_dev = torch.from_numpy(vals.view(np.int32)).cuda()
        del vals
        caps = (counts + 3) // 4 + 4 * counts
        comp_off = np.zeros(m, dtype=np.uint64)
        np.cumsum(caps[:-1], out=comp_off[1:])
        u64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()
        d_counts, d_in_off, d_comp_off = u64(counts), u64(offs[:-1]), u64(comp_off)
        comp = torch.empty(int(caps.sum()), dtype=torch.uint8, device="cuda")
        sizes = torch.empty(m, dtype=torch.int64, device="cuda")
        starts = torch.zeros(m, dtype=torch.int32, device="cuda")
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        svb.svb_encode_batch(m, d_counts, d_in_off, x_dev, d_comp_off, comp, sizes, starts, total)
        args = (m, d_counts, d_comp_off, sizes, comp, d_in_off, out, starts, total, err)
        n = total
        fn = lambda: svb.svb_decode_batch(*args)
        check = lambda: bool(torch.equal(out, x_dev)) and int(err.item()) == 0
    else:
        n = 1 << (26 if kind == "delta26" else 28)
        x = inputs.stress_lengths(n, seed=3) if kind == "plain28" else inputs.docids(n, seed=2)[0]
        x_dev = torch.from_numpy(x.view(np.int32)).cuda()
        del x
        comp = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.int64, device="cuda")
        delta = kind != "plain28"
        (svb.svb_delta_encode(n, x_dev, comp, 0, size) if delta else svb.svb_encode(n, x_dev, comp, size))
        torch.cuda.synchronize()
        nb = int(size.item())
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        if kind == "encode28":
            fn = lambda: svb.svb_delta_encode(n, x_dev, comp, 0, size)
            check = lambda: int(size.item()) == nb
        elif delta:
            fn = lambda: svb.svb_delta_decode(n, comp, nb, out, 0, err)
            check = lambda: bool(torch.equal(out, x_dev)) and int(err.item()) == 0
        else:
            fn = lambda: svb.svb_decode(n, comp, nb, out, err)
            check = lambda: bool(torch.equal(out, x_dev)) and int(err.item()) == 0
    for _ in range(warmup):
        fl()
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        fl()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    med = ms[len(ms) // 2]
    ok = check()
    if kind == "seek8":
        svb.svb_seek_index_destroy(index)
    del x_dev, comp, flush
    ca = torch.empty(COPY_WORDS, dtype=torch.int32, device="cuda").fill_(7)
    cb = torch.empty_like(ca)
    svb.svb_copy_u32(COPY_WORDS, ca, cb)
    torch.cuda.synchronize()
    ok &= bool(torch.equal(ca, cb))
    print(json.dumps({"only": kind, "variant": variant, "n": n, "steps": steps, "warmup": warmup, "median_ms": med,
                      "uint32_per_s": n / (med * 1e-3), "ok": ok}))
    if not ok:
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--only", choices=ONLY_KINDS, default=None,
                    help="run one kind of call only (for profiler runs) and print its median time")
    ap.add_argument("--decode-variant", type=int, default=None,
                    help="with --only: the decoder variant to set first (svb_set_decode_variant)")
    ap.add_argument("--dirty-flush", action="store_true",
                    help="with --only: evict the caches by writing the 1 GiB buffer instead of reading it")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2p28", action="store_true", help="skip the 2^28 sub-measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 200,000-list batched measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-seek", action="store_true", help="skip the seek/select measurement")
    ap.add_argument("--no-append", action="store_true", help="skip the append measurement")
    ap.add_argument("--no-zero-control", action="store_true", help="skip the zero-control variant measurement")
    ap.add_argument("--no-compare", action="store_true", help="skip the VByte / varint-GB comparison")
    ap.add_argument("--no-per-list", action="store_true",
                    help="skip the one-call-per-list baseline of the batched measurement")
    ap.add_argument("--serve-slots", type=int, default=16, help="stream slots of the serving runtime")
    ap.add_argument("--serve-depth", type=int, default=16384, help="with --only serve: queries outstanding")
    ap.add_argument("--serve-batch-lists", type=int, default=16384, help="most lists per serving batch")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of each open-loop serving window (seconds of arrivals)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_MD"))
    ap.add_argument("--counter-command", default="rocprofv3 --pmc {COUNTER} --output-format csv -d "
                    "prof_out/pmc_{COUNTER} -o p -- python3 bench.py --steps 5 --warmup 2 --no-cpu-baseline "
                    "--no-2p28 --no-batched --no-serving --no-seek --no-append --no-zero-control --no-compare")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG",
                    help="OUT_MD TITLE CSV [CSV ...]: summary of rocprofv3 --pmc runs (every kernel); the "
                         "commands that made them go in --pmc-command, once each")
    ap.add_argument("--pmc-command", action="append", default=[])
    ap.add_argument("--pmc-only", action="append", default=None,
                    help="with --summarize-pmc: only kernels whose name holds this fragment (repeatable)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("STATS_CSV", "OUT_MD", "TITLE"))
    ap.add_argument("--trace-command", default="rocprofv3 --kernel-trace --stats --output-format csv -d "
                    "prof_out/prof_kt -o kt -- python3 bench.py --steps 5 --warmup 2 --no-cpu-baseline "
                    "--no-2p28 --no-batched --no-serving --no-seek --no-append --no-zero-control --no-compare")
    ap.add_argument("--trace-bench-json", default=None,
                    help="bench line printed by the traced command (for --summarize-trace)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, command=args.trace_command, bench_json=args.trace_bench_json)
        return
    if args.summarize_pmc:
        if len(args.summarize_pmc) < 3:
            ap.error("--summarize-pmc needs OUT_MD TITLE CSV [CSV ...]")
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.pmc_command, args.summarize_pmc[2:],
                      args.pmc_only)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, command=args.counter_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)." % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.only == "serve":
        profile_serve(args.steps, depth=args.serve_depth, slots=args.serve_slots, max_batch_lists=args.serve_batch_lists)
        return
    if args.only:
        profile_only(args.only, args.steps, args.warmup, args.decode_variant, args.dirty_flush)
        return

    import numpy as np
    import torch

    import paper_1709_08990_amd as svb
    from paper_1709_08990_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    svb.lib()
    log("generating %d document ids" % N_HEAD)
    x, _ = inputs.docids(N_HEAD, seed=2)
    x_dev = torch.from_numpy(x.view(np.int32)).cuda()
    flush = Flush(svb, torch)
    log("delta decode: %d warmup + %d timed steps (at least %d flushed reps)" % (args.warmup, args.steps, MIN_REPS))
    r = measure_delta(svb, torch, x_dev, args.steps, args.warmup, flush)
    assert r["round_trip_ok"], "delta decode did not reproduce the input"
    dom_name = max(r["kernels_ms"], key=r["kernels_ms"].get)
    dom_ms = r["kernels_ms"][dom_name]
    log("delta decode %.4f ms/call (flushed median); dominant kernel %s %.4f ms"
        % (r["ms_per_call"], dom_name, dom_ms))
    copy = measure_copy(svb, torch, max(5, args.steps // 2))
    log("copy %.1f GB/s" % copy["GBps"])

    line = {
        "metric": METRIC,
        "value": r["uint32_per_s"],
        "unit": "uint32/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N_HEAD, "compressed_bytes": r["compressed_bytes"],
                   "bits_per_int": round(r["bits_per_int"], 4), "parallelism": "none (1 GPU)",
                   "timing": "median of %d calls, each after a 1 GiB cache-evicting read (HIP events)"
                             % r["protocol"]["reps"]},
        # the dominant kernel reads the control and data bytes and writes every integer: its
        # algorithmic bytes are the call's
        "roofline": {"bound": "hbm", "achieved": gbs(r["alg_bytes_per_call"], dom_ms), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs(r["alg_bytes_per_call"], dom_ms) / HBM_PEAK_GBS,
                     "traffic": stored_traffic(), "kernel": dom_name, "kernel_ms": dom_ms,
                     "alg_bytes_per_launch": r["alg_bytes_per_call"],
                     "whole_call": {"ms": r["ms_per_call"], "GBps": r["call_GBps"],
                                    "frac": r["call_frac_of_peak"]}},
        "kernels_ms": r["kernels_ms"],
        "timed_region_s": r["protocol"]["timed_region_s"],
        "protocol": r["protocol"],
        "dirty_flush": r["dirty_flush"],
        "unflushed": r["unflushed"],
        "encode": r["encode"],
        "copy": copy,
    }
    del x_dev
    if not args.no_2p28:
        n2 = 1 << 28
        log("generating %d document ids" % n2)
        x2, _ = inputs.docids(n2, seed=2)
        x2_dev = torch.from_numpy(x2.view(np.int32)).cuda()
        del x2
        r2 = measure_delta(svb, torch, x2_dev, MIN_REPS, 2, flush)
        assert r2["round_trip_ok"], "2^28 delta decode did not reproduce the input"
        del x2_dev
        log("2^28 delta decode %.4f ms/call (%.1f%% of peak, flushed median)"
            % (r2["ms_per_call"], 100 * r2["call_frac_of_peak"]))
        line["at_2p28"] = {"delta_docids": {k: r2[k] for k in (
            "n", "compressed_bytes", "ms_per_call", "uint32_per_s", "call_GBps", "call_frac_of_peak", "kernels_ms",
            "dirty_flush", "unflushed", "encode")}}
        log("2^28 delta encode %.4f ms/call (%.1f%% of peak)"
            % (r2["encode"]["ms_per_call"], 100 * r2["encode"]["frac_of_peak"]))
        log("generating %d stress integers" % n2)
        x3 = inputs.stress_lengths(n2, seed=3)
        x3_dev = torch.from_numpy(x3.view(np.int32)).cuda()
        del x3
        r3 = measure_plain(svb, torch, x3_dev, MIN_REPS, 2, flush)
        assert r3["round_trip_ok"], "2^28 plain decode did not reproduce the input"
        del x3_dev
        log("2^28 plain decode %.4f ms/call (%.1f%% of peak)" % (r3["ms_per_call"], 100 * r3["call_frac_of_peak"]))
        line["at_2p28"]["plain_stress"] = r3
    del flush
    if not args.no_batched:
        log("batched: generating 200,000 posting lists")
        rb = measure_batched(svb, torch, np, inputs, max(5, args.steps // 2), 2, per_list=not args.no_per_list)
        assert rb["round_trip_ok"], "batched decode mismatch"
        single = line.get("at_2p28", {}).get("delta_docids", {}).get("uint32_per_s", line["value"])
        rb["vs_single_array"] = rb["uint32_per_s"] / single
        if "one_call_per_list" in rb:
            assert rb["one_call_per_list"]["round_trip_ok"], "per-list decode mismatch"
            rb["vs_one_call_per_list"] = rb["uint32_per_s"] / rb["one_call_per_list"]["uint32_per_s"]
        line["batched"] = rb
        log("batched delta decode %.4f ms/call, %.3g ints/s (%.2fx single array; %.2fx one array of the same ints)"
            % (rb["ms_per_call"], rb["uint32_per_s"], rb["vs_single_array"], rb["vs_single_array_same_ints"]))
    if not args.no_seek:
        log("seek/select: 2^20 lists of 256 integers, 2^22 queries per call")
        rk = measure_seek(svb, torch, np, inputs, max(5, args.steps // 2), 2)
        assert all(r["sample_matches_input"] for r in rk.values()), "seek/select mismatch"
        line["seek_select"] = rk
        for b, r in rk.items():
            log("seek %s: %.3g queries/s (%.1f%% of HBM peak), select %.3g queries/s"
                % (b, r["seek"]["queries_per_s"], 100 * r["seek"]["frac_of_peak"], r["select"]["queries_per_s"]))
    if not args.no_append:
        log("append: 2^22 document ids appended to a stream of 2^26")
        ra = measure_append(svb, torch, np, inputs, max(5, args.steps // 2), 2)
        assert ra["matches_full_encode"], "append mismatch"
        line["append"] = ra
        log("append %.4f ms/call, %.0f GB/s (%.1f%% of peak); oracle %.1f ms"
            % (ra["ms_per_call"], ra["GBps"], 100 * ra["frac_of_peak"], ra["cpu_oracle"]["ms_per_call"]))
    if not args.no_zero_control:
        log("zero-control variant: 2^28 running sums of deltas below 2^8")
        rz = measure_zero_control(svb, torch, np, max(5, args.steps // 2), 2)
        assert rz["variant0"]["round_trip_ok"] and rz["variant1"]["round_trip_ok"], "zero-control decode mismatch"
        line["zero_control"] = rz
        log("zero-control variant: general %.4f ms, zero-control %.4f ms (%.2fx)"
            % (rz["variant0"]["ms_per_call"], rz["variant1"]["ms_per_call"], rz["speedup"]))
    if not args.no_compare:
        log("comparison formats: Stream VByte, VByte, varint-GB on the 2^26 document-id gaps")
        rc = measure_compare(svb, torch, np, inputs, max(5, args.steps // 2), 2)
        assert all(rc[f]["round_trip_ok"] for f in ("stream_vbyte", "vbyte", "varint_gb")), "comparison mismatch"
        line["compare"] = rc
        log("decode ms: Stream VByte %.4f, VByte %.4f, varint-GB %.4f; bits/int %.2f / %.2f / %.2f"
            % (rc["stream_vbyte"]["decode_ms"], rc["vbyte"]["decode_ms"], rc["varint_gb"]["decode_ms"],
               rc["stream_vbyte"]["bits_per_int"], rc["vbyte"]["bits_per_int"], rc["varint_gb"]["bits_per_int"]))
    if not args.no_serving:
        log("serving: building the 10^6-list pool on the GPU")
        rs = measure_serving(svb, torch, np, inputs, args.serve_seconds, slots=args.serve_slots,
                             max_batch_lists=args.serve_batch_lists)
        single = line.get("at_2p28", {}).get("delta_docids", {}).get("uint32_per_s", line["value"])
        rs["saturation_vs_single_array"] = rs["saturation_uint32_per_s"] / single
        rs["saturation_vs_single_array_same_ints"] = (rs["saturation_uint32_per_s"] /
                                                      rs["single_array_same_ints"]["uint32_per_s"])
        log("serving saturation %.3g ints/s: %.2fx the 2^28 document-id array, %.2fx the pool's integers as one "
            "array" % (rs["saturation_uint32_per_s"], rs["saturation_vs_single_array"],
                       rs["saturation_vs_single_array_same_ints"]))
        line["serving"] = rs
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = run_cpu_baseline(x)
    line["source_digest"] = source_digest()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
