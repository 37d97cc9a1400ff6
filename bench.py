#!/usr/bin/env python3
"""Stream VByte on one MI355X: delta-decode throughput against the HBM roofline.

One step = one delta decode (svb_delta_decode: control-byte lengths, byte-offset
scan, byte gather, fused wrap-around prefix sum, store) of 2^26 sorted document
ids whose gaps are geometric with mean 8 (probability 0.99) or uniform in
[2^8, 2^20) (probability 0.01), start value 0.  The compressed input is made by
the library's own delta encoder and is resident in HBM before timing starts.

Prints one JSON line.  Besides the headline it carries:
  roofline      the decode kernel's algorithmic bytes per launch over its average
                duration (HIP events on the launch stream) against 8 TB/s;
  cpu_baseline  the scalar C oracle, single-threaded, on the host cores;
  encode        delta encode of the same array, timed the same way;
  flushed       the decode kernel with a 1 GiB cache-evicting write before each launch;
  at_2p28       delta decode (and encode) of the same generator at 2^28 integers.
"""
import argparse
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


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def source_digest():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1709_08990_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(name):
    """HBM bytes per launch from a committed counter summary, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name)
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


def time_launches(fn, steps, torch, before=None):
    """Runs fn() `steps` times on the current stream with an event pair around each launch.
    Returns (wall seconds for the whole loop, mean per-launch milliseconds)."""
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
    ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    return wall, ms


def run_cpu_baseline(x, min_seconds=10.0):
    """The oracle as it stands: single-threaded scalar C delta decode of the whole array, repeated."""
    import oracle
    stream = oracle.encode(x, delta=True, start=0)
    times = []
    t_end = time.perf_counter() + min_seconds
    while len(times) < 3 or time.perf_counter() < t_end:
        t0 = time.perf_counter()
        vals, _ = oracle.decode(stream, x.size, delta=True, start=0)
        times.append(time.perf_counter() - t0)
        if len(times) >= 200:
            break
    times.sort()
    med = times[len(times) // 2]
    model, ncpu = host_cpu()
    return {"value": x.size / med, "unit": "uint32/s", "cores": 1, "kind": "oracle",
            "sample": "full %d-integer delta decode, %d repetitions (median), host memory" % (x.size, len(times)),
            "host_cpu": model, "host_threads_available": ncpu}


def measure_decode(svb, torch, n, x_dev, steps, warmup, flush_buf=None):
    """Encode once on the GPU, then time delta decodes.  Returns a dict of results."""
    comp = torch.empty(svb.svb_max_compressed_bytes(n), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    svb.svb_delta_encode(n, x_dev, comp, 0, size)
    torch.cuda.synchronize()
    nbytes = int(size.item())
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    def dec():
        svb.svb_delta_decode(n, comp, nbytes, out, 0, err)

    def enc():
        svb.svb_delta_encode(n, x_dev, comp, 0, size)

    for _ in range(warmup):
        dec()
    wall, ms = time_launches(dec, steps, torch)
    torch.cuda.synchronize()
    ok = bool(torch.equal(out, x_dev)) and int(err.item()) == 0
    alg = nbytes + 4 * n
    res = {"n": n, "compressed_bytes": nbytes, "bits_per_int": 8.0 * nbytes / n,
           "alg_bytes_per_launch": alg, "wall_s": wall, "kernel_ms": ms, "round_trip_ok": ok,
           "decode_uint32_per_s": n / (ms * 1e-3), "decode_GBps": alg / (ms * 1e-3) / 1e9}
    res["decode_frac_of_peak"] = res["decode_GBps"] / HBM_PEAK_GBS
    if flush_buf is not None:
        fl = lambda: svb.svb_fill_u32(flush_buf.numel(), flush_buf, 0)
        _, fms = time_launches(dec, max(3, steps // 2), torch, before=fl)
        res["flushed"] = {"kernel_ms": fms, "GBps": alg / (fms * 1e-3) / 1e9,
                          "frac_of_peak": alg / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "note": "1 GiB fill before each launch evicts L2 and the 256 MB MALL"}
    for _ in range(max(1, warmup // 2)):
        enc()
    _, ems = time_launches(enc, steps, torch)
    torch.cuda.synchronize()
    res["encode"] = {"kernel_ms": ems, "uint32_per_s": n / (ems * 1e-3),
                     "GBps": alg / (ems * 1e-3) / 1e9, "frac_of_peak": alg / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "size_ok": int(size.item()) == nbytes}
    del comp, out
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2p28", action="store_true", help="skip the 2^28 sub-measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_08990_amd as svb
    from paper_1709_08990_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    svb.lib()
    n = 1 << 26
    log("generating %d document ids" % n)
    x, _ = inputs.docids(n, seed=2)
    x_dev = torch.from_numpy(x.view(np.int32)).cuda()
    flush = torch.empty(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB
    log("timing delta decode, %d warmup + %d steps" % (args.warmup, args.steps))
    r = measure_decode(svb, torch, n, x_dev, args.steps, args.warmup, flush_buf=flush)
    assert r["round_trip_ok"], "delta decode did not reproduce the input"
    log("decode %.4f ms/launch, %.1f GB/s" % (r["kernel_ms"], r["decode_GBps"]))

    traffic = stored_traffic("counters_delta_decode_docids_2p26.md")
    line = {
        "metric": METRIC,
        "value": n * args.steps / r["wall_s"],
        "unit": "uint32/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": n, "compressed_bytes": r["compressed_bytes"],
                   "bits_per_int": round(r["bits_per_int"], 4), "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": r["decode_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["decode_frac_of_peak"], "traffic": traffic,
                     "kernel": "svb::decode_kernel<4, true>", "kernel_ms": r["kernel_ms"],
                     "alg_bytes_per_launch": r["alg_bytes_per_launch"]},
        "flushed": r.get("flushed"),
        "encode": r["encode"],
    }
    del x_dev
    if not args.no_2p28:
        n2 = 1 << 28
        log("generating %d document ids" % n2)
        x2, _ = inputs.docids(n2, seed=2)
        x2_dev = torch.from_numpy(x2.view(np.int32)).cuda()
        del x2
        r2 = measure_decode(svb, torch, n2, x2_dev, max(5, args.steps // 2), 2, flush_buf=flush)
        assert r2["round_trip_ok"], "2^28 delta decode did not reproduce the input"
        line["at_2p28"] = {k: r2[k] for k in ("n", "compressed_bytes", "kernel_ms", "decode_uint32_per_s",
                                               "decode_GBps", "decode_frac_of_peak", "flushed", "encode")}
        log("2^28 decode %.4f ms/launch, %.1f GB/s" % (r2["kernel_ms"], r2["decode_GBps"]))
        del x2_dev
    del flush
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = run_cpu_baseline(x)
    line["source_digest"] = source_digest()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
