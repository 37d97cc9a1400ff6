"""Stream VByte on AMD Instinct MI355X: Python binding of libsvb.so.

The functions named ``svb_*`` mirror the C ABI of ``include/svb.h`` one to one:
they only marshal arguments (torch tensors -> device pointers, the current HIP
stream) and raise ``SvbError`` on a non-zero status.  Every step of encoding
and decoding runs in the HIP kernels of the library; there is no CPU path.

The convenience wrappers ``encode`` / ``decode`` allocate outputs with torch.
Integer arrays are torch ``int32`` tensors holding the uint32 bit patterns.
"""
import ctypes
import os

__all__ = [
    "SvbError", "lib", "svb_control_bytes", "svb_max_compressed_bytes", "svb_encode",
    "svb_delta_encode", "svb_decode", "svb_delta_decode", "svb_delta_decode_noalloc", "svb_encode_batch",
    "svb_decode_batch",
    "svb_strerror", "svb_release_workspace", "svb_version", "svb_copy_u32", "svb_fill_u32",
    "svb_set_kernel_timing", "svb_kernel_times", "svb_autotune_decode_batch", "svb_autotune_encode_batch",
    "svb_set_batch_chunk", "svb_server_create", "svb_server_submit", "svb_server_step", "svb_server_poll",
    "svb_server_release", "svb_server_arena", "svb_server_stats", "svb_server_destroy", "svb_server_replay",
    "svb_server_replay_poisson",
    "svb_server_set_batching", "svb_seek_index_create", "svb_seek_batch", "svb_select_batch",
    "svb_seek_index_destroy", "svb_append", "svb_delta_append", "svb_autotune_decode", "svb_set_decode_variant",
    "encode", "decode",
    "LIB_PATH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsvb.so")
SVB_DECODE_CORRUPT = 1
SVB_BATCH_OVERFLOW = 3
SVB_QUERY_OUT_OF_RANGE = 4

_lib = None


class SvbError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (what, _strerror(status), status))


def lib():
    """The loaded libsvb.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsvb.so is not built (%s); run `python -m paper_1709_08990_amd.build`"
                               % LIB_PATH)
        # torch ships its own HIP runtime under the same soname as the system one.  Loading torch
        # first makes libsvb.so bind to that runtime, so the process has one HIP runtime, whose
        # device pointers and streams the tensors carry (the other one need not even see the GPU).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, vp, i32, f64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sigs = {
            "svb_control_bytes": (u64, [u64]),
            "svb_max_compressed_bytes": (u64, [u64]),
            "svb_encode": (i32, [u64, vp, vp, vp, vp]),
            "svb_delta_encode": (i32, [u64, vp, vp, u32, vp, vp]),
            "svb_decode": (i32, [u64, vp, u64, vp, vp, vp]),
            "svb_delta_decode": (i32, [u64, vp, u64, vp, u32, vp, vp]),
            "svb_delta_decode_noalloc": (i32, [u64, vp, u64, vp, u32, vp, vp]),
            "svb_encode_batch": (i32, [u32, vp, vp, vp, vp, vp, vp, vp, u64, vp]),
            "svb_decode_batch": (i32, [u32, vp, vp, vp, vp, vp, vp, vp, u64, vp, vp]),
            "svb_autotune_decode_batch": (i32, [u32, vp, vp, vp, vp, vp, vp, vp, u64, vp, vp, vp]),
            "svb_autotune_encode_batch": (i32, [u32, vp, vp, vp, vp, vp, vp, vp, u64, vp, vp]),
            "svb_set_batch_chunk": (i32, [i32, u32]),
            "svb_server_create": (i32, [u32, vp, vp, vp, vp, vp, u64, u32, u32, vp]),
            "svb_server_submit": (i32, [vp, u64, u32, vp]),
            "svb_server_step": (i32, [vp, i32]),
            "svb_server_poll": (i32, [vp, vp, vp, vp, u32]),
            "svb_server_release": (i32, [vp, u64]),
            "svb_server_arena": (vp, [vp]),
            "svb_server_stats": (i32, [vp, vp, u32]),
            "svb_server_destroy": (i32, [vp]),
            "svb_server_replay": (i32, [vp, u64, vp, vp, vp, u32, vp, vp]),
            "svb_server_replay_poisson": (i32, [vp, u64, vp, vp, f64, f64, f64, u64, vp, u32]),
            "svb_server_set_batching": (i32, [vp, u32, u32]),
            "svb_seek_index_create": (i32, [u32, vp, vp, vp, vp, vp, u64, vp, vp]),
            "svb_seek_batch": (i32, [vp, u32, vp, vp, vp, vp, vp, vp]),
            "svb_select_batch": (i32, [vp, u32, vp, vp, vp, vp, vp]),
            "svb_seek_index_destroy": (i32, [vp]),
            "svb_append": (i32, [u64, vp, u64, u64, vp, vp, vp, vp]),
            "svb_autotune_decode": (i32, [u64, vp, u64, vp, u32, i32, vp, vp, vp]),
            "svb_set_decode_variant": (i32, [i32, i32]),
            "svb_delta_append": (i32, [u64, vp, u64, u64, vp, u32, vp, vp, vp]),
            "svb_vbyte_max_bytes": (u64, [u64]),
            "svb_vbyte_encode": (i32, [u64, vp, vp, vp, vp]),
            "svb_vbyte_decode": (i32, [u64, vp, u64, vp, vp, vp]),
            "svb_varintgb_max_bytes": (u64, [u64]),
            "svb_varintgb_encode": (i32, [u64, vp, vp, vp, vp]),
            "svb_varintgb_decode": (i32, [u64, vp, u64, vp, vp, vp]),
            "svb_strerror": (ctypes.c_char_p, [i32]),
            "svb_release_workspace": (None, []),
            "svb_version": (ctypes.c_char_p, []),
            "svb_copy_u32": (i32, [u64, vp, vp, vp]),
            "svb_fill_u32": (i32, [u64, vp, u32, vp]),
            "svb_set_kernel_timing": (i32, [i32]),
            "svb_kernel_times": (i32, [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float), i32]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(status):
    try:
        return lib().svb_strerror(int(status)).decode()
    except Exception:  # pragma: no cover - only while reporting another error
        return "status %d" % status


def _ptr(t):
    """Device address of a tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status, what):
    if status != 0:
        raise SvbError(status, what)
    return status


def _check_count(status, what):
    """For calls that return a count (>= 0) or a negative svb_status."""
    if status < 0:
        raise SvbError(status, what)
    return status


# ------------------------------------------------------------------ C ABI mirror

def svb_control_bytes(n):
    return int(lib().svb_control_bytes(int(n)))


def svb_max_compressed_bytes(n):
    return int(lib().svb_max_compressed_bytes(int(n)))


def svb_encode(n, inp, out, out_bytes=None, stream=None):
    return _check(lib().svb_encode(int(n), _ptr(inp), _ptr(out), _ptr(out_bytes), _stream(stream)),
                  "svb_encode")


def svb_delta_encode(n, inp, out, start=0, out_bytes=None, stream=None):
    return _check(lib().svb_delta_encode(int(n), _ptr(inp), _ptr(out), int(start) & 0xFFFFFFFF,
                                         _ptr(out_bytes), _stream(stream)), "svb_delta_encode")


def svb_decode(n, inp, in_bytes, out, err=None, stream=None):
    return _check(lib().svb_decode(int(n), _ptr(inp), int(in_bytes), _ptr(out), _ptr(err),
                                   _stream(stream)), "svb_decode")


def svb_delta_decode(n, inp, in_bytes, out, start=0, err=None, stream=None):
    return _check(lib().svb_delta_decode(int(n), _ptr(inp), int(in_bytes), _ptr(out),
                                         int(start) & 0xFFFFFFFF, _ptr(err), _stream(stream)),
                  "svb_delta_decode")


SVB_NOALLOC_MAX_N = 1 << 30


def svb_delta_decode_noalloc(n, inp, in_bytes, out, start=0, err=None, stream=None):
    return _check(lib().svb_delta_decode_noalloc(int(n), _ptr(inp), int(in_bytes), _ptr(out),
                                                 int(start) & 0xFFFFFFFF, _ptr(err), _stream(stream)),
                  "svb_delta_decode_noalloc")


def _total_ints(total_ints):
    """The batched calls size their task table from total_ints, an upper bound on the integers of
    all lists: with 0 every list must fit one 1024-integer segment, and a longer one makes the call
    do nothing but flag SVB_BATCH_OVERFLOW.  So the binding asks for the bound explicitly."""
    if total_ints is None:
        raise ValueError("total_ints is required: an upper bound on the integers of all lists")
    return int(total_ints)


def svb_encode_batch(m, counts, in_off, inp, out_off, out, out_bytes=None, starts=None, total_ints=None,
                     stream=None):
    total_ints = _total_ints(total_ints)
    return _check(lib().svb_encode_batch(int(m), _ptr(counts), _ptr(in_off), _ptr(inp), _ptr(out_off),
                                         _ptr(out), _ptr(out_bytes), _ptr(starts), int(total_ints),
                                         _stream(stream)), "svb_encode_batch")


def svb_decode_batch(m, counts, in_off, in_bytes, inp, out_off, out, starts=None, total_ints=None, err=None,
                     stream=None):
    total_ints = _total_ints(total_ints)
    return _check(lib().svb_decode_batch(int(m), _ptr(counts), _ptr(in_off), _ptr(in_bytes), _ptr(inp),
                                         _ptr(out_off), _ptr(out), _ptr(starts), int(total_ints), _ptr(err),
                                         _stream(stream)), "svb_decode_batch")


def svb_autotune_decode_batch(m, counts, in_off, in_bytes, inp, out_off, out, starts=None, total_ints=None,
                              err=None, stream=None):
    """Times each chunk choice (consecutive tasks per wave) on this batch, keeps the fastest for
    later calls of this kind; returns it."""
    total_ints = _total_ints(total_ints)
    chosen = ctypes.c_uint32(0)
    _check(lib().svb_autotune_decode_batch(int(m), _ptr(counts), _ptr(in_off), _ptr(in_bytes), _ptr(inp),
                                           _ptr(out_off), _ptr(out), _ptr(starts), int(total_ints), _ptr(err),
                                           ctypes.addressof(chosen), _stream(stream)), "svb_autotune_decode_batch")
    return int(chosen.value)


def svb_autotune_encode_batch(m, counts, in_off, inp, out_off, out, out_bytes=None, starts=None, total_ints=None,
                              stream=None):
    total_ints = _total_ints(total_ints)
    chosen = ctypes.c_uint32(0)
    _check(lib().svb_autotune_encode_batch(int(m), _ptr(counts), _ptr(in_off), _ptr(inp), _ptr(out_off),
                                           _ptr(out), _ptr(out_bytes), _ptr(starts), int(total_ints),
                                           ctypes.addressof(chosen), _stream(stream)), "svb_autotune_encode_batch")
    return int(chosen.value)


SVB_BATCH_QUEUE = 0x100


def svb_set_batch_chunk(kind, chunk):
    """kind = 2 * encode + delta; chunk (consecutive tasks per wave) in {1, 2, 4, 8, 16}, or for
    decoding chunk | SVB_BATCH_QUEUE (the work-queue schedule)."""
    return _check(lib().svb_set_batch_chunk(int(kind), int(chunk)), "svb_set_batch_chunk")


def svb_strerror(status):
    return _strerror(status)


def svb_release_workspace():
    lib().svb_release_workspace()


def svb_version():
    return lib().svb_version().decode()


def svb_copy_u32(n, inp, out, stream=None):
    return _check(lib().svb_copy_u32(int(n), _ptr(inp), _ptr(out), _stream(stream)), "svb_copy_u32")


def svb_fill_u32(n, out, value, stream=None):
    return _check(lib().svb_fill_u32(int(n), _ptr(out), int(value) & 0xFFFFFFFF, _stream(stream)),
                  "svb_fill_u32")


def svb_set_kernel_timing(enable):
    return _check(lib().svb_set_kernel_timing(1 if enable else 0), "svb_set_kernel_timing")


def svb_kernel_times(cap=4096):
    """[(kernel name, milliseconds)] recorded by the calling thread since the previous call
    (synchronises on them; records beyond ``cap`` are dropped)."""
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_float * cap)()
    n = lib().svb_kernel_times(names, ms, cap)
    if n < 0:
        raise SvbError(n, "svb_kernel_times")
    return [(names[i].decode(), float(ms[i])) for i in range(min(n, cap))]


def svb_server_create(m, counts, in_off, in_bytes, inp, starts, arena_bytes, streams=4, max_batch_lists=8192):
    """Returns the server handle (an int)."""
    h = ctypes.c_void_p()
    _check(lib().svb_server_create(int(m), _ptr(counts), _ptr(in_off), _ptr(in_bytes), _ptr(inp), _ptr(starts),
                                   int(arena_bytes), int(streams), int(max_batch_lists), ctypes.addressof(h)),
           "svb_server_create")
    return h.value


def svb_server_submit(server, query_id, list_ids):
    """list_ids: host sequence of list indices."""
    import numpy as np
    ids = np.ascontiguousarray(list_ids, dtype=np.uint32)
    return _check(lib().svb_server_submit(server, int(query_id), int(ids.size), ids.ctypes.data), "svb_server_submit")


def svb_server_step(server, block=False):
    """Returns the number of completed queries not yet polled."""
    return _check_count(lib().svb_server_step(server, 1 if block else 0), "svb_server_step")


def svb_server_poll(server, cap=4096):
    """[(query id, arena offset, integers)] of queries completed since the last poll."""
    import numpy as np
    ids = np.zeros(cap, dtype=np.uint64)
    off = np.zeros(cap, dtype=np.uint64)
    n = np.zeros(cap, dtype=np.uint64)
    k = _check_count(lib().svb_server_poll(server, ids.ctypes.data, off.ctypes.data, n.ctypes.data, int(cap)),
               "svb_server_poll")
    return [(int(ids[i]), int(off[i]), int(n[i])) for i in range(k)]


def svb_server_release(server, query_id):
    return _check(lib().svb_server_release(server, int(query_id)), "svb_server_release")


def svb_server_arena(server):
    return lib().svb_server_arena(server)


SERVER_STATS = ("batches", "lists", "integers", "admitted", "completed", "peak_busy_slots", "err",
                "arena_peak_ints", "waiting", "admitted_not_launched", "arena_in_use_ints", "steps", "slow_steps",
                "max_step_us")


def svb_server_stats(server):
    import numpy as np
    out = np.zeros(len(SERVER_STATS), dtype=np.uint64)
    _check(lib().svb_server_stats(server, out.ctypes.data, len(SERVER_STATS)), "svb_server_stats")
    return {k: int(v) for k, v in zip(SERVER_STATS, out)}


def svb_server_set_batching(server, min_lists, max_wait_us):
    return _check(lib().svb_server_set_batching(server, int(min_lists), int(max_wait_us)), "svb_server_set_batching")


def svb_server_destroy(server):
    return _check(lib().svb_server_destroy(server), "svb_server_destroy")


def svb_autotune_decode(n, inp, in_bytes, out, start=0, delta=False, err=None, stream=None):
    """Times the decoder variants of this kind (plain: 0..1; delta: 0..3, bit 1 = value sums by
    decoding) on this stream; keeps and returns the fastest."""
    v = ctypes.c_int(-1)
    _check(lib().svb_autotune_decode(int(n), _ptr(inp), int(in_bytes), _ptr(out), int(start) & 0xFFFFFFFF,
                                     int(bool(delta)), _ptr(err), ctypes.addressof(v), _stream(stream)),
           "svb_autotune_decode")
    return v.value


def svb_set_decode_variant(delta, variant):
    return _check(lib().svb_set_decode_variant(int(bool(delta)), int(variant)), "svb_set_decode_variant")


def svb_append(n, inp, in_bytes, k, vals, out, out_bytes=None, stream=None):
    return _check(lib().svb_append(int(n), _ptr(inp), int(in_bytes), int(k), _ptr(vals), _ptr(out), _ptr(out_bytes),
                                   _stream(stream)), "svb_append")


def svb_delta_append(n, inp, in_bytes, k, vals, prev, out, out_bytes=None, stream=None):
    return _check(lib().svb_delta_append(int(n), _ptr(inp), int(in_bytes), int(k), _ptr(vals), int(prev) & 0xFFFFFFFF,
                                         _ptr(out), _ptr(out_bytes), _stream(stream)), "svb_delta_append")


def svb_vbyte_max_bytes(n):
    return int(lib().svb_vbyte_max_bytes(int(n)))


def svb_vbyte_encode(n, inp, out, out_bytes=None, stream=None):
    return _check(lib().svb_vbyte_encode(int(n), _ptr(inp), _ptr(out), _ptr(out_bytes), _stream(stream)),
                  "svb_vbyte_encode")


def svb_vbyte_decode(n, inp, in_bytes, out, err=None, stream=None):
    return _check(lib().svb_vbyte_decode(int(n), _ptr(inp), int(in_bytes), _ptr(out), _ptr(err), _stream(stream)),
                  "svb_vbyte_decode")


def svb_varintgb_max_bytes(n):
    return int(lib().svb_varintgb_max_bytes(int(n)))


def svb_varintgb_encode(n, inp, out, out_bytes=None, stream=None):
    return _check(lib().svb_varintgb_encode(int(n), _ptr(inp), _ptr(out), _ptr(out_bytes), _stream(stream)),
                  "svb_varintgb_encode")


def svb_varintgb_decode(n, inp, in_bytes, out, err=None, stream=None):
    return _check(lib().svb_varintgb_decode(int(n), _ptr(inp), int(in_bytes), _ptr(out), _ptr(err), _stream(stream)),
                  "svb_varintgb_decode")


def svb_seek_index_create(m, counts, in_off, in_bytes, inp, starts, total_ints, stream=None):
    """Skip index for seek/select over m resident lists; returns the handle (an int)."""
    h = ctypes.c_void_p()
    _check(lib().svb_seek_index_create(int(m), _ptr(counts), _ptr(in_off), _ptr(in_bytes), _ptr(inp), _ptr(starts),
                                       int(total_ints), ctypes.addressof(h), _stream(stream)),
           "svb_seek_index_create")
    return h.value


def svb_seek_batch(index, q, lists, targets, pos, value, err=None, stream=None):
    return _check(lib().svb_seek_batch(index, int(q), _ptr(lists), _ptr(targets), _ptr(pos), _ptr(value), _ptr(err),
                                       _stream(stream)), "svb_seek_batch")


def svb_select_batch(index, q, lists, idx, value, err=None, stream=None):
    return _check(lib().svb_select_batch(index, int(q), _ptr(lists), _ptr(idx), _ptr(value), _ptr(err),
                                         _stream(stream)), "svb_select_batch")


def svb_seek_index_destroy(index):
    return _check(lib().svb_seek_index_destroy(index), "svb_seek_index_destroy")


def svb_server_replay(server, picks, arrivals=None, outstanding=0):
    """Replays queries open loop at ``arrivals`` (seconds) or, with arrivals None, closed loop with
    ``outstanding`` queries in flight.  picks: a sequence of list-id arrays, or a pair (qoff, ids)
    with query i asking for ids[qoff[i]:qoff[i+1]].  Returns (latencies in seconds, wall seconds)."""
    import numpy as np
    if isinstance(picks, tuple) and len(picks) == 2:
        qoff = np.ascontiguousarray(picks[0], dtype=np.uint64)
        ids = np.ascontiguousarray(picks[1], dtype=np.uint32)
        nq = qoff.size - 1
    else:
        nq = len(picks)
        qoff = np.zeros(nq + 1, dtype=np.uint64)
        np.cumsum([len(p) for p in picks], out=qoff[1:])
        ids = np.ascontiguousarray(np.concatenate(picks) if nq else np.zeros(0), dtype=np.uint32)
    if ids.size == 0:
        ids = np.zeros(1, dtype=np.uint32)
    arr = None if arrivals is None else np.ascontiguousarray(arrivals, dtype=np.float64)
    if arr is not None and arr.size != nq:
        raise ValueError("one arrival time per query")
    lat = np.zeros(max(1, nq), dtype=np.float64)
    wall = ctypes.c_double(0.0)
    _check(lib().svb_server_replay(server, nq, qoff.ctypes.data, ids.ctypes.data,
                                   None if arr is None else arr.ctypes.data, int(outstanding),
                                   lat.ctypes.data, ctypes.addressof(wall)), "svb_server_replay")
    return lat[:nq], wall.value


def svb_server_replay_poisson(server, trace, qps, seconds, warmup_s=0.25, seed=0):
    """Open loop with arrivals drawn in the call: query i asks for the lists of trace entry
    i mod nbase (trace = (qoff, ids), entry e asking for ids[qoff[e]:qoff[e+1]]) and arrives at
    the i-th point of a Poisson process of rate ``qps`` for ``seconds``; queries arriving before
    ``warmup_s`` are served but not counted.  Returns a dict of the figures."""
    import numpy as np
    qoff = np.ascontiguousarray(trace[0], dtype=np.uint64)
    ids = np.ascontiguousarray(trace[1], dtype=np.uint32)
    out = np.zeros(8, dtype=np.float64)
    _check(lib().svb_server_replay_poisson(server, qoff.size - 1, qoff.ctypes.data, ids.ctypes.data, float(qps),
                                           float(seconds), float(warmup_s), int(seed), out.ctypes.data, 8),
           "svb_server_replay_poisson")
    keys = ("queries", "ints", "wall_s", "p50_s", "p99_s", "mean_s", "generated", "batches")
    return dict(zip(keys, out.tolist()))


# ------------------------------------------------------------------ conveniences

def encode(x, delta=False, start=0, stream=None):
    """Encode a device int32 tensor (uint32 bit patterns).  Returns the stream as a uint8 tensor
    of exact size (this reads the size back, so it synchronises the stream)."""
    import torch
    n = x.numel()
    out = torch.empty(max(1, svb_max_compressed_bytes(n)), dtype=torch.uint8, device=x.device)
    size = torch.zeros(1, dtype=torch.int64, device=x.device)
    if delta:
        svb_delta_encode(n, x, out, start, size, stream)
    else:
        svb_encode(n, x, out, size, stream)
    return out[: int(size.item())]


def decode(s, n, delta=False, start=0, out=None, stream=None, check=True):
    """Decode ``n`` integers from a device uint8 tensor.  Returns an int32 tensor.  With
    ``check`` the corruption flag is read back (a synchronisation) and raises SvbError."""
    import torch
    if out is None:
        out = torch.empty(max(1, n), dtype=torch.int32, device=s.device)
    err = torch.zeros(1, dtype=torch.int32, device=s.device) if check else None
    if delta:
        svb_delta_decode(n, s, s.numel(), out, start, err, stream)
    else:
        svb_decode(n, s, s.numel(), out, err, stream)
    if check and int(err.item()) != 0:
        raise SvbError(-2, "decode")
    return out[:n]
