"""Stream VByte oracle: a scalar C codec (``svb_ref.c``) plus a pure-Python twin (``ref.py``).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1709_08990_amd``), and neither imports the
other.  The C part is compiled with gcc into ``oracle/libsvbref.so``.

Every function here follows the plain definition of the format (Section 3,
Section 4 and Fig. 3 of the paper), of differential coding (Section 2), and of
the two operations on compressed lists benchmarked in Section 5 (seek: the
first position whose value reaches a target; select: the value at a position),
and of the two comparison formats of Table 1 (VByte, Section 1; varint-GB,
Section 3 and Fig. 1).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "svb_ref.c")
_LIB_PATH = os.path.join(_HERE, "libsvbref.so")
_lib = None


def build(force=True):
    """Compile svb_ref.c with gcc -O2 into oracle/libsvbref.so."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
                           "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.svbref_length.argtypes = [ctypes.c_uint32]
        L.svbref_length.restype = ctypes.c_uint32
        L.svbref_control_bytes_of.argtypes = [ctypes.c_uint8]
        L.svbref_control_bytes_of.restype = ctypes.c_uint32
        L.svbref_length_histogram.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.svbref_length_histogram.restype = None
        L.svbref_encode.argtypes = [u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, u8p]
        L.svbref_encode.restype = ctypes.c_uint64
        L.svbref_decode.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_uint32, u32p]
        L.svbref_decode.restype = ctypes.c_int64
        L.svbref_encoded_size.argtypes = [u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32]
        L.svbref_encoded_size.restype = ctypes.c_uint64
        L.svbref_seek.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                  ctypes.c_uint32, u32p]
        L.svbref_seek.restype = ctypes.c_int64
        L.svbref_select.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                    ctypes.c_uint64, u32p]
        L.svbref_select.restype = ctypes.c_int
        L.svbref_append.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, u32p, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_uint32, u8p]
        L.svbref_append.restype = ctypes.c_int64
        L.vbref_length.argtypes = [ctypes.c_uint32]
        L.vbref_length.restype = ctypes.c_uint32
        for name in ("vbref_encode", "gbref_encode"):
            getattr(L, name).argtypes = [u32p, ctypes.c_uint64, u8p]
            getattr(L, name).restype = ctypes.c_uint64
        for name in ("vbref_decode", "gbref_decode"):
            getattr(L, name).argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, u32p]
            getattr(L, name).restype = ctypes.c_int64
        _lib = L
    return _lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def max_compressed_bytes(n):
    """ceil(n/4) control bytes plus at most four data bytes per integer."""
    return (n + 3) // 4 + 4 * n


def encode(x, delta=False, start=0):
    """Encode a uint32 array; returns the stream as a uint8 numpy array of exact size."""
    x, xp = _u32(x)
    n = x.size
    out = np.zeros(max(1, max_compressed_bytes(n)), dtype=np.uint8)
    _, op = _u8(out)
    size = lib().svbref_encode(xp, n, int(bool(delta)), int(start) & 0xFFFFFFFF, op)
    return out[:size].copy()


def decode(stream, n, delta=False, start=0):
    """Decode ``n`` integers from a uint8 stream.  Returns (values, bytes_consumed);
    raises ValueError if the stream is too short for what its control bytes describe."""
    s, sp = _u8(stream)
    out = np.zeros(max(1, n), dtype=np.uint32)
    _, op = _u32(out)
    used = lib().svbref_decode(sp, s.size, n, int(bool(delta)), int(start) & 0xFFFFFFFF, op)
    if used < 0:
        raise ValueError("corrupt or truncated Stream VByte stream")
    return out[:n].copy(), int(used)


def encoded_size(x, delta=False, start=0):
    x, xp = _u32(x)
    return int(lib().svbref_encoded_size(xp, x.size, int(bool(delta)), int(start) & 0xFFFFFFFF))


def length(v):
    return int(lib().svbref_length(int(v)))


def control_bytes_of(c):
    return int(lib().svbref_control_bytes_of(int(c)))


def length_histogram():
    """Counts of byte lengths 1..4 over every 32-bit value (a 2^32-step C loop, a few seconds)."""
    h = (ctypes.c_uint64 * 4)()
    lib().svbref_length_histogram(h)
    return [int(v) for v in h]


# --- operations on the compressed stream (Section 5: seek and select) --------

def seek(stream, n, target, delta=False, start=0):
    """(position, value) of the first integer whose value is >= target, by walking the stream in
    order; (n, 0) if there is none.  Raises ValueError on a stream too short for the walk."""
    s, sp = _u8(stream)
    v = np.zeros(1, dtype=np.uint32)
    _, vp = _u32(v)
    pos = lib().svbref_seek(sp, s.size, int(n), int(bool(delta)), int(start) & 0xFFFFFFFF,
                            int(target) & 0xFFFFFFFF, vp)
    if pos < 0:
        raise ValueError("corrupt or truncated Stream VByte stream")
    return int(pos), int(v[0])


def select(stream, n, i, delta=False, start=0):
    """Value of integer i (from 0), walking the stream up to it.  Raises IndexError if i >= n and
    ValueError on a stream too short for the walk."""
    if not 0 <= int(i) < int(n):
        raise IndexError("select index past the end of the list")
    s, sp = _u8(stream)
    v = np.zeros(1, dtype=np.uint32)
    _, vp = _u32(v)
    if lib().svbref_select(sp, s.size, int(n), int(bool(delta)), int(start) & 0xFFFFFFFF, int(i), vp) != 0:
        raise ValueError("corrupt or truncated Stream VByte stream")
    return int(v[0])


def append(stream, n, x, delta=False, prev=0):
    """The stream of the n integers held in `stream` (its exact bytes) followed by the integers x,
    built without re-encoding the old ones; the first new difference is taken from `prev`.
    Returns a uint8 array; raises ValueError if `stream` is not exactly what its control bytes
    describe."""
    s, sp = _u8(stream)
    x, xp = _u32(x)
    out = np.zeros(max(1, max_compressed_bytes(int(n) + x.size)), dtype=np.uint8)
    _, op = _u8(out)
    size = lib().svbref_append(sp, s.size, int(n), xp, x.size, int(bool(delta)), int(prev) & 0xFFFFFFFF, op)
    if size < 0:
        raise ValueError("stream size does not match its control bytes")
    return out[:size].copy()


# --- batched: Stream VByte applied to each list on its own -------------------

def encode_lists(lists, delta=False, starts=None):
    """Encode each list as its own stream; returns a list of uint8 arrays."""
    out = []
    for i, x in enumerate(lists):
        s = 0 if starts is None else int(starts[i])
        out.append(encode(x, delta=delta, start=s))
    return out


def decode_lists(streams, counts, delta=False, starts=None):
    out = []
    for i, (s, n) in enumerate(zip(streams, counts)):
        st = 0 if starts is None else int(starts[i])
        out.append(decode(s, int(n), delta=delta, start=st)[0])
    return out


# ------------------------------------------------------------------ comparison formats (Table 1; VByte Section 1, varint-GB Section 3)

def vbyte_length(v):
    """VByte bytes of v: the smallest L >= 1 with v < 2^(7L) (1..5)."""
    return int(lib().vbref_length(int(v) & 0xFFFFFFFF))


def vbyte_max_bytes(n):
    return 5 * n


def vbyte_encode(x):
    """VByte stream of a uint32 array (7 bits per byte, least significant first, top bit 1 = more
    bytes follow); uint8 numpy array of exact size."""
    x, xp = _u32(x)
    out = np.zeros(max(1, vbyte_max_bytes(x.size)), dtype=np.uint8)
    _, op = _u8(out)
    size = lib().vbref_encode(xp, x.size, op)
    return out[:size].copy()


def vbyte_decode(stream, n):
    """(values, bytes_consumed); ValueError if an integer runs past the stream or takes more than 5 bytes."""
    s, sp = _u8(stream)
    out = np.zeros(max(1, n), dtype=np.uint32)
    _, op = _u32(out)
    used = lib().vbref_decode(sp, s.size, n, op)
    if used < 0:
        raise ValueError("corrupt or truncated VByte stream")
    return out[:n].copy(), int(used)


def varintgb_max_bytes(n):
    return max_compressed_bytes(n)


def varintgb_encode(x):
    """varint-GB stream of a uint32 array (per block of four: control byte, then the data bytes)."""
    x, xp = _u32(x)
    out = np.zeros(max(1, varintgb_max_bytes(x.size)), dtype=np.uint8)
    _, op = _u8(out)
    size = lib().gbref_encode(xp, x.size, op)
    return out[:size].copy()


def varintgb_decode(stream, n):
    """(values, bytes_consumed); ValueError if a block runs past the stream."""
    s, sp = _u8(stream)
    out = np.zeros(max(1, n), dtype=np.uint32)
    _, op = _u32(out)
    used = lib().gbref_decode(sp, s.size, n, op)
    if used < 0:
        raise ValueError("corrupt or truncated varint-GB stream")
    return out[:n].copy(), int(used)
