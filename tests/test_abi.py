"""CPU checks of the C ABI: the library loads, exports every declared symbol, and the
host-only paths (sizes, strings, argument validation) behave without touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

import paper_1709_08990_amd as svb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(svb_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_codec():
    names = declared_functions()
    for required in ("svb_encode", "svb_decode", "svb_delta_encode", "svb_delta_decode",
                     "svb_encode_batch", "svb_decode_batch", "svb_control_bytes",
                     "svb_max_compressed_bytes", "svb_strerror", "svb_release_workspace"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(svb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_python_binding_mirrors_the_abi():
    for name in declared_functions():
        assert hasattr(svb, name), name


def test_sizes():
    assert svb.svb_control_bytes(0) == 0
    assert svb.svb_control_bytes(1) == 1
    assert svb.svb_control_bytes(4) == 1
    assert svb.svb_control_bytes(5) == 2
    assert svb.svb_max_compressed_bytes(5) == 2 + 20
    assert svb.svb_max_compressed_bytes(1 << 28) == (1 << 26) + (1 << 30)


def test_strings():
    assert svb.svb_strerror(0) == "ok"
    assert "corrupt" in svb.svb_strerror(-2)
    assert svb.svb_version().startswith("svb-gfx950")


def test_argument_errors_are_synchronous():
    """These return before any HIP call, so they run on a machine without a GPU."""
    L = svb.lib()
    assert L.svb_decode(5, None, 10, None, None, None) == -1          # null pointers
    assert L.svb_decode(9, 4096, 2, 4096, None, None) == -1           # in_bytes < ceil(n/4)
    assert L.svb_decode(8, 4096, 64, 4098, None, None) == -1          # misaligned uint32 out
    assert L.svb_decode(1 << 41, 4096, 1 << 50, 4096, None, None) == -1  # n too large
    assert L.svb_encode(4, 4098, 4096, None, None) == -1              # misaligned uint32 in
    assert L.svb_encode(4, 4096, 4096, 4100, None) == -1              # misaligned out_bytes
    assert L.svb_encode(0, None, None, None, None) == 0               # n = 0, nothing to write
    assert L.svb_decode(0, None, 0, None, None, None) == 0
    assert L.svb_copy_u32(4, 4098, 4096, None) == -1


def test_serving_replay_argument_errors():
    """A null server or a bad trace or rate is refused before any HIP call."""
    L = svb.lib()
    q = (ctypes.c_uint64 * 3)(0, 2, 3)
    ids = (ctypes.c_uint32 * 3)(1, 2, 3)
    out = (ctypes.c_double * 8)()
    assert L.svb_server_replay_poisson(None, 2, q, ids, 1e6, 1.0, 0.1, 1, out, 8) == -1
    assert L.svb_server_replay(None, 2, q, ids, None, 4, out, None) == -1
    srv = ctypes.c_void_p(4096)  # never dereferenced: the checks below fail first
    assert L.svb_server_replay_poisson(srv, 0, q, ids, 1e6, 1.0, 0.1, 1, out, 8) == -1     # empty trace
    assert L.svb_server_replay_poisson(srv, 2, q, ids, 0.0, 1.0, 0.1, 1, out, 8) == -1     # rate
    assert L.svb_server_replay_poisson(srv, 2, q, ids, 1e6, 1.0, 1.0, 1, out, 8) == -1     # warm-up >= window
    assert L.svb_server_replay_poisson(srv, 2, q, ids, 1e6, 1.0, 0.1, 1, None, 8) == -1    # no output


def test_comparison_format_sizes_and_argument_errors():
    """VByte and varint-GB entry points: worst-case sizes, and the checks that return before any
    HIP call."""
    assert svb.svb_vbyte_max_bytes(7) == 35
    assert svb.svb_varintgb_max_bytes(5) == 2 + 20
    L = svb.lib()
    for dec in (L.svb_vbyte_decode, L.svb_varintgb_decode):
        assert dec(5, None, 10, None, None, None) == -1           # null pointers
        assert dec(8, 4096, 64, 4098, None, None) == -1           # misaligned uint32 out
        assert dec(1 << 41, 4096, 1 << 50, 4096, None, None) == -1  # n too large
        assert dec(0, None, 0, None, None, None) == 0
    assert L.svb_vbyte_decode(9, 4096, 8, 4096, None, None) == -1      # fewer bytes than integers
    assert L.svb_varintgb_decode(8, 4096, 9, 4096, None, None) == -1   # below n + ceil(n/4)
    for enc in (L.svb_vbyte_encode, L.svb_varintgb_encode):
        assert enc(4, 4098, 4096, None, None) == -1               # misaligned uint32 in
        assert enc(4, 4096, 4096, 4100, None) == -1               # misaligned out_bytes
        assert enc(0, None, None, None, None) == 0


def test_decoder_variant_is_checked():
    assert svb.lib().svb_set_decode_variant(1, 4) == -1
    assert svb.lib().svb_set_decode_variant(0, 2) == -1
    assert svb.lib().svb_set_decode_variant(1, -2) == -1


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_batched_bindings_require_the_integer_bound():
    """Without total_ints the task table would be sized for lists of one segment each; the binding
    refuses the call before it reaches the library."""
    import pytest
    for f, args in ((svb.svb_decode_batch, (1, 0, 0, 0, 0, 0, 0)), (svb.svb_encode_batch, (1, 0, 0, 0, 0, 0)),
                    (svb.svb_autotune_decode_batch, (1, 0, 0, 0, 0, 0, 0)),
                    (svb.svb_autotune_encode_batch, (1, 0, 0, 0, 0, 0))):
        with pytest.raises(ValueError):
            f(*args)
