"""Pure-Python Stream VByte codec, the second, independent oracle.

TEST INFRASTRUCTURE ONLY: imported by the test-suite (and the smoke check) to
cross-check the C oracle on small inputs.  It is written from the format's
definition with different primitives than the C oracle (``int.bit_length``,
``int.to_bytes`` / ``int.from_bytes`` and explicit bit strings) so that a
slip in one formulation does not repeat in the other.

Format (Stream VByte, Section 4 and Fig. 3): for N integers, ceil(N/4)
control bytes come first, then the data bytes.  Integer i takes
L_i = max(1, ceil(log_256(x_i + 1))) little-endian bytes (Section 3); its
2-bit code L_i - 1 sits in bits [2(i mod 4), 2(i mod 4) + 1] of control byte
floor(i/4).  With differential coding (Section 2), the encoder stores
d_i = x_i - x_{i-1} (mod 2^32, x_{-1} = start) and the decoder takes the
running sum.
"""

MASK32 = 0xFFFFFFFF


def byte_length(v: int) -> int:
    """Byte length of one 32-bit integer: ceil(bits / 8), at least one byte (Section 3)."""
    if not 0 <= v <= MASK32:
        raise ValueError("value outside [0, 2^32)")
    return max(1, (v.bit_length() + 7) // 8)


def deltas(values, start=0):
    """Successive differences mod 2^32 with the value before the first taken as ``start`` (Section 2)."""
    out = []
    prev = start
    for v in values:
        out.append((v - prev) & MASK32)
        prev = v
    return out


def prefix_sum(ds, start=0):
    """Running sum mod 2^32 starting from ``start`` (Section 2, "Differential Coding")."""
    out = []
    acc = start
    for d in ds:
        acc = (acc + d) & MASK32
        out.append(acc)
    return out


def encode(values, delta=False, start=0) -> bytes:
    """Stream VByte encoding of a list of 32-bit integers (Section 4)."""
    vals = deltas(values, start) if delta else list(values)
    n = len(vals)
    lengths = [byte_length(v) for v in vals]
    # control stream: build each control byte as a bit string, highest field first
    control = bytearray()
    for b in range((n + 3) // 4):
        fields = lengths[4 * b: 4 * b + 4]
        codes = [L - 1 for L in fields] + [0] * (4 - len(fields))
        bits = "".join(format(c, "02b") for c in reversed(codes))
        control.append(int(bits, 2))
    data = b"".join(v.to_bytes(L, "little") for v, L in zip(vals, lengths))
    return bytes(control) + data


def decode(stream: bytes, n: int, delta=False, start=0):
    """Decode ``n`` integers; raises ValueError if the stream is too short (Section 4)."""
    ncontrol = (n + 3) // 4
    if len(stream) < ncontrol:
        raise ValueError("stream shorter than its control bytes")
    control = stream[:ncontrol]
    pos = ncontrol
    vals = []
    for i in range(n):
        bits = format(control[i // 4], "08b")  # bit 7 first
        j = i % 4
        code = int(bits[6 - 2 * j: 8 - 2 * j], 2)
        L = code + 1
        if pos + L > len(stream):
            raise ValueError("stream shorter than the data its control bytes describe")
        vals.append(int.from_bytes(stream[pos: pos + L], "little"))
        pos += L
    return prefix_sum(vals, start) if delta else vals


def encoded_size(values, delta=False, start=0) -> int:
    """ceil(N/4) + sum of byte lengths (Section 3 and Section 4)."""
    vals = deltas(values, start) if delta else list(values)
    return (len(vals) + 3) // 4 + sum(byte_length(v) for v in vals)


def seek(stream: bytes, n: int, target: int, delta=False, start=0):
    """First position whose decoded value is >= target, with that value; (n, 0) if none
    (Section 5's seek on a compressed stream, stated on the decoded values)."""
    vals = decode(stream, n, delta, start)
    for i, v in enumerate(vals):
        if v >= target:
            return i, v
    return n, 0


def select(stream: bytes, n: int, i: int, delta=False, start=0):
    """Decoded value at position i (Section 5's select)."""
    if not 0 <= i < n:
        raise IndexError("select index past the end of the list")
    return decode(stream, n, delta, start)[i]


def append(stream: bytes, n: int, values, delta=False, prev=0) -> bytes:
    """The stream of the n integers in `stream` followed by `values`, assembled from the old
    stream's codes and bytes (they are not re-encoded) and the new integers' codes and bytes."""
    ncontrol = (n + 3) // 4
    codes = [(stream[i // 4] >> (2 * (i % 4))) & 3 for i in range(n)]
    old_data = bytes(stream[ncontrol:])
    if len(old_data) != sum(c + 1 for c in codes):
        raise ValueError("stream size does not match its control bytes")
    vals = deltas(values, prev) if delta else list(values)
    lengths = [byte_length(v) for v in vals]
    codes += [L - 1 for L in lengths]
    control = bytearray()
    for b in range((len(codes) + 3) // 4):
        fields = codes[4 * b: 4 * b + 4] + [0] * (4 - len(codes[4 * b: 4 * b + 4]))
        control.append(int("".join(format(c, "02b") for c in reversed(fields)), 2))
    return bytes(control) + old_data + b"".join(v.to_bytes(L, "little") for v, L in zip(vals, lengths))
