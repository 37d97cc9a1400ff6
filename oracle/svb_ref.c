/*
 * Stream VByte reference codec: plain, scalar, one byte at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * What it computes (Lemire, Kurz, Rupp, "Stream VByte: Faster Byte-Oriented
 * Integer Compression", Information Processing Letters 2018):
 *
 *  - Byte length of an integer x in [0, 2^32): ceil(log_256(x + 1)) bytes,
 *    one of {1, 2, 3, 4}; stored as a 2-bit code (Section 3, the varint-GB
 *    description, and Fig. 1).  x = 0 is given length 1, the only length in
 *    {1,2,3,4} that can hold it.
 *  - Four 2-bit codes per control byte; integer 4b+j uses bits [2j, 2j+1] of
 *    control byte b, code = length - 1 (Fig. 1 and Fig. 3; the bit order is a
 *    convention the paper leaves open, taken least-significant-first here).
 *  - All ceil(N/4) control bytes come first, then the data bytes of all
 *    integers, back to back (Section 4, Fig. 3).  N is stored out of band.
 *  - Each integer's data bytes are little-endian (the decoder of Section 4
 *    shuffles bytes into little-endian 32-bit lanes).
 *  - Differential coding (Section 2, "Differential Coding", and Section 5):
 *    the encoder stores d_i = x_i - x_{i-1} with x_0 = start, the decoder
 *    rebuilds x_i = d_i + x_{i-1}.  Both run modulo 2^32, so every array of
 *    32-bit integers round-trips, sorted or not.
 *
 * Every loop below visits one integer at a time in stream order; there is no
 * lookup table, no blocking and no vector code.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* Byte length of v (Section 3): the smallest L in {1,2,3,4} with
 * v < 256^L, written as the chain of comparisons it is. */
uint32_t svbref_length(uint32_t v)
{
    if (v < (1u << 8)) return 1;
    if (v < (1u << 16)) return 2;
    if (v < (1u << 24)) return 3;
    return 4;
}

/* Number of data bytes described by one control byte whose four codes are
 * all in use (Section 4: between 4 and 16). */
uint32_t svbref_control_bytes_of(uint8_t control)
{
    uint32_t total = 0;
    for (int j = 0; j < 4; ++j) total += ((control >> (2 * j)) & 3u) + 1u;
    return total;
}

/* Histogram of svbref_length over every v in [0, 2^32) (hist[L-1] += 1).
 * Used to pin the length rule against its closed form. */
void svbref_length_histogram(uint64_t hist[4])
{
    hist[0] = hist[1] = hist[2] = hist[3] = 0;
    uint32_t v = 0;
    do {
        hist[svbref_length(v) - 1] += 1;
        v += 1;
    } while (v != 0);
}

/* Encode n integers (Section 4).  If delta != 0 the stored values are the
 * successive differences modulo 2^32 with x_0 = start (Section 2).
 * out must hold at least ceil(n/4) + 4n bytes.  Returns the number of bytes
 * written: ceil(n/4) + sum of the byte lengths. */
uint64_t svbref_encode(const uint32_t *x, uint64_t n, int delta, uint32_t start,
                       uint8_t *out)
{
    uint64_t ncontrol = (n + 3) / 4;
    memset(out, 0, (size_t)ncontrol);
    uint64_t p = ncontrol;
    uint32_t prev = start;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = delta ? (uint32_t)(x[i] - prev) : x[i];
        prev = x[i];
        uint32_t len = svbref_length(v);
        out[i / 4] |= (uint8_t)((len - 1u) << (2u * (uint32_t)(i % 4)));
        for (uint32_t k = 0; k < len; ++k) out[p + k] = (uint8_t)((v >> (8u * k)) & 0xFFu);
        p += len;
    }
    return p;
}

/* Decode n integers from in[0, in_bytes) (Section 4: one pointer walks the
 * control bytes, one walks the data bytes and advances by each integer's
 * length).  With delta != 0 the decoded values are deltas and the output is
 * their running sum modulo 2^32 starting from start (Section 2).
 * Returns the number of bytes consumed, or -1 if the stream is shorter than
 * the control stream or than the data its control bytes describe.  Codes of
 * the unused fields of a partial last control byte are never read. */
int64_t svbref_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, int delta,
                      uint32_t start, uint32_t *out)
{
    uint64_t ncontrol = (n + 3) / 4;
    if (in_bytes < ncontrol) return -1;
    uint64_t p = ncontrol;
    uint32_t prev = start;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t code = (in[i / 4] >> (2u * (uint32_t)(i % 4))) & 3u;
        uint32_t len = code + 1u;
        if (p + len > in_bytes) return -1;
        uint32_t v = 0;
        for (uint32_t k = 0; k < len; ++k) v |= (uint32_t)in[p + k] << (8u * k);
        p += len;
        if (delta) {
            prev = prev + v;
            out[i] = prev;
        } else {
            out[i] = v;
        }
    }
    return (int64_t)p;
}

/* Size of the stream svbref_encode would write, without writing it
 * (ceil(n/4) control bytes plus the byte lengths, Section 3). */
uint64_t svbref_encoded_size(const uint32_t *x, uint64_t n, int delta, uint32_t start)
{
    uint64_t total = (n + 3) / 4;
    uint32_t prev = start;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = delta ? (uint32_t)(x[i] - prev) : x[i];
        prev = x[i];
        total += svbref_length(v);
    }
    return total;
}

/* Operations on the compressed stream itself (Section 5, the seek and select
 * benchmark): both walk the stream one integer at a time, as the decoder
 * above does, and stop at the answer.  A value is the running sum when
 * delta != 0 and the stored integer otherwise.
 *
 * Seek: the position of the first integer whose value is >= target, its value
 * in *value.  Returns n (and *value = 0) if none is, or -1 if the stream is
 * shorter than its control stream or than the data read before the answer. */
int64_t svbref_seek(const uint8_t *in, uint64_t in_bytes, uint64_t n, int delta, uint32_t start,
                    uint32_t target, uint32_t *value)
{
    uint64_t ncontrol = (n + 3) / 4;
    if (in_bytes < ncontrol) return -1;
    uint64_t p = ncontrol;
    uint32_t prev = start;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t len = ((in[i / 4] >> (2u * (uint32_t)(i % 4))) & 3u) + 1u;
        if (p + len > in_bytes) return -1;
        uint32_t v = 0;
        for (uint32_t k = 0; k < len; ++k) v |= (uint32_t)in[p + k] << (8u * k);
        p += len;
        if (delta) {
            prev = prev + v;
            v = prev;
        }
        if (v >= target) {
            *value = v;
            return (int64_t)i;
        }
    }
    *value = 0;
    return (int64_t)n;
}

/* Select: the value of integer i (counted from 0) in *value.  Returns 0, or
 * -1 if i >= n or the stream is shorter than what is read up to integer i. */
int svbref_select(const uint8_t *in, uint64_t in_bytes, uint64_t n, int delta, uint32_t start,
                  uint64_t i, uint32_t *value)
{
    uint64_t ncontrol = (n + 3) / 4;
    if (i >= n || in_bytes < ncontrol) return -1;
    uint64_t p = ncontrol;
    uint32_t prev = start;
    for (uint64_t k = 0; k <= i; ++k) {
        uint32_t len = ((in[k / 4] >> (2u * (uint32_t)(k % 4))) & 3u) + 1u;
        if (p + len > in_bytes) return -1;
        uint32_t v = 0;
        for (uint32_t b = 0; b < len; ++b) v |= (uint32_t)in[p + b] << (8u * b);
        p += len;
        prev = delta ? prev + v : v;
    }
    *value = prev;
    return 0;
}

/* Append (the paper's closing remark on appending to a stream without
 * re-encoding it: the data grow at the end, the control stream grows too):
 * writes to `out` the stream of the n integers held in `in` followed by the k
 * integers of x.  The old integers' codes keep their places (their last,
 * partial control byte takes the first new codes), the new codes follow; the
 * old data bytes are copied unchanged, the new integers' bytes follow.  With
 * delta != 0 the new integers are stored as differences, the first from
 * `prev` (the old stream's last value, or its start when n = 0).  in_bytes is
 * the old stream's exact size.  Returns the new size, or -1 if the old control
 * bytes describe more data than in_bytes holds. */
int64_t svbref_append(const uint8_t *in, uint64_t in_bytes, uint64_t n, const uint32_t *x, uint64_t k, int delta,
                      uint32_t prev, uint8_t *out)
{
    uint64_t c_old = (n + 3) / 4, c_new = (n + k + 3) / 4;
    if (in_bytes < c_old) return -1;
    uint64_t d_old = 0;
    for (uint64_t i = 0; i < n; ++i) d_old += ((in[i / 4] >> (2u * (uint32_t)(i % 4))) & 3u) + 1u;
    if (c_old + d_old != in_bytes) return -1;
    for (uint64_t b = 0; b < c_new; ++b) out[b] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t code = (in[i / 4] >> (2u * (uint32_t)(i % 4))) & 3u;
        out[i / 4] = (uint8_t)(out[i / 4] | (code << (2u * (uint32_t)(i % 4))));
    }
    for (uint64_t b = 0; b < d_old; ++b) out[c_new + b] = in[c_old + b];
    uint64_t p = c_new + d_old;
    for (uint64_t j = 0; j < k; ++j) {
        uint32_t v = delta ? (uint32_t)(x[j] - prev) : x[j];
        prev = x[j];
        uint32_t len = svbref_length(v);
        uint64_t i = n + j;
        out[i / 4] = (uint8_t)(out[i / 4] | ((len - 1u) << (2u * (uint32_t)(i % 4))));
        for (uint32_t b = 0; b < len; ++b) out[p + b] = (uint8_t)(v >> (8u * b));
        p += len;
    }
    return (int64_t)p;
}

/* ------------------------------------------------------------------------
 * The two byte-oriented comparison formats of Table 1.
 *
 * VByte (Section 1): an integer is written from its least significant bits
 * up, seven bits per byte; the top bit of a byte says whether another byte of
 * the same integer follows.  The paper's examples (32 is the single byte
 * 0x20, 128 is 0x80 then 0x01) fix the flag: 1 = more bytes follow, 0 = last
 * byte.  A 32-bit integer takes 1 to 5 bytes.
 *
 * varint-GB (Section 3, Fig. 1): blocks of four integers, each a control
 * byte (the four 2-bit codes, integer j of the block in bits 2j..2j+1, code =
 * length - 1) followed by the four integers' little-endian data bytes.  A last block with
 * fewer than four integers holds only their data bytes, its unused codes 0;
 * n is kept out of band.
 * ------------------------------------------------------------------------ */

/* VByte length of v: the smallest L >= 1 with v < 2^(7L), as the chain of
 * comparisons it is. */
uint32_t vbref_length(uint32_t v)
{
    if (v < (1u << 7)) return 1;
    if (v < (1u << 14)) return 2;
    if (v < (1u << 21)) return 3;
    if (v < (1u << 28)) return 4;
    return 5;
}

/* VByte encoding of x[0..n); returns the bytes written. */
uint64_t vbref_encode(const uint32_t *x, uint64_t n, uint8_t *out)
{
    uint64_t p = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = x[i];
        while (v >= 128u) {
            out[p++] = (uint8_t)(0x80u | (v & 0x7Fu));
            v >>= 7;
        }
        out[p++] = (uint8_t)v;
    }
    return p;
}

/* Decodes n integers from in[0..in_bytes): each integer's bytes are read
 * until one with the top bit clear; value = sum of (byte & 0x7F) * 2^(7k)
 * modulo 2^32.  Returns the bytes consumed, or -1 if an integer runs past
 * in_bytes or takes more than five bytes (no 32-bit integer needs more).
 * Bytes after the n-th integer are not read. */
int64_t vbref_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t *out)
{
    uint64_t p = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t v = 0;
        uint32_t k = 0;
        for (;;) {
            if (p >= in_bytes || k == 5) return -1;
            uint8_t b = in[p++];
            v |= (uint32_t)(b & 0x7Fu) << (7u * k);
            ++k;
            if ((b & 0x80u) == 0) break;
        }
        out[i] = v;
    }
    return (int64_t)p;
}

/* varint-GB encoding of x[0..n); returns the bytes written. */
uint64_t gbref_encode(const uint32_t *x, uint64_t n, uint8_t *out)
{
    uint64_t p = 0;
    for (uint64_t b = 0; b * 4 < n; ++b) {
        uint64_t ctrl_at = p++;
        uint8_t ctrl = 0;
        for (uint32_t j = 0; j < 4 && b * 4 + j < n; ++j) {
            uint32_t v = x[b * 4 + j];
            uint32_t len = svbref_length(v);
            ctrl = (uint8_t)(ctrl | ((len - 1u) << (2u * j)));
            for (uint32_t k = 0; k < len; ++k) out[p++] = (uint8_t)(v >> (8u * k));
        }
        out[ctrl_at] = ctrl;
    }
    return p;
}

/* Decodes n integers from a varint-GB stream: a control byte, then the data
 * bytes of the block's (up to four) integers.  Returns the bytes consumed, or
 * -1 if a block runs past in_bytes.  The codes of absent integers in a last
 * partial block are ignored. */
int64_t gbref_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t *out)
{
    uint64_t p = 0;
    for (uint64_t b = 0; b * 4 < n; ++b) {
        if (p >= in_bytes) return -1;
        uint8_t ctrl = in[p++];
        for (uint32_t j = 0; j < 4 && b * 4 + j < n; ++j) {
            uint32_t len = ((ctrl >> (2u * j)) & 3u) + 1u;
            if (p + len > in_bytes) return -1;
            uint32_t v = 0;
            for (uint32_t k = 0; k < len; ++k) v |= (uint32_t)in[p + k] << (8u * k);
            p += len;
            out[b * 4 + j] = v;
        }
    }
    return (int64_t)p;
}
