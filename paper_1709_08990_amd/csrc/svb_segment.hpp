// One wave's unit of work for the Stream VByte kernels: a segment of 1024
// integers (256 control bytes).  Lane l owns control bytes (blocks) l, l + 64,
// l + 128 and l + 192 of the segment, so each of its four 16-byte store or
// load instructions covers 1 KiB contiguous.  Shared by the single-stream and
// the batched kernels; a stream is described by a DecodeArgs (in, in_bytes,
// n, out).
#pragma once

#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

static_assert(kWaves == 4, "a block of groups is one workgroup of four waves, one group each");

// Data-stream byte offset of group g.
__device__ __forceinline__ uint64_t group_offset(const DecodeArgs &p, uint64_t g) {
    const uint64_t b = g / 4;
    uint64_t o = p.boff32 ? (uint64_t)p.boff32[b] : p.boff[b];
    const uint32_t i = (uint32_t)(g & 3u);
    const u32x4a x = *(const u32x4a *)(p.gbytes + 4 * b);
    return o + (i > 0 ? x.x : 0u) + (i > 1 ? x.y : 0u) + (i > 2 ? x.z : 0u);
}

// Running sum (mod 2^32, from start) before group g.
__device__ __forceinline__ uint32_t group_carry(const DecodeArgs &p, uint64_t g) {
    const uint64_t b = g / 4;
    const uint32_t i = (uint32_t)(g & 3u);
    const u32x4a x = *(const u32x4a *)(p.gvsum + 4 * b);
    return p.bvpre[b] + (i > 0 ? x.x : 0u) + (i > 1 ? x.y : 0u) + (i > 2 ? x.z : 0u);
}


// Per-wave LDS staging area.  The segment's data bytes start kStagePad bytes
// in, so that the 8 aligned bytes read around an integer never fall below the
// area; 16 x 257 bytes of data (the largest 16-byte-aligned span a segment's
// 4096 data bytes can touch), 16 bytes of over-read for blocks past the end
// and the 8-byte read window fit below kStageBytes.
constexpr uint32_t kStagePad = 64;
constexpr uint32_t kStageBytes = 4224;

__device__ __forceinline__ bool segment_full(const DecodeArgs &p, uint64_t s) { return (s + 1) * kSegInts <= p.n; }

// Integers of block 64 k + lane of segment s (0..4).  The segment's remaining
// count is wave-uniform; the per-block part is 32-bit arithmetic.
__device__ __forceinline__ uint32_t block_ints(const DecodeArgs &p, uint64_t s, uint32_t k, uint32_t lane) {
    const uint64_t i0 = s * kSegInts;
    const int32_t rem = i0 >= p.n ? 0 : (int32_t)((p.n - i0) < kSegInts ? (p.n - i0) : kSegInts);
    const int32_t left = rem - (int32_t)(4u * (kWave * k + lane));
    return left <= 0 ? 0u : (left >= 4 ? 4u : (uint32_t)left);
}

// The lane's control bytes of segment s: c[k] is control byte 64 k + lane of
// the segment, with the codes of integers past n cleared.  Blocks past the end
// read as 0.
struct SegCtrl {
    uint32_t c[4];
};

__device__ __forceinline__ SegCtrl load_seg_ctrl(const DecodeArgs &p, uint64_t s, uint32_t lane) {
    const uint8_t *cp = p.in + s * kSegCtrl + lane;
    SegCtrl r;
    if (segment_full(p, s)) {
        // all 256 control bytes lie below ceil(n/4) <= in_bytes
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) r.c[k] = gptr(cp)[kWave * k];
    } else {
        // all four loads are issued before any is used (a block past the end
        // reads the last control byte instead, and is masked to no codes), so
        // a short segment costs one round trip to memory, not four
        const uint64_t nblocks = (p.n + 3) >> 2;
        const uint64_t b0 = s * kSegCtrl + lane;
        uint32_t raw[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint64_t b = b0 + kWave * k;
            raw[k] = gptr(p.in)[b < nblocks ? b : nblocks - 1];
        }
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t m = block_ints(p, s, k, lane);
            r.c[k] = m ? (raw[k] & ((1u << (2 * m)) - 1u)) : 0u;
        }
    }
    return r;
}

// Per-segment scan state: the lane's control bytes, each of its blocks' byte
// offset inside the segment's data, and the segment's byte total.
struct SegPlan {
    SegCtrl sc;
    uint32_t off[4];
    uint32_t total;
};

__device__ __forceinline__ SegPlan plan_segment(const DecodeArgs &p, uint64_t s, const SegCtrl &sc, uint32_t lane) {
    SegPlan sp;
    sp.sc = sc;
    const bool full = segment_full(p, s);
    uint32_t nb[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t m = full ? 4u : block_ints(p, s, k, lane);
        nb[k] = m + __builtin_popcount(sc.c[k]) + __builtin_popcount(sc.c[k] & 0xAAu);
    }
    // Two rows per wave scan, one in each 16-bit half: a row's bytes total
    // at most 64 x 16 = 1024, so the low half never carries into the high.
    uint32_t run = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; k += 2) {
        const uint32_t incl = wave_incl_scan(nb[k] | (nb[k + 1] << 16));
        const uint32_t tot = wave_last(incl);
        sp.off[k] = run + (incl & 0xFFFFu) - nb[k];
        run += tot & 0xFFFFu;
        sp.off[k + 1] = run + (incl >> 16) - nb[k + 1];
        run += tot >> 16;
    }
    sp.total = run;
    return sp;
}

// A segment's data span in flight: up to 5 x 64 chunks of 16 bytes,
// [abase, abase + 16 nch), where abase is the span start rounded down to 16.
// Lane c takes chunks c, c + 64, ...; each chunk that overlaps the buffer
// [in, in + in_bytes) is one aligned 16-byte load.  Such a load cannot fault:
// an aligned 16-byte chunk never straddles a page, and it holds at least one
// byte of the buffer.  Its bytes outside the buffer are staged but never
// decide a value (an integer's bytes always lie inside its span).  A chunk
// wholly outside the buffer (only on corrupt input, whose span runs past the
// end) is not loaded and stages as zeros.
struct Span {
    const uint8_t *abase;
    uint32_t nch;
    u32x4a w[5];
};

// The tests are wave-uniform where they can be: slots wholly past the span
// are skipped, and a span that lies inside the buffer (every segment's but
// possibly a stream's first and last) loads its chunks without a per-chunk
// bounds test.  The register and address work of slots and tests is a large
// share of a segment's instructions, and the value-sum pass is bound by
// instruction issue.
__device__ __forceinline__ void span_load(const DecodeArgs &p, Span &sp, uint32_t lane) {
    const uint8_t *hi = p.in + p.in_bytes;
    const bool inside = sp.abase >= p.in && sp.abase + 16ull * sp.nch <= hi;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        if (kWave * i >= sp.nch) break;
        const uint32_t c = lane + kWave * i;
        const uint8_t *cp = sp.abase + 16 * c;
        if (inside) {
            if (c < sp.nch) sp.w[i] = *gptr((const u32x4a *)cp);
        } else {
            sp.w[i] = u32x4a{0u, 0u, 0u, 0u};
            if (c < sp.nch && cp < hi && cp + 16 > p.in) sp.w[i] = *gptr((const u32x4a *)cp);
        }
    }
}

// Stages the chunks below nch (only those span_load filled).
__device__ __forceinline__ void span_to_lds(const DecodeArgs &, const Span &sp, uint8_t *stage, uint32_t lane) {
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        if (kWave * i >= sp.nch) break;
        const uint32_t c = lane + kWave * i;
        if (c < sp.nch) *(u32x4a *)(stage + kStagePad + 16 * c) = sp.w[i];
    }
}

// Walks consecutive segments [s, s_end) of one wave with a software pipeline
// D segments deep (1 or 2): when segment s is staged into LDS, the data of
// segments s + 1 .. s + D and the control bytes of s + D + 1 have been
// requested, so they are in flight while s is decoded and stored.  Depth 2
// keeps twice the bytes in flight per wave at the cost of occupancy: it pays
// where the walk waits on memory (plain decoding), not where extraction work
// dominates (the delta passes).
struct WalkSlot {
    SegPlan plan;
    uint32_t sh16;  // (data + boff) mod 16
    uint64_t boff;  // byte offset of the segment in the data stream
    Span sp;
};

template <uint32_t D>
struct Walker {
    static_assert(D == 1 || D == 2, "walker depth 1 or 2");
    const uint8_t *data;    // start of the data stream
    uint64_t data_bytes;    // bytes of the buffer from `data` on
    uint64_t s, s_end;
    WalkSlot q[D];          // q[0]: segment s, q[D - 1]: segment s + D - 1
    SegCtrl ahead;          // control bytes of segment s + D
    bool corrupt;
};

// Plans segment t from its control bytes and requests its data.
__device__ __forceinline__ void walker_issue(const DecodeArgs &p, const uint8_t *data, uint64_t t, const SegCtrl &c,
                                             uint64_t boff, uint32_t lane, WalkSlot &q) {
    q.plan = plan_segment(p, t, c, lane);
    q.boff = boff;
    const uint8_t *at = data + boff;
    q.sh16 = (uint32_t)((uintptr_t)at & 15u);
    q.sp.abase = at - q.sh16;
    q.sp.nch = (q.sh16 + q.plan.total + 15) >> 4;
    span_load(p, q.sp, lane);
}

template <uint32_t D>
__device__ __forceinline__ void walker_begin(const DecodeArgs &p, Walker<D> &w, uint64_t s0, uint64_t s_end,
                                             uint64_t boff, uint32_t lane) {
    const uint64_t nblocks = (p.n + 3) >> 2;
    w.data = p.in + nblocks;
    w.data_bytes = p.in_bytes - nblocks;
    w.s = s0;
    w.s_end = s_end;
    w.corrupt = false;
    walker_issue(p, w.data, s0, load_seg_ctrl(p, s0, lane), boff, lane, w.q[0]);
    if (D == 2 && s0 + 1 < s_end)
        walker_issue(p, w.data, s0 + 1, load_seg_ctrl(p, s0 + 1, lane), boff + w.q[0].plan.total, lane, w.q[D - 1]);
    w.ahead = SegCtrl{{0u, 0u, 0u, 0u}};
    if (s0 + D < s_end) w.ahead = load_seg_ctrl(p, s0 + D, lane);
}

// Stages segment w.s into `stage`, returns its plan and data alignment, and
// advances the walker to w.s + 1 (requesting the data of w.s + D).
template <uint32_t D>
__device__ __forceinline__ void walker_step(const DecodeArgs &p, Walker<D> &w, uint8_t *stage, uint32_t lane,
                                            SegPlan &seg, uint32_t &seg_sh16) {
    if (w.q[0].boff + w.q[0].plan.total > w.data_bytes) w.corrupt = true;
    span_to_lds(p, w.q[0].sp, stage, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    seg = w.q[0].plan;
    seg_sh16 = w.q[0].sh16;
    const uint64_t next_boff = w.q[D - 1].boff + w.q[D - 1].plan.total;
    if (D == 2) w.q[0] = w.q[D - 1];
    ++w.s;
    const uint64_t t = w.s + D - 1;  // the segment whose data is requested now
    if (t < w.s_end) {
        walker_issue(p, w.data, t, w.ahead, next_boff, lane, w.q[D - 1]);
        if (t + 1 < w.s_end) w.ahead = load_seg_ctrl(p, t + 1, lane);
    }
}

// After a staged segment has been read: the next step overwrites the staging
// area, and LDS operations of one wave complete in order.
__device__ __forceinline__ void walker_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The lane's 16 integers of a staged segment; integers past n read as 0.
// Integer j of a block ends at byte o_{j+1} - 1 of the staged span.  With
// y_j = 3 - code_j = 4 - L_j and R_j = kStagePad - 4 + o_{j+1} - 4 (j + 1),
// which falls by y_j per integer, the 4 bytes ending at the integer's last
// byte start at R_j + 4 (j + 1); they are cut out of the aligned 8 bytes
// around them, and their top L_j bytes are the integer.
//
// ZC (the zero-control variant): a row whose 64 control bytes are all zero
// holds 256 one-byte integers, so a lane's block is the 4 bytes at its offset:
// one aligned 8-byte read, one funnel shift, byte extracts (Section 4's
// decoder also special-cases blocks of single-byte integers).  Worth it only
// where such rows are common, so it is a separate kernel variant.
template <bool ZC = false>
__device__ __forceinline__ void extract_segment(const DecodeArgs &p, uint64_t s, const uint8_t *stage,
                                                const SegPlan &seg, uint32_t sh16, uint32_t lane,
                                                uint32_t (&v)[4][4]) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (ZC && __ballot(seg.sc.c[k] != 0u) == 0ull) {
            const uint32_t b = kStagePad + sh16 + seg.off[k];
            const uint32_t a = b & ~3u;
            const uint32_t w = __builtin_amdgcn_alignbyte(*(const uint32_t *)(stage + a + 4),
                                                          *(const uint32_t *)(stage + a), b & 3u);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) v[k][j] = (w >> (8 * j)) & 0xFFu;
            continue;
        }
        uint32_t R = kStagePad - 4 + sh16 + seg.off[k];
        const uint32_t nc = ~seg.sc.c[k];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t y = (nc >> (2 * j)) & 3u;
            R -= y;
            const uint32_t a = (R & ~3u) + 4 * (j + 1);
            const uint32_t lo = *(const uint32_t *)(stage + a);
            const uint32_t hi = *(const uint32_t *)(stage + a + 4);
            v[k][j] = __builtin_amdgcn_alignbyte(0u, __builtin_amdgcn_alignbyte(hi, lo, R & 3u), y);
        }
    }
    if (!segment_full(p, s)) {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t m = block_ints(p, s, k, lane);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) v[k][j] = (j < m) ? v[k][j] : 0u;
        }
    }
}

// Running sum over the segment in integer order (Section 2), continuing from
// `carry`, which it advances past the segment.
__device__ __forceinline__ void running_sum(uint32_t (&v)[4][4], uint32_t &carry) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        v[k][1] += v[k][0];
        v[k][2] += v[k][1];
        v[k][3] += v[k][2];
        const uint32_t li = wave_incl_scan(v[k][3]);
        const uint32_t add = carry + li - v[k][3];
        carry += wave_last(li);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) v[k][j] += add;
    }
}

__device__ __forceinline__ void store_segment(const DecodeArgs &p, uint64_t s, uint32_t lane, const uint32_t (&v)[4][4],
                                              uint32_t add) {
    uint32_t *o = p.out + s * kSegInts + 4ull * lane;
    if (segment_full(p, s)) {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
            __builtin_nontemporal_store(u32x4{v[k][0] + add, v[k][1] + add, v[k][2] + add, v[k][3] + add},
                                        gptr((u32x4 *)(o + 4 * kWave * k)));
    } else {
        // whole blocks of a partial segment still take one 16-byte store
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t m = block_ints(p, s, k, lane);
            uint32_t *ok = o + 4 * kWave * k;
            if (m == 4) {
                __builtin_nontemporal_store(u32x4{v[k][0] + add, v[k][1] + add, v[k][2] + add, v[k][3] + add},
                                            gptr((u32x4 *)ok));
            } else {
#pragma unroll
                for (uint32_t j = 0; j < 3; ++j)
                    if (j < m) gptr(ok)[j] = v[k][j] + add;
            }
        }
    }
}

// --------------------------------------------------------------------------
// control-byte counts

// Data bytes described by the P control bytes [first + P lane, first + P lane
// + P) of stream p (Section 4: each control byte stands for 4 integers plus
// the sum of its codes), counting only integers below n.  Reads aligned dwords
// when the whole run of the wave lies inside the stream, else byte by byte.
template <uint32_t P>
__device__ __forceinline__ uint32_t lane_ctrl_bytes(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint64_t first,
                                                    uint32_t lane) {
    static_assert(P % 4 == 0, "whole dwords per lane");
    const uint64_t nblocks = (n + 3) >> 2;
    const uint8_t *gp = in + first;
    const uint32_t sh = (uint32_t)((uintptr_t)gp & 3u);
    // every block of the wave's run is full (4 integers); the aligned dwords
    // around a lane's bytes each hold at least one of them, so none crosses a
    // page the stream does not touch (the one past the end is read only when
    // the bytes are misaligned)
    if ((first + (uint64_t)P * kWave) * 4 <= n) {
        const uint32_t *base = (const uint32_t *)(gp - sh) + (P / 4) * lane;
        const uint32_t keep = 0xFFFFFFFFu << (8u * sh);
        uint32_t codes = 0;
#pragma unroll
        for (uint32_t i = 0; i < P / 4; ++i) {
            const uint32_t x = (i == 0) ? (gptr(base)[i] & keep) : gptr(base)[i];
            codes += __builtin_popcount(x) + __builtin_popcount(x & 0xAAAAAAAAu);
        }
        const uint32_t e = sh ? (gptr(base)[P / 4] & ~keep) : 0u;
        codes += __builtin_popcount(e) + __builtin_popcount(e & 0xAAAAAAAAu);
        return 4u * P + codes;
    }
    const uint32_t last_r = (n & 3) ? (uint32_t)(n & 3) : 4u;
    const uint64_t b0 = first + (uint64_t)P * lane;
    uint32_t c[P];
#pragma unroll
    for (uint32_t i = 0; i < P; ++i) c[i] = (b0 + i < nblocks) ? (uint32_t)in[b0 + i] : 0u;
    uint32_t bytes = 0;
#pragma unroll
    for (uint32_t i = 0; i < P; ++i) {
        const uint64_t b = b0 + i;
        if (b < nblocks) bytes += control_data_bytes(c[i], (b == nblocks - 1) ? last_r : 4u);
    }
    return bytes;
}

// --------------------------------------------------------------------------
// encoding one segment

constexpr uint32_t kEncStageBytes = 4160;  // 16 x 257 bytes of span + padding

// The lane's four blocks of segment s: the values (or differences, Section 2)
// to store, each block's control byte (Section 3: L = 1 + [v >= 2^8] +
// [v >= 2^16] + [v >= 2^24], code L - 1 in bits 2j..2j+1) and data bytes.
// Integers past n contribute nothing.
struct SegValues {
    uint32_t v[4][4];
    uint32_t c[4];
    uint32_t nb[4];
};

template <bool DELTA>
__device__ __forceinline__ void load_segment_values(const EncodeStream &e, uint64_t s, uint32_t lane, SegValues &sv) {
    const bool full = (s + 1) * kSegInts <= e.n;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint64_t b = s * kSegCtrl + kWave * k + lane;
        const uint32_t *src = e.in + 4 * b;
        uint32_t x[4] = {0u, 0u, 0u, 0u};
        uint32_t r = 4, pv = 0;
        if (full) {
            const u32x4 w = *gptr((const u32x4 *)src);
            x[0] = w.x; x[1] = w.y; x[2] = w.z; x[3] = w.w;
            if (DELTA) pv = b ? gptr(src)[-1] : e.start;
        } else {
            const uint64_t i0 = 4 * b;
            r = i0 < e.n ? (uint32_t)((e.n - i0) < 4 ? (e.n - i0) : 4) : 0u;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j)
                if (j < r) x[j] = gptr(src)[j];
            if (DELTA && r) pv = b ? gptr(src)[-1] : e.start;
        }
        uint32_t ctrl = 0, bytes = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t val = DELTA ? x[j] - (j ? x[j - 1] : pv) : x[j];
            sv.v[k][j] = val;
            const uint32_t L = byte_length(val);
            ctrl |= (j < r) ? ((L - 1u) << (2 * j)) : 0u;
            bytes += (j < r) ? L : 0u;
        }
        sv.c[k] = ctrl;
        sv.nb[k] = bytes;
    }
}

// Data bytes of the lane's blocks of a loaded segment, summed over the wave.
__device__ __forceinline__ uint32_t segment_data_bytes(const SegValues &sv) {
    return wave_last(wave_incl_scan(sv.nb[0] + sv.nb[1] + sv.nb[2] + sv.nb[3]));
}

// Writes segment s of stream e: its control bytes, and its data bytes at byte
// `boff` of the data stream (which starts at out + ceil(n/4)).  The data are
// packed little-endian into the wave's LDS area laid out like the 16-byte
// aligned global span that holds them, then written with 16-byte stores
// inside the span and byte stores at its two edges (neighbouring segments own
// the rest of those 16-byte chunks).  Returns the segment's data bytes.
template <bool DELTA>
__device__ __forceinline__ uint32_t encode_segment(const EncodeStream &e, uint64_t s, uint64_t boff, uint32_t lane,
                                                   uint32_t *stage) {
    SegValues sv;
    load_segment_values<DELTA>(e, s, lane, sv);
    uint32_t off[4], run = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t incl = wave_incl_scan(sv.nb[k]);
        off[k] = run + incl - sv.nb[k];
        run += wave_last(incl);
    }
    const uint32_t total = run;
    const uint64_t nblocks = (e.n + 3) >> 2;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint64_t b = s * kSegCtrl + kWave * k + lane;
        if (b < nblocks) gptr(e.out)[b] = (uint8_t)sv.c[k];
    }
    uint8_t *dst = e.out + nblocks + boff;
    const uint32_t sh = (uint32_t)((uintptr_t)dst & 15u);
    uint8_t *abase = dst - sh;
    const uint32_t nch = (sh + total + 15) >> 4;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        const uint32_t c = lane + kWave * i;
        if (c < nch) ((u32x4a *)stage)[c] = u32x4a{0u, 0u, 0u, 0u};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool full = (s + 1) * kSegInts <= e.n;  // wave-uniform: no integer of the segment lies past n
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        uint32_t pos = sh + off[k];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t code = (sv.c[k] >> (2 * j)) & 3u;
            const uint64_t i = (s * kSegCtrl + kWave * k + lane) * 4 + j;  // integers past n are not written
            if (full || i < e.n) {
                const uint32_t val = sv.v[k][j];
                const uint32_t w = pos >> 2, sb = pos & 3u;
                atomicOr(stage + w, val << (8u * sb));
                if (sb + code + 1u > 4u) atomicOr(stage + w + 1, val >> (32u - 8u * sb));
                pos += code + 1u;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t end = sh + total;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        const uint32_t c = lane + kWave * i;
        const uint32_t lo = 16 * c;
        if (c < nch && lo >= sh && lo + 16 <= end) *gptr((u32x4a *)(abase + lo)) = ((const u32x4a *)stage)[c];
    }
    // the span's first and last chunk, when neighbouring segments own part of
    // them: one byte per lane (lanes 0-15 the first chunk, 16-31 the last),
    // only the bytes inside [sh, end)
    if (lane < 32) {
        const uint32_t c = lane < 16 ? 0u : nch - 1;
        const uint32_t q = 16 * c + (lane & 15u);
        const bool first_edge = sh != 0 || end < 16;  // chunk 0 is partial
        const bool last_edge = end != 16 * nch;       // chunk nch - 1 is partial (the same chunk when nch = 1)
        const bool mine = lane < 16 ? first_edge : (last_edge && nch > 1);
        if (nch && mine && q >= sh && q < end) gptr(abase)[q] = (uint8_t)(stage[q >> 2] >> (8u * (q & 3u)));
    }
    // the next segment clears this area: LDS operations of a wave complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return total;
}

}  // namespace svb
