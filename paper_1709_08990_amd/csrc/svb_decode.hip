// Stream VByte decoding for gfx950: plain decode, delta decode, and the pass
// that finds where each piece of the data stream starts.
//
// The paper's decoder (Section 4, Fig. 4) walks the control stream one byte at
// a time: look up the four lengths, shuffle 16 data bytes into four integers,
// advance the data pointer by the byte count C.  Differential coding (Section
// 2) adds a running sum on top.  Both the pointer advance and the running sum
// are prefix sums, so here they become scans:
//
//   1. group_bytes_kernel: data bytes of every group (kGroupInts integers)
//      and each segment's byte offset inside its group, from the control
//      stream alone: 4 integers per control byte plus the sum of its codes;
//   2. scan_kernel: exclusive scan of the group byte counts -> each group's
//      offset in the data stream;
//   3. decode_kernel: one wave per group walks its segments (1024 integers =
//      256 control bytes each) in order.  Plain decoding stores the integers.
//      Delta decoding runs it twice: first summing each group's stored
//      differences (nothing stored), then -- after a scan of those sums
//      modulo 2^32 from `start` -- storing the running sum.
//
// Inside a segment, lane l owns control bytes l, l + 64, l + 128, l + 192, so
// each of its four store instructions writes 64 consecutive 16-byte slots.
// Four wave scans of per-block byte counts give every block's offset, the
// segment's data bytes are copied into LDS with coalesced 16-byte loads, and
// each integer is cut out of the aligned 8 bytes around the 4 bytes that end
// at its last byte with two byte-align instructions: the byte shuffle of
// Fig. 4 without a shuffle table.  A wave loads segment s + 1 while it
// decodes segment s.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

// Per-wave LDS staging area.  The segment's data bytes start kStagePad bytes
// in, so that the 8 aligned bytes read around an integer never fall below the
// area; 16 x 257 bytes of data (the largest 16-byte-aligned span a segment's
// 4096 data bytes can touch), 16 bytes of over-read for blocks past the end
// and the 8-byte read window fit below kStageBytes.
constexpr uint32_t kStagePad = 64;
constexpr uint32_t kStageBytes = 4224;

// --------------------------------------------------------------------------
// 1. data bytes per group (and, on request, each segment's byte offset inside
// its group)

__global__ __launch_bounds__(kThreads) void group_bytes_kernel(GroupBytesArgs p) {
    constexpr uint32_t kPerLane = kGroupCtrl / kWave;      // control bytes per lane
    constexpr uint32_t kLanesPerSeg = kSegCtrl / kPerLane;  // lanes covering one segment
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const uint64_t g = (uint64_t)blockIdx.x * kWaves + wave;
    if (g >= p.groups) return;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint64_t first = g * kGroupCtrl;  // the group's first control byte
    const uint8_t *gp = p.in + first;
    const uint32_t sh = (uint32_t)((uintptr_t)gp & 3u);
    uint32_t bytes = 0;
    if ((g + 1) * kGroupInts <= p.n && first >= sh && first + kGroupCtrl + 4 <= p.in_bytes) {
        // the lane's kPerLane control bytes: the aligned dwords around them,
        // minus the bytes outside
        const uint32_t *base = (const uint32_t *)(gp - sh) + (kPerLane / 4) * lane;
        const uint32_t keep = 0xFFFFFFFFu << (8u * sh);
        uint32_t codes = 0;
#pragma unroll
        for (uint32_t i = 0; i < kPerLane / 4; ++i) {
            const uint32_t x = (i == 0) ? (base[i] & keep) : base[i];
            codes += __builtin_popcount(x) + __builtin_popcount(x & 0xAAAAAAAAu);
        }
        const uint32_t e = base[kPerLane / 4] & ~keep;
        codes += __builtin_popcount(e) + __builtin_popcount(e & 0xAAAAAAAAu);
        bytes = 4u * kPerLane + codes;
    } else {
        const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;
        const uint64_t b0 = first + (uint64_t)kPerLane * lane;
        for (uint32_t i = 0; i < kPerLane; ++i) {
            const uint64_t b = b0 + i;
            if (b < nblocks) bytes += control_data_bytes(p.in[b], (b == nblocks - 1) ? last_r : 4u);
        }
    }
    const uint32_t incl = wave_incl_scan(bytes);
    if (p.seg_loc && (lane % kLanesPerSeg) == 0) {
        const uint64_t s = g * kGroupSegs + lane / kLanesPerSeg;
        if (s * kSegInts < p.n) p.seg_loc[s] = incl - bytes;
    }
    if (lane == kWave - 1) p.gbytes[g] = incl;
}

// --------------------------------------------------------------------------
// 2. exclusive scan by one workgroup of 1024 threads, 16 values per thread per
// step.  WIDE: 64-bit sums (byte offsets); otherwise modulo 2^32 from `start`.

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

template <bool WIDE>
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *in, void *out, uint64_t m, uint32_t start) {
    constexpr uint32_t kT = 1024, kPer = 16, kW = kT / kWave;
    __shared__ uint32_t s_wtot[kW];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    uint64_t carry = WIDE ? 0u : start;
    for (uint64_t base = 0; base < m; base += (uint64_t)kT * kPer) {
        const uint64_t i0 = base + (uint64_t)tid * kPer;
        const bool whole = i0 + kPer <= m;
        uint32_t x[kPer];
        if (whole) {
#pragma unroll
            for (uint32_t j = 0; j < kPer; j += 4) {
                const u32x4 w = *(const u32x4 *)(in + i0 + j);
                x[j] = w.x; x[j + 1] = w.y; x[j + 2] = w.z; x[j + 3] = w.w;
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kPer; ++j) x[j] = (i0 + j < m) ? in[i0 + j] : 0u;
        }
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) sum += x[j];
        const uint32_t incl = wave_incl_scan(sum);
        if (lane == kWave - 1) s_wtot[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            const uint32_t t = lane < kW ? s_wtot[lane] : 0u;
            const uint32_t ti = wave_incl_scan(t);
            if (lane < kW) s_wtot[lane] = ti - t;
            if (lane == kWave - 1) s_total = ti;
        }
        __syncthreads();
        uint32_t y[kPer];
        uint32_t run = s_wtot[wave] + incl - sum;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            y[j] = run;
            run += x[j];
        }
        if (whole) {
            if (WIDE) {
                u64x2 *o = (u64x2 *)((uint64_t *)out + i0);
#pragma unroll
                for (uint32_t j = 0; j < kPer; j += 2) o[j / 2] = u64x2{carry + y[j], carry + y[j + 1]};
            } else {
                uint32_t *o = (uint32_t *)out + i0;
                const uint32_t c32 = (uint32_t)carry;
#pragma unroll
                for (uint32_t j = 0; j < kPer; j += 4)
                    *(u32x4 *)(o + j) = u32x4{c32 + y[j], c32 + y[j + 1], c32 + y[j + 2], c32 + y[j + 3]};
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kPer; ++j) {
                if (i0 + j < m) {
                    if (WIDE)
                        ((uint64_t *)out)[i0 + j] = carry + y[j];
                    else
                        ((uint32_t *)out)[i0 + j] = (uint32_t)carry + y[j];
                }
            }
        }
        carry += s_total;
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// 3. segments

__device__ __forceinline__ bool segment_full(const DecodeArgs &p, uint64_t s) { return (s + 1) * kSegInts <= p.n; }

// Integers of block 64 k + lane of segment s (0..4).
__device__ __forceinline__ uint32_t block_ints(const DecodeArgs &p, uint64_t s, uint32_t k, uint32_t lane) {
    const uint64_t i0 = s * kSegInts + 4ull * (kWave * k + lane);
    return i0 < p.n ? (uint32_t)((p.n - i0) < 4 ? (p.n - i0) : 4) : 0u;
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
        for (uint32_t k = 0; k < 4; ++k) r.c[k] = cp[kWave * k];
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t m = block_ints(p, s, k, lane);
            r.c[k] = m ? (cp[kWave * k] & ((1u << (2 * m)) - 1u)) : 0u;
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
    uint32_t run = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t m = full ? 4u : block_ints(p, s, k, lane);
        const uint32_t nb = m + __builtin_popcount(sc.c[k]) + __builtin_popcount(sc.c[k] & 0xAAu);
        const uint32_t incl = wave_incl_scan(nb);
        sp.off[k] = run + incl - nb;
        run += wave_last(incl);
    }
    sp.total = run;
    return sp;
}

// A segment's data span in flight: up to 5 x 64 chunks of 16 bytes,
// [abase, abase + 16 nch), where abase is the span start rounded down to 16.
// Inside the buffer every chunk is one aligned 16-byte load into registers
// (lane c takes chunks c, c + 64, ...); at the edges of the buffer the chunks
// are assembled byte by byte when they are staged, bytes outside
// [in, in + in_bytes) reading as 0.
struct Span {
    const uint8_t *abase;
    uint32_t nch;
    bool inside;
    u32x4a w[5];
};

__device__ __forceinline__ void span_load(const DecodeArgs &p, Span &sp, uint32_t lane) {
    sp.inside = sp.abase >= p.in && sp.abase + 16ull * sp.nch <= p.in + p.in_bytes;
    if (sp.inside) {
#pragma unroll
        for (uint32_t i = 0; i < 5; ++i) {
            const uint32_t c = lane + kWave * i;
            if (c < sp.nch) sp.w[i] = *(const u32x4a *)(sp.abase + 16 * c);
        }
    }
}

__device__ __forceinline__ void span_to_lds(const DecodeArgs &p, const Span &sp, uint8_t *stage, uint32_t lane) {
    if (sp.inside) {
#pragma unroll
        for (uint32_t i = 0; i < 5; ++i) {
            const uint32_t c = lane + kWave * i;
            if (c < sp.nch) *(u32x4a *)(stage + kStagePad + 16 * c) = sp.w[i];
        }
    } else {
        for (uint32_t c = lane; c < sp.nch; c += kWave) {
            uint32_t d[4] = {0u, 0u, 0u, 0u};
            for (uint32_t b = 0; b < 16; ++b) {
                const uint8_t *a = sp.abase + 16 * c + b;
                if (a >= p.in && a < p.in + p.in_bytes) d[b >> 2] |= (uint32_t)*a << (8 * (b & 3));
            }
            *(u32x4a *)(stage + kStagePad + 16 * c) = u32x4a{d[0], d[1], d[2], d[3]};
        }
    }
}

// Walks consecutive segments [s, s_end) of one wave with a one-segment
// software pipeline: each step stages segment s into LDS and, before
// returning, requests segment s + 1's data and segment s + 2's control bytes,
// so that they are in flight while s is decoded and stored.
struct Walker {
    const uint8_t *data;    // start of the data stream
    uint64_t data_bytes;    // bytes of the buffer from `data` on
    uint64_t s, s_end;
    uint64_t boff;          // byte offset of segment s in the data stream
    SegPlan cur;            // plan of segment s
    uint32_t sh16;          // (data + boff) mod 16
    Span sp;                // segment s's data in flight
    SegCtrl ahead;          // control bytes of segment s + 1
    bool corrupt;
};

__device__ __forceinline__ void walker_begin(const DecodeArgs &p, Walker &w, uint64_t s0, uint64_t s_end,
                                             uint64_t boff, uint32_t lane) {
    const uint64_t nblocks = (p.n + 3) >> 2;
    w.data = p.in + nblocks;
    w.data_bytes = p.in_bytes - nblocks;
    w.s = s0;
    w.s_end = s_end;
    w.boff = boff;
    w.corrupt = false;
    w.cur = plan_segment(p, s0, load_seg_ctrl(p, s0, lane), lane);
    w.sh16 = (uint32_t)((uintptr_t)(w.data + boff) & 15u);
    w.sp.abase = w.data + boff - w.sh16;
    w.sp.nch = (w.sh16 + w.cur.total + 15) >> 4;
    span_load(p, w.sp, lane);
    w.ahead = SegCtrl{{0u, 0u, 0u, 0u}};
    if (s0 + 1 < s_end) w.ahead = load_seg_ctrl(p, s0 + 1, lane);
}

// Stages segment w.s into `stage`, returns its plan and data alignment, and
// advances the walker to w.s + 1 (requesting its data).
__device__ __forceinline__ void walker_step(const DecodeArgs &p, Walker &w, uint8_t *stage, uint32_t lane,
                                            SegPlan &seg, uint32_t &seg_sh16) {
    if (w.boff + w.cur.total > w.data_bytes) w.corrupt = true;
    span_to_lds(p, w.sp, stage, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    seg = w.cur;
    seg_sh16 = w.sh16;
    w.boff += seg.total;
    ++w.s;
    if (w.s < w.s_end) {
        w.cur = plan_segment(p, w.s, w.ahead, lane);
        const uint8_t *q = w.data + w.boff;
        w.sh16 = (uint32_t)((uintptr_t)q & 15u);
        w.sp.abase = q - w.sh16;
        w.sp.nch = (w.sh16 + w.cur.total + 15) >> 4;
        span_load(p, w.sp, lane);
        if (w.s + 1 < w.s_end) w.ahead = load_seg_ctrl(p, w.s + 1, lane);
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
__device__ __forceinline__ void extract_segment(const DecodeArgs &p, uint64_t s, const uint8_t *stage,
                                                const SegPlan &seg, uint32_t sh16, uint32_t lane,
                                                uint32_t (&v)[4][4]) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
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
                                        (u32x4 *)(o + 4 * kWave * k));
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t m = block_ints(p, s, k, lane);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j)
                if (j < m) o[4 * kWave * k + j] = v[k][j] + add;
        }
    }
}

// --------------------------------------------------------------------------
// 4. kernels

// Group-per-wave decode: wave w of workgroup b decodes group 4 b + w,
// segment by segment.
//   kPlain: store the integers.
//   kDelta: store their running sum (Section 2), continuing from gvpre[group].
//   kSums:  store nothing; write the group's sum of decoded values to gvsum.
template <int MODE>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const uint64_t g = (uint64_t)blockIdx.x * kWaves + wave;
    if (g >= p.groups) return;
    uint8_t *stage = s_stage + wave * kStageBytes;
    const uint64_t segs = (p.n + kSegInts - 1) / kSegInts;
    const uint64_t s0 = g * kGroupSegs;
    const uint64_t s_end = s0 + kGroupSegs < segs ? s0 + kGroupSegs : segs;
    uint32_t carry = (MODE == kDelta) ? p.gvpre[g] : 0u;
    Walker w;
    walker_begin(p, w, s0, s_end, p.goff[g], lane);
    for (uint64_t s = s0; s < s_end; ++s) {
        SegPlan seg;
        uint32_t sh16;
        walker_step(p, w, stage, lane, seg, sh16);
        uint32_t v[4][4];
        extract_segment(p, s, stage, seg, sh16, lane, v);
        walker_release();
        if (MODE == kSums) {
            uint32_t t = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) t += v[k][0] + v[k][1] + v[k][2] + v[k][3];
            carry += wave_last(wave_incl_scan(t));
        } else {
            if (MODE == kDelta) running_sum(v, carry);
            store_segment(p, s, lane, v, 0u);
        }
    }
    if (w.corrupt && p.err && lane == 0) *p.err = SVB_DECODE_CORRUPT;
    if (MODE == kSums && lane == 0) p.gvsum[g] = carry;
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_group_bytes(const GroupBytesArgs &a, hipStream_t s) {
    const uint64_t grid = (a.groups + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(group_bytes_kernel, dim3((uint32_t)grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *in, void *out, uint64_t m, bool wide, uint32_t start, hipStream_t s) {
    if (wide)
        hipLaunchKernelGGL((scan_kernel<true>), dim3(1), dim3(1024), 0, s, in, out, m, start);
    else
        hipLaunchKernelGGL((scan_kernel<false>), dim3(1), dim3(1024), 0, s, in, out, m, start);
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs &a, int mode, hipStream_t s) {
    const uint32_t grid = (uint32_t)((a.groups + kWaves - 1) / kWaves);
    if (mode == kPlain)
        hipLaunchKernelGGL((decode_kernel<kPlain>), dim3(grid), dim3(kThreads), 0, s, a);
    else if (mode == kDelta)
        hipLaunchKernelGGL((decode_kernel<kDelta>), dim3(grid), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((decode_kernel<kSums>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svb
