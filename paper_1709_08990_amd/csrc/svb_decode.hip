// Stream VByte decoding for gfx950: plain decode, delta decode, and the pass
// that finds where each piece of the data stream starts.
//
// The paper's decoder (Section 4, Fig. 4) walks the control stream one byte at
// a time: look up the four lengths, shuffle 16 data bytes into four integers,
// advance the data pointer by the byte count C.  Differential coding (Section
// 2) adds a running sum on top.  Both the pointer advance and the running sum
// are prefix sums, so here they become scans:
//
//   1. group_bytes_kernel: data bytes of every group (kGroupInts integers),
//      from the control stream alone: 4 integers per control byte plus the
//      sum of its codes, and of every block of four groups (one per wave);
//   2. a device scan (svb_scan.hip) of the block byte counts -> each block's
//      offset in the data stream (a group's is its block's plus the groups
//      before it in the block);
//   3. decode_kernel: one wave per group walks its segments (1024 integers =
//      256 control bytes each) in order.  Plain decoding stores the integers.
//      Delta decoding first needs each group's sum of stored differences
//      (svb_delta.hip takes it without decoding; the kSums mode below takes
//      it by decoding, for dense streams), then -- after a scan of those sums
//      modulo 2^32 from `start` -- stores the running sum.
//
// Inside a segment, lane l owns control bytes l, l + 64, l + 128, l + 192, so
// each of its four store instructions writes 64 consecutive 16-byte slots.
// Four wave scans of per-block byte counts give every block's offset, the
// segment's data bytes are copied into LDS with coalesced 16-byte loads, and
// each integer is cut out of the aligned 8 bytes around the 4 bytes that end
// at its last byte with two byte-align instructions: the byte shuffle of
// Fig. 4 without a shuffle table.  A wave loads the next segment (the next
// two, for plain decoding) while it decodes segment s.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

// --------------------------------------------------------------------------
// 1. data bytes per group

// One block of four groups per wave: lane l reads control bytes 16 l ..
// 16 l + 15 of each of the four groups (four 16-byte loads in flight, and one
// more dword each when the stream is not 4-byte aligned).  Each control byte
// stands for 4 integers plus the sum of its codes (Section 4).  A group's
// data bytes are at most 16,384, so two groups share one wave sum; lane 0
// writes the four group totals and the block's.  (Measured at 2^28 against
// one group per wave: delta decode 0.3059 -> 0.3045 ms per call, plain
// decode 0.3077 -> 0.3065.)
static_assert(kGroupCtrl == 16 * kWave, "16 control bytes per lane and group");

__global__ __launch_bounds__(kThreads) void group_bytes_kernel(GroupBytesArgs p) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const uint64_t blk = (uint64_t)blockIdx.x * kWaves + wave;
    const uint64_t blocks = (p.groups + kWaves - 1) / kWaves;
    if (blk >= blocks) return;
    const uint64_t full = p.n / kGroupInts;  // groups whose 1024 control bytes all lie below ceil(n/4)
    const uint64_t g0 = blk * kWaves;
    uint32_t bytes[kWaves];
    if (g0 + kWaves <= full) {
        const uint8_t *cp = p.in + g0 * kGroupCtrl + 16ull * lane;
        const uint32_t sh = (uint32_t)((uintptr_t)cp & 3u);
        const uint32_t *ap = (const uint32_t *)(cp - sh);
        u32x4 w[kWaves];
        uint32_t w4[kWaves];
#pragma unroll
        for (uint32_t j = 0; j < kWaves; ++j) w[j] = *gptr((const u32x4 *)(ap + j * (kGroupCtrl / 4)));
#pragma unroll
        for (uint32_t j = 0; j < kWaves; ++j) w4[j] = sh ? gptr(ap + j * (kGroupCtrl / 4))[4] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < kWaves; ++j) {
            const uint32_t x[4] = {__builtin_amdgcn_alignbyte(w[j].y, w[j].x, sh),
                                   __builtin_amdgcn_alignbyte(w[j].z, w[j].y, sh),
                                   __builtin_amdgcn_alignbyte(w[j].w, w[j].z, sh),
                                   __builtin_amdgcn_alignbyte(w4[j], w[j].w, sh)};
            uint32_t codes = 0;
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) codes += __builtin_popcount(x[i]) + __builtin_popcount(x[i] & 0xAAAAAAAAu);
            bytes[j] = 64u + codes;
        }
    } else {
        // the block of the stream's last, partial group: byte loads, integers
        // past n not counted, groups past the last 0
        const uint64_t nblocks = (p.n + 3) >> 2;
        const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;
#pragma unroll
        for (uint32_t j = 0; j < kWaves; ++j) {
            bytes[j] = 0;
            const uint64_t g = g0 + j;
            if (g >= p.groups) continue;
            for (uint32_t i = 0; i < 16; ++i) {
                const uint64_t b = g * kGroupCtrl + 16ull * lane + i;
                if (b < nblocks) bytes[j] += control_data_bytes(gptr(p.in)[b], b == nblocks - 1 ? last_r : 4u);
            }
        }
    }
    const uint32_t s01 = wave_last(wave_incl_scan(bytes[0] | (bytes[1] << 16)));
    const uint32_t s23 = wave_last(wave_incl_scan(bytes[2] | (bytes[3] << 16)));
    if (lane == 0) {
        const u32x4 t = u32x4{s01 & 0xFFFFu, s01 >> 16, s23 & 0xFFFFu, s23 >> 16};
        *(u32x4 *)(p.gbytes + g0) = t;  // 0 past the last group (the array holds whole blocks)
        p.bbytes[blk] = t.x + t.y + t.z + t.w;
    }
}

// --------------------------------------------------------------------------
// 2. decode kernels

// Group-per-wave decode: wave w of workgroup b decodes group 4 b + w,
// segment by segment.
//   kPlain: store the integers.
//   kDelta: store their running sum (Section 2), continuing from the group's carry.
//   kSums:  store nothing; write the group's sum of decoded values to gvsum,
//           and the block's to bvsum.
//   ZC: rows of all-zero control bytes take the widening path of
//       extract_segment (the zero-control variant).
// Delta decoding takes the groups last to first: the value-sum pass has just
// read the stream front to back, so the end of it is still in the
// memory-side cache when the decode starts (measured at 2^28 document ids:
// 0.385 ms per call against 0.400 front to back; no change at 2^26, whose
// whole stream stays cached either way).
// Segments a wave keeps in flight (walker depth).  Measured at 2^28: plain
// decode of the stress integers 0.310 ms at depth 2 (3 waves per SIMD) and
// 0.311 at depth 1 (5 waves per SIMD); delta decode of the document ids
// 0.315 ms at depth 1, 0.328 at depth 2.
#ifndef SVB_PLAIN_DEPTH
#define SVB_PLAIN_DEPTH 2
#endif
#ifndef SVB_DELTA_DEPTH
#define SVB_DELTA_DEPTH 1
#endif
#ifndef SVB_DECODE_REVERSE
#define SVB_DECODE_REVERSE 1
#endif
template <int MODE, bool ZC>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    __shared__ uint32_t s_part[kWaves];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const uint64_t gl = (uint64_t)blockIdx.x * kWaves + wave;
    if (MODE != kSums && gl >= p.groups) return;  // (the sums mode's waves all reach the block total)
    const uint64_t g = (MODE == kDelta && SVB_DECODE_REVERSE) ? p.groups - 1 - gl : gl;
    uint8_t *stage = s_stage + wave * kStageBytes;
    const uint64_t segs = (p.n + kSegInts - 1) / kSegInts;
    const uint64_t s0 = g * kGroupSegs;
    const uint64_t s_end = g >= p.groups ? s0 : (s0 + kGroupSegs < segs ? s0 + kGroupSegs : segs);
    uint32_t carry = (MODE == kDelta) ? group_carry(p, g) : 0u;
    Walker<MODE == kPlain ? SVB_PLAIN_DEPTH : SVB_DELTA_DEPTH> w;
    if (s0 < s_end) walker_begin(p, w, s0, s_end, group_offset(p, g), lane);
    for (uint64_t s = s0; s < s_end; ++s) {
        SegPlan seg;
        uint32_t sh16;
        walker_step(p, w, stage, lane, seg, sh16);
        uint32_t v[4][4];
        extract_segment<ZC>(p, s, stage, seg, sh16, lane, v);
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
    if (s0 < s_end && w.corrupt && p.err && lane == 0) *p.err = SVB_DECODE_CORRUPT;
    if (MODE == kSums) {
        if (lane == 0) {
            p.gvsum[g] = carry;  // 0 past the last group (the array holds whole blocks)
            s_part[wave] = carry;
        }
        __syncthreads();
        if (threadIdx.x == 0) p.bvsum[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    }
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_group_bytes(const GroupBytesArgs &a, hipStream_t s) {
    const uint64_t blocks = (a.groups + kWaves - 1) / kWaves;  // one per wave
    hipLaunchKernelGGL(group_bytes_kernel, dim3((uint32_t)((blocks + kWaves - 1) / kWaves)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs &a, int mode, hipStream_t s, bool zc) {
    const uint32_t grid = (uint32_t)((a.groups + kWaves - 1) / kWaves);
    if (mode == kPlain) {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kPlain, true>), dim3(grid), dim3(kThreads), 0, s, a);
        else
            hipLaunchKernelGGL((decode_kernel<kPlain, false>), dim3(grid), dim3(kThreads), 0, s, a);
    } else if (mode == kDelta) {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kDelta, true>), dim3(grid), dim3(kThreads), 0, s, a);
        else
            hipLaunchKernelGGL((decode_kernel<kDelta, false>), dim3(grid), dim3(kThreads), 0, s, a);
    } else {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kSums, true>), dim3(grid), dim3(kThreads), 0, s, a);
        else
            hipLaunchKernelGGL((decode_kernel<kSums, false>), dim3(grid), dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace svb
