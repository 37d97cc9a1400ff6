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
//   2. a device scan (svb_scan.hip) of the group byte counts -> each group's
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
// Fig. 4 without a shuffle table.  A wave loads the next segment (the next
// two, for plain decoding) while it decodes segment s.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

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
    const uint32_t bytes = lane_ctrl_bytes<kPerLane>(p.in, p.in_bytes, p.n, g * kGroupCtrl, lane);
    const uint32_t incl = wave_incl_scan(bytes);
    if (p.seg_loc && (lane % kLanesPerSeg) == 0) {
        const uint64_t s = g * kGroupSegs + lane / kLanesPerSeg;
        if (s * kSegInts < p.n) p.seg_loc[s] = incl - bytes;
    }
    if (lane == kWave - 1) p.gbytes[g] = incl;
}

// --------------------------------------------------------------------------
// 2. decode kernels

// Group-per-wave decode: wave w of workgroup b decodes group 4 b + w,
// segment by segment.
//   kPlain: store the integers.
//   kDelta: store their running sum (Section 2), continuing from gvpre[group].
//   kSums:  store nothing; write the group's sum of decoded values to gvsum.
//   ZC: rows of all-zero control bytes take the widening path of
//       extract_segment (the zero-control variant).
template <int MODE, bool ZC>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs p, const uint32_t *goff32) {
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
    Walker<MODE == kPlain ? 2 : 1> w;  // plain decoding waits on memory: two segments in flight
    walker_begin(p, w, s0, s_end, goff32 ? (uint64_t)goff32[g] : p.goff[g], lane);
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

hipError_t launch_decode(const DecodeArgs &a, int mode, hipStream_t s, bool zc, const uint32_t *goff32) {
    const uint32_t grid = (uint32_t)((a.groups + kWaves - 1) / kWaves);
    if (mode == kPlain) {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kPlain, true>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
        else
            hipLaunchKernelGGL((decode_kernel<kPlain, false>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
    } else if (mode == kDelta) {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kDelta, true>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
        else
            hipLaunchKernelGGL((decode_kernel<kDelta, false>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
    } else {
        if (zc)
            hipLaunchKernelGGL((decode_kernel<kSums, true>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
        else
            hipLaunchKernelGGL((decode_kernel<kSums, false>), dim3(grid), dim3(kThreads), 0, s, a, goff32);
    }
    return hipGetLastError();
}

}  // namespace svb
