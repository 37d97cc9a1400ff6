// Stream VByte encoding for gfx950 (plain and delta), plus a copy and a fill
// kernel used for measurement.
//
// The paper's encoder (Section 3) writes each integer's control bits and then
// appends its bytes after the previous integer's.  Where the bytes go is a
// prefix sum of the lengths, so here encoding takes two passes over the
// values, with no workgroup ever waiting for another:
//   1. encode_sizes_kernel: one wave per segment (1024 integers) computes the
//      lengths (of the differences, Section 2, for delta coding) and writes
//      the segment's data bytes;
//   2. an exclusive scan of those counts (svb_scan.hip) -> each segment's byte
//      offset in the data stream;
//   3. encode_pack_kernel: one wave per segment computes the lengths again,
//      writes the 256 control bytes, packs the data bytes into LDS and writes
//      them out (encode_segment); the wave of the last segment writes the
//      stream size.
// A single pass with a decoupled look-back between tiles was built and
// measured first: it was 1.6x slower on MI355X, where each look-back poll is
// a device-coherent read that bypasses the per-XCD L2.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

// --------------------------------------------------------------------------
// two-pass encoding: data bytes of every segment, an exclusive scan of them
// (svb_scan.hip), then one wave per segment packs it at its offset.  The
// values are read twice; no workgroup waits for another.

template <bool DELTA>
__global__ __launch_bounds__(kThreads) void encode_sizes_kernel(EncodeStream e, uint32_t *seg_bytes, uint64_t segs) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t s = (uint64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (s >= segs) return;
    SegValues sv;
    load_segment_values<DELTA>(e, s, lane, sv);
    const uint32_t t = segment_data_bytes(sv);
    if (lane == 0) seg_bytes[s] = t;
}

// The pack pass takes the segments last to first: the size pass has just read
// the values front to back, so the end of them is still in the memory-side
// cache (measured at 2^28 document ids: 0.441 ms per delta encode against
// 0.446 front to back).
#ifndef SVB_PACK_REVERSE
#define SVB_PACK_REVERSE 1
#endif
template <bool DELTA>
__global__ __launch_bounds__(kThreads) void encode_pack_kernel(EncodeStream e, const uint64_t *seg_off,
                                                               const uint32_t *seg_off32, uint64_t segs,
                                                               uint64_t *out_bytes) {
    __shared__ __attribute__((aligned(16))) uint32_t s_stage[kWaves * (kEncStageBytes / 4)];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t sl = (uint64_t)blockIdx.x * kWaves + wave;
    if (sl >= segs) return;
    const uint64_t s = SVB_PACK_REVERSE ? segs - 1 - sl : sl;
    const uint64_t off = seg_off32 ? (uint64_t)seg_off32[s] : seg_off[s];
    const uint32_t t = encode_segment<DELTA>(e, s, off, lane, s_stage + wave * (kEncStageBytes / 4));
    if (s == segs - 1 && lane == 0 && out_bytes) *out_bytes = (e.n + 3) / 4 + off + t;
}

__global__ __launch_bounds__(kThreads) void copy_kernel(const uint32_t *in, uint32_t *out, uint64_t n) {
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load((const u32x4 *)(in + 4 * i)), (u32x4 *)(out + 4 * i));
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) out[4 * n4 + threadIdx.x] = in[4 * n4 + threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void fill_kernel(uint32_t *out, uint64_t n, uint32_t value) {
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
        *(u32x4 *)(out + 4 * i) = u32x4{value, value, value, value};
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) out[4 * n4 + threadIdx.x] = value;
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_encode_sizes(const EncodeStream &e, bool delta, uint32_t *seg_bytes, uint64_t segs, hipStream_t s) {
    const uint32_t grid = (uint32_t)((segs + kWaves - 1) / kWaves);
    if (delta)
        hipLaunchKernelGGL((encode_sizes_kernel<true>), dim3(grid), dim3(kThreads), 0, s, e, seg_bytes, segs);
    else
        hipLaunchKernelGGL((encode_sizes_kernel<false>), dim3(grid), dim3(kThreads), 0, s, e, seg_bytes, segs);
    return hipGetLastError();
}

hipError_t launch_encode_pack(const EncodeStream &e, bool delta, const uint64_t *seg_off, uint64_t segs,
                              uint64_t *out_bytes, hipStream_t s, const uint32_t *seg_off32) {
    const uint32_t grid = (uint32_t)((segs + kWaves - 1) / kWaves);
    if (delta)
        hipLaunchKernelGGL((encode_pack_kernel<true>), dim3(grid), dim3(kThreads), 0, s, e, seg_off, seg_off32, segs,
                           out_bytes);
    else
        hipLaunchKernelGGL((encode_pack_kernel<false>), dim3(grid), dim3(kThreads), 0, s, e, seg_off, seg_off32, segs,
                           out_bytes);
    return hipGetLastError();
}

hipError_t launch_copy(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s) {
    const uint64_t want = (n / 4 + kThreads - 1) / kThreads;
    const uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > 16384 ? 16384 : want));
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kThreads), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t *out, uint64_t n, uint32_t value, hipStream_t s) {
    const uint64_t want = (n / 4 + kThreads - 1) / kThreads;
    const uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(kThreads), 0, s, out, n, value);
    return hipGetLastError();
}

}  // namespace svb
