// Batched Stream VByte: m independent lists (the paper's posting lists,
// Section 5: many lists of very uneven length) decoded or encoded by one
// sequence of launches whose work list is built on the device.
//
// Every list is cut into items of G segments (G * 1024 integers); an item is
// one wave's work.  The host never reads the list arrays, so the item list is
// built on the device:
//   1. batch_count_kernel:  items per list (0 for an empty or invalid list);
//   2. scan -> each list's first item, and the item total;
//   3. batch_map_kernel:    item -> list;
//   4. batch_item_bytes_kernel: data bytes of every item that is not the last
//      of its list (control bytes only when decoding; the values' byte lengths
//      when encoding), then a scan -> each item's byte offset in its list's
//      data stream (global scan minus the value at the list's first item);
//   5. delta decoding only: batch_item_sums_kernel sums the stored differences
//      of every item that is not the last of its list, then a scan -> each
//      item's carry;
//   6. batch_decode_kernel / batch_encode_kernel: one wave per item.
// A list that fits in one item skips steps 4-5 entirely (offset 0, carry =
// start), so short lists cost one pass over their bytes.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

namespace {

constexpr uint32_t kEncStageWords = kEncStageBytes / 4;

__device__ __forceinline__ uint32_t items_of(uint64_t count, uint32_t G) {
    const uint64_t per = (uint64_t)G * kSegInts;
    return (uint32_t)((count + per - 1) / per);
}

template <uint32_t G>
__global__ __launch_bounds__(kThreads) void batch_count_kernel(BatchArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.m) return;
    const uint64_t c = a.counts[i];
    uint32_t items = 0;
    if (c > SVB_MAX_N) {
        if (a.err) *a.err = SVB_DECODE_CORRUPT;
        if (a.out_bytes) a.out_bytes[i] = ~0ull;
    } else if (a.in_bytes && a.in_bytes[i] < (c + 3) / 4) {
        if (a.err) *a.err = SVB_DECODE_CORRUPT;  // control stream longer than the list's bytes
    } else {
        items = items_of(c, G);
        if (c == 0 && a.out_bytes) a.out_bytes[i] = 0;
    }
    a.litems[i] = items;
}

__global__ __launch_bounds__(kThreads) void batch_map_kernel(BatchArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.m) return;
    if (a.lbase[a.m] > a.t_cap) {
        // the caller's integer bound was too small: nothing is done
        if (i == 0 && a.err) *a.err = SVB_BATCH_OVERFLOW;
        if (a.out_bytes) a.out_bytes[i] = ~0ull;
        return;
    }
    const uint32_t b = a.lbase[i], e = b + a.litems[i];
    for (uint32_t t = b; t < e; ++t) a.item_list[t] = (uint32_t)i;
}

// The item a wave works on, and its place in its list.
struct ItemRef {
    bool valid;
    uint32_t list;
    uint32_t first_item;  // the list's first item
    uint32_t piece;       // item index inside the list
    bool last;
};

__device__ __forceinline__ ItemRef item_ref(const BatchArgs &a, uint64_t t) {
    ItemRef r = {false, 0u, 0u, 0u, false};
    const uint32_t total = a.lbase[a.m];
    if (total > a.t_cap || t >= total) return r;
    r.valid = true;
    r.list = a.item_list[t];
    r.first_item = a.lbase[r.list];
    r.piece = (uint32_t)t - r.first_item;
    r.last = r.piece + 1 == a.litems[r.list];
    return r;
}

__device__ __forceinline__ DecodeArgs list_stream(const BatchArgs &a, uint32_t i) {
    DecodeArgs p = {};
    p.in = a.in8 + a.in_off[i];
    p.in_bytes = a.in_bytes[i];
    p.n = a.counts[i];
    p.out = a.out32 + a.out_off[i];
    p.err = a.err;
    return p;
}

__device__ __forceinline__ EncodeStream list_values(const BatchArgs &a, uint32_t i) {
    EncodeStream e;
    e.in = a.in32 + a.in_off[i];
    e.n = a.counts[i];
    e.out = a.out8 + a.out_off[i];
    e.start = a.starts ? a.starts[i] : 0u;
    return e;
}

__device__ __forceinline__ uint64_t wave_item(uint32_t wave) { return (uint64_t)blockIdx.x * kWaves + wave; }

// Data bytes of every item that is not the last of its list.
template <uint32_t G, bool ENCODE, bool DELTA>
__global__ __launch_bounds__(kThreads) void batch_item_bytes_kernel(BatchArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t t = wave_item(wave);
    const ItemRef r = item_ref(a, t);
    if (!r.valid) return;
    uint32_t bytes = 0;
    if (!r.last) {
        if (ENCODE) {
            const EncodeStream e = list_values(a, r.list);
#pragma unroll 1
            for (uint32_t g = 0; g < G; ++g) {
                SegValues sv;
                load_segment_values<DELTA>(e, (uint64_t)r.piece * G + g, lane, sv);
                bytes += segment_data_bytes(sv);
            }
        } else {
            const DecodeArgs p = list_stream(a, r.list);
            const uint32_t lb = lane_ctrl_bytes<4 * G>(p.in, p.in_bytes, p.n, (uint64_t)r.piece * G * kSegCtrl, lane);
            bytes = wave_last(wave_incl_scan(lb));
        }
    }
    if (lane == 0) a.ibytes[t] = bytes;
}

// Sum of the stored differences of every item that is not the last of its list.
template <uint32_t G>
__global__ __launch_bounds__(kThreads) void batch_item_sums_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t t = wave_item(wave);
    const ItemRef r = item_ref(a, t);
    if (!r.valid) return;
    uint32_t sum = 0;
    if (!r.last) {
        uint8_t *stage = s_stage + wave * kStageBytes;
        const DecodeArgs p = list_stream(a, r.list);
        const uint64_t s0 = (uint64_t)r.piece * G;
        Walker w;
        walker_begin(p, w, s0, s0 + G, a.ioff[t] - a.ioff[r.first_item], lane);
#pragma unroll 1
        for (uint64_t s = s0; s < s0 + G; ++s) {
            SegPlan seg;
            uint32_t sh16;
            walker_step(p, w, stage, lane, seg, sh16);
            uint32_t v[4][4];
            extract_segment(p, s, stage, seg, sh16, lane, v);
            walker_release();
            uint32_t x = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) x += v[k][0] + v[k][1] + v[k][2] + v[k][3];
            sum += wave_last(wave_incl_scan(x));
        }
        if (w.corrupt && a.err && lane == 0) *a.err = SVB_DECODE_CORRUPT;
    }
    if (lane == 0) a.ivsum[t] = sum;
}

template <uint32_t G, bool DELTA>
__global__ __launch_bounds__(kThreads) void batch_decode_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t t = wave_item(wave);
    const ItemRef r = item_ref(a, t);
    if (!r.valid) return;
    uint8_t *stage = s_stage + wave * kStageBytes;
    const DecodeArgs p = list_stream(a, r.list);
    const uint64_t segs = (p.n + kSegInts - 1) / kSegInts;
    const uint64_t s0 = (uint64_t)r.piece * G;
    const uint64_t s_end = s0 + G < segs ? s0 + G : segs;
    const uint64_t boff = r.piece ? a.ioff[t] - a.ioff[r.first_item] : 0ull;
    uint32_t carry = 0;
    if (DELTA) carry = a.starts[r.list] + (r.piece ? a.ivpre[t] - a.ivpre[r.first_item] : 0u);
    Walker w;
    walker_begin(p, w, s0, s_end, boff, lane);
#pragma unroll 1
    for (uint64_t s = s0; s < s_end; ++s) {
        SegPlan seg;
        uint32_t sh16;
        walker_step(p, w, stage, lane, seg, sh16);
        uint32_t v[4][4];
        extract_segment(p, s, stage, seg, sh16, lane, v);
        walker_release();
        if (DELTA) running_sum(v, carry);
        store_segment(p, s, lane, v, 0u);
    }
    if (w.corrupt && a.err && lane == 0) *a.err = SVB_DECODE_CORRUPT;
}

template <uint32_t G, bool DELTA>
__global__ __launch_bounds__(kThreads) void batch_encode_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t s_stage[kWaves * kEncStageWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t t = wave_item(wave);
    const ItemRef r = item_ref(a, t);
    if (!r.valid) return;
    uint32_t *stage = s_stage + wave * kEncStageWords;
    const EncodeStream e = list_values(a, r.list);
    const uint64_t segs = (e.n + kSegInts - 1) / kSegInts;
    const uint64_t s0 = (uint64_t)r.piece * G;
    const uint64_t s_end = s0 + G < segs ? s0 + G : segs;
    uint64_t boff = r.piece ? a.ioff[t] - a.ioff[r.first_item] : 0ull;
#pragma unroll 1
    for (uint64_t s = s0; s < s_end; ++s) boff += encode_segment<DELTA>(e, s, boff, lane, stage);
    if (r.last && lane == 0 && a.out_bytes) a.out_bytes[r.list] = (e.n + 3) / 4 + boff;
}

uint32_t list_grid(uint32_t m) { return (m + kThreads - 1) / kThreads; }
uint32_t item_grid(uint32_t t_cap) { return (t_cap + kWaves - 1) / kWaves; }

template <uint32_t G>
hipError_t launch_batch_g(const BatchArgs &a, int phase, bool encode, bool delta, hipStream_t s) {
    switch (phase) {
        case kBatchCount:
            hipLaunchKernelGGL((batch_count_kernel<G>), dim3(list_grid(a.m)), dim3(kThreads), 0, s, a);
            break;
        case kBatchItemBytes:
            if (!encode)
                hipLaunchKernelGGL((batch_item_bytes_kernel<G, false, false>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0,
                                   s, a);
            else if (delta)
                hipLaunchKernelGGL((batch_item_bytes_kernel<G, true, true>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0,
                                   s, a);
            else
                hipLaunchKernelGGL((batch_item_bytes_kernel<G, true, false>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0,
                                   s, a);
            break;
        case kBatchItemSums:
            hipLaunchKernelGGL((batch_item_sums_kernel<G>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            break;
        case kBatchWork:
            if (encode) {
                if (delta)
                    hipLaunchKernelGGL((batch_encode_kernel<G, true>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0, s, a);
                else
                    hipLaunchKernelGGL((batch_encode_kernel<G, false>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            } else {
                if (delta)
                    hipLaunchKernelGGL((batch_decode_kernel<G, true>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0, s, a);
                else
                    hipLaunchKernelGGL((batch_decode_kernel<G, false>), dim3(item_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            }
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchArgs &a, uint32_t item_segs, int phase, bool encode, bool delta, hipStream_t s) {
    if (phase == kBatchMap) {
        hipLaunchKernelGGL(batch_map_kernel, dim3(list_grid(a.m)), dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    switch (item_segs) {
        case 1: return launch_batch_g<1>(a, phase, encode, delta, s);
        case 2: return launch_batch_g<2>(a, phase, encode, delta, s);
        case 4: return launch_batch_g<4>(a, phase, encode, delta, s);
        case 8: return launch_batch_g<8>(a, phase, encode, delta, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace svb
