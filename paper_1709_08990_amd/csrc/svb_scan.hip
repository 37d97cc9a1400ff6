// Device-wide exclusive prefix sums of uint32 arrays, used by the decoders and
// the batched calls to turn per-piece byte counts and value sums into offsets
// and carries (the paper's serial "advance the data pointer" and running sum,
// Sections 2 and 4, become scans).
//
// WIDE: 64-bit sums (byte offsets).  Otherwise sums modulo 2^32 plus `start`
// (delta carries).  A wide scan's values are byte counts of at most a few
// tens of thousands (a group, segment or task), below 2^18, so one
// workgroup step of at most 16384 of them sums below 2^32: inside a step the
// wide scan uses the 32-bit wave scan, and only the carry between steps and
// tiles is 64-bit.  An optional `total` receives the sum of all m values
// (64-bit, or 32-bit plus start modulo 2^32).
//
// Up to kSingleMax (16384) values: one workgroup of 1024 threads.  Above
// that: reduce-then-scan over tiles of 4096 values, one 256-thread workgroup
// each, in two launches (tile sums; then each tile adds up the sums of the
// tiles before it and scans its values from there), so that a few hundred
// thousand values already spread over most of the chip.  Measured at 65,536
// values: one workgroup taking them in one step of 64 per thread, 18.5 us;
// three launches (with a one-workgroup scan of the tile sums between), about
// 10 us; the two launches save the middle one.
#include <type_traits>

#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

namespace {

constexpr uint32_t kScanThreads = 1024;                 // the single-workgroup scan
constexpr uint32_t kScanPer = 16;
constexpr uint32_t kScanTile = kScanThreads * kScanPer;  // values per workgroup step
constexpr uint64_t kSingleMax = kScanTile;
constexpr uint32_t kTileThreads = 256;                   // the multi-workgroup scan
constexpr uint32_t kTileVals = kTileThreads * kScanPer;

template <bool WIDE>
using acc_t = typename std::conditional<WIDE, uint64_t, uint32_t>::type;

// Inclusive wave scan in the accumulator type.
__device__ __forceinline__ uint32_t wave_scan_acc(uint32_t x) { return wave_incl_scan(x); }
__device__ __forceinline__ uint64_t wave_scan_acc(uint64_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Loads the 16 values of thread `tid` from base on, 0 past m.
__device__ __forceinline__ void load16(const uint32_t *in, uint64_t base, uint64_t m, uint32_t tid,
                                       uint32_t (&x)[kScanPer]) {
    const uint64_t i0 = base + (uint64_t)tid * kScanPer;
    if (i0 + kScanPer <= m) {
#pragma unroll
        for (uint32_t j = 0; j < kScanPer; j += 4) {
            const u32x4 w = *(const u32x4 *)(in + i0 + j);
            x[j] = w.x; x[j + 1] = w.y; x[j + 2] = w.z; x[j + 3] = w.w;
        }
    } else {
#pragma unroll
        for (uint32_t j = 0; j < kScanPer; ++j) x[j] = (i0 + j < m) ? in[i0 + j] : 0u;
    }
}

// Workgroup-wide exclusive prefix of each thread's value over a workgroup of
// W waves; returns the thread's prefix and writes the workgroup total to
// *total (all threads).  s_wtot holds W + 1 entries.
template <uint32_t W, typename A>
__device__ __forceinline__ A block_prefix(A sum, A *s_wtot, A *total) {
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const A incl = wave_scan_acc(sum);
    if (lane == kWave - 1) s_wtot[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const A t = lane < W ? s_wtot[lane] : (A)0;
        const A ti = wave_scan_acc(t);
        if (lane < W) s_wtot[lane] = ti - t;
        if (lane == kWave - 1) s_wtot[W] = ti;
    }
    __syncthreads();
    const A pre = s_wtot[wave] + incl - sum;
    *total = s_wtot[W];
    __syncthreads();
    return pre;
}

// Writes thread `tid`'s 16 outputs: carry + pre + the exclusive sums of x.
// The running sum inside the thread's 16 values stays 32-bit (for WIDE: the
// 16 values and pre sum below 2^32, see above); wide outputs go out as
// 16-byte stores of two 64-bit values.
template <bool WIDE>
__device__ __forceinline__ void store16(void *out, uint64_t base, uint64_t m, uint32_t tid, acc_t<WIDE> carry,
                                        uint32_t pre, const uint32_t (&x)[kScanPer]) {
    const uint64_t i0 = base + (uint64_t)tid * kScanPer;
    uint32_t r[kScanPer];
    uint32_t run = WIDE ? pre : (uint32_t)carry + pre;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) {
        r[j] = run;
        run += x[j];
    }
    if (WIDE) {
        const uint64_t c = (uint64_t)carry;
        uint64_t *o = (uint64_t *)out + i0;
        if (i0 + kScanPer <= m) {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j += 2) {
                const uint64_t y0 = c + r[j], y1 = c + r[j + 1];
                *(u32x4 *)(o + j) = u32x4{(uint32_t)y0, (uint32_t)(y0 >> 32), (uint32_t)y1, (uint32_t)(y1 >> 32)};
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; ++j)
                if (i0 + j < m) o[j] = c + r[j];
        }
    } else {
        uint32_t *o = (uint32_t *)out + i0;
        if (i0 + kScanPer <= m) {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; j += 4) *(u32x4 *)(o + j) = u32x4{r[j], r[j + 1], r[j + 2], r[j + 3]};
        } else {
#pragma unroll
            for (uint32_t j = 0; j < kScanPer; ++j)
                if (i0 + j < m) o[j] = r[j];
        }
    }
}

template <bool WIDE>
__device__ __forceinline__ void write_total(void *total, acc_t<WIDE> v) {
    if (!total) return;
    if (WIDE)
        *(uint64_t *)total = v;
    else
        *(uint32_t *)total = (uint32_t)v;
}

// One workgroup over the whole array.
template <bool WIDE>
__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(const uint32_t *in, void *out, uint64_t m,
                                                                   uint32_t start, void *total) {
    typedef acc_t<WIDE> A;
    constexpr uint32_t W = kScanThreads / kWave;
    __shared__ uint32_t s_wtot[W + 1];
    const uint32_t tid = threadIdx.x;
    A carry = WIDE ? (A)0 : (A)start;
    for (uint64_t base = 0; base < m; base += kScanTile) {
        uint32_t x[kScanPer];
        load16(in, base, m, tid, x);
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < kScanPer; ++j) sum += x[j];
        uint32_t step_total;
        const uint32_t pre = block_prefix<W, uint32_t>(sum, s_wtot, &step_total);
        store16<WIDE>(out, base, m, tid, carry, pre, x);
        carry += (A)step_total;
    }
    if (tid == 0) write_total<WIDE>(total, carry);
}

// Tile t's sum into sums[t] (64-bit for WIDE).
template <bool WIDE>
__global__ __launch_bounds__(kTileThreads) void scan_tile_sums_kernel(const uint32_t *in, uint64_t m, uint32_t *sums) {
    constexpr uint32_t W = kTileThreads / kWave;
    __shared__ uint32_t s_wtot[W + 1];
    const uint64_t base = (uint64_t)blockIdx.x * kTileVals;
    uint32_t x[kScanPer];
    load16(in, base, m, threadIdx.x, x);
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) sum += x[j];
    uint32_t tot;
    (void)block_prefix<W, uint32_t>(sum, s_wtot, &tot);
    if (threadIdx.x == 0) {
        if (WIDE) {
            // split into two 32-bit words so the tile sums scan as u32 pairs below
            sums[2 * blockIdx.x] = (uint32_t)tot;
            sums[2 * blockIdx.x + 1] = (uint32_t)((uint64_t)tot >> 32);
        } else {
            sums[blockIdx.x] = (uint32_t)tot;
        }
    }
}

// Per-tile scan that takes its own carry, the sum of the tile sums before it
// (`start` on top, when not WIDE), so that no separate scan of the tile sums
// runs between the two passes.  Tile t reads t sums: a few per thread up to
// millions of values (2^22 values, 1024 tiles: at most 4 per thread).  The
// last tile writes the total.

template <bool WIDE>
__global__ __launch_bounds__(kTileThreads) void scan_tile_carry_final_kernel(const uint32_t *in, void *out, uint64_t m,
                                                                             const uint32_t *sums, uint32_t start,
                                                                             void *total) {
    typedef acc_t<WIDE> A;
    constexpr uint32_t W = kTileThreads / kWave;
    __shared__ A s_acc[W + 1];
    __shared__ uint32_t s_wtot[W + 1];
    const uint64_t tile = blockIdx.x;
    A c = 0;
    for (uint64_t t = threadIdx.x; t < tile; t += kTileThreads)
        c += WIDE ? (A)(sums[2 * t] | ((uint64_t)sums[2 * t + 1] << 32)) : (A)sums[t];
    A before;
    (void)block_prefix<W, A>(c, s_acc, &before);
    const A carry = (WIDE ? (A)0 : (A)start) + before;
    const uint64_t base = tile * kTileVals;
    uint32_t x[kScanPer];
    load16(in, base, m, threadIdx.x, x);
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) sum += x[j];
    uint32_t tot;
    const uint32_t p = block_prefix<W, uint32_t>(sum, s_wtot, &tot);
    store16<WIDE>(out, base, m, threadIdx.x, carry, p, x);
    if (tile == gridDim.x - 1 && threadIdx.x == 0) write_total<WIDE>(total, carry + (A)tot);
}

}  // namespace

uint64_t scan_scratch_bytes(uint64_t m) {
    if (m <= kSingleMax) return 0;
    const uint64_t tiles = (m + kTileVals - 1) / kTileVals;
    return 8 * tiles;  // tile sums (two words each when wide)
}

hipError_t launch_scan(const uint32_t *in, void *out, uint64_t m, bool wide, uint32_t start, hipStream_t s,
                       void *total, void *scratch) {
    if (m <= kSingleMax) {
        if (wide)
            hipLaunchKernelGGL((scan_single_kernel<true>), dim3(1), dim3(kScanThreads), 0, s, in, out, m, start, total);
        else
            hipLaunchKernelGGL((scan_single_kernel<false>), dim3(1), dim3(kScanThreads), 0, s, in, out, m, start, total);
        return hipGetLastError();
    }
    if (!scratch) return hipErrorInvalidValue;
    const uint64_t tiles = (m + kTileVals - 1) / kTileVals;
    uint32_t *sums = (uint32_t *)scratch;
    if (wide) {
        hipLaunchKernelGGL((scan_tile_sums_kernel<true>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, in, m, sums);
        hipLaunchKernelGGL((scan_tile_carry_final_kernel<true>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, in,
                           out, m, sums, start, total);
    } else {
        hipLaunchKernelGGL((scan_tile_sums_kernel<false>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, in, m, sums);
        hipLaunchKernelGGL((scan_tile_carry_final_kernel<false>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, in,
                           out, m, sums, start, total);
    }
    return hipGetLastError();
}

}  // namespace svb
