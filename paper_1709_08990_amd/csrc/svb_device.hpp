// Device-side building blocks shared by the Stream VByte kernels (gfx950, wave64).
//
//  - wave-level inclusive scans with DPP row shifts and row broadcasts,
//  - a decoupled look-back over per-tile 64-bit status words (the encoder's
//    serial "append after the previous integer's bytes" becomes an exclusive
//    scan over tiles).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "svb_internal.hpp"

namespace svb {

// 16-byte vector whose only alignment requirement is 4 bytes: global
// loads/stores of it become one dwordx4 access.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(4)));
// Same with natural 16-byte alignment (LDS).
typedef uint32_t u32x4a __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kThreads = 256;           // 4 waves per workgroup
constexpr int kWaves = kThreads / kWave;

// ---------------------------------------------------------------- wave scans

// Inclusive prefix sum over the 64 lanes of a wave (mod 2^32).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, true);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false); // row_bcast:15 -> rows 1,3
    x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false); // row_bcast:31 -> rows 2,3
    return x;
}

__device__ __forceinline__ uint32_t wave_last(uint32_t x) {
    return __builtin_amdgcn_readlane(x, kWave - 1);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------- control bytes

// Data bytes described by control byte c when its first r (0..4) integers are in
// use: r plus the sum of their 2-bit codes (Section 4: between 4 and 16 for r = 4).
__device__ __forceinline__ uint32_t control_data_bytes(uint32_t c, uint32_t r) {
    const uint32_t keep = (r >= 4) ? 0xFFu : ((1u << (2u * r)) - 1u);
    c &= keep;
    return r + __builtin_popcount(c & 0x55u) + 2u * __builtin_popcount(c & 0xAAu);
}

// Byte length of one integer (Section 3): 1 + floor(log2(v|1)) / 8.
__device__ __forceinline__ uint32_t byte_length(uint32_t v) {
    return ((31u - (uint32_t)__builtin_clz(v | 1u)) >> 3) + 1u;
}

// ---------------------------------------------------------------- tickets

// Next tile for this workgroup (>= q.num_tiles once its class has none left).
// Each class's tiles are handed out in increasing order to running workgroups,
// so a tile's predecessors are always held by workgroups that make progress.
__device__ __forceinline__ uint32_t take_tile(const TileQueue &q) {
    const uint32_t cls = blockIdx.x % q.classes;
    const uint32_t j = atomicAdd(q.counters + cls * kCounterStride, 1u) - q.base[cls];
    return j * q.classes + cls;
}

// ---------------------------------------------------------------- look-back

// A tile's status word: [epoch | status(2) | value(VB)].  status 1 = the tile's
// own aggregate, 2 = inclusive prefix up to and including the tile.  The epoch
// (20 bits) tells words written by the current launch from stale ones, so the
// status array never needs clearing between launches.
constexpr uint32_t kEpochBits = 20;
constexpr uint32_t kAggregate = 1;
constexpr uint32_t kInclusive = 2;

template <int VB>
__device__ __forceinline__ uint64_t flag_word(uint32_t epoch, uint32_t status, uint64_t value) {
    return ((uint64_t)epoch << (VB + 2)) | ((uint64_t)status << VB) | (value & ((1ull << VB) - 1ull));
}

template <int VB>
__device__ __forceinline__ void flag_publish(uint64_t *flags, uint32_t tile, uint32_t epoch,
                                             uint32_t status, uint64_t value) {
    __hip_atomic_store(flags + (uint64_t)tile * kFlagStride, flag_word<VB>(epoch, status, value), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Polls of predecessor words before a look-back gives up (each poll is a
// round trip to memory plus a short sleep, about a microsecond): a safety net
// that turns a wait that cannot end into a reported error instead of a hung
// device.  Every predecessor is held by a running workgroup, so in normal
// operation the limit is never reached.
constexpr uint32_t kLookbackPollLimit = 1u << 22;

// Predecessor words each lane reads per poll: one poll covers
// kLookbackPerLane * 64 predecessors.  Each poll is a device-coherent read
// that bypasses the per-XCD L2, and many waves poll at once, so a wider window
// costs more than it saves (measured on MI355X: 4 or 16 words per lane made a
// look-back-bound kernel 2.4x and 10x slower than 1).
#ifndef SVB_LOOKBACK_PER_LANE
#define SVB_LOOKBACK_PER_LANE 1
#endif
constexpr uint32_t kLookbackPerLane = SVB_LOOKBACK_PER_LANE;

// Exclusive prefix of tile `tile` from the words of tiles 0..tile-1, run by
// one full wave.  The tile's own aggregate is published right after the first
// window of predecessor words has been requested, so the wave never waits for
// its own store before reading.  Tiles are handed out in increasing order to
// running workgroups, so every predecessor is held by a workgroup that makes
// progress: the wait always ends.  Sums are modulo 2^VB.  The caller publishes
// the inclusive prefix (excl + total) when it suits it.  `stalled` is set (and
// 0 returned) when the poll limit is reached.
template <int VB>
__device__ uint64_t lookback(uint64_t *flags, uint32_t tile, uint32_t epoch, uint64_t total, bool &stalled) {
    constexpr uint32_t P = kLookbackPerLane;
    const uint32_t lane = lane_id();
    const uint64_t vmask = (1ull << VB) - 1ull;
    stalled = false;
    if (tile == 0) return 0;
    uint64_t excl = 0;
    int64_t pos = (int64_t)tile - 1;  // nearest predecessor not summed yet
    bool published = false;
    uint32_t polls = 0;
    for (;;) {
        // lane l covers predecessors pos - P l - j, j = 0..P-1 (nearest first)
        for (;;) {
            uint64_t w[P];
#pragma unroll
            for (uint32_t j = 0; j < P; ++j) {
                const int64_t idx = pos - (int64_t)(P * lane + j);
                w[j] = idx >= 0 ? __hip_atomic_load(flags + idx * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : 0ull;
            }
            if (!published) {
                if (lane == 0) flag_publish<VB>(flags, tile, epoch, kAggregate, total);
                published = true;
            }
            // per lane: the first inclusive word (fi = P if none) and whether a
            // word before it has not been published by this launch
            uint32_t fi = P;
            bool bad = false;
#pragma unroll
            for (uint32_t j = 0; j < P; ++j) {
                const int64_t idx = pos - (int64_t)(P * lane + j);
                uint32_t st = kInclusive;  // before tile 0: an inclusive prefix of zero
                if (idx >= 0) st = ((uint32_t)(w[j] >> (VB + 2)) == epoch) ? (uint32_t)((w[j] >> VB) & 3u) : 0u;
                if (fi == P) {
                    if (st == kInclusive)
                        fi = j;
                    else if (st == 0)
                        bad = true;
                }
            }
            const uint64_t has_incl = __ballot(fi < P);
            const uint64_t first = has_incl & (~has_incl + 1ull);        // nearest lane with an inclusive word
            const uint64_t before = has_incl ? (first - 1ull) : ~0ull;   // lanes that must be all aggregates
            if ((__ballot(bad) & (before | first)) == 0) {
                const bool whole = (before >> lane) & 1ull;
                const bool part = (first >> lane) & 1ull;
                uint64_t mine = 0;
#pragma unroll
                for (uint32_t j = 0; j < P; ++j) {
                    const int64_t idx = pos - (int64_t)(P * lane + j);
                    const uint64_t val = idx >= 0 ? (w[j] & vmask) : 0ull;
                    if (whole || (part && j <= fi)) mine += val;
                }
                excl = (excl + wave_sum_u64(mine)) & vmask;
                if (has_incl) return excl;
                break;
            }
            if (++polls >= kLookbackPollLimit) {
                stalled = true;
                return 0;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        pos -= (int64_t)P * kWave;
    }
}

}  // namespace svb
