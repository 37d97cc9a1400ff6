// Device-side building blocks shared by the Stream VByte kernels (gfx950, wave64).
//
//  - wave-level inclusive scans with DPP row shifts and row broadcasts,
//  - a decoupled look-back over per-tile 64-bit status words (the serial
//    "advance the data pointer by C" chain of the paper's decoder, Section 4,
//    becomes an exclusive scan over tiles),
//  - byte-window loads that never touch memory outside the stream.
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

// Low L bytes of v (L in 1..4).
__device__ __forceinline__ uint32_t low_bytes(uint32_t v, uint32_t L) {
    return v & (0xFFFFFFFFu >> (32u - 8u * L));
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

// Exclusive prefix of tile `tile` from the words of tiles 0..tile-1, run by
// one full wave.  The tile's own aggregate is published right after the first
// window of predecessor words has been requested, so the wave never waits for
// its own store before reading.  Tiles of one ticket class are handed out in
// increasing order to running workgroups, so every predecessor is held by a
// workgroup that makes progress: the wait always ends.  Sums are modulo 2^VB.
// The caller publishes the inclusive prefix (excl + total) when it suits it.
template <int VB>
__device__ uint64_t lookback(uint64_t *flags, uint32_t tile, uint32_t epoch, uint64_t total) {
    const uint32_t lane = lane_id();
    const uint64_t vmask = (1ull << VB) - 1ull;
    if (tile == 0) return 0;
    uint64_t excl = 0;
    int64_t pos = (int64_t)tile - 1;
    bool published = false;
    for (;;) {
        const int64_t idx = pos - (int64_t)lane;
        for (;;) {
            uint64_t w = 0;
            if (idx >= 0) w = __hip_atomic_load(flags + idx * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!published) {
                if (lane == 0) flag_publish<VB>(flags, tile, epoch, kAggregate, total);
                published = true;
            }
            uint32_t st;
            if (idx >= 0)
                st = ((uint32_t)(w >> (VB + 2)) == epoch) ? (uint32_t)((w >> VB) & 3u) : 0u;
            else
                st = kInclusive;  // before tile 0: an inclusive prefix of zero
            const uint64_t val = (idx >= 0) ? (w & vmask) : 0ull;
            const uint64_t invalid = __ballot(st == 0);
            const uint64_t incl = __ballot(st == kInclusive);
            const uint64_t first = incl & (~incl + 1ull);           // nearest inclusive lane
            const uint64_t below = incl ? (first - 1ull) : ~0ull;   // lanes that must be aggregates
            if ((invalid & below) == 0) {
                const uint64_t take = incl ? (below | first) : ~0ull;
                const uint64_t mine = ((take >> lane) & 1ull) ? val : 0ull;
                excl = (excl + wave_sum_u64(mine)) & vmask;
                if (incl) return excl;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        pos -= kWave;
    }
}

// ---------------------------------------------------------------- byte windows

// The 16 bytes at in[a .. a+16) as four little-endian dwords, reading only
// [a, limit) (bytes at or past limit read as 0).  `in` has any alignment.
// Used for the first and last tiles of a stream, where a 20-byte window
// could leave the buffer.
__device__ __forceinline__ void load_window16_checked(const uint8_t *in, uint64_t a, uint64_t limit,
                                                      uint32_t &d0, uint32_t &d1, uint32_t &d2, uint32_t &d3) {
    uint32_t d[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t byte = (a + i < limit) ? (uint32_t)in[a + i] : 0u;
        d[i >> 2] |= byte << (8 * (i & 3));
    }
    d0 = d[0]; d1 = d[1]; d2 = d[2]; d3 = d[3];
}

// Raw 20-byte window around in[a]: the dword-aligned dwords covering
// [a, a + 16), plus the byte shift of a inside the first one.  The caller
// guarantees the window lies inside the buffer.
struct Window {
    u32x4 w;
    uint32_t w4;
    uint32_t sh;
};

__device__ __forceinline__ Window load_window(const uint8_t *in, uint64_t a) {
    const uint8_t *pa = in + a;
    Window r;
    r.sh = (uint32_t)((uintptr_t)pa & 3u);
    const uint8_t *base = pa - r.sh;
    r.w = *(const u32x4 *)base;
    r.w4 = *(const uint32_t *)(base + 16);
    return r;
}

__device__ __forceinline__ void align_window(const Window &r, uint32_t &d0, uint32_t &d1, uint32_t &d2,
                                             uint32_t &d3) {
    d0 = __builtin_amdgcn_alignbyte(r.w.y, r.w.x, r.sh);
    d1 = __builtin_amdgcn_alignbyte(r.w.z, r.w.y, r.sh);
    d2 = __builtin_amdgcn_alignbyte(r.w.w, r.w.z, r.sh);
    d3 = __builtin_amdgcn_alignbyte(r.w4, r.w.w, r.sh);
}

// Select word q (0..3) of (d0,d1,d2,d3) without dynamic register indexing.
__device__ __forceinline__ uint32_t pick4(uint32_t q, uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3) {
    const uint32_t lo = (q & 1u) ? d1 : d0;
    const uint32_t hi = (q & 1u) ? d3 : d2;
    return (q & 2u) ? hi : lo;
}

// The four integers of one block from its 16-byte window (Section 4: the
// shuffle of Fig. 4 done with byte-align instructions).  c = control byte.
__device__ __forceinline__ void gather_block(uint32_t c, uint32_t d0, uint32_t d1, uint32_t d2,
                                             uint32_t d3, uint32_t &v0, uint32_t &v1, uint32_t &v2,
                                             uint32_t &v3) {
    const uint32_t L0 = (c & 3u) + 1u;
    const uint32_t L1 = ((c >> 2) & 3u) + 1u;
    const uint32_t L2 = ((c >> 4) & 3u) + 1u;
    const uint32_t L3 = ((c >> 6) & 3u) + 1u;
    const uint32_t o1 = L0;            // 1..4
    const uint32_t o2 = o1 + L1;       // 2..8
    const uint32_t o3 = o2 + L2;       // 3..12
    v0 = low_bytes(d0, L0);
    {
        const uint32_t q = o1 >> 2, s = o1 & 3u;
        const uint32_t lo = q ? d1 : d0, hi = q ? d2 : d1;
        v1 = low_bytes(__builtin_amdgcn_alignbyte(hi, lo, s), L1);
    }
    {
        const uint32_t q = o2 >> 2, s = o2 & 3u;
        const uint32_t lo = pick4(q, d0, d1, d2, d3), hi = pick4(q + 1u, d0, d1, d2, d3);
        v2 = low_bytes(__builtin_amdgcn_alignbyte(hi, lo, s), L2);
    }
    {
        const uint32_t q = o3 >> 2, s = o3 & 3u;
        const uint32_t lo = pick4(q, d0, d1, d2, d3), hi = pick4(q + 1u, d0, d1, d2, d3);
        v3 = low_bytes(__builtin_amdgcn_alignbyte(hi, lo, s), L3);
    }
}

}  // namespace svb
