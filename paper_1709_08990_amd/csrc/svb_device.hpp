// Device-side building blocks shared by the Stream VByte kernels (gfx950, wave64).
//
//  - wave-level inclusive scans with DPP row shifts and row broadcasts,
//  - the length rules of the format (Sections 3 and 4).
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

// Global-memory views of pointers.  A pointer read out of memory (a batched
// call's task descriptor) is generic to the compiler, and generic accesses
// become FLAT instructions, which the LDS wait counter also tracks: every wait
// before an LDS read would then wait for the next task's prefetched loads
// too.  Every stream and output access goes through these views.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

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

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------- byte windows

// 16 bytes starting at byte o (0..15) of the 32 bytes lo:hi (little-endian).
__device__ __forceinline__ u32x4a shift_window(const u32x4a &lo, const u32x4a &hi, uint32_t o) {
    const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    const uint32_t q = o >> 2, rb = o & 3u;
    uint32_t r[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        // dwords q + i and q + i + 1, q in 0..3
        const uint32_t a0 = q == 0 ? w[i] : q == 1 ? w[i + 1] : q == 2 ? w[i + 2] : w[i + 3];
        const uint32_t a1 = q == 0 ? w[i + 1] : q == 1 ? w[i + 2] : q == 2 ? w[i + 3] : w[i + 4];
        r[i] = __builtin_amdgcn_alignbyte(a1, a0, rb);
    }
    return u32x4a{r[0], r[1], r[2], r[3]};
}

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

}  // namespace svb
