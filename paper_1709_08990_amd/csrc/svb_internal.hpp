// Internal interface between the C ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/svb.h"

namespace svb {

// Blocks (control bytes) per thread per tile: a tile is 256 * 4 blocks = 4096 integers.
constexpr int kWorkgroupThreads = 256;
constexpr int kBlocksPerThread = 4;
constexpr uint64_t kTileInts = 256ull * kBlocksPerThread * 4ull;

struct DecodeArgs {
    const uint8_t *in;
    uint64_t in_bytes;
    uint64_t n;
    uint32_t *out;
    uint32_t start;
    uint32_t *err;
    uint32_t *counters;    // [0] tile ticket, [1] finished workgroups
    uint64_t *byte_flags;  // one status word per tile (byte offsets)
    uint64_t *val_flags;   // one status word per tile (delta values)
    uint32_t epoch;
    uint32_t num_tiles;
};

struct EncodeArgs {
    const uint32_t *in;
    uint64_t n;
    uint8_t *out;
    uint32_t start;
    uint64_t *out_bytes;
    uint32_t *counters;
    uint64_t *byte_flags;
    uint32_t epoch;
    uint32_t num_tiles;
};

hipError_t launch_decode(const DecodeArgs &a, bool delta, hipStream_t s);
hipError_t launch_encode(const EncodeArgs &a, bool delta, hipStream_t s);
hipError_t launch_copy(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n, uint32_t value, hipStream_t s);

// Workgroups for a persistent launch of `kernel` over `num_tiles` tiles:
// resident workgroups per CU (from the occupancy calculator) times the CU count,
// capped by the number of tiles.
uint32_t persistent_grid(const void *kernel, uint32_t num_tiles);

}  // namespace svb
