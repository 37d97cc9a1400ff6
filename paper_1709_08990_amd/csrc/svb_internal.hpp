// Internal interface between the C ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/svb.h"

namespace svb {

// Blocks (control bytes) per thread per tile: a tile is 256 * K blocks = 1024 K integers.
constexpr int kWorkgroupThreads = 256;
#ifndef SVB_BLOCKS_PER_THREAD
#define SVB_BLOCKS_PER_THREAD 4
#endif
constexpr int kBlocksPerThread = SVB_BLOCKS_PER_THREAD;
constexpr uint64_t kTileInts = 256ull * kBlocksPerThread * 4ull;

// Words between consecutive tiles' status words (1 = packed).
#ifndef SVB_FLAG_STRIDE
#define SVB_FLAG_STRIDE 1
#endif
constexpr uint64_t kFlagStride = SVB_FLAG_STRIDE;

// Tiles are handed out by kTicketClasses ticket counters.  Workgroup b belongs
// to class b % classes (the dispatcher places workgroups on the eight XCDs
// round-robin, so a class is an XCD) and takes tiles t with t % classes equal
// to its class, in increasing order.  One shared counter would serialise every
// ticket on a single address; eight spread the atomics over eight lines.
constexpr uint32_t kTicketClasses = 8;
constexpr uint32_t kCounterStride = 32;  // uint32 words between counters (128 bytes)

// Tickets each workgroup takes beyond the last tile of its class, per kernel.
constexpr uint32_t kEncodeTicketsPastEnd = 1;
constexpr uint32_t kDecodeTicketsPastEnd = 3;       // the decoder asks three tiles ahead

struct TileQueue {
    uint32_t *counters;             // kTicketClasses counters, kCounterStride words apart
    uint32_t base[kTicketClasses];  // value of each counter when the launch starts
    uint32_t classes;               // min(kTicketClasses, grid)
    uint32_t num_tiles;
};

// A decode tile is four sub-tiles (one per data wave) of 64 x K blocks; a
// super-tile (one workgroup of the control reduction) covers 256 threads x 64
// blocks = kSubsPerSuper sub-tiles.
constexpr uint32_t kSubsPerTile = 4;
constexpr uint32_t kSubsPerSuper = 256 / kBlocksPerThread;
constexpr uint64_t kSuperInts = 256ull * 64ull * 4ull;

struct ReduceArgs {
    const uint8_t *in;     // stream; its first ceil(n/4) bytes are the control stream
    uint64_t in_bytes;
    uint64_t n;
    uint32_t *sub_loc;     // out: data byte offset of each sub-tile inside its super-tile
    uint32_t *sup_bytes;   // out: data bytes of each super-tile
    uint64_t num_subs;
    uint64_t num_supers;
};

struct DecodeArgs {
    const uint8_t *in;
    uint64_t in_bytes;
    uint64_t n;
    uint32_t *out;
    uint32_t start;
    uint32_t *err;
    TileQueue q;
    const uint32_t *sub_loc;   // byte offset of each sub-tile inside its super-tile
    const uint64_t *sup_off;   // data-stream byte offset of each super-tile
    uint32_t *sub_vloc;        // value offset of each sub-tile inside its tile (written by SUMS)
    uint32_t *tile_sum;        // value sum of each tile (written by SUMS)
    const uint32_t *tile_vpre; // exclusive value prefix of each tile (read by DELTA)
    uint64_t num_subs;
};

struct EncodeArgs {
    const uint32_t *in;
    uint64_t n;
    uint8_t *out;
    uint32_t start;
    uint64_t *out_bytes;
    TileQueue q;
    uint64_t *byte_flags;
    uint32_t epoch;
};

// Persistent grid size for the codec kernels over `num_tiles` tiles.
uint32_t decode_grid(int mode, uint32_t num_tiles);  // mode: 0 plain, 1 delta, 2 value sums
uint32_t encode_grid(bool delta, uint32_t num_tiles);
hipError_t launch_control_reduce(const ReduceArgs &a, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, void *out, uint64_t m, bool wide, hipStream_t s);
hipError_t launch_decode(const DecodeArgs &a, int mode, uint32_t grid, hipStream_t s);
hipError_t launch_encode(const EncodeArgs &a, bool delta, uint32_t grid, hipStream_t s);
hipError_t launch_copy(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n, uint32_t value, hipStream_t s);

// Workgroups for a persistent launch of `kernel` over `num_tiles` tiles:
// resident workgroups per CU (from the occupancy calculator) times the CU count,
// capped by the number of tiles.
uint32_t persistent_grid(const void *kernel, uint32_t num_tiles, uint32_t block_threads);

}  // namespace svb
