// The two byte-oriented formats the paper compares Stream VByte with (Table 1):
//
//   VByte (Section 1): seven data bits per byte, least significant first; the
//   top bit of a byte is 1 when another byte of the same integer follows.
//   varint-GB (Section 3, Fig. 1): per block of four integers a control byte
//   (the same 2-bit codes as Stream VByte) followed by the block's data bytes.
//
// Encoding is the Stream VByte scheme: byte counts per 1024-integer segment,
// a scan, then each segment packed in LDS and copied out.
//
// VByte decodes without a dependency chain: an integer ends at every byte
// whose top bit is clear, so a tile of 1024 bytes counts its ends, a scan
// turns the counts into integer indices, and each lane decodes the integers
// ending in its 16 bytes (looking back at most 8 bytes for the start of the
// first one).
//
// varint-GB keeps the chain Section 3 describes: where block k + 1 starts
// depends on block k's control byte.  It is broken by speculation.  Each lane
// owns a 128-byte chunk; since a block takes at most 17 bytes, the first
// block starting in a chunk starts at one of its first 17 bytes, and for each
// of these 17 entries the lane walks the control bytes to the chunk's end,
// giving a map entry -> (exit offset into the next chunk, blocks started).
// Maps compose: 64 chunk maps make a tile map (8 KiB), 64 tile maps a
// supertile map (512 KiB).  One wave then follows the true chain (entry 0)
// across supertiles, waves per supertile follow it across tiles, and the
// decode pass follows it across the chunks of its tile and decodes.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

namespace {

constexpr uint32_t kCmpPer = kSegInts / kWave;     // 16 integers per lane
constexpr uint32_t kVbTile = 16 * kWave;           // VByte decode: 1024 bytes per wave
constexpr uint32_t kGbChunk = 128;                 // varint-GB: bytes per lane
constexpr uint32_t kGbTile = kGbChunk * kWave;     // 8192 bytes per wave
constexpr uint32_t kGbEntries = 17;                // a block spans at most 17 bytes
constexpr uint32_t kGbEnd = 31;                    // exit marker: the walk reached in_bytes
constexpr uint32_t kGbStage = kGbTile + 32;        // a tile and the bytes its last blocks may spill into
// In LDS a chunk takes 132 bytes (33 dwords, an odd count), so that the 64
// lanes, each reading its own chunk at the same offset, hit different banks
// (a 128-byte pitch puts them all in one).
constexpr uint32_t kGbPitch = kGbChunk + 4;
constexpr uint32_t kGbLdsMap = kWave * kGbPitch;          // a tile
constexpr uint32_t kGbLdsDecode = (kWave + 1) * kGbPitch; // a tile and its spill bytes
constexpr uint32_t kStageMax = 5 * kSegInts;       // bytes of one encoded segment, at most

__device__ __forceinline__ uint64_t wave_index() { return (uint64_t)blockIdx.x * kWaves + threadIdx.x / kWave; }

// Bytes [pos, pos + 16) of the stream [in, in + len), from the aligned
// 16-byte chunks that overlap the stream only (such a chunk never crosses a
// page).  Bytes outside the stream are unspecified.
__device__ __forceinline__ u32x4a load_window(const uint8_t *in, uint64_t len, uint64_t pos) {
    const uintptr_t s0 = (uintptr_t)in, S = s0 + pos, Sa = S & ~(uintptr_t)15;
    const uint32_t o = (uint32_t)(S & 15u);
    const uintptr_t s_end = s0 + len;
    u32x4a lo = {0u, 0u, 0u, 0u}, hi = {0u, 0u, 0u, 0u};
    if (Sa < s_end) lo = *gptr((const u32x4a *)Sa);
    if (o && Sa + 16 < s_end) hi = *gptr((const u32x4a *)(Sa + 16));
    return shift_window(lo, hi, o);
}

__device__ __forceinline__ uint32_t byte_of(const u32x4a &w, uint32_t j) {
    const uint32_t d = j < 4 ? w.x : j < 8 ? w.y : j < 12 ? w.z : w.w;
    return (d >> (8 * (j & 3u))) & 0xFFu;
}

// ---------------------------------------------------------------- encoders

template <int FMT>
__device__ __forceinline__ uint32_t int_bytes(uint32_t v) {
    if (FMT == kFmtVByte) return v < (1u << 7) ? 1u : v < (1u << 14) ? 2u : v < (1u << 21) ? 3u : v < (1u << 28) ? 4u : 5u;
    return byte_length(v);
}

// The lane's 16 integers (0 past n) and how many of them exist.
__device__ __forceinline__ uint32_t load_ints(const uint32_t *in, uint64_t n, uint64_t i0, uint32_t (&x)[kCmpPer]) {
    if (i0 + kCmpPer <= n) {
#pragma unroll
        for (uint32_t j = 0; j < kCmpPer; j += 4) {
            const u32x4 w = *gptr((const u32x4 *)(in + i0 + j));
            x[j] = w.x; x[j + 1] = w.y; x[j + 2] = w.z; x[j + 3] = w.w;
        }
        return kCmpPer;
    }
#pragma unroll
    for (uint32_t j = 0; j < kCmpPer; ++j) x[j] = i0 + j < n ? gptr(in)[i0 + j] : 0u;
    return i0 >= n ? 0u : (uint32_t)(n - i0);
}

// Encoded bytes of the lane's r integers (varint-GB adds one control byte per
// block; i0 is a multiple of 4, so its blocks are the lane's own).
template <int FMT>
__device__ __forceinline__ uint32_t lane_bytes(const uint32_t (&x)[kCmpPer], uint32_t r) {
    uint32_t b = FMT == kFmtVarintGB ? (r + 3) / 4 : 0u;
#pragma unroll
    for (uint32_t j = 0; j < kCmpPer; ++j) b += j < r ? int_bytes<FMT>(x[j]) : 0u;
    return b;
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void cmp_sizes_kernel(CmpEncodeArgs a) {
    const uint64_t seg = wave_index();
    if (seg >= a.segs) return;
    const uint32_t lane = lane_id();
    uint32_t x[kCmpPer];
    const uint32_t r = load_ints(a.in, a.n, seg * kSegInts + (uint64_t)lane * kCmpPer, x);
    const uint32_t tot = wave_last(wave_incl_scan(lane_bytes<FMT>(x, r)));
    if (lane == 0) gptr(a.seg_bytes)[seg] = tot;
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void cmp_pack_kernel(CmpEncodeArgs a) {
    __shared__ uint8_t s_stage[kWaves][kStageMax];
    const uint64_t seg = wave_index();
    if (seg >= a.segs) return;
    const uint32_t lane = lane_id();
    uint8_t *stage = s_stage[threadIdx.x / kWave];
    uint32_t x[kCmpPer];
    const uint32_t r = load_ints(a.in, a.n, seg * kSegInts + (uint64_t)lane * kCmpPer, x);
    const uint32_t mine = lane_bytes<FMT>(x, r);
    const uint32_t incl = wave_incl_scan(mine);
    const uint32_t total = wave_last(incl);
    uint32_t p = incl - mine;
    if (FMT == kFmtVByte) {
#pragma unroll
        for (uint32_t j = 0; j < kCmpPer; ++j) {
            if (j < r) {
                uint32_t v = x[j];
                while (v >= 128u) {
                    stage[p++] = (uint8_t)(0x80u | (v & 0x7Fu));
                    v >>= 7;
                }
                stage[p++] = (uint8_t)v;
            }
        }
    } else {
#pragma unroll
        for (uint32_t q = 0; q < kCmpPer / 4; ++q) {
            if (4 * q < r) {
                const uint32_t at = p++;
                uint32_t ctrl = 0;
#pragma unroll
                for (uint32_t jj = 0; jj < 4; ++jj) {
                    if (4 * q + jj < r) {
                        const uint32_t v = x[4 * q + jj];
                        const uint32_t len = byte_length(v);
                        ctrl |= (len - 1u) << (2u * jj);
                        for (uint32_t k = 0; k < len; ++k) stage[p++] = (uint8_t)(v >> (8u * k));
                    }
                }
                stage[at] = (uint8_t)ctrl;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t off = a.seg_off[seg];
    for (uint32_t i = lane; i < total; i += kWave) gptr(a.out)[off + i] = stage[i];
    if (a.out_bytes && seg + 1 == a.segs && lane == 0) *gptr(a.out_bytes) = off + total;
}

// ---------------------------------------------------------------- VByte decoder

// Bit j set: byte j of the window ends an integer (top bit clear) and lies
// before the stream's end (rem bytes left from the window's start).
__device__ __forceinline__ uint32_t end_mask(const u32x4a &w, uint64_t rem) {
    const uint32_t d[4] = {w.x, w.y, w.z, w.w};
    uint32_t m = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t t = ~d[q] & 0x80808080u;
        m |= (((t >> 7) & 1u) | ((t >> 14) & 2u) | ((t >> 21) & 4u) | ((t >> 28) & 8u)) << (4 * q);
    }
    return rem < 16 ? m & ((1u << rem) - 1u) : m;
}

__global__ __launch_bounds__(kThreads) void vb_count_kernel(VbDecodeArgs a) {
    const uint64_t tile = wave_index();
    if (tile >= a.tiles) return;
    const uint32_t lane = lane_id();
    const uint64_t pos = tile * kVbTile + 16ull * lane;
    uint32_t c = 0;
    if (pos < a.in_bytes) c = __builtin_popcount(end_mask(load_window(a.in, a.in_bytes, pos), a.in_bytes - pos));
    const uint32_t tot = wave_last(wave_incl_scan(c));
    if (lane == 0) gptr(a.tcount)[tile] = tot;
}

__global__ __launch_bounds__(kThreads) void vb_decode_kernel(VbDecodeArgs a) {
    __shared__ uint32_t s_vals[kWaves][kVbTile];
    const uint64_t tile = wave_index();
    if (tile >= a.tiles) return;
    const uint32_t lane = lane_id();
    uint32_t *vals = s_vals[threadIdx.x / kWave];
    const uint64_t pos = tile * kVbTile + 16ull * lane;
    u32x4a w = {0u, 0u, 0u, 0u};
    uint32_t m = 0;
    if (pos < a.in_bytes) {
        w = load_window(a.in, a.in_bytes, pos);
        m = end_mask(w, a.in_bytes - pos);
    }
    // The 8 bytes before pos: the previous lane's last 8, the previous tile's
    // for lane 0; before the stream they count as integer ends.
    uint32_t pz = __shfl_up(w.z, 1, kWave), pw = __shfl_up(w.w, 1, kWave);
    if (lane == 0) {
        pz = pw = 0u;
        if (tile > 0) {
            const u32x4a b = load_window(a.in, a.in_bytes, pos - 16);
            pz = b.z;
            pw = b.w;
        }
    }
    // The integer running into this lane's bytes: the continuation bytes
    // right before pos (at most 8 looked at; more makes it too long anyway).
    const uint64_t pv = ((uint64_t)pw << 32) | pz;
    uint32_t ends = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) ends |= ((uint32_t)(pv >> (8 * i + 7)) & 1u ? 0u : 1u) << i;
    const uint32_t run = ends ? 7u - (31u - (uint32_t)__builtin_clz(ends)) : 8u;
    uint32_t acc = 0, k = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
        if (i >= 8 - run) {
            if (k < 5) acc |= ((uint32_t)(pv >> (8 * i)) & 0x7Fu) << (7 * k);
            ++k;
        }
    }
    const uint32_t cnt = __builtin_popcount(m);
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t in_tile = wave_last(incl);
    const uint64_t first = a.toff[tile];
    uint32_t r = incl - cnt;
    bool bad = false;
    const uint64_t rem = pos < a.in_bytes ? a.in_bytes - pos : 0;
#pragma unroll
    for (uint32_t j = 0; j < 16; ++j) {
        if (j < rem) {
            if (k < 5) acc |= (byte_of(w, j) & 0x7Fu) << (7 * k);
            ++k;
            if ((m >> j) & 1u) {
                vals[r] = acc;
                if (k > 5 && first + r < a.n) bad = true;
                ++r;
                acc = 0;
                k = 0;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = lane; i < in_tile; i += kWave) {
        const uint64_t g = first + i;
        if (g < a.n) gptr(a.out)[g] = vals[i];
    }
    if (a.err) {
        if (bad) *gptr(a.err) = SVB_DECODE_CORRUPT;
        if (tile == 0 && lane == 0 && *a.total < a.n) *gptr(a.err) = SVB_DECODE_CORRUPT;
    }
}

// ---------------------------------------------------------------- varint-GB decoder

// LDS offset of byte x of a tile (chunks kGbPitch apart).
__device__ __forceinline__ uint32_t gb_lds(uint32_t x) { return (x / kGbChunk) * kGbPitch + x % kGbChunk; }

// Stages bytes [base, base + len) of the stream (len a multiple of 16) at
// stage[gb_lds(0 .. len)); bytes outside the stream are unspecified.
__device__ __forceinline__ void gb_stage(const GbDecodeArgs &a, uint64_t base, uint32_t len, uint8_t *stage,
                                         uint32_t lane) {
    for (uint32_t i = lane; 16 * i < len; i += kWave) {
        const uint64_t pos = base + 16ull * i;
        if (pos < a.in_bytes) {
            const u32x4a w = load_window(a.in, a.in_bytes, pos);
            uint32_t *d = (uint32_t *)(stage + gb_lds(16 * i));
            d[0] = w.x;
            d[1] = w.y;
            d[2] = w.z;
            d[3] = w.w;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Size of a block of four integers with control byte c.
__device__ __forceinline__ uint32_t gb_block_bytes(uint32_t c) { return 1u + control_data_bytes(c, 4); }

// Chunk maps (entry e -> exit | blocks << 5) and the tile map (entry ->
// exit | blocks << 8) of one 8 KiB tile.
__global__ __launch_bounds__(kThreads) void gb_map_kernel(GbDecodeArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves][kGbLdsMap];
    __shared__ uint16_t s_map[kWaves][kWave * kGbEntries];
    const uint64_t tile = wave_index();
    if (tile >= a.tiles) return;
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint8_t *stage = s_stage[wv];
    uint16_t *map = s_map[wv];
    const uint64_t base = tile * kGbTile;
    gb_stage(a, base, kGbTile, stage, lane);
    const uint64_t cbase = base + (uint64_t)lane * kGbChunk;
    const uint8_t *chunk = stage + lane * kGbPitch;
    for (uint32_t e = 0; e < kGbEntries; ++e) {
        uint32_t p = e, cnt = 0, exit = kGbEnd;
        for (;;) {
            if (p >= kGbChunk) {
                exit = p - kGbChunk;
                break;
            }
            if (cbase + p >= a.in_bytes) break;
            p += gb_block_bytes(chunk[p]);
            ++cnt;
        }
        const uint16_t v = (uint16_t)(exit | (cnt << 5));
        map[lane * kGbEntries + e] = v;
        gptr(a.cmap)[(tile * kWave + lane) * kGbEntries + e] = v;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < kGbEntries) {
        uint32_t x = lane, cnt = 0;
        for (uint32_t c = 0; c < kWave && x != kGbEnd; ++c) {
            const uint32_t v = map[c * kGbEntries + x];
            cnt += v >> 5;
            x = v & 31u;
        }
        gptr(a.tmap)[tile * kGbEntries + lane] = x | (cnt << 8);
    }
}

// Supertile maps: 64 tile maps composed.
__global__ __launch_bounds__(kThreads) void gb_super_kernel(GbDecodeArgs a) {
    __shared__ uint32_t s_map[kWaves][kWave * kGbEntries];
    const uint64_t sup = wave_index();
    if (sup >= a.supers) return;
    const uint32_t lane = lane_id();
    uint32_t *map = s_map[threadIdx.x / kWave];
    const uint64_t t0 = sup * kWave;
    const uint32_t nt = (uint32_t)(a.tiles - t0 < kWave ? a.tiles - t0 : kWave);
    for (uint32_t i = lane; i < nt * kGbEntries; i += kWave) map[i] = a.tmap[t0 * kGbEntries + i];
    __builtin_amdgcn_wave_barrier();
    if (lane < kGbEntries) {
        uint32_t x = lane, cnt = 0;
        for (uint32_t t = 0; t < nt && x != kGbEnd; ++t) {
            const uint32_t v = map[t * kGbEntries + x];
            cnt += v >> 8;
            x = v & 31u;
        }
        gptr(a.smap)[sup * kGbEntries + lane] = x | (cnt << 8);
    }
}

// The true chain across supertiles: entry and first block index of each, and
// the number of blocks that start inside the stream.  One wave.
__global__ __launch_bounds__(kWave) void gb_top_kernel(GbDecodeArgs a) {
    __shared__ uint32_t s_map[kWave * kGbEntries];
    const uint32_t lane = lane_id();
    uint32_t x = 0;
    uint64_t blocks = 0;
    for (uint64_t s0 = 0; s0 < a.supers; s0 += kWave) {
        const uint32_t ns = (uint32_t)(a.supers - s0 < kWave ? a.supers - s0 : kWave);
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < ns * kGbEntries; i += kWave) s_map[i] = a.smap[s0 * kGbEntries + i];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            for (uint32_t s = 0; s < ns; ++s) {
                gptr(a.sentry)[s0 + s] = x;
                gptr(a.sbase)[s0 + s] = blocks;
                if (x != kGbEnd) {
                    const uint32_t v = s_map[s * kGbEntries + x];
                    blocks += v >> 8;
                    x = v & 31u;
                }
            }
        }
    }
    if (lane == 0) *gptr(a.total) = blocks;
}

// The true chain across the tiles of each supertile.
__global__ __launch_bounds__(kThreads) void gb_tiles_kernel(GbDecodeArgs a) {
    __shared__ uint32_t s_map[kWaves][kWave * kGbEntries];
    const uint64_t sup = wave_index();
    if (sup >= a.supers) return;
    const uint32_t lane = lane_id();
    uint32_t *map = s_map[threadIdx.x / kWave];
    const uint64_t t0 = sup * kWave;
    const uint32_t nt = (uint32_t)(a.tiles - t0 < kWave ? a.tiles - t0 : kWave);
    for (uint32_t i = lane; i < nt * kGbEntries; i += kWave) map[i] = a.tmap[t0 * kGbEntries + i];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        uint32_t x = a.sentry[sup];
        uint64_t blocks = a.sbase[sup];
        for (uint32_t t = 0; t < nt; ++t) {
            gptr(a.tentry)[t0 + t] = x;
            gptr(a.tbase)[t0 + t] = blocks;
            if (x != kGbEnd) {
                const uint32_t v = map[t * kGbEntries + x];
                blocks += v >> 8;
                x = v & 31u;
            }
        }
    }
}

// Decodes the blocks that start in one tile: the chain across its chunks from
// the tile's entry, then each lane decodes the blocks of its chunk.
__global__ __launch_bounds__(kThreads) void gb_decode_kernel(GbDecodeArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves][kGbLdsDecode];
    __shared__ uint16_t s_map[kWaves][kWave * kGbEntries];
    __shared__ uint32_t s_entry[kWaves][kWave], s_first[kWaves][kWave];
    const uint64_t tile = wave_index();
    if (tile >= a.tiles) return;
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint8_t *stage = s_stage[wv];
    uint16_t *map = s_map[wv];
    const uint64_t base = tile * kGbTile;
    gb_stage(a, base, kGbStage, stage, lane);
    for (uint32_t i = lane; i < kWave * kGbEntries; i += kWave) map[i] = a.cmap[tile * kWave * kGbEntries + i];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        uint32_t x = a.tentry[tile], blocks = 0;
        for (uint32_t c = 0; c < kWave; ++c) {
            s_entry[wv][c] = x;
            s_first[wv][c] = blocks;
            if (x != kGbEnd) {
                const uint32_t v = map[c * kGbEntries + x];
                blocks += v >> 5;
                x = v & 31u;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t nblocks = (a.n + 3) / 4;
    const uint64_t cbase = base + (uint64_t)lane * kGbChunk;
    uint32_t p = s_entry[wv][lane];
    uint64_t b = a.tbase[tile] + s_first[wv][lane];
    bool bad = false;
    if (p != kGbEnd) {
        while (p < kGbChunk && cbase + p < a.in_bytes && b < nblocks) {
            const uint32_t c = stage[lane * kGbPitch + p];
            const uint64_t left = a.n - 4 * b;
            const uint32_t r = left < 4 ? (uint32_t)left : 4u;
            const uint32_t size = 1u + control_data_bytes(c, r);
            if (cbase + p + size > a.in_bytes) {
                bad = true;
                break;
            }
            uint32_t v[4] = {0u, 0u, 0u, 0u};
            uint32_t q = lane * kGbChunk + p + 1;  // tile offset of the block's data
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                if (j < r) {
                    const uint32_t len = ((c >> (2 * j)) & 3u) + 1u;
                    uint32_t val = 0;
                    for (uint32_t t = 0; t < len; ++t) val |= (uint32_t)stage[gb_lds(q + t)] << (8 * t);
                    v[j] = val;
                    q += len;
                }
            }
            uint32_t *o = a.out + 4 * b;
            if (r == 4) {
                *gptr((u32x4 *)o) = u32x4{v[0], v[1], v[2], v[3]};
            } else {
                for (uint32_t j = 0; j < r; ++j) gptr(o)[j] = v[j];
            }
            p += size;
            ++b;
        }
    }
    if (a.err) {
        if (bad) *gptr(a.err) = SVB_DECODE_CORRUPT;
        if (tile == 0 && lane == 0 && *a.total < nblocks) *gptr(a.err) = SVB_DECODE_CORRUPT;
    }
}

uint32_t wave_grid(uint64_t waves) { return (uint32_t)((waves + kWaves - 1) / kWaves); }

}  // namespace

uint64_t vb_tiles(uint64_t in_bytes) { return (in_bytes + kVbTile - 1) / kVbTile; }
uint64_t gb_tiles(uint64_t in_bytes) { return (in_bytes + kGbTile - 1) / kGbTile; }
uint64_t gb_supers(uint64_t tiles) { return (tiles + kWave - 1) / kWave; }

hipError_t launch_cmp_encode(const CmpEncodeArgs &a, int fmt, bool sizes, hipStream_t s) {
    if (a.segs == 0) return hipSuccess;
    const dim3 g(wave_grid(a.segs)), b(kThreads);
    if (sizes) {
        if (fmt == kFmtVByte)
            hipLaunchKernelGGL(cmp_sizes_kernel<kFmtVByte>, g, b, 0, s, a);
        else
            hipLaunchKernelGGL(cmp_sizes_kernel<kFmtVarintGB>, g, b, 0, s, a);
    } else {
        if (fmt == kFmtVByte)
            hipLaunchKernelGGL(cmp_pack_kernel<kFmtVByte>, g, b, 0, s, a);
        else
            hipLaunchKernelGGL(cmp_pack_kernel<kFmtVarintGB>, g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_vb_decode(const VbDecodeArgs &a, bool count, hipStream_t s) {
    if (a.tiles == 0) return hipSuccess;
    const dim3 g(wave_grid(a.tiles)), b(kThreads);
    if (count)
        hipLaunchKernelGGL(vb_count_kernel, g, b, 0, s, a);
    else
        hipLaunchKernelGGL(vb_decode_kernel, g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gb_decode(const GbDecodeArgs &a, int phase, hipStream_t s) {
    if (a.tiles == 0) return hipSuccess;
    switch (phase) {
        case kGbMap: hipLaunchKernelGGL(gb_map_kernel, dim3(wave_grid(a.tiles)), dim3(kThreads), 0, s, a); break;
        case kGbSuper: hipLaunchKernelGGL(gb_super_kernel, dim3(wave_grid(a.supers)), dim3(kThreads), 0, s, a); break;
        case kGbTop: hipLaunchKernelGGL(gb_top_kernel, dim3(1), dim3(kWave), 0, s, a); break;
        case kGbTiles: hipLaunchKernelGGL(gb_tiles_kernel, dim3(wave_grid(a.supers)), dim3(kThreads), 0, s, a); break;
        default: hipLaunchKernelGGL(gb_decode_kernel, dim3(wave_grid(a.tiles)), dim3(kThreads), 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace svb
