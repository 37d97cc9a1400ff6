// Single-stream Stream VByte kernels for gfx950: decode, delta decode, encode,
// delta encode, plus a copy and a fill kernel used for measurement.
//
// Work decomposition (shared by all four codec kernels):
//  - a block is one control byte = 4 integers (Section 4);
//  - a tile is kThreads * K blocks; thread t of the workgroup owns blocks
//    t, t + 256, ..., t + 256 (K-1) of the tile, so each wave touches 64
//    consecutive control bytes and 64 consecutive 16-byte output slots;
//  - workgroups are persistent and take tiles from an atomic ticket, in
//    increasing order, which makes the decoupled look-back safe;
//  - the paper's serial "advance the data pointer by C" (Section 4) becomes an
//    exclusive scan of per-block byte counts: wave DPP scan -> LDS -> tile
//    total -> look-back over earlier tiles' status words;
//  - delta decoding (Section 2) is a second scan of the same shape over the
//    decoded values, fused into the same pass.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

// --------------------------------------------------------------------------
// shared tile prologue pieces

struct TileTicket {
    uint32_t *counters;  // [0] ticket, [1] workgroups finished
};

// Last workgroup to leave resets the ticket so the next launch starts at 0.
__device__ __forceinline__ void retire_workgroup(uint32_t *counters) {
    if (threadIdx.x == 0) {
        const uint32_t done = atomicAdd(counters + 1, 1u);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(counters + 0, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(counters + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Exclusive scan over the tile's K x 256 per-block byte counts in block order
// (step k, then wave, then lane).  Returns the tile total; pre[k] + x[k] is the
// block's offset inside the tile.
template <int K>
__device__ __forceinline__ uint32_t tile_scan(const uint32_t (&v)[K], uint32_t (&x)[K],
                                              uint32_t (&pre)[K], uint32_t *s_tot) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t incl = wave_incl_scan(v[k]);
        x[k] = incl - v[k];
        if (lane == kWave - 1) s_tot[k * kWaves + wave] = incl;
    }
    __syncthreads();
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = s_tot[k * kWaves + w];
            if ((uint32_t)w == wave) pre[k] = run;
            run += t;
        }
    }
    return run;
}

// Publish this tile's aggregate, look back, publish the inclusive prefix.
// Run by wave 0; returns the tile's exclusive prefix in every lane of wave 0.
template <int VB>
__device__ __forceinline__ uint64_t tile_prefix(uint64_t *flags, uint32_t tile, uint32_t epoch,
                                                uint64_t total) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (tile == 0) {
        if (lane == 0) flag_publish<VB>(flags, 0, epoch, kInclusive, total);
        return 0;
    }
    if (lane == 0) flag_publish<VB>(flags, tile, epoch, kAggregate, total);
    const uint64_t excl = lookback<VB>(flags, tile, epoch);
    if (lane == 0) flag_publish<VB>(flags, tile, epoch, kInclusive, excl + total);
    return excl;
}

constexpr int kByteBits = 42;   // byte prefixes: up to 4 TiB
constexpr int kValueBits = 32;  // delta values: modulo 2^32

// --------------------------------------------------------------------------
// decode

template <int K, bool DELTA>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs p) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_btot[K * kWaves];
    __shared__ uint32_t s_vtot[K * kWaves];
    __shared__ uint64_t s_bbase;
    __shared__ uint32_t s_vcarry;

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / kWave;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(p.counters, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= p.num_tiles) break;
        const uint64_t b0 = (uint64_t)tile * (kThreads * K) + tid;

        // control bytes -> per-block data byte counts (Section 4: C in [4, 16])
        uint32_t c[K], r[K], nb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t b = b0 + (uint64_t)k * kThreads;
            r[k] = (b < nblocks) ? ((b == nblocks - 1) ? last_r : 4u) : 0u;
            c[k] = r[k] ? (uint32_t)p.in[b] : 0u;
            nb[k] = control_data_bytes(c[k], r[k]);
        }

        // byte offsets: scan inside the tile, look back across tiles
        uint32_t bx[K], bpre[K];
        const uint32_t tile_bytes = tile_scan<K>(nb, bx, bpre, s_btot);
        if (wave == 0) {
            const uint64_t e = tile_prefix<kByteBits>(p.byte_flags, tile, p.epoch, tile_bytes);
            if (tid == 0) s_bbase = e;
        }
        __syncthreads();
        const uint64_t data0 = nblocks + s_bbase;

        // gather each block's four integers from its 16-byte window
        uint32_t v[K][4];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k][0] = v[k][1] = v[k][2] = v[k][3] = 0u;
            if (r[k]) {
                const uint64_t a = data0 + bpre[k] + bx[k];
                if (a + nb[k] > p.in_bytes) {
                    bad = true;
                } else {
                    uint32_t d0, d1, d2, d3;
                    load_window16(p.in, a, p.in_bytes, d0, d1, d2, d3);
                    gather_block(c[k], d0, d1, d2, d3, v[k][0], v[k][1], v[k][2], v[k][3]);
                    if (r[k] < 4) {
                        if (r[k] < 2) v[k][1] = 0u;
                        if (r[k] < 3) v[k][2] = 0u;
                        v[k][3] = 0u;
                    }
                }
            }
        }
        if (bad && p.err) *p.err = SVB_DECODE_CORRUPT;

        if (DELTA) {
            // running sum modulo 2^32 (Section 2): inside the block, then across
            // blocks of the tile, then across tiles
            uint32_t bs[K], vx[K], vpre[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                v[k][1] += v[k][0];
                v[k][2] += v[k][1];
                v[k][3] += v[k][2];
                bs[k] = v[k][3];
            }
            const uint32_t tile_sum = tile_scan<K>(bs, vx, vpre, s_vtot);
            if (wave == 0) {
                const uint64_t e = tile_prefix<kValueBits>(p.val_flags, tile, p.epoch, tile_sum);
                if (tid == 0) s_vcarry = (uint32_t)e;
            }
            __syncthreads();
            const uint32_t base = p.start + s_vcarry;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t add = base + vpre[k] + vx[k];
                v[k][0] += add;
                v[k][1] += add;
                v[k][2] += add;
                v[k][3] += add;
            }
        }

#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t b = b0 + (uint64_t)k * kThreads;
            uint32_t *o = p.out + 4 * b;
            if (r[k] == 4) {
                *(u32x4 *)o = u32x4{v[k][0], v[k][1], v[k][2], v[k][3]};
            } else if (r[k]) {
                o[0] = v[k][0];
                if (r[k] > 1) o[1] = v[k][1];
                if (r[k] > 2) o[2] = v[k][2];
            }
        }
        __syncthreads();  // LDS words are reused by the next tile
    }
    retire_workgroup(p.counters);
}

// --------------------------------------------------------------------------
// encode

template <int K, bool DELTA>
__global__ __launch_bounds__(kThreads) void encode_kernel(EncodeArgs p) {
    constexpr uint32_t kStageWords = (kThreads * K * 16 + 32) / 4;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_btot[K * kWaves];
    __shared__ uint64_t s_bbase;
    __shared__ __attribute__((aligned(16))) uint32_t s_stage[kStageWords];

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / kWave;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(p.counters, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= p.num_tiles) break;
        const uint64_t b0 = (uint64_t)tile * (kThreads * K) + tid;

        // values (or deltas, Section 2) -> byte lengths (Section 3) -> control byte
        uint32_t v[K][4], r[K], c[K], nb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t b = b0 + (uint64_t)k * kThreads;
            r[k] = (b < nblocks) ? ((b == nblocks - 1) ? last_r : 4u) : 0u;
            uint32_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
            const uint32_t *src = p.in + 4 * b;
            if (r[k] == 4) {
                const u32x4 w = *(const u32x4 *)src;
                x0 = w.x; x1 = w.y; x2 = w.z; x3 = w.w;
            } else if (r[k]) {
                x0 = src[0];
                if (r[k] > 1) x1 = src[1];
                if (r[k] > 2) x2 = src[2];
            }
            if (DELTA && r[k]) {
                const uint32_t prev = (b == 0) ? p.start : src[-1];
                v[k][0] = x0 - prev;
                v[k][1] = x1 - x0;
                v[k][2] = x2 - x1;
                v[k][3] = x3 - x2;
            } else {
                v[k][0] = x0; v[k][1] = x1; v[k][2] = x2; v[k][3] = x3;
            }
            uint32_t ctrl = 0, bytes = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t L = byte_length(v[k][j]);
                const bool used = (uint32_t)j < r[k];
                ctrl |= used ? ((L - 1u) << (2 * j)) : 0u;
                bytes += used ? L : 0u;
            }
            c[k] = ctrl;
            nb[k] = bytes;
            if (r[k]) p.out[b] = (uint8_t)ctrl;
        }

        uint32_t bx[K], bpre[K];
        const uint32_t tile_bytes = tile_scan<K>(nb, bx, bpre, s_btot);
        if (wave == 0) {
            const uint64_t e = tile_prefix<kByteBits>(p.byte_flags, tile, p.epoch, tile_bytes);
            if (tid == 0) s_bbase = e;
        }
        __syncthreads();

        // The tile's data bytes go to out[g0, g0 + tile_bytes).  They are packed
        // into LDS laid out like the 16-byte-aligned global span that holds them,
        // then written with full 16-byte stores inside and byte stores at the two
        // edges, which other tiles share.
        const uint64_t g0 = nblocks + s_bbase;
        const uintptr_t gabs = (uintptr_t)p.out + g0;
        const uintptr_t gal = gabs & ~(uintptr_t)15;
        const uint32_t sh = (uint32_t)(gabs - gal);
        const uint32_t span = sh + tile_bytes;
        const uint32_t nwords = (span + 7) / 4;
        for (uint32_t i = tid; i < nwords; i += kThreads) s_stage[i] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!r[k]) continue;
            uint32_t pos = sh + bpre[k] + bx[k];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((uint32_t)j >= r[k]) break;
                const uint32_t L = ((c[k] >> (2 * j)) & 3u) + 1u;
                const uint32_t val = v[k][j];
                const uint32_t w = pos >> 2, s = pos & 3u;
                atomicOr(&s_stage[w], val << (8u * s));
                if (s + L > 4u) atomicOr(&s_stage[w + 1], val >> (32u - 8u * s));
                pos += L;
            }
        }
        __syncthreads();
        const uint32_t nchunks = (span + 15) / 16;
        for (uint32_t ch = tid; ch < nchunks; ch += kThreads) {
            const uint32_t lo = ch * 16, hi = lo + 16;
            uint8_t *dst = (uint8_t *)gal;
            if (lo >= sh && hi <= span) {
                *(u32x4a *)(dst + lo) = *(const u32x4a *)(&s_stage[lo / 4]);
            } else {
                const uint32_t from = lo > sh ? lo : sh;
                const uint32_t to = hi < span ? hi : span;
                for (uint32_t i = from; i < to; ++i)
                    dst[i] = (uint8_t)(s_stage[i >> 2] >> (8u * (i & 3u)));
            }
        }
        if (tile == p.num_tiles - 1 && tid == 0 && p.out_bytes) *p.out_bytes = g0 + tile_bytes;
        __syncthreads();
    }
    retire_workgroup(p.counters);
}

// --------------------------------------------------------------------------
// measurement kernels

__global__ __launch_bounds__(kThreads) void copy_kernel(const uint32_t *in, uint32_t *out, uint64_t n) {
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
        *(u32x4 *)(out + 4 * i) = *(const u32x4 *)(in + 4 * i);
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

template <typename Kern, typename Args>
static hipError_t launch_persistent(Kern kern, const Args &a, uint32_t num_tiles, hipStream_t s) {
    const uint32_t grid = persistent_grid((const void *)kern, num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs &a, bool delta, hipStream_t s) {
    if (delta) return launch_persistent(decode_kernel<kBlocksPerThread, true>, a, a.num_tiles, s);
    return launch_persistent(decode_kernel<kBlocksPerThread, false>, a, a.num_tiles, s);
}

hipError_t launch_encode(const EncodeArgs &a, bool delta, hipStream_t s) {
    if (delta) return launch_persistent(encode_kernel<kBlocksPerThread, true>, a, a.num_tiles, s);
    return launch_persistent(encode_kernel<kBlocksPerThread, false>, a, a.num_tiles, s);
}

hipError_t launch_copy(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s) {
    const uint64_t want = (n / 4 + kThreads - 1) / kThreads;
    const uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
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
