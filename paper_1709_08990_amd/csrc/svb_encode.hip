// Stream VByte encoding for gfx950 (plain and delta), plus a copy and a fill
// kernel used for measurement.
//
// Work decomposition:
//  - a block is one control byte = 4 integers (Section 4);
//  - a tile is kThreads * K blocks; thread t of the workgroup owns blocks
//    t, t + 256, ..., t + 256 (K-1) of the tile;
//  - workgroups are persistent and take tiles from per-class atomic tickets
//    in increasing order, which makes the decoupled look-back safe;
//  - where the paper's encoder appends each integer's bytes after the
//    previous ones, here a tile's byte offset is the exclusive scan of the
//    byte counts of all earlier tiles, chained by a look-back over their
//    status words; inside the tile it is a workgroup scan.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

// --------------------------------------------------------------------------
// shared tile prologue pieces

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
// Run by one full wave; returns the tile's exclusive prefix in all its lanes
// (0, with `stalled` set, if the look-back gave up).
template <int VB>
__device__ __forceinline__ uint64_t tile_prefix(uint64_t *flags, uint32_t tile, uint32_t epoch,
                                                uint64_t total, bool &stalled) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t excl = lookback<VB>(flags, tile, epoch, total, stalled);
    if (lane == 0) flag_publish<VB>(flags, tile, epoch, kInclusive, excl + total);
    return excl;
}

constexpr int kByteBits = 42;  // byte prefixes: up to 4 TiB

// --------------------------------------------------------------------------
// encode

template <int K, bool DELTA>
__global__ __launch_bounds__(kThreads) void encode_kernel(EncodeArgs p) {
    constexpr uint32_t kStageWords = (kThreads * K * 16 + 32) / 4;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_btot[K * kWaves];
    __shared__ uint64_t s_bbase;
    __shared__ uint32_t s_stalled;
    __shared__ __attribute__((aligned(16))) uint32_t s_stage[kStageWords];

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / kWave;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;

    for (;;) {
        if (tid == 0) s_tile = take_tile(p.q);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= p.q.num_tiles) break;
        const uint64_t b0 = (uint64_t)tile * (kThreads * K) + tid;
        // the staging words are cleared while the inputs are in flight
        for (uint32_t i = tid; i < kStageWords; i += kThreads) s_stage[i] = 0u;

        // values (or deltas, Section 2) -> byte lengths (Section 3) -> control byte
        const bool full = (uint64_t)(tile + 1) * (kThreads * K * 4) <= p.n;
        uint32_t v[K][4], r[K], c[K], nb[K];
        if (full) {
            // all loads at once: the four values of each block and, for delta
            // coding, the value before the block (index clamped at 0)
            u32x4 w[K];
            uint32_t prev[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t b = b0 + (uint64_t)k * kThreads;
                w[k] = *(const u32x4 *)(p.in + 4 * b);
                if (DELTA) prev[k] = p.in[b ? 4 * b - 1 : 0];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the first use
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t b = b0 + (uint64_t)k * kThreads;
                r[k] = 4u;
                if (DELTA) {
                    const uint32_t pv = b ? prev[k] : p.start;
                    v[k][0] = w[k].x - pv;
                    v[k][1] = w[k].y - w[k].x;
                    v[k][2] = w[k].z - w[k].y;
                    v[k][3] = w[k].w - w[k].z;
                } else {
                    v[k][0] = w[k].x; v[k][1] = w[k].y; v[k][2] = w[k].z; v[k][3] = w[k].w;
                }
            }
        } else {
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
                    const uint32_t pv = (b == 0) ? p.start : src[-1];
                    v[k][0] = x0 - pv;
                    v[k][1] = x1 - x0;
                    v[k][2] = x2 - x1;
                    v[k][3] = x3 - x2;
                } else {
                    v[k][0] = x0; v[k][1] = x1; v[k][2] = x2; v[k][3] = x3;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
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
        }

        uint32_t bx[K], bpre[K];
        const uint32_t tile_bytes = tile_scan<K>(nb, bx, bpre, s_btot);
        if (wave == 0) {
            bool stalled;
            const uint64_t e = tile_prefix<kByteBits>(p.byte_flags, tile, p.epoch, tile_bytes, stalled);
            if (tid == 0) {
                s_bbase = e;
                s_stalled = stalled;
            }
        }
        __syncthreads();
        if (s_stalled) {
            // the tile's offset is unknown: write nothing, report the stall
            if (tid == 0 && p.out_bytes) *p.out_bytes = ~0ull;
            __syncthreads();
            continue;
        }

        // The tile's data bytes go to out[g0, g0 + tile_bytes).  They are packed
        // into LDS laid out like the 16-byte-aligned global span that holds them,
        // then written with full 16-byte stores inside and byte stores at the two
        // edges, which other tiles share.
        const uint64_t g0 = nblocks + s_bbase;
        const uintptr_t gabs = (uintptr_t)p.out + g0;
        const uintptr_t gal = gabs & ~(uintptr_t)15;
        const uint32_t sh = (uint32_t)(gabs - gal);
        const uint32_t span = sh + tile_bytes;
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
        // control bytes, then the data bytes of the tile
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r[k]) p.out[b0 + (uint64_t)k * kThreads] = (uint8_t)c[k];
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
        if (tile == p.q.num_tiles - 1 && tid == 0 && p.out_bytes) *p.out_bytes = g0 + tile_bytes;
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// measurement kernels

// Streaming copy with nontemporal 16-byte loads and stores: the practical
// HBM ceiling the codec kernels are compared with, and the reference that
// scales the hardware byte counters (it moves exactly 4n bytes each way).
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

uint32_t encode_grid(bool delta, uint32_t num_tiles) {
    return delta ? persistent_grid((const void *)encode_kernel<kBlocksPerThread, true>, num_tiles, kThreads)
                 : persistent_grid((const void *)encode_kernel<kBlocksPerThread, false>, num_tiles, kThreads);
}

hipError_t launch_encode(const EncodeArgs &a, bool delta, uint32_t grid, hipStream_t s) {
    if (delta)
        hipLaunchKernelGGL((encode_kernel<kBlocksPerThread, true>), dim3(grid), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((encode_kernel<kBlocksPerThread, false>), dim3(grid), dim3(kThreads), 0, s, a);
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
