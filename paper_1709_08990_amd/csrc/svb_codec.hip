// Single-stream Stream VByte kernels for gfx950: decode, delta decode, encode,
// delta encode, plus a copy and a fill kernel used for measurement.
//
// Work decomposition (shared by all four codec kernels):
//  - a block is one control byte = 4 integers (Section 4);
//  - a tile is kThreads * K blocks; thread t of the workgroup owns blocks
//    t, t + 256, ..., t + 256 (K-1) of the tile, so each wave touches 64
//    consecutive control bytes and 64 consecutive 16-byte output slots;
//  - workgroups are persistent and take tiles from per-class atomic tickets
//    in increasing order, which makes the decoupled look-back safe;
//  - the paper's serial "advance the data pointer by C" (Section 4) becomes an
//    exclusive scan of per-block byte counts: wave DPP scan -> LDS -> tile
//    total -> tile offset.  Decoding takes tile offsets from a pre-pass over
//    the control stream; encoding chains them with a look-back over earlier
//    tiles' status words;
//  - delta decoding (Section 2) is a second scan of the same shape over the
//    decoded values, chained across tiles by a look-back in the same pass.
#include "svb_device.hpp"
#include "svb_internal.hpp"

namespace svb {

// --------------------------------------------------------------------------
// shared tile prologue pieces

// Next tile for this workgroup (>= q.num_tiles once its class has none left).
// Each class's tiles are handed out in increasing order to running workgroups,
// so a tile's predecessors are always held by workgroups that make progress.
__device__ __forceinline__ uint32_t take_tile(const TileQueue &q) {
    const uint32_t cls = blockIdx.x % q.classes;
    const uint32_t j = atomicAdd(q.counters + cls * kCounterStride, 1u) - q.base[cls];
    return j * q.classes + cls;
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
// Run by one full wave; returns the tile's exclusive prefix in all its lanes.
template <int VB>
__device__ __forceinline__ uint64_t tile_prefix(uint64_t *flags, uint32_t tile, uint32_t epoch,
                                                uint64_t total) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t excl = lookback<VB>(flags, tile, epoch, total);
    if (lane == 0) flag_publish<VB>(flags, tile, epoch, kInclusive, excl + total);
    return excl;
}

// Control bytes of the K blocks lane `lane` owns in sub-tile `sub` (a wave's
// 64 x K consecutive blocks; lane l takes blocks l, l + 64, ...), none past the
// end of the stream or when sub >= num_subs.
template <int K>
__device__ __forceinline__ void load_sub_control(const uint8_t *in, uint64_t n, uint64_t sub,
                                                 uint64_t num_subs, uint32_t lane, uint32_t (&c)[K]) {
    const uint64_t nblocks = (n + 3) >> 2;
    const uint64_t b0 = sub * (kWave * K) + lane;
    if (sub < num_subs && (sub + 1) * (kWave * K * 4) <= n) {
#pragma unroll
        for (int k = 0; k < K; ++k) c[k] = in[b0 + (uint64_t)k * kWave];
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t b = b0 + (uint64_t)k * kWave;
            c[k] = (sub < num_subs && b < nblocks) ? (uint32_t)in[b] : 0u;
        }
    }
}

constexpr int kByteBits = 42;   // byte prefixes: up to 4 TiB
constexpr int kValueBits = 32;  // delta values: modulo 2^32

// --------------------------------------------------------------------------
// decoding: reduce, then scan, then decode
//
// The paper's decoder advances its data pointer by C bytes after every control
// byte (Section 4) and, for differential coding, carries a running sum
// (Section 2).  Both are prefix sums; here they are computed without any chain
// between workgroups:
//   1. control_reduce_kernel: per sub-tile byte offset inside its super-tile,
//      and each super-tile's byte total (reads the control stream only);
//   2. scan_kernel: exclusive scan of the super-tile totals (one workgroup);
//   3. (delta only) decode_kernel<SUMS>: decodes without storing and writes each
//      tile's value sum and each sub-tile's value offset inside its tile;
//   4. (delta only) scan_kernel over the tile sums;
//   5. decode_kernel<PLAIN|DELTA>: decodes every sub-tile at its byte offset,
//      adds the value carry, stores.
// Sizes: a sub-tile is one wave's 64 x K blocks, a tile four sub-tiles, a
// super-tile 256 threads x 64 blocks = kSubsPerSuper sub-tiles.

template <int K>
__global__ __launch_bounds__(kThreads) void control_reduce_kernel(ReduceArgs p) {
    __shared__ uint32_t s_wtot[kWaves];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;
    for (uint64_t sup = blockIdx.x; sup < p.num_supers; sup += gridDim.x) {
        const uint64_t first = sup * (kThreads * 64) + (uint64_t)tid * 64;  // first block of this thread
        uint32_t bytes = 0;
        if (first >= 4 && first + 64 < nblocks && first + 68 <= p.in_bytes) {
            // 64 whole blocks, none of them the last: 256 + the sum of all codes
            const uint8_t *pa = p.in + first;
            const uint32_t sh = (uint32_t)((uintptr_t)pa & 3u);
            const uint8_t *base = pa - sh;
            u32x4 w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = *(const u32x4 *)(base + 16 * i);
            const uint32_t w16 = *(const uint32_t *)(base + 64);
            const uint32_t d[17] = {w[0].x, w[0].y, w[0].z, w[0].w, w[1].x, w[1].y, w[1].z, w[1].w,
                                    w[2].x, w[2].y, w[2].z, w[2].w, w[3].x, w[3].y, w[3].z, w[3].w, w16};
            uint32_t codes = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t x = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
                codes += __builtin_popcount(x & 0x55555555u) + 2u * __builtin_popcount(x & 0xAAAAAAAAu);
            }
            bytes = 256u + codes;
        } else {
            for (uint32_t i = 0; i < 64; ++i) {
                const uint64_t b = first + i;
                if (b >= nblocks) break;
                bytes += control_data_bytes(p.in[b], (b == nblocks - 1) ? last_r : 4u);
            }
        }
        const uint32_t incl = wave_incl_scan(bytes);
        if (lane == kWave - 1) s_wtot[wave] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = s_wtot[w];
            if ((uint32_t)w < wave) before += t;
            total += t;
        }
        if (tid % K == 0) {
            const uint64_t sub = (sup * kThreads + tid) / K;
            if (sub < p.num_subs) p.sub_loc[sub] = before + incl - bytes;
        }
        if (tid == 0) p.sup_bytes[sup] = total;
        __syncthreads();
    }
}

// Exclusive prefix sums of m uint32 values by one workgroup of 1024 threads,
// 16384 values per step.  WIDE: 64-bit sums (byte offsets); otherwise modulo
// 2^32 (delta values).
template <bool WIDE>
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *in, void *out, uint64_t m) {
    constexpr int kT = 1024, kPer = 16, kW = kT / kWave;
    __shared__ uint32_t s_wtot[kW];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < m; base += (uint64_t)kT * kPer) {
        uint32_t x[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = base + (uint64_t)tid * kPer + j;
            x[j] = i < m ? in[i] : 0u;
            sum += x[j];
        }
        const uint32_t incl = wave_incl_scan(sum);
        if (lane == kWave - 1) s_wtot[wave] = incl;
        __syncthreads();
        uint32_t before = 0;
        if (wave == 0) {
            const uint32_t t = lane < kW ? s_wtot[lane] : 0u;
            const uint32_t ti = wave_incl_scan(t);
            if (lane < kW) s_wtot[lane] = ti - t;
            if (lane == kWave - 1) s_total = ti;
        }
        __syncthreads();
        before = s_wtot[wave] + incl - sum;
        uint32_t run = before;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t i = base + (uint64_t)tid * kPer + j;
            if (i < m) {
                if (WIDE)
                    ((uint64_t *)out)[i] = carry + run;
                else
                    ((uint32_t *)out)[i] = (uint32_t)carry + run;
            }
            run += x[j];
        }
        carry += s_total;
        __syncthreads();
    }
}

// One wave's sub-tile.  issue_sub plans the sub-tile from its control bytes
// (byte counts, offsets) and, for an interior sub-tile -- every 20-byte
// window inside the buffer -- requests all its windows at once; gather_sub
// later turns them into integers.  Sub-tiles at the edges of the stream take
// a checked byte-by-byte path in gather_sub instead.
template <int K>
struct SubLoads {
    Window win[K];
    uint32_t r[K];
    uint64_t soff;
    bool interior;
};

template <int K>
__device__ __forceinline__ void plan_blocks(const DecodeArgs &p, uint64_t sub, const uint32_t (&c)[K],
                                            uint32_t (&r)[K], uint32_t (&nb)[K], uint32_t (&off)[K],
                                            uint32_t &total) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint32_t last_r = (p.n & 3) ? (uint32_t)(p.n & 3) : 4u;
    const uint64_t b0 = sub * (kWave * K) + lane;
    const bool full = (sub + 1) * (kWave * K * 4) <= p.n;
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t b = b0 + (uint64_t)k * kWave;
        r[k] = full ? 4u : ((b < nblocks) ? ((b == nblocks - 1) ? last_r : 4u) : 0u);
        nb[k] = control_data_bytes(c[k], r[k]);
        const uint32_t incl = wave_incl_scan(nb[k]);
        off[k] = run + incl - nb[k];
        run += wave_last(incl);
    }
    total = run;
}

template <int K>
__device__ __forceinline__ void issue_sub(const DecodeArgs &p, uint64_t sub, const uint32_t (&c)[K],
                                          uint64_t soff, SubLoads<K> &sl) {
    uint32_t nb[K], off[K], total;
    plan_blocks<K>(p, sub, c, sl.r, nb, off, total);
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint64_t data0 = nblocks + soff;
    const bool full = (sub + 1) * (kWave * K * 4) <= p.n;
    sl.soff = soff;
    sl.interior = full && data0 >= 3 && data0 + total + 20 <= p.in_bytes;
    if (sl.interior) {
#pragma unroll
        for (int k = 0; k < K; ++k) sl.win[k] = load_window(p.in, data0 + off[k]);
    }
}

// Returns false if the sub-tile's data runs past in_bytes (corrupt stream).
template <int K>
__device__ __forceinline__ bool gather_sub(const DecodeArgs &p, uint64_t sub, const uint32_t (&c)[K],
                                           const SubLoads<K> &sl, uint32_t (&v)[K][4]) {
    if (sl.interior) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            uint32_t d0, d1, d2, d3;
            align_window(sl.win[k], d0, d1, d2, d3);
            gather_block(c[k], d0, d1, d2, d3, v[k][0], v[k][1], v[k][2], v[k][3]);
        }
        return true;
    }
    uint32_t r[K], nb[K], off[K], total;
    plan_blocks<K>(p, sub, c, r, nb, off, total);
    const uint64_t data0 = ((p.n + 3) >> 2) + sl.soff;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k][0] = v[k][1] = v[k][2] = v[k][3] = 0u;
        if (r[k]) {
            const uint64_t a = data0 + off[k];
            if (a + nb[k] > p.in_bytes) {
                ok = false;
            } else {
                uint32_t d0, d1, d2, d3;
                load_window16_checked(p.in, a, p.in_bytes, d0, d1, d2, d3);
                gather_block(c[k], d0, d1, d2, d3, v[k][0], v[k][1], v[k][2], v[k][3]);
                if (r[k] < 4) {
                    if (r[k] < 2) v[k][1] = 0u;
                    if (r[k] < 3) v[k][2] = 0u;
                    v[k][3] = 0u;
                }
            }
        }
    }
    return ok;
}

template <int K>
__device__ __forceinline__ void store_sub(uint32_t *out, uint64_t sub, const uint32_t (&r)[K],
                                          const uint32_t (&v)[K][4]) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t b0 = sub * (kWave * K) + lane;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint32_t *o = out + 4 * (b0 + (uint64_t)k * kWave);
        if (r[k] == 4) {
            __builtin_nontemporal_store(u32x4{v[k][0], v[k][1], v[k][2], v[k][3]}, (u32x4 *)o);
        } else if (r[k]) {
            o[0] = v[k][0];
            if (r[k] > 1) o[1] = v[k][1];
            if (r[k] > 2) o[2] = v[k][2];
        }
    }
}

// Byte offset of sub-tile `sub` in the data stream, and (delta) its value carry.
__device__ __forceinline__ uint64_t sub_offset(const DecodeArgs &p, uint64_t sub) {
    return p.sup_off[sub / kSubsPerSuper] + p.sub_loc[sub];
}

// Everything a wave requests for a sub-tile one iteration before planning it.
template <int K>
struct SubAhead {
    uint32_t c[K];
    uint64_t soff;
    uint32_t carry;
};

template <int K, int MODE>
__device__ __forceinline__ void request_sub(const DecodeArgs &p, uint32_t tile, uint32_t T, SubAhead<K> &a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t sub = (uint64_t)tile * kWaves + wave;
    load_sub_control<K>(p.in, p.n, sub, p.num_subs, lane, a.c);
    const bool have = tile < T && sub < p.num_subs;
    a.soff = have ? sub_offset(p, sub) : 0;
    a.carry = (MODE == 1 && have) ? p.start + p.tile_vpre[tile] + p.sub_vloc[sub] : 0u;
}

// The decoder.  Four data waves per workgroup, one sub-tile each per tile,
// software-pipelined over three tiles: in the iteration that gathers tile i,
// a wave first requests the control bytes and offsets of tile i+2, then plans
// tile i+1 and requests its data windows, and only then waits for tile i's
// windows.  Vector memory loads retire in issue order, so this keeps two tiles
// of data windows in flight per wave; stores go last.  Tiles come from the
// class tickets, three ahead.
//   PLAIN: store the integers.
//   DELTA: store their running sum (Section 2): inside each block, over the
//          wave's blocks, plus the carry from the scans (start + tile prefix +
//          sub-tile offset inside the tile).
//   SUMS:  store nothing; write the tile's value sum and each sub-tile's value
//          offset inside the tile (input of the value scan).
enum DecodeMode { kPlain = 0, kDelta = 1, kSums = 2 };

template <int K, int MODE>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs p) {
    __shared__ uint32_t s_tiles[4];  // tile of iteration j at j % 4
    __shared__ uint32_t s_sums[2][kWaves];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint32_t T = p.q.num_tiles;
    const uint64_t S = p.num_subs;

    if (tid == 0) {
        s_tiles[0] = take_tile(p.q);
        s_tiles[1] = take_tile(p.q);
        s_tiles[2] = take_tile(p.q);
    }
    __syncthreads();
    uint32_t t0 = s_tiles[0], t1 = s_tiles[1], t2 = s_tiles[2];
    SubAhead<K> a0, a1, a2;
    request_sub<K, MODE>(p, t0, T, a0);
    request_sub<K, MODE>(p, t1, T, a1);
    SubLoads<K> l0, l1;
    issue_sub<K>(p, (uint64_t)t0 * kWaves + wave, a0.c, a0.soff, l0);
    uint32_t it = 0;

    while (t0 < T) {
        // 1. tile i+2: control bytes and offsets; the ticket of tile i+3
        request_sub<K, MODE>(p, t2, T, a2);
        uint32_t ticket = 0;
        if (tid == 0) ticket = take_tile(p.q);
        // 2. tile i+1: plan, request its windows
        issue_sub<K>(p, (uint64_t)t1 * kWaves + wave, a1.c, a1.soff, l1);
        // 3. tile i: gather
        const uint64_t sub = (uint64_t)t0 * kWaves + wave;
        uint32_t v[K][4];
        const bool ok = gather_sub<K>(p, sub, a0.c, l0, v);
        if (!ok && p.err) *p.err = SVB_DECODE_CORRUPT;

        if (MODE == kPlain) {
            store_sub<K>(p.out, sub, l0.r, v);
        } else if (MODE == kDelta) {
            uint32_t run = a0.carry;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                v[k][1] += v[k][0];
                v[k][2] += v[k][1];
                v[k][3] += v[k][2];
                const uint32_t incl = wave_incl_scan(v[k][3]);
                const uint32_t add = run + incl - v[k][3];
                run += wave_last(incl);
#pragma unroll
                for (int j = 0; j < 4; ++j) v[k][j] += add;
            }
            store_sub<K>(p.out, sub, l0.r, v);
        } else {
            uint32_t sum = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) sum += v[k][0] + v[k][1] + v[k][2] + v[k][3];
            sum = wave_last(wave_incl_scan(sum));
            if (lane == 0) s_sums[it & 1][wave] = sum;
        }
        if (tid == 0) s_tiles[(it + 3) & 3] = ticket;
        __syncthreads();
        if (MODE == kSums && wave == 0 && lane < kWaves) {
            uint32_t before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t x = s_sums[it & 1][w];
                if ((uint32_t)w < lane) before += x;
                total += x;
            }
            const uint64_t my = (uint64_t)t0 * kWaves + lane;
            if (my < S) p.sub_vloc[my] = before;
            if (lane == 0) p.tile_sum[t0] = total;
        }
        t0 = t1;
        t1 = t2;
        t2 = s_tiles[(it + 3) & 3];
        a0 = a1;
        a1 = a2;
        l0 = l1;
        ++it;
    }
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

uint32_t decode_grid(int mode, uint32_t num_tiles) {
    const void *k = mode == kPlain ? (const void *)decode_kernel<kBlocksPerThread, kPlain>
                  : mode == kDelta ? (const void *)decode_kernel<kBlocksPerThread, kDelta>
                                   : (const void *)decode_kernel<kBlocksPerThread, kSums>;
    return persistent_grid(k, num_tiles, kThreads);
}

uint32_t encode_grid(bool delta, uint32_t num_tiles) {
    return delta ? persistent_grid((const void *)encode_kernel<kBlocksPerThread, true>, num_tiles, kThreads)
                 : persistent_grid((const void *)encode_kernel<kBlocksPerThread, false>, num_tiles, kThreads);
}

hipError_t launch_control_reduce(const ReduceArgs &a, hipStream_t s) {
    const uint64_t want = a.num_supers;
    const uint32_t grid = (uint32_t)(want > 65536 ? 65536 : (want < 1 ? 1 : want));
    hipLaunchKernelGGL((control_reduce_kernel<kBlocksPerThread>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *in, void *out, uint64_t m, bool wide, hipStream_t s) {
    if (wide)
        hipLaunchKernelGGL((scan_kernel<true>), dim3(1), dim3(1024), 0, s, in, out, m);
    else
        hipLaunchKernelGGL((scan_kernel<false>), dim3(1), dim3(1024), 0, s, in, out, m);
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs &a, int mode, uint32_t grid, hipStream_t s) {
    if (mode == kPlain)
        hipLaunchKernelGGL((decode_kernel<kBlocksPerThread, kPlain>), dim3(grid), dim3(kThreads), 0, s, a);
    else if (mode == kDelta)
        hipLaunchKernelGGL((decode_kernel<kBlocksPerThread, kDelta>), dim3(grid), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((decode_kernel<kBlocksPerThread, kSums>), dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
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
