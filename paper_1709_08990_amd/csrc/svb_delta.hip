// Value sums of the delta decoder for gfx950: the running sum of Section 2
// over the decoder of Section 4.
//
// Differential coding stores x_i - x_{i-1}; decoding is a running sum over the
// decoded differences, started from `start`.  The decoder of Section 4 keeps
// that sum in a register while it walks the stream; here every wave decodes
// its own group of kGroupInts integers at the same time, so each wave needs the
// sum of every difference stored before its group (its carry).  The delta
// decode therefore runs in two passes: every group's sum of stored
// differences, a device scan of the sums from `start`, then the decode pass
// (svb_decode.hip), each group starting from its carry.
//
// Sum of a group's values without decoding them.  A value of L bytes is
// sum_k byte_k 256^k, so the sum of the values is the plain sum of all the
// group's data bytes plus, for each integer of L >= 2 bytes, its value minus
// the sum of its bytes.  The plain byte sum needs no integer boundaries: it is
// a sum over the group's contiguous data span (four SAD instructions per 16
// bytes).  The corrections are needed only for blocks whose control byte is
// not zero (a zero control byte stands for four one-byte integers): on
// document-id gaps (mostly one-byte differences) about 4 % of the blocks.  The
// group's span is known before any load (its offset and the next group's come
// from the scan of the group byte counts), so the control bytes and the whole
// span are requested together, one round trip to memory; the span is staged
// in LDS as it is summed, and the corrections read their blocks from there (a
// block past the staging area, only in a group of long integers, takes its
// two aligned chunks from memory).  About half the instructions of decoding
// the group, and few enough registers for eight waves per SIMD.  Streams of
// long integers (more than about 1.1 bytes per integer on average), where
// nearly every block needs a correction, take their sums by decoding
// (decode_kernel<kSums>) instead.
//
// One-pass schedules were built and measured slower on this chip (see the
// design notes): a chained scan across groups advances one window of groups
// per device-scope round trip; a tree of block sums filled by atomics waits
// for the slowest sum before each group; and taking the sums a generation of
// workgroups ahead of the decode puts their memory latency into every
// decoding wave's lifetime.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

namespace {

static_assert(kGroupCtrl == 16 * kWave, "the value-sum step gives each lane 16 control bytes of a group");

constexpr uint32_t kSpanStage = 4608;  // 288 chunks: a document-id group's span fits
constexpr uint32_t kCorrList = 64;     // blocks with a non-zero control byte listed for one pass
constexpr uint32_t kSumLds = kSpanStage + 4 * kCorrList;

__device__ __forceinline__ uint32_t sad_bytes(uint32_t x, uint32_t acc) { return __builtin_amdgcn_sad_u8(x, 0u, acc); }

__device__ __forceinline__ uint32_t sad_chunk(const u32x4a &w, uint32_t acc) {
    acc = sad_bytes(w.x, acc);
    acc = sad_bytes(w.y, acc);
    acc = sad_bytes(w.z, acc);
    return sad_bytes(w.w, acc);
}

// The low L bytes of a dword, L in 1..4.
__device__ __forceinline__ uint32_t int_mask(uint32_t L) { return 0xFFFFFFFFu >> (32u - 8u * L); }

// Bytes [0, k) of a dword, k in 0..4.
__device__ __forceinline__ uint32_t low_bytes_mask(int32_t k) {
    return k <= 0 ? 0u : (k >= 4 ? 0xFFFFFFFFu : ((1u << (8 * k)) - 1u));
}

template <class T>
__device__ __forceinline__ T pick4(uint32_t i, T a0, T a1, T a2, T a3) {
    return i == 0 ? a0 : (i == 1 ? a1 : (i == 2 ? a2 : a3));
}

// Dword i (0..7) of the 32 bytes a:b, by selects (no indexed registers).
__device__ __forceinline__ uint32_t pick8(uint32_t i, const u32x4a &a, const u32x4a &b) {
    const uint32_t x = pick4(i & 3u, a.x, a.y, a.z, a.w), y = pick4(i & 3u, b.x, b.y, b.z, b.w);
    return i < 4 ? x : y;
}

// The 16-byte aligned chunk at cp, or zeros when it holds no byte of the
// buffer [lo, hi) (only on a corrupt stream whose span runs past the end).
__device__ __forceinline__ u32x4a load_chunk(const uint8_t *cp, const uint8_t *lo, const uint8_t *hi) {
    u32x4a w = u32x4a{0u, 0u, 0u, 0u};
    if (cp < hi && cp + 16 > lo) w = *gptr((const u32x4a *)cp);
    return w;
}

// Group g's byte offset in the data stream, and its data bytes, from one load
// of its block's byte counts.
__device__ __forceinline__ uint64_t group_span(const DecodeArgs &p, uint64_t g, uint32_t &bytes) {
    const uint64_t b = g / 4;
    const uint64_t o = p.boff32 ? (uint64_t)p.boff32[b] : p.boff[b];
    const uint32_t i = (uint32_t)(g & 3u);
    const u32x4a x = *(const u32x4a *)(p.gbytes + 4 * b);
    bytes = pick4(i, x.x, x.y, x.z, x.w);
    return o + (i > 0 ? x.x : 0u) + (i > 1 ? x.y : 0u) + (i > 2 ? x.z : 0u);
}

// A group's value sum in two halves, so that its loads can be in flight
// while the wave does something else: group_sum_issue requests the control
// bytes and the data span into registers, group_sum_finish stages the span in
// LDS and adds up.  The group's data span is bytes [gofs, gend) of the data
// stream (from the scan of the group byte counts; gend <= the data stream's
// length, checked by the caller).  Reads stay inside the aligned chunks that
// overlap the buffer.
struct SumLoads {
    uint64_t g, gofs;
    uint32_t total, sh16, nch;
    u32x4a cw;      // full group: the aligned dwords around the lane's 16 control bytes
    uint32_t cw4;   //   (a fifth dword when they are not 4-byte aligned)
    uint32_t csh;   //   and their byte alignment
    uint32_t c[4];  // the stream's last group: the lane's 16 control bytes (blocks 16 l .. 16 l + 15)
    uint32_t ints;  // integers of those blocks
    u32x4a w[5];    // chunks lane, lane + 64, ... of the span's first 288 chunks
};

__device__ __forceinline__ void group_sum_issue(const DecodeArgs &p, uint64_t g, uint64_t gofs, uint64_t gend,
                                                uint32_t lane, SumLoads &sl) {
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint8_t *data = p.in + nblocks;
    sl.g = g;
    sl.gofs = gofs;
    sl.total = (uint32_t)(gend - gofs);
    const uint8_t *at = data + gofs;
    sl.sh16 = (uint32_t)((uintptr_t)at & 15u);
    const uint8_t *abase = at - sl.sh16;
    sl.nch = (sl.sh16 + sl.total + 15) >> 4;
    const uint8_t *lo = p.in, *hi = p.in + p.in_bytes;
    const bool inside = abase >= lo && abase + 16ull * sl.nch <= hi;
    const uint64_t b0 = g * kGroupCtrl + 16ull * lane;
    if ((g + 1) * kGroupInts <= p.n) {
        // at any byte alignment: the aligned dwords around them each hold at least one of them
        const uint8_t *cp = p.in + b0;
        const uint32_t sh = (uint32_t)((uintptr_t)cp & 3u);
        const uint32_t *ap = (const uint32_t *)(cp - sh);
        // (aligned in group_sum_finish, so that the span's loads below are
        // issued before anything waits for these)
        sl.cw = *gptr((const u32x4a *)ap);
        sl.cw4 = sh ? gptr(ap)[4] : 0u;
        sl.csh = sh;
        sl.ints = 64;
    } else {
        // the stream's last group: blocks past the end read as 0, and the
        // codes of integers past n in the last block are cleared
        const uint32_t last_r = (uint32_t)(p.n & 3);
        sl.cw = u32x4a{0u, 0u, 0u, 0u};
        sl.cw4 = 0u;
        sl.csh = 0u;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) sl.c[i] = 0u;
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) {
            const uint64_t b = b0 + i;
            uint32_t x = b < nblocks ? (uint32_t)gptr(p.in)[b] : 0u;
            if (b == nblocks - 1 && last_r) x &= (1u << (2 * last_r)) - 1u;
            sl.c[i >> 2] |= x << (8 * (i & 3));
        }
        const uint64_t i0 = 4 * b0;
        sl.ints = i0 >= p.n ? 0u : (uint32_t)((p.n - i0) < 64 ? (p.n - i0) : 64);
    }
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        sl.w[i] = u32x4a{0u, 0u, 0u, 0u};
        if (kWave * i >= sl.nch) break;
        const uint32_t ch = kWave * i + lane;
        const uint8_t *cp = abase + 16 * ch;
        if (ch < sl.nch && ch < kSpanStage / 16) sl.w[i] = inside ? *gptr((const u32x4a *)cp) : load_chunk(cp, lo, hi);
    }
}

// Sum modulo 2^32 of the values stored in the group of `sl`.  `lds` is the
// wave's area (kSumLds bytes).
__device__ __forceinline__ uint32_t group_sum_finish(const DecodeArgs &p, const SumLoads &sl, uint32_t lane,
                                                     uint8_t *lds) {
    uint8_t *stage = lds;
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint8_t *abase = p.in + nblocks + sl.gofs - sl.sh16;
    const uint8_t *lo = p.in, *hi = p.in + p.in_bytes;
    const uint32_t sh16 = sl.sh16, total = sl.total, nch = sl.nch;
    // the span: whole chunks staged and summed, then the bytes of the first
    // and last chunk outside it taken back out; chunks past the staging area
    // (a group of long integers) are summed from memory
    const bool inside = abase >= lo && abase + 16ull * nch <= hi;
    uint32_t acc = 0;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) {
        if (kWave * i >= nch) break;
        const uint32_t ch = kWave * i + lane;
        if (ch < nch && ch < kSpanStage / 16) *(u32x4a *)(stage + 16 * ch) = sl.w[i];
        acc = sad_chunk(sl.w[i], acc);
    }
    for (uint32_t ch = kSpanStage / 16 + lane; ch < nch; ch += kWave) {
        const uint8_t *cp = abase + 16 * ch;
        acc = sad_chunk(inside ? *gptr((const u32x4a *)cp) : load_chunk(cp, lo, hi), acc);
    }
    const uint32_t staged = 16 * (nch < kSpanStage / 16 ? nch : kSpanStage / 16);

    // the lane's control bytes; per word, the codes before it and the top bit
    // of each of its non-zero bytes (a block that needs a correction)
    const bool full_group = (sl.g + 1) * kGroupInts <= p.n;
    uint32_t c[4];
    if (full_group) {
        c[0] = __builtin_amdgcn_alignbyte(sl.cw.y, sl.cw.x, sl.csh);
        c[1] = __builtin_amdgcn_alignbyte(sl.cw.z, sl.cw.y, sl.csh);
        c[2] = __builtin_amdgcn_alignbyte(sl.cw.w, sl.cw.z, sl.csh);
        c[3] = __builtin_amdgcn_alignbyte(sl.cw4, sl.cw.w, sl.csh);
    } else {
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) c[i] = sl.c[i];
    }
    uint32_t codes = 0, nzc = 0, pre[4], nz[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        pre[i] = codes;
        codes += __builtin_popcount(c[i]) + __builtin_popcount(c[i] & 0xAAAAAAAAu);
        nz[i] = (((c[i] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | c[i]) & 0x80808080u;
        nzc += __builtin_popcount(nz[i]);
    }
    // one scan for both the lane's byte offset in the span and its first
    // slot in the correction list (a group's data bytes, at most 16,384, and
    // its blocks, 1024, each fit 16 bits)
    const uint32_t bytes = sl.ints + codes;
    const uint32_t both = wave_incl_scan(bytes | (nzc << 16));
    const uint32_t off = (both & 0xFFFFu) - bytes;
    const uint32_t nzi = both >> 16;
    const uint32_t nz_total = wave_last(nzi);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // the span's edges: lane 0 takes back bytes [0, sh16) of the first chunk,
    // lane 1 the bytes of the last chunk from the span's end on (its chunk sum
    // minus its first e bytes), both read from the staged copy when it holds
    // them
    if (lane < 2) {
        const uint32_t ch = lane ? nch - 1 : 0u;
        const int32_t k = lane ? (int32_t)(sh16 + total - 16 * (nch - 1)) : (int32_t)sh16;
        const u32x4a w = 16 * ch + 16 <= staged ? *(const u32x4a *)(stage + 16 * ch) : load_chunk(abase + 16 * ch, lo, hi);
        const uint32_t pfx = sad_bytes(w.x & low_bytes_mask(k), 0u) + sad_bytes(w.y & low_bytes_mask(k - 4), 0u) +
                             sad_bytes(w.z & low_bytes_mask(k - 8), 0u) + sad_bytes(w.w & low_bytes_mask(k - 12), 0u);
        acc -= lane ? sad_chunk(w, 0u) - pfx : pfx;
    }

    // corrections: each block with a non-zero control byte, read from the
    // staged span (an integer's 4-byte read starts at most 12 bytes into its
    // block and reads 8 aligned bytes, so a block whose first byte lies 24
    // bytes or more before the staged part's end reads only staged bytes;
    // bytes past the span never reach a value, masked to the integer's
    // length), or else from its two aligned chunks in memory.  Every block is
    // taken as four integers: in the stream's last block the codes of the
    // integers past n were cleared above, and a one-byte integer needs no
    // correction (its value is its byte sum).
    // the correction of one block: its first byte at pos (from abase), control byte cb
    auto block_corr = [&](uint32_t pos, uint32_t cb) -> uint32_t {
        uint32_t corr = 0;
        if (pos + 24 <= staged) {
            uint32_t q = pos;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t L = ((cb >> (2 * j)) & 3u) + 1u;
                const uint32_t *src = (const uint32_t *)stage;
                const uint32_t x = __builtin_amdgcn_alignbyte(src[(q >> 2) + 1], src[q >> 2], q & 3u);
                const uint32_t v = x & int_mask(L);
                corr += v - sad_bytes(v, 0u);
                q += L;
            }
        } else {
            // past the staged part: the two aligned chunks around the block, in registers
            const uint32_t o = pos & 15u;
            const uint32_t C = 4u + __builtin_popcount(cb) + __builtin_popcount(cb & 0xAAu);
            const uint8_t *cp = abase + (pos - o);
            const u32x4a w0 = load_chunk(cp, lo, hi);
            const u32x4a w1 = (o + C > 16) ? load_chunk(cp + 16, lo, hi) : u32x4a{0u, 0u, 0u, 0u};
            uint32_t q = o;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t L = ((cb >> (2 * j)) & 3u) + 1u;
                const uint32_t x = __builtin_amdgcn_alignbyte(pick8((q >> 2) + 1, w0, w1), pick8(q >> 2, w0, w1), q & 3u);
                const uint32_t v = x & int_mask(L);
                corr += v - sad_bytes(v, 0u);
                q += L;
            }
        }
        return corr;
    };
    // Every block of the lane with a non-zero control byte, word by word
    // (so that each word's control bytes and code count are known without
    // selecting among registers): f(pos, cb) with its first byte at pos (from
    // abase) and its control byte.
    auto each_block = [&](auto f) {
        const uint32_t base = sh16 + off;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            uint32_t y = nz[i];
            while (y) {
                const uint32_t sft = (uint32_t)__builtin_ctz(y) - 7u;  // 8 k for byte k of the word
                y &= y - 1u;
                const uint32_t low = c[i] & ((1u << sft) - 1u);
                const uint32_t pos = base + 16u * i + pre[i] + (sft >> 1) + __builtin_popcount(low) +
                                     __builtin_popcount(low & 0xAAAAAAAAu);
                f(pos, __builtin_amdgcn_ubfe(c[i], sft, 8));
            }
        }
    };
    // the blocks with a non-zero control byte are few on most streams but
    // unevenly spread over the lanes: up to kCorrList of them are listed in
    // LDS and taken one per lane; more are taken by their own lanes
    uint32_t corr = 0;
    if (nz_total <= kCorrList) {
        uint32_t *list = (uint32_t *)(stage + kSpanStage);
        uint32_t slot = nzi - nzc;
        each_block([&](uint32_t pos, uint32_t cb) { list[slot++] = pos | (cb << 20); });
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < nz_total) {
            const uint32_t e = list[lane];
            corr = block_corr(e & 0xFFFFFu, e >> 20);
        }
    } else {
        each_block([&](uint32_t pos, uint32_t cb) { corr += block_corr(pos, cb); });
    }
    // the next use of the area overwrites it: LDS operations of a wave complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return wave_last(wave_incl_scan(acc + corr));
}

__device__ __forceinline__ uint32_t group_sum(const DecodeArgs &p, uint64_t g, uint64_t gofs, uint64_t gend,
                                              uint32_t lane, uint8_t *lds) {
    SumLoads sl;
    group_sum_issue(p, g, gofs, gend, lane, sl);
    return group_sum_finish(p, sl, lane, lds);
}

// The two-pass schedule's value-sum pass: one wave per group; nothing waits
// for another wave.
#ifndef SVB_SUMS_WPE
#define SVB_SUMS_WPE 8
#endif
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(SVB_SUMS_WPE, 8))) void group_sums_kernel(
    DecodeArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kWaves * kSumLds];
    __shared__ uint32_t s_part[kWaves];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t g = (uint64_t)blockIdx.x * kWaves + wave;
    uint32_t sum = 0;
    if (g < p.groups) {
        const uint64_t data_bytes = p.in_bytes - ((p.n + 3) >> 2);
        uint32_t gbytes;
        const uint64_t gofs = group_span(p, g, gbytes);
        const uint64_t gend = gofs + gbytes;
        if (gend > data_bytes) {
            if (p.err && lane == 0) *p.err = SVB_DECODE_CORRUPT;
        } else {
            sum = group_sum(p, g, gofs, gend, lane, s_lds + wave * kSumLds);
        }
    }
    // the block's total too (waves past the last group count 0)
    if (lane == 0) {
        p.gvsum[g] = sum;
        s_part[wave] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) p.bvsum[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

}  // namespace

hipError_t launch_group_sums(const DecodeArgs &a, hipStream_t s) {
    const uint32_t grid = (uint32_t)((a.groups + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(group_sums_kernel, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svb
