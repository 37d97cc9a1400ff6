// One-pass delta decoding for gfx950.
//
// Differential coding (Section 2) stores x_i - x_{i-1}; decoding is a running
// sum over the decoded differences, started from `start`.  The decoder of
// Section 4 keeps that sum in a register while it walks the stream; here every
// wave decodes its own group of kGroupInts integers at the same time, so each
// wave needs the sum of every difference stored before its group (its carry)
// before it can store anything.
//
// The two-pass schedule (svb_decode.hip) reads the stream twice from memory:
// a pass that sums each group's differences, a scan, then the decode pass.
// This kernel reads it once.  Each wave:
//
//   A. sums its group's differences without decoding them (below), which also
//      brings the group's control and data bytes into the L2;
//   B. publishes that sum and finds its carry by a chained scan with a
//      decoupled look-back over the groups before it (a status word per
//      group: the group's own sum, or the inclusive running sum once known);
//   C. decodes the group like the two-pass decode pass, adding the carry,
//      from bytes that pass A left in the caches.
//
// Sum of a group's values without decoding them.  A value of L bytes is
// sum_k byte_k 256^k, so the sum of the values is the plain sum of all the
// group's data bytes plus, for each integer of L >= 2 bytes, its value minus
// the sum of its bytes.  The plain byte sum needs no integer boundaries: it
// is a sum over the group's contiguous data span (four SAD instructions per
// 16 bytes).  The corrections are needed only for blocks whose control byte
// is not zero (a zero control byte stands for four one-byte integers), which
// are compacted into a list and handled 64 at a time.  On document-id gaps
// (mostly one-byte differences) that is about 4 % of the blocks.
//
// Forward progress: groups are taken in the order workgroups start (a ticket
// counter), so every group a wave waits on belongs to a workgroup that is
// already running.  The status words carry a call counter in their tag, so
// they need no clearing between calls; the last workgroup to finish resets
// the ticket and advances the counter for the next call.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

namespace {

static_assert(kGroupCtrl == 16 * kWave, "the value-sum step gives each lane 16 control bytes of a group");
static_assert(4 * kGroupInts <= 0xFFFF, "a group's data bytes fit the 16-bit halves of the packed scan");

constexpr uint32_t kEntBytes = 4 * kGroupCtrl;  // compacted blocks with a non-zero control byte
constexpr uint32_t kWinBytes = 32 * kWave;      // a 32-byte window per lane
constexpr uint32_t kWaveLds = (kEntBytes + kWinBytes) > kStageBytes ? (kEntBytes + kWinBytes) : kStageBytes;

__device__ __forceinline__ uint32_t sad_bytes(uint32_t x, uint32_t acc) { return __builtin_amdgcn_sad_u8(x, 0u, acc); }

__device__ __forceinline__ uint32_t sad_chunk(const u32x4a &w, uint32_t acc) {
    acc = sad_bytes(w.x, acc);
    acc = sad_bytes(w.y, acc);
    acc = sad_bytes(w.z, acc);
    return sad_bytes(w.w, acc);
}

// Bytes [0, k) of a dword, k in 0..4.
__device__ __forceinline__ uint32_t low_bytes_mask(int32_t k) {
    return k <= 0 ? 0u : (k >= 4 ? 0xFFFFFFFFu : ((1u << (8 * k)) - 1u));
}

template <class T>
__device__ __forceinline__ T pick4(uint32_t i, T a0, T a1, T a2, T a3) {
    return i == 0 ? a0 : (i == 1 ? a1 : (i == 2 ? a2 : a3));
}

// The 16-byte aligned chunk at cp, or zeros when it holds no byte of the
// buffer [lo, hi) (only on a corrupt stream whose span runs past the end).
__device__ __forceinline__ u32x4a load_chunk(const uint8_t *cp, const uint8_t *lo, const uint8_t *hi) {
    u32x4a w = u32x4a{0u, 0u, 0u, 0u};
    if (cp < hi && cp + 16 > lo) w = *gptr((const u32x4a *)cp);
    return w;
}

// Sum modulo 2^32 of the values stored in group g, whose data start at byte
// `gofs` of the data stream `data` (of `data_bytes` bytes).  `lds` is the
// wave's area (kWaveLds bytes).  Sets `bad` if the group's data would run past
// the buffer; nothing is read outside it.
__device__ uint32_t group_value_sum(const DecodeArgs &p, const uint8_t *data, uint64_t data_bytes, uint64_t g,
                                    uint64_t gofs, uint32_t lane, uint8_t *lds, bool &bad) {
    const uint64_t nblocks = (p.n + 3) >> 2;
    const uint64_t b0 = g * kGroupCtrl + 16ull * lane;  // the lane's first control byte
    uint32_t c[4];
    uint32_t ints;
    if ((g + 1) * kGroupInts <= p.n) {
        // 16 control bytes at any byte alignment: the aligned dwords around
        // them each hold at least one of them
        const uint8_t *cp = p.in + b0;
        const uint32_t sh = (uint32_t)((uintptr_t)cp & 3u);
        const uint32_t *ap = (const uint32_t *)(cp - sh);
        const u32x4 w = *gptr((const u32x4 *)ap);
        const uint32_t w4 = sh ? gptr(ap)[4] : 0u;
        c[0] = __builtin_amdgcn_alignbyte(w.y, w.x, sh);
        c[1] = __builtin_amdgcn_alignbyte(w.z, w.y, sh);
        c[2] = __builtin_amdgcn_alignbyte(w.w, w.z, sh);
        c[3] = __builtin_amdgcn_alignbyte(w4, w.w, sh);
        ints = 64;
    } else {
        // the stream's last group: blocks past the end read as 0, and the
        // codes of integers past n in the last block are cleared
        const uint32_t last_r = (uint32_t)(p.n & 3);
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) c[i] = 0u;
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) {
            const uint64_t b = b0 + i;
            uint32_t x = b < nblocks ? (uint32_t)gptr(p.in)[b] : 0u;
            if (b == nblocks - 1 && last_r) x &= (1u << (2 * last_r)) - 1u;
            c[i >> 2] |= x << (8 * (i & 3));
        }
        const uint64_t i0 = 4 * b0;
        ints = i0 >= p.n ? 0u : (uint32_t)((p.n - i0) < 64 ? (p.n - i0) : 64);
    }
    // data bytes of the lane's blocks (4 per block plus its codes), the code
    // bits before each dword, and which control bytes are not zero
    uint32_t codes = 0, nzm = 0, pre[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        pre[i] = codes;
        codes += __builtin_popcount(c[i]) + __builtin_popcount(c[i] & 0xAAAAAAAAu);
        const uint32_t y = (((c[i] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | c[i]) & 0x80808080u;  // top bit of each non-zero byte
        nzm |= ((((y >> 7) * 0x00204081u) >> 21) & 0xFu) << (4 * i);                     // ... gathered into a nibble
    }
    const uint32_t bytes = ints + codes;
    const uint32_t K = __builtin_popcount(nzm);
    // one scan for both: byte offsets in the low half, list positions in the high
    const uint32_t incl = wave_incl_scan(bytes | (K << 16));
    const uint32_t tot = wave_last(incl);
    const uint32_t off = (incl & 0xFFFFu) - bytes;
    uint32_t kpos = (incl >> 16) - K;
    const uint32_t total = tot & 0xFFFFu, ktot = tot >> 16;
    if (gofs + total > data_bytes) {
        bad = true;
        return 0u;
    }

    // plain sum of the span's bytes: whole aligned 16-byte chunks, then the
    // bytes of the first and last chunk outside the span taken back out
    const uint8_t *at = data + gofs;
    const uint32_t sh16 = (uint32_t)((uintptr_t)at & 15u);
    const uint8_t *abase = at - sh16;
    const uint32_t nch = (sh16 + total + 15) >> 4;
    const uint8_t *lo = p.in, *hi = p.in + p.in_bytes;
    const bool inside = abase >= lo && abase + 16ull * nch <= hi;
    uint32_t acc = 0;
    for (uint32_t c0 = 0; c0 < nch; c0 += 8 * kWave) {
        u32x4a w[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            w[i] = u32x4a{0u, 0u, 0u, 0u};
            if (c0 + kWave * i >= nch) break;
            const uint32_t ch = c0 + kWave * i + lane;
            const uint8_t *cp = abase + 16 * ch;
            if (ch < nch) w[i] = inside ? *gptr((const u32x4a *)cp) : load_chunk(cp, lo, hi);
        }
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            if (c0 + kWave * i >= nch) break;
            acc = sad_chunk(w[i], acc);
        }
    }
    if (lane < 2) {
        // lane 0: bytes [0, sh16) of the first chunk; lane 1: the last
        // chunk's bytes from the span's end on
        const uint32_t ch = lane ? nch - 1 : 0u;
        const int32_t xlo = lane ? (int32_t)(sh16 + total - 16 * (nch - 1)) : 0;
        const int32_t xhi = lane ? 16 : (int32_t)sh16;
        if (xlo < xhi) {
            const u32x4a w = load_chunk(abase + 16 * ch, lo, hi);
            const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
            uint32_t x = 0;
#pragma unroll
            for (int32_t i = 0; i < 4; ++i)
                x = sad_bytes(wd[i] & low_bytes_mask(xhi - 4 * i) & ~low_bytes_mask(xlo - 4 * i), x);
            acc -= x;
        }
    }

    // compact the blocks whose control byte is not zero: (byte offset in
    // the group's data, control byte, integers - 1) per entry
    uint32_t *ent = (uint32_t *)lds;
    const uint64_t last_block = nblocks - 1;
    const uint32_t last_r1 = (uint32_t)((p.n - 1) & 3);  // integers in the stream's last block, minus 1
    uint32_t m = nzm;
    while (m) {
        const uint32_t b = __builtin_ctz(m);
        m &= m - 1u;
        const uint32_t i = b >> 2, k = b & 3u;
        const uint32_t ci = pick4(i, c[0], c[1], c[2], c[3]);
        const uint32_t low = ci & low_bytes_mask((int32_t)k);
        const uint32_t boff = off + 4 * b + pick4(i, pre[0], pre[1], pre[2], pre[3]) + __builtin_popcount(low) +
                              __builtin_popcount(low & 0xAAAAAAAAu);
        const uint32_t r1 = (b0 + b == last_block) ? last_r1 : 3u;
        ent[kpos++] = (r1 << 24) | (((ci >> (8 * k)) & 0xFFu) << 16) | boff;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // each listed block: the sum of its values minus the sum of its bytes,
    // from the two aligned chunks around it, staged in the lane's window
    uint32_t corr = 0;
    uint32_t *win = (uint32_t *)(lds + kEntBytes) + 8 * lane;
    for (uint32_t e0 = 0; e0 < ktot; e0 += kWave) {
        const uint32_t e = e0 + lane;
        if (e < ktot) {
            const uint32_t en = ent[e];
            const uint32_t cb = (en >> 16) & 0xFFu, r = (en >> 24) + 1u;
            const uint8_t *bp = at + (en & 0xFFFFu);
            const uint32_t o = (uint32_t)((uintptr_t)bp & 15u);
            const uint32_t C = r + __builtin_popcount(cb) + __builtin_popcount(cb & 0xAAu);
            const u32x4a w0 = load_chunk(bp - o, lo, hi);
            const u32x4a w1 = (o + C > 16) ? load_chunk(bp - o + 16, lo, hi) : u32x4a{0u, 0u, 0u, 0u};
            *(u32x4a *)win = w0;
            *(u32x4a *)(win + 4) = w1;
            uint32_t q = o;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t L = ((cb >> (2 * j)) & 3u) + 1u;
                const uint32_t x = __builtin_amdgcn_alignbyte(win[(q >> 2) + 1], win[q >> 2], q & 3u);
                const uint32_t v = (j < r) ? (x & low_bytes_mask((int32_t)L)) : 0u;
                corr += v - sad_bytes(v, 0u);
                q += L;
            }
        }
    }
    return wave_last(wave_incl_scan(acc + corr));
}

__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void status_store(uint64_t *p, uint32_t tag, uint32_t value) {
    __hip_atomic_store(p, ((uint64_t)tag << 32) | value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chained scan over the groups: publishes group g's own sum `agg`, finds the
// sum of everything before it (start included) by looking back over the status
// words of its predecessors, 64 at a time, and publishes its inclusive sum.
// The value travels in the same 64-bit word as its tag, so relaxed atomics
// suffice.  Returns the group's carry.  The wait is bounded: after
// `spin_limit` polls without progress the wave gives up, sets `stalled` and
// publishes what it has, so that every wave still ends.
__device__ uint32_t look_back(uint64_t *status, uint64_t g, uint32_t epoch, uint32_t agg, uint32_t start,
                              uint32_t lane, uint32_t spin_limit, bool &stalled) {
    const uint32_t tag_agg = epoch << 1, tag_incl = tag_agg | 1u;
    if (g == 0) {
        if (lane == 0) status_store(status, tag_incl, start + agg);
        return start;
    }
    if (lane == 0) status_store(status + g, tag_agg, agg);
    uint32_t carry = 0, idle = 0;
    int64_t j = (int64_t)g - 1;  // lane l examines group j - l
    for (;;) {
        const int64_t idx = j - (int64_t)lane;
        uint32_t tag = tag_incl, val = start;  // before group 0: the start value, inclusive
        if (idx >= 0) {
            const uint64_t w = status_load(status + idx);
            tag = (uint32_t)(w >> 32);
            val = (uint32_t)w;
        }
        const uint64_t not_ready = __ballot((tag | 1u) != tag_incl);
        const uint64_t inclusive = __ballot(tag == tag_incl);
        const uint32_t f_nr = not_ready ? (uint32_t)__builtin_ctzll(not_ready) : 64u;
        const uint32_t f_in = inclusive ? (uint32_t)__builtin_ctzll(inclusive) : 64u;
        const uint32_t take = f_in < f_nr ? f_in + 1 : f_nr;  // lanes [0, take) add their values
        const uint32_t s = wave_incl_scan(lane < take ? val : 0u);
        if (take) carry += __builtin_amdgcn_readlane(s, take - 1);
        if (f_in < f_nr) break;
        j -= take;
        if (take == 0) {
            if (++idle > spin_limit) {
                stalled = true;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    if (lane == 0) status_store(status + g, tag_incl, carry + agg);
    return carry;
}

// Wave w of the workgroup with ticket t decodes group 4 t + w.
template <bool ZC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void delta_onepass_kernel(DecodeArgs p, const uint32_t *goff32, OnePassArgs op) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kWaves * kWaveLds];
    __shared__ uint32_t s_ticket[2];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (threadIdx.x == 0) {
        s_ticket[0] = __hip_atomic_fetch_add(&op.ctl->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ticket[1] = __hip_atomic_load(&op.ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t ticket = s_ticket[0];
    const uint32_t epoch = s_ticket[1] + 1u;  // 1 .. 2^31 - 1: a zero tag is never valid
    const uint64_t g = (uint64_t)ticket * kWaves + wave;
    if (g < p.groups) {
        uint8_t *lds = s_lds + wave * kWaveLds;
        const uint64_t nblocks = (p.n + 3) >> 2;
        const uint8_t *data = p.in + nblocks;
        const uint64_t data_bytes = p.in_bytes - nblocks;
        const uint64_t gofs = goff32 ? (uint64_t)goff32[g] : p.goff[g];
        bool bad = false;
        const uint32_t agg = group_value_sum(p, data, data_bytes, g, gofs, lane, lds, bad);
        const uint64_t segs = (p.n + kSegInts - 1) / kSegInts;
        const uint64_t s0 = g * kGroupSegs;
        const uint64_t s_end = s0 + kGroupSegs < segs ? s0 + kGroupSegs : segs;
        // the first segment's loads are in flight during the look-back
        Walker<1> w;
        walker_begin(p, w, s0, s_end, gofs, lane);
        bool stalled = false;
        uint32_t carry = look_back(op.status, g, epoch, agg, op.start, lane, op.spin_limit, stalled);
        for (uint64_t s = s0; s < s_end; ++s) {
            SegPlan seg;
            uint32_t sh16;
            walker_step(p, w, lds, lane, seg, sh16);
            uint32_t v[4][4];
            extract_segment<ZC>(p, s, lds, seg, sh16, lane, v);
            walker_release();
            running_sum(v, carry);
            store_segment(p, s, lane, v, 0u);
        }
        if ((w.corrupt || bad) && p.err && lane == 0) *p.err = SVB_DECODE_CORRUPT;
        if (stalled && p.err && lane == 0) *p.err = SVB_DECODE_STALLED;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&op.ctl->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (d == gridDim.x - 1) {
            // every workgroup has its ticket: reset for the next call
            __hip_atomic_store(&op.ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&op.ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&op.ctl->epoch, epoch == 0x7FFFFFFFu ? 0u : epoch, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

hipError_t launch_delta_onepass(const DecodeArgs &a, const uint32_t *goff32, const OnePassArgs &op, bool zc,
                                hipStream_t s) {
    const uint32_t grid = (uint32_t)((a.groups + kWaves - 1) / kWaves);
    if (zc)
        hipLaunchKernelGGL(delta_onepass_kernel<true>, dim3(grid), dim3(kThreads), 0, s, a, goff32, op);
    else
        hipLaunchKernelGGL(delta_onepass_kernel<false>, dim3(grid), dim3(kThreads), 0, s, a, goff32, op);
    return hipGetLastError();
}

}  // namespace svb
