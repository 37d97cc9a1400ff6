// Seek and select on resident compressed lists (the two operations on the
// compressed stream that Section 5 benchmarks): seek(list, target) gives the
// first position whose value is >= target, with that value; select(list, i)
// gives the value at position i.  A value is the running sum for delta-coded
// lists (Section 2) and the stored integer otherwise.
//
// Skip index, built once over the lists: the batched decoder's task index (per
// 1024-integer segment: its byte offset in the list's data stream and the
// running sum before it) plus, per segment, the running maximum of the list's
// values up to the segment's end.  The running maximum never decreases, so the
// segment holding a seek's answer is the first whose running maximum reaches
// the target, found by a 64-way search, whether or not the list is sorted;
// select's segment is i / 1024.  Each query is one wave that decodes that one
// segment with the single-stream decoder's segment code.
#include <algorithm>

#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

namespace {

__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32) | (uint64_t)uniform32((uint32_t)x);
}

// Inclusive running maximum over the 64 lanes of a wave (the DPP pattern of
// wave_incl_scan with max in place of +; lanes that a step does not reach see
// 0, which leaves the maximum of unsigned values unchanged).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, true));   // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, true));   // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, true));   // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, true));   // row_shr:8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return x;
}

// The first of a lane's four integers (j = 0..3, in order) that is a valid
// position with a value >= target, or 4 if none.
__device__ __forceinline__ uint32_t first_at_least(const uint32_t (&v)[4], uint32_t valid_n, uint32_t c0,
                                                   uint32_t target) {
    uint32_t jf = 4;
#pragma unroll
    for (int j = 3; j >= 0; --j)
        if (c0 + (uint32_t)j < valid_n && v[j] >= target) jf = (uint32_t)j;
    return jf;
}

// One segment of one list, as the task index describes it (wave-uniform).
struct SegRef {
    DecodeArgs p;
    uint64_t s;
    uint64_t boff;
    uint32_t carry;
};

__device__ __forceinline__ SegRef load_seg(const TaskDesc *desc, uint64_t t) {
    const TaskDesc d = desc[t];
    SegRef r;
    r.p = DecodeArgs{};
    r.p.in = (const uint8_t *)uniform64(d.in);
    r.p.in_bytes = uniform64(d.in_bytes);
    r.p.n = uniform64(d.n);
    r.s = uniform32(d.s);
    r.boff = uniform64(d.boff);
    r.carry = uniform32(d.carry);
    return r;
}

// Decodes the segment into the lane's 16 values (block 64 k + lane, integer j
// in v[k][j]; integers past the list's end read as 0).  Returns true if the
// segment's data run past the list's bytes (corrupt input; the values are then
// meaningless, and no load left the list's bytes).
__device__ __forceinline__ bool decode_seg(const SegRef &r, bool delta, uint8_t *stage, uint32_t lane,
                                           uint32_t (&v)[4][4]) {
    const SegCtrl sc = load_seg_ctrl(r.p, r.s, lane);
    const SegPlan plan = plan_segment(r.p, r.s, sc, lane);
    const uint64_t nblocks = (r.p.n + 3) >> 2;
    const uint8_t *q = r.p.in + nblocks + r.boff;
    Span sp;
    const uint32_t sh16 = (uint32_t)((uintptr_t)q & 15u);
    sp.abase = q - sh16;
    sp.nch = (sh16 + plan.total + 15) >> 4;
    const bool corrupt = r.boff + plan.total > r.p.in_bytes - nblocks;
    span_load(r.p, sp, lane);
    span_to_lds(r.p, sp, stage, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    extract_segment(r.p, r.s, stage, plan, sh16, lane, v);
    if (delta) {
        uint32_t carry = r.carry;
        running_sum(v, carry);
    }
    return corrupt;
}

// A segment of at most 256 integers (a short list, or a list's last segment)
// uses one row of the four: lane l holds block l only.  Decoding just that row
// saves three quarters of the scans, extraction and comparisons, and queries
// are bound by instruction issue.  v[j] is integer 4 lane + j (0 past the
// end).
__device__ __forceinline__ bool decode_row(const SegRef &r, uint32_t rem, bool delta, uint8_t *stage, uint32_t lane,
                                           uint32_t (&v)[4]) {
    const uint64_t nblocks = (r.p.n + 3) >> 2;
    const uint32_t nb_seg = (rem + 3) >> 2;  // control bytes of the segment (1..64)
    const int32_t left = (int32_t)rem - (int32_t)(4 * lane);
    const uint32_t m = left <= 0 ? 0u : (left >= 4 ? 4u : (uint32_t)left);
    const uint64_t b = r.s * kSegCtrl + (lane < nb_seg ? lane : nb_seg - 1);
    const uint32_t raw = gptr(r.p.in)[b];
    const uint32_t c = m ? (raw & ((1u << (2 * m)) - 1u)) : 0u;
    const uint32_t nb = m + __builtin_popcount(c) + __builtin_popcount(c & 0xAAu);
    const uint32_t incl = wave_incl_scan(nb);
    const uint32_t total = wave_last(incl);
    const uint8_t *q = r.p.in + nblocks + r.boff;
    Span sp;
    const uint32_t sh16 = (uint32_t)((uintptr_t)q & 15u);
    sp.abase = q - sh16;
    sp.nch = (sh16 + total + 15) >> 4;
    const bool corrupt = r.boff + total > r.p.in_bytes - nblocks;
    span_load(r.p, sp, lane);
    span_to_lds(r.p, sp, stage, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // as extract_segment, for the one row
    uint32_t R = kStagePad - 4 + sh16 + (incl - nb);
    const uint32_t nc = ~c;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t y = (nc >> (2 * j)) & 3u;
        R -= y;
        const uint32_t a = (R & ~3u) + 4 * (j + 1);
        const uint32_t lo = *(const uint32_t *)(stage + a);
        const uint32_t hi = *(const uint32_t *)(stage + a + 4);
        v[j] = j < m ? __builtin_amdgcn_alignbyte(0u, __builtin_amdgcn_alignbyte(hi, lo, R & 3u), y) : 0u;
    }
    if (delta) {
        v[1] += v[0];
        v[2] += v[1];
        v[3] += v[2];
        const uint32_t li = wave_incl_scan(v[3]);
        const uint32_t add = r.carry + li - v[3];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) v[j] += add;
    }
    return corrupt;
}

// The value at local position li (0..255) of a decoded row, on every lane.
__device__ __forceinline__ uint32_t row_value_at(const uint32_t (&v)[4], uint32_t li) {
    const uint32_t j = li & 3u, owner = (li >> 2) & (kWave - 1);
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t jj = 0; jj < 4; ++jj)
        if (jj == j) mine = v[jj];
    return (uint32_t)__builtin_amdgcn_readlane((int)mine, (int)owner);
}

// The value at local position li (0..1023) of a decoded segment, on every lane.
__device__ __forceinline__ uint32_t value_at(const uint32_t (&v)[4][4], uint32_t li) {
    const uint32_t k = li >> 8, j = li & 3u, owner = (li >> 2) & (kWave - 1);
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t kk = 0; kk < 4; ++kk)
#pragma unroll
        for (uint32_t jj = 0; jj < 4; ++jj)
            if (kk == k && jj == j) mine = v[kk][jj];
    return (uint32_t)__builtin_amdgcn_readlane((int)mine, (int)owner);
}

// Index build, pass 1: the largest value of every segment (one wave per task).
__global__ __launch_bounds__(kThreads) void seg_max_kernel(SeekArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t t = (uint64_t)blockIdx.x * kWaves + wave;
    if (t >= a.tasks) return;
    const SegRef r = load_seg(a.desc, t);
    const uint64_t rem = r.p.n - r.s * kSegInts;
    uint32_t x = 0;
    bool corrupt;
    if (rem <= kSegInts / 4) {
        uint32_t v[4];
        corrupt = decode_row(r, (uint32_t)rem, a.delta, s_stage + wave * kStageBytes, lane, v);
        // positions past the end hold 0 (plain) or the last running value (delta)
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) x = max(x, v[j]);
    } else {
        uint32_t v[4][4];
        corrupt = decode_seg(r, a.delta, s_stage + wave * kStageBytes, lane, v);
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) x = max(x, v[k][j]);  // as above
    }
    x = wave_incl_max(x);
    if (lane == kWave - 1) a.rmax[t] = x;
    if (corrupt && lane == 0) *a.err = SVB_DECODE_CORRUPT;
}

// Index build, pass 2: within each list, the running maximum of the segment
// maxima (one wave per list, 64 segments per step).
__global__ __launch_bounds__(kThreads) void run_max_kernel(SeekArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t l = (uint64_t)blockIdx.x * kWaves + wave;
    if (l >= a.m) return;
    const uint32_t first = a.lbase[l], end = a.lbase[l + 1];
    uint32_t carry = 0;
    for (uint32_t b = first; b < end; b += kWave) {
        const uint32_t t = b + lane;
        uint32_t x = t < end ? a.rmax[t] : 0u;
        x = max(wave_incl_max(x), carry);
        if (t < end) a.rmax[t] = x;
        carry = (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
    }
}

// Index build, pass 3: one line per list (one thread each).
__global__ __launch_bounds__(kThreads) void list_rec_kernel(SeekArgs a) {
    const uint32_t l = blockIdx.x * kThreads + threadIdx.x;
    if (l >= a.m) return;
    const uint32_t first = a.lbase[l], segs = a.lbase[l + 1] - first;
    SeekList r = {};
    r.first = first;
    r.segs = segs;
    if (segs) {
        const TaskDesc &d = a.desc[first];
        r.in = d.in;
        r.in_bytes = d.in_bytes;
        r.n = d.n;
        r.carry = d.carry;
        r.top = a.rmax[first + segs - 1];
    }
    a.lists[l] = r;
}

// Marks query `qi` as refused.
__device__ __forceinline__ void refuse(const SeekArgs &a, uint32_t qi, uint32_t code, uint32_t lane) {
    if (lane != 0) return;
    if (a.pos) a.pos[qi] = ~0ull;
    a.value[qi] = 0u;
    if (a.err) *a.err = code;
}

// Query qi, answered by one wave.  SEEK: the first position of list[qi] whose
// value is >= target[qi] (the list's length if none, value 0).  Otherwise
// select: the value at position idx[qi].  A list id past m, or a select
// position past the list's end, is refused with SVB_QUERY_OUT_OF_RANGE.
template <bool SEEK>
__device__ __forceinline__ void answer(const SeekArgs &a, uint32_t qi, uint8_t *stage, uint32_t lane) {
    // the query's list and its target or position are requested together
    const uint32_t t_raw = SEEK ? a.target[qi] : 0u;
    const uint64_t i_raw = SEEK ? 0ull : a.idx[qi];
    const uint32_t l = uniform32(a.list[qi]);
    if (l >= a.m) {
        refuse(a, qi, SVB_QUERY_OUT_OF_RANGE, lane);
        return;
    }
    const uint32_t first = uniform32(a.lbase[l]);
    const uint32_t segs = uniform32(a.lbase[l + 1]) - first;
    uint64_t s;
    uint32_t target = 0;
    uint64_t idx = 0;
    SegRef r;
    if (SEEK) {
        target = uniform32(t_raw);
        if (segs == 0) {
            if (lane == 0) {
                a.pos[qi] = 0ull;
                a.value[qi] = 0u;
            }
            return;
        }
        // the list's largest value and its first segment's descriptor are
        // requested together (a list of one segment needs nothing else)
        const uint32_t top_raw = a.rmax[first + segs - 1];
        r = load_seg(a.desc, first);
        if (uniform32(top_raw) < target) {
            // no value reaches the target: the list's length
            if (lane == 0) {
                a.pos[qi] = r.p.n;
                a.value[qi] = 0u;
            }
            return;
        }
        // the first segment whose running maximum reaches the target lies in
        // [lo, hi]; each step probes 64 evenly spaced segments of the range
        uint32_t lo = 0, hi = segs - 1;
        while (lo < hi) {
            const uint32_t step = (hi - lo + kWave) / kWave;  // ceil((hi - lo + 1) / 64)
            const uint32_t p = lo + lane * step;
            const bool valid = p <= hi;
            const bool below = valid && a.rmax[first + p] < target;
            const uint32_t n_below = __builtin_popcountll(__ballot(below));
            const uint32_t nvalid = __builtin_popcountll(__ballot(valid));
            const uint32_t new_lo = n_below ? lo + (n_below - 1) * step + 1 : lo;
            const uint32_t new_hi = n_below < nvalid ? lo + n_below * step : hi;
            lo = new_lo;
            hi = new_hi;
        }
        s = lo;
        if (s) r = load_seg(a.desc, first + s);
    } else {
        // every segment's descriptor holds the list's length
        idx = uniform64(i_raw);
        s = idx / kSegInts;
        if (s >= segs) {
            refuse(a, qi, SVB_QUERY_OUT_OF_RANGE, lane);
            return;
        }
        r = load_seg(a.desc, first + s);
        if (idx >= r.p.n) {
            refuse(a, qi, SVB_QUERY_OUT_OF_RANGE, lane);
            return;
        }
    }
    const uint64_t base = s * kSegInts;
    const uint64_t rem64 = r.p.n - base;
    uint32_t li, val;
    if (rem64 <= kSegInts / 4) {
        // a segment of one row
        uint32_t v[4];
        if (decode_row(r, (uint32_t)rem64, a.delta, stage, lane, v)) {
            refuse(a, qi, SVB_DECODE_CORRUPT, lane);
            return;
        }
        if (SEEK) {
            // the row holds a value >= target: the first lane that has one,
            // then its first such integer
            const uint32_t jf = first_at_least(v, (uint32_t)rem64, 4 * lane, target);
            const uint64_t mask = __ballot(jf < 4);
            const uint32_t owner = mask ? (uint32_t)__builtin_ctzll(mask) : 0u;
            li = 4 * owner + (uint32_t)__builtin_amdgcn_readlane((int)jf, (int)owner);
        } else {
            li = (uint32_t)(idx - base);
        }
        val = row_value_at(v, li);
    } else {
        uint32_t v[4][4];
        if (decode_seg(r, a.delta, stage, lane, v)) {
            refuse(a, qi, SVB_DECODE_CORRUPT, lane);
            return;
        }
        if (SEEK) {
            // the segment holds a value >= target (its running maximum reaches
            // the target, the previous segment's does not): the first row
            // with one, its first lane with one, that lane's first such integer
            const uint32_t rem = (uint32_t)(rem64 < kSegInts ? rem64 : kSegInts);
            li = 0;
            bool found = false;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) {
                const uint32_t jf = first_at_least(v[k], rem, 4 * (kWave * k + lane), target);
                const uint64_t mask = __ballot(jf < 4);
                if (!found && mask) {
                    const uint32_t owner = (uint32_t)__builtin_ctzll(mask);
                    li = 4 * (kWave * k + owner) + (uint32_t)__builtin_amdgcn_readlane((int)jf, (int)owner);
                    found = true;
                }
            }
        } else {
            li = (uint32_t)(idx - base);
        }
        val = value_at(v, li);
    }
    if (lane == 0) {
        if (SEEK) a.pos[qi] = base + li;
        a.value[qi] = val;
    }
}

// Four queries per wave, 16 lanes each, for lists of at most 256 integers
// (one segment of one row: 64 control bytes).  Lane g of a group takes
// control bytes 4 g .. 4 g + 3 (16 integers): the lengths, a 16-lane scan of
// the byte counts (DPP row shifts stay inside a row of 16 lanes), the row's
// data bytes staged in the group's quarter of the wave's LDS area, the
// integers cut out with two byte-align instructions each, the running sum
// for delta lists (in the lane, then across the group).  A query whose list
// has more than one segment, or more than 256 integers, is left to the
// one-wave path: the return value says which groups answered.
constexpr uint32_t kGroupLanes = 16;
constexpr uint32_t kRowCtrl = 64, kRowInts = 4 * kRowCtrl;
constexpr uint32_t kGroupStage = kStageBytes / (kWave / kGroupLanes);  // 1056: 1024 data bytes, 15 before, 8 after
static_assert(kGroupStage >= 4 * kRowInts + 16 + 16, "a group's staging area holds a row's data bytes");

__device__ __forceinline__ uint32_t row16_incl_scan(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, true);  // row_shr:8
    return x;
}

template <bool SEEK>
__device__ __forceinline__ bool answer_rows4(const SeekArgs &a, uint64_t qi, bool active, uint8_t *stage,
                                             uint32_t lane) {
    const uint32_t gl = lane & (kGroupLanes - 1);
    const uint32_t gbase = lane & ~(kGroupLanes - 1);
    uint8_t *gs = stage + (lane / kGroupLanes) * kGroupStage;
    if (!active) return true;
    const uint32_t l = a.list[qi];
    const uint32_t t_raw = SEEK ? a.target[qi] : 0u;
    const uint64_t idx = SEEK ? 0ull : a.idx[qi];
    if (l >= a.m) {
        if (gl == 0) refuse(a, (uint32_t)qi, SVB_QUERY_OUT_OF_RANGE, 0);
        return true;
    }
    const SeekList &rec = a.lists[l];
    const uint32_t segs = rec.segs;
    if (segs == 0) {
        // an empty list: a seek answers position 0, a select is out of range
        if (gl == 0) {
            if (SEEK) {
                a.pos[qi] = 0ull;
                a.value[qi] = 0u;
            } else {
                refuse(a, (uint32_t)qi, SVB_QUERY_OUT_OF_RANGE, 0);
            }
        }
        return true;
    }
    if (segs != 1) return false;
    const uint64_t n = rec.n;
    if (n > kRowInts) return false;
    const uint8_t *in = (const uint8_t *)rec.in;
    const uint64_t in_bytes = rec.in_bytes;
    const uint32_t carry = rec.carry;
    if (SEEK) {
        if (rec.top < t_raw) {
            // no value reaches the target: the list's length
            if (gl == 0) {
                a.pos[qi] = n;
                a.value[qi] = 0u;
            }
            return true;
        }
    } else if (idx >= n) {
        if (gl == 0) refuse(a, (uint32_t)qi, SVB_QUERY_OUT_OF_RANGE, 0);
        return true;
    }
    // the lane's four control bytes, codes of integers past n cleared
    const uint32_t nblocks = (uint32_t)((n + 3) >> 2);
    uint32_t c[4], m[4], bytes = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t b = 4 * gl + k;
        const int32_t left = (int32_t)n - (int32_t)(4 * b);
        m[k] = left <= 0 ? 0u : (left >= 4 ? 4u : (uint32_t)left);
        const uint32_t raw = b < nblocks ? (uint32_t)gptr(in)[b] : 0u;
        c[k] = m[k] ? (raw & ((1u << (2 * m[k])) - 1u)) : 0u;
        bytes += m[k] + __builtin_popcount(c[k]) + __builtin_popcount(c[k] & 0xAAu);
    }
    const uint32_t incl = row16_incl_scan(bytes);
    const uint32_t total = (uint32_t)__shfl((int)incl, (int)(gbase + kGroupLanes - 1));
    if (total > in_bytes - nblocks) {  // the index build checked in_bytes >= nblocks
        if (gl == 0) refuse(a, (uint32_t)qi, SVB_DECODE_CORRUPT, 0);
        return true;
    }
    // the row's data bytes (the whole data stream of a list of one segment)
    // into the group's staging area, 16-byte chunks from the aligned address
    // below the first
    const uint8_t *q0 = in + nblocks;
    const uint32_t sh16 = (uint32_t)((uintptr_t)q0 & 15u);
    const uint8_t *abase = q0 - sh16;
    const uint32_t nch = (sh16 + total + 15) >> 4;
    const uint8_t *lo = in, *hi = in + in_bytes;
#pragma unroll
    for (uint32_t i = 0; i < (kGroupStage - 16) / (16 * kGroupLanes) + 1; ++i) {
        const uint32_t ch = gl + kGroupLanes * i;
        if (ch < nch) {
            const uint8_t *cp = abase + 16 * ch;
            u32x4a w = u32x4a{0u, 0u, 0u, 0u};
            if (cp < hi && cp + 16 > lo) w = *gptr((const u32x4a *)cp);
            *(u32x4a *)(gs + 16 * ch) = w;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the lane's 16 integers, cut from the staged bytes in two passes (no
    // array of them: a wave of this kernel holds few registers): the first
    // sums them (delta lists), the second runs the values and keeps the one
    // the query asks for
    const uint32_t *w32 = (const uint32_t *)gs;
    const uint32_t q_lane = sh16 + incl - bytes;
    auto int_at = [&](uint32_t &q, uint32_t k, uint32_t j, bool &valid) -> uint32_t {
        const uint32_t L = ((c[k] >> (2 * j)) & 3u) + 1u;
        valid = j < m[k];
        const uint32_t x = __builtin_amdgcn_alignbyte(w32[(q >> 2) + 1], w32[q >> 2], q & 3u);
        q += valid ? L : 0u;
        return valid ? (L == 4 ? x : x & ((1u << (8 * L)) - 1u)) : 0u;
    };
    // sixteen one-byte integers (every control byte of the lane zero, none
    // past n, as on lists of small differences): the lane's 16 data bytes,
    // cut from five aligned dwords, summed by SAD and unpacked by bit-field
    // extracts; otherwise integer by integer
    const bool zc = (c[0] | c[1] | c[2] | c[3]) == 0 && m[0] + m[1] + m[2] + m[3] == 16;
    uint32_t X[4] = {0u, 0u, 0u, 0u};
    uint32_t run = 0;
    if (zc) {
        const uint32_t d = q_lane >> 2, o = q_lane & 3u;
        uint32_t prev = w32[d];
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            const uint32_t nxt = w32[d + 1 + i];
            X[i] = __builtin_amdgcn_alignbyte(nxt, prev, o);
            prev = nxt;
        }
    }
    if (a.delta) {
        uint32_t sum = 0;
        if (zc) {
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) sum = __builtin_amdgcn_sad_u8(X[i], 0u, sum);
        } else {
            uint32_t q = q_lane;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
                for (uint32_t j = 0; j < 4; ++j) {
                    bool valid;
                    sum += int_at(q, k, j, valid);
                }
        }
        run = carry + row16_incl_scan(sum) - sum;  // the running value before the lane's first integer
    }
    // SEEK: the lane's first valid value >= target (jf = 16 if none); select:
    // the value at idx, held by lane idx / 16
    const uint32_t jsel = SEEK ? 16u : (uint32_t)(idx & 15u);
    uint32_t jf = 16, mine = 0;
    auto visit = [&](uint32_t i, uint32_t x, bool valid) {
        const uint32_t vv = a.delta ? (run += x) : x;
        if (SEEK) {
            if (jf == 16 && valid && vv >= t_raw) {
                jf = i;
                mine = vv;
            }
        } else if (i == jsel) {
            mine = vv;
        }
    };
    if (zc) {
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) visit(i, __builtin_amdgcn_ubfe(X[i >> 2], 8 * (i & 3u), 8), true);
    } else {
        uint32_t q = q_lane;
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                bool valid;
                const uint32_t x = int_at(q, k, j, valid);
                visit(4 * k + j, x, valid);
            }
    }
    uint32_t pos, val;
    if (SEEK) {
        // the row holds a value >= target: the first lane of the group with one
        const uint64_t mask = (__ballot(jf < 16) >> gbase) & 0xFFFFull;
        const uint32_t owner = mask ? (uint32_t)__builtin_ctzll(mask) : 0u;
        const uint32_t ojf = (uint32_t)__shfl((int)jf, (int)(gbase + owner));
        val = (uint32_t)__shfl((int)mine, (int)(gbase + owner));
        pos = 16 * owner + ojf;
    } else {
        val = (uint32_t)__shfl((int)mine, (int)(gbase + (uint32_t)(idx >> 4)));
        pos = (uint32_t)idx;
    }
    if (gl == 0) {
        if (SEEK) a.pos[qi] = pos;
        a.value[qi] = val;
    }
    return true;
}

// Each wave answers a run of a.chunk consecutive queries, so that a large
// batch does not cost one workgroup launch per four queries.  Throughput
// follows the number of resident waves (each query is a chain of dependent
// loads), so the kernel is held to eight waves per SIMD.  (Keeping the next
// queries' index loads in flight while one decodes was measured no faster:
// it cost more registers, hence waves, than it saved in waiting.)
#ifndef SVB_QUERY_WPE
#define SVB_QUERY_WPE 6
#endif
template <bool SEEK>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(SVB_QUERY_WPE, 8))) void query_kernel(SeekArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t q0 = ((uint64_t)blockIdx.x * kWaves + wave) * a.chunk;
    const uint64_t q1 = q0 + a.chunk < a.q ? q0 + a.chunk : a.q;
    uint8_t *stage = s_stage + wave * kStageBytes;
#pragma unroll 1
    for (uint64_t qb = q0; qb < q1; qb += kWave / kGroupLanes) {
        // four queries at once, 16 lanes each; the ones that need a whole wave after
        const uint64_t qi = qb + lane / kGroupLanes;
        const bool done = answer_rows4<SEEK>(a, qi, qi < q1, stage, lane);
        const uint64_t rest = __ballot(!done);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t g = 0; g < kWave / kGroupLanes; ++g) {
            if (!((rest >> (kGroupLanes * g)) & 1ull)) continue;
            answer<SEEK>(a, (uint32_t)(qb + g), stage, lane);
            // the next query overwrites the staging area: LDS operations of a
            // wave complete in order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

}  // namespace

hipError_t launch_seek_index(const SeekArgs &a, hipStream_t s) {
    if (a.tasks)
        hipLaunchKernelGGL(seg_max_kernel, dim3((uint32_t)((a.tasks + kWaves - 1) / kWaves)), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(run_max_kernel, dim3((a.m + kWaves - 1) / kWaves), dim3(kThreads), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(list_rec_kernel, dim3((a.m + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seek_queries(const SeekArgs &a, bool seek, hipStream_t s) {
    if (a.q == 0 || a.chunk == 0) return hipSuccess;
    const uint64_t waves = (a.q + a.chunk - 1) / a.chunk;
    const dim3 grid((uint32_t)((waves + kWaves - 1) / kWaves));
    if (seek)
        hipLaunchKernelGGL(query_kernel<true>, grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(query_kernel<false>, grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svb

// ---------------------------------------------------------------- C ABI

namespace {

struct SeekIndex {
    int device = 0;
    uint32_t m = 0;
    bool delta = false;
    uint32_t tasks = 0;
    svb::TaskDesc *desc = nullptr;
    uint32_t *lbase = nullptr;
    uint32_t *rmax = nullptr;
    svb::SeekList *lists = nullptr;
};

void free_index(SeekIndex *x) {
    if (!x) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(x->device);
    (void)hipDeviceSynchronize();
    if (x->desc) (void)hipFree(x->desc);
    if (x->lbase) (void)hipFree(x->lbase);
    if (x->rmax) (void)hipFree(x->rmax);
    if (x->lists) (void)hipFree(x->lists);
    (void)hipSetDevice(cur);
    delete x;
}

bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

int queries(void *index, uint32_t q, const uint32_t *list, const uint32_t *target, const uint64_t *idx,
            uint64_t *pos, uint32_t *value, uint32_t *err, bool seek, void *stream) {
    SeekIndex *x = (SeekIndex *)index;
    if (!x) return SVB_ERR_INVALID;
    if (q == 0) return SVB_OK;
    if (!list || !value || (seek ? (!target || !pos) : !idx)) return SVB_ERR_INVALID;
    if (!aligned(list, 4) || !aligned(value, 4) || (target && !aligned(target, 4)) || (idx && !aligned(idx, 8)) ||
        (pos && !aligned(pos, 8)) || (err && !aligned(err, 4)))
        return SVB_ERR_INVALID;
    if (q > (1u << 31)) return SVB_ERR_INVALID;
    svb::SeekArgs a = {};
    a.m = x->m;
    a.tasks = x->tasks;
    a.desc = x->desc;
    a.lbase = x->lbase;
    a.rmax = x->rmax;
    a.lists = x->lists;
    a.delta = x->delta;
    a.q = q;
    // queries per wave: four (one per 16-lane group) while that still leaves
    // tens of thousands of waves, up to 16
    a.chunk = std::min<uint32_t>(16u, std::max<uint32_t>(4u, (q / 32768u) & ~3u));
    a.list = list;
    a.target = target;
    a.idx = idx;
    a.pos = seek ? pos : nullptr;
    a.value = value;
    a.err = err;
    return svb::launch_seek_queries(a, seek, (hipStream_t)stream) == hipSuccess ? SVB_OK : SVB_ERR_HIP;
}

}  // namespace

extern "C" {

int svb_seek_index_create(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                          const uint8_t *in, const uint32_t *starts, uint64_t total_ints, void **index,
                          void *stream) {
    if (!index) return SVB_ERR_INVALID;
    *index = nullptr;
    hipStream_t s = (hipStream_t)stream;
    SeekIndex *x = new SeekIndex();
    (void)hipGetDevice(&x->device);
    x->m = m;
    x->delta = starts != nullptr;
    int st = svb::build_pool_index(m, counts, in_off, in_bytes, in, starts, total_ints, &x->desc, &x->lbase,
                                   &x->tasks, s);
    uint32_t *d_err = nullptr;
    if (st == SVB_OK && hipMalloc((void **)&x->rmax, 4ull * (x->tasks ? x->tasks : 1)) != hipSuccess)
        st = SVB_ERR_NOMEM;
    if (st == SVB_OK && hipMalloc((void **)&x->lists, sizeof(svb::SeekList) * (m ? m : 1)) != hipSuccess)
        st = SVB_ERR_NOMEM;
    if (st == SVB_OK && hipMalloc((void **)&d_err, 4) != hipSuccess) st = SVB_ERR_NOMEM;
    uint32_t h_err = 0;
    if (st == SVB_OK) {
        svb::SeekArgs a = {};
        a.m = m;
        a.tasks = x->tasks;
        a.desc = x->desc;
        a.lbase = x->lbase;
        a.rmax = x->rmax;
        a.lists = x->lists;
        a.delta = x->delta;
        a.err = d_err;
        if (svb::launch_fill(d_err, 1, 0u, s) != hipSuccess || svb::launch_seek_index(a, s) != hipSuccess ||
            hipMemcpyAsync(&h_err, d_err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = SVB_ERR_HIP;
        else if (h_err != 0)
            st = SVB_ERR_INVALID;
    }
    if (d_err) (void)hipFree(d_err);
    if (st != SVB_OK) {
        free_index(x);
        return st;
    }
    *index = x;
    return SVB_OK;
}

int svb_seek_batch(void *index, uint32_t q, const uint32_t *list, const uint32_t *target, uint64_t *pos,
                   uint32_t *value, uint32_t *err, void *stream) {
    return queries(index, q, list, target, nullptr, pos, value, err, true, stream);
}

int svb_select_batch(void *index, uint32_t q, const uint32_t *list, const uint64_t *idx, uint32_t *value,
                     uint32_t *err, void *stream) {
    return queries(index, q, list, nullptr, idx, nullptr, value, err, false, stream);
}

int svb_seek_index_destroy(void *index) {
    free_index((SeekIndex *)index);
    return SVB_OK;
}

}  // extern "C"
