// Batched Stream VByte: m independent lists (the paper's posting lists,
// Section 5: many lists of very uneven length) decoded or encoded by one fixed
// sequence of launches whose work list is built on the device.
//
// A task is one 1024-integer segment of one list.  Tasks are numbered list by
// list; the host never reads the list arrays, so the task list is built on
// the device:
//   1. batch_count_kernel:  segments per list (0 for an empty or invalid list);
//   2. scan -> each list's first task, and the task total;
//   3. task -> (list, last segment of its list?), first task of its list (a
//      binary search per task), and the data bytes of every task that is not
//      the last segment of its list (decoding: batch_map_bytes_kernel, one
//      kernel: each lane searches for one task, then 8 lanes read a segment's
//      256 control bytes; encoding: batch_map_kernel, then one task per wave
//      takes the byte lengths of its 1024 values), then a scan -> each task's
//      byte offset in its list's data stream (global scan minus the value at
//      the list's first task);
//   4. delta decoding only: batch_sums_runs_kernel sums the stored
//      differences of every task that is not the last of its list (walking
//      each list's consecutive tasks as one run), then a scan;
//   5. batch_desc_kernel: one 64-byte descriptor per task (stream, output,
//      segment, byte offset, and for delta decoding the carry: global scan
//      minus the value at the list's first task, plus the list's start), so a
//      wave needs a single load to start a task;
//   6. batch_walk_kernel / batch_encode_kernel: each wave takes a run of
//      `chunk` consecutive tasks (the tuned parameter).  The decoder keeps a
//      pipeline three tasks deep: while one segment is decoded from LDS, the
//      next task's data, the control bytes of the one after and the
//      descriptor of the third are in flight.
// A list of one segment needs none of steps 4-5: offset 0, carry = start.
#include "svb_device.hpp"
#include "svb_internal.hpp"
#include "svb_segment.hpp"

namespace svb {

namespace {

constexpr uint32_t kEncStageWords = kEncStageBytes / 4;
constexpr uint32_t kLastBit = 1u << 31;

template <bool ENCODE>
__global__ __launch_bounds__(kThreads) void batch_count_kernel(BatchArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.m) return;
    const uint64_t c = a.counts[i];
    uint32_t segs = 0;
    if (c > SVB_MAX_N) {
        if (!ENCODE && a.err) *a.err = SVB_DECODE_CORRUPT;
        if (ENCODE && a.out_bytes) a.out_bytes[i] = ~0ull;
    } else if (!ENCODE && a.in_bytes[i] < (c + 3) / 4) {
        if (a.err) *a.err = SVB_DECODE_CORRUPT;  // control stream longer than the list's bytes
    } else {
        segs = (uint32_t)((c + kSegInts - 1) / kSegInts);
        if (ENCODE && c == 0 && a.out_bytes) a.out_bytes[i] = 0;
    }
    a.litems[i] = segs;
}

// The list i with lbase[i] <= t < lbase[i + 1] (t below lbase[m]), by a
// binary search over the list bases, so finding it costs the same however the
// tasks are spread over the lists.
__device__ __forceinline__ uint32_t find_list(const uint32_t *lbase, uint32_t m, uint64_t t) {
    uint32_t lo = 0, hi = m;  // invariant: lbase[lo] <= t < lbase[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (lbase[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Encoding: task -> list, one thread per task.  If the tasks overflow the
// caller's integer bound, nothing is done and every list's size is marked.
__global__ __launch_bounds__(kThreads) void batch_map_kernel(BatchArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint32_t total = a.lbase[a.m];
    if (total > a.t_cap) {
        if (t < a.m && a.out_bytes) a.out_bytes[t] = ~0ull;
        return;
    }
    if (t >= total) return;
    const uint32_t lo = find_list(a.lbase, a.m, t);
    const uint32_t e = a.lbase[lo + 1];
    a.item_list[t] = lo | ((uint32_t)t + 1 == e ? kLastBit : 0u);
    a.item_first[t] = a.lbase[lo];
}

// Total tasks, or 0 if they overflow the scratch.
__device__ __forceinline__ uint32_t task_total(const BatchArgs &a) {
    const uint32_t total = a.lbase[a.m];
    return total > a.t_cap ? 0u : total;
}

// ---------------------------------------------------------------- decoding

// Wave-uniform copies of descriptor fields (in scalar registers).  The
// builtin works on int: each half goes back to uint32_t before widening, so
// no half is sign-extended.
__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32) | (uint64_t)uniform32((uint32_t)x);
}

// Descriptors, written once every task's byte offset (and carry) is known.
template <bool ENCODE>
__global__ __launch_bounds__(kThreads) void batch_desc_kernel(BatchArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= task_total(a)) return;
    const uint32_t word = a.item_list[t];
    const uint32_t first = a.item_first[t];
    const uint32_t i = word & ~kLastBit;
    TaskDesc d = {};
    if (ENCODE) {
        d.in = (uint64_t)(a.in32 + a.in_off[i]);
        d.out = (uint64_t)(a.out8 + a.out_off[i]);
        d.carry = a.starts ? a.starts[i] : 0u;
    } else {
        d.in = (uint64_t)(a.in8 + a.in_off[i]);
        d.in_bytes = a.in_bytes[i];
        d.out = a.out_off ? (uint64_t)(a.out32 + a.out_off[i]) : 0ull;  // none in a task index
        if (a.starts) d.carry = a.starts[i] + (a.ivpre[t] - a.ivpre[first]);
    }
    d.n = a.counts[i];
    d.boff = a.ioff[t] - a.ioff[first];
    d.s = (uint32_t)t - first;
    d.word = word;
    a.desc[t] = d;
}

// A decode task as a wave sees it (wave-uniform).
struct TaskHdr {
    bool valid;
    bool last;
    DecodeArgs p;
    uint64_t s;
    uint64_t boff;
    uint32_t carry;
};

__device__ __forceinline__ TaskHdr load_hdr(const BatchArgs &a, uint64_t t, uint64_t t_end) {
    TaskHdr h = {};
    h.valid = t < t_end;
    if (!h.valid) return h;
    const TaskDesc d = a.desc[t];
    h.p.in = (const uint8_t *)uniform64(d.in);
    h.p.in_bytes = uniform64(d.in_bytes);
    h.p.n = uniform64(d.n);
    h.p.out = (uint32_t *)uniform64(d.out);
    h.p.err = a.err;
    h.boff = uniform64(d.boff);
    h.s = uniform32(d.s);
    h.carry = uniform32(d.carry);
    h.last = (uniform32(d.word) & kLastBit) != 0;
    return h;
}

// A task's segment in flight: its plan and its data loads.
struct Pending {
    SegPlan plan;
    uint32_t sh16;
    Span sp;
};

__device__ __forceinline__ void issue_task(const TaskHdr &k, const SegCtrl &sc, uint32_t lane, Pending &pd) {
    pd.plan = plan_segment(k.p, k.s, sc, lane);
    const uint8_t *q = k.p.in + (k.p.n + 3) / 4 + k.boff;
    pd.sh16 = (uint32_t)((uintptr_t)q & 15u);
    pd.sp.abase = q - pd.sh16;
    pd.sp.nch = (pd.sh16 + pd.plan.total + 15) >> 4;
    span_load(k.p, pd.sp, lane);
}

// Walks tasks [t0, t_end) of the task list with a pipeline three tasks
// deep: in the iteration that decodes task t, the data of t + 1, the control
// bytes of t + 2 and the descriptor of t + 3 are requested, each from what the
// previous iteration loaded.
// kPlain / kDelta: decode and store (delta: running sum from the task's
// carry).
template <int MODE>
__device__ __forceinline__ void walk_tasks(const BatchArgs &a, uint64_t t0, uint64_t t_end, uint8_t *stage,
                                           uint32_t lane, bool &corrupt) {
    constexpr bool DELTA = MODE == kDelta;
    auto active = [&](const TaskHdr &k) { return k.valid; };
    TaskHdr h0 = load_hdr(a, t0, t_end);
    Pending pend;
    if (active(h0)) issue_task(h0, load_seg_ctrl(h0.p, h0.s, lane), lane, pend);
    TaskHdr h1 = load_hdr(a, t0 + 1, t_end);
    TaskHdr h2 = load_hdr(a, t0 + 2, t_end);
    SegCtrl c1 = {{0u, 0u, 0u, 0u}};
    if (active(h1)) c1 = load_seg_ctrl(h1.p, h1.s, lane);

#pragma unroll 1
    for (uint64_t t = t0; t < t_end; ++t) {
        const TaskHdr k = h0;
        const bool work = active(k);
        SegPlan seg;
        uint32_t sh16 = 0;
        if (work) {
            if (k.boff + pend.plan.total > k.p.in_bytes - (k.p.n + 3) / 4) corrupt = true;
            span_to_lds(k.p, pend.sp, stage, lane);
            seg = pend.plan;
            sh16 = pend.sh16;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (active(h1)) issue_task(h1, c1, lane, pend);
        SegCtrl c2 = {{0u, 0u, 0u, 0u}};
        if (active(h2)) c2 = load_seg_ctrl(h2.p, h2.s, lane);
        const TaskHdr h3 = load_hdr(a, t + 3, t_end);

        if (work) {
            uint32_t v[4][4];
            extract_segment(k.p, k.s, stage, seg, sh16, lane, v);
            uint32_t carry = k.carry;
            if (DELTA) running_sum(v, carry);
            store_segment(k.p, k.s, lane, v, 0u);
        }
        walker_release();
        h0 = h1;
        h1 = h2;
        h2 = h3;
        c1 = c2;
    }
}

// The decode walk.  Static schedule (QUEUE false): wave w takes tasks
// [w chunk, (w + 1) chunk).  Work queue (QUEUE true, a.queue set): a grid of
// a few waves per SIMD, each wave grabbing the next `chunk` tasks from a
// device counter until none are left.  The two schedules are separate
// instantiations so that the static one carries none of the queue loop's
// registers.  Five waves per SIMD: the delta walk fits 96 registers without
// spilling, and was measured 12% faster there than at four.
#ifndef SVB_WALK_WPE
#define SVB_WALK_WPE 5
#endif
template <int MODE, bool QUEUE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(SVB_WALK_WPE, 8))) void batch_walk_kernel(BatchArgs a) {
    static_assert(MODE == kPlain || MODE == kDelta, "the value sums walk in runs (batch_sums_runs_kernel)");
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t total = task_total(a);
    uint8_t *stage = s_stage + wave * kStageBytes;
    bool corrupt = false;
    if (QUEUE) {
#pragma unroll 1
        for (;;) {
            uint32_t t0 = 0;
            if (lane == 0) t0 = atomicAdd(a.queue, a.chunk);
            t0 = __builtin_amdgcn_readfirstlane(t0);
            if (t0 >= total) break;  // every wave reaches this once the counter passes the last task
            const uint64_t t_end = (uint64_t)t0 + a.chunk < total ? (uint64_t)t0 + a.chunk : total;
            walk_tasks<MODE>(a, t0, t_end, stage, lane, corrupt);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        const uint64_t t0 = ((uint64_t)blockIdx.x * kWaves + wave) * a.chunk;
        if (t0 >= total) return;
        const uint64_t t_end = t0 + a.chunk < total ? t0 + a.chunk : total;
        walk_tasks<MODE>(a, t0, t_end, stage, lane, corrupt);
    }
    if (corrupt && a.err && lane == 0) *a.err = SVB_DECODE_CORRUPT;
}

// Delta decoding, value sums in runs: a wave takes kSumsChunk consecutive
// tasks, and each stretch of them that belongs to one list (every task but
// the list's last) is a run of consecutive full segments, walked like a
// single stream (Walker<1>): the run's list and byte offset are read once
// (it runs before the descriptors exist), byte offsets are chained from
// segment to segment, and the next segment's data is in flight while one is
// summed.  Writes each task's sum of stored differences to ivsum (0 for the
// last task of a list, whose sum no carry needs).
constexpr uint32_t kSumsChunk = 8;  // measured on C4: 8 tasks 175-179 us, 4 186-188, 6 178-180, 16 and 32 slower
// Seven waves per SIMD (72 registers, no spill): the whole batched C4 call
// measured 0.648-0.652 ms against 0.668 at five and 0.660 at six; a walker
// two segments deep (four waves per SIMD, 119 registers) 0.717.
#ifndef SVB_SUMS_RUN_WPE
#define SVB_SUMS_RUN_WPE 7
#endif
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(SVB_SUMS_RUN_WPE, 8))) void batch_sums_runs_kernel(
    BatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves * kStageBytes];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t total = task_total(a);
    const uint64_t t0 = ((uint64_t)blockIdx.x * kWaves + wave) * kSumsChunk;
    if (t0 >= total) return;
    const uint64_t t_end = t0 + kSumsChunk < total ? t0 + kSumsChunk : total;
    uint8_t *stage = s_stage + wave * kStageBytes;
    bool corrupt = false;
    uint64_t t = t0;
#pragma unroll 1
    while (t < t_end) {
        const uint32_t word = uniform32(a.item_list[t]);
        if (word & kLastBit) {
            if (lane == 0) a.ivsum[t] = 0u;
            ++t;
            continue;
        }
        const uint32_t li = word & ~kLastBit;
        const uint32_t first = uniform32(a.item_first[t]);
        DecodeArgs p = {};
        p.in = a.in8 + uniform64(a.in_off[li]);
        p.in_bytes = uniform64(a.in_bytes[li]);
        p.n = uniform64(a.counts[li]);
        const uint64_t s0 = t - first;
        const uint64_t boff = uniform64(a.ioff[t]) - uniform64(a.ioff[first]);
        // the run: tasks t .. u - 1, up to the list's last task (excluded) or the chunk's end
        const uint64_t segs = (p.n + kSegInts - 1) / kSegInts;
        const uint64_t list_last = t + (segs - 1 - s0);
        const uint64_t u = list_last < t_end ? list_last : t_end;
        Walker<1> w;
        walker_begin(p, w, s0, s0 + (u - t), boff, lane);
#pragma unroll 1
        for (uint64_t i = 0; i < u - t; ++i) {
            SegPlan seg;
            uint32_t sh16;
            walker_step(p, w, stage, lane, seg, sh16);
            uint32_t v[4][4];
            extract_segment(p, s0 + i, stage, seg, sh16, lane, v);
            walker_release();
            uint32_t x = 0;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) x += v[q][0] + v[q][1] + v[q][2] + v[q][3];
            x = wave_last(wave_incl_scan(x));
            if (lane == 0) a.ivsum[t + i] = x;
        }
        corrupt |= w.corrupt;
        t = u;
    }
    if (corrupt && a.err && lane == 0) *a.err = SVB_DECODE_CORRUPT;
}

// Decoding: task -> list and the data bytes of every task, 64 tasks per wave.
// Lane l finds the list of task 64 w + l; then the wave counts the bytes of its
// 64 tasks eight at a time, lanes 8 j .. 8 j + 7 reading the 256 control bytes
// of one task, 32 each.  The last task of a list writes 0.  If the tasks
// overflow the caller's integer bound, nothing is done and the call reports
// SVB_BATCH_OVERFLOW.
__global__ __launch_bounds__(kThreads) void batch_map_bytes_kernel(BatchArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t total = a.lbase[a.m];
    const uint64_t tw = ((uint64_t)blockIdx.x * kWaves + wave) * kWave;
    if (total > a.t_cap) {
        if (tw == 0 && lane == 0 && a.err) *a.err = SVB_BATCH_OVERFLOW;
        return;
    }
    if (tw >= total) return;
    const uint64_t t = tw + lane;
    uint32_t body = 0;
    uint64_t ctrl = 0;  // address of the task's first control byte
    if (t < total) {
        const uint32_t i = find_list(a.lbase, a.m, t);
        const uint32_t first = a.lbase[i];
        body = t + 1 < a.lbase[i + 1] ? 1u : 0u;
        a.item_list[t] = i | (body ? 0u : kLastBit);
        a.item_first[t] = first;
        ctrl = (uint64_t)(a.in8 + a.in_off[i] + (t - first) * kSegCtrl);
    }
    const uint32_t part = lane & 7u;
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t g = 0; g < kWave / 8; ++g) {
        const uint32_t q = 8 * g + lane / 8;  // the task of this lane's group
        const uint32_t qb = __shfl(body, q, kWave);
        const uint64_t qc = ((uint64_t)__shfl((uint32_t)(ctrl >> 32), q, kWave) << 32) |
                            (uint64_t)__shfl((uint32_t)ctrl, q, kWave);
        uint32_t bytes = 0;
        if (qb) {
            // a segment that is not the last of its list is full, and more
            // bytes of the list follow its control bytes; the aligned dwords
            // around the lane's 32 bytes each hold at least one of them, so
            // none crosses a page the list does not touch
            const uint8_t *gp = (const uint8_t *)qc + 32u * part;
            const uint32_t sh = (uint32_t)((uintptr_t)gp & 3u);
            const uint32_t *base = (const uint32_t *)(gp - sh);
            const uint32_t keep = 0xFFFFFFFFu << (8u * sh);
            uint32_t codes = 0;
#pragma unroll
            for (uint32_t w = 0; w < 8; ++w) {
                const uint32_t x = (w == 0) ? (gptr(base)[w] & keep) : gptr(base)[w];
                codes += __builtin_popcount(x) + __builtin_popcount(x & 0xAAAAAAAAu);
            }
            const uint32_t e = sh ? (gptr(base)[8] & ~keep) : 0u;
            codes += __builtin_popcount(e) + __builtin_popcount(e & 0xAAAAAAAAu);
            bytes = 128u + codes;
        }
        // sum over each group of 8 lanes; lane q takes task q's total
        bytes += __shfl_xor(bytes, 1, kWave);
        bytes += __shfl_xor(bytes, 2, kWave);
        bytes += __shfl_xor(bytes, 4, kWave);
        const uint32_t v = __shfl(bytes, 8 * (lane & 7u), kWave);
        if (lane / 8 == g) mine = v;
    }
    if (t < total) a.ibytes[t] = body ? mine : 0u;
}

// ---------------------------------------------------------------- encoding

struct EncTask {
    bool valid;
    bool last;
    uint32_t list;
    EncodeStream e;
    uint64_t s;
    uint64_t boff;
};

__device__ __forceinline__ EncTask load_enc_task(const BatchArgs &a, uint64_t t, uint64_t t_end) {
    EncTask k = {};
    k.valid = t < t_end;
    if (!k.valid) return k;
    const uint32_t word = a.item_list[t];
    const uint32_t first = a.item_first[t];
    k.list = word & ~kLastBit;
    k.last = (word & kLastBit) != 0;
    k.e.in = a.in32 + a.in_off[k.list];
    k.e.n = a.counts[k.list];
    k.e.out = a.out8 + a.out_off[k.list];
    k.e.start = a.starts ? a.starts[k.list] : 0u;
    k.s = t - first;
    k.boff = a.ioff[t] - a.ioff[first];
    return k;
}

// Data bytes of one encode task per wave (the last task of a list writes 0).
template <bool DELTA>
__global__ __launch_bounds__(kThreads) void batch_task_bytes_encode_kernel(BatchArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t total = task_total(a);
    const uint64_t t = (uint64_t)blockIdx.x * kWaves + wave;
    if (t >= total) return;
    const EncTask k = load_enc_task(a, t, total);
    uint32_t bytes = 0;
    if (!k.last) {
        SegValues sv;
        load_segment_values<DELTA>(k.e, k.s, lane, sv);
        bytes = segment_data_bytes(sv);
    }
    if (lane == 0) a.ibytes[t] = bytes;
}

template <bool DELTA>
__global__ __launch_bounds__(kThreads) void batch_encode_kernel(BatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t s_stage[kWaves * kEncStageWords];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t total = task_total(a);
    const uint64_t t0 = ((uint64_t)blockIdx.x * kWaves + wave) * a.chunk;
    if (t0 >= total) return;
    const uint64_t t_end = t0 + a.chunk < total ? t0 + a.chunk : total;
    uint32_t *stage = s_stage + wave * kEncStageWords;
#pragma unroll 1
    for (uint64_t t = t0; t < t_end; ++t) {
        const TaskDesc d = a.desc[t];
        EncodeStream e;
        e.in = (const uint32_t *)uniform64(d.in);
        e.n = uniform64(d.n);
        e.out = (uint8_t *)uniform64(d.out);
        e.start = uniform32(d.carry);
        const uint64_t boff = uniform64(d.boff);
        const uint32_t word = uniform32(d.word);
        const uint32_t bytes = encode_segment<DELTA>(e, uniform32(d.s), boff, lane, stage);
        if ((word & kLastBit) && lane == 0 && a.out_bytes) a.out_bytes[word & ~kLastBit] = (e.n + 3) / 4 + boff + bytes;
    }
}

uint32_t list_grid(uint32_t m) { return (m + kThreads - 1) / kThreads; }
constexpr uint64_t kQueueWaves = 256 * 4 * 5;
uint32_t wave_grid(uint64_t waves) { return (uint32_t)((waves + kWaves - 1) / kWaves); }

// ---------------------------------------------------------------- serving

// One serving batch's descriptors: task t finds its batch list j (base[j] <=
// t < base[j + 1], a binary search over the batch's small, cache-resident
// table) and copies the index descriptor of that list's segment t - base[j],
// pointed at the list's arena range.  One thread per task, so a list's
// segments are copied in parallel.
__global__ __launch_bounds__(kThreads) void serve_desc_kernel(ServeDescArgs a) {
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t tasks = a.base[a.m];
    if (t >= tasks) return;
    uint32_t lo = 0, hi = a.m;  // invariant: base[lo] <= t < base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.base[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    TaskDesc d = a.pool_desc[a.pool_lbase[a.list[lo]] + (t - a.base[lo])];
    d.out = (uint64_t)(a.arena + a.out_off[lo]);
    a.desc[t] = d;
}

// One serving batch's table, built on the device from the integer counts of
// its lists (in query order, the queries' results back to back from
// out_base): each list's first task (its segments, ceil(count / 1024), summed
// over the lists before it) and arena offset (the integers of the lists
// before it; a batch holds fewer than 2^32).  One workgroup: kPlanPer lists
// per thread per step, wave scans of both sums, the 16 wave totals scanned in
// LDS, the carry into the next step.
constexpr uint32_t kPlanThreads = 1024, kPlanPer = 8, kPlanWaves = kPlanThreads / kWave;

__global__ __launch_bounds__(kPlanThreads) void serve_plan_kernel(ServePlanArgs a) {
    __shared__ uint32_t s_ints[kPlanWaves + 1], s_tasks[kPlanWaves + 1];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t carry_i = 0, carry_t = 0;
    for (uint32_t c0 = 0; c0 < a.m; c0 += kPlanThreads * kPlanPer) {
        uint32_t ci[kPlanPer], ct[kPlanPer];
        uint32_t si = 0, st = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPlanPer; ++j) {
            const uint32_t idx = c0 + tid * kPlanPer + j;
            ci[j] = idx < a.m ? a.counts[idx] : 0u;
            ct[j] = (ci[j] + kSegInts - 1) / kSegInts;
            si += ci[j];
            st += ct[j];
        }
        const uint32_t ii = wave_incl_scan(si), it = wave_incl_scan(st);
        if (lane == kWave - 1) {
            s_ints[wave] = ii;
            s_tasks[wave] = it;
        }
        __syncthreads();
        if (wave == 0) {
            const uint32_t wi = lane < kPlanWaves ? s_ints[lane] : 0u, wt = lane < kPlanWaves ? s_tasks[lane] : 0u;
            const uint32_t xi = wave_incl_scan(wi), xt = wave_incl_scan(wt);
            if (lane < kPlanWaves) {
                s_ints[lane] = xi - wi;
                s_tasks[lane] = xt - wt;
            }
            if (lane == kWave - 1) {
                s_ints[kPlanWaves] = xi;
                s_tasks[kPlanWaves] = xt;
            }
        }
        __syncthreads();
        uint32_t pi = carry_i + s_ints[wave] + ii - si;
        uint32_t pt = carry_t + s_tasks[wave] + it - st;
#pragma unroll
        for (uint32_t j = 0; j < kPlanPer; ++j) {
            const uint32_t idx = c0 + tid * kPlanPer + j;
            if (idx < a.m) {
                a.out_off[idx] = a.out_base + pi;
                a.base[idx] = pt;
            }
            pi += ci[j];
            pt += ct[j];
        }
        carry_i += s_ints[kPlanWaves];
        carry_t += s_tasks[kPlanWaves];
        __syncthreads();  // the next step rewrites the totals
    }
    if (tid == 0) a.base[a.m] = carry_t;
}

}  // namespace

hipError_t launch_serve_plan(const ServePlanArgs &a, hipStream_t s) {
    if (a.m == 0) return hipSuccess;
    hipLaunchKernelGGL(serve_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs &a, int phase, bool encode, bool delta, hipStream_t s) {
    const uint64_t chunk_waves = (a.t_cap + a.chunk - 1) / a.chunk;
    switch (phase) {
        case kBatchCount:
            if (encode)
                hipLaunchKernelGGL((batch_count_kernel<true>), dim3(list_grid(a.m)), dim3(kThreads), 0, s, a);
            else
                hipLaunchKernelGGL((batch_count_kernel<false>), dim3(list_grid(a.m)), dim3(kThreads), 0, s, a);
            break;
        case kBatchMap:
            // one thread per task (t_cap >= m, so the overflow path also reaches every list)
            if (!encode) return hipErrorInvalidValue;
            hipLaunchKernelGGL(batch_map_kernel, dim3(list_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            break;
        case kBatchDesc:
            if (encode)
                hipLaunchKernelGGL((batch_desc_kernel<true>), dim3(list_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            else
                hipLaunchKernelGGL((batch_desc_kernel<false>), dim3(list_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            break;
        case kBatchItemBytes:
            if (!encode)
                hipLaunchKernelGGL(batch_map_bytes_kernel, dim3(list_grid(a.t_cap)), dim3(kThreads), 0, s, a);
            else if (delta)
                hipLaunchKernelGGL((batch_task_bytes_encode_kernel<true>), dim3(wave_grid(a.t_cap)), dim3(kThreads), 0, s,
                                   a);
            else
                hipLaunchKernelGGL((batch_task_bytes_encode_kernel<false>), dim3(wave_grid(a.t_cap)), dim3(kThreads), 0, s,
                                   a);
            break;
        case kBatchItemSums:
            hipLaunchKernelGGL(batch_sums_runs_kernel, dim3(wave_grid((a.t_cap + kSumsChunk - 1) / kSumsChunk)),
                               dim3(kThreads), 0, s, a);
            break;
        case kBatchWork:
            if (encode) {
                if (delta)
                    hipLaunchKernelGGL((batch_encode_kernel<true>), dim3(wave_grid(chunk_waves)), dim3(kThreads), 0, s, a);
                else
                    hipLaunchKernelGGL((batch_encode_kernel<false>), dim3(wave_grid(chunk_waves)), dim3(kThreads), 0, s, a);
            } else {
                // with a work queue: at most five waves per SIMD of a 256-CU chip, each looping
                const uint64_t waves = a.queue && chunk_waves > kQueueWaves ? kQueueWaves : chunk_waves;
                const dim3 grid(wave_grid(waves));
                if (delta) {
                    if (a.queue)
                        hipLaunchKernelGGL((batch_walk_kernel<kDelta, true>), grid, dim3(kThreads), 0, s, a);
                    else
                        hipLaunchKernelGGL((batch_walk_kernel<kDelta, false>), grid, dim3(kThreads), 0, s, a);
                } else {
                    if (a.queue)
                        hipLaunchKernelGGL((batch_walk_kernel<kPlain, true>), grid, dim3(kThreads), 0, s, a);
                    else
                        hipLaunchKernelGGL((batch_walk_kernel<kPlain, false>), grid, dim3(kThreads), 0, s, a);
                }
            }
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_serve_desc(const ServeDescArgs &a, uint32_t tasks, hipStream_t s) {
    if (a.m == 0 || tasks == 0) return hipSuccess;
    hipLaunchKernelGGL(serve_desc_kernel, dim3((tasks + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svb
