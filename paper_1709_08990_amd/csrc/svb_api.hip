// C ABI of libsvb.so (declared in include/svb.h): argument checks, per-stream
// scratch workspaces and kernel launches.  No codec arithmetic happens here.
#include <algorithm>
#include <map>
#include <vector>
#include <mutex>
#include <utility>

#include "svb_internal.hpp"

namespace svb {
namespace {

// Scratch owned by the library for one (device, stream): per-piece byte
// counts, offsets and value sums of the reduce-then-scan passes.
struct Workspace {
    uint8_t *scratch = nullptr;
    uint64_t scratch_bytes = 0;
};

std::mutex g_mu;
std::map<std::pair<int, uintptr_t>, Workspace> g_ws;

int hip_status(hipError_t e) { return e == hipSuccess ? SVB_OK : SVB_ERR_HIP; }

// Optional per-kernel timing (svb_set_kernel_timing): each codec kernel launch
// of the calling thread is bracketed by a pair of HIP events recorded on the
// launch stream; svb_kernel_times reads and forgets the recorded pairs.
struct KernelTiming {
    const char *name;
    hipEvent_t begin, end;
};
bool g_timing = false;
thread_local std::vector<KernelTiming> t_timings;     // recorded, not read yet
thread_local std::vector<KernelTiming> t_event_pool;  // events ready for reuse

// Runs launch() bracketed by events when timing is on.
template <class F>
hipError_t timed(const char *name, hipStream_t s, F launch) {
    if (!g_timing) return launch();
    KernelTiming k;
    if (!t_event_pool.empty()) {
        k = t_event_pool.back();
        t_event_pool.pop_back();
    } else {
        if (hipEventCreate(&k.begin) != hipSuccess) return hipErrorOutOfMemory;
        if (hipEventCreate(&k.end) != hipSuccess) return hipErrorOutOfMemory;
    }
    k.name = name;
    hipError_t e = hipEventRecord(k.begin, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(k.end, s);
    t_timings.push_back(k);
    return e;
}

// Workspace of the calling thread's device and stream `s`.  Caller holds g_mu.
int acquire_locked(hipStream_t s, Workspace **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVB_ERR_HIP;
    *out = &g_ws[std::make_pair(dev, (uintptr_t)s)];
    return SVB_OK;
}

// At least `bytes` of decoder scratch (contents undefined).  Caller holds g_mu.
int ensure_scratch(Workspace &w, uint64_t bytes, hipStream_t s) {
    if (bytes <= w.scratch_bytes) return SVB_OK;
    uint64_t cap = 1ull << 16;
    while (cap < bytes) cap <<= 1;
    if (w.scratch) {
        if (hipStreamSynchronize(s) != hipSuccess) return SVB_ERR_HIP;
        (void)hipFree(w.scratch);
        w.scratch = nullptr;
        w.scratch_bytes = 0;
    }
    if (hipMalloc((void **)&w.scratch, cap) != hipSuccess) {
        w.scratch = nullptr;
        return SVB_ERR_NOMEM;
    }
    w.scratch_bytes = cap;
    return SVB_OK;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }
bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int zero_u64(uint64_t *p, hipStream_t s) {
    if (!p) return SVB_OK;
    return hip_status(launch_fill((uint32_t *)p, 2, 0u, s));
}

// Encoding in two passes over the values: data bytes of every segment, an
// exclusive scan of them, then each segment packed at its offset.
int do_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint32_t start, uint64_t *out_bytes,
              bool delta, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (out_bytes && !aligned8(out_bytes)) return SVB_ERR_INVALID;
    if (n == 0) return zero_u64(out_bytes, s);
    if (!in || !out || !aligned4(in)) return SVB_ERR_INVALID;
    const uint64_t segs = (n + kSegInts - 1) / kSegInts;
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    const uint64_t o_bytes = 0, o_off = up16(4 * segs), o_scan = o_off + up16(8 * segs);
    const uint64_t need = o_scan + up16(scan_scratch_bytes(segs));
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *w;
    int st = acquire_locked(s, &w);
    if (st != SVB_OK) return st;
    if ((st = ensure_scratch(*w, need, s)) != SVB_OK) return st;
    uint8_t *sc = w->scratch;
    EncodeStream e;
    e.in = in;
    e.n = n;
    e.out = out;
    e.start = start;
    uint32_t *seg_bytes = (uint32_t *)(sc + o_bytes);
    uint64_t *seg_off = (uint64_t *)(sc + o_off);
    if ((st = hip_status(timed("encode_sizes", s, [&] { return launch_encode_sizes(e, delta, seg_bytes, segs, s); }))) !=
        SVB_OK)
        return st;
    // offsets that fit 32 bits whatever the values (n below about 1.01e9) scan
    // in 32 bits: half the bytes written and read
    const bool off32 = (n + 3) / 4 + 4 * n < (1ull << 32);
    if ((st = hip_status(timed("scan_offsets", s, [&] {
             return launch_scan(seg_bytes, seg_off, segs, !off32, 0u, s, nullptr, sc + o_scan);
         }))) != SVB_OK)
        return st;
    const uint32_t *seg_off32 = off32 ? (const uint32_t *)seg_off : nullptr;
    return hip_status(timed(delta ? "encode_delta" : "encode", s,
                            [&] { return launch_encode_pack(e, delta, seg_off, segs, out_bytes, s, seg_off32); }));
}

// Decoder variant per (device, delta), once tuned or set: bit 0 = the
// zero-control variant; bit 1 (delta only) = the value sums by decoding each
// group instead of from its byte sum and corrections.  Unset: the general
// decoder, and for delta decoding the value sums chosen from the stream's mean
// bytes per group (byte sums where a group's span usually fits the staging
// area of the value-sum kernel, decoding above).
std::map<std::pair<int, int>, int> g_variant;
constexpr int kVariantZC = 1, kVariantSumsByDecoding = 2;
constexpr uint64_t kByteSumsMaxSpan = 4480;  // mean data bytes per group (staging area 4608)

int variant_choice(bool delta) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = g_variant.find(std::make_pair(dev, delta ? 1 : 0));
    return it == g_variant.end() ? -1 : it->second;
}

// Scratch layout of a decode of n integers: per group its data bytes (u32)
// and value sum (u32), per block of four groups (one workgroup of the passes
// that take a group per wave) the same two totals, the block's data offset
// (u32 when the stream is under 4 GiB, else u64) and value prefix (u32), then
// the scans' partial sums.  Group arrays hold whole blocks.
struct DecodeLayout {
    uint64_t groups, blocks, o_gbytes, o_bbytes, o_boff, o_gvsum, o_bvsum, o_bvpre, o_scan, need;
};

DecodeLayout decode_layout(uint64_t n) {
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    DecodeLayout L;
    L.groups = (n + kGroupInts - 1) / kGroupInts;
    L.blocks = (L.groups + 3) / 4;
    L.o_gbytes = 0;
    L.o_bbytes = L.o_gbytes + up16(16 * L.blocks);
    L.o_boff = L.o_bbytes + up16(4 * L.blocks);
    L.o_gvsum = L.o_boff + up16(8 * (L.blocks + 1));
    L.o_bvsum = L.o_gvsum + up16(16 * L.blocks);
    L.o_bvpre = L.o_bvsum + up16(4 * L.blocks);
    L.o_scan = L.o_bvpre + up16(4 * L.blocks);
    L.need = L.o_scan + up16(scan_scratch_bytes(L.blocks));
    return L;
}

// The decoder's launches on stream s over scratch sc (L.need bytes; nothing
// in it needs to start at any value).  Arguments are checked by the caller,
// n > 0; g_mu held.  With `timing`, launches may be bracketed by the
// per-kernel timing events.
int decode_launches(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start, uint32_t *err,
                    bool delta, hipStream_t s, int chosen, uint8_t *sc, const DecodeLayout &L, bool timing) {
    auto run = [&](const char *name, auto launch) { return hip_status(timing ? timed(name, s, launch) : launch()); };
    const uint64_t groups = L.groups;
    const bool zc = chosen > 0 && (chosen & kVariantZC) != 0;
    const bool sums_by_decoding = chosen < 0 ? (in_bytes - (n + 3) / 4) / groups > kByteSumsMaxSpan
                                             : (chosen & kVariantSumsByDecoding) != 0;
    int st;
    // data bytes of every group and block of groups, from the control stream
    GroupBytesArgs ga;
    ga.in = in;
    ga.in_bytes = in_bytes;
    ga.n = n;
    ga.groups = groups;
    ga.gbytes = (uint32_t *)(sc + L.o_gbytes);
    ga.bbytes = (uint32_t *)(sc + L.o_bbytes);
    if ((st = run("group_bytes", [&] { return launch_group_bytes(ga, s); })) != SVB_OK) return st;
    // block offsets below 2^32 (a data stream under 4 GiB) scan in 32 bits
    const bool off32 = in_bytes < (1ull << 32);
    if ((st = run("scan_offsets", [&] {
             return launch_scan(ga.bbytes, sc + L.o_boff, L.blocks, !off32, 0u, s, nullptr, sc + L.o_scan);
         })) != SVB_OK)
        return st;

    DecodeArgs a = {};
    a.in = in;
    a.in_bytes = in_bytes;
    a.n = n;
    a.out = out;
    a.err = err;
    a.groups = groups;
    a.gbytes = ga.gbytes;
    a.boff32 = off32 ? (const uint32_t *)(sc + L.o_boff) : nullptr;
    a.boff = off32 ? nullptr : (const uint64_t *)(sc + L.o_boff);
    a.gvsum = (uint32_t *)(sc + L.o_gvsum);
    a.bvsum = (uint32_t *)(sc + L.o_bvsum);
    a.bvpre = (const uint32_t *)(sc + L.o_bvpre);
    if (delta) {
        // value sum of every group and block, then start + the blocks' exclusive prefix
        if ((st = run("group_sums", [&] {
                 return sums_by_decoding ? launch_decode(a, kSums, s, zc) : launch_group_sums(a, s);
             })) != SVB_OK)
            return st;
        if ((st = run("scan_sums", [&] {
                 return launch_scan(a.bvsum, sc + L.o_bvpre, L.blocks, false, start, s, nullptr, sc + L.o_scan);
             })) != SVB_OK)
            return st;
    }
    return run(delta ? "decode_delta" : "decode", [&] { return launch_decode(a, delta ? kDelta : kPlain, s, zc); });
}

// Argument checks shared by the decode entry points: SVB_OK to go on, 1 for
// nothing to do (n = 0), else an error.
int check_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, const uint32_t *out, const uint32_t *err) {
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (err && !aligned4(err)) return SVB_ERR_INVALID;
    if (n == 0) return 1;
    if (!in || !out || !aligned4(out)) return SVB_ERR_INVALID;
    if (in_bytes < (n + 3) / 4) return SVB_ERR_INVALID;
    return SVB_OK;
}

// variant: -1 = the chosen variant for this kind of call, else the bits above.
int do_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start,
              uint32_t *err, bool delta, void *stream, int variant = -1) {
    hipStream_t s = (hipStream_t)stream;
    int st = check_decode(n, in, in_bytes, out, err);
    if (st != SVB_OK) return st == 1 ? SVB_OK : st;
    const DecodeLayout L = decode_layout(n);
    std::lock_guard<std::mutex> lock(g_mu);
    const int chosen = variant < 0 ? variant_choice(delta) : variant;
    Workspace *w;
    if ((st = acquire_locked(s, &w)) != SVB_OK) return st;
    if ((st = ensure_scratch(*w, L.need, s)) != SVB_OK) return st;
    return decode_launches(n, in, in_bytes, out, start, err, delta, s, chosen, w->scratch, L, true);
}

// Scratch of svb_delta_decode_noalloc: one file-scope array per device (each
// device holds its own copy for the life of the process).  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): the address each device gives for it is looked up once,
// with that device current, and kept in g_static_scratch.
constexpr uint64_t kStaticScratchBytes = 8ull << 20;  // n up to SVB_NOALLOC_MAX_N = 2^30 needs about 5 MiB
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
uint8_t *g_static_scratch[kMaxDevices] = {};

// The calling thread's device's address of `scratch`.  Caller holds g_mu.
int static_scratch_locked(uint8_t **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVB_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return SVB_ERR_INVALID;
    if (!g_static_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SVB_ERR_HIP;
        g_static_scratch[dev] = (uint8_t *)ptr;
    }
    *out = g_static_scratch[dev];
    return SVB_OK;
}

// Times the decoder variants (plain: general and zero-control; delta: those
// two with each way of taking the value sums) on the caller's stream, median
// of five calls after two untimed ones each, and keeps the fastest for this
// kind of call on the current device.
int autotune_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start, uint32_t *err,
                    bool delta, int *chosen, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SVB_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SVB_ERR_HIP;
    }
    const int nvar = delta ? 4 : 2;
    float best_ms[4] = {1e30f, 1e30f, 1e30f, 1e30f};
    int st = SVB_OK;
    for (int v = 0; v < nvar && st == SVB_OK; ++v) {
        for (int warm = 0; warm < 2 && st == SVB_OK; ++warm) st = do_decode(n, in, in_bytes, out, start, err, delta, stream, v);
        constexpr int kReps = 5;
        float times[kReps];
        for (int r = 0; r < kReps && st == SVB_OK; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK) st = do_decode(n, in, in_bytes, out, start, err, delta, stream, v);
            if (st == SVB_OK && hipEventRecord(e1, s) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK && hipEventSynchronize(e1) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK && hipEventElapsedTime(&times[r], e0, e1) != hipSuccess) st = SVB_ERR_HIP;
        }
        if (st == SVB_OK) {
            std::sort(times, times + kReps);
            best_ms[v] = times[kReps / 2];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SVB_OK) return st;
    int best = 0;
    for (int v = 1; v < nvar; ++v)
        if (best_ms[v] < best_ms[best]) best = v;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_variant[std::make_pair(dev, delta ? 1 : 0)] = best;
    }
    if (chosen) *chosen = best;
    return SVB_OK;
}

// Append without re-encoding the stored integers: the new integers are
// encoded into scratch by the single-stream encoder, then the result is
// assembled by byte copies (old control bytes, merged control bytes, old
// data, new data).
int do_append(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint64_t k, const uint32_t *vals, uint32_t prev,
              bool delta, uint8_t *out, uint64_t *out_bytes, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N || k > SVB_MAX_N || n + k > SVB_MAX_N) return SVB_ERR_INVALID;
    if (out_bytes && !aligned8(out_bytes)) return SVB_ERR_INVALID;
    const uint64_t c_old = (n + 3) / 4, c_new = (n + k + 3) / 4, c_k = (k + 3) / 4;
    if (in_bytes < c_old || (in_bytes && !in)) return SVB_ERR_INVALID;
    if (k && (!vals || !aligned4(vals))) return SVB_ERR_INVALID;
    if (!out && (in_bytes || k)) return SVB_ERR_INVALID;
    const uint64_t d_old = in_bytes - c_old;
    if (k == 0) return hip_status(launch_copy_bytes(in, out, in_bytes, nullptr, 0, out_bytes, 0, s));
    const uint64_t segs = (k + kSegInts - 1) / kSegInts;
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    const uint64_t o_tmp = 0, o_sb = up16(c_k + 4 * k), o_so = o_sb + up16(4 * segs), o_size = o_so + up16(8 * segs);
    const uint64_t o_scan = o_size + 16, need = o_scan + up16(scan_scratch_bytes(segs));
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *w;
    int st = acquire_locked(s, &w);
    if (st != SVB_OK) return st;
    if ((st = ensure_scratch(*w, need, s)) != SVB_OK) return st;
    uint8_t *sc = w->scratch;
    uint8_t *tmp = sc + o_tmp;
    uint64_t *tmp_size = (uint64_t *)(sc + o_size);
    EncodeStream e;
    e.in = vals;
    e.n = k;
    e.out = tmp;
    e.start = prev;
    uint32_t *seg_bytes = (uint32_t *)(sc + o_sb);
    uint64_t *seg_off = (uint64_t *)(sc + o_so);
    auto ok = [](hipError_t x) { return x == hipSuccess; };
    if (!ok(timed("encode_sizes", s, [&] { return launch_encode_sizes(e, delta, seg_bytes, segs, s); })) ||
        !ok(timed("scan_offsets", s, [&] { return launch_scan(seg_bytes, seg_off, segs, true, 0u, s, nullptr, sc + o_scan); })) ||
        !ok(timed(delta ? "encode_delta" : "encode", s,
                  [&] { return launch_encode_pack(e, delta, seg_off, segs, tmp_size, s); })) ||
        !ok(timed("append_copy", s, [&] { return launch_copy_bytes(in, out, n / 4, nullptr, 0, nullptr, 0, s); })) ||
        !ok(timed("append_ctrl", s, [&] { return launch_merge_ctrl(in, tmp, out, n, k, s); })) ||
        !ok(timed("append_copy", s,
                  [&] { return launch_copy_bytes(in + c_old, out + c_new, d_old, nullptr, 0, nullptr, 0, s); })) ||
        !ok(timed("append_copy", s, [&] {
            return launch_copy_bytes(tmp + c_k, out + c_new + d_old, 4 * k, tmp_size, c_k, out_bytes, c_new + d_old, s);
        })))
        return SVB_ERR_HIP;
    return SVB_OK;
}

// ---------------------------------------------------------------- batched calls

// Tasks (segments) per wave of the main pass, per (device, kind); kind = 2 encode + delta.
std::map<std::pair<int, int>, uint32_t> g_chunk;
constexpr uint32_t kDefaultChunk = 4;
constexpr uint32_t kQueueBit = SVB_BATCH_QUEUE;  // the decode walk's work-queue schedule
constexpr uint32_t kChunkChoices[] = {1, 2, 4, 8, 16};
constexpr uint32_t kQueueChoices[] = {kQueueBit | 1, kQueueBit | 2, kQueueBit | 4, kQueueBit | 8};

bool valid_chunk(uint32_t c) {
    const uint32_t k = c & ~kQueueBit;
    return k == 1 || k == 2 || k == 4 || k == 8 || k == 16;
}

uint32_t tuned_chunk(int kind) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = g_chunk.find(std::make_pair(dev, kind));
    return it == g_chunk.end() ? kDefaultChunk : it->second;
}

struct BatchCall {
    bool encode;
    uint32_t m;
    const uint64_t *counts, *in_off, *in_bytes;
    const void *in;
    const uint64_t *out_off;
    void *out;
    uint64_t *out_bytes;
    const uint32_t *starts;
    uint64_t total_ints;
    uint32_t *err;
};

// Scratch layout of a batched call over at most T tasks and M lists.
struct BatchLayout {
    uint64_t o_litems, o_lbase, o_ilist, o_ifirst, o_ibytes, o_ioff, o_ivsum, o_ivpre, o_desc, o_queue, o_scan, need;
};

BatchLayout batch_layout(uint64_t M, uint64_t T) {
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    BatchLayout L;
    L.o_litems = 0;
    L.o_lbase = L.o_litems + up16(4 * M);
    L.o_ilist = L.o_lbase + up16(4 * (M + 1));
    L.o_ifirst = L.o_ilist + up16(4 * T);
    L.o_ibytes = L.o_ifirst + up16(4 * T);
    L.o_ioff = L.o_ibytes + up16(4 * T);
    L.o_ivsum = L.o_ioff + up16(8 * T);
    L.o_ivpre = L.o_ivsum + up16(4 * T);
    L.o_desc = (L.o_ivpre + up16(4 * T) + 63) & ~63ull;
    L.o_queue = L.o_desc + 64 * T;
    L.o_scan = L.o_queue + 16;
    L.need = L.o_scan + up16(std::max(scan_scratch_bytes(M), scan_scratch_bytes(T)));
    return L;
}

// Argument checks shared by the batched calls; t_cap receives the task bound.
// Only a task index (no_out) comes without an output.
int check_batch(const BatchCall &c, bool no_out, uint64_t *t_cap) {
    if (c.m >= (1u << 31)) return SVB_ERR_INVALID;
    if (!c.counts || !c.in_off || !c.in) return SVB_ERR_INVALID;
    if (no_out ? (c.out || c.out_off || c.encode) : (!c.out || !c.out_off)) return SVB_ERR_INVALID;
    if (!c.encode && !c.in_bytes) return SVB_ERR_INVALID;
    if (!aligned8(c.counts) || !aligned8(c.in_off) || (c.out_off && !aligned8(c.out_off))) return SVB_ERR_INVALID;
    if ((c.in_bytes && !aligned8(c.in_bytes)) || (c.out_bytes && !aligned8(c.out_bytes))) return SVB_ERR_INVALID;
    if ((c.starts && !aligned4(c.starts)) || (c.err && !aligned4(c.err))) return SVB_ERR_INVALID;
    if (c.encode ? !aligned4(c.in) : (c.out && !aligned4(c.out))) return SVB_ERR_INVALID;
    const uint64_t t = (uint64_t)c.m + (c.total_ints + kSegInts - 1) / kSegInts;
    if (c.total_ints > (1ull << 50) || t >= (1ull << 31)) return SVB_ERR_INVALID;
    *t_cap = t;
    return SVB_OK;
}

// Builds the task table of a batched call in scratch `sc` (laid out by
// batch_layout): tasks, byte offsets, descriptors, and for delta decoding the
// carries.  Leaves `a` ready for the walk.
int prepare_batch(const BatchCall &c, uint32_t C, uint64_t T, uint8_t *sc, BatchArgs &a, hipStream_t s) {
    const bool delta = c.starts != nullptr;
    const uint64_t M = c.m;
    const BatchLayout L = batch_layout(M, T);
    a = BatchArgs{};
    a.m = c.m;
    a.counts = c.counts;
    a.in_off = c.in_off;
    a.in_bytes = c.encode ? nullptr : c.in_bytes;
    a.in8 = c.encode ? nullptr : (const uint8_t *)c.in;
    a.in32 = c.encode ? (const uint32_t *)c.in : nullptr;
    a.out_off = c.out_off;
    a.out32 = c.encode ? nullptr : (uint32_t *)c.out;
    a.out8 = c.encode ? (uint8_t *)c.out : nullptr;
    a.out_bytes = c.encode ? c.out_bytes : nullptr;
    a.starts = c.starts;
    a.err = c.encode ? nullptr : c.err;
    a.litems = (uint32_t *)(sc + L.o_litems);
    a.lbase = (uint32_t *)(sc + L.o_lbase);
    a.item_list = (uint32_t *)(sc + L.o_ilist);
    a.item_first = (uint32_t *)(sc + L.o_ifirst);
    a.t_cap = (uint32_t)T;
    a.chunk = C & ~kQueueBit;
    a.queue = (C & kQueueBit) && !c.encode ? (uint32_t *)(sc + L.o_queue) : nullptr;
    a.ibytes = (uint32_t *)(sc + L.o_ibytes);
    a.ioff = (uint64_t *)(sc + L.o_ioff);
    a.ivsum = (uint32_t *)(sc + L.o_ivsum);
    a.ivpre = (uint32_t *)(sc + L.o_ivpre);
    a.desc = (TaskDesc *)(sc + L.o_desc);
    void *scan_scr = sc + L.o_scan;
    int st;
    auto run = [&](const char *name, int phase) {
        return hip_status(timed(name, s, [&] { return launch_batch(a, phase, c.encode, delta, s); }));
    };
    if ((st = run("batch_count", kBatchCount)) != SVB_OK) return st;
    if ((st = hip_status(timed("batch_scan_lists", s, [&] {
             return launch_scan(a.litems, a.lbase, M, false, 0u, s, a.lbase + M, scan_scr);
         }))) != SVB_OK)
        return st;
    if (c.encode && (st = run("batch_map", kBatchMap)) != SVB_OK) return st;
    if ((st = run(c.encode ? "batch_task_bytes" : "batch_map_bytes", kBatchItemBytes)) != SVB_OK) return st;
    if ((st = hip_status(timed("batch_scan_offsets", s, [&] {
             return launch_scan(a.ibytes, a.ioff, T, true, 0u, s, nullptr, scan_scr);
         }))) != SVB_OK)
        return st;
    if (!c.encode && delta) {
        if ((st = run("batch_task_sums", kBatchItemSums)) != SVB_OK) return st;
        if ((st = hip_status(timed("batch_scan_sums", s, [&] {
                 return launch_scan(a.ivsum, a.ivpre, T, false, 0u, s, nullptr, scan_scr);
             }))) != SVB_OK)
            return st;
    }
    if (a.queue && (st = hip_status(launch_fill(a.queue, 1, 0u, s))) != SVB_OK) return st;
    // descriptors last: for delta decoding they carry each task's running sum
    return run("batch_desc", kBatchDesc);
}

// chunk = 0: the tuned choice for this kind of call.
int do_batch(const BatchCall &c, uint32_t chunk, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (c.m == 0) return SVB_OK;
    uint64_t T = 0;
    int st = check_batch(c, false, &T);
    if (st != SVB_OK) return st;
    const bool delta = c.starts != nullptr;
    const int kind = 2 * (c.encode ? 1 : 0) + (delta ? 1 : 0);
    std::lock_guard<std::mutex> lock(g_mu);
    const uint32_t C = chunk ? chunk : tuned_chunk(kind);
    if (!valid_chunk(C)) return SVB_ERR_INVALID;
    Workspace *w;
    if ((st = acquire_locked(s, &w)) != SVB_OK) return st;
    if ((st = ensure_scratch(*w, batch_layout(c.m, T).need, s)) != SVB_OK) return st;
    BatchArgs a;
    if ((st = prepare_batch(c, C, T, w->scratch, a, s)) != SVB_OK) return st;
    return hip_status(timed(c.encode ? "batch_encode" : "batch_decode", s,
                            [&] { return launch_batch(a, kBatchWork, c.encode, delta, s); }));
}

// Times each chunk choice on the caller's batch (median of five calls after
// two untimed ones) and keeps the fastest.
int autotune_batch(const BatchCall &c, uint32_t *chosen, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SVB_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SVB_ERR_HIP;
    }
    uint32_t best = kDefaultChunk;
    float best_ms = 1e30f;
    int st = SVB_OK;
    // static chunks for every call; the work-queue schedule for decoding
    std::vector<uint32_t> choices(std::begin(kChunkChoices), std::end(kChunkChoices));
    if (!c.encode) choices.insert(choices.end(), std::begin(kQueueChoices), std::end(kQueueChoices));
    for (uint32_t g : choices) {
        for (int warm = 0; warm < 2 && st == SVB_OK; ++warm) st = do_batch(c, g, stream);
        if (st != SVB_OK) break;
        constexpr int kReps = 5;
        float times[kReps];
        for (int r = 0; r < kReps && st == SVB_OK; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK) st = do_batch(c, g, stream);
            if (st == SVB_OK && hipEventRecord(e1, s) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK && hipEventSynchronize(e1) != hipSuccess) st = SVB_ERR_HIP;
            if (st == SVB_OK && hipEventElapsedTime(&times[r], e0, e1) != hipSuccess) st = SVB_ERR_HIP;
        }
        if (st != SVB_OK) break;
        std::sort(times, times + kReps);
        const float med = times[kReps / 2];
        if (med < best_ms) {
            best_ms = med;
            best = g;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SVB_OK) return st;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_chunk[std::make_pair(dev, 2 * (c.encode ? 1 : 0) + (c.starts ? 1 : 0))] = best;
    }
    if (chosen) *chosen = best;
    return SVB_OK;
}

}  // namespace

// Task index of a serving pool: the batched decoder's task table for every
// list of the pool, built once (descriptors with no output address, the first
// task of each list).  The caller owns *desc and *lbase (hipFree).  Returns
// SVB_ERR_INVALID if a list is corrupt (its control stream longer than its
// bytes) or too long.
int build_pool_index(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                     const uint8_t *in, const uint32_t *starts, uint64_t total_ints, TaskDesc **desc,
                     uint32_t **lbase, uint32_t *tasks, hipStream_t s) {
    *desc = nullptr;
    *lbase = nullptr;
    *tasks = 0;
    BatchCall c = {false, m, counts, in_off, in_bytes, in, nullptr, nullptr, nullptr, starts, total_ints, nullptr};
    uint64_t T = 0;
    int st = check_batch(c, true, &T);
    if (st != SVB_OK || m == 0) return m == 0 ? SVB_ERR_INVALID : st;
    const BatchLayout L = batch_layout(m, T);
    uint8_t *sc = nullptr;
    uint32_t *d_err = nullptr;
    if (hipMalloc((void **)&sc, L.need) != hipSuccess) return SVB_ERR_NOMEM;
    if (hipMalloc((void **)&d_err, 4) != hipSuccess) {
        (void)hipFree(sc);
        return SVB_ERR_NOMEM;
    }
    c.err = d_err;
    BatchArgs a;
    uint32_t h_err = 0, h_tasks = 0;
    st = hip_status(launch_fill(d_err, 1, 0u, s));
    if (st == SVB_OK) {
        std::lock_guard<std::mutex> lock(g_mu);
        st = prepare_batch(c, kDefaultChunk, T, sc, a, s);
    }
    if (st == SVB_OK && (hipMemcpyAsync(&h_tasks, a.lbase + m, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipMemcpyAsync(&h_err, d_err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        st = SVB_ERR_HIP;
    if (st == SVB_OK && (h_err != 0 || h_tasks > T)) st = SVB_ERR_INVALID;
    if (st == SVB_OK) {
        if (hipMalloc((void **)desc, 64ull * (h_tasks ? h_tasks : 1)) != hipSuccess ||
            hipMalloc((void **)lbase, 4ull * (m + 1)) != hipSuccess)
            st = SVB_ERR_NOMEM;
        else if (hipMemcpyAsync(*desc, a.desc, 64ull * h_tasks, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                 hipMemcpyAsync(*lbase, a.lbase, 4ull * (m + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess)
            st = SVB_ERR_HIP;
    }
    (void)hipFree(sc);
    (void)hipFree(d_err);
    if (st != SVB_OK) {
        if (*desc) (void)hipFree(*desc);
        if (*lbase) (void)hipFree(*lbase);
        *desc = nullptr;
        *lbase = nullptr;
        return st;
    }
    *tasks = h_tasks;
    return SVB_OK;
}

// The walk of a serving batch whose descriptors are in a.desc (tasks
// a.lbase[a.m]); chunk 0 = the tuned choice for batched decoding.
int serve_walk(BatchArgs &a, bool delta, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        a.chunk = tuned_chunk(delta ? 1 : 0) & ~kQueueBit;  // a serving batch walks on the static schedule
    }
    a.queue = nullptr;
    return hip_status(launch_batch(a, kBatchWork, false, delta, s));
}

// The comparison formats (Table 1).  Encoding: bytes per segment, a scan,
// the pack.
int do_cmp_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, int fmt, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (out_bytes && !aligned8(out_bytes)) return SVB_ERR_INVALID;
    if (n == 0) return zero_u64(out_bytes, s);
    if (!in || !out || !aligned4(in)) return SVB_ERR_INVALID;
    const uint64_t segs = (n + kSegInts - 1) / kSegInts;
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    const uint64_t o_bytes = 0, o_off = up16(4 * segs), o_scan = o_off + up16(8 * segs);
    const uint64_t need = o_scan + up16(scan_scratch_bytes(segs));
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *w;
    int st = acquire_locked(s, &w);
    if (st != SVB_OK) return st;
    if ((st = ensure_scratch(*w, need, s)) != SVB_OK) return st;
    uint8_t *sc = w->scratch;
    CmpEncodeArgs a;
    a.in = in;
    a.n = n;
    a.out = out;
    a.seg_bytes = (uint32_t *)(sc + o_bytes);
    a.seg_off = (const uint64_t *)(sc + o_off);
    a.segs = segs;
    a.out_bytes = out_bytes;
    const char *name = fmt == kFmtVByte ? "vbyte_encode" : "varintgb_encode";
    if ((st = hip_status(timed("cmp_sizes", s, [&] { return launch_cmp_encode(a, fmt, true, s); }))) != SVB_OK)
        return st;
    if ((st = hip_status(timed("scan_offsets", s, [&] {
             return launch_scan(a.seg_bytes, sc + o_off, segs, true, 0u, s, nullptr, sc + o_scan);
         }))) != SVB_OK)
        return st;
    return hip_status(timed(name, s, [&] { return launch_cmp_encode(a, fmt, false, s); }));
}

// VByte decoding: integer ends per tile, a scan of them, the decode pass.
int do_vb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (err && !aligned4(err)) return SVB_ERR_INVALID;
    if (n == 0) return SVB_OK;
    if (!in || !out || !aligned4(out)) return SVB_ERR_INVALID;
    if (in_bytes < n) return SVB_ERR_INVALID;
    const uint64_t tiles = vb_tiles(in_bytes);
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    const uint64_t o_cnt = 0, o_off = up16(4 * tiles), o_tot = o_off + up16(8 * tiles), o_scan = o_tot + 16;
    const uint64_t need = o_scan + up16(scan_scratch_bytes(tiles));
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *w;
    int st = acquire_locked(s, &w);
    if (st != SVB_OK) return st;
    if ((st = ensure_scratch(*w, need, s)) != SVB_OK) return st;
    uint8_t *sc = w->scratch;
    VbDecodeArgs a;
    a.in = in;
    a.in_bytes = in_bytes;
    a.n = n;
    a.tiles = tiles;
    a.tcount = (uint32_t *)(sc + o_cnt);
    a.toff = (const uint64_t *)(sc + o_off);
    a.total = (const uint64_t *)(sc + o_tot);
    a.out = out;
    a.err = err;
    if ((st = hip_status(timed("vbyte_ends", s, [&] { return launch_vb_decode(a, true, s); }))) != SVB_OK) return st;
    if ((st = hip_status(timed("scan_offsets", s, [&] {
             return launch_scan(a.tcount, sc + o_off, tiles, true, 0u, s, sc + o_tot, sc + o_scan);
         }))) != SVB_OK)
        return st;
    return hip_status(timed("vbyte_decode", s, [&] { return launch_vb_decode(a, false, s); }));
}

// varint-GB decoding: chunk and tile maps, supertile maps, the chain across
// supertiles and tiles, the decode pass.
int do_gb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (err && !aligned4(err)) return SVB_ERR_INVALID;
    if (n == 0) return SVB_OK;
    if (!in || !out || !aligned4(out)) return SVB_ERR_INVALID;
    if (in_bytes < n + (n + 3) / 4) return SVB_ERR_INVALID;
    const uint64_t tiles = gb_tiles(in_bytes), supers = gb_supers(tiles);
    auto up16 = [](uint64_t b) { return (b + 15) & ~15ull; };
    const uint64_t o_cmap = 0;
    const uint64_t o_tmap = o_cmap + up16(2 * 17 * 64 * tiles);
    const uint64_t o_smap = o_tmap + up16(4 * 17 * tiles);
    const uint64_t o_sentry = o_smap + up16(4 * 17 * supers);
    const uint64_t o_sbase = o_sentry + up16(4 * supers);
    const uint64_t o_tentry = o_sbase + up16(8 * supers);
    const uint64_t o_tbase = o_tentry + up16(4 * tiles);
    const uint64_t o_total = o_tbase + up16(8 * tiles);
    const uint64_t need = o_total + 16;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *w;
    int st = acquire_locked(s, &w);
    if (st != SVB_OK) return st;
    if ((st = ensure_scratch(*w, need, s)) != SVB_OK) return st;
    uint8_t *sc = w->scratch;
    GbDecodeArgs a;
    a.in = in;
    a.in_bytes = in_bytes;
    a.n = n;
    a.tiles = tiles;
    a.supers = supers;
    a.cmap = (uint16_t *)(sc + o_cmap);
    a.tmap = (uint32_t *)(sc + o_tmap);
    a.smap = (uint32_t *)(sc + o_smap);
    a.sentry = (uint32_t *)(sc + o_sentry);
    a.sbase = (uint64_t *)(sc + o_sbase);
    a.tentry = (uint32_t *)(sc + o_tentry);
    a.tbase = (uint64_t *)(sc + o_tbase);
    a.total = (uint64_t *)(sc + o_total);
    a.out = out;
    a.err = err;
    static const char *const names[] = {"varintgb_maps", "varintgb_super", "varintgb_top", "varintgb_tiles",
                                        "varintgb_decode"};
    for (int ph = kGbMap; ph <= kGbDecode; ++ph)
        if ((st = hip_status(timed(names[ph], s, [&] { return launch_gb_decode(a, ph, s); }))) != SVB_OK) return st;
    return SVB_OK;
}

}  // namespace svb

using namespace svb;

extern "C" {

uint64_t svb_control_bytes(uint64_t n) { return (n + 3) / 4; }

uint64_t svb_max_compressed_bytes(uint64_t n) { return (n + 3) / 4 + 4 * n; }

int svb_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream) {
    return do_encode(n, in, out, 0u, out_bytes, false, stream);
}

int svb_delta_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint32_t start, uint64_t *out_bytes,
                     void *stream) {
    return do_encode(n, in, out, start, out_bytes, true, stream);
}

int svb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err, void *stream) {
    return do_decode(n, in, in_bytes, out, 0u, err, false, stream);
}

int svb_delta_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start,
                     uint32_t *err, void *stream) {
    return do_decode(n, in, in_bytes, out, start, err, true, stream);
}

int svb_delta_decode_noalloc(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start,
                             uint32_t *err, void *stream) {
    int st = check_decode(n, in, in_bytes, out, err);
    if (st != SVB_OK) return st == 1 ? SVB_OK : st;
    if (n > SVB_NOALLOC_MAX_N) return SVB_ERR_INVALID;
    const DecodeLayout L = decode_layout(n);
    if (L.need > kStaticScratchBytes) return SVB_ERR_INVALID;  // not reached for n <= SVB_NOALLOC_MAX_N
    std::lock_guard<std::mutex> lock(g_mu);
    uint8_t *sc = nullptr;
    if ((st = static_scratch_locked(&sc)) != SVB_OK) return st;
    return decode_launches(n, in, in_bytes, out, start, err, true, (hipStream_t)stream, variant_choice(true), sc, L,
                           false);
}


int svb_encode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint32_t *in,
                     const uint64_t *out_off, uint8_t *out, uint64_t *out_bytes, const uint32_t *starts,
                     uint64_t total_ints, void *stream) {
    BatchCall c = {true, m, counts, in_off, nullptr, in, out_off, out, out_bytes, starts, total_ints, nullptr};
    return do_batch(c, 0, stream);
}

int svb_autotune_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start, int delta,
                        uint32_t *err, int *variant, void *stream) {
    return autotune_decode(n, in, in_bytes, out, start, err, delta != 0, variant, stream);
}

int svb_set_decode_variant(int delta, int variant) {
    if (variant < -1 || variant > (delta ? 3 : 1)) return SVB_ERR_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVB_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (variant < 0)
        g_variant.erase(std::make_pair(dev, delta ? 1 : 0));
    else
        g_variant[std::make_pair(dev, delta ? 1 : 0)] = variant;
    return SVB_OK;
}

int svb_append(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint64_t k, const uint32_t *vals, uint8_t *out,
               uint64_t *out_bytes, void *stream) {
    return do_append(n, in, in_bytes, k, vals, 0u, false, out, out_bytes, stream);
}

int svb_delta_append(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint64_t k, const uint32_t *vals, uint32_t prev,
                     uint8_t *out, uint64_t *out_bytes, void *stream) {
    return do_append(n, in, in_bytes, k, vals, prev, true, out, out_bytes, stream);
}

uint64_t svb_vbyte_max_bytes(uint64_t n) { return 5 * n; }

int svb_vbyte_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream) {
    return do_cmp_encode(n, in, out, out_bytes, kFmtVByte, stream);
}

int svb_vbyte_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err, void *stream) {
    return do_vb_decode(n, in, in_bytes, out, err, stream);
}

uint64_t svb_varintgb_max_bytes(uint64_t n) { return (n + 3) / 4 + 4 * n; }

int svb_varintgb_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream) {
    return do_cmp_encode(n, in, out, out_bytes, kFmtVarintGB, stream);
}

int svb_varintgb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err,
                        void *stream) {
    return do_gb_decode(n, in, in_bytes, out, err, stream);
}

int svb_decode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                     const uint8_t *in, const uint64_t *out_off, uint32_t *out, const uint32_t *starts,
                     uint64_t total_ints, uint32_t *err, void *stream) {
    BatchCall c = {false, m, counts, in_off, in_bytes, in, out_off, out, nullptr, starts, total_ints, err};
    return do_batch(c, 0, stream);
}

int svb_autotune_decode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                              const uint8_t *in, const uint64_t *out_off, uint32_t *out, const uint32_t *starts,
                              uint64_t total_ints, uint32_t *err, uint32_t *chunk, void *stream) {
    BatchCall c = {false, m, counts, in_off, in_bytes, in, out_off, out, nullptr, starts, total_ints, err};
    return autotune_batch(c, chunk, stream);
}

int svb_autotune_encode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint32_t *in,
                              const uint64_t *out_off, uint8_t *out, uint64_t *out_bytes, const uint32_t *starts,
                              uint64_t total_ints, uint32_t *chunk, void *stream) {
    BatchCall c = {true, m, counts, in_off, nullptr, in, out_off, out, out_bytes, starts, total_ints, nullptr};
    return autotune_batch(c, chunk, stream);
}

int svb_set_batch_chunk(int kind, uint32_t chunk) {
    if (kind < 0 || kind > 3 || !valid_chunk(chunk) || ((chunk & kQueueBit) && kind >= 2)) return SVB_ERR_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVB_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    g_chunk[std::make_pair(dev, kind)] = chunk;
    return SVB_OK;
}

const char *svb_strerror(int status) {
    switch (status) {
        case SVB_OK: return "ok";
        case SVB_ERR_INVALID: return "invalid argument";
        case SVB_ERR_CORRUPT: return "corrupt stream";
        case SVB_ERR_HIP: return "HIP runtime error";
        case SVB_ERR_NOMEM: return "out of device memory for scratch workspace";
        default: return "unknown status";
    }
}

void svb_release_workspace(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        if (kv.second.scratch) (void)hipFree(kv.second.scratch);
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
}

int svb_set_kernel_timing(int enable) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_timing = enable != 0;
    return SVB_OK;
}

int svb_kernel_times(const char **names, float *ms, int cap) {
    if (cap < 0 || (cap > 0 && (!names || !ms))) return SVB_ERR_INVALID;
    const int n = (int)t_timings.size();
    int st = n;
    for (int i = 0; i < n; ++i) {
        const KernelTiming &k = t_timings[i];
        if (i < cap && st >= 0) {
            float t = 0.f;
            if (hipEventSynchronize(k.end) != hipSuccess || hipEventElapsedTime(&t, k.begin, k.end) != hipSuccess)
                st = SVB_ERR_HIP;
            names[i] = k.name;
            ms[i] = t;
        }
        t_event_pool.push_back(k);
    }
    t_timings.clear();
    return st;
}

const char *svb_version(void) { return "svb-gfx950 0.1.0"; }

int svb_copy_u32(uint64_t n, const uint32_t *in, uint32_t *out, void *stream) {
    if (n == 0) return SVB_OK;
    if (!in || !out || !aligned4(in) || !aligned4(out)) return SVB_ERR_INVALID;
    return hip_status(launch_copy(in, out, n, (hipStream_t)stream));
}

int svb_fill_u32(uint64_t n, uint32_t *out, uint32_t value, void *stream) {
    if (n == 0) return SVB_OK;
    if (!out || !aligned4(out)) return SVB_ERR_INVALID;
    return hip_status(launch_fill(out, n, value, (hipStream_t)stream));
}

}  // extern "C"
