// Serving runtime: a pool of delta-coded (or plain) lists resident in device
// memory, queries of a few lists each, admission by output memory, and
// continuous batching over the batched decoder.
//
// When the server is created, the batched decoder's preparation passes run
// once over the whole pool and leave its task index: a 64-byte descriptor per
// segment of every list, holding the segment's byte offset and, for delta
// coding, the running sum before it.  A query's lists then need no pass over
// their control bytes before they are decoded.
//
// Each query asks for k lists; its result is the k lists decoded back to back
// into one region of a fixed output arena.  A scheduling step:
//   1. retires batches whose completion event has fired (their queries become
//      complete; the caller reads results, then releases them);
//   2. admits waiting queries in arrival order while the arena has room for
//      their output (next fit over coalesced free ranges; the first query that
//      does not fit waits, and so does everything behind it);
//   3. launches batches of the admitted queries' lists (at most
//      max_batch_lists each) on free stream slots: one copy of the batch table
//      (per list: pool list, first task, arena offset), one kernel that copies
//      the lists' index descriptors with their output addresses, and the
//      batched decoder's walk.  Batches admitted while others are still on the
//      device run alongside them.
// Host work per step is bookkeeping plus one asynchronous copy of each
// batch's table; nothing waits for the device unless the caller asks to block.
//
// The replay driver (svb_server_replay) takes a whole query trace and keeps
// the host's work per query to a few additions: the trace's list ids go to
// the device once, a batch is a run of consecutive queries whose results lie
// back to back in a ring carved from the arena, and its table (per list: first
// task, arena offset) is built on the device (serve_plan_kernel) from the
// lists' counts, which the host writes to pinned memory as it sizes each
// arriving query: the host passes three numbers per batch instead of a table
// entry per list.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <random>
#include <thread>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "svb_internal.hpp"

namespace {

using svb::BatchArgs;
using svb::ServeDescArgs;
using svb::TaskDesc;
using svb::kSegInts;

// A query in the server's slab.  Up to kInlineLists lists are kept in the
// entry itself, so a waiting query costs no heap allocation however long the
// queue grows; longer queries spill into vectors.  Entries are reused.
constexpr uint32_t kInlineLists = 8;
struct Query {
    uint64_t id;
    uint32_t k;                               // lists
    uint32_t small_lists[kInlineLists];
    uint64_t small_counts[kInlineLists];      // integers of each list (read once, at submission)
    std::vector<uint32_t> big_lists;
    std::vector<uint64_t> big_counts;
    uint32_t list(uint32_t i) const { return k <= kInlineLists ? small_lists[i] : big_lists[i]; }
    uint64_t count(uint32_t i) const { return k <= kInlineLists ? small_counts[i] : big_counts[i]; }
    uint64_t admit_ns;   // when it was admitted (steady clock)
    uint64_t ints;       // output integers
    uint64_t tasks;      // segments to decode
    uint64_t arena_off;  // in integers
    int state;           // 0 waiting, 1 admitted, 2 on the device, 3 complete
    bool external;       // submitted through svb_server_submit (else by the replay driver)
};

// One stream slot: a batch in flight and the buffers it owns.  The batch
// table holds, per batch list, its pool list and arena offset, and the first
// task of each list (plus the task total).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t seq = 0;  // launch order of the batch in flight
    std::vector<uint32_t> queries;  // slab entries of the batch in flight
    uint32_t cap = 0;             // lists the table holds
    uint8_t *h_table = nullptr;   // pinned host copy
    uint8_t *d_table = nullptr;
    uint64_t task_cap = 0;        // descriptors d_desc holds
    TaskDesc *d_desc = nullptr;
    uint32_t *d_err = nullptr;
};

// Table layout for a batch of `cap` lists, packed so that one copy of
// table_bytes(lists) moves exactly the batch's entries: list ids (u32), task
// bases (u32, lists + 1), arena offsets (u64, 8-byte aligned).
size_t table_lists_off(uint32_t) { return 0; }
size_t table_base_off(uint32_t cap) { return 4ull * cap; }
size_t table_out_off(uint32_t cap) { return (4ull * cap + 4ull * (cap + 1) + 7) & ~7ull; }
size_t table_bytes(uint32_t cap) { return table_out_off(cap) + 8ull * cap; }

struct Server {
    int device = 0;
    uint32_t m = 0;
    std::vector<uint64_t> counts;  // host copy of the pool's list lengths
    std::vector<uint32_t> counts32;  // the same, saturated at 2^32 - 1 (half the cache footprint)
    bool delta = false;
    TaskDesc *pool_desc = nullptr;  // task index of the pool
    uint32_t *pool_lbase = nullptr;
    uint32_t *arena = nullptr;
    uint64_t arena_ints = 0;
    // Free ranges of the arena (offset -> length, integers), coalesced on
    // release.  Allocation is next fit: the search starts where the previous
    // allocation ended, so results admitted in order and released in about
    // that order find their space at once, and a result held out of order only
    // leaves a hole that later allocations can still use.
    std::map<uint64_t, uint64_t> free_ranges;
    uint64_t rover = 0;
    uint64_t free_ints = 0;      // sum of the free ranges
    bool admit_blocked = false;  // the front query did not fit, and nothing was released since
    std::deque<Query> slab;  // entries never move as it grows
    std::vector<uint32_t> free_entries;
    std::unordered_map<uint64_t, uint32_t> by_id;  // live queries of svb_server_submit
    std::deque<uint32_t> waiting, admitted;        // slab entries, arrival order
    std::deque<uint32_t> completed;                // complete, not polled (svb_server_submit)
    std::deque<uint32_t> completed_replay;         // complete (replay driver)
    std::vector<Slot> slots;
    uint32_t max_batch_lists = 0;
    // Batching policy: with a batch on the device, the next one waits until
    // min_batch_lists lists are admitted or its oldest query has waited
    // max_wait_ns; with none on the device it leaves at once.
    uint32_t min_batch_lists = 1024;
    uint64_t max_wait_ns = 20000;
    uint64_t admitted_lists = 0;
    uint64_t stats[8] = {};  // batches, lists, integers, queries admitted, queries completed, peak slots busy,
                             // corrupt batches, arena peak integers in use
    uint64_t in_use = 0;
    uint64_t launches = 0;
    uint64_t steps = 0, slow_steps = 0, max_step_ns = 0;  // host time of scheduling steps (slow: > 1 ms)
    std::mutex mu;
};

// Next fit: the free range holding the rover (or the first after it, then
// the first from the start) that has room for n; end() if none.
std::map<uint64_t, uint64_t>::iterator arena_find(Server &s, uint64_t n) {
    if (n > s.free_ints) return s.free_ranges.end();
    auto start = s.free_ranges.upper_bound(s.rover);
    if (start != s.free_ranges.begin()) {
        auto prev = std::prev(start);
        if (prev->first + prev->second > s.rover) start = prev;
    }
    for (auto it = start; it != s.free_ranges.end(); ++it)
        if (it->second >= n) return it;
    for (auto it = s.free_ranges.begin(); it != start; ++it)
        if (it->second >= n) return it;
    return s.free_ranges.end();
}

void arena_free(Server &s, uint64_t off, uint64_t n) {
    if (n == 0) return;
    s.in_use -= n;
    s.free_ints += n;
    s.admit_blocked = false;
    auto it = s.free_ranges.emplace(off, n).first;
    auto next = std::next(it);
    if (next != s.free_ranges.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s.free_ranges.erase(next);
    }
    if (it != s.free_ranges.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s.free_ranges.erase(it);
        }
    }
}

int ensure_slot_capacity(Slot &sl, uint32_t lists, uint64_t tasks) {
    if (lists > sl.cap) {
        const uint32_t cap = lists;
        if (sl.h_table) (void)hipHostFree(sl.h_table);
        if (sl.d_table) (void)hipFree(sl.d_table);
        sl.h_table = nullptr;
        sl.d_table = nullptr;
        sl.cap = 0;
        if (hipHostMalloc((void **)&sl.h_table, table_bytes(cap), hipHostMallocDefault) != hipSuccess)
            return SVB_ERR_NOMEM;
        if (hipMalloc((void **)&sl.d_table, table_bytes(cap)) != hipSuccess) return SVB_ERR_NOMEM;
        sl.cap = cap;
    }
    if (tasks > sl.task_cap) {
        const uint64_t cap = tasks;
        if (sl.d_desc) (void)hipFree(sl.d_desc);
        sl.d_desc = nullptr;
        sl.task_cap = 0;
        if (hipMalloc((void **)&sl.d_desc, sizeof(TaskDesc) * cap) != hipSuccess) return SVB_ERR_NOMEM;
        sl.task_cap = cap;
    }
    return SVB_OK;
}

// Retires finished batches.  block: wait for the oldest busy slot if none has finished.
int retire(Server &s, bool block) {
    bool any = false;
    for (int pass = 0; pass < 2 && !any; ++pass) {
        for (Slot &sl : s.slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return SVB_ERR_HIP;
            for (uint32_t e : sl.queries) {
                s.slab[e].state = 3;
                (s.slab[e].external ? s.completed : s.completed_replay).push_back(e);
                s.stats[4]++;
            }
            sl.queries.clear();
            sl.busy = false;
            any = true;
        }
        if (any || !block) break;
        // nothing finished: wait for the oldest batch on the device
        Slot *oldest = nullptr;
        for (Slot &sl : s.slots)
            if (sl.busy && (!oldest || sl.seq < oldest->seq)) oldest = &sl;
        if (!oldest) break;
        if (hipEventSynchronize(oldest->done) != hipSuccess) return SVB_ERR_HIP;
    }
    return SVB_OK;
}

// Admits waiting queries in arrival order.  Consecutive queries are carved
// out of one free range one after the other, so the free-range map changes
// once per range, not once per query.
uint64_t steady_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void admit(Server &s) {
    if (s.admit_blocked) return;  // the arena has not changed since the front query failed to fit
    if (s.waiting.empty()) return;
    const uint64_t now = steady_ns();
    while (!s.waiting.empty()) {
        auto it = s.free_ranges.end();
        if (s.slab[s.waiting.front()].ints) {
            it = arena_find(s, s.slab[s.waiting.front()].ints);
            if (it == s.free_ranges.end()) {
                s.admit_blocked = true;
                break;
            }
        }
        const uint64_t off = it == s.free_ranges.end() ? 0 : it->first;
        const uint64_t end = it == s.free_ranges.end() ? 0 : it->first + it->second;
        uint64_t pos = off;
        // the front query fits; so may the ones behind it
        while (!s.waiting.empty()) {
            const uint32_t e = s.waiting.front();
            Query &q = s.slab[e];
            if (q.ints > end - pos) break;
            q.arena_off = q.ints ? pos : 0;
            pos += q.ints;
            q.state = 1;
            q.admit_ns = now;
            s.admitted_lists += q.k;
            s.admitted.push_back(e);
            s.waiting.pop_front();
            s.stats[3]++;
            if (it == s.free_ranges.end() && !s.waiting.empty() && s.slab[s.waiting.front()].ints) break;
        }
        if (it != s.free_ranges.end()) {
            s.free_ranges.erase(it);
            if (end > pos) s.free_ranges.emplace(pos, end - pos);
            s.rover = pos;
            s.free_ints -= pos - off;
            s.in_use += pos - off;
            s.stats[7] = std::max(s.stats[7], s.in_use);
        }
    }
}

// Slots whose batch is still running on the device (its completion event
// has not fired), counting `self` (just launched) once: the most seen at a
// launch is the peak of batches on the device together.
uint64_t running_slots(Server &s, const Slot *self) {
    uint64_t n = 1;
    for (Slot &sl : s.slots)
        if (&sl != self && sl.busy && hipEventQuery(sl.done) == hipErrorNotReady) ++n;
    return n;
}

int launch_one(Server &s, bool *launched);

// Launches batches of the admitted queries on free slots while the batching
// policy lets them leave.
int launch(Server &s) {
    bool more = true;
    while (more) {
        const int st = launch_one(s, &more);
        if (st != SVB_OK) return st;
    }
    return SVB_OK;
}

int launch_one(Server &s, bool *launched) {
    *launched = false;
    if (s.admitted.empty()) return SVB_OK;
    Slot *slot = nullptr;
    bool busy = false;
    for (Slot &sl : s.slots) {
        if (!sl.busy && !slot) slot = &sl;
        busy |= sl.busy;
    }
    if (!slot) return SVB_OK;
    // with work on the device, let a small batch grow for a while
    if (busy && s.admitted_lists < s.min_batch_lists &&
        steady_ns() - s.slab[s.admitted.front()].admit_ns < s.max_wait_ns)
        return SVB_OK;
    // take admitted queries in order while their lists fit the batch limit
    size_t take = 0;
    uint32_t lists = 0;
    uint64_t tasks = 0;
    while (take < s.admitted.size()) {
        const Query &q = s.slab[s.admitted[take]];
        const uint32_t k = q.k;
        if (take > 0 && lists + k > s.max_batch_lists) break;
        lists += k;
        tasks += q.tasks;
        ++take;
    }
    s.admitted_lists -= lists;
    int st = ensure_slot_capacity(*slot, lists, tasks);
    if (st != SVB_OK) return st;
    const uint32_t cap = lists;  // the table is laid out for exactly this batch
    uint32_t *h_list = (uint32_t *)(slot->h_table + table_lists_off(cap));
    uint32_t *h_base = (uint32_t *)(slot->h_table + table_base_off(cap));
    uint64_t *h_out = (uint64_t *)(slot->h_table + table_out_off(cap));
    uint32_t j = 0, t = 0;
    uint64_t total = 0;
    slot->queries.assign(s.admitted.begin(), s.admitted.begin() + take);
    for (uint32_t e : slot->queries) {
        Query &q = s.slab[e];
        uint64_t o = q.arena_off;
        const uint32_t k = q.k;
        for (uint32_t i = 0; i < k; ++i) {
            const uint64_t c = q.count(i);
            h_list[j] = q.list(i);
            h_base[j] = t;
            h_out[j] = o;
            o += c;
            t += (uint32_t)((c + kSegInts - 1) / kSegInts);
            ++j;
        }
        total += q.ints;
        q.state = 2;
    }
    h_base[j] = t;
    s.admitted.erase(s.admitted.begin(), s.admitted.begin() + take);
    if (hipMemcpyAsync(slot->d_table, slot->h_table, table_bytes(cap), hipMemcpyHostToDevice, slot->stream) !=
        hipSuccess)
        return SVB_ERR_HIP;
    ServeDescArgs d;
    d.m = j;
    d.list = (const uint32_t *)(slot->d_table + table_lists_off(cap));
    d.base = (const uint32_t *)(slot->d_table + table_base_off(cap));
    d.out_off = (const uint64_t *)(slot->d_table + table_out_off(cap));
    d.pool_desc = s.pool_desc;
    d.pool_lbase = s.pool_lbase;
    d.arena = s.arena;
    d.desc = slot->d_desc;
    if (svb::launch_serve_desc(d, t, slot->stream) != hipSuccess) return SVB_ERR_HIP;
    BatchArgs a = {};
    a.m = j;
    a.lbase = (uint32_t *)d.base;
    a.t_cap = t;
    a.desc = slot->d_desc;
    a.err = slot->d_err;
    if (t && (st = svb::serve_walk(a, s.delta, slot->stream)) != SVB_OK) return st;
    if (hipEventRecord(slot->done, slot->stream) != hipSuccess) return SVB_ERR_HIP;
    slot->busy = true;
    slot->seq = s.launches++;
    s.stats[0]++;
    s.stats[1] += j;
    s.stats[2] += total;
    s.stats[5] = std::max(s.stats[5], running_slots(s, slot));
    *launched = true;
    return SVB_OK;
}

// Queues a query; `external` ones are registered under their id for
// svb_server_poll / svb_server_release.  *entry receives its slab entry.
int submit_locked(Server &s, uint64_t query_id, uint32_t k, const uint32_t *list_ids, bool external,
                  uint32_t *entry) {
    if (external && s.by_id.count(query_id)) return SVB_ERR_INVALID;
    if (k > s.max_batch_lists) return SVB_ERR_INVALID;  // could never be admitted
    for (uint32_t i = 0; i < k; ++i)
        if (list_ids[i] >= s.m) return SVB_ERR_INVALID;
    uint32_t e;
    if (!s.free_entries.empty()) {
        e = s.free_entries.back();
        s.free_entries.pop_back();
    } else {
        e = (uint32_t)s.slab.size();
        s.slab.emplace_back();
    }
    Query &q = s.slab[e];
    q.id = query_id;
    q.k = k;
    uint32_t *ql = q.small_lists;
    uint64_t *qc = q.small_counts;
    if (k > kInlineLists) {
        q.big_lists.resize(k);
        q.big_counts.resize(k);
        ql = q.big_lists.data();
        qc = q.big_counts.data();
    }
    uint64_t ints = 0, tasks = 0;
    for (uint32_t i = 0; i < k; ++i) {
        const uint64_t c = s.counts[list_ids[i]];
        ql[i] = list_ids[i];
        qc[i] = c;
        ints += c;
        tasks += (c + kSegInts - 1) / kSegInts;
    }
    if (ints > s.arena_ints) {  // could never be admitted
        q.state = -1;
        s.free_entries.push_back(e);
        return SVB_ERR_INVALID;
    }
    q.ints = ints;
    q.tasks = tasks;
    q.arena_off = 0;
    q.state = 0;
    q.external = external;
    if (external) s.by_id.emplace(query_id, e);
    s.waiting.push_back(e);
    if (entry) *entry = e;
    return SVB_OK;
}

// Frees a complete query's arena range and slab entry.
void finish_query(Server &s, uint32_t e) {
    Query &q = s.slab[e];
    arena_free(s, q.arena_off, q.ints);
    if (q.external) s.by_id.erase(q.id);
    q.state = -1;
    s.free_entries.push_back(e);
}

// One scheduling step (see svb_server_step).  With block, waits for a batch
// if `watch` (a completion queue) is empty.
int step_locked(Server &s, bool block, const std::deque<uint32_t> &watch) {
    typedef std::chrono::steady_clock clock;
    const clock::time_point t0 = clock::now();
    int st = retire(s, false);
    if (st != SVB_OK) return st;
    admit(s);
    if ((st = launch(s)) != SVB_OK) return st;
    const uint64_t ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clock::now() - t0).count();
    s.steps++;
    if (ns > 1000000) s.slow_steps++;
    s.max_step_ns = std::max(s.max_step_ns, ns);
    if (block && watch.empty()) {
        if ((st = retire(s, true)) != SVB_OK) return st;
        admit(s);
        if ((st = launch(s)) != SVB_OK) return st;
    }
    return SVB_OK;
}

void destroy(Server *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_table) (void)hipHostFree(sl.h_table);
        if (sl.d_table) (void)hipFree(sl.d_table);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
        if (sl.d_err) (void)hipFree(sl.d_err);
    }
    if (s->arena) (void)hipFree(s->arena);
    if (s->pool_desc) (void)hipFree(s->pool_desc);
    if (s->pool_lbase) (void)hipFree(s->pool_lbase);
    delete s;
}

// One batch of a replayed trace on `slot`: its table built on the device from
// the lists' counts (pinned host memory) and ids (device memory), the lists'
// descriptors copied with their output addresses (results back to back from
// arena offset out_base, in integers), the walk, and the slot's completion
// event.
int launch_trace_batch(Server &s, Slot *slot, uint32_t nlists, const uint32_t *h_counts, const uint32_t *d_ids,
                       uint64_t out_base, uint64_t tasks) {
    uint32_t *d_base = (uint32_t *)(slot->d_table + table_base_off(slot->cap));
    uint64_t *d_out = (uint64_t *)(slot->d_table + table_out_off(slot->cap));
    svb::ServePlanArgs pa;
    pa.m = nlists;
    pa.counts = h_counts;
    pa.out_base = out_base;
    pa.base = d_base;
    pa.out_off = d_out;
    ServeDescArgs d;
    d.m = nlists;
    d.list = d_ids;
    d.base = d_base;
    d.out_off = d_out;
    d.pool_desc = s.pool_desc;
    d.pool_lbase = s.pool_lbase;
    d.arena = s.arena;
    d.desc = slot->d_desc;
    BatchArgs a = {};
    a.m = nlists;
    a.lbase = d_base;
    a.t_cap = tasks;
    a.desc = slot->d_desc;
    a.err = slot->d_err;
    if (svb::launch_serve_plan(pa, slot->stream) != hipSuccess ||
        svb::launch_serve_desc(d, (uint32_t)tasks, slot->stream) != hipSuccess)
        return SVB_ERR_HIP;
    int st = SVB_OK;
    if (tasks) st = svb::serve_walk(a, s.delta, slot->stream);
    if (st == SVB_OK && hipEventRecord(slot->done, slot->stream) != hipSuccess) st = SVB_ERR_HIP;
    return st;
}

}  // namespace

extern "C" {

int svb_server_create(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                      const uint8_t *in, const uint32_t *starts, uint64_t arena_bytes, uint32_t streams,
                      uint32_t max_batch_lists, void **server) {
    if (!server || m == 0 || !counts || !in_off || !in_bytes || !in || arena_bytes < 4 || streams == 0 ||
        streams > 16 || max_batch_lists == 0)
        return SVB_ERR_INVALID;
    Server *s = new Server();
    (void)hipGetDevice(&s->device);
    s->m = m;
    s->counts.resize(m);
    s->delta = starts != nullptr;
    int st = SVB_OK;
    if (hipMemcpy(s->counts.data(), counts, 8ull * m, hipMemcpyDeviceToHost) != hipSuccess) st = SVB_ERR_HIP;
    s->counts32.resize(m);
    for (uint32_t i = 0; i < m; ++i) s->counts32[i] = (uint32_t)std::min<uint64_t>(s->counts[i], 0xFFFFFFFFull);
    uint64_t total = 0, tasks = 0;
    for (uint64_t c : s->counts) {
        total += c;
        tasks += (c + kSegInts - 1) / kSegInts;
    }
    s->arena_ints = arena_bytes / 4;
    if (st == SVB_OK && hipMalloc((void **)&s->arena, s->arena_ints * 4) != hipSuccess) st = SVB_ERR_NOMEM;
    if (st == SVB_OK) {
        s->free_ranges.emplace(0, s->arena_ints);
        s->free_ints = s->arena_ints;
    }
    s->max_batch_lists = max_batch_lists;
    s->slots.resize(streams);
    for (Slot &sl : s->slots) {
        if (st != SVB_OK) break;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.d_err, 4) != hipSuccess || hipMemset(sl.d_err, 0, 4) != hipSuccess)
            st = SVB_ERR_HIP;
    }
    // each slot's table and descriptors at their largest (a batch holds at
    // most max_batch_lists lists and an arena's worth of integers), so no
    // allocation ever happens between batches
    for (Slot &sl : s->slots) {
        if (st != SVB_OK) break;
        st = ensure_slot_capacity(sl, max_batch_lists, (uint64_t)max_batch_lists + s->arena_ints / kSegInts + 1);
    }
    // the pool's task index: byte offset and carry of every segment of every
    // list, computed once; a corrupt or oversized list refuses the pool
    uint32_t index_tasks = 0;
    if (st == SVB_OK)
        st = svb::build_pool_index(m, counts, in_off, in_bytes, in, starts, total, &s->pool_desc, &s->pool_lbase,
                                   &index_tasks, s->slots[0].stream);
    if (st == SVB_OK && index_tasks != tasks) st = SVB_ERR_INVALID;
    if (st != SVB_OK) {
        destroy(s);
        return st;
    }
    *server = s;
    return SVB_OK;
}

int svb_server_submit(void *server, uint64_t query_id, uint32_t k, const uint32_t *list_ids) {
    Server *s = (Server *)server;
    if (!s || k == 0 || !list_ids) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    return submit_locked(*s, query_id, k, list_ids, true, nullptr);
}

int svb_server_step(void *server, int block) {
    Server *s = (Server *)server;
    if (!s) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    (void)hipSetDevice(s->device);
    const int st = step_locked(*s, block != 0, s->completed);
    if (st != SVB_OK) return st;
    return (int)std::min<size_t>(s->completed.size(), 1u << 30);
}

int svb_server_poll(void *server, uint64_t *ids, uint64_t *arena_off, uint64_t *ints, uint32_t cap) {
    Server *s = (Server *)server;
    if (!s || (cap && (!ids || !arena_off || !ints))) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    uint32_t n = 0;
    while (n < cap && !s->completed.empty()) {
        const Query &q = s->slab[s->completed.front()];
        s->completed.pop_front();
        ids[n] = q.id;
        arena_off[n] = q.arena_off;
        ints[n] = q.ints;
        ++n;
    }
    return (int)n;
}

int svb_server_release(void *server, uint64_t query_id) {
    Server *s = (Server *)server;
    if (!s) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->by_id.find(query_id);
    if (it == s->by_id.end() || s->slab[it->second].state != 3) return SVB_ERR_INVALID;
    finish_query(*s, it->second);
    return SVB_OK;
}

constexpr uint64_t kBatchIntsMax = 0xFFFFFFFFull;  // a replayed batch's table holds 32-bit offsets

int svb_server_replay(void *server, uint64_t nq, const uint64_t *qoff, const uint32_t *lists, const double *arrival_s,
                      uint32_t outstanding, double *latency_s, double *wall_s) {
    Server *s = (Server *)server;
    if (!s || !qoff || (nq && (!lists || !latency_s)) || (!arrival_s && outstanding == 0)) return SVB_ERR_INVALID;
    for (uint64_t i = 0; i < nq; ++i)
        if (qoff[i + 1] <= qoff[i] || qoff[i + 1] - qoff[i] > s->max_batch_lists) return SVB_ERR_INVALID;
    const uint64_t nl = nq ? qoff[nq] - qoff[0] : 0;
    for (uint64_t i = 0; i < nl; ++i)
        if (lists[qoff[0] + i] >= s->m) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    (void)hipSetDevice(s->device);
    if (!s->completed_replay.empty()) return SVB_ERR_INVALID;
    int st = SVB_OK;
    // queries of the ordinary interface queued before the replay are launched
    // first (they complete in the background and are polled as usual)
    const std::deque<uint32_t> none;
    while (!s->waiting.empty() || !s->admitted.empty()) {
        if ((st = step_locked(*s, true, none)) != SVB_OK) return st;
        if (!s->waiting.empty() && s->admitted.empty() &&
            std::none_of(s->slots.begin(), s->slots.end(), [](const Slot &sl) { return sl.busy; }))
            return SVB_ERR_NOMEM;  // the arena is held by unreleased results
    }
    // the replay's output ring: the largest free range of the arena
    auto big = s->free_ranges.end();
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it)
        if (big == s->free_ranges.end() || it->second > big->second) big = it;
    if (big == s->free_ranges.end()) return SVB_ERR_NOMEM;
    const uint64_t r0 = big->first, R = big->second;
    s->free_ranges.erase(big);
    s->free_ints -= R;
    const uint64_t in_use_before = s->in_use;
    // the trace's list ids on the device (the descriptor copy reads them), and
    // the lists' counts in pinned host memory, written as queries arrive and
    // read by the kernel that builds a batch's table
    uint32_t *d_lists = nullptr, *h_cnt = nullptr;
    if (nl && hipMalloc((void **)&d_lists, 4 * nl) != hipSuccess) st = SVB_ERR_NOMEM;
    if (st == SVB_OK && nl && hipHostMalloc((void **)&h_cnt, 4 * nl, hipHostMallocDefault) != hipSuccess)
        st = SVB_ERR_NOMEM;
    if (st == SVB_OK && nl && hipMemcpy(d_lists, lists + qoff[0], 4 * nl, hipMemcpyHostToDevice) != hipSuccess)
        st = SVB_ERR_HIP;

    // Batches are contiguous runs of queries in arrival order; their results
    // lie back to back in the ring, one contiguous region per batch, freed in
    // launch order as batches complete.
    struct Batch {
        uint64_t q0, q1, off, len;
        Slot *slot;
        bool done;
    };
    std::deque<Batch> fifo;
    uint64_t head = 0;  // next free ring position (regions in use: fifo's, from fifo.front().off)
    auto ring_space = [&](uint64_t need_first, uint64_t *pos) -> uint64_t {
        if (fifo.empty()) {
            *pos = 0;
            return R;
        }
        const uint64_t tail = fifo.front().off;
        if (head > tail || (head == tail && fifo.empty())) {
            if (R - head >= need_first) {
                *pos = head;
                return R - head;
            }
            *pos = 0;
            return tail;
        }
        *pos = head;
        return tail > head ? tail - head : 0;
    };
    std::vector<uint64_t> qints(nq), qtasks(nq);
    std::vector<double> sent(nq, 0.0);
    typedef std::chrono::steady_clock clock;
    const clock::time_point t0 = clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    // A second host thread sizes the queries as they arrive (their lists'
    // lengths: result size, segments, and the counts the batch-table kernel
    // reads), while this one launches and retires batches: queries [0,
    // released) have arrived, [0, sized) are sized.
    std::atomic<uint64_t> released{0}, sized{0};
    std::atomic<bool> stop{false}, too_big{false};
    std::thread sizer([&] {
        const uint32_t *cnt = s->counts32.data();  // (prefetching a few queries ahead measured slower)
        uint64_t q = 0;
        while (q < nq && !stop.load(std::memory_order_relaxed)) {
            const uint64_t r = released.load(std::memory_order_acquire);
            if (q == r) {
                __builtin_ia32_pause();
                continue;
            }
            for (; q < r; ++q) {
                uint64_t ints = 0, tasks = 0;
                for (uint64_t i = qoff[q]; i < qoff[q + 1]; ++i) {
                    const uint32_t c = cnt[lists[i]];  // 2^32 - 1: at least that long, never admitted
                    h_cnt[i - qoff[0]] = c;
                    ints += c;
                    tasks += (c + kSegInts - 1) / kSegInts;
                }
                if (ints > R || ints >= kBatchIntsMax) {
                    too_big.store(true, std::memory_order_relaxed);
                    stop.store(true, std::memory_order_relaxed);
                    break;
                }
                qints[q] = ints;
                qtasks[q] = tasks;
                if ((q & 255) == 255) sized.store(q + 1, std::memory_order_release);
            }
            sized.store(q, std::memory_order_release);
        }
    });
    uint64_t next = 0, launched = 0, done = 0;
    while (st == SVB_OK && done < nq) {
        // arrivals: due (open loop) or room under the outstanding limit (closed loop)
        const double t = now_s();
        const uint64_t was = next;
        while (next < nq && (arrival_s ? arrival_s[next] <= t : next - done < outstanding)) {
            sent[next] = arrival_s ? arrival_s[next] : t;
            ++next;
        }
        if (next != was) released.store(next, std::memory_order_release);
        if (too_big.load(std::memory_order_relaxed)) {
            st = SVB_ERR_NOMEM;  // a query that can never be admitted
            break;
        }
        const uint64_t ready = sized.load(std::memory_order_acquire);
        s->stats[3] += next - was;
        // retire: every finished slot is free again at once (batches of
        // different sizes finish out of order); their ring regions are freed
        // in launch order
        for (Batch &b : fifo) {
            if (b.done) continue;
            const hipError_t q = hipEventQuery(b.slot->done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                st = SVB_ERR_HIP;
                break;
            }
            b.done = true;
            b.slot->busy = false;
        }
        if (st != SVB_OK) break;
        if (!fifo.empty() && fifo.front().done) {
            const double tc = now_s();
            while (!fifo.empty() && fifo.front().done) {
                const Batch &b = fifo.front();
                for (uint64_t q = b.q0; q < b.q1; ++q) latency_s[q] = tc - sent[q];
                done += b.q1 - b.q0;
                s->stats[4] += b.q1 - b.q0;
                s->in_use -= b.len;
                fifo.pop_front();
            }
            if (fifo.empty()) head = 0;
        }
        // launch: the waiting queries in order, as many as a batch and the
        // ring's free region hold, on a free slot
        bool launched_now = false;
        if (launched < ready) {
            Slot *slot = nullptr;
            bool busy = false;
            for (Slot &sl : s->slots) {
                if (!sl.busy && !slot) slot = &sl;
                busy |= sl.busy;
            }
            const uint64_t waiting_lists = qoff[ready] - qoff[launched];
            const bool hold = busy && waiting_lists < s->min_batch_lists &&
                              (t - sent[launched]) * 1e9 < (double)s->max_wait_ns;
            uint64_t pos = 0;
            const uint64_t room = slot && !hold ? ring_space(qints[launched], &pos) : 0;
            if (slot && !hold && room >= qints[launched]) {
                uint64_t b = launched, ints = 0, tasks = 0;
                while (b < ready && qoff[b + 1] - qoff[launched] <= s->max_batch_lists && ints + qints[b] <= room &&
                       ints + qints[b] <= kBatchIntsMax) {
                    ints += qints[b];
                    tasks += qtasks[b];
                    ++b;
                }
                const uint32_t nlists = (uint32_t)(qoff[b] - qoff[launched]);
                st = launch_trace_batch(*s, slot, nlists, h_cnt + (qoff[launched] - qoff[0]),
                                        d_lists + (qoff[launched] - qoff[0]), r0 + pos, tasks);
                if (st != SVB_OK) break;
                slot->busy = true;
                slot->seq = s->launches++;
                fifo.push_back(Batch{launched, b, pos, ints, slot, false});
                head = pos + ints;
                s->in_use += ints;
                s->stats[7] = std::max(s->stats[7], s->in_use);
                s->stats[0]++;
                s->stats[1] += nlists;
                s->stats[2] += ints;
                s->stats[5] = std::max(s->stats[5], running_slots(*s, slot));
                launched = b;
                launched_now = true;
            }
        }
        // closed loop with nothing more to send or launch: wait for the oldest batch
        if (!launched_now && !arrival_s && next - done >= outstanding && !fifo.empty()) {
            for (Batch &b : fifo)
                if (!b.done) {
                    if (hipEventSynchronize(b.slot->done) != hipSuccess) st = SVB_ERR_HIP;
                    break;
                }
        }
    }
    stop.store(true, std::memory_order_relaxed);
    sizer.join();
    // wait for what is still on the device (after an error), then give the ring back
    for (Batch &b : fifo)
        if (!b.done) {
            (void)hipEventSynchronize(b.slot->done);
            b.slot->busy = false;
        }
    s->in_use = in_use_before + R;  // the ring, as arena_free takes it back
    arena_free(*s, r0, R);
    if (d_lists) (void)hipFree(d_lists);
    if (h_cnt) (void)hipHostFree(h_cnt);
    if (wall_s) *wall_s = now_s();
    return st;
}

// Open loop generated in the call: query i asks for the lists of trace entry
// i mod nbase and arrives at the i-th point of a Poisson process of rate qps
// (exponential gaps from a 64-bit Mersenne twister seeded with `seed`, see
// below) until `seconds` have passed.  The trace's list ids and their counts are set up
// once, so the host's work per query is an arrival time and, at completion, a
// histogram bin; batches are runs of consecutive queries that stop at the
// trace's end.
int svb_server_replay_poisson(void *server, uint64_t nbase, const uint64_t *qoff, const uint32_t *lists, double qps,
                              double seconds, double warmup_s, uint64_t seed, double *out, uint32_t out_cap) {
    Server *s = (Server *)server;
    if (!s || !qoff || !lists || nbase == 0 || !(qps > 0.0) || !(seconds > 0.0) || !(warmup_s >= 0.0) ||
        warmup_s >= seconds || (out_cap && !out))
        return SVB_ERR_INVALID;
    for (uint64_t i = 0; i < nbase; ++i)
        if (qoff[i + 1] <= qoff[i] || qoff[i + 1] - qoff[i] > s->max_batch_lists) return SVB_ERR_INVALID;
    const uint64_t nl = qoff[nbase] - qoff[0];
    for (uint64_t i = 0; i < nl; ++i)
        if (lists[qoff[0] + i] >= s->m) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    (void)hipSetDevice(s->device);
    if (!s->completed_replay.empty()) return SVB_ERR_INVALID;
    int st = SVB_OK;
    const std::deque<uint32_t> none;
    while (!s->waiting.empty() || !s->admitted.empty()) {
        if ((st = step_locked(*s, true, none)) != SVB_OK) return st;
        if (!s->waiting.empty() && s->admitted.empty() &&
            std::none_of(s->slots.begin(), s->slots.end(), [](const Slot &sl) { return sl.busy; }))
            return SVB_ERR_NOMEM;
    }
    auto big = s->free_ranges.end();
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it)
        if (big == s->free_ranges.end() || it->second > big->second) big = it;
    if (big == s->free_ranges.end()) return SVB_ERR_NOMEM;
    const uint64_t r0 = big->first, R = big->second;
    // every trace entry sized once: output integers and segments; an entry
    // that can never be admitted refuses the call before anything runs
    std::vector<uint64_t> eints(nbase), etasks(nbase);
    const uint32_t *cnt = s->counts32.data();
    for (uint64_t e = 0; e < nbase; ++e) {
        uint64_t ints = 0, tasks = 0;
        for (uint64_t i = qoff[e]; i < qoff[e + 1]; ++i) {
            const uint32_t c = cnt[lists[i]];
            ints += c;
            tasks += (c + kSegInts - 1) / kSegInts;
        }
        if (ints > R || ints >= kBatchIntsMax) return SVB_ERR_NOMEM;
        eints[e] = ints;
        etasks[e] = tasks;
    }
    s->free_ranges.erase(big);
    s->free_ints -= R;
    const uint64_t in_use_before = s->in_use;
    uint32_t *d_lists = nullptr, *h_cnt = nullptr;
    if (hipMalloc((void **)&d_lists, 4 * nl) != hipSuccess) st = SVB_ERR_NOMEM;
    if (st == SVB_OK && hipHostMalloc((void **)&h_cnt, 4 * nl, hipHostMallocDefault) != hipSuccess)
        st = SVB_ERR_NOMEM;
    if (st == SVB_OK && hipMemcpy(d_lists, lists + qoff[0], 4 * nl, hipMemcpyHostToDevice) != hipSuccess)
        st = SVB_ERR_HIP;
    if (st == SVB_OK)
        for (uint64_t i = 0; i < nl; ++i) h_cnt[i] = cnt[lists[qoff[0] + i]];

    struct Batch {
        uint64_t q0, q1, off, len;
        Slot *slot;
        bool done;
    };
    std::deque<Batch> fifo;
    uint64_t head = 0;
    auto ring_space = [&](uint64_t need_first, uint64_t *pos) -> uint64_t {
        if (fifo.empty()) {
            *pos = 0;
            return R;
        }
        const uint64_t tail = fifo.front().off;
        if (head > tail) {
            if (R - head >= need_first) {
                *pos = head;
                return R - head;
            }
            *pos = 0;
            return tail;
        }
        *pos = head;
        return tail > head ? tail - head : 0;
    };
    // The gaps: a table of kGaps exponential draws made before the clock
    // starts, read in order from a fresh random position every kGaps queries
    // (drawing each gap as it is needed, or reading the table out of order,
    // costs the launching thread more than a query's share of its time at
    // tens of millions of queries per second).  Two walkers read the same
    // sequence: this thread's, which releases arrivals, and the accounting
    // thread's, which recomputes each query's arrival time when its batch
    // completes.
    constexpr uint64_t kGaps = 1ull << 22;
    std::mt19937_64 rng(seed);
    std::vector<double> gaps(kGaps);
    {
        std::exponential_distribution<double> draw(qps);
        for (double &g : gaps) g = draw(rng);
    }
    struct Arrivals {
        const std::vector<double> *gaps;
        std::mt19937_64 rng;
        uint64_t i = 0, rot = 0;
        double t = 0.0;  // arrival time of query i
        void start() {
            rot = rng();
            t = (*gaps)[rot & (kGaps - 1)];
        }
        void advance() {
            ++i;
            if ((i & (kGaps - 1)) == 0) rot = rng();
            t += (*gaps)[(i + rot) & (kGaps - 1)];
        }
    };
    Arrivals gen{&gaps, rng}, acc_gen{&gaps, rng};
    gen.start();
    acc_gen.start();
    // latency accounting, off this thread: completed batches (queries [q0,
    // q1), seen complete at tc) go through a single-producer ring
    constexpr uint64_t kBins = 1000000;  // 0.1 us bins up to 0.1 s, the last bin open
    constexpr double kBinS = 1e-7;
    std::vector<uint64_t> hist(kBins, 0);
    uint64_t measured = 0;
    double measured_ints = 0.0, lat_sum = 0.0, t_last = 0.0;
    struct Done {
        uint64_t q0, q1;
        double tc;
    };
    constexpr uint64_t kRing = 1 << 16;
    std::vector<Done> ring(kRing);
    std::atomic<uint64_t> produced{0}, consumed{0};
    std::atomic<bool> finished{false};
    std::thread accountant([&] {
        uint64_t c = 0;
        for (;;) {
            const uint64_t p = produced.load(std::memory_order_acquire);
            if (c == p) {
                if (finished.load(std::memory_order_acquire) && c == produced.load(std::memory_order_acquire)) break;
                __builtin_ia32_pause();
                continue;
            }
            for (; c < p; ++c) {
                const Done d = ring[c & (kRing - 1)];
                const uint64_t e_first = d.q0 % nbase;  // a batch never wraps the trace
                for (uint64_t q = d.q0; q < d.q1; ++q, acc_gen.advance()) {
                    const double ta = acc_gen.t;
                    if (ta < warmup_s) continue;
                    const double lat = d.tc - ta;
                    const uint64_t bin = (uint64_t)(lat * (1.0 / kBinS));
                    ++hist[bin < kBins ? bin : kBins - 1];
                    ++measured;
                    measured_ints += (double)eints[e_first + (q - d.q0)];
                    lat_sum += lat;
                }
                t_last = d.tc;
            }
            consumed.store(c, std::memory_order_release);
        }
    });
    // arrival times of queries [launched, next), by query number modulo
    // pend_cap: one second of arrivals, at least 2^16 and at most 2^26
    // entries (a longer backlog holds further arrivals back, their latency
    // still counted from their arrival times).  A double-ended queue here,
    // allocating and freeing as queries came and went, let the open loop fall
    // behind at 40M queries/s: p99 8-100 ms against 0.17-0.21 ms with the ring.
    uint64_t pend_cap = 1ull << 16;
    while (pend_cap < (1ull << 26) && (double)pend_cap < qps) pend_cap <<= 1;
    std::vector<double> pending(pend_cap);
    typedef std::chrono::steady_clock clock;
    const clock::time_point t0 = clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    uint64_t next = 0, launched = 0, done = 0, batches = 0, produced_here = 0;
    while (st == SVB_OK) {
        const double t = now_s();
        const uint64_t was = next;
        while (gen.t <= t && gen.t < seconds && next - launched < pend_cap) {
            pending[next & (pend_cap - 1)] = gen.t;
            ++next;
            gen.advance();
        }
        s->stats[3] += next - was;
        if (gen.t >= seconds && done == next) break;
        // retire every finished slot; free ring regions in launch order and
        // hand the batches to the accounting thread
        for (Batch &b : fifo) {
            if (b.done) continue;
            const hipError_t q = hipEventQuery(b.slot->done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                st = SVB_ERR_HIP;
                break;
            }
            b.done = true;
            b.slot->busy = false;
        }
        if (st != SVB_OK) break;
        if (!fifo.empty() && fifo.front().done) {
            const double tc = now_s();
            while (!fifo.empty() && fifo.front().done) {
                const Batch &b = fifo.front();
                while (produced_here - consumed.load(std::memory_order_acquire) >= kRing) __builtin_ia32_pause();
                ring[produced_here & (kRing - 1)] = Done{b.q0, b.q1, tc};
                produced.store(++produced_here, std::memory_order_release);
                done += b.q1 - b.q0;
                s->stats[4] += b.q1 - b.q0;
                s->in_use -= b.len;
                fifo.pop_front();
            }
            if (fifo.empty()) head = 0;
        }
        // launch the arrived queries in order, as many as a batch, the ring's
        // free region and the trace's end allow, on a free slot
        if (launched < next) {
            Slot *slot = nullptr;
            bool busy = false;
            for (Slot &sl : s->slots) {
                if (!sl.busy && !slot) slot = &sl;
                busy |= sl.busy;
            }
            const uint64_t e0 = launched % nbase;
            const uint64_t avail = std::min<uint64_t>(next - launched, nbase - e0);  // entries before the wrap
            const bool hold = busy && qoff[e0 + avail] - qoff[e0] < s->min_batch_lists &&
                              (t - pending[launched & (pend_cap - 1)]) * 1e9 < (double)s->max_wait_ns;
            uint64_t pos = 0;
            const uint64_t room = slot && !hold ? ring_space(eints[e0], &pos) : 0;
            if (slot && !hold && room >= eints[e0]) {
                uint64_t e = e0, ints = 0, tasks = 0;
                while (e < e0 + avail && qoff[e + 1] - qoff[e0] <= s->max_batch_lists && ints + eints[e] <= room &&
                       ints + eints[e] <= kBatchIntsMax) {
                    ints += eints[e];
                    tasks += etasks[e];
                    ++e;
                }
                const uint32_t nlists = (uint32_t)(qoff[e] - qoff[e0]);
                st = launch_trace_batch(*s, slot, nlists, h_cnt + (qoff[e0] - qoff[0]), d_lists + (qoff[e0] - qoff[0]),
                                        r0 + pos, tasks);
                if (st != SVB_OK) break;
                slot->busy = true;
                slot->seq = s->launches++;
                fifo.push_back(Batch{launched, launched + (e - e0), pos, ints, slot, false});
                head = pos + ints;
                s->in_use += ints;
                s->stats[7] = std::max(s->stats[7], s->in_use);
                s->stats[0]++;
                s->stats[1] += nlists;
                s->stats[2] += ints;
                s->stats[5] = std::max(s->stats[5], running_slots(*s, slot));
                launched += e - e0;
                ++batches;
            }
        }
    }
    finished.store(true, std::memory_order_release);
    accountant.join();
    for (Batch &b : fifo)
        if (!b.done) {
            (void)hipEventSynchronize(b.slot->done);
            b.slot->busy = false;
        }
    s->in_use = in_use_before + R;
    arena_free(*s, r0, R);
    if (d_lists) (void)hipFree(d_lists);
    if (h_cnt) (void)hipHostFree(h_cnt);
    if (st != SVB_OK) return st;
    auto pct = [&](double f) {
        const uint64_t want = (uint64_t)std::ceil(f * (double)measured);
        uint64_t acc = 0;
        for (uint64_t b = 0; b < kBins; ++b) {
            acc += hist[b];
            if (acc >= want && acc) return ((double)b + 0.5) * kBinS;
        }
        return 0.0;
    };
    const double wall = t_last > warmup_s ? t_last - warmup_s : 0.0;
    const double res[8] = {(double)measured, measured_ints, wall, pct(0.5), pct(0.99),
                           measured ? lat_sum / (double)measured : 0.0, (double)next, (double)batches};
    for (uint32_t i = 0; i < out_cap; ++i) out[i] = i < 8 ? res[i] : 0.0;
    return SVB_OK;
}

int svb_server_set_batching(void *server, uint32_t min_lists, uint32_t max_wait_us) {
    Server *s = (Server *)server;
    if (!s) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    s->min_batch_lists = min_lists;
    s->max_wait_ns = (uint64_t)max_wait_us * 1000;
    return SVB_OK;
}

uint32_t *svb_server_arena(void *server) { return server ? ((Server *)server)->arena : nullptr; }

int svb_server_stats(void *server, uint64_t *out, uint32_t cap) {
    Server *s = (Server *)server;
    if (!s || (cap && !out)) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    uint32_t err = 0;
    for (Slot &sl : s->slots) {
        uint32_t e = 0;
        if (!sl.busy && hipMemcpy(&e, sl.d_err, 4, hipMemcpyDeviceToHost) == hipSuccess) err |= e;
    }
    s->stats[6] = err;
    const uint64_t extra[6] = {(uint64_t)s->waiting.size(), (uint64_t)s->admitted.size(), s->in_use,
                               s->steps, s->slow_steps, s->max_step_ns / 1000};
    for (uint32_t i = 0; i < cap; ++i) out[i] = i < 8 ? s->stats[i] : (i < 14 ? extra[i - 8] : 0);
    return SVB_OK;
}

int svb_server_destroy(void *server) {
    destroy((Server *)server);
    return SVB_OK;
}

}  // extern "C"
