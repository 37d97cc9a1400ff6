// Serving runtime: a pool of delta-coded (or plain) lists resident in device
// memory, queries of a few lists each, admission by output memory, and
// continuous batching over the batched decoder.
//
// Each query asks for k lists; its result is the k lists decoded back to back
// into one region of a fixed output arena.  A scheduling step:
//   1. retires batches whose completion event has fired (their queries become
//      complete; the caller reads results, then releases them);
//   2. admits waiting queries in arrival order while the arena has room for
//      their output (first fit over free ranges; the first query that does not
//      fit waits, and so does everything behind it);
//   3. launches one batched decode of every admitted query's lists on a free
//      stream slot, so batches admitted while others are still on the device
//      run alongside them.
// Host work per step is bookkeeping plus one asynchronous copy of the batch's
// list table; nothing waits for the device unless the caller asks to block.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "svb_internal.hpp"

namespace svb {
int serve_decode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                       const uint8_t *in, const uint64_t *out_off, uint32_t *out, const uint32_t *starts,
                       uint64_t total_ints, uint32_t *err, void *stream);
}

namespace {

using svb::serve_decode_batch;

struct Query {
    uint64_t id;
    std::vector<uint32_t> lists;
    uint64_t ints;       // output integers
    uint64_t arena_off;  // in integers
    int state;           // 0 waiting, 1 admitted, 2 on the device, 3 complete
};

// One stream slot: a batch in flight and the buffers it owns.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t seq = 0;  // launch order of the batch in flight
    std::vector<uint64_t> queries;
    uint32_t cap = 0;           // lists the buffers hold
    uint64_t *h_table = nullptr;  // pinned: counts | in_off | in_bytes | out_off (4 x cap u64) + starts (cap u32)
    uint64_t *d_table = nullptr;
    uint32_t *d_err = nullptr;
};

struct Server {
    int device = 0;
    uint32_t m = 0;
    std::vector<uint64_t> counts, in_off, in_bytes;  // host copies of the pool table
    std::vector<uint32_t> starts;
    bool delta = false;
    const uint8_t *in = nullptr;
    uint32_t *arena = nullptr;
    uint64_t arena_ints = 0;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> length (integers)
    std::deque<uint64_t> waiting;
    std::vector<uint64_t> admitted;
    std::unordered_map<uint64_t, Query> queries;
    std::deque<uint64_t> completed;
    std::vector<Slot> slots;
    uint32_t max_batch_lists = 0;
    uint64_t stats[8] = {};  // batches, lists, integers, queries admitted, queries completed, peak slots busy,
                             // corrupt batches, arena peak integers in use
    uint64_t in_use = 0;
    uint64_t launches = 0;
    std::mutex mu;
};

bool arena_alloc(Server &s, uint64_t n, uint64_t *off) {
    if (n == 0) {
        *off = 0;
        return true;
    }
    for (auto it = s.free_ranges.begin(); it != s.free_ranges.end(); ++it) {
        if (it->second >= n) {
            *off = it->first;
            const uint64_t rest = it->second - n;
            const uint64_t roff = it->first + n;
            s.free_ranges.erase(it);
            if (rest) s.free_ranges[roff] = rest;
            s.in_use += n;
            s.stats[7] = std::max(s.stats[7], s.in_use);
            return true;
        }
    }
    return false;
}

void arena_free(Server &s, uint64_t off, uint64_t n) {
    if (n == 0) return;
    s.in_use -= n;
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

int ensure_slot_capacity(Slot &sl, uint32_t lists) {
    if (lists <= sl.cap) return SVB_OK;
    uint32_t cap = std::max<uint32_t>(1024, sl.cap);
    while (cap < lists) cap *= 2;
    if (sl.h_table) (void)hipHostFree(sl.h_table);
    if (sl.d_table) (void)hipFree(sl.d_table);
    sl.h_table = nullptr;
    sl.d_table = nullptr;
    sl.cap = 0;
    const size_t bytes = (size_t)cap * (4 * sizeof(uint64_t) + sizeof(uint32_t));
    if (hipHostMalloc((void **)&sl.h_table, bytes, hipHostMallocDefault) != hipSuccess) return SVB_ERR_NOMEM;
    if (hipMalloc((void **)&sl.d_table, bytes) != hipSuccess) return SVB_ERR_NOMEM;
    sl.cap = cap;
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
            for (uint64_t id : sl.queries) {
                s.queries[id].state = 3;
                s.completed.push_back(id);
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

void admit(Server &s) {
    while (!s.waiting.empty()) {
        Query &q = s.queries[s.waiting.front()];
        uint64_t off;
        if (!arena_alloc(s, q.ints, &off)) break;
        q.arena_off = off;
        q.state = 1;
        s.admitted.push_back(q.id);
        s.waiting.pop_front();
        s.stats[3]++;
    }
}

int launch(Server &s) {
    if (s.admitted.empty()) return SVB_OK;
    Slot *slot = nullptr;
    for (Slot &sl : s.slots)
        if (!sl.busy) {
            slot = &sl;
            break;
        }
    if (!slot) return SVB_OK;
    // take admitted queries in order while their lists fit the batch limit
    size_t take = 0;
    uint32_t lists = 0;
    while (take < s.admitted.size()) {
        const uint32_t k = (uint32_t)s.queries[s.admitted[take]].lists.size();
        if (take > 0 && lists + k > s.max_batch_lists) break;
        lists += k;
        ++take;
    }
    int st = ensure_slot_capacity(*slot, lists);
    if (st != SVB_OK) return st;
    const uint32_t cap = slot->cap;
    uint64_t *h_counts = slot->h_table, *h_in_off = h_counts + cap, *h_in_bytes = h_in_off + cap,
             *h_out_off = h_in_bytes + cap;
    uint32_t *h_starts = (uint32_t *)(h_out_off + cap);
    uint32_t j = 0;
    uint64_t total = 0;
    slot->queries.assign(s.admitted.begin(), s.admitted.begin() + take);
    for (uint64_t id : slot->queries) {
        Query &q = s.queries[id];
        uint64_t o = q.arena_off;
        for (uint32_t list : q.lists) {
            h_counts[j] = s.counts[list];
            h_in_off[j] = s.in_off[list];
            h_in_bytes[j] = s.in_bytes[list];
            h_out_off[j] = o;
            h_starts[j] = s.delta ? s.starts[list] : 0u;
            o += s.counts[list];
            total += s.counts[list];
            ++j;
        }
        q.state = 2;
    }
    s.admitted.erase(s.admitted.begin(), s.admitted.begin() + take);
    const size_t bytes = (size_t)cap * (4 * sizeof(uint64_t) + sizeof(uint32_t));
    if (hipMemcpyAsync(slot->d_table, slot->h_table, bytes, hipMemcpyHostToDevice, slot->stream) != hipSuccess)
        return SVB_ERR_HIP;
    uint64_t *d_counts = slot->d_table, *d_in_off = d_counts + cap, *d_in_bytes = d_in_off + cap,
             *d_out_off = d_in_bytes + cap;
    uint32_t *d_starts = (uint32_t *)(d_out_off + cap);
    st = serve_decode_batch(j, d_counts, d_in_off, d_in_bytes, s.in, d_out_off, s.arena, s.delta ? d_starts : nullptr,
                            total, slot->d_err, slot->stream);
    if (st != SVB_OK) return st;
    if (hipEventRecord(slot->done, slot->stream) != hipSuccess) return SVB_ERR_HIP;
    slot->busy = true;
    slot->seq = s.launches++;
    s.stats[0]++;
    s.stats[1] += j;
    s.stats[2] += total;
    uint64_t busy = 0;
    for (Slot &sl : s.slots) busy += sl.busy ? 1 : 0;
    s.stats[5] = std::max(s.stats[5], busy);
    return SVB_OK;
}

int submit_locked(Server &s, uint64_t query_id, uint32_t k, const uint32_t *list_ids) {
    if (s.queries.count(query_id)) return SVB_ERR_INVALID;
    Query q;
    q.id = query_id;
    q.lists.assign(list_ids, list_ids + k);
    q.ints = 0;
    for (uint32_t l : q.lists) {
        if (l >= s.m) return SVB_ERR_INVALID;
        q.ints += s.counts[l];
    }
    if (q.ints > s.arena_ints || k > s.max_batch_lists) return SVB_ERR_INVALID;  // could never be admitted
    q.arena_off = 0;
    q.state = 0;
    s.queries.emplace(query_id, std::move(q));
    s.waiting.push_back(query_id);
    return SVB_OK;
}

// One scheduling step (see svb_server_step).
int step_locked(Server &s, bool block) {
    int st = retire(s, false);
    if (st != SVB_OK) return st;
    admit(s);
    if ((st = launch(s)) != SVB_OK) return st;
    if (block && s.completed.empty()) {
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
        if (sl.d_err) (void)hipFree(sl.d_err);
    }
    if (s->arena) (void)hipFree(s->arena);
    delete s;
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
    s->in_off.resize(m);
    s->in_bytes.resize(m);
    s->delta = starts != nullptr;
    int st = SVB_OK;
    if (hipMemcpy(s->counts.data(), counts, 8ull * m, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(s->in_off.data(), in_off, 8ull * m, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(s->in_bytes.data(), in_bytes, 8ull * m, hipMemcpyDeviceToHost) != hipSuccess)
        st = SVB_ERR_HIP;
    if (st == SVB_OK && s->delta) {
        s->starts.resize(m);
        if (hipMemcpy(s->starts.data(), starts, 4ull * m, hipMemcpyDeviceToHost) != hipSuccess) st = SVB_ERR_HIP;
    }
    s->in = in;
    s->arena_ints = arena_bytes / 4;
    if (st == SVB_OK && hipMalloc((void **)&s->arena, s->arena_ints * 4) != hipSuccess) st = SVB_ERR_NOMEM;
    if (st == SVB_OK) s->free_ranges[0] = s->arena_ints;
    s->max_batch_lists = max_batch_lists;
    s->slots.resize(streams);
    for (Slot &sl : s->slots) {
        if (st != SVB_OK) break;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.d_err, 4) != hipSuccess || hipMemset(sl.d_err, 0, 4) != hipSuccess)
            st = SVB_ERR_HIP;
    }
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
    return submit_locked(*s, query_id, k, list_ids);
}

int svb_server_step(void *server, int block) {
    Server *s = (Server *)server;
    if (!s) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    (void)hipSetDevice(s->device);
    const int st = step_locked(*s, block != 0);
    if (st != SVB_OK) return st;
    return (int)std::min<size_t>(s->completed.size(), 1u << 30);
}

int svb_server_poll(void *server, uint64_t *ids, uint64_t *arena_off, uint64_t *ints, uint32_t cap) {
    Server *s = (Server *)server;
    if (!s || (cap && (!ids || !arena_off || !ints))) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    uint32_t n = 0;
    while (n < cap && !s->completed.empty()) {
        const uint64_t id = s->completed.front();
        s->completed.pop_front();
        const Query &q = s->queries[id];
        ids[n] = id;
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
    auto it = s->queries.find(query_id);
    if (it == s->queries.end() || it->second.state != 3) return SVB_ERR_INVALID;
    arena_free(*s, it->second.arena_off, it->second.ints);
    s->queries.erase(it);
    return SVB_OK;
}

int svb_server_replay(void *server, uint64_t nq, const uint64_t *qoff, const uint32_t *lists, const double *arrival_s,
                      uint32_t outstanding, uint64_t id_base, double *latency_s, double *wall_s) {
    Server *s = (Server *)server;
    if (!s || !qoff || (nq && (!lists || !latency_s)) || (!arrival_s && outstanding == 0)) return SVB_ERR_INVALID;
    for (uint64_t i = 0; i < nq; ++i)
        if (qoff[i + 1] <= qoff[i] || qoff[i + 1] - qoff[i] > 0xFFFFFFFFull) return SVB_ERR_INVALID;
    std::lock_guard<std::mutex> lock(s->mu);
    (void)hipSetDevice(s->device);
    for (uint64_t i = 0; i < nq; ++i)
        if (s->queries.count(id_base + i)) return SVB_ERR_INVALID;
    typedef std::chrono::steady_clock clock;
    const clock::time_point t0 = clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    std::vector<double> sent(nq, 0.0);
    std::vector<uint64_t> other;  // completions of queries submitted outside this replay stay pollable
    uint64_t next = 0, done = 0;
    int st = SVB_OK;
    while (done < nq) {
        // arrivals that are due (open loop) or room under the outstanding limit (closed loop)
        const double t = now_s();
        while (next < nq && (arrival_s ? arrival_s[next] <= t : next - done < outstanding)) {
            sent[next] = arrival_s ? arrival_s[next] : t;
            st = submit_locked(*s, id_base + next, (uint32_t)(qoff[next + 1] - qoff[next]), lists + qoff[next]);
            if (st != SVB_OK) return st;
            ++next;
        }
        // closed loop: nothing else can happen until a batch finishes, so wait for one
        const bool block = !arrival_s && next - done >= outstanding;
        if ((st = step_locked(*s, block)) != SVB_OK) return st;
        if (s->completed.empty() && !s->waiting.empty() && s->admitted.empty() &&
            std::none_of(s->slots.begin(), s->slots.end(), [](const Slot &sl) { return sl.busy; }))
            return SVB_ERR_NOMEM;  // nothing on the device and the arena is held by unreleased results
        if (!s->completed.empty()) {
            const double tc = now_s();
            while (!s->completed.empty()) {
                const uint64_t id = s->completed.front();
                s->completed.pop_front();
                auto it = s->queries.find(id);
                if (id >= id_base && id - id_base < nq) {
                    latency_s[id - id_base] = tc - sent[id - id_base];
                    arena_free(*s, it->second.arena_off, it->second.ints);
                    s->queries.erase(it);
                    ++done;
                } else {
                    other.push_back(id);
                }
            }
        }
    }
    for (uint64_t id : other) s->completed.push_back(id);
    if (wall_s) *wall_s = now_s();
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
    const uint64_t extra[3] = {(uint64_t)s->waiting.size(), (uint64_t)s->admitted.size(), s->in_use};
    for (uint32_t i = 0; i < cap; ++i) out[i] = i < 8 ? s->stats[i] : (i < 11 ? extra[i - 8] : 0);
    return SVB_OK;
}

int svb_server_destroy(void *server) {
    destroy((Server *)server);
    return SVB_OK;
}

}  // extern "C"
