// C ABI of libsvb.so (declared in include/svb.h): argument checks, per-stream
// scratch workspaces and kernel launches.  No codec arithmetic happens here.
#include <map>
#include <mutex>
#include <utility>

#include "svb_internal.hpp"

namespace svb {
namespace {

// Scratch owned by the library for one (device, stream): the tile ticket and
// finish counters and the per-tile status words of the look-back scans.
struct Workspace {
    uint32_t *counters = nullptr;  // 16 words
    uint64_t *flags = nullptr;     // 2 * cap words: byte prefixes, then value prefixes
    uint64_t cap = 0;              // tiles
    uint32_t epoch = 0;
};

std::mutex g_mu;
std::map<std::pair<int, uintptr_t>, Workspace> g_ws;

constexpr uint32_t kEpochLimit = 1u << 20;  // status words carry a 20-bit epoch

int hip_status(hipError_t e) { return e == hipSuccess ? SVB_OK : SVB_ERR_HIP; }

// Workspace for the calling thread's device and `s`, with room for `tiles`
// tiles, and a fresh epoch for one launch.
int acquire(hipStream_t s, uint64_t tiles, Workspace **out, uint32_t *epoch) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVB_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace &w = g_ws[std::make_pair(dev, (uintptr_t)s)];
    if (!w.counters) {
        if (hipMalloc((void **)&w.counters, 16 * sizeof(uint32_t)) != hipSuccess) {
            w.counters = nullptr;
            return SVB_ERR_NOMEM;
        }
        if (launch_fill(w.counters, 16, 0u, s) != hipSuccess) return SVB_ERR_HIP;
    }
    if (tiles > w.cap) {
        uint64_t cap = 1024;
        while (cap < tiles) cap <<= 1;
        if (w.flags) {
            if (hipStreamSynchronize(s) != hipSuccess) return SVB_ERR_HIP;
            (void)hipFree(w.flags);
            w.flags = nullptr;
            w.cap = 0;
        }
        if (hipMalloc((void **)&w.flags, 2 * cap * sizeof(uint64_t)) != hipSuccess) {
            w.flags = nullptr;
            return SVB_ERR_NOMEM;
        }
        if (launch_fill((uint32_t *)w.flags, 4 * cap, 0u, s) != hipSuccess) return SVB_ERR_HIP;
        w.cap = cap;
        w.epoch = 0;
    }
    w.epoch += 1;
    if (w.epoch >= kEpochLimit) {
        // every epoch value has been used: clear the words and start over
        if (launch_fill((uint32_t *)w.flags, 4 * w.cap, 0u, s) != hipSuccess) return SVB_ERR_HIP;
        w.epoch = 1;
    }
    *out = &w;
    *epoch = w.epoch;
    return SVB_OK;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }
bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int zero_u64(uint64_t *p, hipStream_t s) {
    if (!p) return SVB_OK;
    return hip_status(launch_fill((uint32_t *)p, 2, 0u, s));
}

int do_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint32_t start, uint64_t *out_bytes,
              bool delta, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (out_bytes && !aligned8(out_bytes)) return SVB_ERR_INVALID;
    if (n == 0) return zero_u64(out_bytes, s);
    if (!in || !out || !aligned4(in)) return SVB_ERR_INVALID;
    const uint64_t tiles = (n + kTileInts - 1) / kTileInts;
    Workspace *w;
    EncodeArgs a;
    int st = acquire(s, tiles, &w, &a.epoch);
    if (st != SVB_OK) return st;
    a.in = in;
    a.n = n;
    a.out = out;
    a.start = start;
    a.out_bytes = out_bytes;
    a.counters = w->counters;
    a.byte_flags = w->flags;
    a.num_tiles = (uint32_t)tiles;
    return hip_status(launch_encode(a, delta, s));
}

int do_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start,
              uint32_t *err, bool delta, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n > SVB_MAX_N) return SVB_ERR_INVALID;
    if (err && !aligned4(err)) return SVB_ERR_INVALID;
    if (n == 0) return SVB_OK;
    if (!in || !out || !aligned4(out)) return SVB_ERR_INVALID;
    if (in_bytes < (n + 3) / 4) return SVB_ERR_INVALID;
    const uint64_t tiles = (n + kTileInts - 1) / kTileInts;
    Workspace *w;
    DecodeArgs a;
    int st = acquire(s, tiles, &w, &a.epoch);
    if (st != SVB_OK) return st;
    a.in = in;
    a.in_bytes = in_bytes;
    a.n = n;
    a.out = out;
    a.start = start;
    a.err = err;
    a.counters = w->counters;
    a.byte_flags = w->flags;
    a.val_flags = w->flags + w->cap;
    a.num_tiles = (uint32_t)tiles;
    return hip_status(launch_decode(a, delta, s));
}

}  // namespace

uint32_t persistent_grid(const void *kernel, uint32_t num_tiles) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, uint32_t> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    uint32_t grid = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(std::make_pair(dev, kernel));
        if (it != cache.end()) {
            grid = it->second;
        } else {
            int cus = 0, per_cu = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
                cus = 256;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWorkgroupThreads, 0) != hipSuccess ||
                per_cu <= 0)
                per_cu = 4;
            grid = (uint32_t)(cus * per_cu);
            cache[std::make_pair(dev, kernel)] = grid;
        }
    }
    if (grid > num_tiles) grid = num_tiles;
    return grid ? grid : 1u;
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
        if (kv.second.counters) (void)hipFree(kv.second.counters);
        if (kv.second.flags) (void)hipFree(kv.second.flags);
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
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
