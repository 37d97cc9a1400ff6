// Internal interface between the C ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/svb.h"

namespace svb {

// Geometry.  A segment is what one wave decodes or encodes at a time: 64 lanes
// x 16 integers, lane l owning control bytes l, l + 64, l + 128, l + 192.  A group is
// kGroupSegs consecutive segments, walked in order by one wave; the pre-pass
// and the scans work per group.
constexpr uint32_t kSegInts = 1024;
constexpr uint32_t kSegCtrl = kSegInts / 4;
#ifndef SVB_GROUP_SEGS
#define SVB_GROUP_SEGS 4  // measured: 4 as fast as 8 or faster (2^28 delta 0.378 vs 0.385-0.413 ms), 16 slower
#endif
constexpr uint32_t kGroupSegs = SVB_GROUP_SEGS;
constexpr uint64_t kGroupInts = (uint64_t)kSegInts * kGroupSegs;
constexpr uint64_t kGroupCtrl = kGroupInts / 4;
static_assert(kGroupSegs >= 4 && kGroupSegs <= 64 && (64 % kGroupSegs) == 0, "group of 4..64 segments");

// Groups come in blocks of kWaves (one workgroup of the passes that take one
// group per wave): the passes that produce per-group byte counts and value
// sums also write each block's total, and the scans run over the block
// totals; a group's offset or carry is its block's prefix plus the at most
// kWaves - 1 group values before it in the block.
struct GroupBytesArgs {
    const uint8_t *in;     // stream; its first ceil(n/4) bytes are the control stream
    uint64_t in_bytes;
    uint64_t n;
    uint64_t groups;
    uint32_t *gbytes;      // out: data bytes of each group (an array of whole blocks)
    uint32_t *bbytes;      // out: data bytes of each block of groups
};

struct DecodeArgs {
    const uint8_t *in;
    uint64_t in_bytes;
    uint64_t n;
    uint32_t *out;
    uint32_t *err;
    uint64_t groups;
    const uint32_t *gbytes;  // data bytes of each group (an array of whole blocks)
    const uint32_t *boff32;  // data-stream byte offset of each block of groups, 32-bit (a stream under 4 GiB),
    const uint64_t *boff;    //   else 64-bit
    uint32_t *gvsum;         // value sum of each group (written by the value-sum pass; whole blocks)
    uint32_t *bvsum;         // value sum of each block of groups (written by the value-sum pass)
    const uint32_t *bvpre;   // start + exclusive value prefix of each block (read in delta mode)
};

// Decoding: mode 0 plain, 1 delta (running sum), 2 value sums per group.
enum DecodeMode { kPlain = 0, kDelta = 1, kSums = 2 };
hipError_t launch_group_bytes(const GroupBytesArgs &a, hipStream_t s);
// Exclusive prefix sums of m uint32 values into `out`: 64-bit (wide) or modulo
// 2^32 plus `start`.  `total` (may be null) receives the sum (u64 when wide,
// else u32 start + sum).  Above a few tens of thousands of values the scan
// needs scan_scratch_bytes(m) bytes of device scratch.
uint64_t scan_scratch_bytes(uint64_t m);
hipError_t launch_scan(const uint32_t *in, void *out, uint64_t m, bool wide, uint32_t start, hipStream_t s,
                       void *total = nullptr, void *scratch = nullptr);
// zc: the zero-control variant (rows of all-zero control bytes widen bytes).
hipError_t launch_decode(const DecodeArgs &a, int mode, hipStream_t s, bool zc = false);

// Delta decoding's value sums (gvsum per group, bvsum per block) without
// decoding: the plain sum of each group's data bytes plus a correction per
// block whose control byte is not zero (svb_delta.hip).
hipError_t launch_group_sums(const DecodeArgs &a, hipStream_t s);

// Batched calls.  A task is one 1024-integer segment of one list; each wave of
// the main pass takes `chunk` consecutive tasks.
//
// Per-task descriptor: everything a wave needs to start the task, so that a
// task costs one 64-byte load before its control bytes can be requested.
struct alignas(64) TaskDesc {
    uint64_t in;        // decode: the list's stream; encode: the list's values
    uint64_t in_bytes;  // decode: bytes readable at `in`
    uint64_t n;         // integers in the list
    uint64_t out;       // decode: the list's output (uint32); encode: the list's stream
    uint64_t boff;      // byte offset of the segment's data in the list's data stream
    uint32_t s;         // segment index inside the list
    uint32_t carry;     // delta decode: running sum before the segment; delta encode: start
    uint32_t word;      // list index, bit 31 set on the list's last segment
    uint32_t pad[3];
};
static_assert(sizeof(TaskDesc) == 64, "one 64-byte descriptor per task");

struct BatchArgs {
    uint32_t m;
    const uint64_t *counts;
    const uint64_t *in_off;    // decode: byte offset of each stream; encode: uint32 index of each list
    const uint64_t *in_bytes;  // decode only (null when encoding)
    const uint8_t *in8;        // decode input
    const uint32_t *in32;      // encode input
    const uint64_t *out_off;   // decode: uint32 index of each list; encode: byte offset of each stream
    uint32_t *out32;           // decode output
    uint8_t *out8;             // encode output
    uint64_t *out_bytes;       // encode: stream sizes (may be null)
    const uint32_t *starts;    // null: plain
    uint32_t *err;             // decode: corruption / overflow flag (may be null)
    uint32_t *litems;          // per list: tasks (segments)
    uint32_t *lbase;           // per list + 1: first task of each list; lbase[m] = tasks in all
    uint32_t *item_list;       // per task: its list, bit 31 set on a list's last task
    uint32_t *item_first;      // per task: first task of its list
    uint32_t t_cap;            // task capacity of the scratch arrays
    uint32_t chunk;            // tasks per wave in the main pass (per grab, with a work queue)
    uint32_t *queue;           // decode walk: counter of the next task to grab (zeroed before the walk),
                               // or null for the static schedule (wave w takes tasks [w chunk, (w + 1) chunk))
    uint32_t *ibytes;          // per task: data bytes (tasks that are not the last of their list)
    uint64_t *ioff;            // per task: exclusive scan of ibytes
    uint32_t *ivsum;           // per task: sum of stored differences (delta decoding)
    uint32_t *ivpre;           // per task: exclusive scan of ivsum
    TaskDesc *desc;            // per task
};
enum BatchPhase {
    kBatchCount = 0,
    kBatchMap = 1,      // encoding (decoding maps tasks in its byte counts)
    kBatchItemBytes = 2,
    kBatchItemSums = 3,
    kBatchWork = 4,
    kBatchDesc = 5      // descriptors from the byte offsets (and for delta decoding the value-sum prefixes)
};
hipError_t launch_batch(const BatchArgs &a, int phase, bool encode, bool delta, hipStream_t s);

// Serving: the descriptors of one batch, copied from the pool's task index
// (built once by the batched decoder's preparation passes) with each list's
// output address in the arena.
struct ServeDescArgs {
    uint32_t m;                  // lists in the batch
    const uint32_t *list;        // pool list of each batch list
    const uint64_t *out_off;     // arena offset (uint32 units) of each batch list
    const uint32_t *base;        // first task of each batch list; base[m] = tasks in the batch
    const TaskDesc *pool_desc;   // task index of the pool (no output addresses)
    const uint32_t *pool_lbase;  // first index task of each pool list
    uint32_t *arena;
    TaskDesc *desc;              // out: the batch's descriptors
};
hipError_t launch_serve_desc(const ServeDescArgs &a, uint32_t tasks, hipStream_t s);  // tasks = base[m]
// A serving batch's table on the device: per batch list its first task and
// arena offset, from the lists' integer counts.
struct ServePlanArgs {
    uint32_t m;               // lists in the batch
    const uint32_t *counts;   // integers of each batch list (query order; may be pinned host memory);
                              // they sum below 2^32
    uint64_t out_base;        // arena offset (uint32 units) of the batch's first list
    uint32_t *base;           // out: first task of each batch list; base[m] = tasks in the batch
    uint64_t *out_off;        // out: arena offset of each batch list
};
hipError_t launch_serve_plan(const ServePlanArgs &a, hipStream_t s);
int build_pool_index(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                     const uint8_t *in, const uint32_t *starts, uint64_t total_ints, TaskDesc **desc,
                     uint32_t **lbase, uint32_t *tasks, hipStream_t s);
int serve_walk(BatchArgs &a, bool delta, hipStream_t s);

// Seek and select over a task index (built by build_pool_index): per task the
// running maximum of its list's values up to the task's segment's end.
// Per list, what a query of a short list needs in one 64-byte line: its
// stream, its length, its first task and segment count, the running sum it
// starts from and its largest value.
struct alignas(64) SeekList {
    uint64_t in;        // the list's stream
    uint64_t in_bytes;  // bytes of it
    uint64_t n;         // integers
    uint32_t first;     // first task in the index
    uint32_t segs;      // segments
    uint32_t carry;     // delta lists: the start value
    uint32_t top;       // the running maximum at the list's end (0 for an empty list)
    uint32_t pad[6];
};
static_assert(sizeof(SeekList) == 64, "one line per list");

struct SeekArgs {
    uint32_t m;               // lists
    SeekList *lists;          // per list (written by the index build)
    uint64_t tasks;           // segments of the index
    const TaskDesc *desc;     // task index (no output addresses)
    const uint32_t *lbase;    // first task of each list; lbase[m] = tasks
    uint32_t *rmax;           // per task: running maximum (written by the index build)
    bool delta;
    uint32_t q;               // queries
    uint32_t chunk;           // queries per wave
    const uint32_t *list;     // list of each query
    const uint32_t *target;   // seek targets
    const uint64_t *idx;      // select positions
    uint64_t *pos;            // seek: out
    uint32_t *value;          // out
    uint32_t *err;            // flag word (required by the index build, may be null for queries)
};
hipError_t launch_seek_index(const SeekArgs &a, hipStream_t s);
hipError_t launch_seek_queries(const SeekArgs &a, bool seek, hipStream_t s);

// Encoding (two passes: data bytes per segment, scan, pack).
// A stream to encode: n values at `in`; the stream (control bytes first) is
// written at `out`.  Delta encoding starts from `start`.
struct EncodeStream {
    const uint32_t *in;
    uint64_t n;
    uint8_t *out;
    uint32_t start;
};
hipError_t launch_encode_sizes(const EncodeStream &e, bool delta, uint32_t *seg_bytes, uint64_t segs, hipStream_t s);
// seg_off32 (may be null): 32-bit segment offsets, used instead of seg_off.
hipError_t launch_encode_pack(const EncodeStream &e, bool delta, const uint64_t *seg_off, uint64_t segs,
                              uint64_t *out_bytes, hipStream_t s, const uint32_t *seg_off32 = nullptr);
hipError_t launch_copy(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s);
// Append: a byte copy at any alignments (the count is len, or *len_dev -
// len_sub when len_dev is set, at most len; size_out, if set, receives
// size_base + the count), and the merged control bytes from floor(n/4) on.
hipError_t launch_copy_bytes(const uint8_t *src, uint8_t *dst, uint64_t len, const uint64_t *len_dev,
                             uint64_t len_sub, uint64_t *size_out, uint64_t size_base, hipStream_t s);
hipError_t launch_merge_ctrl(const uint8_t *old_ctrl, const uint8_t *new_ctrl, uint8_t *out, uint64_t n, uint64_t k,
                             hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n, uint32_t value, hipStream_t s);

// The comparison formats of Table 1: VByte and varint-GB.
constexpr int kFmtVByte = 0, kFmtVarintGB = 1;
// Encoding: bytes per 1024-integer segment (sizes pass), a scan, the pack.
struct CmpEncodeArgs {
    const uint32_t *in;
    uint64_t n;
    uint8_t *out;
    uint32_t *seg_bytes;
    const uint64_t *seg_off;
    uint64_t segs;
    uint64_t *out_bytes;
};
hipError_t launch_cmp_encode(const CmpEncodeArgs &a, int fmt, bool sizes, hipStream_t s);
// VByte decoding: integer ends per 1024-byte tile (count pass), a scan
// (toff, total), the decode pass.
struct VbDecodeArgs {
    const uint8_t *in;
    uint64_t in_bytes, n, tiles;
    uint32_t *tcount;
    const uint64_t *toff;
    const uint64_t *total;
    uint32_t *out;
    uint32_t *err;
};
uint64_t vb_tiles(uint64_t in_bytes);
hipError_t launch_vb_decode(const VbDecodeArgs &a, bool count, hipStream_t s);
// varint-GB decoding, in five passes (kGbMap .. kGbDecode).
enum GbPhase { kGbMap = 0, kGbSuper, kGbTop, kGbTiles, kGbDecode };
struct GbDecodeArgs {
    const uint8_t *in;
    uint64_t in_bytes, n, tiles, supers;
    uint16_t *cmap;    // 17 entries per 128-byte chunk
    uint32_t *tmap;    // 17 entries per 8 KiB tile
    uint32_t *smap;    // 17 entries per 64 tiles
    uint32_t *sentry;  // chain entry and first block of each supertile
    uint64_t *sbase;
    uint32_t *tentry;  // ... and of each tile
    uint64_t *tbase;
    uint64_t *total;   // blocks starting inside the stream
    uint32_t *out;
    uint32_t *err;
};
uint64_t gb_tiles(uint64_t in_bytes);
uint64_t gb_supers(uint64_t tiles);
hipError_t launch_gb_decode(const GbDecodeArgs &a, int phase, hipStream_t s);

}  // namespace svb
