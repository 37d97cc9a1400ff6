/*
 * svb.h -- Stream VByte on AMD Instinct MI355X (gfx950): C ABI of libsvb.so.
 *
 * Format (Lemire, Kurz, Rupp, "Stream VByte: Faster Byte-Oriented Integer
 * Compression", Section 4 and Fig. 3).  A stream of n unsigned 32-bit
 * integers is one byte buffer:
 *
 *     [ control stream: ceil(n/4) bytes | data stream: sum of L_i bytes ]
 *
 *  - L_i = max(1, ceil(log_256(x_i + 1))) in {1,2,3,4} (Section 3).
 *  - Control byte b holds the 2-bit codes L_i - 1 of integers 4b..4b+3,
 *    integer 4b+j in bits [2j, 2j+1].  Unused fields of a partial last
 *    control byte are written as 0 and ignored when read.
 *  - Integer i occupies L_i consecutive data bytes, little-endian.
 *  - n is not stored in the stream; every call takes it as an argument.
 *
 * Differential ("delta") variant (Section 2, "Differential Coding", and
 * Section 5): the stored values are d_i = x_i - x_{i-1} modulo 2^32 with
 * x_{-1} = start; decoding returns the running sum modulo 2^32 from start.
 * Any uint32 array round-trips, sorted or not.
 *
 * Conventions shared by every call:
 *  - Every buffer pointer is a DEVICE pointer on the current HIP device,
 *    owned by the caller.  The library never frees or retains them.
 *  - uint32_t arrays must be 4-byte aligned; byte streams have no alignment
 *    requirement.  uint64_t arrays must be 8-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream: results are valid after the
 *    stream is synchronised.  Argument errors are returned synchronously.
 *  - Calls on different streams may run concurrently: the library keeps a
 *    separate scratch workspace per (device, stream).  Calls on one stream
 *    are ordered by the stream.
 *  - The only library-owned memory is that scratch workspace (and, for a
 *    serving pool, the server's own buffers): 12 bytes per encoder segment of
 *    1024 integers (byte count, byte offset), about 13 bytes per decoder
 *    group of 4096 integers (byte total and value sum per group; byte total,
 *    value sum, byte offset and value prefix per block of four groups), about
 *    96 bytes per batched segment, plus the scans' partial sums; grown on
 *    demand, freed by svb_release_workspace.
 *  - Return value: SVB_OK (0) or a negative svb_status.  The library never
 *    aborts the process.
 */
#ifndef SVB_H
#define SVB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum svb_status {
    SVB_OK = 0,
    SVB_ERR_INVALID = -1,   /* bad argument: null pointer with n > 0, misaligned uint32 array,
                               in_bytes smaller than the control stream, n too large */
    SVB_ERR_CORRUPT = -2,   /* reported through the `err` word of decode calls, see below */
    SVB_ERR_HIP = -3,       /* a HIP runtime call failed (launch, allocation of scratch) */
    SVB_ERR_NOMEM = -4      /* scratch workspace could not be allocated */
};

/* Value a decode kernel writes to the caller's device `err` word when the
 * control bytes describe more data than in_bytes holds. */
#define SVB_DECODE_CORRUPT 1u

/* (Value 2 is not used: no kernel of the library waits for another
 * workgroup, so none can stall.) */

/* Value a batched decode writes to `err` when the lists hold more integers
 * than the caller's total_ints bound (nothing is decoded then). */
#define SVB_BATCH_OVERFLOW 3u

/* Value a seek or select call writes to `err` when a query names a list past
 * the index's last one, or selects a position past its list's end. */
#define SVB_QUERY_OUT_OF_RANGE 4u

/* Largest n accepted by the single-stream calls (2^40 integers). */
#define SVB_MAX_N (((uint64_t)1) << 40)

/* ceil(n/4): size of the control stream (Section 4). */
uint64_t svb_control_bytes(uint64_t n);

/* ceil(n/4) + 4n: the largest stream n integers can need.  Section 3 gives
 * each integer a byte length of 1 to 4 (4 for values of 2^24 and above), and
 * the layout of Section 4 stores one control byte per 4 integers followed by
 * the integers' bytes, so the worst case is every integer 4 bytes long. */
uint64_t svb_max_compressed_bytes(uint64_t n);

/*
 * svb_encode -- Section 4 (format) and Section 3 (byte lengths).
 *   n          number of integers in `in`.
 *   in         device uint32[n], 4-byte aligned.
 *   out        device byte buffer of at least svb_max_compressed_bytes(n)
 *              bytes; receives the stream.  Bytes past the stream's size are
 *              not written.
 *   out_bytes  device uint64: receives the stream size ceil(n/4) + sum L_i.
 *              May be NULL.
 * The encoding is unique (minimal lengths), so the output is byte-exact.
 */
int svb_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream);

/* svb_delta_encode -- svb_encode of d_i = in[i] - in[i-1] (mod 2^32), in[-1] = start
 * (Section 2, "Differential Coding"; Section 5). */
int svb_delta_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint32_t start,
                     uint64_t *out_bytes, void *stream);

/*
 * svb_decode -- Section 4 (the decoding procedure of Fig. 4, done as a
 * parallel scan of control-byte lengths instead of a pointer chase).
 *   n          number of integers to decode.
 *   in         device stream of in_bytes bytes (no alignment requirement).
 *   in_bytes   bytes readable at `in`; must be >= ceil(n/4).  The stream
 *              may be followed by unrelated bytes (in_bytes larger than the
 *              stream): they are never interpreted.
 *   out        device uint32[n], 4-byte aligned.
 *   err        device uint32 or NULL.  Set to SVB_DECODE_CORRUPT when the
 *              control bytes describe more data bytes than in_bytes - ceil(n/4);
 *              left untouched otherwise (initialise it to 0).  On corrupt
 *              input the contents of `out` are unspecified, and nothing
 *              outside out[0..n) is written.  Reads stay inside the aligned
 *              16-byte chunks that overlap [in, in + in_bytes): such a chunk
 *              never crosses a page, so the decoder cannot fault on memory
 *              next to the stream, and bytes outside the stream never change
 *              a decoded value.
 */
int svb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err,
               void *stream);

/* svb_delta_decode -- svb_decode followed by the running sum modulo 2^32
 * starting from `start` (Section 2, "Differential Coding"; Section 5).  Each
 * group of 4096 integers first has its sum of stored differences taken (its
 * plain byte sum plus a correction per block of multi-byte integers, or by
 * decoding it, see the decoder variants), the sums are scanned from `start`,
 * then every group decodes from its carry with the running sum fused into the
 * decode. */
int svb_delta_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out,
                     uint32_t start, uint32_t *err, void *stream);

/* svb_delta_decode_noalloc -- svb_delta_decode for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, output, error behaviour
 * and kernels as svb_delta_decode, but its scratch is a fixed 8 MiB array in
 * the library's device code instead of the per-stream workspace: it never
 * calls hipMalloc, hipFree or any allocating routine.  Each device the
 * library runs on holds its own copy of the array until the process ends;
 * the first call on a device looks up that device's address of it.  n is
 * limited to SVB_NOALLOC_MAX_N (2^30): larger n is SVB_ERR_INVALID.  Every
 * call on one device shares that device's array, whose contents carry no
 * meaning from one call to the next (nothing in it needs to start at any
 * value): calls that overlap on one device -- on different streams, or from
 * different threads without ordering -- race on it and give wrong results.
 * Per-kernel timing (svb_set_kernel_timing) does not apply to it. */
#define SVB_NOALLOC_MAX_N (((uint64_t)1) << 30)
int svb_delta_decode_noalloc(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out,
                             uint32_t start, uint32_t *err, void *stream);

/*
 * Batched calls (Section 5's posting lists: many lists of very uneven
 * length): m independent lists decoded or encoded by one fixed sequence of
 * launches whose work list is built on the device.  A task is one
 * 1024-integer segment of one list; each wave of the main pass takes a tuned
 * number of consecutive tasks.  Lists longer than one segment first get
 * per-segment byte offsets (and, for delta decoding, per-segment value
 * carries) from a scan.  All array arguments are DEVICE arrays of m entries;
 * the host never reads them.
 *
 * total_ints (host value) is an upper bound on sum(counts[i]); it sizes the
 * library's scratch (about 96 bytes per segment, m + total_ints/1024
 * segments at most).  If the counts add up to more,
 * nothing is done: decode sets err to SVB_BATCH_OVERFLOW and encode writes
 * UINT64_MAX to every out_bytes[i].
 *
 * svb_encode_batch
 *   counts[i]     integers in list i (<= SVB_MAX_N; a larger count is
 *                 skipped and its out_bytes[i] set to UINT64_MAX).
 *   in_off[i]     index (in uint32 units) of list i's first integer in `in`.
 *   out_off[i]    byte offset in `out` where stream i is written; the caller
 *                 reserves svb_max_compressed_bytes(counts[i]) bytes there and
 *                 reserved regions must not overlap.
 *   out_bytes[i]  receives stream i's size (may be NULL).
 *   starts        NULL: plain encoding.  Otherwise delta encoding of list i
 *                 from starts[i].
 * The streams are byte-identical to svb_encode / svb_delta_encode of each list.
 */
int svb_encode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint32_t *in,
                     const uint64_t *out_off, uint8_t *out, uint64_t *out_bytes, const uint32_t *starts,
                     uint64_t total_ints, void *stream);

/*
 * svb_decode_batch
 *   counts[i]     integers in list i.
 *   in_off[i]     byte offset of stream i in `in`.
 *   in_bytes[i]   bytes readable at in + in_off[i] (a value below
 *                 ceil(counts[i]/4) makes list i corrupt: it is skipped).
 *   out_off[i]    index (uint32 units) where list i's integers are written;
 *                 output ranges must not overlap.
 *   starts        NULL: plain decoding.  Otherwise delta decoding of list i
 *                 from starts[i].
 *   err           device uint32 or NULL; set to SVB_DECODE_CORRUPT if any
 *                 stream is corrupt (see svb_decode), SVB_BATCH_OVERFLOW as
 *                 above.
 */
int svb_decode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off,
                     const uint64_t *in_bytes, const uint8_t *in, const uint64_t *out_off,
                     uint32_t *out, const uint32_t *starts, uint64_t total_ints, uint32_t *err,
                     void *stream);

/*
 * Autotuning of the batched calls: the number of consecutive tasks a wave
 * takes (1, 2, 4, 8 or 16 segments of 1024 integers) and, for decoding, the
 * schedule (static: wave w takes tasks w chunk .. (w + 1) chunk - 1; work
 * queue, chunk | SVB_BATCH_QUEUE: a grid of a few waves per SIMD, each
 * grabbing the next chunk of tasks from a device counter until none are
 * left) are chosen per device and per kind of call (decode or encode, plain
 * or delta).
 * svb_autotune_decode_batch times each candidate on the given batch (the
 * arguments of svb_decode_batch; it decodes the batch several times and
 * synchronises the stream), keeps the fastest for later calls of that kind on
 * the current device, and writes it to *chunk.  svb_autotune_encode_batch
 * does the same for encoding.  svb_set_batch_chunk(kind, chunk) sets the
 * choice directly; kind = 2 * (encode ? 1 : 0) + (delta ? 1 : 0); the queue
 * bit is refused for encoding kinds.  The default is 4 (static).  Serving
 * batches use the tuned chunk on the static schedule.
 */
#define SVB_BATCH_QUEUE 0x100u
int svb_autotune_decode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off,
                              const uint64_t *in_bytes, const uint8_t *in, const uint64_t *out_off,
                              uint32_t *out, const uint32_t *starts, uint64_t total_ints, uint32_t *err,
                              uint32_t *chunk, void *stream);
int svb_autotune_encode_batch(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint32_t *in,
                              const uint64_t *out_off, uint8_t *out, uint64_t *out_bytes,
                              const uint32_t *starts, uint64_t total_ints, uint32_t *chunk, void *stream);
int svb_set_batch_chunk(int kind, uint32_t chunk);

/*
 * Serving runtime: a pool of lists resident in device memory and queries of
 * a few lists each, decoded with admission by output memory and continuous
 * batching over the batched decoder (the paper's setting of Section 5: a
 * search engine decoding the posting lists a query asks for).
 *
 * svb_server_create takes a pool of m lists whose streams lie in `in` at
 * in_off[i] (in_bytes[i] bytes, counts[i] integers), delta-coded from
 * starts[i] if `starts` is not NULL (all device arrays; `in` must stay valid
 * while the server lives).  It copies the counts to the host and builds the
 * pool's task index on the device once (64 bytes per segment of 1024
 * integers: each segment's byte offset and running-sum carry), refusing a
 * pool with a corrupt list with SVB_ERR_INVALID.  The server owns an output
 * arena of arena_bytes, `streams` stream slots (1..16; a slot runs one batch
 * at a time) and launches at most max_batch_lists lists per batch.
 *
 * svb_server_submit queues query `query_id` (unique among live queries) for
 * the k lists list_ids[] (host array).  Its result is the k lists decoded back
 * to back into one arena range.  A query whose output exceeds the arena, or
 * with k > max_batch_lists, is refused with SVB_ERR_INVALID.
 *
 * svb_server_step runs one scheduling step: retire finished batches, admit
 * waiting queries in arrival order while the arena has room for their output,
 * and launch batches of the admitted queries (at most max_batch_lists lists
 * each) on free slots.  With block != 0
 * and nothing complete yet, it waits for the oldest batch on the device.  It
 * returns the number of complete queries not yet polled (or a negative status).
 *
 * svb_server_poll hands out up to `cap` complete queries: id, arena offset and
 * length (in uint32 units); their arena ranges stay reserved until
 * svb_server_release(query_id).  svb_server_arena returns the arena's device
 * address.  svb_server_stats writes up to `cap` counters: batches, lists,
 * integers, queries admitted, queries completed, most batches running on the
 * device at once (counted at each launch: slots whose batch had not finished), the
 * decoders' err flags (OR), arena peak (integers), queries waiting, admitted
 * but not launched, arena integers in use, scheduling steps, steps whose host
 * work took over 1 ms, the longest step (microseconds).  svb_server_destroy waits for the
 * device and frees everything.  One server may be driven from one thread at a
 * time (calls are serialised by a lock).
 */
int svb_server_create(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                      const uint8_t *in, const uint32_t *starts, uint64_t arena_bytes, uint32_t streams,
                      uint32_t max_batch_lists, void **server);
int svb_server_submit(void *server, uint64_t query_id, uint32_t k, const uint32_t *list_ids);
int svb_server_step(void *server, int block);
int svb_server_poll(void *server, uint64_t *ids, uint64_t *arena_off, uint64_t *ints, uint32_t cap);
int svb_server_release(void *server, uint64_t query_id);
uint32_t *svb_server_arena(void *server);
int svb_server_stats(void *server, uint64_t *out, uint32_t cap);
/* Batching policy of svb_server_step: while a batch is on the device, the
 * next one is launched only once min_lists lists are admitted or its oldest
 * query has waited max_wait_us microseconds (with nothing on the device it
 * leaves at once).  Defaults 1024 lists, 20 us; (0, 0) launches whenever a
 * slot is free.  Larger batches cost the host less per query. */
int svb_server_set_batching(void *server, uint32_t min_lists, uint32_t max_wait_us);
int svb_server_destroy(void *server);

/*
 * svb_server_replay drives the server from the calling thread with a query
 * trace and measures latency (a load generator for the serving loop).  Query i
 * asks for lists[qoff[i] .. qoff[i+1]) (host arrays; every query names at
 * least one list).  Open loop (arrival_s != NULL): query i is submitted once
 * arrival_s[i] seconds have passed since the call began; its latency runs
 * from arrival_s[i] to the moment the host sees its batch complete.  Closed
 * loop (arrival_s == NULL): `outstanding` queries are kept in the system,
 * latency runs from submission.  Queries of svb_server_submit waiting when
 * the replay starts are launched first (and polled as usual); the replayed
 * queries' results go to a ring in the largest free range of the arena and
 * are released as soon as they complete (never polled).  A replayed batch is
 * a run of consecutive queries; its per-list table is built on the device.  latency_s[i] receives
 * seconds; *wall_s (if not NULL) the call's duration.  Returns SVB_OK, or a
 * negative status (bad trace, a query that can never be admitted, an arena
 * held by unreleased results, a HIP error) with the server's state as of the
 * failure.
 */
int svb_server_replay(void *server, uint64_t nq, const uint64_t *qoff, const uint32_t *lists, const double *arrival_s,
                      uint32_t outstanding, double *latency_s, double *wall_s);

/*
 * svb_server_replay_poisson: an open loop whose arrivals are drawn in the
 * call, for windows longer than a host trace could hold.  Query i (i = 0, 1,
 * ...) asks for the lists of trace entry i mod nbase (lists[qoff[e] ..
 * qoff[e+1]), host arrays, at least one list each) and arrives at the i-th
 * point of a Poisson process of rate qps queries per second, for `seconds`
 * of arrivals (exponential gaps: 2^22 draws of a 64-bit Mersenne twister
 * seeded with `seed`, read in order from a fresh random position every 2^22
 * queries).  Queries are served like svb_server_replay's (results released
 * unread); those arriving before warmup_s (< seconds) are served but left
 * out of the figures.  out[0 .. out_cap) receives, as doubles: queries
 * measured, their integers, seconds from warmup_s to the last completion,
 * the 50th and 99th percentile and the mean latency in seconds (arrival to
 * the host seeing the batch complete; percentiles from 0.1 us bins up to
 * 0.1 s), queries generated, batches launched.  Returns SVB_OK, or a
 * negative status as svb_server_replay (SVB_ERR_NOMEM also for a trace entry
 * larger than the arena's largest free range).  The serving setting is
 * Section 5's: posting lists decoded per query.
 */
int svb_server_replay_poisson(void *server, uint64_t nbase, const uint64_t *qoff, const uint32_t *lists, double qps,
                              double seconds, double warmup_s, uint64_t seed, double *out, uint32_t out_cap);

/*
 * Decoder variants (the paper's decoder special-cases control bytes of
 * single-byte integers, Section 4).  Bit 0 of a variant: 0 = the general
 * decoder; 1 = also decode every row of 64 blocks whose control bytes are all
 * zero (256 one-byte integers) by widening bytes, which pays only where such
 * rows are common (small deltas everywhere) and costs a test per row
 * elsewhere.  Bit 1, delta decoding only (how each group's sum of stored
 * differences is taken before the running sum, Section 2): 0 = from the
 * group's plain byte sum plus a correction per block of multi-byte integers;
 * 1 = by decoding the group.  Plain decoding takes variants 0..1, delta decoding
 * 0..3.  svb_autotune_decode times every variant of the kind on the caller's
 * stream (the arguments of svb_decode / svb_delta_decode; it decodes several
 * times and synchronises the stream), keeps the fastest for later calls of
 * that kind (plain or delta) on the current device and writes it to
 * *variant; svb_set_decode_variant sets it directly (-1: back to the
 * automatic choice below; SVB_ERR_INVALID for a variant out of range).  All variants give identical output.  Until one is
 * tuned or set, the general decoder is used, and delta decoding takes the sums
 * from byte sums unless the stream averages more than 4480 data bytes per
 * group (about 1.1 bytes per integer), where it decodes them.
 */
int svb_autotune_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t start, int delta,
                        uint32_t *err, int *variant, void *stream);
int svb_set_decode_variant(int delta, int variant);

/*
 * Append without re-encoding the stored integers (the paper's closing remark:
 * data added at the end of a stream, its control stream grown).  svb_append
 * writes to `out` the stream of the n integers held in `in` followed by the
 * k integers at `vals` (device uint32, 4-byte aligned): the old codes keep
 * their bit positions (the last, partial control byte takes the first new
 * codes), the old data bytes are copied unchanged, and only the new integers
 * are encoded.  The result is byte-identical to encoding all n + k integers.
 * svb_delta_append stores the new integers as differences, the first from
 * `prev` (the old stream's last value, or its start when n = 0); the result
 * is then the delta stream of all n + k integers from the old stream's start.
 *   in_bytes   the old stream's exact size (as the encoder reported it);
 *              below ceil(n/4) is SVB_ERR_INVALID.  A size that does not
 *              match the control bytes gives a stream that is not valid.
 *   out        ceil((n+k)/4) + (in_bytes - ceil(n/4)) + 4k bytes at most;
 *              must not overlap `in` or `vals`.
 *   out_bytes  device uint64 (may be NULL): the new stream's size.
 * Uses the encoder's scratch (about 4.3 bytes per new integer).
 */
int svb_append(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint64_t k, const uint32_t *vals, uint8_t *out,
               uint64_t *out_bytes, void *stream);
int svb_delta_append(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint64_t k, const uint32_t *vals,
                     uint32_t prev, uint8_t *out, uint64_t *out_bytes, void *stream);

/*
 * The two comparison formats of Table 1, for measuring Stream VByte against
 * them on the same data (Section 5 compares speed and size).
 *
 * VByte (Section 1): each integer in 1 to 5 bytes of seven data bits, least
 * significant first; a byte's top bit is 1 when another byte of the same
 * integer follows (the paper's examples: 32 -> 0x20, 128 -> 0x80 0x01).
 * varint-GB (Section 3, Fig. 1): per block of four integers, a control byte
 * (integer j of the block in bits 2j..2j+1, code = byte length - 1) followed
 * by the block's little-endian data bytes; a last block of fewer than four
 * integers holds only their bytes (its unused codes 0).  n is kept out of
 * band for both.
 *
 * Encoders: `in` device uint32 (4-byte aligned); `out` at least
 * svb_vbyte_max_bytes(n) / svb_varintgb_max_bytes(n) bytes, any alignment;
 * out_bytes device uint64 (may be NULL) receives the stream's size.  The
 * encoding is unique (minimal lengths), so streams compare byte for byte.
 *
 * Decoders: in_bytes may exceed the stream (later bytes are not used); below
 * n (VByte) or n + ceil(n/4) (varint-GB) it is SVB_ERR_INVALID.  `out`
 * device uint32, 4-byte aligned, n values.  *err (device uint32, may be
 * NULL) is set to SVB_DECODE_CORRUPT when the stream ends before the n-th
 * integer, or (VByte) one of the first n integers takes more than 5 bytes;
 * the output is then unspecified and nothing outside it is written.  VByte
 * decodes in three passes (integer ends per 1 KiB tile, a scan, the decode);
 * varint-GB, whose block positions form a chain through the control bytes,
 * in five (chunk maps of the chain from each of the 17 possible entry offsets,
 * their composition over 8 KiB tiles and 512 KiB supertiles, the true chain,
 * the decode).  Scratch: VByte 12 bytes per KiB of stream; varint-GB about
 * 280 bytes per KiB.
 */
uint64_t svb_vbyte_max_bytes(uint64_t n);
int svb_vbyte_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream);
int svb_vbyte_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err, void *stream);
uint64_t svb_varintgb_max_bytes(uint64_t n);
int svb_varintgb_encode(uint64_t n, const uint32_t *in, uint8_t *out, uint64_t *out_bytes, void *stream);
int svb_varintgb_decode(uint64_t n, const uint8_t *in, uint64_t in_bytes, uint32_t *out, uint32_t *err,
                        void *stream);

/*
 * Seek and select on resident compressed lists (Section 5 benchmarks both
 * operations on the compressed stream).  For list L, value x_i is its i-th
 * integer after the running sum from starts[L] when the lists are
 * delta-coded (Section 2), else the stored integer.
 *   seek(L, target)  the first position i with x_i >= target, and x_i; the
 *                    list's length and 0 if no value reaches the target;
 *   select(L, i)     x_i.
 * Both are exact for any list, sorted or not.
 *
 * svb_seek_index_create builds a skip index over m lists laid out as for
 * svb_server_create (device arrays counts, in_off, in_bytes, starts or NULL;
 * streams in `in`, which must stay valid and unchanged while the index
 * lives; total_ints bounds sum(counts)).  Per 1024-integer segment of each
 * list the index keeps the segment's byte offset, the running sum before it
 * and the running maximum of the list's values up to its end (68 bytes per
 * segment, 4 per list).  It synchronises `stream`.  Returns SVB_ERR_INVALID
 * if a list is corrupt (data shorter than its control bytes describe) or the
 * counts exceed total_ints.
 *
 * svb_seek_batch answers q seeks: list[k] and target[k] (device arrays) give
 * pos[k] (uint64) and value[k].  svb_select_batch answers q selects: list[k]
 * and idx[k] (uint64) give value[k].  One wave decodes the one segment that
 * holds each answer.  A query naming a list >= m, or a select position past
 * its list's end, gets pos = UINT64_MAX and value 0 and sets the device word
 * err (may be NULL) to SVB_QUERY_OUT_OF_RANGE.  Asynchronous on `stream`.
 * svb_seek_index_destroy frees the index (after the device is done with it).
 */
int svb_seek_index_create(uint32_t m, const uint64_t *counts, const uint64_t *in_off, const uint64_t *in_bytes,
                          const uint8_t *in, const uint32_t *starts, uint64_t total_ints, void **index,
                          void *stream);
int svb_seek_batch(void *index, uint32_t q, const uint32_t *list, const uint32_t *target, uint64_t *pos,
                   uint32_t *value, uint32_t *err, void *stream);
int svb_select_batch(void *index, uint32_t q, const uint32_t *list, const uint64_t *idx, uint32_t *value,
                     uint32_t *err, void *stream);
int svb_seek_index_destroy(void *index);

/* Message for a status code (static string).  A support call of this
 * library's interface: the paper defines no error reporting, so the codes
 * above are this library's own (a corrupt stream is the one condition that
 * the format itself can present, Section 4's length code read past the
 * data bytes). */
const char *svb_strerror(int status);

/* Frees every scratch workspace the library holds (all devices and streams).
 * Synchronises the devices first.  Later calls allocate again.  A support
 * call of this library's interface: the scratch holds the per-group byte
 * counts, offsets and value sums that turn the serial pointer advance and
 * running sum of Sections 2 and 4 into scans; the paper's decoder, a single
 * pass in registers, needs none. */
void svb_release_workspace(void);

/*
 * Per-kernel timing (measurement aid).  svb_set_kernel_timing(1) makes every
 * later codec call record a pair of HIP events on its stream around each
 * kernel it launches; 0 turns recording off.  svb_kernel_times reads the
 * records of the calling thread made since its previous call, oldest first:
 * it synchronises on them, writes up to `cap` kernel names (static strings)
 * and durations in milliseconds, forgets all of them, and returns how many
 * there were (or a negative svb_status).  Kernel names: "group_bytes",
 * "scan_offsets", "group_sums", "scan_sums", "decode", "decode_delta",
 * "encode", "encode_delta", and for the batched calls "batch_count",
 * "batch_scan_lists", "batch_map" and "batch_task_bytes" (encoding),
 * "batch_map_bytes" (decoding), "batch_scan_offsets", "batch_task_sums",
 * "batch_scan_sums", "batch_desc", "batch_decode", "batch_encode", for the
 * comparison formats "cmp_sizes", "vbyte_encode", "varintgb_encode",
 * "vbyte_ends", "vbyte_decode", "varintgb_maps", "varintgb_super",
 * "varintgb_top", "varintgb_tiles", "varintgb_decode" (a scan of more than
 * 16384 values is three kernels under one name).
 */
int svb_set_kernel_timing(int enable);
int svb_kernel_times(const char **names, float *ms, int cap);

/* Library version string. */
const char *svb_version(void);

/*
 * Measurement helpers (not part of the codec): a plain copy kernel of the
 * same launch style, used as the practical bandwidth ceiling and to scale
 * hardware byte counters, and a kernel that writes `bytes` bytes of scratch
 * to evict caches between timed runs.
 */
int svb_copy_u32(uint64_t n, const uint32_t *in, uint32_t *out, void *stream);
int svb_fill_u32(uint64_t n, uint32_t *out, uint32_t value, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SVB_H */
