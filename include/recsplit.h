/*
 * librecsplit -- RecSplit minimal perfect hashing on AMD Instinct MI355X (gfx950).
 *
 * A minimal perfect hash function (MPHF) maps a fixed set S of n keys one-to-one
 * onto [0, n) (paper Sec. 1); values for keys outside S are unspecified but
 * deterministic.  RecSplit (Esposito, Mueller Graf, Vigna 2019) builds it by
 * hashing keys to 128-bit signatures, distributing them into buckets of
 * average size b (Sec. 4, Sec. 6.1), and searching, for every bucket, a
 * splitting tree whose inner nodes store the first hash index that splits the
 * node's keys into parts of prescribed sizes and whose leaves (at most l keys)
 * store the first index that is a bijection (Sec. 4, Sec. 5).  Indices are
 * Golomb-Rice coded (eq. (4), Sec. 6.2) and the bucket prefix sums and bit
 * offsets are kept in a double Elias-Fano list (Sec. 6.3, Sec. 7.4).
 *
 * Conventions for every entry point:
 *   - All functions return an rs_status; nothing aborts or throws across the ABI.
 *   - On error, output parameters are left untouched and rs_last_error() returns
 *     a message for the calling thread.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *   - The caller owns key, query and output buffers and must keep them valid
 *     until the work enqueued on the stream has completed.
 *   - The library owns rs_blob objects; free them with rs_blob_free.
 */
#ifndef RECSPLIT_H
#define RECSPLIT_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RS_OK = 0,
    RS_EINVAL = 1,      /* bad argument: l outside [1,24], b = 0, n = 0, NULL pointer,
                           non-monotone offsets, key kind differing from the blob's */
    RS_EDUPLICATE = 2,  /* two keys share a 128-bit signature (duplicate keys), or two keys
                           of one bucket share the lower signature word */
    RS_ENOMEM = 3,      /* a device or host allocation failed */
    RS_EDEVICE = 4,     /* a HIP runtime call failed */
    RS_ESEARCH = 5,     /* an index search reached the seed cap (2^56 unless lowered) */
    RS_EFORMAT = 6,     /* serialized blob has a bad magic, version or size */
    RS_EBUSY = 7        /* serving queue full */
} rs_status;

enum { RS_KEYS_U64 = 1, RS_KEYS_BYTES = 2 };

/* A key set resident in device memory.
 *   RS_KEYS_U64:   data -> uint64_t[n]; offsets = NULL.
 *   RS_KEYS_BYTES: data -> concatenated key bytes; offsets -> uint64_t[n+1], key i is
 *                  data[offsets[i] .. offsets[i+1]); offsets must be non-decreasing. */
typedef struct {
    uint32_t kind;
    const void* data;
    const uint64_t* offsets;
    uint64_t n;
} rs_keys;

typedef struct rs_blob rs_blob; /* opaque; immutable after build; safe for concurrent lookups */

/* Device memory.  Every device buffer of the library (a call's workspace, the
 * per-size tables, blob arenas, plan buffers, the autotuner's calibration keys)
 * comes from one process-wide allocator, by default stream-ordered
 * hipMallocAsync / hipFreeAsync.  rs_set_allocator installs the caller's
 * instead, e.g. PyTorch's caching allocator (the Python binding does so), so
 * that the library's memory is counted and reused with the caller's own.
 *   alloc(bytes, stream, ctx): return 256-byte aligned device memory of at
 *     least `bytes` bytes on the current device, for work enqueued on `stream`
 *     (a hipStream_t); NULL = out of memory, and the call fails with RS_ENOMEM.
 *   release(ptr, stream, ctx): give ptr back.  With a non-NULL stream the
 *     memory may still be in use by work already enqueued on that stream (it
 *     is free once that work is done, as with hipFreeAsync); with stream ==
 *     NULL no device work uses it any more.
 * Both NULL restores the default; exactly one NULL is RS_EINVAL.  The setting
 * applies to allocations made after the call, from any thread; memory keeps
 * the allocator that made it and is released through it, so alloc, release
 * and ctx must stay valid until every blob, plan and server created while they
 * were installed has been freed.  The functions may be called from the
 * library's server threads and must be thread-safe.  No device is needed. */
typedef void* (*rs_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*rs_free_fn)(void* ptr, void* stream, void* ctx);
int rs_set_allocator(rs_alloc_fn alloc, rs_free_fn release, void* ctx);

/* Build options (all-zero = defaults).
 *   seed_cap  : lowers the search cap of every split and bijection index
 *               (0 = 2^56); it exists to exercise the RS_ESEARCH path.
 *   gr_table_max: splits of more than this many keys take their Golomb-Rice
 *               parameter from the paper's integer approximation for large
 *               buckets (Sec. 7.2), every other node from eq. (4) (0 = eq. (4)
 *               for every node).  The value is recorded in the structure
 *               (header word 7, bits 16 and up), so lookups and
 *               rs_blob_from_host follow it.
 *   flags     : RS_OPT_TIMING records HIP events around each construction phase
 *               on the build stream (read them with rs_last_build_stats); the
 *               build then waits for the stream before returning.
 *               RS_OPT_TUNED takes each build's search schedule from the
 *               process-wide schedule table (rs_autotune, rs_schedule_set) when
 *               the table has an entry for its (l, b); builds without an entry
 *               use the built-in schedule.
 *               RS_OPT_NO_SAMPLES builds blobs without select samples (see
 *               rs_blob_bytes): about 0.5 byte per bucket less device memory,
 *               and lookups start their selects at the two-level inventory.
 *   stage_from, group_max, waves: schedule overrides for every build of the
 *               call (0 = keep the table's or built-in value), as in rs_schedule.
 *   wait_limit: when several wavefronts share a bucket's tree, a wavefront
 *               waiting for a node whose parent is still being searched waits
 *               as long as some wavefront of the bucket reports progress; it
 *               gives up (and the build fails with RS_EDEVICE, "search
 *               scheduling failed") only after wait_limit sleeps of about
 *               0.1 us with no progress at all, which the node order rules out
 *               in a correct build.  0 = 2^25 (several seconds).  Small values
 *               exist to exercise that error path.
 *   leaf_slack: 0 builds the minimal structure.  A value in [1, 255] builds
 *               the non-minimal variant that Sec. 9 proposes (a larger
 *               codomain): every leaf of m >= 2 keys takes the first index
 *               whose hash is injective into m + ceil(m leaf_slack / 256)
 *               values, a subtree covers the sum of its parts' ranges, and
 *               the first Elias-Fano list holds the prefix sums of the
 *               buckets' ranges instead of their sizes.  Lookups then map the
 *               n keys one-to-one into [0, R), R = the sum of all bucket
 *               ranges (the last entry of that list); the value is recorded
 *               in the structure (header word 7, bits 40-47).  RS_EINVAL when
 *               l + ceil(l leaf_slack / 256) exceeds 32.
 * Schedules never change the result, only the time it takes. */
enum { RS_OPT_TIMING = 1, RS_OPT_TUNED = 2, RS_OPT_NO_SAMPLES = 4 };
typedef struct {
    uint64_t seed_cap;
    uint32_t flags;
    uint32_t stage_from;
    uint32_t group_max;
    uint32_t waves;
    uint32_t wait_limit;
    uint32_t gr_table_max;
    uint32_t leaf_slack;
} rs_options;

/* Search schedule of one (l, b) pair.  The seed search runs one workgroup per
 * bucket; these knobs set how its lanes and wavefronts share the work.
 *   stage_from: leaves of at least this many keys use the staged (early-exit)
 *               bijection search, smaller ones try 64 candidates on every key
 *               (2..25; 25 = none of 16 keys or fewer; built-in 9).  Leaves of
 *               17 or more keys are always staged.
 *   group_max : 1 + the largest log2 of lanes that share one split candidate
 *               (1 = one lane per candidate .. 7 = up to 64; built-in 7).  The
 *               lanes per candidate of each node size come from its expected
 *               number of trials, capped here.
 *   waves     : wavefronts per bucket workgroup: 1, 2, 4 or 8.  Built-in, by
 *               the buckets B of the whole call: for l <= 8, 4 if B <= 4096,
 *               2 if B <= 40000, else 1; for 9 <= l <= 12, 8 if B <= 256,
 *               else 4; for l > 12, 4.
 *   search_ms : rs_autotune: time of the calibration search with this schedule.
 *   default_ms: rs_autotune: time of the same search with the built-in schedule.
 *   tune_ms   : rs_autotune: wall time the tuning took. */
typedef struct {
    uint32_t stage_from;
    uint32_t group_max;
    uint32_t waves;
    uint32_t variants;  /* rs_autotune: schedules timed */
    double search_ms;
    double default_ms;
    double tune_ms;
} rs_schedule;

/* Pick the search schedule of (leaf, bucket) by timing the seed search on a
 * synthetic calibration key set in device memory (distinct uniform random
 * 64-bit keys).
 *   keys_hint: size of the builds the schedule is for (the sum over a batch);
 *              the calibration set has that many keys, at most 2^25 and at most
 *              what about ten searches within the budget allow.  0 = ten times
 *              the bucket workgroups the device holds at once.
 *   budget_ms: search time to spend (0 = 3000 ms).  The built-in schedule and
 *              one variant are always timed.
 * The search runs for at least 100 ms before any timing (clocks ramp up
 * under load).  The built-in schedule is timed first.  Then each knob is
 * tried in turn (wavefronts per bucket, stage_from, group_max), and a change
 * is kept only when it is more than 2% faster.  The winner is stored in the
 * process-wide table and returned in *out (which may be NULL).  Work is
 * enqueued on stream, and the call waits for it.
 * Errors: RS_EINVAL (l outside [1,24], b = 0), RS_ENOMEM, RS_EDEVICE. */
int rs_autotune(uint32_t leaf, uint32_t bucket, uint64_t keys_hint, double budget_ms, void* stream,
                rs_schedule* out);

/* Read (RS_EINVAL if the table has no entry) or write the process-wide table
 * entry of (leaf, bucket); set validates the knobs (RS_EINVAL if out of range)
 * and is how a caller restores a schedule saved from an earlier process.
 * Thread-safe.  rs_schedule_clear empties the table. */
int rs_schedule_get(uint32_t leaf, uint32_t bucket, rs_schedule* out);
int rs_schedule_set(uint32_t leaf, uint32_t bucket, const rs_schedule* schedule);
void rs_schedule_clear(void);

/* Per-phase device times (milliseconds, from HIP events on the build stream)
 * and sizes of the calling thread's last successful rs_build_ex with
 * RS_OPT_TIMING. */
typedef struct {
    double ms_signature;  /* signatures + bucket histogram + prefix sums */
    double ms_scatter;    /* bucket-contiguous scatter */
    double ms_search;     /* seed search kernel (the hot loop) */
    double ms_offsets;    /* bit-length prefix sums and Elias-Fano gaps */
    double ms_fill;       /* Elias-Fano bits and Golomb-Rice streams */
    double ms_device;     /* first to last event */
    uint64_t n, nb, maxm, tree_bits, blob_bytes;
    uint64_t arena_bytes; /* device memory the blob lives in: blob_bytes when the
                             arena was sized after the search; larger when a single
                             build of a shape seen before on this thread filled an
                             arena guessed from it, before the call's one wait */
    uint64_t refills;     /* 1 if the guessed arena was too small and the blob was
                             filled again into an exact one */
} rs_build_stats;

int rs_last_build_stats(rs_build_stats* out);

/* Build the MPHF of a key set (construction of Sec. 4-6 of the paper).
 *   keys   : device key set, n >= 1 distinct keys.
 *   leaf   : leaf size l, 1 <= l <= 24 (Sec. 5: l <= 24 keeps Golomb-Rice parameters
 *            below 32).
 *   bucket : average bucket size b >= 1; nb = ceil(n / b) buckets (Sec. 6.1), at
 *            most 2^28 (268,435,456) in one call, counting every build of a
 *            batch (RS_EINVAL beyond).
 *   stream : HIP stream; all device work is enqueued on it.  The call waits on the
 *            stream once, for the blob size: the search is sized for a
 *            bucket-size cap estimated from n and b (a bucket count is
 *            exceeded with probability below 1e-6); if a bucket is larger
 *            (skewed keys), the construction runs again sized for the
 *            largest bucket, with the same result.  When the calling thread's
 *            last single build had this shape (leaf, bucket, gr_table_max,
 *            leaf_slack, select samples or not) and a key count within a
 *            factor of two, the blob is written before that wait
 *            into memory sized from the earlier build (with
 *            a 1/8 margin; the environment variable RS_ARENA_GUESS scales it,
 *            0 turns it off); a blob that does not fit is written again after
 *            the wait into memory of its exact size.
 *   out    : receives the new blob; its device bytes are valid once the stream
 *            reaches the end of the enqueued work.
 * Errors: RS_EINVAL, RS_EDUPLICATE, RS_ENOMEM, RS_EDEVICE, RS_ESEARCH. */
int rs_build(const rs_keys* keys, uint32_t leaf, uint32_t bucket, void* stream, rs_blob** out);

/* rs_build with options (opts may be NULL). */
int rs_build_ex(const rs_keys* keys, uint32_t leaf, uint32_t bucket, const rs_options* opts, void* stream,
                rs_blob** out);

/* Build many independent MPHFs in one call (buckets of all builds are independent,
 * Sec. 4): one signature pass, one search launch over the buckets of every
 * build (one workgroup per bucket), one encoding pass; each blob is
 * byte-identical to the one rs_build makes for the same keys, l and b.
 *   sets[count]            : device key sets (kinds may differ between builds).
 *   leaf[count], bucket[count]: per-build l and b.
 *   outs[count]            : receives one blob per successful build, NULL otherwise.
 *   per_build_status[count]: optional; an rs_status per build.
 * Returns RS_OK if every build succeeded, else the status of the first failed build
 * (the other builds' blobs are still returned).  The blobs of one call share one
 * device allocation, released when the last of them is freed. */
int rs_build_batch(const rs_keys* sets, uint32_t count, const uint32_t* leaf, const uint32_t* bucket,
                   const rs_options* opts, void* stream, rs_blob** outs, int* per_build_status);

/* Build plans: the whole construction of a fixed batch shape (the same key
 * buffers, sizes, l and b) captured once into a HIP graph, for callers that
 * rebuild the same sets again and again as their contents change.  A run is
 * one graph launch and one wait, with no host round trip between phases.
 *   rs_plan_create: makes an ordinary rs_build_batch first; its blobs go to
 *     first_outs (NULL: freed) and its statuses to per_build_status.  The plan
 *     then sizes the search for a bucket cap (the largest bucket seen plus
 *     four standard deviations of a Poisson count, within the local data
 *     share) and the blob arena for a word cap (the blobs' words plus 1/8),
 *     and captures every phase on a stream of its own.  Fails, without a plan,
 *     if any build of the first call fails.  The key buffers in sets must stay
 *     allocated, at the same addresses and sizes, until rs_plan_destroy.
 *   rs_plan_run: rebuilds every set from the buffers' current contents on
 *     stream and returns new blobs, exactly as rs_build_batch would (and owned
 *     like them).  If a bucket or the blobs exceed the caps, that run falls
 *     back to an ordinary rs_build_batch (counted in rs_plan_info).  One
 *     thread at a time per plan.
 *   rs_plan_info: bucket cap, arena words, runs and fallbacks so far.
 * Errors: RS_EINVAL, RS_ENOMEM, RS_EDEVICE, and the build errors of
 * rs_build_batch. */
typedef struct rs_plan rs_plan;
int rs_plan_create(const rs_keys* sets, uint32_t count, const uint32_t* leaf, const uint32_t* bucket,
                   const rs_options* opts, void* stream, rs_plan** out, rs_blob** first_outs,
                   int* per_build_status);
int rs_plan_run(rs_plan* plan, void* stream, rs_blob** outs, int* per_build_status);
int rs_plan_info(const rs_plan* plan, uint32_t* bucket_cap, uint64_t* capacity_words, uint64_t* runs,
                 uint64_t* fallbacks);
void rs_plan_destroy(rs_plan* plan);

/* rs_build for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It calls no hipMalloc,
 * hipFree, pinned-host or other allocating device routine (host bookkeeping
 * uses a few small heap objects).  The workspace and tables of the call live
 * in a device array of 64 MiB that every GPU the library runs on holds from
 * the time the library's kernels are loaded there until the process ends; key
 * sets whose workspace (about 44 bytes per key plus 24 per bucket) and tables
 * do not fit are refused with RS_EINVAL and a message, before any device work.
 *   keys, leaf, bucket: as for rs_build.
 *   blob_dev, blob_cap: the caller's device buffer and its size in bytes; the
 *     serialized structure (the bytes rs_blob_to_host gives for rs_build's
 *     blob of the same keys, l and b) is written there.
 *   blob_bytes: receives the structure's size.  If blob_dev is NULL or
 *     blob_cap is smaller, the call fails with RS_EINVAL and still sets
 *     *blob_bytes to the size needed (after the whole search has run).
 *   stream: all device work is enqueued on it; the call waits for it three
 *     times and returns when the structure is complete.
 * All calls on a GPU share that GPU's array, which keeps the last call's
 * contents (every call rewrites what it reads).  Calls that overlapped on one
 * GPU would race on it, so the library serializes them: one call at a time
 * per process, and a call returns only once its device work is done.
 * Errors: as rs_build, and RS_EINVAL for key sets beyond the array. */
int rs_build_noalloc(const rs_keys* keys, uint32_t leaf, uint32_t bucket, void* blob_dev, uint64_t blob_cap,
                     uint64_t* blob_bytes, void* stream);

/* Rank of each query (lookup of Sec. 4 and Sec. 6.2): ranks_dev[i] = f(queries[i]).
 * Members of the built set get distinct values in [0, n).  Other keys get a
 * deterministic value in [0, n] (n only when their bucket is the last one and
 * is empty), the same value the CPU reference computes.
 *   queries  : device key set of the same kind as the blob.
 *   ranks_dev: device uint64_t[queries->n], written asynchronously on stream (which
 *              first waits for the blob's construction if that ran on another stream).
 * Errors: RS_EINVAL (NULL, kind mismatch), RS_EDEVICE. */
int rs_lookup(const rs_blob* blob, const rs_keys* queries, uint64_t* ranks_dev, void* stream);

/* Size in bytes of the serialized structure (header + Elias-Fano + trees).  A blob
 * also holds, in device memory beside the structure, its select samples (the
 * position of every 16th one of both Elias-Fano upper-bits arrays, 4 bytes each,
 * about 0.5 byte per bucket), from which rs_lookup starts its selects; they are not
 * part of the serialized bytes.  A structure of more than (2^32 - 1) / 3 - 1 buckets,
 * whose bit positions would not fit 32 bits, has none: its lookups start at the
 * two-level inventory. */
uint64_t rs_blob_bytes(const rs_blob* blob);

/* Copy the serialized structure to host memory dst (capacity cap bytes); waits until
 * the blob is complete.  Errors: RS_EINVAL (cap too small, NULL). */
int rs_blob_to_host(const rs_blob* blob, void* dst, uint64_t cap);

/* Load a serialized structure from host memory into a new device blob (its select
 * samples, within the bucket bound given at rs_blob_bytes, are computed from the
 * structure's inventory).
 * Errors: RS_EFORMAT (magic, version, size), RS_ENOMEM, RS_EDEVICE. */
int rs_blob_from_host(const void* src, uint64_t bytes, void* stream, rs_blob** out);

/* Device address of the serialized bytes (read-only; rs_blob_bytes long). */
const void* rs_blob_device_ptr(const rs_blob* blob);

/* Number of keys, leaf size and bucket size the blob was built with. */
int rs_blob_info(const rs_blob* blob, uint64_t* n, uint32_t* leaf, uint32_t* bucket);

/* Release a blob (waits until it is complete; blobs of one rs_build_batch call share
 * one allocation, freed with the last of them).  NULL is ignored. */
void rs_blob_free(rs_blob* blob);

/* Message describing the last error of the calling thread ("" if none). */
const char* rs_last_error(void);

/* ---- Serving loop ---------------------------------------------------------------
 * Build and lookup requests of uneven sizes arrive over time.  Build requests wait
 * in first-in first-out order and are admitted when their estimated device
 * footprint (about 56 bytes per key) fits in the free part of the budget (one is
 * always admitted when nothing is in flight).  Each of `build_workers` workers owns
 * a stream and runs the request at the head of the queue and every admissible
 * waiting request of the same leaf size as one rs_build_batch call (the requests of
 * a batch complete together, so short and long searches are not mixed), so
 * requests that arrive while a batch is on the device overlap with it in the next
 * worker's batch.  Lookups run on their own stream.  A request's result is the same
 * as rs_build / rs_lookup on the same inputs.
 * The caller keeps key and query buffers valid until the request completes. */
typedef struct rs_server rs_server;

typedef struct {
    uint64_t batches, batched_requests, max_batch, max_concurrent_batches;
    uint64_t peak_in_flight_bytes, budget_bytes;
    uint32_t max_queue;
    uint32_t lookup_cus;  /* compute units kept free of build work (0: none) */
} rs_server_stats;

/* Start a server with a device-memory budget for builds in flight (bytes) and
 * `build_workers` build streams (0 = 2, at most 8); opts as for rs_build_ex (its
 * RS_OPT_TIMING flag is ignored). */
int rs_server_create(uint64_t hbm_budget_bytes, uint32_t build_workers, const rs_options* opts, rs_server** out);

/* Server configuration for rs_server_create_ex.
 *   hbm_budget_bytes, build_workers: as for rs_server_create.
 *   lookup_cus: compute units that heavy builds (a modelled search of 0.25 s
 *     or more) never use (a CU mask on the stream they run on), taken evenly
 *     from every XCD; lookups and light builds run on all CUs and so always
 *     find these free, even when every other CU runs long seed-search
 *     workgroups.  0 = none; at most the CU count of one XCD (32 on
 *     MI355X), best a multiple of the XCD count (8). */
typedef struct {
    uint64_t hbm_budget_bytes;
    uint32_t build_workers;
    uint32_t lookup_cus;
    uint32_t reserved[4];
} rs_server_config;

int rs_server_create_ex(const rs_server_config* config, const rs_options* opts, rs_server** out);

/* Enqueue a build; *ticket identifies it.  Errors: RS_EINVAL, RS_EBUSY (stopping). */
int rs_server_submit_build(rs_server* srv, const rs_keys* keys, uint32_t leaf, uint32_t bucket, uint64_t* ticket);

/* Enqueue a lookup of queries against a built blob; ranks_dev as for rs_lookup. */
int rs_server_submit_lookup(rs_server* srv, const rs_blob* blob, const rs_keys* queries, uint64_t* ranks_dev,
                            uint64_t* ticket);

/* Non-blocking: *done = 0 while running; when done, the request's status, its blob
 * (builds; the caller then owns it), its latency (submission to completion, ms) and
 * the number of requests of its batch are returned and the ticket is retired. */
int rs_server_poll(rs_server* srv, uint64_t ticket, int* done, int* status, rs_blob** blob, double* latency_ms,
                   uint32_t* batch_size);

/* Blocking variant of rs_server_poll. */
int rs_server_wait(rs_server* srv, uint64_t ticket, int* status, rs_blob** blob, double* latency_ms,
                   uint32_t* batch_size);

int rs_server_get_stats(rs_server* srv, rs_server_stats* out);

/* Finish every queued request, stop the workers and free the server (blobs that
 * were never collected are freed). */
void rs_server_destroy(rs_server* srv);

/* The per-size tables a structure with leaf size l uses, for node sizes
 * m = 0..maxm (host arrays of maxm+1 entries each, written by the call):
 *   r[m]: Golomb-Rice parameter of a node of m keys, eq. (4) with the exact
 *         success probability of eq. (2) (leaves: m!/m^m, Sec. 5);
 *   F[m]: fixed-part bits of a whole subtree on m keys (Sec. 6.2);
 *   N[m]: coded nodes of that subtree (nodes with at least 2 keys).
 * Host only; no device is needed.  Errors: RS_EINVAL (l outside [1,24], NULL),
 * RS_ENOMEM. */
int rs_tables(uint32_t leaf, uint32_t maxm, uint32_t* r, uint32_t* F, uint32_t* N);

/* rs_tables of a structure built with rs_options.gr_table_max = gr_table_max:
 * r of split nodes above that size follows the integer approximation of
 * Sec. 7.2 (and F with it). */
int rs_tables_ex(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t* r, uint32_t* F, uint32_t* N);

/* The same tables as one 32-bit word per size (footnote of Sec. 7.2: one such
 * table suffices for l >= 4 and b <= 2000): bits 0-4 hold r[m], bits 5-15
 * N[m] and bits 16-31 F[m].  Lookups read it instead of the three arrays when
 * every size of the structure fits.  packed: host array of maxm+1 words.
 * Errors: RS_EINVAL (l outside [1,24], NULL, or some size up to maxm does not
 * fit the fields), RS_ENOMEM. */
int rs_tables_packed(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t* packed);

/* rs_tables_ex of a structure built with rs_options.leaf_slack = leaf_slack,
 * plus Q[m], the output values of a subtree of m keys (m for the minimal
 * structure; leaves m + ceil(m leaf_slack / 256); splits the sum over their
 * parts).  r of a leaf follows its injection probability
 * prod_{i<m} (M - i) / M with M = Q[m].  Host arrays of maxm+1 entries.
 * Errors: RS_EINVAL (l outside [1,24], leaf_slack > 255, a leaf range above
 * 32, NULL), RS_ENOMEM. */
int rs_tables_range(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t leaf_slack, uint32_t* r,
                    uint32_t* F, uint32_t* N, uint32_t* Q);

/* Library version string. */
const char* rs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RECSPLIT_H */
