// Host-side helpers shared by the translation units of librecsplit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "launch.h"
#include "rs_internal.h"

namespace rs {

// Device memory of the library: the caller's allocator (rs_set_allocator) or,
// by default, stream-ordered hipMallocAsync / hipFreeAsync.  Every owner of
// device memory (a call's workspace, a blob arena, a plan) keeps the Alloc
// that made it and frees through it, so the process-wide choice may change
// while older memory is alive.
struct Alloc {
    rs_alloc_fn alloc = nullptr;  // null: the default
    rs_free_fn release = nullptr;
    void* ctx = nullptr;
    // bytes (at least 256) for use on stream s; RS_ENOMEM or RS_EDEVICE on failure
    int get(void** p, size_t bytes, hipStream_t s) const;
    // return p after the work enqueued so far on s (null p is ignored)
    void put(void* p, hipStream_t s) const;
    // return p that no stream uses any more
    void put_idle(void* p) const;
};
Alloc current_alloc();

struct BlobArena;
void release_arena(BlobArena* a);
}  // namespace rs

struct rs_blob {
    uint64_t* words = nullptr;   // serialized structure on the device
    uint64_t bytes = 0;
    uint32_t* tables = nullptr;  // device r, F, N for sizes 0..tab_stride-1, tab_stride words each
    uint32_t tab_stride = 0;
    const uint32_t* samples = nullptr;  // select samples on the device (null: the inventory alone)
    uint64_t header[rs::kHeaderWords] = {};
    hipEvent_t ready = nullptr;      // recorded after the last write of the blob (shared with the arena)
    int device = 0;
    rs::BlobArena* arena = nullptr;  // shared with the other blobs of one build call (null: own memory)
    rs::Alloc al;                    // frees words and tables when the blob owns them
    bool packed = false;             // the packed per-size words hold every size up to the largest bucket
};

namespace rs {

// Sets the calling thread's error message and returns code.
int fail(int code, const char* fmt, ...);
void clear_error();


// Blob geometry decoded from a header.
struct Layout {
    uint64_t n, leaf, bucket, nb, maxm, kind;
    uint32_t Ws, Wz;
    uint32_t gr_max;  // splits above this size take the Sec. 7.2 parameter approximation (0: none)
    uint32_t slack;   // non-minimal variant: leaves map into leaf_range(m, slack) values (0: minimal)
    uint64_t delta_s;
    int64_t delta_z;
    uint64_t beta;
    uint64_t us_words, uz_words, lower_words, tree_words, tree_bits;
    uint64_t hi_words, lo_words;  // inventory
    // word offsets from the start of the blob
    uint64_t lower_off, us_off, uz_off, inv_hi_off, inv_lo_off, tree_off, total_words;
};
Layout layout_of(const uint64_t* header);

// Upload the per-size tables of (leaf, maxm, gr_max, slack) into dst
// (kTableCount * (maxm + 1) u32).
int upload_tables(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack, uint32_t* dst, hipStream_t s);

// Search schedules: the built-in one of a leaf size for a launch over
// `buckets` buckets in all, range checks, and the process-wide table filled by
// the autotuner.
// Built-in search schedule of builds with leaf size `leaf` and bucket size
// `bucket` (0: not known) in a call of `buckets` buckets.
rs_schedule builtin_schedule(uint32_t leaf, uint64_t buckets, uint32_t bucket = 0);
// Expected hash evaluations of the seed searches of n keys in buckets of b
// (trials 1/p times keys for every node of the strategy, bucket sizes taken as
// Poisson(n / ceil(n / b))); the serving loop's model of a request's device work.
double expected_search_evals(uint32_t leaf, uint32_t bucket, uint64_t n);
bool schedule_valid(const rs_schedule& s);
bool schedule_lookup(uint32_t leaf, uint32_t bucket, rs_schedule* out);
void schedule_store(uint32_t leaf, uint32_t bucket, const rs_schedule& s);

}  // namespace rs

#define RS_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return rs::fail(RS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)
