// Construction of a RecSplit structure on the GPU (Sec. 4-7 of the paper).
//
// Pipeline for one or many independent builds at once, all on the caller's
// stream: signatures + bin histogram -> bin offsets -> scatter into bin order
// -> per-bin bucket sort (prefix sums s_i, keys in bucket order) -> seed search
// (one workgroup per bucket, one lane per candidate index) -> scan of bucket
// bit lengths (offsets o_i) -> Elias-Fano minimum gaps per build -> blob
// geometry -> Elias-Fano bits + Golomb-Rice streams written into the blobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <string>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rs_host.h"
#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

// Status words of a call and n zeroed counters; and in_words words of the
// call's bases and descriptors read from pinned host memory (in_words = 0
// when a copy brought them).
__global__ void k_reset(DevStatus* st, unsigned long long* counters, uint64_t n, uint64_t* __restrict__ in_dst,
                        const uint64_t* __restrict__ in_src, uint64_t in_words) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (uint64_t)gridDim.x * blockDim.x;
    if (t == 0) {
        st->maxm = 0;
        st->flags = 0;
        st->delta_s = ~0ull;
        st->delta_z = 0x7fffffffffffffffll;
    }
    for (uint64_t i = t; i < n; i += step) counters[i] = 0;
    for (uint64_t i = t; i < in_words; i += step) in_dst[i] = in_src[i];
}

// ---------------------------------------------------------------------------
// Builds of one call.  Several independent key sets are built together: their
// keys and buckets are numbered consecutively (key_base, bucket_base) and every
// kernel finds the build of an index by binary search over those bases.
// ---------------------------------------------------------------------------
struct BuildDesc {
    const void* data;
    const uint64_t* offsets;
    uint64_t n, key_base, nb, bucket_base;
    uint32_t kind, leaf, lower, upper;
    uint32_t tab;      // index of this build's leaf-size tables in the table arena
    uint32_t aligned;  // byte keys start on an 8-byte boundary
    // search schedule of this build
    uint32_t stage_from;  // leaves of at least this many keys use the staged bijection search
    uint32_t group_cap;   // cap on log2 lanes per split candidate
    uint32_t waves;       // wavefronts of the bucket's workgroup that take nodes
    uint32_t bucket;      // the caller's bucket size b (header word)
    uint32_t gr_max;      // splits above this size use the Sec. 7.2 approximation (0: none; header)
    uint32_t slack;       // non-minimal variant: leaves map into leaf_range(m, slack) values (0: minimal)
    // written by the device
    uint32_t maxm, flags;
    unsigned long long delta_s;
    long long delta_z;
    unsigned long long total_bits;
    unsigned long long range_total;  // last value of the first Elias-Fano list (n for the minimal structure)
    // written by the host once the sizes are known
    unsigned long long* blob;  // null: no blob for this build
    uint64_t beta;
    uint64_t lower_off, us_off, uz_off, inv_hi_off, inv_lo_off, tree_off;
    uint64_t samples_off;  // select samples after the blob in its arena slot (0: none)
    uint32_t Ws, Wz;
};

// Largest j with base[j] <= x (base[0] = 0, strictly increasing, count entries).
__device__ __forceinline__ uint32_t find_build(const uint64_t* __restrict__ base, uint32_t count, uint64_t x) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Signatures (Sec. 6.1) and the bin histogram.
//
// Keys reach bucket order by a two-level counting sort.  Buckets are grouped
// into bins of 2^shift consecutive global bucket numbers (a few thousand keys
// each).  The signature pass counts keys per bin in LDS and adds each block's
// counts to the global bin counters.  The bin scatter moves (lower word, bucket) pairs
// into bin order, a contiguous run per (block, bin).  One workgroup per bin
// then counts its buckets in LDS, writes their prefix sums and places each key
// in its bucket.  Order inside a bucket is irrelevant: every later step is a
// function of the bucket's key set.
// ---------------------------------------------------------------------------
constexpr uint32_t kSigItems = 32;                 // keys per thread in the signature and bin passes
constexpr uint32_t kSigTile = kBlock * kSigItems;  // keys per block
constexpr uint32_t kMaxBins = 4096;
constexpr uint32_t kMaxBinShift = 16;              // at most 65536 buckets per bin (eight pieces)
constexpr uint32_t kSortSpan = 8192;               // buckets a per-bin sort counts at once in LDS
constexpr uint32_t kSortBlock = 512;               // threads of the per-bin sort
constexpr uint32_t kSortItems = 8;                 // keys a thread of the sort loads at once

// dynamic LDS: nbins u32 counters
__global__ __launch_bounds__(kBlock) void k_signature(const BuildDesc* __restrict__ descs, BuildDesc* __restrict__ wdescs,
                                                     const uint64_t* __restrict__ key_base, uint32_t count,
                                                     uint64_t total, uint64_t* __restrict__ lo_out,
                                                     uint32_t* __restrict__ bid, uint32_t shift, uint32_t nbins,
                                                     uint32_t nxcd, unsigned long long* __restrict__ bin_cnt) {
    extern __shared__ uint32_t hist[];
    for (uint32_t c = threadIdx.x; c < nbins; c += kBlock) hist[c] = 0;
    __syncthreads();
    const uint64_t tile0 = (uint64_t)blockIdx.x * kSigTile;
    const uint64_t base = tile0 + threadIdx.x;
    const uint64_t tile_last = min(total, tile0 + kSigTile) - 1;
    const uint32_t j0 = __builtin_amdgcn_readfirstlane(find_build(key_base, count, tile0));
    const uint32_t j1 = __builtin_amdgcn_readfirstlane(find_build(key_base, count, tile_last));
    auto emit = [&](uint64_t i, const BuildDesc& B, uint64_t hi, uint64_t lo) {
        const uint32_t b = (uint32_t)(bucket_of(hi, B.nb) + B.bucket_base);
        lo_out[i] = lo;
        bid[i] = b;
        atomicAdd(&hist[b >> shift], 1u);
    };
    constexpr uint32_t kGroup = 8;
    if (j0 == j1) {
        // the whole tile belongs to one build: groups of independent loads
        const BuildDesc& B = descs[j0];
        const uint64_t kb = B.key_base;
        if (B.kind == RS_KEYS_U64) {
            const uint64_t* keys = static_cast<const uint64_t*>(B.data);
#pragma unroll
            for (uint32_t g = 0; g < kSigItems; g += kGroup) {
                uint64_t key[kGroup];
#pragma unroll
                for (uint32_t u = 0; u < kGroup; u++) {
                    const uint64_t i = base + (uint64_t)(g + u) * kBlock;
                    key[u] = i < total ? keys[i - kb] : 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kGroup; u++) {
                    const uint64_t i = base + (uint64_t)(g + u) * kBlock;
                    if (i >= total) continue;
                    uint64_t hi, lo;
                    signature_u64(key[u], hi, lo);
                    emit(i, B, hi, lo);
                }
            }
        } else {
            // four strings at a time: their words and states in registers (eight
            // held 158 VGPRs, three wavefronts per SIMD)
            constexpr uint32_t kGroupS = 4;
            const uint64_t* off = B.offsets;
            const uint8_t* data = static_cast<const uint8_t*>(B.data);
            const uint64_t bytes = off[B.n];
            const bool aligned = B.aligned != 0;
            for (uint32_t g = 0; g < kSigItems; g += kGroupS) {
                uint64_t st[kGroupS], en[kGroupS], a[kGroupS], c[kGroupS];
                uint64_t longest = 0;
#pragma unroll
                for (uint32_t u = 0; u < kGroupS; u++) {
                    const uint64_t i = base + (uint64_t)(g + u) * kBlock;
                    st[u] = en[u] = 0;
                    if (i < total) {
                        st[u] = off[i - kb];
                        en[u] = off[i - kb + 1];
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kGroupS; u++) {
                    if (en[u] < st[u] || en[u] > bytes) {
                        atomicOr(&wdescs[j0].flags, kFlagOffsets);
                        en[u] = st[u] = min(st[u], bytes);
                    }
                    const uint64_t len = en[u] - st[u];
                    a[u] = kSigHi ^ len;
                    c[u] = kSigLo ^ len;
                    longest = max(longest, len);
                }
                for (uint64_t p = 0; p < longest; p += 8) {
#pragma unroll
                    for (uint32_t u = 0; u < kGroupS; u++) {
                        if (st[u] + p < en[u]) {
                            const uint64_t w = string_word(data, bytes, aligned, st[u] + p, en[u]);
                            a[u] = mix64(a[u] ^ w);
                            c[u] = mix64(c[u] + w);
                        }
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kGroupS; u++) {
                    const uint64_t i = base + (uint64_t)(g + u) * kBlock;
                    if (i < total) emit(i, B, mix64(a[u]), mix64(c[u]));
                }
            }
        }
    } else {
        for (uint32_t it = 0; it < kSigItems; it++) {
            const uint64_t i = base + (uint64_t)it * kBlock;
            if (i >= total) break;
            const uint32_t j = find_build(key_base, count, i);
            const BuildDesc& B = descs[j];
            const uint64_t k = i - B.key_base;
            uint64_t hi, lo;
            if (B.kind == RS_KEYS_U64) {
                signature_u64(static_cast<const uint64_t*>(B.data)[k], hi, lo);
            } else {
                const uint64_t* off = B.offsets;
                uint64_t s = off[k], e = off[k + 1], bytes = off[B.n];
                if (e < s || e > bytes) {
                    atomicOr(&wdescs[j].flags, kFlagOffsets);
                    e = s = min(s, bytes);
                }
                signature_bytes(static_cast<const uint8_t*>(B.data), bytes, B.aligned != 0, s, e, hi, lo);
            }
            emit(i, B, hi, lo);
        }
    }
    __syncthreads();
    const uint32_t x = blockIdx.x % nxcd;
    for (uint32_t c = threadIdx.x; c < nbins; c += kBlock)
        if (hist[c]) atomicAdd(&bin_cnt[c * nxcd + x], (unsigned long long)hist[c]);
}

// dynamic LDS: nbins u64 bases, then nbins u32 counters
__global__ __launch_bounds__(kBlock) void k_bin_scatter(const uint64_t* __restrict__ lo, const uint32_t* __restrict__ bid,
                                                       uint64_t total, uint32_t shift, uint32_t nbins,
                                                       uint32_t nxcd, unsigned long long* __restrict__ bin_cur,
                                                       uint64_t* __restrict__ bin_lo, uint32_t* __restrict__ bin_bid) {
    extern __shared__ unsigned long long bases[];
    uint32_t* hist = reinterpret_cast<uint32_t*>(bases + nbins);
    for (uint32_t c = threadIdx.x; c < nbins; c += kBlock) hist[c] = 0;
    __syncthreads();
    // every load of the tile is issued before the first use (independent loads
    // keep the memory pipeline full; a loop of dependent steps would wait on each)
    const uint64_t base = (uint64_t)blockIdx.x * kSigTile + threadIdx.x;
    uint32_t b[kSigItems];
#pragma unroll
    for (uint32_t it = 0; it < kSigItems; it++) {
        const uint64_t i = base + (uint64_t)it * kBlock;
        b[it] = i < total ? bid[i] : ~0u;
    }
#pragma unroll
    for (uint32_t it = 0; it < kSigItems; it++)
        if (b[it] != ~0u) atomicAdd(&hist[b[it] >> shift], 1u);
    __syncthreads();
    // reserve this block's run in every bin it touches, inside the part of the bin
    // that blocks of its XCD fill (consecutive runs then meet in one L2); the
    // counters restart as cursors
    const uint32_t x = blockIdx.x % nxcd;
    for (uint32_t c = threadIdx.x; c < nbins; c += kBlock) {
        const uint32_t h = hist[c];
        if (h) bases[c] = atomicAdd(&bin_cur[c * nxcd + x], (unsigned long long)h);
        hist[c] = 0;
    }
    __syncthreads();
    constexpr uint32_t kGroup = 8;
#pragma unroll
    for (uint32_t g = 0; g < kSigItems; g += kGroup) {
        uint64_t v[kGroup];
#pragma unroll
        for (uint32_t u = 0; u < kGroup; u++) {
            const uint64_t i = base + (uint64_t)(g + u) * kBlock;
            v[u] = i < total ? lo[i] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kGroup; u++) {
            if (b[g + u] == ~0u) continue;
            const uint32_t c = b[g + u] >> shift;
            const uint64_t pos = bases[c] + atomicAdd(&hist[c], 1u);
            bin_lo[pos] = v[u];
            bin_bid[pos] = b[g + u];
        }
    }
}

// The same scatter with the tile reordered by bin in LDS first, so that the
// writes of a block's run in each bin leave from consecutive lanes to
// consecutive addresses (the plain scatter sends every lane's key to another
// bin and its partial-line writes multiply the bytes written).  kScatterBlock
// threads, kScatterItems keys each (the same 8192-key tile as the signature
// pass); at most kScatterMaxBins bins.  Dynamic LDS: the tile's lower words
// and bucket numbers (12 B per key), then per bin the global run base (u64),
// the count (u32) and the tile-local start (u32).
constexpr uint32_t kScatterBlock = 512;
constexpr uint32_t kScatterItems = kSigTile / kScatterBlock;
constexpr uint32_t kScatterMaxBins = 1024;
static_assert(kScatterItems * kScatterBlock == kSigTile, "the scatter takes the signature pass's tiles");

size_t staged_scatter_lds(uint32_t nbins) { return (size_t)kSigTile * 12 + (size_t)nbins * 16; }

__global__ __launch_bounds__(kScatterBlock) void k_bin_scatter_staged(
    const uint64_t* __restrict__ lo, const uint32_t* __restrict__ bid, uint64_t total, uint32_t shift, uint32_t nbins,
    uint32_t nxcd, unsigned long long* __restrict__ bin_cur, uint64_t* __restrict__ bin_lo,
    uint32_t* __restrict__ bin_bid) {
    extern __shared__ uint64_t smem[];
    uint64_t* s_lo = smem;
    uint32_t* s_bid = reinterpret_cast<uint32_t*>(s_lo + kSigTile);
    unsigned long long* bases = reinterpret_cast<unsigned long long*>(s_bid + kSigTile);
    uint32_t* hist = reinterpret_cast<uint32_t*>(bases + nbins);
    uint32_t* lstart = hist + nbins;
    __shared__ uint32_t wsum[kScatterBlock / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (uint32_t c = tid; c < nbins; c += kScatterBlock) hist[c] = 0;
    __syncthreads();
    const uint64_t tile0 = (uint64_t)blockIdx.x * kSigTile;
    const uint32_t count = (uint32_t)min<uint64_t>(kSigTile, total - tile0);
    // bucket numbers in, and each key's rank among the tile's keys of its bin
    uint32_t b[kScatterItems], r[kScatterItems];
#pragma unroll
    for (uint32_t it = 0; it < kScatterItems; it++) {
        const uint32_t e = it * kScatterBlock + tid;
        b[it] = e < count ? bid[tile0 + e] : ~0u;
    }
#pragma unroll
    for (uint32_t it = 0; it < kScatterItems; it++)
        r[it] = b[it] != ~0u ? atomicAdd(&hist[b[it] >> shift], 1u) : 0;
    __syncthreads();
    // tile-local bin starts (exclusive scan, two bins per thread) and the
    // block's run in every bin it touches, inside its XCD's part of the bin
    const uint32_t c0 = 2 * tid;
    const uint32_t h0 = c0 < nbins ? hist[c0] : 0, h1 = c0 + 1 < nbins ? hist[c0 + 1] : 0;
    uint32_t x = h0 + h1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (uint32_t w = 0; w < kScatterBlock / 64; w++) pre += w < wid ? wsum[w] : 0;
    const uint32_t ex = pre + x - (h0 + h1);
    const uint32_t xcd = blockIdx.x % nxcd;
    if (c0 < nbins) {
        lstart[c0] = ex;
        if (h0) bases[c0] = atomicAdd(&bin_cur[c0 * nxcd + xcd], (unsigned long long)h0);
    }
    if (c0 + 1 < nbins) {
        lstart[c0 + 1] = ex + h0;
        if (h1) bases[c0 + 1] = atomicAdd(&bin_cur[(c0 + 1) * nxcd + xcd], (unsigned long long)h1);
    }
    __syncthreads();
    // the tile into LDS in bin order
#pragma unroll
    for (uint32_t it = 0; it < kScatterItems; it++) {
        const uint32_t e = it * kScatterBlock + tid;
        if (b[it] == ~0u) continue;
        const uint32_t slot = lstart[b[it] >> shift] + r[it];
        s_lo[slot] = lo[tile0 + e];
        s_bid[slot] = b[it];
    }
    __syncthreads();
    // out in bin order: consecutive lanes write consecutive positions of a run
    for (uint32_t e = tid; e < count; e += kScatterBlock) {
        const uint32_t bk = s_bid[e], c = bk >> shift;
        const uint64_t pos = bases[c] + (e - lstart[c]);
        bin_lo[pos] = s_lo[e];
        bin_bid[pos] = bk;
    }
}

// One workgroup per bin: bucket counts in LDS, their prefix sums (bstart of
// the bin's buckets), the largest bucket, and the keys in bucket order.  A bin
// of more than `piece` buckets is done `piece` buckets at a time (each
// piece reads the bin's keys again and keeps those of its buckets).
// piece = min(2^shift, kSortSpan, nbuckets); dynamic LDS: 2 * piece u32 (counts,
// then offsets).
__global__ __launch_bounds__(kSortBlock) void k_bucket_sort(const uint64_t* __restrict__ bin_start,
                                                           const uint64_t* __restrict__ bin_lo,
                                                           const uint32_t* __restrict__ bin_bid, uint32_t shift,
                                                           uint32_t piece, uint64_t nbuckets,
                                                           uint64_t* __restrict__ bstart, uint64_t* __restrict__ sorted,
                                                           uint32_t* __restrict__ maxm) {
    extern __shared__ uint32_t cnt[];
    __shared__ uint32_t wsum[kSortBlock / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t g0 = (uint64_t)blockIdx.x << shift;
    const uint32_t span = (uint32_t)min<uint64_t>(1ull << shift, nbuckets - g0);
    uint32_t* offs = cnt + piece;
    const uint64_t s = bin_start[blockIdx.x], e = bin_start[blockIdx.x + 1];
    uint64_t base = s;  // sorted position of the first key of the current piece
    for (uint32_t sub = 0; sub < span; sub += piece) {
        const uint32_t len = min(piece, span - sub);
        const uint32_t first = (uint32_t)(g0 + sub);  // global number of the piece's first bucket
        for (uint32_t j = tid; j < len; j += kSortBlock) cnt[j] = 0;
        __syncthreads();
        // keys are taken kSortItems per thread at a time, every load issued
        // before the first use (a loop of one key per step waits on each)
        for (uint64_t i0 = s + tid; i0 < e; i0 += (uint64_t)kSortItems * kSortBlock) {
            uint32_t b[kSortItems];
#pragma unroll
            for (uint32_t u = 0; u < kSortItems; u++) {
                const uint64_t i = i0 + (uint64_t)u * kSortBlock;
                b[u] = i < e ? bin_bid[i] - first : ~0u;  // wraps above len for buckets outside the piece
            }
#pragma unroll
            for (uint32_t u = 0; u < kSortItems; u++)
                if (b[u] < len) atomicAdd(&cnt[b[u]], 1u);
        }
        __syncthreads();
        // exclusive scan of cnt[0, len): each thread sums a chunk, the block scans the chunk sums
        const uint32_t chunk = (len + kSortBlock - 1) / kSortBlock;
        const uint32_t j0 = min(len, tid * chunk), j1 = min(len, j0 + chunk);
        uint32_t sum = 0, mx = 0;
        for (uint32_t j = j0; j < j1; j++) {
            sum += cnt[j];
            mx = max(mx, cnt[j]);
        }
        uint32_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= (uint32_t)o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if (lane == 0 && mx) atomicMax(maxm, mx);
        __syncthreads();
        uint32_t pre = 0, piece_total = 0;
        for (uint32_t w = 0; w < kSortBlock / 64; w++) {
            pre += w < wid ? wsum[w] : 0;
            piece_total += wsum[w];
        }
        uint32_t run = pre + x - sum;
        for (uint32_t j = j0; j < j1; j++) {
            offs[j] = run;
            bstart[first + j] = base + run;
            run += cnt[j];
        }
        __syncthreads();
        for (uint32_t j = tid; j < len; j += kSortBlock) cnt[j] = 0;
        __syncthreads();
        for (uint64_t i0 = s + tid; i0 < e; i0 += (uint64_t)kSortItems * kSortBlock) {
            uint32_t b[kSortItems];
            uint64_t lo[kSortItems];
#pragma unroll
            for (uint32_t u = 0; u < kSortItems; u++) {
                const uint64_t i = i0 + (uint64_t)u * kSortBlock;
                b[u] = i < e ? bin_bid[i] - first : ~0u;
                lo[u] = i < e ? bin_lo[i] : 0;
            }
#pragma unroll
            for (uint32_t u = 0; u < kSortItems; u++)
                if (b[u] < len) sorted[base + offs[b[u]] + atomicAdd(&cnt[b[u]], 1u)] = lo[u];
        }
        base += piece_total;
        __syncthreads();
    }
    if (blockIdx.x + 1 == gridDim.x && tid == 0) bstart[nbuckets] = e;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Exclusive scan (three passes: tile sums, scan of tile sums, tile scan).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_inclusive_sum(uint64_t x) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up(x, off, 64);
        if (lane >= (uint32_t)off) x += y;
    }
    return x;
}

// Exclusive block sum of v over kBlock threads; *total receives the block sum.
__device__ uint64_t block_exclusive_sum(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[kBlock / 64];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t x = wave_inclusive_sum(v);
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBlock / 64; w++) {
        uint64_t s = wsum[w];
        pre += w < wid ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const T* __restrict__ in, uint64_t n,
                                                      uint64_t* __restrict__ tile_sums, uint32_t* maxout) {
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    uint32_t mx = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
        if (i < n) {
            uint64_t v = (uint64_t)in[i];
            s += v;
            mx = max(mx, (uint32_t)min(v, (uint64_t)0xffffffffu));
        }
    }
    uint64_t tot;
    block_exclusive_sum(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
    if (maxout) {
        for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(maxout, mx);
    }
}

// Single block: exclusive scan of the tile sums in place.
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(uint64_t* sums, uint64_t ntiles) {
    __shared__ uint64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (uint64_t base = 0; base < ntiles; base += kBlock) {
        uint64_t i = base + threadIdx.x;
        uint64_t v = i < ntiles ? sums[i] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_sum(v, &tot);
        uint64_t carry = carry_s;
        if (i < ntiles) sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + tot;
        __syncthreads();
    }
}

// Single block: exclusive prefix sums of the (bin, XCD) counters in bin-major
// order.  bin_cur receives them (each XCD's part of each bin starts there) and
// bin_start[c] the start of bin c (nbins + 1 entries).
__global__ __launch_bounds__(kBlock) void k_bin_offsets(const unsigned long long* __restrict__ bin_cnt,
                                                       uint32_t nbins, uint32_t nxcd,
                                                       uint64_t* __restrict__ bin_start,
                                                       unsigned long long* __restrict__ bin_cur) {
    // each thread takes kBinItems consecutive counters per round: their loads
    // are independent (one memory round trip, not one per kBlock counters)
    constexpr uint32_t kBinItems = 16;
    __shared__ uint64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const uint32_t n = nbins * nxcd;
    for (uint32_t base = 0; base < n; base += kBlock * kBinItems) {
        const uint32_t i0 = base + threadIdx.x * kBinItems;
        uint64_t v[kBinItems], sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBinItems; k++) {
            v[k] = i0 + k < n ? bin_cnt[i0 + k] : 0;
            sum += v[k];
        }
        uint64_t tot;
        const uint64_t carry = carry_s;
        uint64_t run = carry + block_exclusive_sum(sum, &tot);
        uint32_t bin = i0 / nxcd, x = i0 % nxcd;
#pragma unroll
        for (uint32_t k = 0; k < kBinItems; k++) {
            if (i0 + k < n) {
                bin_cur[i0 + k] = run;
                if (x == 0) bin_start[bin] = run;
            }
            run += v[k];
            if (++x == nxcd) {
                x = 0;
                bin++;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) bin_start[nbins] = carry_s;
}

// out[i] = sum_{j<i} in[j] for i in [0, n]; each thread owns kScanItems
// consecutive items of the block's tile (tile_off = null: a single tile).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const T* __restrict__ in, uint64_t n,
                                                      const uint64_t* __restrict__ tile_off,
                                                      uint64_t* __restrict__ out) {
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t vals[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        uint64_t i = base + k;
        vals[k] = i < n ? (uint64_t)in[i] : 0;
        s += vals[k];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_sum(s, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += vals[k];
        if (i + 1 == n) out[n] = run;
    }
}


// ---------------------------------------------------------------------------
// Seed search (Sec. 4, 5): one 64-lane wavefront per bucket walks the bucket's
// splitting tree in preorder.  Every node's index is the FIRST index that
// works; lanes test candidates in increasing order and the lowest successful
// candidate of the first group that contains one is returned.
// ---------------------------------------------------------------------------
struct SearchArgs {
    const uint64_t* sorted;
    uint64_t* tmp;
    const uint64_t* bstart;
    uint64_t* seeds;
    uint32_t* msz;  // size of every coded node, at the same preorder position as its index
    uint64_t* blen;
    const BuildDesc* descs;
    BuildDesc* wdescs;
    const uint64_t* bucket_base;
    uint32_t count;
    uint64_t nbuckets;
    const uint32_t* tables;     // per table set: kTableCount arrays of `stride` words (r, F, N, G, P, Q, S, C)
    uint32_t stride;
    uint64_t seed_cap;
    uint32_t key_words;   // 64-bit words of dynamic LDS before the node slots (largest bucket)
    uint32_t wait_limit;  // sleeps a slot wait tolerates without any search progress in the bucket
    uint64_t bucket0;     // bucket of block 0 of this launch (the search is launched in chunks)
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// Returned by a search that stopped (seed cap, duplicate keys): the bucket is
// abandoned and the flag in DevStatus makes the build fail.
constexpr uint64_t kNoSeed = ~0ull;

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lane_value(uint64_t x, uint32_t lane) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Orders this wavefront's LDS accesses (the queues are private to one wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shared state of one bucket's workgroup (LDS).  Every wavefront that is
// searching adds to `beat` at regular intervals: a wavefront waiting for a
// slot gives up only when `beat` stops moving (no wavefront of the bucket is
// making progress, which the slot order rules out unless the tables and the
// strategy disagree), never because a search simply takes long.
struct QueueState {
    uint32_t head;   // next slot to claim
    uint32_t tail;   // next slot to fill
    uint32_t abort;  // set by a wavefront that abandons the bucket
    uint32_t beat;   // search progress counter
    unsigned long long bits;
};

// Default number of s_sleep(4) rounds (about 0.1-0.15 us each) a slot wait
// tolerates while `beat` does not move: several seconds, against search
// steps that bump it every few milliseconds at most.
constexpr uint32_t kDefaultWaitLimit = 1u << 25;

// Progress report of a searching wavefront, and whether the bucket was
// abandoned meanwhile (wave-uniform).
__device__ __forceinline__ bool search_poll(QueueState* qs) {
    if (lane_id() == 0) __hip_atomic_fetch_add(&qs->beat, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t ab = __hip_atomic_load(&qs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_amdgcn_readfirstlane(ab) != 0;
}

// ---- bijections --------------------------------------------------------------
// A trial fails at its first collision, so candidates are filtered in up to
// three stages: every new candidate is tried on the first C1 keys; survivors
// (about a third to a half) wait in an LDS queue in candidate order and are
// tried in groups of 64 on keys C1..C2-1; their survivors wait in a second
// queue and are finished on keys C2..M-1.  Queues are first-in first-out and
// candidates enter them in increasing order, so the first success found in the
// last stage is the first index that works.  Cut points minimise the expected
// VALU work (M^M/M! trials plus half the candidates needed to fill one group
// of the last stage) x sum_stages P(stage reached) * keys(stage), with P the
// collision-free probabilities prod (1 - i/M); 1 or 2 stages where filling the
// groups costs more than it saves.
constexpr int kQ = 128;  // ring capacity (at most 64 + 63 entries wait)
struct LeafQueues {
    uint64_t seed[2][kQ];
    uint32_t mask[2][kQ];
};
__device__ constexpr int kCut1[25] = {0, 1, 2, 3, 4, 5, 6, 3, 4, 4, 4, 4, 5, 5, 5, 5, 6, 6, 6, 6, 6, 7, 7, 7, 7};
__device__ constexpr int kCut2[25] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 5, 6, 6, 7, 8, 8, 8, 9, 10, 10, 10, 10, 11, 11, 12, 12};

template <int M, int LO, int HI>
__device__ __forceinline__ uint32_t leaf_bits(const uint64_t (&k)[M], uint64_t S, uint32_t mask) {
#pragma unroll
    for (int i = LO; i < HI; i++) mask |= 1u << __umulhi(mix64_hi32(k[i] + S), (uint32_t)M);
    return mask;
}

// Search steps (of 64 candidates) between two progress reports of a bijection search.
constexpr uint64_t kLeafPollMask = 64ull * 64 - 1;

template <int M>
__device__ __forceinline__ uint64_t leaf_search(const uint64_t* keys, uint32_t depth, uint64_t cap, uint32_t* flags,
                                                LeafQueues* q, bool staged, QueueState* qs) {
    constexpr int C1 = kCut1[M], C2 = kCut2[M];
    constexpr uint32_t full = (1u << M) - 1u;
    uint64_t k[M];
#pragma unroll
    for (int i = 0; i < M; i++) k[i] = uniform64(keys[i]);
    const uint32_t lane = lane_id();
    const uint64_t D = (uint64_t)depth << 56;
    const uint64_t step = 64ull * kGamma;
    uint64_t S = (D + lane) * kGamma;
    if (C1 == M || !staged) {
        // Key i of candidate base + lane is hashed at kl[i] + base * gamma: the
        // per-lane part is added once, the per-step part is a scalar register
        // pair (one vector add per evaluation and none per step; the empty asm
        // keeps the compiler from turning the sum back into one vector
        // induction variable per key).  Only the step that reaches the cap
        // checks lanes against it.
        uint64_t kl[M];
#pragma unroll
        for (int i = 0; i < M; i++) kl[i] = k[i] + S;
        const uint64_t last = cap ? (cap - 1) & ~63ull : 0;
        uint64_t O = 0;
        for (uint64_t base = 0; cap; base += 64, O += step) {
            uint64_t Os = O;
            asm volatile("" : "+s"(Os));
            uint32_t mask = leaf_bits<M, 0, M>(kl, Os, 0);
            bool ok = mask == full;
            const bool at_end = base == last;
            if (at_end) ok &= lane < (uint32_t)(cap - base);
            uint64_t bal = __ballot(ok);
            if (bal) return base + (uint64_t)__builtin_ctzll(bal);
            if (at_end) break;
            if ((base & kLeafPollMask) == kLeafPollMask - 63 && search_poll(qs)) return kNoSeed;
        }
    } else if constexpr (C1 < M) {
        uint32_t a_head = 0, a_tail = 0, b_head = 0, b_tail = 0;
        uint64_t found = kNoSeed;
        // Stage 3: finish queued candidates on keys [C2, M); full groups only,
        // unless flushing at the seed cap.
        auto drain_b = [&](bool flush) {
            while (b_tail - b_head >= 64 || (flush && b_tail != b_head)) {
                const uint32_t cb = min(64u, b_tail - b_head);
                const bool ab = lane < cb;
                const uint32_t pb = (b_head + lane) & (kQ - 1);
                uint64_t w = ab ? q->seed[1][pb] : 0;
                uint32_t m3 = ab ? q->mask[1][pb] : 0;
                b_head += cb;
                m3 = leaf_bits<M, C2, M>(k, (D + w) * kGamma, m3);
                uint64_t b3 = __ballot(ab && m3 == full);
                wave_lds_sync();
                if (b3) {
                    found = lane_value(w, (uint32_t)__builtin_ctzll(b3));
                    return;
                }
            }
        };
        for (uint64_t base = 0; base < cap; base += 64, S += step) {
            const bool last = base + 64 >= cap;
            // stage 1: 64 new candidates on keys [0, C1)
            uint32_t m1 = leaf_bits<M, 0, C1>(k, S, 0);
            bool s1 = __popc(m1) == C1 && base + lane < cap;
            uint64_t b1 = __ballot(s1);
            if (s1) {
                uint32_t p = (a_tail + lanes_below(b1)) & (kQ - 1);
                q->seed[0][p] = base + lane;
                q->mask[0][p] = m1;
            }
            a_tail += (uint32_t)__popcll(b1);
            wave_lds_sync();
            // stage 2: groups of (up to) 64 queued candidates on keys [C1, C2)
            while (a_tail - a_head >= 64 || (last && a_tail != a_head)) {
                const uint32_t cnt = min(64u, a_tail - a_head);
                const bool act = lane < cnt;
                const uint32_t pa = (a_head + lane) & (kQ - 1);
                uint64_t v = act ? q->seed[0][pa] : 0;
                uint32_t m2 = act ? q->mask[0][pa] : 0;
                a_head += cnt;
                m2 = leaf_bits<M, C1, C2>(k, (D + v) * kGamma, m2);
                if constexpr (C2 == M) {
                    uint64_t b2 = __ballot(act && m2 == full);
                    if (b2) return lane_value(v, (uint32_t)__builtin_ctzll(b2));
                } else {
                    bool s2 = act && __popc(m2) == C2;
                    uint64_t b2 = __ballot(s2);
                    wave_lds_sync();
                    if (s2) {
                        uint32_t p = (b_tail + lanes_below(b2)) & (kQ - 1);
                        q->seed[1][p] = v;
                        q->mask[1][p] = m2;
                    }
                    b_tail += (uint32_t)__popcll(b2);
                    wave_lds_sync();
                    drain_b(false);
                    if (found != kNoSeed) return found;
                }
                wave_lds_sync();
            }
            if constexpr (C2 != M) {
                if (last) {  // every older candidate has left stage 2: flush stage 3
                    drain_b(true);
                    if (found != kNoSeed) return found;
                }
            }
            if (last) break;
            if ((base & kLeafPollMask) == kLeafPollMask - 63 && search_poll(qs)) return kNoSeed;
        }
    }
    if (lane == 0) atomicOr(flags, kFlagSearch);
    return kNoSeed;
}

// Bijection search of the non-minimal variant: the first index whose hash
// sends the M keys to M distinct values out of `range` >= M (at most 32, so
// one 32-bit mask per candidate holds them).  Same candidate order and early
// exit as the plain loop of leaf_search.
template <int M>
__device__ __forceinline__ uint64_t leaf_search_wide(const uint64_t* keys, uint32_t depth, uint64_t cap,
                                                     uint32_t range, uint32_t* flags, QueueState* qs) {
    const uint32_t lane = lane_id();
    const uint64_t step = 64ull * kGamma;
    const uint64_t S = (((uint64_t)depth << 56) + lane) * kGamma;
    uint64_t kl[M];
#pragma unroll
    for (int i = 0; i < M; i++) kl[i] = uniform64(keys[i]) + S;
    const uint64_t last = cap ? (cap - 1) & ~63ull : 0;
    uint64_t O = 0;
    for (uint64_t base = 0; cap; base += 64, O += step) {
        uint64_t Os = O;
        asm volatile("" : "+s"(Os));
        uint32_t mask = 0;
#pragma unroll
        for (int i = 0; i < M; i++) mask |= 1u << __umulhi(mix64_hi32(kl[i] + Os), range);
        bool ok = __popc(mask) == M;
        const bool at_end = base == last;
        if (at_end) ok &= lane < (uint32_t)(cap - base);
        const uint64_t bal = __ballot(ok);
        if (bal) return base + (uint64_t)__builtin_ctzll(bal);
        if (at_end) break;
        if ((base & kLeafPollMask) == kLeafPollMask - 63 && search_poll(qs)) return kNoSeed;
    }
    if (lane == 0) atomicOr(flags, kFlagSearch);
    return kNoSeed;
}

// True if two of the m <= 64 keys are equal (wave-uniform result).
__device__ bool has_duplicate(const uint64_t* keys, uint32_t m) {
    uint32_t lane = lane_id();
    uint64_t mine = lane < m ? keys[lane] : 0;
    bool dup = false;
    for (uint32_t j = 0; j < m; j++) dup |= lane < m && lane > j && keys[j] == mine;
    return __ballot(dup) != 0;
}

// Inlined into each search kernel: as a call shared by the kernels it costs
// the calling convention's register saves and the uniformity of its arguments.
template <int MAXL, bool WIDE>
__device__ __forceinline__ uint64_t leaf_dispatch(const uint64_t* keys, uint32_t m, uint32_t depth, uint64_t cap,
                                                  uint32_t* flags, LeafQueues* q, uint32_t stage_from,
                                                  QueueState* qs, uint32_t range) {
    // Equal lower words never separate: copies that reach a leaf together are
    // caught here (more copies than any part of a split holds stop that split's
    // search instead, see split_search).
    if (has_duplicate(keys, m)) {
        if (lane_id() == 0) atomicOr(flags, kFlagDuplicate);
        return kNoSeed;
    }
    switch (m) {
#define RS_LEAF_CASE(M)                                                                    \
    case M:                                                                                \
        if constexpr (M <= MAXL && WIDE) return leaf_search_wide<M>(keys, depth, cap, range, flags, qs); \
        if constexpr (M <= MAXL && !WIDE)                                                  \
            return leaf_search<M>(keys, depth, cap, flags, q, M > 16 || M >= stage_from, qs); \
        return kNoSeed;
        RS_LEAF_CASE(2) RS_LEAF_CASE(3) RS_LEAF_CASE(4) RS_LEAF_CASE(5) RS_LEAF_CASE(6) RS_LEAF_CASE(7)
        RS_LEAF_CASE(8) RS_LEAF_CASE(9) RS_LEAF_CASE(10) RS_LEAF_CASE(11) RS_LEAF_CASE(12) RS_LEAF_CASE(13)
        RS_LEAF_CASE(14) RS_LEAF_CASE(15) RS_LEAF_CASE(16) RS_LEAF_CASE(17) RS_LEAF_CASE(18) RS_LEAF_CASE(19)
        RS_LEAF_CASE(20) RS_LEAF_CASE(21) RS_LEAF_CASE(22) RS_LEAF_CASE(23) RS_LEAF_CASE(24)
#undef RS_LEAF_CASE
        default:
            return kNoSeed;
    }
}

// ---- splits -----------------------------------------------------------------
// The first v such that the parts receive exactly (u, ..., u, last) keys.
// 2^g lanes share one candidate (each takes every 2^g-th key) and reduce their
// counts with cross-lane shuffles, so 64 >> g candidates are tried per step:
// few lanes per candidate for nodes that need many trials, many for nodes that
// need few (less overshoot past the first success).  Counting:
//   thresholds: phi >= t*u exactly when the upper hash word is >= T_t =
//               ceil(t*u*2^32/m); one counter per boundary (fanout <= 4).
//   packed:     j = floor(phi/u) by a reciprocal multiply, and 1 << (j*w) is
//               added to one 64-bit word of w-bit fields (fanout >= 5 when
//               fanout * w <= 64).
//   one-hot:    fanout 4 and m < 256: as packed, with four 8-bit fields in one
//               32-bit word (4 vector instructions per key after the hash
//               against 6 for three thresholds).
constexpr uint32_t kMaxThresholds = 8;  // fanout <= max(s, t) = 9 for l <= 24
enum CountMode { kCountThresholds = 0, kCountPacked = 1, kCountOneHot = 2 };

__device__ __forceinline__ uint32_t split_count_mode(uint32_t m, uint32_t fanout) {
    if (fanout == 4 && m < 256) return kCountOneHot;
    const uint32_t w = 32 - __clz(m);
    return fanout >= 5 && fanout * w <= 64 ? kCountPacked : kCountThresholds;
}

struct SplitCtl {
    uint32_t m, unit, fanout, last;
    uint32_t g;      // log2 lanes per candidate
    uint32_t w;      // packed field width (bits)
    uint32_t recip;  // ceil(2^32 / unit)
    uint64_t want;   // packed target
};

// True if two of the m keys are equal (any m; wave-uniform result).  Lane i
// holds key c0 + i and compares it with every later key (same LDS address for
// all lanes: one broadcast read per comparison).  m^2/128 comparisons.
__device__ bool node_has_duplicate(const uint64_t* keys, uint32_t m) {
    const uint32_t lane = lane_id();
    bool dup = false;
    for (uint32_t c0 = 0; c0 < m; c0 += 64) {
        const uint32_t i = c0 + lane;
        const uint64_t mine = i < m ? keys[i] : 0;
        for (uint32_t j = c0 + 1; j < m; j++) dup |= j > i && i < m && keys[j] == mine;
    }
    return __ballot(dup) != 0;
}

// Split search steps between two progress reports.
constexpr uint32_t kSplitPollSteps = 16;

// Equal keys always land in the same part.  A group of equal keys larger than
// every part can therefore never be split, and the search would not end; a
// group that fits travels on and is caught by the leaf that receives it.  So
// once a split search has tried 64 m candidates (the expected number of
// trials of every node the strategy makes is far below that for small nodes,
// and the check then costs well under 1% of the work already spent), and
// again each time that count doubles, the node's keys are compared pairwise,
// and equal keys end the search with the duplicate flag.  The check changes
// no result: without duplicates the search simply goes on.
//
// The search covers candidates [lo, min(hi, cap)) (lo a multiple of the
// candidates per step) and returns the first that works there.  With best
// null it is the node's whole search (lo = 0, hi = cap): duplicates are
// checked as above and reaching the cap raises the search flag.  Otherwise
// it is one chunk of a search shared by several wavefronts: it stops early
// once *best (the smallest success any of them found) is at or below the
// candidates still to try, and the owner of the node handles duplicates and
// the cap.
//
// EXACT: every part has u keys (m = f u).  Then the part of a key,
// floor(floor(h m / 2^32) / u), equals floor(h f / 2^32) (nested floors of
// an integer division), one multiply instead of two: h >> 30 for the
// one-hot mode's fanout of 4.
template <int NT, int MODE, bool EXACT>
__device__ __forceinline__ uint64_t split_search(const uint64_t* keys, uint32_t depth, const SplitCtl& c, const uint32_t* T,
                                 uint64_t lo, uint64_t hi, uint64_t cap, const unsigned long long* best,
                                 uint32_t* flags, QueueState* qs) {
    constexpr int NA = NT > 0 ? NT : 1;  // NT = 0 in the packed modes
    uint32_t thr[NA];
#pragma unroll
    for (int t = 0; t < NT; t++) thr[t] = T[t];
    const uint32_t lane = lane_id();
    const uint32_t g = __builtin_amdgcn_readfirstlane(c.g);
    const uint32_t G = 1u << g, gl = lane & (G - 1), gi = lane >> g, per_step = 64u >> g;
    const uint32_t m = __builtin_amdgcn_readfirstlane(c.m);
    const uint64_t step = (uint64_t)per_step * kGamma;
    // Keys are dealt to the G lanes of a candidate in blocks of 4 consecutive
    // keys (lane gl takes keys 4 gl .. 4 gl + 3 of every block of 4 G, so one
    // address serves all four loads); every lane runs the same number of
    // blocks, and the last m mod 4 G keys are dealt one at a time.
    const uint32_t quads = m / (4 * G);
    const uint32_t tail = quads * 4 * G;
    uint64_t S = (((uint64_t)depth << 56) + lo + gi) * kGamma;
    uint64_t next_check = 64ull * m;
    uint32_t steps = 0;
    const uint64_t end = min(hi, cap);
    for (uint64_t base = lo; base < end; base += per_step, S += step) {
        // a success at or below `base` elsewhere makes the rest of the chunk useless
        if (best && uniform64(__hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) <= base)
            return kNoSeed;
        uint32_t cnt[NA];
        uint64_t packed = 0;
        uint32_t onehot = 0;
#pragma unroll
        for (int t = 0; t < NT; t++) cnt[t] = 0;
        const uint64_t* kp = keys + 4 * gl;
        for (uint32_t q4 = 0; q4 < quads; q4++, kp += 4 * G) {
            uint32_t h[4];
#pragma unroll
            for (int u = 0; u < 4; u++) h[u] = mix64_hi32(kp[u] + S);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if constexpr (MODE == kCountPacked) {
                    uint32_t j = EXACT ? __umulhi(h[u], c.fanout) : __umulhi(__umulhi(h[u], m), c.recip);
                    packed += 1ull << (j * c.w);
                } else if constexpr (MODE == kCountOneHot) {
                    uint32_t j = EXACT ? h[u] >> 30 : __umulhi(__umulhi(h[u], m), c.recip);
                    onehot += 1u << (j * c.w);
                } else {
#pragma unroll
                    for (int t = 0; t < NT; t++) cnt[t] += (uint32_t)(h[u] < thr[t]);
                }
            }
        }
        for (uint32_t i = tail + gl; i < m; i += G) {
            uint32_t h = mix64_hi32(keys[i] + S);
            if constexpr (MODE == kCountPacked) {
                uint32_t j = EXACT ? __umulhi(h, c.fanout) : __umulhi(__umulhi(h, m), c.recip);
                packed += 1ull << (j * c.w);
            } else if constexpr (MODE == kCountOneHot) {
                uint32_t j = EXACT ? h >> 30 : __umulhi(__umulhi(h, m), c.recip);
                onehot += 1u << (j * c.w);
            } else {
#pragma unroll
                for (int t = 0; t < NT; t++) cnt[t] += (uint32_t)(h < thr[t]);
            }
        }
        for (uint32_t o = 1; o < G; o <<= 1) {
            if constexpr (MODE == kCountPacked) {
                packed += (uint64_t)__shfl_xor((unsigned long long)packed, (int)o, 64);
            } else if constexpr (MODE == kCountOneHot) {
                onehot += (uint32_t)__shfl_xor((int)onehot, (int)o, 64);
            } else {
#pragma unroll
                for (int t = 0; t < NT; t++) cnt[t] += (uint32_t)__shfl_xor((int)cnt[t], (int)o, 64);
            }
        }
        bool ok = gl == 0 && base + gi < cap;
        if constexpr (MODE == kCountPacked) {
            ok &= packed == c.want;
        } else if constexpr (MODE == kCountOneHot) {
            ok &= onehot == (uint32_t)c.want;
        } else {
#pragma unroll
            for (int t = 0; t < NT; t++) ok &= cnt[t] == (uint32_t)(t + 1) * c.unit;
        }
        uint64_t bal = __ballot(ok);
        if (bal) return base + (uint64_t)(__builtin_ctzll(bal) >> c.g);
        if (++steps == kSplitPollSteps) {
            steps = 0;
            if (search_poll(qs)) return kNoSeed;
        }
        if (!best && base + per_step >= next_check) {
            if (node_has_duplicate(keys, m)) {
                if (lane == 0) atomicOr(flags, kFlagDuplicate);
                return kNoSeed;
            }
            next_check *= 2;
        }
    }
    if (!best && lane == 0) atomicOr(flags, kFlagSearch);
    return kNoSeed;
}

template <int MAXNT>
__device__ __forceinline__ uint64_t split_dispatch(const uint64_t* keys, uint32_t depth, const SplitCtl& c, const uint32_t* T,
                                   uint32_t mode, uint64_t lo, uint64_t hi, uint64_t cap,
                                   const unsigned long long* best, uint32_t* flags, QueueState* qs) {
    const bool exact = c.last == c.unit;
    if (mode == kCountPacked)
        return exact ? split_search<0, kCountPacked, true>(keys, depth, c, T, lo, hi, cap, best, flags, qs)
                     : split_search<0, kCountPacked, false>(keys, depth, c, T, lo, hi, cap, best, flags, qs);
    if (mode == kCountOneHot)
        return exact ? split_search<0, kCountOneHot, true>(keys, depth, c, T, lo, hi, cap, best, flags, qs)
                     : split_search<0, kCountOneHot, false>(keys, depth, c, T, lo, hi, cap, best, flags, qs);
    switch (c.fanout - 1) {
#define RS_SPLIT_CASE(NT)                                                                                       \
    case NT:                                                                                                    \
        if constexpr (NT <= MAXNT)                                                                              \
            return split_search<NT, kCountThresholds, false>(keys, depth, c, T, lo, hi, cap, best, flags, qs);  \
        return kNoSeed;
        RS_SPLIT_CASE(1) RS_SPLIT_CASE(2) RS_SPLIT_CASE(3) RS_SPLIT_CASE(4) RS_SPLIT_CASE(5) RS_SPLIT_CASE(6)
        RS_SPLIT_CASE(7) RS_SPLIT_CASE(8)
#undef RS_SPLIT_CASE
        default:
            return kNoSeed;
    }
}

// Largest fanout - 1 of any node for leaf sizes up to MAXL (max(s, t) - 1).
__host__ __device__ constexpr int max_thresholds(int maxl) {
    int sv = (35 * maxl + 149) / 100;
    sv = sv < 2 ? 2 : sv;
    int tv = maxl < 7 ? 2 : (21 * maxl + 189) / 100;
    return (sv > tv ? sv : tv) - 1;
}

// Workgroup-scope ordering of one wavefront's global and LDS accesses (used
// where a wave hands data to its own lanes through memory).
__device__ __forceinline__ void wave_mem_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Reorder the node's keys so that child j occupies [j*unit, ...) (one
// wavefront): every key goes to its final place in a scratch array and the
// keys are copied back.  The scratch is the wavefront's LDS area of the
// bijection queues (free while it works on a split) when the node fits there,
// else global memory.  The LDS scratch is addressed through an LDS-qualified
// pointer, so that its stores are LDS stores and not generic ones.
typedef __attribute__((address_space(3))) uint64_t lds_u64;

__device__ __forceinline__ void partition(uint64_t* keys, uint32_t m, uint32_t depth, uint64_t v, const uint32_t* T,
                                          uint32_t nt, uint32_t unit, uint64_t* lds_tmp, uint32_t lds_cap,
                                          uint64_t* gtmp) {
    const uint32_t lane = lane_id();
    const uint64_t S = stream_offset(depth, v);
    auto scatter = [&](auto* dst) {
        uint32_t cursor[kMaxThresholds + 1];
#pragma unroll
        for (uint32_t q = 0; q <= kMaxThresholds; q++) cursor[q] = q * unit;
        for (uint32_t c0 = 0; c0 < m; c0 += 64) {
            uint32_t i = c0 + lane;
            bool act = i < m;
            uint64_t x = act ? keys[i] : 0;
            uint32_t h = mix64_hi32(x + S);
            uint32_t j = 0;
            for (uint32_t t = 0; t < nt; t++) j += (uint32_t)(h >= T[t]);
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t q = 0; q <= kMaxThresholds; q++) {
                if (q <= nt) {
                    uint64_t bal = __ballot(act && j == q);
                    if (act && j == q) pos = cursor[q] + lanes_below(bal);
                    cursor[q] += (uint32_t)__popcll(bal);
                }
            }
            if (act) dst[pos] = x;
        }
    };
    if (m <= lds_cap) {
        lds_u64* tmp = (lds_u64*)lds_tmp;
        scatter(tmp);
        wave_lds_sync();
        for (uint32_t i = lane; i < m; i += 64) keys[i] = tmp[i];
        wave_lds_sync();
    } else {
        scatter(gtmp);
        wave_mem_sync();
        for (uint32_t i = lane; i < m; i += 64) keys[i] = gtmp[i];
        wave_mem_sync();
    }
}

// One workgroup of WAVES wavefronts per bucket of every build of the call (the
// hardware hands workgroups to compute units as they free up, so uneven
// buckets balance dynamically).  The bucket's keys sit in LDS.
// Every coded node of the bucket's tree gets one slot of an LDS queue (the
// number of coded nodes, N(m), is known from the strategy): wavefronts claim
// slots in order with an atomic counter, wait until the slot has been
// published, search the node's index, partition its keys if it is a split and
// publish its children in later slots.  A parent's slot always precedes its
// children's, so a claimed slot is always filled by a wavefront that is not
// waiting, and the bucket is done when every slot has been claimed.  A node's
// preorder position (where its index is stored) is its parent's position + 1
// + the coded nodes of its earlier siblings, j * N(u).  Waits end early if
// another wavefront abandons the bucket.  A wait never times out while some
// wavefront of the bucket reports search progress (the chain of waits always
// ends at a searching wavefront, so a long search only means a long wait);
// if no progress is reported for wait_limit sleeps, which the slot order rules
// out, the bucket fails with the scheduling flag instead of hanging.
struct NodeSlot {
    uint32_t off, d, idx;
    uint32_t m;  // published last (release); 0 = not yet filled
};

// A split search shared by the wavefronts of a bucket.  The owner of a heavy
// split node (the tables flag sizes whose expected trials x keys exceed
// kCoopEvals) publishes it on its board entry; wavefronts that wait for a
// slot meanwhile help.  Candidates are cut into chunks of kCoopSteps search
// steps, claimed in increasing order from `next`; each chunk is searched from
// its start, and `best` keeps the smallest success found.  Once a success is
// known no chunk above it is started, and chunks above it that are running
// stop at their next step, so when every claimed chunk has ended (the owner
// stops claiming and waits for `outstanding` to return to zero) `best` is the
// first index that works: the result of the plain search.
constexpr uint32_t kCoopSteps = 32;
struct CoopNode {
    uint32_t active;       // chunks may be claimed (release / acquire)
    uint32_t outstanding;  // helpers inside the node (never reset: returns to 0)
    uint32_t failed;       // the owner stopped the search (duplicate keys)
    uint32_t pad0;
    unsigned long long next;  // next chunk
    unsigned long long best;  // smallest success found (kNoSeed: none)
    uint32_t off, depth, mode, pad;
    SplitCtl c;
};

// Claim chunks of the shared search `cn` and search them until none below the
// best success (or the cap) is left; returns the success this wavefront
// found, if any.  The owner also compares the node's keys pairwise once its
// chunks pass 64 m candidates and at each doubling (duplicate keys: the
// search is stopped for every wavefront and the duplicate flag raised).
template <int MAXNT>
__device__ __forceinline__ uint64_t coop_search(CoopNode& cn, const uint64_t* keys, const uint32_t* T, uint64_t cap,
                                uint32_t* flags, QueueState* qs, bool owner) {
    const uint32_t lane = lane_id();
    // the node's parameters, wave-uniform (scalar registers)
    SplitCtl c;
    c.m = __builtin_amdgcn_readfirstlane(cn.c.m);
    c.unit = __builtin_amdgcn_readfirstlane(cn.c.unit);
    c.fanout = __builtin_amdgcn_readfirstlane(cn.c.fanout);
    c.last = __builtin_amdgcn_readfirstlane(cn.c.last);
    c.g = __builtin_amdgcn_readfirstlane(cn.c.g);
    c.w = __builtin_amdgcn_readfirstlane(cn.c.w);
    c.recip = __builtin_amdgcn_readfirstlane(cn.c.recip);
    c.want = uniform64(cn.c.want);
    const uint32_t depth = __builtin_amdgcn_readfirstlane(cn.depth);
    const uint32_t mode = __builtin_amdgcn_readfirstlane(cn.mode);
    const uint64_t K = (uint64_t)(64u >> c.g) * kCoopSteps;
    uint64_t next_check = 64ull * c.m;
    for (;;) {
        unsigned long long ci = 0;
        if (lane == 0) ci = __hip_atomic_fetch_add(&cn.next, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint64_t c64 = uniform64(ci);
        const uint64_t lo = c64 < cap / K + 1 ? c64 * K : cap;  // (no product overflow)
        const uint64_t bst = uniform64(__hip_atomic_load(&cn.best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        const uint32_t stop = __hip_atomic_load(&cn.failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) |
                              __hip_atomic_load(&qs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (lo >= min(bst, cap) || __builtin_amdgcn_readfirstlane(stop)) return kNoSeed;
        if (owner && lo >= next_check) {
            while (next_check <= lo) next_check *= 2;
            if (node_has_duplicate(keys, c.m)) {
                if (lane == 0) {
                    atomicOr(flags, kFlagDuplicate);
                    __hip_atomic_store(&cn.failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_store(&cn.best, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                return kNoSeed;
            }
        }
        const uint64_t v = split_dispatch<MAXNT>(keys, depth, c, T, mode, lo, lo + K, cap, &cn.best, flags, qs);
        if (v != kNoSeed) {
            if (lane == 0)
                __hip_atomic_fetch_min(&cn.best, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return v;  // every later chunk lies above this success
        }
    }
}

// A waiting wavefront's help with the shared search `cn` of another.  The
// helper counts itself in before it looks at `active`, and the owner closes
// the node before it reads the count (both sequentially consistent): a helper
// that the owner did not see finds the node closed, and the owner waits for
// every helper it saw.
template <int MAXNT>
__device__ __forceinline__ void coop_help(CoopNode& cn, const uint64_t* lds_keys, const uint32_t* T, uint64_t cap, uint32_t* flags,
                          QueueState* qs) {
    if (lane_id() == 0) __hip_atomic_fetch_add(&cn.outstanding, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t open = __hip_atomic_load(&cn.active, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (__builtin_amdgcn_readfirstlane(open)) {
        const uint32_t off = __builtin_amdgcn_readfirstlane(cn.off);
        (void)coop_search<MAXNT>(cn, lds_keys + off, T, cap, flags, qs, false);
    }
    wave_lds_sync();
    if (lane_id() == 0) __hip_atomic_fetch_sub(&cn.outstanding, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP);
}


// WIDE: the call holds a build of the non-minimal variant; leaves search
// injections into their build's leaf_range (equal to m for slack 0).
template <int MAXL, int WAVES, bool WIDE>
__global__ __launch_bounds__(64 * WAVES) void k_search(SearchArgs a) {
    extern __shared__ uint64_t lds_dyn[];
    __shared__ QueueState qs;
    __shared__ uint32_t thr_s[WAVES][kMaxThresholds];
    __shared__ LeafQueues queues[WAVES];
    __shared__ CoopNode board[WAVES];
    const uint32_t lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t* lds_keys = lds_dyn;
    NodeSlot* slots = reinterpret_cast<NodeSlot*>(lds_dyn + a.key_words);
    uint32_t* thr = thr_s[wave];
    {
        const uint64_t b = a.bucket0 + blockIdx.x;
        const uint32_t j = find_build(a.bucket_base, a.count, b);
        const BuildDesc& B = a.descs[j];
        // the descriptor is also written by this kernel (flags), so its fields are
        // loaded per lane: make the build's parameters wave-uniform explicitly
        const uint32_t leaf = __builtin_amdgcn_readfirstlane(B.leaf);
        const uint32_t lower = __builtin_amdgcn_readfirstlane(B.lower);
        const uint32_t upper = __builtin_amdgcn_readfirstlane(B.upper);
        const uint32_t stage_from = __builtin_amdgcn_readfirstlane(B.stage_from);
        const uint32_t group_cap = __builtin_amdgcn_readfirstlane(B.group_cap);
        const uint32_t slack = WIDE ? __builtin_amdgcn_readfirstlane(B.slack) : 0;
        // waves beyond the build's count only join the barriers
        const uint32_t active = __builtin_amdgcn_readfirstlane(min(B.waves, (uint32_t)WAVES));
        const uint32_t* R = a.tables + (size_t)__builtin_amdgcn_readfirstlane(B.tab) * kTableCount * a.stride;
        const uint32_t* Nt = R + 2 * a.stride;
        const uint32_t* Gt = R + 3 * a.stride;
        uint32_t* bflags = &a.wdescs[j].flags;
        const uint64_t start = a.bstart[b];
        const uint32_t m0 = (uint32_t)(a.bstart[b + 1] - start);
        if (m0 > a.key_words) {  // larger than the LDS this launch was sized for (a reused plan)
            if (threadIdx.x == 0) {
                atomicOr(bflags, kFlagTooBig);
                a.blen[b] = 0;
            }
            return;
        }
        const uint32_t total = Nt[m0];
        for (uint32_t i = threadIdx.x; i < m0; i += 64 * WAVES) lds_keys[i] = a.sorted[start + i];
        for (uint32_t i = threadIdx.x; i < total; i += 64 * WAVES) slots[i].m = 0;
        __syncthreads();
        if (threadIdx.x < WAVES) {
            board[threadIdx.x].active = 0;
            board[threadIdx.x].outstanding = 0;
        }
        if (threadIdx.x == 0) {
            qs.head = 0;
            qs.tail = total ? 1 : 0;
            qs.abort = 0;
            qs.beat = 0;
            qs.bits = 0;
            if (total) {
                slots[0].off = 0;
                slots[0].d = 0;
                slots[0].idx = 0;
                slots[0].m = m0;
            }
        }
        __syncthreads();
        unsigned long long bits = 0;
        for (; wave < active;) {
            uint32_t h = 0;
            if (lane == 0) h = __hip_atomic_fetch_add(&qs.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            h = __builtin_amdgcn_readfirstlane(h);
            if (h >= total) break;
            // wait for the slot while some wavefront of the bucket makes progress,
            // and help the shared split searches of other wavefronts meanwhile
            uint32_t m = 0, stop = 0, idle = 0;
            uint32_t seen = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(&qs.beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            for (;;) {
                m = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&slots[h].m, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
                if (m) break;
                if (__builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(&qs.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))) {
                    stop = 1;
                    break;
                }
                if constexpr (WAVES > 1) {
                    uint32_t e = WAVES;
                    for (uint32_t w2 = 0; w2 < WAVES; w2++)
                        if (e == WAVES &&
                            __hip_atomic_load(&board[w2].active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                            e = w2;
                    e = __builtin_amdgcn_readfirstlane(e);
                    if (e < WAVES) {
                        coop_help<max_thresholds(MAXL)>(board[e], lds_keys, thr_s[e], a.seed_cap, bflags, &qs);
                        idle = 0;
                        __builtin_amdgcn_s_sleep(1);  // (a node whose chunks are all taken is retried)
                        continue;
                    }
                }
                const uint32_t now = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&qs.beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                if (now != seen) {
                    seen = now;
                    idle = 0;
                } else if (++idle >= a.wait_limit) {
                    if (lane == 0) {
                        atomicOr(bflags, kFlagStack);
                        __hip_atomic_store(&qs.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            if (stop) break;
            const uint32_t off = __builtin_amdgcn_readfirstlane(slots[h].off);
            const uint32_t d = __builtin_amdgcn_readfirstlane(slots[h].d);
            const uint32_t idx = __builtin_amdgcn_readfirstlane(slots[h].idx);
            wave_mem_sync();
            uint64_t v;
            bool fail;
            SplitShape sh{};
            if (m <= leaf) {
                v = leaf_dispatch<MAXL, WIDE>(lds_keys + off, m, d, a.seed_cap, bflags, &queues[wave], stage_from,
                                              &qs, leaf_range(m, slack));
                fail = v == kNoSeed;
            } else {
                sh = split_shape(m, leaf, lower, upper);
                if (sh.unit == 1 && has_duplicate(lds_keys + off, m)) {  // l = 1: parts of one key each
                    if (lane == 0) atomicOr(bflags, kFlagDuplicate);
                    v = kNoSeed;
                    fail = true;
                } else {
                    const uint32_t nt = sh.fanout - 1;
                    if (lane < nt) thr[lane] = (uint32_t)((((uint64_t)(lane + 1) * sh.unit << 32) + m - 1) / m);
                    wave_lds_sync();
                    SplitCtl c;
                    c.m = m;
                    c.unit = sh.unit;
                    c.fanout = sh.fanout;
                    c.last = sh.last;
                    const uint32_t gw = Gt[m];
                    c.g = __builtin_amdgcn_readfirstlane(min(gw & kGroupMask, group_cap));
                    const uint32_t mode = split_count_mode(m, sh.fanout);
                    c.w = mode == kCountOneHot ? 8 : 32 - __clz(m);
                    c.recip = mode != kCountThresholds ? (uint32_t)(((1ull << 32) + sh.unit - 1) / sh.unit) : 0;
                    c.want = 0;
                    if (mode != kCountThresholds)
                        for (uint32_t q = 0; q < sh.fanout; q++)
                            c.want += (uint64_t)(q + 1 == sh.fanout ? sh.last : sh.unit) << (q * c.w);
                    if (WAVES > 1 && active > 1 && (gw & kCoopFlag)) {
                        // a heavy node: searched in chunks with the help of waiting wavefronts
                        CoopNode& cn = board[wave];
                        if (lane == 0) {
                            cn.c = c;
                            cn.off = off;
                            cn.depth = d;
                            cn.mode = mode;
                            cn.next = 0;
                            cn.failed = 0;
                            cn.best = kNoSeed;
                            __hip_atomic_store(&cn.active, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        wave_lds_sync();
                        (void)coop_search<max_thresholds(MAXL)>(cn, lds_keys + off, thr, a.seed_cap, bflags, &qs,
                                                                true);
                        if (lane == 0)
                            __hip_atomic_store(&cn.active, 0u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP);
                        // every helper the node had ends its chunk (each stops at the next
                        // step once the best success lies below it)
                        uint32_t wait_idle = 0, wseen = 0;
                        while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(
                            &cn.outstanding, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WORKGROUP))) {
                            const uint32_t now = __builtin_amdgcn_readfirstlane(
                                __hip_atomic_load(&qs.beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                            if (now != wseen) {
                                wseen = now;
                                wait_idle = 0;
                            } else if (++wait_idle >= a.wait_limit) {
                                if (lane == 0) {
                                    atomicOr(bflags, kFlagStack);
                                    __hip_atomic_store(&qs.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                }
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        const uint32_t failed = __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&cn.failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) |
                            __hip_atomic_load(&qs.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                        v = failed ? kNoSeed
                                   : uniform64(__hip_atomic_load(&cn.best, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP));
                        if (!failed && v == kNoSeed && lane == 0) atomicOr(bflags, kFlagSearch);  // the cap
                    } else {
                        v = split_dispatch<max_thresholds(MAXL)>(lds_keys + off, d, c, thr, mode, 0, a.seed_cap,
                                                                 a.seed_cap, nullptr, bflags, &qs);
                    }
                    fail = v == kNoSeed;  // counts do not match the parts: no partition
                    if (!fail)
                        partition(lds_keys + off, m, d, v, thr, nt, sh.unit, reinterpret_cast<uint64_t*>(&queues[wave]),
                                  (uint32_t)(sizeof(LeafQueues) / sizeof(uint64_t)), a.tmp + start + off);
                }
            }
            if (fail) {
                if (lane == 0) __hip_atomic_store(&qs.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                break;
            }
            if (lane == 0) {
                a.seeds[start + idx] = v;
                a.msz[start + idx] = m;
            }
            const uint32_t r = R[m];
            bits += r + (v >> r) + 1;
            if (m > leaf && lane == 0) {
                for (uint32_t q = 0; q < sh.fanout; q++) {
                    const uint32_t cm = q + 1 == sh.fanout ? sh.last : sh.unit;
                    if (cm < 2) continue;
                    const uint32_t t =
                        __hip_atomic_fetch_add(&qs.tail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (t >= total) {  // more children than coded nodes: tables and strategy disagree
                        atomicOr(bflags, kFlagStack);
                        __hip_atomic_store(&qs.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        break;
                    }
                    slots[t].off = off + q * sh.unit;
                    slots[t].d = d + 1;
                    slots[t].idx = idx + 1 + q * Nt[sh.unit];
                    __hip_atomic_store(&slots[t].m, cm, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        if (lane == 0) atomicAdd(&qs.bits, bits);
        __syncthreads();
        if (threadIdx.x == 0) a.blen[b] = qs.bits;
    }
}

// ---------------------------------------------------------------------------
// Elias-Fano of s_i and z_i = o_i - floor(beta s_i / 2^16) (Sec. 6.3, 7.4),
// per build: minimum gaps, largest bucket and total tree bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t z_of(uint64_t o, uint64_t s, uint64_t beta) {
    return (int64_t)o - (int64_t)((beta * s) >> 16);
}

struct GapArgs {
    const uint64_t* bstart;  // global prefix sums of bucket sizes (nbuckets + 1)
    const uint64_t* qstart;  // global prefix sums of bucket output ranges (bstart for minimal builds)
    const uint64_t* ostart;  // global prefix sums of bucket bit lengths (nbuckets + 1)
    const BuildDesc* descs;
    BuildDesc* wdescs;
    const uint64_t* bucket_base;
    uint32_t count;
    uint64_t nbuckets;
};

// Gap, size and bit-length statistics of one bucket g (0 <= g < nbuckets).
struct GapStat {
    unsigned long long gs;
    long long gz;
    uint32_t mx;
};

__device__ __forceinline__ GapStat gap_of(const GapArgs& a, uint32_t j, uint64_t g) {
    const BuildDesc& B = a.descs[j];
    const uint64_t bb = B.bucket_base, s0 = a.qstart[bb], o0 = a.ostart[bb];
    const uint64_t bits = a.ostart[bb + B.nb] - o0;
    const uint64_t range = a.qstart[bb + B.nb] - s0;
    const uint64_t beta = (bits << 16) / range;
    const uint64_t s_i = a.qstart[g] - s0, s_i1 = a.qstart[g + 1] - s0;
    GapStat r;
    r.gs = s_i1 - s_i;
    r.gz = z_of(a.ostart[g + 1] - o0, s_i1, beta) - z_of(a.ostart[g] - o0, s_i, beta);
    r.mx = (uint32_t)(a.bstart[g + 1] - a.bstart[g]);
    if (g == bb) {
        a.wdescs[j].total_bits = bits;
        a.wdescs[j].range_total = range;
    }
    return r;
}

constexpr uint32_t kGapItems = 8;  // buckets per thread
constexpr uint32_t kGapTile = kBlock * kGapItems;

// Minimum gaps of both Elias-Fano sequences, largest bucket and total tree
// bits of every build.  A block whose buckets all belong to one build reduces
// in LDS and updates the build with one atomic per statistic (many buckets
// per build would otherwise all update the same three words).
__global__ __launch_bounds__(kBlock) void k_ef_gaps(GapArgs a) {
    __shared__ unsigned long long r_gs[kBlock / 64];
    __shared__ long long r_gz[kBlock / 64];
    __shared__ uint32_t r_mx[kBlock / 64];
    const uint64_t tile = (uint64_t)blockIdx.x * kGapTile;
    const uint64_t last = min(a.nbuckets, tile + kGapTile) - 1;
    const uint32_t j0 = __builtin_amdgcn_readfirstlane(find_build(a.bucket_base, a.count, tile));
    const uint32_t j1 = __builtin_amdgcn_readfirstlane(find_build(a.bucket_base, a.count, last));
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (j0 == j1) {
        unsigned long long gs = ~0ull;
        long long gz = 0x7fffffffffffffffll;
        uint32_t mx = 0;
        for (uint32_t k = 0; k < kGapItems; k++) {
            const uint64_t g = tile + (uint64_t)k * kBlock + threadIdx.x;
            if (g < a.nbuckets) {
                const GapStat r = gap_of(a, j0, g);
                gs = min(gs, r.gs);
                gz = min(gz, r.gz);
                mx = max(mx, r.mx);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            gs = min(gs, (unsigned long long)__shfl_xor(gs, off, 64));
            gz = min(gz, (long long)__shfl_xor(gz, off, 64));
            mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
        }
        if (lane == 0) {
            r_gs[wid] = gs;
            r_gz[wid] = gz;
            r_mx[wid] = mx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (uint32_t w = 1; w < kBlock / 64; w++) {
                gs = min(gs, r_gs[w]);
                gz = min(gz, r_gz[w]);
                mx = max(mx, r_mx[w]);
            }
            if (gs != ~0ull) {
                atomicMin(&a.wdescs[j0].delta_s, gs);
                atomicMin(&a.wdescs[j0].delta_z, gz);
                atomicMax(&a.wdescs[j0].maxm, mx);
            }
        }
        return;
    }
    // the block spans several builds: reduce per wavefront where its lanes share a build
    for (uint32_t k = 0; k < kGapItems; k++) {
        const uint64_t g = tile + (uint64_t)k * kBlock + threadIdx.x;
        uint32_t j = 0;
        GapStat r{~0ull, 0x7fffffffffffffffll, 0};
        if (g < a.nbuckets) {
            j = find_build(a.bucket_base, a.count, g);
            r = gap_of(a, j, g);
        }
        const uint32_t jw = __builtin_amdgcn_readfirstlane(j);
        if (__ballot(g < a.nbuckets && j != jw) == 0) {
            for (int off = 32; off > 0; off >>= 1) {
                r.gs = min(r.gs, (unsigned long long)__shfl_xor(r.gs, off, 64));
                r.gz = min(r.gz, (long long)__shfl_xor(r.gz, off, 64));
                r.mx = max(r.mx, (uint32_t)__shfl_xor((int)r.mx, off, 64));
            }
            if (lane == 0 && r.gs != ~0ull) {
                atomicMin(&a.wdescs[jw].delta_s, r.gs);
                atomicMin(&a.wdescs[jw].delta_z, r.gz);
                atomicMax(&a.wdescs[jw].maxm, r.mx);
            }
        } else if (g < a.nbuckets) {
            atomicMin(&a.wdescs[j].delta_s, r.gs);
            atomicMin(&a.wdescs[j].delta_z, r.gz);
            atomicMax(&a.wdescs[j].maxm, r.mx);
        }
    }
}

__device__ __forceinline__ void or_bits(unsigned long long* a, uint64_t pos, uint64_t val, uint32_t nbits) {
    if (nbits == 0) return;
    uint64_t w = pos >> 6;
    uint32_t o = (uint32_t)(pos & 63);
    atomicOr(&a[w], (unsigned long long)(val << o));
    if (o + nbits > 64) atomicOr(&a[w + 1], (unsigned long long)(val >> (64 - o)));
}

__device__ __forceinline__ void or_bits_lds(unsigned long long* a, uint64_t pos, uint64_t val, uint32_t nbits) {
    if (nbits == 0) return;
    const uint32_t w = (uint32_t)(pos >> 6), o = (uint32_t)(pos & 63);
    atomicOr(&a[w], (unsigned long long)(val << o));
    if (o + nbits > 64) atomicOr(&a[w + 1], (unsigned long long)(val >> (64 - o)));
}

struct FillArgs {
    const uint64_t* bstart;
    const uint64_t* qstart;  // first Elias-Fano list (bstart for minimal builds)
    const uint64_t* ostart;
    const uint64_t* seeds;
    const uint32_t* msz;
    const BuildDesc* descs;
    const uint64_t* bucket_base;
    const uint64_t* entry_base;  // bucket_base[j] + j: nb_j + 1 Elias-Fano entries per build
    uint32_t count;
    uint64_t nbuckets;
    const uint32_t* tables;
    uint32_t stride;
    uint64_t g0;             // k_tree_bits: bucket of the launch's first lane group
    const uint64_t* headers;  // k_ef_fill: kHeaderWords per build
};

// One thread per Elias-Fano entry i = 0..nb of every build.
__device__ __forceinline__ void ef_fill_entry(const FillArgs& a, uint64_t e) {
    if (e >= a.nbuckets + a.count) {  // the threads past the entries write the headers
        const uint64_t hw = e - (a.nbuckets + a.count);
        if (hw < (uint64_t)a.count * kHeaderWords) {
            const uint32_t j = (uint32_t)(hw / kHeaderWords), w = (uint32_t)(hw % kHeaderWords);
            if (a.descs[j].blob) a.descs[j].blob[w] = a.headers[hw];
        }
        return;
    }
    const uint32_t j = find_build(a.entry_base, a.count, e);
    const BuildDesc& B = a.descs[j];
    if (!B.blob) return;
    const uint64_t i = e - a.entry_base[j];
    const uint64_t bb = B.bucket_base;
    const uint64_t s = a.qstart[bb + i] - a.qstart[bb];
    const int64_t z = z_of(a.ostart[bb + i] - a.ostart[bb], s, B.beta);
    const uint64_t ys = s - i * B.delta_s;
    const uint64_t yz = (uint64_t)(z - (int64_t)i * B.delta_z);
    const uint64_t lpos = i * (uint64_t)(B.Ws + B.Wz);
    const uint64_t ms = B.Ws ? (~0ull >> (64 - B.Ws)) : 0, mz = B.Wz ? (~0ull >> (64 - B.Wz)) : 0;
    unsigned long long* blob = B.blob;
    or_bits(blob + B.lower_off, lpos, ys & ms, B.Ws);
    or_bits(blob + B.lower_off, lpos + B.Ws, yz & mz, B.Wz);
    const uint64_t ps = (ys >> B.Ws) + i, pz = (yz >> B.Wz) + i;
    or_bits(blob + B.us_off, ps, 1, 1);
    or_bits(blob + B.uz_off, pz, 1, 1);
    if (B.samples_off && (i & (kSelectSample - 1)) == 0) {
        // positions below 2^32 (select_samples_fit)
        uint32_t* smp = reinterpret_cast<uint32_t*>(blob + B.samples_off);
        const uint64_t groups = select_sample_groups(B.nb + 1);
        smp[i / kSelectSample] = (uint32_t)ps;
        smp[groups + i / kSelectSample] = (uint32_t)pz;
    }
    // two-level inventory (Sec. 7.4), s and z interleaved
    if ((i & ((1u << kInvHi) - 1)) == 0) {
        blob[B.inv_hi_off + 2 * (i >> kInvHi)] = ps;
        blob[B.inv_hi_off + 2 * (i >> kInvHi) + 1] = pz;
    }
    if ((i & ((1u << kInvLo) - 1)) == 0) {
        // the anchor: the one of index i rounded down to a multiple of 2^14
        const uint64_t an = i & ~(uint64_t)((1u << kInvHi) - 1);
        const uint64_t sa = a.qstart[bb + an] - a.qstart[bb];
        const int64_t za = z_of(a.ostart[bb + an] - a.ostart[bb], sa, B.beta);
        const uint64_t pa_s = ((sa - an * B.delta_s) >> B.Ws) + an;
        const uint64_t pa_z = ((uint64_t)(za - (int64_t)an * B.delta_z) >> B.Wz) + an;
        const uint64_t ds = ps - pa_s, dz = pz - pa_z;
        const uint64_t vs = ds < kInvOverflow ? ds : kInvOverflow, vz = dz < kInvOverflow ? dz : kInvOverflow;
        const uint64_t e = 2 * (i >> kInvLo);  // s entry; z is e + 1, in the same word
        atomicOr(&blob[B.inv_lo_off + e / 4], (unsigned long long)((vs | vz << 16) << (16 * (e % 4))));
    }
}

__global__ void k_ef_fill(FillArgs a) { ef_fill_entry(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x); }

// Golomb-Rice streams (Sec. 6.2): per bucket, the fixed parts of all coded
// nodes in preorder, then their unary parts (q zeros and a one) in preorder.
// A group of kTreeLanes lanes per bucket, one lane per coded node: the search
// left every node's index and size at its preorder position, so each node's
// two bit offsets are prefix sums over the nodes before it (segmented
// shuffles within the group; a group returns or loops as a whole).  The
// bucket's stream is assembled in an LDS window of kTreeWords words and then
// ORed into the blob one word at a time (the first and last words may be
// shared with the neighbouring buckets); a longer stream is ORed into the blob
// directly.
constexpr uint32_t kTreeLanes = 16;
constexpr uint32_t kTreeWords = 64;
static_assert(64 % kTreeLanes == 0 && kBlock % kTreeLanes == 0, "bucket groups inside one wavefront");

__device__ __forceinline__ uint64_t group_inclusive_sum(uint64_t x, uint32_t gl) {
#pragma unroll
    for (uint32_t off = 1; off < kTreeLanes; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, kTreeLanes);
        if (gl >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ void tree_bits_block(const FillArgs& a, uint64_t block,
                                                unsigned long long (*window)[kTreeWords]) {
    const uint64_t g = a.g0 + (block * kBlock + threadIdx.x) / kTreeLanes;
    const uint32_t gl = threadIdx.x & (kTreeLanes - 1);
    if (g >= a.nbuckets) return;
    const uint32_t j = find_build(a.bucket_base, a.count, g);
    const BuildDesc& B = a.descs[j];
    if (!B.blob) return;
    const uint64_t start = a.bstart[g];
    const uint32_t m0 = (uint32_t)(a.bstart[g + 1] - start);
    if (m0 <= 1) return;
    const uint32_t* R = a.tables + (size_t)B.tab * kTableCount * a.stride;
    const uint32_t* F = R + a.stride;
    const uint32_t nodes = R[2 * a.stride + m0];
    unsigned long long* tree = B.blob + B.tree_off;
    const uint64_t o0 = a.ostart[B.bucket_base];
    const uint64_t first = a.ostart[g] - o0, end = a.ostart[g + 1] - o0;
    const uint64_t w0 = first >> 6, words = ((end + 63) >> 6) - w0;
    const bool in_lds = words <= kTreeWords;
    unsigned long long* win = window[threadIdx.x / kTreeLanes];
    if (in_lds) {
        for (uint32_t i = gl; i < kTreeWords; i += kTreeLanes) win[i] = 0;
        wave_lds_sync();
    }
    // bit positions relative to word w0 in the window, absolute in the blob
    unsigned long long* dst = in_lds ? nullptr : tree;
    const uint64_t base = in_lds ? w0 << 6 : 0;
    uint64_t fp = first - base, up = first + F[m0] - base;
    for (uint32_t c = 0; c < nodes; c += kTreeLanes) {
        const uint32_t k = c + gl;
        const bool act = k < nodes;
        const uint64_t v = act ? a.seeds[start + k] : 0;
        const uint32_t r = act ? R[a.msz[start + k]] : 0;
        const uint64_t q = v >> r;               // zeros of the unary part
        const uint64_t len = act ? q + 1 : 0;    // unary part with its one
        const uint64_t rs = group_inclusive_sum(r, gl), us = group_inclusive_sum(len, gl);
        if (act) {
            const uint64_t fixed = r ? (v & (~0ull >> (64 - r))) : 0;
            if (in_lds) {
                or_bits_lds(win, fp + rs - r, fixed, r);
                or_bits_lds(win, up + us - len + q, 1, 1);
            } else {
                or_bits(dst, fp + rs - r, fixed, r);
                or_bits(dst, up + us - len + q, 1, 1);
            }
        }
        fp += __shfl(rs, kTreeLanes - 1, kTreeLanes);
        up += __shfl(us, kTreeLanes - 1, kTreeLanes);
    }
    if (in_lds) {
        wave_lds_sync();
        for (uint32_t i = gl; i < words; i += kTreeLanes) {
            const unsigned long long x = win[i];
            if (x) atomicOr(&tree[w0 + i], x);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_tree_bits(FillArgs a) {
    __shared__ unsigned long long window[kBlock / kTreeLanes][kTreeWords];
    tree_bits_block(a, blockIdx.x, window);
}

// Both writers in one launch: the first ef_blocks blocks take the
// Elias-Fano entries and headers, the others the Golomb-Rice streams.  The
// two write disjoint words of the blobs, and each is bound by the latency of
// its loads and atomics, so running them side by side hides much of it.
__global__ __launch_bounds__(kBlock) void k_fill(FillArgs a, uint32_t ef_blocks) {
    __shared__ unsigned long long window[kBlock / kTreeLanes][kTreeWords];
    if (blockIdx.x < ef_blocks) ef_fill_entry(a, (uint64_t)blockIdx.x * kBlock + threadIdx.x);
    else tree_bits_block(a, blockIdx.x - ef_blocks, window);
}

// Output range of every bucket of a call that holds a non-minimal build: Q of
// the bucket's size under its build's tables (the size itself for minimal
// builds, whose Q is the identity).  Their prefix sums are the first
// Elias-Fano list.  A bucket above the tables' largest size fails its build
// anyway (the search flags it), so it takes its size.
__global__ void k_range_sizes(const uint64_t* __restrict__ bstart, const BuildDesc* __restrict__ descs,
                              const uint64_t* __restrict__ bucket_base, uint32_t count, uint64_t nbuckets,
                              const uint32_t* __restrict__ tables, uint32_t stride, uint32_t tab_maxm,
                              uint64_t* __restrict__ out) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbuckets) return;
    const uint32_t j = find_build(bucket_base, count, g);
    const uint64_t m = bstart[g + 1] - bstart[g];
    out[g] = m <= tab_maxm ? tables[((size_t)descs[j].tab * kTableCount + 5) * stride + m] : m;
}

// Elias-Fano lower width: the largest W >= 0 with N * 2^W <= U.
__device__ uint32_t ef_width(uint64_t N, uint64_t U) {
    uint32_t W = 0;
    while (W < 62 && (N << (W + 1)) >> (W + 1) == N && (N << (W + 1)) <= U) W++;
    return W;
}

// Blob geometry of every build once its sizes are known: beta, the
// Elias-Fano widths, the header words, the word offsets of the arrays and the
// blob's size (raw_words; rounded up to 256 bytes in the arena).  Builds with
// an error flag get no blob (size 0).  One block: builds are taken 256 at a
// time and their rounded sizes are scanned into the arena offsets off[0..K].
__device__ uint64_t geometry_of(BuildDesc& d, uint64_t* h) {
    const uint64_t n = d.n, nb = d.nb, N = nb + 1, bits = d.total_bits, U = d.range_total;
    const uint64_t beta = (bits << 16) / U;
    const uint64_t ys_last = U - nb * (uint64_t)d.delta_s;
    const int64_t z_last = (int64_t)bits - (int64_t)((beta * U) >> 16);
    const uint64_t yz_last = (uint64_t)(z_last - (int64_t)nb * (int64_t)d.delta_z);
    const uint32_t Ws = ef_width(N, ys_last), Wz = ef_width(N, yz_last);
    h[0] = kMagic;
    h[1] = kVersion | ((uint64_t)d.kind << 32);
    h[2] = n;
    h[3] = d.leaf;
    h[4] = d.bucket;
    h[5] = nb;
    h[6] = d.maxm;
    h[7] = (uint64_t)Ws | ((uint64_t)Wz << 8) | ((uint64_t)d.gr_max << 16) | ((uint64_t)d.slack << 40);
    h[8] = d.delta_s;
    h[9] = (uint64_t)d.delta_z;
    h[10] = beta;
    const uint64_t us_words = ((ys_last >> Ws) + N + 63) / 64, uz_words = ((yz_last >> Wz) + N + 63) / 64;
    const uint64_t lower_words = (N * (Ws + Wz) + 63) / 64 + 1, tree_words = (bits + 63) / 64 + 1;
    h[11] = us_words;
    h[12] = uz_words;
    h[13] = lower_words;
    h[14] = tree_words;
    h[15] = bits;

    d.beta = beta;
    d.Ws = Ws;
    d.Wz = Wz;
    d.lower_off = kHeaderWords;
    d.us_off = d.lower_off + lower_words;
    d.uz_off = d.us_off + us_words;
    d.inv_hi_off = d.uz_off + uz_words;
    d.inv_lo_off = d.inv_hi_off + inv_hi_words(N);
    d.tree_off = d.inv_lo_off + inv_lo_words(N);
    return d.tree_off + tree_words;
}

// with_samples: each arena slot also holds the build's select samples
// (select_samples_words after the blob, which is rounded to 256 bytes).
__global__ __launch_bounds__(kBlock) void k_layout(BuildDesc* __restrict__ descs, uint32_t count,
                                                  uint64_t* __restrict__ hdr, uint64_t* __restrict__ raw_words,
                                                  uint64_t* __restrict__ off, uint32_t with_samples) {
    __shared__ uint64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (uint32_t base = 0; base < count; base += kBlock) {
        const uint32_t j = base + threadIdx.x;
        uint64_t w = 0;
        if (j < count) {
            BuildDesc& d = descs[j];
            uint64_t raw = 0;
            if (!(d.flags & (kFlagDuplicate | kFlagSearch | kFlagOffsets | kFlagStack | kFlagTooBig)))
                raw = geometry_of(d, hdr + (size_t)j * kHeaderWords);
            raw_words[j] = raw;
            w = (raw + 31) & ~uint64_t(31);
            d.samples_off = with_samples && raw && select_samples_fit(d.nb + 1) ? w : 0;
            if (d.samples_off) w += (select_samples_words(d.nb + 1) + 31) & ~uint64_t(31);
        }
        uint64_t tot;
        const uint64_t ex = block_exclusive_sum(w, &tot);
        const uint64_t carry = carry_s;
        if (j < count) off[j] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[count] = carry_s;
}

// Blob addresses inside an arena of `capacity` words at the scanned offsets
// (a build that does not fit gets no blob and raises the capacity flag), and
// the first clear_words words of the arena zeroed (the Elias-Fano and
// Golomb-Rice writers OR their bits in).  One launch: the two parts touch
// different memory.
__global__ void k_set_blobs(BuildDesc* __restrict__ descs, uint32_t count, unsigned long long* arena,
                            const uint64_t* __restrict__ off, uint64_t capacity, uint32_t* __restrict__ flags,
                            uint64_t clear_words) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        const uint32_t j = (uint32_t)t;
        if (!arena || off[j + 1] == off[j]) {
            descs[j].blob = nullptr;
        } else if (off[j + 1] > capacity) {
            descs[j].blob = nullptr;
            atomicOr(flags, kFlagCapacity);
        } else {
            descs[j].blob = arena + off[j];
        }
    }
    if (arena)
        for (uint64_t i = t; i < clear_words; i += (uint64_t)gridDim.x * blockDim.x) arena[i] = 0;
}

uint64_t grid_for(uint64_t n, uint64_t block) { return std::max<uint64_t>(1, (n + block - 1) / block); }

// Launch with the grid checked against the dispatch limits (launch.h).
#define RS_LAUNCH(kern, blocks, threads, lds, stream, ...)                                            \
    do {                                                                                              \
        const uint64_t blocks_ = (blocks);                                                            \
        if (!grid_fits(blocks_, (threads)))                                                           \
            return fail(RS_EINVAL, "grid of %llu blocks of %s does not fit one launch",               \
                        (unsigned long long)blocks_, #kern);                                          \
        kern<<<dim3((uint32_t)blocks_), dim3((uint32_t)(threads)), (lds), (stream)>>>(__VA_ARGS__);   \
    } while (0)

// Exclusive scan of n values into out[0..n]; tiles holds ceil(n/kScanTile)+1 words.
template <typename T>
int scan(const T* in, uint64_t n, uint64_t* out, uint64_t* tiles, uint32_t* maxout, hipStream_t s) {
    uint64_t ntiles = std::max<uint64_t>(1, (n + kScanTile - 1) / kScanTile);
    if (ntiles == 1 && !maxout) {  // one tile: one launch (small builds)
        RS_LAUNCH(k_scan_apply<T>, 1, kBlock, 0, s, in, n, nullptr, out);
    } else {
        RS_LAUNCH(k_scan_tiles<T>, ntiles, kBlock, 0, s, in, n, tiles, maxout);
        RS_LAUNCH(k_scan_tile_sums, 1, kBlock, 0, s, tiles, ntiles);
        RS_LAUNCH(k_scan_apply<T>, ntiles, kBlock, 0, s, in, n, tiles, out);
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}


// Grow-only pinned host staging buffer of the calling thread.  Copies from it
// are asynchronous, so an event recorded after the last copy of a call guards
// its reuse by the next call.
struct Staging {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
thread_local Staging g_staging;        // descriptors, bases, headers, sizes
thread_local Staging g_table_staging;  // the call's per-size tables

void* pinned(size_t bytes, Staging& st = g_staging) {
    if (st.pending) {
        (void)hipEventSynchronize(st.done);
        st.pending = false;
    }
    if (st.cap < bytes) {
        if (st.p) (void)hipHostFree(st.p);
        size_t want = std::max<size_t>(bytes, 1 << 16);
        // mapped (on every device) and coherent: kernels read it directly
        // (k_reset, k_copy_words)
        const unsigned flags = hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable;
        if (hipHostMalloc(&st.p, want, flags) != hipSuccess) {
            st.p = nullptr;
            st.cap = 0;
            return nullptr;
        }
        st.cap = want;
    }
    return st.p;
}

// After the last copy of a call from either staging buffer.
void pinned_release(hipStream_t s) {
    for (Staging* st : {&g_staging, &g_table_staging}) {
        if (!st->p) continue;
        if (!st->done && hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
            st->done = nullptr;
            (void)hipStreamSynchronize(s);
            return;
        }
        if (hipEventRecord(st->done, s) == hipSuccess) st->pending = true;
        else (void)hipStreamSynchronize(s);
    }
}

thread_local rs_build_stats g_stats;
thread_local bool g_stats_valid = false;

struct PhaseEvents {
    hipEvent_t ev[7] = {};
    bool on = false;
    int create(bool enable) {
        on = enable;
        if (!on) return RS_OK;
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(RS_EDEVICE, "hipEventCreate failed");
        return RS_OK;
    }
    void record(int i, hipStream_t s) {
        if (on) (void)hipEventRecord(ev[i], s);
    }
    double ms(int a, int b) {
        float t = 0;
        (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
    ~PhaseEvents() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

int max_lds_bytes() {
    static int v = -1;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        v = hipGetDeviceProperties(&prop, dev) == hipSuccess ? (int)prop.sharedMemPerBlock : 65536;
    });
    return v;
}

// Accelerator complex dies (XCDs) of the current device; workgroups of a
// one-dimensional grid are dealt to them round-robin by workgroup number.
uint32_t xcd_count() {
    static uint32_t v = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, x = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&x, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess) x = 1;
        v = (uint32_t)std::min(std::max(x, 1), 16);
    });
    return v;
}

// Search kernel of a (leaf-size class, wavefronts per workgroup) pair.
using SearchKernel = void (*)(SearchArgs);

template <int MAXL, bool WIDE>
SearchKernel search_kernel_waves(uint32_t waves) {
    switch (waves) {
        case 1: return k_search<MAXL, 1, WIDE>;
        case 2: return k_search<MAXL, 2, WIDE>;
        case 4: return k_search<MAXL, 4, WIDE>;
        default: return k_search<MAXL, 8, WIDE>;
    }
}

// Calls with a non-minimal build take the kernels whose leaves search
// injections into a larger range (three leaf-size classes).
SearchKernel search_kernel(uint32_t max_leaf, uint32_t waves, bool wide) {
    if (wide) {
        if (max_leaf <= 8) return search_kernel_waves<8, true>(waves);
        if (max_leaf <= 16) return search_kernel_waves<16, true>(waves);
        return search_kernel_waves<24, true>(waves);
    }
    if (max_leaf <= 8) return search_kernel_waves<8, false>(waves);
    if (max_leaf <= 12) return search_kernel_waves<12, false>(waves);
    if (max_leaf <= 16) return search_kernel_waves<16, false>(waves);
    return search_kernel_waves<24, false>(waves);
}

// One launch of the search over every bucket of the call: one workgroup of
// `waves` wavefronts per bucket, `lds` bytes of dynamic LDS (keys + node slots).
// Static LDS of a kernel (queried once: a launch may be under graph capture).
int static_lds(const void* k, size_t* out) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, size_t>> known;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& e : known)
        if (e.first == k) {
            *out = e.second;
            return RS_OK;
        }
    hipFuncAttributes attr;
    RS_HIP(hipFuncGetAttributes(&attr, k));
    known.emplace_back(k, attr.sharedSizeBytes);
    *out = attr.sharedSizeBytes;
    return RS_OK;
}

int launch_search(uint32_t max_leaf, uint32_t waves, bool wide, const SearchArgs& sa, size_t lds, hipStream_t s) {
    SearchKernel k = search_kernel(max_leaf, waves, wide);
    size_t static_bytes = 0;
    if (int rc = static_lds(reinterpret_cast<const void*>(k), &static_bytes)) return rc;
    if (lds + static_bytes > (size_t)max_lds_bytes())
        return fail(RS_EINVAL, "largest bucket (%u keys) exceeds the local data share", sa.key_words);
    // one workgroup per bucket, in launches of at most max_grid_blocks() workgroups
    const uint64_t threads = 64ull * waves;
    return for_each_chunk(sa.nbuckets, threads, 1, [&](uint64_t first, uint64_t, uint64_t blocks) -> int {
        if (!grid_fits(blocks, threads))
            return fail(RS_EINVAL, "search grid of %llu blocks does not fit", (unsigned long long)blocks);
        SearchArgs args = sa;
        args.bucket0 = first;
        void* params[] = {&args};
        RS_HIP(hipLaunchKernel(reinterpret_cast<const void*>(k), dim3((uint32_t)blocks), dim3((uint32_t)threads),
                               params, lds, s));
        return RS_OK;
    });
}

}  // namespace

// Shared ownership of the device memory of the blobs of one call.  Blobs may
// outlive the stream they were built on, so they hold an event, not the stream.
struct BlobArena {
    uint64_t* words = nullptr;
    uint32_t* tables = nullptr;
    std::atomic<int> refs{0};
    hipEvent_t ready = nullptr;
    Alloc al;  // the allocator that made words and tables
};

void release_arena(BlobArena* a) {
    if (a && a->refs.fetch_sub(1) == 1) {
        if (a->ready) (void)hipEventSynchronize(a->ready);
        a->al.put_idle(a->words);
        a->al.put_idle(a->tables);
        if (a->ready) (void)hipEventDestroy(a->ready);
        delete a;
    }
}

// RS_DEBUG=1 in the environment prints the construction phases to stderr.
bool debug_trace() {
    static const bool on = [] {
        const char* e = std::getenv("RS_DEBUG");
        return e && *e && *e != '0';
    }();
    return on;
}
#define RS_TRACE(...)                               \
    do {                                            \
        if (debug_trace()) {                        \
            std::fprintf(stderr, "[librecsplit] "); \
            std::fprintf(stderr, __VA_ARGS__);      \
            std::fprintf(stderr, "\n");             \
            std::fflush(stderr);                    \
        }                                           \
    } while (0)

// ---------------------------------------------------------------------------
// Autotuning: the search of one calibration build is launched repeatedly with
// different schedules (the search only reads the scattered keys and rewrites
// the same indices, so repeated launches are independent).
// ---------------------------------------------------------------------------
struct TuneCtx {
    bool probe_only = false;  // time the built-in schedule and report residency only
    double budget_ms = 0;     // search time allowed for the variants
    uint64_t buckets = 0;     // buckets of the calibration build (for the built-in schedule)
    uint32_t bucket = 0;      // its bucket size
    // results
    rs_schedule best{};
    double default_ms = 0;
    double spent_ms = 0;
    uint32_t variants = 0;
    uint64_t resident = 0;  // workgroups of the built-in kernel resident on the whole device
};

int tune_search(TuneCtx& t, uint32_t leaf, BuildDesc* hdesc, BuildDesc* d_desc, const SearchArgs& sa, size_t lds,
                hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RS_EDEVICE, "hipEventCreate failed");
    }
    auto once = [&](const rs_schedule& sc, double* ms) -> int {
        hdesc[0].stage_from = sc.stage_from;
        hdesc[0].group_cap = sc.group_max - 1;
        hdesc[0].waves = sc.waves;
        RS_HIP(hipMemcpyAsync(d_desc, hdesc, sizeof(BuildDesc), hipMemcpyHostToDevice, s));
        RS_HIP(hipEventRecord(e0, s));
        if (int rc = launch_search(leaf, sc.waves, false, sa, lds, s)) return rc;
        RS_HIP(hipEventRecord(e1, s));
        RS_HIP(hipEventSynchronize(e1));
        float f = 0;
        RS_HIP(hipEventElapsedTime(&f, e0, e1));
        *ms = f;
        t.spent_ms += f;
        return RS_OK;
    };
    // short searches are timed three times (minimum), long ones once
    auto measure = [&](const rs_schedule& sc, double* ms) -> int {
        if (int rc = once(sc, ms)) return rc;
        for (int r = 0; r < 2 && *ms < 30.0; r++) {
            double again = 0;
            if (int rc = once(sc, &again)) return rc;
            *ms = std::min(*ms, again);
        }
        return RS_OK;
    };
    int rc = RS_OK;
    rs_schedule cur = builtin_schedule(leaf, t.buckets, t.bucket);
    double warm = 0, warm_total = 0, best_ms = 0;
    // warm-up: the first launches run slower (clocks still ramping), so search
    // for at least 100 ms (at most 20 launches) before timing anything
    for (int r = 0; r < 20 && warm_total < 100.0; r++) {
        if ((rc = once(cur, &warm))) goto done;
        warm_total += warm;
    }
    t.spent_ms = 0;
    if ((rc = measure(cur, &best_ms))) goto done;
    t.default_ms = best_ms;
    if (t.probe_only) {
        int per_cu = 0, cus = 0, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(search_kernel(leaf, cur.waves, false)), 64 * (int)cur.waves, lds) !=
            hipSuccess)
            per_cu = 1;
        t.resident = (uint64_t)std::max(per_cu, 1) * (uint64_t)std::max(cus, 1);
        goto done;
    }
    {
        // one knob at a time: wavefronts per bucket, staged-search threshold, lanes per split candidate
        std::vector<uint32_t> waves_list = leaf <= 8 ? std::vector<uint32_t>{1, 2, 4} : std::vector<uint32_t>{1, 2, 4, 8};
        std::vector<uint32_t> stage_list;
        for (uint32_t v : {7u, 8u, 9u, 11u, 13u, 16u, 25u})
            if (v >= 7 && (v <= leaf || v == 25)) stage_list.push_back(v);
        if (leaf < 7) stage_list.clear();  // no leaf size is ever staged
        const std::vector<uint32_t> group_list{7, 4, 2, 1};
        bool out_of_budget = false;
        for (int knob = 0; knob < 3 && !out_of_budget; knob++) {
            const std::vector<uint32_t>& vals = knob == 0 ? waves_list : knob == 1 ? stage_list : group_list;
            const rs_schedule base = cur;
            for (uint32_t v : vals) {
                rs_schedule cand = base;
                uint32_t& field = knob == 0 ? cand.waves : knob == 1 ? cand.stage_from : cand.group_max;
                if (field == v) continue;
                if (t.variants >= 1 && t.spent_ms >= t.budget_ms) {
                    out_of_budget = true;
                    break;
                }
                field = v;
                double ms = 0;
                if ((rc = measure(cand, &ms))) goto done;
                t.variants++;
                if (ms < best_ms * 0.98) {  // keep a change only beyond timing noise
                    best_ms = ms;
                    cur = cand;
                }
            }
        }
    }
    t.best = cur;
    t.best.search_ms = best_ms;
    t.best.default_ms = t.default_ms;
    t.best.variants = t.variants + 1;
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// ---------------------------------------------------------------------------
// Host orchestration.  A call validates its builds (Batch), carves one device
// workspace and one pinned staging area for them, and enqueues the phases:
//   front:    descriptors in, signatures, two-level sort into bucket order
//   (the host reads the largest bucket: it sizes the tables and the LDS)
//   back:     seed search, bit-length prefix sums, Elias-Fano statistics,
//             blob geometry and arena offsets (all on the device)
//   (the host reads the blob sizes and allocates the arena)
//   fill:     blob addresses, headers, Elias-Fano bits, Golomb-Rice streams
// A plan enqueues the same phases without the two host reads (sizes fixed by
// caps) and captures them into one HIP graph.
// ---------------------------------------------------------------------------
// A set of per-size tables: they depend on the leaf size, the size above
// which splits take the Sec. 7.2 approximation, and the non-minimal slack.
struct TabKey {
    uint32_t leaf, gr_max, slack;
    bool operator==(const TabKey& o) const { return leaf == o.leaf && gr_max == o.gr_max && slack == o.slack; }
};

struct Batch {
    uint32_t count = 0;
    std::vector<int> st;
    std::vector<std::string> why;
    std::vector<BuildDesc> hd;
    std::vector<uint32_t> which;  // desc index -> position in the call
    std::vector<TabKey> tab_keys;  // of each table set
    bool wide = false;             // some build is non-minimal
    bool samples = true;           // arena slots hold select samples (not in allocation-free builds
                                   // nor with RS_OPT_NO_SAMPLES)
    uint64_t total = 0, nbuckets = 0, seed_cap = kDefaultSeedCap;
    uint32_t wait_limit = kDefaultWaitLimit;
    uint32_t K = 0, max_leaf = 1, launch_waves = 1;
    uint32_t shift = 0, nbins = 0, nxcd = 1;
    // device workspace
    size_t ws_bytes = 0;
    uint64_t *d_lo = nullptr, *d_bst = nullptr, *d_sorted = nullptr, *d_tmp = nullptr, *d_seeds = nullptr;
    uint64_t *d_blen = nullptr, *d_ost = nullptr, *d_tiles = nullptr, *d_kb = nullptr, *d_bb = nullptr;
    uint64_t *d_eb = nullptr, *d_hdr = nullptr, *d_raw = nullptr, *d_boff = nullptr;
    uint64_t* d_qst = nullptr;  // prefix sums of bucket ranges (non-minimal calls; else d_bst)
    uint64_t* d_binst = nullptr;
    uint32_t* d_bid = nullptr;
    unsigned long long *d_bincnt = nullptr, *d_bincur = nullptr;
    DevStatus* d_st = nullptr;
    BuildDesc* d_desc = nullptr;
    // pinned staging: descriptors and bases going in; descriptors, headers,
    // blob sizes and offsets and the status words coming back
    size_t pin_bytes = 0, io_in = 0, io_out = 0;
    BuildDesc* h_desc = nullptr;
    uint64_t *h_kb = nullptr, *h_hdr = nullptr, *h_raw = nullptr, *h_boff = nullptr;
    DevStatus* h_st = nullptr;
    // per-size tables and the search's LDS
    uint32_t* d_tab = nullptr;
    uint32_t stride = 0, table_maxm = 0;
    size_t lds = 0;
};

int batch_prepare(Batch& b, const rs_keys* sets, uint32_t count, const uint32_t* leafs, const uint32_t* buckets,
                  const rs_options* opts) {
    if (opts && opts->waves && opts->waves != 1 && opts->waves != 2 && opts->waves != 4 && opts->waves != 8)
        return fail(RS_EINVAL, "waves must be 1, 2, 4 or 8");
    b.count = count;
    b.seed_cap = opts && opts->seed_cap ? std::min(opts->seed_cap, kDefaultSeedCap) : kDefaultSeedCap;
    b.wait_limit = opts && opts->wait_limit ? opts->wait_limit : kDefaultWaitLimit;
    b.samples = !(opts && (opts->flags & RS_OPT_NO_SAMPLES));
    b.st.assign(count, RS_OK);
    b.why.assign(count, std::string());
    for (uint32_t c = 0; c < count; c++) {
        const rs_keys& k = sets[c];
        const uint32_t leaf = leafs[c], bucket = buckets[c];
        const char* bad = nullptr;
        if (k.n == 0) bad = "empty key set";
        else if (leaf < 1 || leaf > kMaxLeaf) bad = "leaf size outside [1, 24]";
        else if (bucket == 0) bad = "bucket size must be positive";
        else if (!k.data) bad = "NULL key data";
        else if (k.kind != RS_KEYS_U64 && k.kind != RS_KEYS_BYTES) bad = "unknown key kind";
        else if (k.kind == RS_KEYS_BYTES && !k.offsets) bad = "NULL offsets for byte keys";
        else if (opts && opts->gr_table_max >= (1u << 24)) bad = "gr_table_max must be below 2^24";
        else if (opts && opts->leaf_slack > kMaxSlack) bad = "leaf_slack must be at most 255";
        else if (opts && leaf_range(leaf, opts->leaf_slack) > kMaxLeafRange)
            bad = "leaf_slack gives leaves more than 32 values";
        if (bad) {
            b.st[c] = RS_EINVAL;
            b.why[c] = bad;
            continue;
        }
        BuildDesc d{};
        d.data = k.data;
        d.offsets = k.offsets;
        d.n = k.n;
        d.key_base = b.total;
        d.nb = (k.n + bucket - 1) / bucket;
        d.bucket_base = b.nbuckets;
        d.kind = k.kind;
        const Strategy sg = make_strategy(leaf);
        d.leaf = leaf;
        d.lower = sg.lower;
        d.upper = sg.upper;
        d.bucket = bucket;
        d.gr_max = opts ? opts->gr_table_max : 0;
        d.slack = opts ? opts->leaf_slack : 0;
        const TabKey key{leaf, d.gr_max, d.slack};
        uint32_t t = 0;
        while (t < b.tab_keys.size() && !(b.tab_keys[t] == key)) t++;
        if (t == b.tab_keys.size()) b.tab_keys.push_back(key);
        d.tab = t;
        d.aligned = ((uintptr_t)k.data & 7) == 0;
        d.delta_s = ~0ull;
        d.delta_z = 0x7fffffffffffffffll;
        // search schedule: built-in, else the table's (RS_OPT_TUNED), then the
        // overrides; the built-in wavefront count depends on the buckets of the
        // whole call and is set once they are all known (waves = 0 until then)
        rs_schedule sc = builtin_schedule(leaf, 0);
        sc.waves = 0;
        if (opts && (opts->flags & RS_OPT_TUNED)) {
            rs_schedule tuned;
            if (schedule_lookup(leaf, bucket, &tuned)) sc = tuned;
        }
        if (opts && opts->stage_from) sc.stage_from = opts->stage_from;
        if (opts && opts->group_max) sc.group_max = std::min<uint32_t>(opts->group_max, 7);
        if (opts && opts->waves) sc.waves = opts->waves;
        d.stage_from = sc.stage_from;
        d.group_cap = sc.group_max - 1;
        d.waves = sc.waves;
        b.total += d.n;
        b.nbuckets += d.nb;
        b.max_leaf = std::max(b.max_leaf, leaf);
        b.wide |= d.slack != 0;
        b.hd.push_back(d);
        b.which.push_back(c);
    }
    b.K = (uint32_t)b.hd.size();
    if (b.K && b.nbuckets >= (1ull << 32)) return fail(RS_EINVAL, "too many buckets in one call");
    for (BuildDesc& d : b.hd) {
        if (!d.waves) d.waves = builtin_schedule(d.leaf, b.nbuckets, d.bucket).waves;
        b.launch_waves = std::max(b.launch_waves, d.waves);
    }
    return RS_OK;
}

// Status of every build of the call (the first failure also becomes the
// thread's error message).
int batch_finish(Batch& b, int* statuses, int rc) {
    int first = RS_OK;
    for (uint32_t c = 0; c < b.count; c++) {
        if (statuses) statuses[c] = b.st[c];
        if (b.st[c] != RS_OK && first == RS_OK) {
            first = b.st[c];
            fail(b.st[c], "build %u: %s", c, b.why[c].c_str());
        }
    }
    return rc != RS_OK ? rc : first;
}

// Bin geometry and the sizes of the workspace and of the pinned staging.
int batch_layout(Batch& b) {
    // bins of the two-level bucket sort: about 16k keys each, at most kMaxBins
    const double keys_per_bucket = (double)b.total / (double)b.nbuckets;
    b.shift = 0;
    // (a bin of more than kSortSpan buckets only when the bin count requires it)
    while ((1u << (b.shift + 1)) <= kSortSpan && (double)(2ull << b.shift) * keys_per_bucket <= 16384.0) b.shift++;
    while (b.shift < kMaxBinShift && ((b.nbuckets + (1ull << b.shift) - 1) >> b.shift) > kMaxBins) b.shift++;
    const uint64_t nbins64 = (b.nbuckets + (1ull << b.shift) - 1) >> b.shift;
    if (nbins64 > kMaxBins)
        return fail(RS_EINVAL, "too many buckets in one call (%llu; at most %llu)", (unsigned long long)b.nbuckets,
                    (unsigned long long)kMaxBins << kMaxBinShift);
    b.nbins = (uint32_t)nbins64;
    b.nxcd = xcd_count();
    const uint64_t T = b.total, NB = b.nbuckets, K = b.K;
    const uint64_t ntiles = (NB + 1 + kScanTile - 1) / kScanTile + 1;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    b.d_lo = (uint64_t*)carve(T * 8);
    b.d_bid = (uint32_t*)carve(T * 4);
    b.d_bincnt = (unsigned long long*)carve((size_t)b.nbins * b.nxcd * 8);
    b.d_binst = (uint64_t*)carve((b.nbins + 1) * 8ull);
    b.d_bincur = (unsigned long long*)carve((size_t)b.nbins * b.nxcd * 8);
    b.d_bst = (uint64_t*)carve((NB + 1) * 8);
    b.d_sorted = (uint64_t*)carve(T * 8);
    b.d_tmp = (uint64_t*)carve(T * 8);
    b.d_seeds = (uint64_t*)carve(T * 8);
    b.d_blen = (uint64_t*)carve(NB * 8);
    b.d_ost = (uint64_t*)carve((NB + 1) * 8);
    b.d_tiles = (uint64_t*)carve(ntiles * 8);
    b.d_qst = b.wide ? (uint64_t*)carve((NB + 1) * 8) : nullptr;
    // one contiguous block, mirrored in the pinned staging, so that one copy
    // takes it in (bases, descriptors) and one brings it back (descriptors,
    // headers, blob sizes and offsets, status words)
    b.io_in = 3 * (K + 1) * 8 + K * sizeof(BuildDesc);
    b.io_out = K * sizeof(BuildDesc) + K * kHeaderWords * 8 + K * 8 + (K + 1) * 8 + sizeof(DevStatus);
    b.pin_bytes = 3 * (K + 1) * 8 + b.io_out;
    b.d_kb = (uint64_t*)carve(b.pin_bytes);
    b.ws_bytes = off;
    return RS_OK;
}

// Rebase the carved offsets on the workspace and fill the pinned staging.
void batch_bind(Batch& b, char* ws, char* pin) {
    auto at = [&](auto& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(ws + (size_t)p); };
    at(b.d_lo); at(b.d_bid); at(b.d_bincnt); at(b.d_binst); at(b.d_bincur); at(b.d_bst); at(b.d_sorted);
    at(b.d_tmp); at(b.d_seeds); at(b.d_blen); at(b.d_ost); at(b.d_tiles); at(b.d_kb);
    if (b.wide) at(b.d_qst);
    else b.d_qst = b.d_bst;
    const uint32_t K = b.K;
    // [key bases | bucket bases | entry bases | descriptors | headers | raw words | offsets | status]
    auto lay = [K](char* base, uint64_t*& kb, BuildDesc*& desc, uint64_t*& hdr, uint64_t*& raw, uint64_t*& boff,
                   DevStatus*& st) {
        kb = (uint64_t*)base;
        desc = (BuildDesc*)(kb + 3 * (K + 1));
        hdr = (uint64_t*)(desc + K);
        raw = hdr + (size_t)K * kHeaderWords;
        boff = raw + K;
        st = (DevStatus*)(boff + (K + 1));
    };
    lay((char*)b.d_kb, b.d_kb, b.d_desc, b.d_hdr, b.d_raw, b.d_boff, b.d_st);
    lay(pin, b.h_kb, b.h_desc, b.h_hdr, b.h_raw, b.h_boff, b.h_st);
    b.d_bb = b.d_kb + (K + 1);
    b.d_eb = b.d_bb + (K + 1);
    memcpy(b.h_desc, b.hd.data(), K * sizeof(BuildDesc));
    uint64_t* h_bb = b.h_kb + (K + 1);
    uint64_t* h_eb = h_bb + (K + 1);
    for (uint32_t j = 0; j < K; j++) {
        b.h_kb[j] = b.hd[j].key_base;
        h_bb[j] = b.hd[j].bucket_base;
        h_eb[j] = b.hd[j].bucket_base + j;
    }
    b.h_kb[K] = b.total;
    h_bb[K] = b.nbuckets;
    h_eb[K] = b.nbuckets + K;
}

#define RS_ENQ(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(RS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Descriptors in, signatures, sort into bucket order (bstart, sorted keys,
// largest bucket in d_st->maxm).  The descriptors are uploaded from h_desc.
// in_src: null, or the device address of the pinned staging, from which the
// first kernel reads the bases and descriptors (a copy would add the host's
// time in the copy call before that kernel can start).
int enqueue_front(Batch& b, hipStream_t s, PhaseEvents* pe, const void* in_src) {
    const uint32_t K = b.K;
    if (pe) pe->record(0, s);
    if (!in_src) RS_ENQ(hipMemcpyAsync(b.d_kb, b.h_kb, b.io_in, hipMemcpyHostToDevice, s));
    const uint64_t ncnt = (uint64_t)b.nbins * b.nxcd, in_words = in_src ? b.io_in / 8 : 0;
    RS_LAUNCH(k_reset, grid_for(std::max(ncnt, in_words), kBlock * 4), kBlock, 0, s, b.d_st, b.d_bincnt, ncnt,
              b.d_kb, static_cast<const uint64_t*>(in_src), in_words);
    RS_LAUNCH(k_signature, grid_for(b.total, kSigTile), kBlock, b.nbins * 4, s, b.d_desc, b.d_desc, b.d_kb, K,
              b.total, b.d_lo, b.d_bid, b.shift, b.nbins, b.nxcd, b.d_bincnt);
    if (pe) pe->record(1, s);
    // before the search, the partition scratch and the index array hold the keys in bin order
    uint64_t* bin_lo = b.d_tmp;
    uint32_t* bin_bid = (uint32_t*)b.d_seeds;
    RS_LAUNCH(k_bin_offsets, 1, kBlock, 0, s, b.d_bincnt, b.nbins, b.nxcd, b.d_binst, b.d_bincur);
    if (b.nbins <= kScatterMaxBins && staged_scatter_lds(b.nbins) + 256 <= (size_t)max_lds_bytes())
        RS_LAUNCH(k_bin_scatter_staged, grid_for(b.total, kSigTile), kScatterBlock, staged_scatter_lds(b.nbins), s,
                  b.d_lo, b.d_bid, b.total, b.shift, b.nbins, b.nxcd, b.d_bincur, bin_lo, bin_bid);
    else
        RS_LAUNCH(k_bin_scatter, grid_for(b.total, kSigTile), kBlock, b.nbins * 12, s, b.d_lo, b.d_bid, b.total,
                  b.shift, b.nbins, b.nxcd, b.d_bincur, bin_lo, bin_bid);
    const uint32_t piece = (uint32_t)std::min<uint64_t>(std::min(1u << b.shift, kSortSpan), b.nbuckets);
    RS_LAUNCH(k_bucket_sort, b.nbins, kSortBlock, 8u * piece, s, b.d_binst, bin_lo, bin_bid, b.shift, piece,
              b.nbuckets, b.d_bst, b.d_sorted, &b.d_st->maxm);
    if (pe) pe->record(2, s);
    RS_ENQ(hipGetLastError());
    return RS_OK;
}

// Per-size tables of every table set of the call for sizes 0..maxm (each set
// kTableCount arrays of maxm + 1 words, table_words(b) words in b.d_tab) and
// the search's dynamic LDS (keys + node slots of the largest possible bucket).
// The host cache may hold a set for many more sizes (the LDS limit probes up
// to ~20,000): only the sizes the call can meet go up.
int prepare_tables(Batch& b, uint32_t maxm) {
    b.table_maxm = maxm;
    b.stride = maxm + 1;
    uint32_t max_nodes = 0;
    for (const TabKey& key : b.tab_keys) {
        const TableView tv = host_tables(key.leaf, maxm, key.gr_max, key.slack);
        if (!tv.data) return fail(RS_ENOMEM, "table allocation failed");
        if (key.slack && !ranges_increasing(tv.Q(), maxm))
            return fail(RS_EINVAL, "leaf_slack %u gives two bucket sizes the same range", key.slack);
        for (uint32_t m = 0; m <= maxm; m++) max_nodes = std::max(max_nodes, tv.N()[m]);
    }
    b.lds = (size_t)maxm * 8 + (size_t)max_nodes * 16;
    return RS_OK;
}

size_t table_words(const Batch& b) { return b.tab_keys.size() * kTableCount * (size_t)b.stride; }

// Words from pinned host memory, read by the kernel itself.
__global__ void k_copy_words(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// stage: null, or pinned host memory of table_words(b) words.  A copy from
// pageable memory returns only once it has been made, i.e. after the work
// queued before it.  From the pinned staging a small kernel reads the tables
// in stream order: a copy engine would add its hand-over from the compute
// queue and back (about 30 us between the bucketing and the search).
int upload_batch_tables(Batch& b, hipStream_t s, uint32_t* stage) {
    if (stage) {
        for (uint32_t t = 0; t < (uint32_t)b.tab_keys.size(); t++) {
            const TabKey& key = b.tab_keys[t];
            const TableView tv = host_tables(key.leaf, b.table_maxm, key.gr_max, key.slack);
            if (!tv.data) return fail(RS_ENOMEM, "table allocation failed");
            for (int a = 0; a < kTableCount; a++)
                memcpy(stage + ((size_t)t * kTableCount + a) * b.stride, tv.data + (size_t)a * (tv.cap + 1),
                       (size_t)b.stride * 4);
        }
        void* src = nullptr;
        RS_ENQ(hipHostGetDevicePointer(&src, stage, 0));
        const uint64_t n = table_words(b);
        RS_LAUNCH(k_copy_words, std::min<uint64_t>(grid_for(n, kBlock), 64), kBlock, 0, s, b.d_tab,
                  static_cast<const uint32_t*>(src), n);
        RS_ENQ(hipGetLastError());
        return RS_OK;
    }
    for (uint32_t t = 0; t < (uint32_t)b.tab_keys.size(); t++) {
        const TabKey& key = b.tab_keys[t];
        const TableView tv = host_tables(key.leaf, b.table_maxm, key.gr_max, key.slack);
        if (!tv.data) return fail(RS_ENOMEM, "table allocation failed");
        uint32_t* dst = b.d_tab + (size_t)t * kTableCount * b.stride;
        for (int a = 0; a < kTableCount; a++)
            RS_ENQ(hipMemcpyAsync(dst + (size_t)a * b.stride, tv.data + (size_t)a * (tv.cap + 1), b.stride * 4ull,
                                  hipMemcpyHostToDevice, s));
    }
    return RS_OK;
}

SearchArgs search_args(const Batch& b) {
    // the bucket numbers of the keys are no longer needed once the keys are
    // in bucket order: their array takes the node sizes
    return SearchArgs{b.d_sorted, b.d_tmp, b.d_bst, b.d_seeds, b.d_bid, b.d_blen, b.d_desc, b.d_desc, b.d_bb, b.K,
                      b.nbuckets, b.d_tab, b.stride, b.seed_cap, b.table_maxm, b.wait_limit, 0};
}

// Seed search, bit-length prefix sums, Elias-Fano statistics, blob geometry
// and the arena offsets (d_boff[K] = arena words).
int enqueue_back(Batch& b, hipStream_t s, PhaseEvents* pe) {
    if (pe) pe->record(3, s);
    if (int rc = launch_search(b.max_leaf, b.launch_waves, b.wide, search_args(b), b.lds, s)) return rc;
    if (pe) pe->record(4, s);
    if (int rc = scan<uint64_t>(b.d_blen, b.nbuckets, b.d_ost, b.d_tiles, nullptr, s)) return rc;
    if (b.wide) {  // bucket ranges into the bit lengths' array (scanned already), then their prefix sums
        RS_LAUNCH(k_range_sizes, grid_for(b.nbuckets, kBlock), kBlock, 0, s, b.d_bst, b.d_desc, b.d_bb, b.K,
                  b.nbuckets, b.d_tab, b.stride, b.table_maxm, b.d_blen);
        if (int rc = scan<uint64_t>(b.d_blen, b.nbuckets, b.d_qst, b.d_tiles, nullptr, s)) return rc;
    }
    GapArgs ga{b.d_bst, b.d_qst, b.d_ost, b.d_desc, b.d_desc, b.d_bb, b.K, b.nbuckets};
    RS_LAUNCH(k_ef_gaps, grid_for(b.nbuckets, kGapTile), kBlock, 0, s, ga);
    RS_LAUNCH(k_layout, 1, kBlock, 0, s, b.d_desc, b.K, b.d_hdr, b.d_raw, b.d_boff, (uint32_t)b.samples);
    if (pe) pe->record(5, s);
    RS_ENQ(hipGetLastError());
    return RS_OK;
}

// Blob addresses in `arena` (capacity words; the first clear_words words are
// zeroed first), headers, Elias-Fano bits and Golomb-Rice streams.
int enqueue_fill(Batch& b, uint64_t* arena, uint64_t capacity, uint64_t clear_words, hipStream_t s) {
    const uint32_t K = b.K;
    const uint64_t clear = arena ? clear_words : 0;
    RS_LAUNCH(k_set_blobs, std::max(grid_for(K, kBlock), grid_for(clear, kBlock * 8)), kBlock, 0, s, b.d_desc, K,
              (unsigned long long*)arena, b.d_boff, capacity, &b.d_st->flags, clear);
    FillArgs fa{b.d_bst, b.d_qst, b.d_ost, b.d_seeds, b.d_bid, b.d_desc, b.d_bb, b.d_eb, K, b.nbuckets, b.d_tab,
                b.stride, 0, b.d_hdr};
    // Elias-Fano entries, then the header words of every build; kTreeLanes
    // lanes per bucket for the trees.  One launch where both fit in one grid.
    const uint64_t ef_blocks = grid_for(b.nbuckets + K + (uint64_t)K * kHeaderWords, kBlock);
    const uint64_t tree_blocks = grid_for(b.nbuckets, kBlock / kTreeLanes);
    if (ef_blocks + tree_blocks <= max_grid_blocks(kBlock)) {
        RS_LAUNCH(k_fill, ef_blocks + tree_blocks, kBlock, 0, s, fa, (uint32_t)ef_blocks);
        RS_ENQ(hipGetLastError());
        return RS_OK;
    }
    RS_LAUNCH(k_ef_fill, ef_blocks, kBlock, 0, s, fa);
    // trees in launches of at most max_grid_blocks() blocks
    if (int rc = for_each_chunk(b.nbuckets, kBlock, kBlock / kTreeLanes, [&](uint64_t g0, uint64_t, uint64_t blocks) -> int {
            fa.g0 = g0;
            RS_LAUNCH(k_tree_bits, blocks, kBlock, 0, s, fa);
            return RS_OK;
        }))
        return rc;
    RS_ENQ(hipGetLastError());
    return RS_OK;
}

// Descriptors, headers, blob sizes and offsets and the status words back to
// the pinned staging.
int enqueue_readback(Batch& b, hipStream_t s) {
    RS_ENQ(hipMemcpyAsync(b.h_desc, b.d_desc, b.io_out, hipMemcpyDeviceToHost, s));
    return RS_OK;
}
#undef RS_ENQ

// Per-build status from the flags the device raised.
void collect_status(Batch& b) {
    for (uint32_t j = 0; j < b.K; j++) {
        const uint32_t c = b.which[j], f = b.h_desc[j].flags;
        if (b.st[c] != RS_OK) continue;
        if (f & kFlagOffsets) {
            b.st[c] = RS_EINVAL;
            b.why[c] = "byte-key offsets are not monotone";
        } else if (f & kFlagDuplicate) {
            b.st[c] = RS_EDUPLICATE;
            b.why[c] = "duplicate keys (equal signatures)";
        } else if (f & kFlagSearch) {
            b.st[c] = RS_ESEARCH;
            b.why[c] = "an index search reached the seed cap";
        } else if (f & kFlagStack) {
            b.st[c] = RS_EDEVICE;
            b.why[c] = "search scheduling failed";
        }
    }
}

// Blob objects of the successful builds over `words` (the arena, laid out at
// h_boff) and `tables`; the arena is freed with the last of them.
void make_blobs(Batch& b, uint64_t* words, uint32_t* tables, uint32_t stride, const Alloc& al, hipStream_t s,
                rs_blob** outs) {
    uint32_t made = 0;
    for (uint32_t j = 0; j < b.K; j++) made += b.st[b.which[j]] == RS_OK;
    for (uint32_t c = 0; c < b.count; c++) outs[c] = nullptr;
    if (!made) {
        al.put(words, s);
        al.put(tables, s);
        return;
    }
    BlobArena* arena = new (std::nothrow) BlobArena;
    if (!arena) {
        for (uint32_t j = 0; j < b.K; j++)
            if (b.st[b.which[j]] == RS_OK) {
                b.st[b.which[j]] = RS_ENOMEM;
                b.why[b.which[j]] = "host allocation failed";
            }
        al.put(words, s);
        al.put(tables, s);
        return;
    }
    arena->words = words;
    arena->tables = tables;
    arena->al = al;
    arena->refs = (int)made;
    if (hipEventCreateWithFlags(&arena->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(arena->ready, s) != hipSuccess) {
        (void)hipStreamSynchronize(s);  // no event: the blobs are complete once the stream is
        if (arena->ready) (void)hipEventDestroy(arena->ready);
        arena->ready = nullptr;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (uint32_t j = 0; j < b.K; j++) {
        const uint32_t c = b.which[j];
        if (b.st[c] != RS_OK) continue;
        rs_blob* blob = new (std::nothrow) rs_blob;
        if (!blob) {
            b.st[c] = RS_ENOMEM;
            b.why[c] = "host allocation failed";
            release_arena(arena);
            continue;
        }
        blob->words = words + b.h_boff[j];
        blob->bytes = b.h_raw[j] * 8;
        blob->samples = b.h_desc[j].samples_off
                            ? reinterpret_cast<const uint32_t*>(words + b.h_boff[j] + b.h_desc[j].samples_off)
                            : nullptr;
        blob->tables = tables + (size_t)b.h_desc[j].tab * kTableCount * stride;
        blob->tab_stride = stride;
        {
            const TabKey& key = b.tab_keys[b.h_desc[j].tab];
            const TableView tv = host_tables(key.leaf, stride - 1, key.gr_max, key.slack);
            blob->packed = !key.slack && tv.data &&
                           packed_valid(tv.P(), (uint32_t)b.h_hdr[(size_t)j * kHeaderWords + 6]);
        }
        memcpy(blob->header, b.h_hdr + (size_t)j * kHeaderWords, sizeof blob->header);
        blob->ready = arena->ready;
        blob->device = dev;
        blob->arena = arena;
        outs[c] = blob;
    }
}

uint32_t lds_bucket_limit(Batch& b);

// Largest bucket that n keys in nb buckets exceed with probability below
// 1e-6: a bucket's count is Binomial(n, 1/nb), bounded by the heavier-tailed
// Poisson(n / nb); the tail is summed downward from far above the mean.
// The last (n, nb) of the calling thread is remembered: repeated builds of
// one shape skip the sum.
uint32_t bucket_size_cap(uint64_t n, uint64_t nb) {
    thread_local uint64_t last_n = 0, last_nb = 0;
    thread_local uint32_t last_cap = 0;
    if (n == last_n && nb == last_nb && last_cap) return last_cap;
    const double lam = (double)n / (double)nb, target = 1e-6 / (double)nb;
    const uint64_t k0 = (uint64_t)lam;
    const uint64_t kmax = k0 + (uint64_t)(20.0 * std::sqrt(lam + 1.0)) + 40;
    std::vector<double> pmf(kmax - k0 + 1);
    double p = std::exp((double)k0 * std::log(lam) - lam - std::lgamma((double)k0 + 1.0));
    for (uint64_t k = k0; k <= kmax; k++) {  // pmf(k + 1) = pmf(k) lam / (k + 1)
        pmf[k - k0] = p;
        p *= lam / (double)(k + 1);
    }
    double tail = 0;  // P(X > c)
    uint64_t c = kmax;
    while (c > k0 && tail + pmf[c - k0] < target) tail += pmf[c-- - k0];
    last_cap = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(c, 1), n);
    last_n = n;
    last_nb = nb;
    return last_cap;
}

// Blob words per key of the calling thread's last single build.  A later
// single build of the same shape (l, b, Golomb-Rice table bound, slack, with
// or without select samples) and of a similar key count (within a factor of
// two: small sets spend more words per key on the header and the index)
// enqueues its fill into an arena of n times that (with a
// margin) before its one wait on the stream, rather
// than waiting for the exact sizes and then filling: the host's wake-up and
// two launches leave the critical path.  A blob beyond the guessed arena is
// flagged by k_set_blobs, and after the wait it is filled again into an
// arena of the exact size (same bytes).  RS_ARENA_GUESS scales the margin
// (0: never guess), read at each call.
struct ArenaMemo {
    uint32_t leaf = 0, bucket = 0, gr_max = 0, slack = 0;
    bool samples = false;
    uint64_t n = 0;
    double words_per_key = 0;
};
thread_local ArenaMemo g_arena_memo;

uint64_t arena_guess(const Batch& b) {
    if (b.K != 1) return 0;
    const BuildDesc& d = b.hd[0];
    const ArenaMemo& m = g_arena_memo;
    if (m.words_per_key <= 0 || m.leaf != d.leaf || m.bucket != d.bucket || m.gr_max != d.gr_max ||
        m.slack != d.slack || m.samples != b.samples || d.n > 2 * m.n || 2 * d.n < m.n)
        return 0;
    double scale = 1.125;
    if (const char* e = std::getenv("RS_ARENA_GUESS"); e && *e) scale = std::atof(e);
    if (!(scale > 0)) return 0;
    return (uint64_t)std::ceil((double)d.n * m.words_per_key * scale) + 256;
}

void arena_remember(const Batch& b) {
    if (b.K != 1 || b.h_boff[1] == 0) return;
    const BuildDesc& d = b.hd[0];
    ArenaMemo& m = g_arena_memo;
    m.leaf = d.leaf;
    m.bucket = d.bucket;
    m.gr_max = d.gr_max;
    m.slack = d.slack;
    m.samples = b.samples;
    m.n = d.n;
    m.words_per_key = (double)b.h_boff[1] / (double)d.n;
}

// maxm_hint: 0 = size the tables and the search's LDS for a bucket-size cap
// estimated from the key and bucket counts, so that the call waits on its
// stream only once (for the blob sizes); if a bucket exceeds the cap, the call
// is made again with the largest bucket the first attempt measured.
int build_batch_impl(const rs_keys* sets, uint32_t count, const uint32_t* leafs, const uint32_t* buckets,
                     const rs_options* opts, hipStream_t s, rs_blob** outs, int* statuses, TuneCtx* tune,
                     uint32_t maxm_hint = 0) {
    if (!sets || !leafs || !buckets || !outs || count == 0) return fail(RS_EINVAL, "NULL argument or empty batch");
    const bool timing = opts && (opts->flags & RS_OPT_TIMING);
    Batch b;
    if (int rc = batch_prepare(b, sets, count, leafs, buckets, opts)) return rc;
    if (b.K == 0) return batch_finish(b, statuses, RS_OK);
    if (int rc = batch_layout(b)) return rc;
    RS_TRACE("build call: %u builds, %llu keys, %llu buckets", b.K, (unsigned long long)b.total,
             (unsigned long long)b.nbuckets);
    PhaseEvents pe;
    if (int rc0 = pe.create(timing)) return rc0;

    const Alloc al = current_alloc();
    char* ws = nullptr;
    if (int rc0 = al.get((void**)&ws, b.ws_bytes, s)) return rc0;
    uint64_t* d_blob = nullptr;
    auto cleanup = [&](int code) {
        pinned_release(s);
        al.put(ws, s);
        if (code != RS_OK) {
            al.put(b.d_tab, s);
            al.put(d_blob, s);
        }
        return code;
    };
#define RS_TRY(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return cleanup(fail(RS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)));          \
    } while (0)
    char* pin = (char*)pinned(b.pin_bytes);
    if (!pin) return cleanup(fail(RS_ENOMEM, "pinned host allocation failed"));
    batch_bind(b, ws, pin);
    void* pin_dev = nullptr;  // the bases and descriptors go in through k_reset
    RS_TRY(hipHostGetDevicePointer(&pin_dev, pin, 0));

    if (int rc = enqueue_front(b, s, &pe, pin_dev)) return cleanup(rc);
    uint32_t maxm = maxm_hint;
    const bool capped = !tune && !maxm_hint;
    if (capped) {
        for (const BuildDesc& d : b.hd) maxm = std::max(maxm, bucket_size_cap(d.n, d.nb));
        maxm = std::min(maxm, lds_bucket_limit(b));
        RS_TRACE("bucket-size cap %u", maxm);
    } else if (!maxm) {
        RS_TRY(hipMemcpyAsync(b.h_st, b.d_st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        RS_TRACE("signatures enqueued; waiting for the largest bucket");
        RS_TRY(hipStreamSynchronize(s));
        maxm = b.h_st->maxm;
        RS_TRACE("largest bucket %u", maxm);
    }
    if (int rc = prepare_tables(b, maxm)) return cleanup(rc);
    if (int rc = al.get((void**)&b.d_tab, table_words(b) * 4, s)) return cleanup(rc);
    uint32_t* stage = static_cast<uint32_t*>(pinned(table_words(b) * 4, g_table_staging));
    if (!stage) return cleanup(fail(RS_ENOMEM, "pinned host allocation failed"));
    if (int rc = upload_batch_tables(b, s, stage)) return cleanup(rc);
    if (tune) {  // calibration only: no blob, the tables are not handed to an arena
        tune->buckets = b.nbuckets;
        tune->bucket = b.hd.empty() ? 0 : b.hd[0].bucket;
        const int trc = tune_search(*tune, b.max_leaf, b.h_desc, b.d_desc, search_args(b), b.lds, s);
        al.put(b.d_tab, s);
        b.d_tab = nullptr;
        return cleanup(trc);
    }
    if (int rc = enqueue_back(b, s, &pe)) return cleanup(rc);
    uint64_t guess = arena_guess(b);
    if (guess && al.get((void**)&d_blob, guess * 8, s) != RS_OK) {
        clear_error();  // no room for a guess: the exact arena after the wait
        (void)hipGetLastError();
        d_blob = nullptr;
        guess = 0;
    }
    if (guess) {
        if (int rc = enqueue_fill(b, d_blob, guess, guess, s)) return cleanup(rc);
        pe.record(6, s);
        RS_TRACE("fill enqueued into a guessed arena of %llu words", (unsigned long long)guess);
    }
    if (int rc = enqueue_readback(b, s)) return cleanup(rc);
    RS_TRACE("search enqueued (class %u); waiting for the sizes", b.max_leaf);
    RS_TRY(hipStreamSynchronize(s));
    if (capped) {
        bool over = false;
        for (uint32_t j = 0; j < b.K; j++) over |= (b.h_desc[j].flags & kFlagTooBig) != 0;
        if (over) {  // a bucket above the cap: again, sized for the largest bucket now known
            const uint32_t exact = std::max(b.h_st->maxm, maxm + 1);
            RS_TRACE("a bucket exceeds the cap %u; again with %u", maxm, exact);
            pinned_release(s);
            al.put(ws, s);
            al.put(b.d_tab, s);
            al.put(d_blob, s);
            return build_batch_impl(sets, count, leafs, buckets, opts, s, outs, statuses, nullptr, exact);
        }
    }
    collect_status(b);
    const uint64_t arena_words = b.h_boff[b.K];
    RS_TRACE("sizes known (%llu blob words)", (unsigned long long)arena_words);
    arena_remember(b);
    uint64_t arena_cap = guess;
    uint32_t refills = 0;
    if (!arena_words || arena_words > guess) {  // no guess, or a blob beyond it: fill an exact arena
        refills = guess && arena_words ? 1 : 0;
        if (refills) RS_TRACE("the guessed arena is too small; filled again");
        al.put(d_blob, s);
        d_blob = nullptr;
        arena_cap = arena_words;
        if (arena_words) {
            if (int rc = al.get((void**)&d_blob, arena_words * 8, s)) return cleanup(rc);
            if (int rc = enqueue_fill(b, d_blob, arena_words, arena_words, s)) return cleanup(rc);
        }
        pe.record(6, s);
    }
    if (timing) {
        RS_TRY(hipStreamSynchronize(s));
        g_stats.ms_signature = pe.ms(0, 1);
        g_stats.ms_scatter = pe.ms(1, 2);
        g_stats.ms_search = pe.ms(3, 4);
        g_stats.ms_offsets = pe.ms(4, 5);
        g_stats.ms_fill = pe.ms(5, 6);
        g_stats.ms_device = pe.ms(0, 6);
        g_stats.n = b.total;
        g_stats.nb = b.nbuckets;
        g_stats.maxm = b.h_st->maxm;
        g_stats.tree_bits = 0;
        for (uint32_t j = 0; j < b.K; j++) g_stats.tree_bits += b.h_desc[j].total_bits;
        g_stats.blob_bytes = arena_words * 8;
        g_stats.arena_bytes = arena_cap * 8;
        g_stats.refills = refills;
        g_stats_valid = true;
    }
    make_blobs(b, d_blob, b.d_tab, b.stride, al, s, outs);
    pinned_release(s);
    al.put(ws, s);
    return batch_finish(b, statuses, RS_OK);
#undef RS_TRY
}

// ---------------------------------------------------------------------------
// Build plans: the construction of a fixed batch shape captured into one HIP
// graph.  The largest bucket and the blob sizes are not known in advance, so
// the plan sizes the search's LDS and the tables for a bucket cap and the blob
// arena for a word cap, both set with a margin from a first ordinary build;
// the kernels flag buckets or blobs beyond the caps and the run then falls
// back to an ordinary build.
// ---------------------------------------------------------------------------
}  // namespace rs

struct rs_plan {
    rs::Batch b;
    std::vector<rs_keys> sets;
    std::vector<uint32_t> leafs, buckets;
    rs_options opts{};
    char* ws = nullptr;
    char* pin = nullptr;
    uint64_t* arena = nullptr;
    uint64_t capacity = 0;
    uint32_t maxm_cap = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // the last run's copies out of the arena
    bool done_pending = false;
    uint64_t runs = 0, fallbacks = 0;
    rs::Alloc al;  // device memory of the plan and of the blobs its runs return
};

namespace rs {

void plan_release(rs_plan* p) {
    if (!p) return;
    if (p->done_pending) (void)hipEventSynchronize(p->done);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->al.put_idle(p->ws);
    p->al.put_idle(p->b.d_tab);
    p->al.put_idle(p->arena);
    if (p->pin) (void)hipHostFree(p->pin);
    delete p;
}

// Largest bucket of which the search still fits the LDS with the tables of
// this batch (binary search over the dynamic LDS the launch would ask for;
// remembered per kernel and table sets, as the search takes ~60 us of host
// time, which a small build would wait for).
uint32_t lds_bucket_limit(Batch& b) {
    SearchKernel k = search_kernel(b.max_leaf, b.launch_waves, b.wide);
    struct Known {
        SearchKernel k;
        std::vector<TabKey> keys;
        uint32_t limit;
    };
    static std::mutex mu;
    static std::vector<Known> known;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Known& e : known)
            if (e.k == k && e.keys == b.tab_keys) return e.limit;
    }
    size_t static_bytes = 0;
    if (static_lds(reinterpret_cast<const void*>(k), &static_bytes)) return 0;
    const size_t avail = (size_t)max_lds_bytes() - static_bytes;
    uint32_t lo = 0, hi = (uint32_t)(avail / 8);
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        uint32_t nodes = 0;
        for (const auto& key : b.tab_keys) {
            TableView tv = host_tables(key.leaf, mid, key.gr_max, key.slack);
            if (!tv.data) return 0;
            for (uint32_t m = 0; m <= mid; m++) nodes = std::max(nodes, tv.N()[m]);
        }
        if ((size_t)mid * 8 + (size_t)nodes * 16 <= avail) lo = mid;
        else hi = mid - 1;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (known.size() < 256) known.push_back(Known{k, b.tab_keys, lo});
    return lo;
}

}  // namespace rs

extern "C" int rs_plan_create(const rs_keys* sets, uint32_t count, const uint32_t* leaf, const uint32_t* bucket,
                              const rs_options* opts, void* stream, rs_plan** out, rs_blob** first_outs,
                              int* per_build_status) {
    rs::clear_error();
    if (!sets || !leaf || !bucket || !out || count == 0) return rs::fail(RS_EINVAL, "NULL argument or empty batch");
    hipStream_t s = (hipStream_t)stream;
    rs_options o{};
    if (opts) o = *opts;
    o.flags &= ~(uint32_t)RS_OPT_TIMING;
    // a first ordinary build: the sizes the caps start from (and the caller's first result)
    std::vector<rs_blob*> first(count, nullptr);
    std::vector<int> status(count, RS_OK);
    int rc = rs::build_batch_impl(sets, count, leaf, bucket, &o, s, first.data(), status.data(), nullptr);
    if (per_build_status)
        for (uint32_t c = 0; c < count; c++) per_build_status[c] = status[c];
    uint32_t maxm0 = 0;
    uint64_t words0 = 0;
    for (uint32_t c = 0; c < count; c++)
        if (first[c]) {
            maxm0 = std::max<uint32_t>(maxm0, (uint32_t)first[c]->header[6]);
            words0 += ((first[c]->bytes / 8) + 31) & ~uint64_t(31);
        }
    auto give_first = [&]() {
        for (uint32_t c = 0; c < count; c++) {
            if (first_outs) first_outs[c] = first[c];
            else if (first[c]) rs_blob_free(first[c]);
        }
    };
    if (rc != RS_OK) {
        give_first();
        return rc;
    }
    rs_plan* p = new (std::nothrow) rs_plan;
    if (!p) {
        give_first();
        return rs::fail(RS_ENOMEM, "host allocation failed");
    }
    p->sets.assign(sets, sets + count);
    p->leafs.assign(leaf, leaf + count);
    p->buckets.assign(bucket, bucket + count);
    p->opts = o;
    rs::Batch& b = p->b;
    auto bail = [&](int code) {
        rs::plan_release(p);
        give_first();
        return code;
    };
    if ((rc = rs::batch_prepare(b, sets, count, leaf, bucket, &o))) return bail(rc);
    if ((rc = rs::batch_layout(b))) return bail(rc);
    p->al = rs::current_alloc();
    if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess)
        return bail(rs::fail(RS_EDEVICE, "stream or event creation failed"));
    if ((rc = p->al.get((void**)&p->ws, b.ws_bytes, p->cap_stream))) return bail(rc);
    if (hipHostMalloc((void**)&p->pin, b.pin_bytes, hipHostMallocDefault) != hipSuccess) {
        p->pin = nullptr;
        return bail(rs::fail(RS_ENOMEM, "pinned host allocation failed"));
    }
    rs::batch_bind(b, p->ws, p->pin);
    // caps: the first build's largest bucket plus four standard deviations of a
    // Poisson count (and a few keys), within what the LDS holds; the arena 1/8 larger
    const uint32_t margin = (uint32_t)std::ceil(4.0 * std::sqrt((double)maxm0)) + 8;
    p->maxm_cap = std::min(maxm0 + margin, rs::lds_bucket_limit(b));
    if (p->maxm_cap < maxm0) return bail(rs::fail(RS_EINVAL, "largest bucket exceeds the local data share"));
    p->capacity = words0 + words0 / 8 + 64ull * b.K + 1024;
    if ((rc = rs::prepare_tables(b, p->maxm_cap)) ||
        (rc = p->al.get((void**)&b.d_tab, rs::table_words(b) * 4, p->cap_stream)) ||
        (rc = p->al.get((void**)&p->arena, p->capacity * 8, p->cap_stream)))
        return bail(rc);
    if ((rc = rs::upload_batch_tables(b, p->cap_stream, nullptr))) return bail(rc);
    if (hipStreamSynchronize(p->cap_stream) != hipSuccess) return bail(rs::fail(RS_EDEVICE, "table upload failed"));
    // capture: every phase, no host read in between
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(rs::fail(RS_EDEVICE, "hipStreamBeginCapture failed"));
    int crc = rs::enqueue_front(b, p->cap_stream, nullptr, nullptr);
    if (!crc) crc = rs::enqueue_back(b, p->cap_stream, nullptr);
    if (!crc) crc = rs::enqueue_fill(b, p->arena, p->capacity, p->capacity, p->cap_stream);
    if (!crc) crc = rs::enqueue_readback(b, p->cap_stream);
    const hipError_t ec = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (crc) return bail(crc);
    if (ec != hipSuccess || !p->graph) return bail(rs::fail(RS_EDEVICE, "hipStreamEndCapture failed"));
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(rs::fail(RS_EDEVICE, "hipGraphInstantiate failed"));
    give_first();
    *out = p;
    return RS_OK;
}

extern "C" int rs_plan_run(rs_plan* p, void* stream, rs_blob** outs, int* per_build_status) {
    rs::clear_error();
    if (!p || !outs) return rs::fail(RS_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    rs::Batch& b = p->b;
    // the previous run's copies read the arena: they finish before it is rewritten
    if (p->done_pending) RS_HIP(hipStreamWaitEvent(s, p->done, 0));
    // the descriptors going in are the plan's originals (a run rewrites the staging)
    memcpy(b.h_desc, b.hd.data(), b.K * sizeof(rs::BuildDesc));
    RS_HIP(hipGraphLaunch(p->exec, s));
    RS_HIP(hipStreamSynchronize(s));
    p->runs++;
    bool over = (b.h_st->flags & rs::kFlagCapacity) != 0;
    for (uint32_t j = 0; j < b.K; j++) over |= (b.h_desc[j].flags & rs::kFlagTooBig) != 0;
    if (over) {  // a bucket or a blob beyond the caps: build this run the ordinary way
        p->fallbacks++;
        p->done_pending = false;
        return rs::build_batch_impl(p->sets.data(), b.count, p->leafs.data(), p->buckets.data(), &p->opts, s, outs,
                                    per_build_status, nullptr);
    }
    // statuses start from validation, then the device flags of this run
    std::vector<int> st0 = b.st;
    std::vector<std::string> why0 = b.why;
    rs::collect_status(b);
    // copy the blobs (one contiguous range) and the tables out of the plan
    const uint64_t words = b.h_boff[b.K];
    uint64_t* dst = nullptr;
    uint32_t* tab = nullptr;
    const size_t tab_words = rs::table_words(b);
    int rc = RS_OK;
    if (words) {
        if ((rc = p->al.get((void**)&dst, words * 8, s)) || (rc = p->al.get((void**)&tab, tab_words * 4, s))) {
            p->al.put(dst, s);
            b.st = st0;
            b.why = why0;
            return rc;
        }
        RS_HIP(hipMemcpyAsync(dst, p->arena, words * 8, hipMemcpyDeviceToDevice, s));
        RS_HIP(hipMemcpyAsync(tab, b.d_tab, tab_words * 4, hipMemcpyDeviceToDevice, s));
        RS_HIP(hipEventRecord(p->done, s));
        p->done_pending = true;
    }
    rs::make_blobs(b, dst, tab, b.stride, p->al, s, outs);
    rc = rs::batch_finish(b, per_build_status, RS_OK);
    b.st = st0;
    b.why = why0;
    return rc;
}

extern "C" int rs_plan_info(const rs_plan* p, uint32_t* bucket_cap, uint64_t* capacity_words, uint64_t* runs,
                            uint64_t* fallbacks) {
    rs::clear_error();
    if (!p) return rs::fail(RS_EINVAL, "NULL argument");
    if (bucket_cap) *bucket_cap = p->maxm_cap;
    if (capacity_words) *capacity_words = p->capacity;
    if (runs) *runs = p->runs;
    if (fallbacks) *fallbacks = p->fallbacks;
    return RS_OK;
}

extern "C" void rs_plan_destroy(rs_plan* p) { rs::plan_release(p); }

namespace rs {

}  // namespace rs

extern "C" int rs_build_batch(const rs_keys* sets, uint32_t count, const uint32_t* leaf, const uint32_t* bucket,
                              const rs_options* opts, void* stream, rs_blob** outs, int* per_build_status) {
    rs::clear_error();
    return rs::build_batch_impl(sets, count, leaf, bucket, opts, (hipStream_t)stream, outs, per_build_status,
                                nullptr);
}

extern "C" int rs_build_ex(const rs_keys* keys, uint32_t leaf, uint32_t bucket, const rs_options* opts, void* stream,
                           rs_blob** out) {
    rs::clear_error();
    if (!keys || !out) return rs::fail(RS_EINVAL, "NULL argument");
    rs_blob* b = nullptr;
    int status = RS_OK;
    int rc = rs::build_batch_impl(keys, 1, &leaf, &bucket, opts, (hipStream_t)stream, &b, &status, nullptr);
    if (rc == RS_OK) *out = b;
    return rc;
}

extern "C" int rs_last_build_stats(rs_build_stats* out) {
    if (!out) return rs::fail(RS_EINVAL, "NULL argument");
    if (!rs::g_stats_valid) return rs::fail(RS_EINVAL, "no timed build on this thread");
    *out = rs::g_stats;
    return RS_OK;
}

extern "C" int rs_build(const rs_keys* keys, uint32_t leaf, uint32_t bucket, void* stream, rs_blob** out) {
    return rs_build_ex(keys, leaf, bucket, nullptr, stream, out);
}

// ---------------------------------------------------------------------------
// Construction without allocation (rs_build_noalloc), for callers that cannot
// allocate device memory.  The workspace and the per-size tables of the call
// live in one file-scope device array, `scratch`; host-side staging lives in
// static host buffers.  Each device holds its own copy of `scratch` from the
// time the library's code object is loaded on it until the process ends.
// Host code never uses the array's name as an address: its device address is
// taken once per device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
namespace rs {
namespace {
constexpr size_t kScratchBytes = 64ull << 20;  // workspace + tables of one call
constexpr uint32_t kScratchDevices = 64;
constexpr uint32_t kNoAllocMaxM = 16384;       // largest bucket (the search's LDS holds fewer keys)
}  // namespace
}  // namespace rs

static __device__ __align__(256) unsigned char scratch[rs::kScratchBytes];

namespace rs {
namespace {

std::mutex g_na_mu;  // one call at a time in this process: the host buffers below are shared
alignas(256) char g_na_host[1 << 14];  // descriptors in, sizes and status out
uint32_t g_na_tab[kTableCount * (kNoAllocMaxM + 1)];
void* g_na_scratch[kScratchDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (dev < 0 || (uint32_t)dev >= kScratchDevices) return fail(RS_EINVAL, "device %d out of range", dev);
    if (!g_na_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_na_scratch[dev] = p;
    }
    *out = g_na_scratch[dev];
    return RS_OK;
}

}  // namespace
}  // namespace rs

extern "C" int rs_build_noalloc(const rs_keys* keys, uint32_t leaf, uint32_t bucket, void* blob_dev,
                                uint64_t blob_cap, uint64_t* blob_bytes, void* stream) {
    using namespace rs;
    clear_error();
    if (!keys || !blob_bytes) return fail(RS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_na_mu);
    hipStream_t s = (hipStream_t)stream;
    char* base = nullptr;
    if (int rc = scratch_address((void**)&base)) return rc;
    Batch b;
    if (int rc = batch_prepare(b, keys, 1, &leaf, &bucket, nullptr)) return rc;
    if (b.K == 0) return batch_finish(b, nullptr, RS_OK);  // invalid arguments
    if (int rc = batch_layout(b)) return rc;
    const size_t ws_bytes = (b.ws_bytes + 255) & ~size_t(255);
    if (ws_bytes > kScratchBytes)
        return fail(RS_EINVAL, "%llu keys need %zu bytes of workspace; the allocation-free build holds %zu",
                    (unsigned long long)keys->n, ws_bytes, kScratchBytes);
    if (b.pin_bytes > sizeof g_na_host) return fail(RS_EINVAL, "host staging too small");
    b.samples = false;  // the caller's buffer holds the blob alone
    batch_bind(b, base, g_na_host);
    // front: signatures and bucket order, then the largest bucket
    if (int rc = enqueue_front(b, s, nullptr, nullptr)) return rc;
    RS_HIP(hipMemcpyAsync(b.h_st, b.d_st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    const uint32_t maxm = b.h_st->maxm;
    if (maxm > kNoAllocMaxM) return fail(RS_EINVAL, "largest bucket (%u keys) exceeds the local data share", maxm);
    // tables after the workspace, filled on the host without allocating
    b.table_maxm = maxm;
    b.stride = maxm + 1;
    const size_t tab_bytes = table_words(b) * 4;
    if (ws_bytes + tab_bytes > kScratchBytes)
        return fail(RS_EINVAL, "workspace and tables exceed the %zu bytes of the allocation-free build",
                    kScratchBytes);
    b.d_tab = reinterpret_cast<uint32_t*>(base + ws_bytes);
    fill_tables(leaf, maxm, g_na_tab);
    uint32_t max_nodes = 0;
    for (uint32_t m = 0; m <= maxm; m++) max_nodes = std::max(max_nodes, g_na_tab[2 * (maxm + 1) + m]);
    b.lds = (size_t)maxm * 8 + (size_t)max_nodes * 16;
    RS_HIP(hipMemcpyAsync(b.d_tab, g_na_tab, tab_bytes, hipMemcpyHostToDevice, s));
    // back: search, offsets, geometry; then the blob size
    if (int rc = enqueue_back(b, s, nullptr)) return rc;
    if (int rc = enqueue_readback(b, s)) return rc;
    RS_HIP(hipStreamSynchronize(s));
    collect_status(b);
    if (b.st[0] != RS_OK) return batch_finish(b, nullptr, RS_OK);
    const uint64_t raw = b.h_raw[0], rounded = b.h_boff[1];
    if (!blob_dev || blob_cap < raw * 8) {
        *blob_bytes = raw * 8;
        return fail(RS_EINVAL, "blob buffer of %llu bytes; the structure needs %llu", (unsigned long long)blob_cap,
                    (unsigned long long)(raw * 8));
    }
    // fill: the blob's own words are cleared and written (k_set_blobs sees the
    // rounded size as capacity; every write stays inside the first raw words)
    if (int rc = enqueue_fill(b, reinterpret_cast<uint64_t*>(blob_dev), rounded, raw, s)) return rc;
    RS_HIP(hipStreamSynchronize(s));
    *blob_bytes = raw * 8;
    return RS_OK;
}

namespace rs {
namespace {

// Calibration keys: distinct uniform random 64-bit words (the SplitMix64
// stream of a fixed seed).
__global__ void k_synth_keys(uint64_t* out, uint64_t n, uint64_t seed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = mix64(seed + (i + 1) * kGamma);
}

int tune_on_sample(uint32_t leaf, uint32_t bucket, uint64_t n, hipStream_t s, TuneCtx& t) {
    const Alloc al = current_alloc();
    uint64_t* keys = nullptr;
    if (int rc = al.get((void**)&keys, n * 8, s)) return rc;
    if (!grid_fits(grid_for(n, kBlock), kBlock)) {
        al.put(keys, s);
        return fail(RS_EINVAL, "calibration set too large");
    }
    k_synth_keys<<<(uint32_t)grid_for(n, kBlock), kBlock, 0, s>>>(keys, n, 0x5eed5eed5eed5eedull + leaf);
    if (hipGetLastError() != hipSuccess) {
        al.put(keys, s);
        return fail(RS_EDEVICE, "calibration key launch failed");
    }
    rs_keys k{RS_KEYS_U64, keys, nullptr, n};
    rs_blob* unused = nullptr;
    int status = RS_OK;
    int rc = build_batch_impl(&k, 1, &leaf, &bucket, nullptr, s, &unused, &status, &t);
    al.put(keys, s);
    return rc;
}

}  // namespace
}  // namespace rs

extern "C" int rs_autotune(uint32_t leaf, uint32_t bucket, uint64_t keys_hint, double budget_ms, void* stream,
                           rs_schedule* out) {
    rs::clear_error();
    if (leaf < 1 || leaf > rs::kMaxLeaf || bucket == 0) return rs::fail(RS_EINVAL, "l outside [1, 24] or b = 0");
    if (!(budget_ms > 0)) budget_ms = 3000.0;
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    constexpr uint64_t kMaxKeys = 1ull << 25;
    const uint64_t max_nb = std::max<uint64_t>(1, kMaxKeys / bucket);
    // buckets of the builds the schedule is for: the hint, else ten times the
    // workgroups resident at once (a steady state, like a large build)
    uint64_t nb_target = keys_hint ? (keys_hint + bucket - 1) / bucket : 0;
    uint64_t nb1 = nb_target ? std::min(nb_target, max_nb) : 0;
    rs::TuneCtx probe;
    if (nb1 == 0 || nb1 > 1024) {
        // probe: 1024 buckets with the built-in schedule (residency, time per round)
        const uint64_t nb0 = std::min<uint64_t>(1024, max_nb);
        probe.probe_only = true;
        if (int rc = rs::tune_on_sample(leaf, bucket, nb0 * bucket, s, probe)) return rc;
        const double resident = (double)std::max<uint64_t>(probe.resident, 1);
        const double ms_per_round = probe.default_ms / std::max(1.0, (double)nb0 / resident);
        if (!nb1) nb1 = std::min<uint64_t>((uint64_t)(10.0 * resident), max_nb);
        // about ten timed searches must fit the budget
        const double affordable = budget_ms / 10.0 / std::max(ms_per_round, 1e-3) * resident;
        if ((double)nb1 > affordable) nb1 = std::max<uint64_t>(nb0, (uint64_t)affordable);
    }
    rs::TuneCtx full;
    full.budget_ms = budget_ms;
    if (int rc = rs::tune_on_sample(leaf, bucket, nb1 * bucket, s, full)) return rc;
    rs_schedule best = full.best;
    best.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    rs::schedule_store(leaf, bucket, best);
    if (out) *out = best;
    return RS_OK;
}
