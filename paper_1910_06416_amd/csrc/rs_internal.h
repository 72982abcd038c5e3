// Internal declarations of librecsplit: format constants, the splitting
// strategy, host tables and the device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/recsplit.h"

namespace rs {

// ---------------------------------------------------------------------------
// Serialized format (little-endian 64-bit words).
//   word 0      magic "RSPLMPHF"
//   word 1      version | key kind << 32
//   words 2-6   n, leaf, bucket, nb, largest bucket size
//   word 7      Elias-Fano lower widths Ws | Wz << 8
//   words 8-10  delta_s, delta_z (two's complement), beta (16.16 fixed point)
//   words 11-15 upper-s words, upper-z words, lower words, tree words, tree bits
// followed by: interleaved lower bits, upper bits of s, upper bits of z, the
// two-level inventory (Sec. 7.4: for every 2^14-th one of each list its
// position as a 64-bit word, s and z interleaved; then for every 2^8-th one
// its distance from that anchor as a 16-bit entry, s and z interleaved, four
// entries per word, 0xffff when the distance does not fit), and the
// concatenated Golomb-Rice streams of all buckets (plus one zero guard word).
// ---------------------------------------------------------------------------
constexpr uint64_t kMagic = 0x4648504D4C505352ull;
constexpr uint64_t kVersion = 2;
constexpr int kHeaderWords = 16;
constexpr uint32_t kInvHi = 14;       // a 64-bit anchor for every 2^14-th one
constexpr uint32_t kInvLo = 8;        // a 16-bit offset for every 2^8-th one
constexpr uint32_t kInvOverflow = 0xffff;

// Words of the inventory of N entries per list: anchors, then packed offsets.
__host__ __device__ inline uint64_t inv_hi_words(uint64_t N) { return 2 * ((N + (1ull << kInvHi) - 1) >> kInvHi); }
__host__ __device__ inline uint64_t inv_lo_words(uint64_t N) {
    return (2 * ((N + (1ull << kInvLo) - 1) >> kInvLo) + 3) / 4;
}

// Select samples (not part of the serialized structure; kept by the library
// beside a blob it builds): the positions of every kSelectSample-th one of the
// two upper-bits arrays, as 32-bit words, s list then z list.  A lookup starts
// its selects there instead of at the two-level inventory, so it scans at
// most kSelectSample - 1 ones instead of up to 255.
constexpr uint32_t kSelectSample = 16;
__host__ __device__ inline uint64_t select_sample_groups(uint64_t N) { return (N + kSelectSample - 1) / kSelectSample; }
__host__ __device__ inline uint64_t select_samples_words(uint64_t N) { return select_sample_groups(N); }
// An upper-bits array of N entries spans fewer than 3 N bits, so its
// positions fit the 32-bit samples while 3 N < 2^32; a larger structure
// keeps none and its lookups start at the inventory.
__host__ __device__ inline bool select_samples_fit(uint64_t N) { return N <= 0xffffffffull / 3; }

constexpr uint64_t kDefaultSeedCap = 1ull << 56;
constexpr uint32_t kMaxLeaf = 24;

// Signature and hash-family constants.
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;  // SplitMix64 increment
constexpr uint64_t kMixA = 0xbf58476d1ce4e5b9ull;
constexpr uint64_t kMixB = 0x94d049bb133111ebull;
constexpr uint64_t kSigHi = 0x243f6a8885a308d3ull;
constexpr uint64_t kSigLo = 0x13198a2e03707344ull;

// Build flags set by the device: duplicate keys, seed cap reached, bad byte offsets,
// search scheduling failure, blob arena too small, bucket larger than the search was sized for.
enum : uint32_t {
    kFlagDuplicate = 1,
    kFlagSearch = 2,
    kFlagOffsets = 4,
    kFlagStack = 8,
    kFlagCapacity = 16,
    kFlagTooBig = 32
};

// Device-side status words of one build.
struct DevStatus {
    uint32_t maxm;
    uint32_t flags;
    unsigned long long delta_s;  // minimum gap of the prefix sums
    long long delta_z;           // minimum gap of z_i = o_i - floor(beta s_i)
    unsigned long long pad[5];
};

// Splitting strategy of Sec. 5: leaves of at most `leaf` keys, a first
// aggregation level of unit `leaf` up to `lower` keys, a second one of unit
// `lower` up to `upper` keys, and 2-way splits above.
struct Strategy {
    uint32_t leaf, lower, upper;
};
Strategy make_strategy(uint32_t leaf);

struct SplitShape {
    uint32_t unit, fanout, last;
};

__host__ __device__ inline SplitShape split_shape(uint32_t m, uint32_t leaf, uint32_t lower, uint32_t upper) {
    SplitShape s;
    if (m > upper) {
        s.unit = ((m / 2 + upper - 1) / upper) * upper;
        s.fanout = 2;
        s.last = m - s.unit;
        return s;
    }
    s.unit = m > lower ? lower : leaf;
    s.fanout = (m + s.unit - 1) / s.unit;
    s.last = m - (s.fanout - 1) * s.unit;
    return s;
}

// Non-minimal variant (the larger codomain that Sec. 9 proposes): a leaf of
// m >= 2 keys maps injectively into m + ceil(m slack / 256) values; slack = 0
// is the minimal structure.
__host__ __device__ inline uint32_t leaf_range(uint32_t m, uint32_t slack) {
    return m <= 1 ? m : m + (m * slack + 255u) / 256u;
}

// Per-size tables for sizes 0..cap (cap >= the requested maxm), laid out as
// r[cap+1], F[cap+1], N[cap+1], G[cap+1], P[cap+1], Q[cap+1], S[cap+1],
// C[cap+1]: Golomb-Rice parameter of a node, fixed bits of a subtree, coded
// nodes of a subtree, log2 of the lanes that share one candidate in the split
// search of a node of that size, r, N and F of the size packed into one word
// (footnote of Sec. 7.2: bits 0-4 r, 5-15 N, 16-31 F; kNoPacked where they do
// not fit), the number of output values of a subtree (m for the minimal
// structure; with slack, leaf_range for a leaf and the sum over the parts for
// a split), the split shape of a node (part size u in bits 0-15, fanout in
// bits 16-23; 0 for leaves and where u >= 2^16), and ceil(2^32 / u) (0 for
// u = 1 and leaves), with which floor(x / u) = umulhi(x, C) for x u < 2^32.
// The host memory is pinned and stays valid for the life of the process.
struct TableView {
    const uint32_t* data;
    uint32_t cap;
    const uint32_t* r() const { return data; }
    const uint32_t* F() const { return data + cap + 1; }
    const uint32_t* N() const { return data + 2 * (cap + 1); }
    const uint32_t* G() const { return data + 3 * (cap + 1); }
    const uint32_t* P() const { return data + 4 * (cap + 1); }
    const uint32_t* Q() const { return data + 5 * (cap + 1); }
    const uint32_t* S() const { return data + 6 * (cap + 1); }
    const uint32_t* C() const { return data + 7 * (cap + 1); }
};
constexpr int kTableCount = 8;
// G holds log2 lanes per split candidate in its low byte; kCoopFlag marks
// split sizes whose expected work (trials x keys) reaches kCoopEvals: their
// search is shared by the wavefronts of the bucket that are waiting.
constexpr uint32_t kGroupMask = 0xffu;
constexpr uint32_t kCoopFlag = 1u << 8;
constexpr double kCoopEvals = 524288.0;
constexpr uint32_t kNoPacked = 0xffffffffu;
__host__ __device__ inline uint32_t packed_r(uint32_t w) { return w & 31u; }
__host__ __device__ inline uint32_t packed_N(uint32_t w) { return (w >> 5) & 2047u; }
__host__ __device__ inline uint32_t packed_F(uint32_t w) { return w >> 16; }
// True if the packed words of sizes 0..maxm are all valid.
bool packed_valid(const uint32_t* P, uint32_t maxm);
// gr_max > 0: split nodes of more than gr_max keys take the integer
// approximation of their Golomb-Rice parameter (Sec. 7.2) instead of eq. (4).
// slack > 0: leaves map into leaf_range(m, slack) values, which changes their
// success probability (and so r) and the output ranges Q.
TableView host_tables(uint32_t leaf, uint32_t maxm, uint32_t gr_max = 0, uint32_t slack = 0);
// The same tables for sizes 0..maxm written into dst (kTableCount * (maxm + 1)
// words, in the order above), without any allocation.
void fill_tables(uint32_t leaf, uint32_t maxm, uint32_t* dst, uint32_t gr_max = 0, uint32_t slack = 0);
// True if the output range Q grows strictly with the size for 0..maxm (the
// lookup recovers a bucket's size from its range).
bool ranges_increasing(const uint32_t* Q, uint32_t maxm);
// Largest slack of the non-minimal variant: ranges stay below 2^32 and a
// leaf's values fit one 32-bit mask.
constexpr uint32_t kMaxSlack = 255;
constexpr uint32_t kMaxLeafRange = 32;

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------
// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * kMixA;
    z = (z ^ (z >> 27)) * kMixB;
    return z ^ (z >> 31);
}

// Upper 32 bits of mix64(z): the final xor-shift by 31 only moves bit 63 into
// the upper half, so the low product word of the last round is not needed.
__device__ __forceinline__ uint32_t mix64_hi32(uint64_t z) {
    z = (z ^ (z >> 30)) * kMixA;
    z = (z ^ (z >> 27)) * kMixB;
    uint32_t h = (uint32_t)(z >> 32);
    return h ^ (h >> 31);
}

// Position of hash function (depth d, index v) in the SplitMix64 stream of a key.
__device__ __forceinline__ uint64_t stream_offset(uint32_t depth, uint64_t v) {
    return (((uint64_t)depth << 56) | v) * kGamma;
}

// phi^m_{d,v}(x): fixed-point reduction of the upper 32 hash bits to [0, m).
__device__ __forceinline__ uint32_t phi(uint64_t x, uint32_t depth, uint64_t v, uint32_t m) {
    return __umulhi(mix64_hi32(x + stream_offset(depth, v)), m);
}

__device__ __forceinline__ void signature_u64(uint64_t key, uint64_t& hi, uint64_t& lo) {
    hi = mix64(key ^ kSigHi);
    lo = mix64(key ^ kSigLo);
}

// 8 bytes of a string starting at byte pos (bytes at or after `end` read as 0).
// Aligned word loads are used where both words lie inside the buffer.
__device__ __forceinline__ uint64_t string_word(const uint8_t* __restrict__ data, uint64_t total, bool aligned,
                                                uint64_t pos, uint64_t end) {
    uint64_t w = 0;
    uint64_t a = pos & ~7ull;
    if (aligned && a + 16 <= total) {
        const uint64_t* wp = reinterpret_cast<const uint64_t*>(data + a);
        uint64_t w0 = wp[0], w1 = wp[1];
        uint32_t sh = (uint32_t)(pos & 7) * 8;
        w = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
    } else {
        for (uint32_t k = 0; k < 8; k++)
            if (pos + k < end) w |= (uint64_t)data[pos + k] << (8 * k);
        return w;
    }
    uint64_t len = end - pos;
    if (len < 8) w &= (1ull << (8 * len)) - 1;
    return w;
}

// Byte-string signature: two chains over the little-endian 64-bit words of the
// string (the last one zero-padded), one absorbing by xor and one by addition,
// each followed by the mixer; both seeded with the length; mixed once more.
__device__ __forceinline__ void signature_bytes(const uint8_t* __restrict__ data, uint64_t total, bool aligned,
                                                uint64_t start, uint64_t end, uint64_t& hi, uint64_t& lo) {
    uint64_t len = end - start;
    uint64_t a = kSigHi ^ len, b = kSigLo ^ len;
    for (uint64_t pos = start; pos < end; pos += 8) {
        uint64_t w = string_word(data, total, aligned, pos, end);
        a = mix64(a ^ w);
        b = mix64(b + w);
    }
    hi = mix64(a);
    lo = mix64(b);
}

__device__ __forceinline__ uint64_t bucket_of(uint64_t hi, uint64_t nb) { return __umul64hi(hi, nb); }

}  // namespace rs
