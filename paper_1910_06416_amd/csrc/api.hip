// Blob management, lookup (Sec. 4 and 6.2-6.3 of the paper) and the error
// plumbing of librecsplit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "rs_host.h"
#include "rs_internal.h"

namespace rs {

namespace {
thread_local std::string g_error;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

namespace {
std::mutex g_alloc_mu;
Alloc g_alloc;
}  // namespace

Alloc current_alloc() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

int Alloc::get(void** p, size_t bytes, hipStream_t s) const {
    *p = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    if (alloc) {
        *p = alloc(bytes, (void*)s, ctx);
        return *p ? RS_OK : fail(RS_ENOMEM, "the caller's allocator returned no memory for %zu bytes", bytes);
    }
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? RS_ENOMEM : RS_EDEVICE, "device allocation of %zu bytes failed: %s",
                    bytes, hipGetErrorString(e));
    }
    return RS_OK;
}

void Alloc::put(void* p, hipStream_t s) const {
    if (!p) return;
    if (release) release(p, (void*)s, ctx);
    else (void)hipFreeAsync(p, s);
}

void Alloc::put_idle(void* p) const {
    if (!p) return;
    if (release) release(p, nullptr, ctx);
    else (void)hipFree(p);
}

Layout layout_of(const uint64_t* h) {
    Layout L;
    L.kind = h[1] >> 32;
    L.n = h[2]; L.leaf = h[3]; L.bucket = h[4]; L.nb = h[5]; L.maxm = h[6];
    L.Ws = (uint32_t)(h[7] & 0xff);
    L.Wz = (uint32_t)((h[7] >> 8) & 0xff);
    L.gr_max = (uint32_t)((h[7] >> 16) & 0xffffff);
    L.slack = (uint32_t)((h[7] >> 40) & 0xff);
    L.delta_s = h[8];
    L.delta_z = (int64_t)h[9];
    L.beta = h[10];
    L.us_words = h[11]; L.uz_words = h[12]; L.lower_words = h[13]; L.tree_words = h[14]; L.tree_bits = h[15];
    L.hi_words = inv_hi_words(L.nb + 1);
    L.lo_words = inv_lo_words(L.nb + 1);
    L.lower_off = kHeaderWords;
    L.us_off = L.lower_off + L.lower_words;
    L.uz_off = L.us_off + L.us_words;
    L.inv_hi_off = L.uz_off + L.uz_words;
    L.inv_lo_off = L.inv_hi_off + L.hi_words;
    L.tree_off = L.inv_lo_off + L.lo_words;
    L.total_words = L.tree_off + L.tree_words;
    return L;
}

int upload_tables(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack, uint32_t* dst, hipStream_t s) {
    TableView tv = host_tables(leaf, maxm, gr_max, slack);
    if (!tv.data) return fail(RS_ENOMEM, "table allocation failed");
    const size_t w = maxm + 1;
    for (int a = 0; a < kTableCount; a++)
        RS_HIP(hipMemcpyAsync(dst + a * w, tv.data + (size_t)a * (tv.cap + 1), w * 4, hipMemcpyHostToDevice, s));
    return RS_OK;
}

namespace {

// ---------------------------------------------------------------------------
// Lookup: one query per lane.
// ---------------------------------------------------------------------------
struct LookupArgs {
    const uint64_t* blob;
    const uint32_t* R;
    const uint32_t* F;
    const uint32_t* N;
    const uint32_t* P;  // r | N << 5 | F << 16 per size (used when every size fits)
    const uint32_t* Q;  // output values of a subtree per size (non-minimal structures)
    const uint32_t* S;  // split shape per size: part size | fanout << 16
    const uint32_t* C;  // ceil(2^32 / part size) per size
    const uint32_t* samples;  // select samples (null: start at the inventory)
    uint64_t nb, beta, delta_s;
    int64_t delta_z;
    uint32_t Ws, Wz;
    uint64_t lower_off, us_off, uz_off, inv_hi_off, inv_lo_off, tree_off;
    uint64_t us_words, uz_words, tree_words;
    uint32_t leaf, lower, upper, maxm, slack;
};

// Position of the k-th set bit (k = 0, 1, ...) inside a 64-bit word (k is
// less than the word's popcount): a binary search over halves of 32, 16, 8, 4,
// 2 and 1 bits, each step a popcount and a compare with no branch (the select
// runs once per lane in a wavefront whose lanes search different words).
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t k) {
    const uint32_t lo = (uint32_t)x;
    uint32_t c = (uint32_t)__popc(lo);
    const bool up = k >= c;
    uint32_t w = up ? (uint32_t)(x >> 32) : lo;
    k -= up ? c : 0;
    uint32_t pos = up ? 32 : 0;
#pragma unroll
    for (uint32_t half = 16; half >= 1; half >>= 1) {
        c = (uint32_t)__popc(w & ((1u << half) - 1));
        const bool hi = k >= c;
        k -= hi ? c : 0;
        w = hi ? w >> half : w;
        pos += hi ? half : 0;
    }
    return pos;
}

// Position of the k-th set bit at or after bit position p of an array of
// `words` words; a position past the end if there is no such bit (only in a
// corrupted structure).  Words after the first are read four at a time (the
// loads are independent, so a long scan costs one memory round trip per four
// words instead of one per word); the loop only finds the word, and the one
// in-word select runs after it.
__device__ __forceinline__ uint64_t select_from(const uint64_t* a, uint64_t words, uint64_t p, uint32_t k) {
    uint64_t w = p >> 6;
    if (w >= words) return words << 6;
    uint64_t x = a[w] & (~0ull << (p & 63));
    const uint32_t c = (uint32_t)__popcll(x);
    if (k >= c) {
        k -= c;
        for (w++;; w += 4) {
            if (w >= words) return words << 6;
            uint64_t y[4];
#pragma unroll
            for (int u = 0; u < 4; u++) y[u] = w + u < words ? a[w + u] : 0;
            const uint32_t s1 = (uint32_t)__popcll(y[0]), s2 = s1 + (uint32_t)__popcll(y[1]);
            const uint32_t s3 = s2 + (uint32_t)__popcll(y[2]), s4 = s3 + (uint32_t)__popcll(y[3]);
            if (k < s4) {  // in this group: pick the word without branches
                const bool b1 = k >= s1, b2 = k >= s2, b3 = k >= s3;
                x = b3 ? y[3] : b2 ? y[2] : b1 ? y[1] : y[0];
                k -= b3 ? s3 : b2 ? s2 : b1 ? s1 : 0;
                w += (uint32_t)b1 + b2 + b3;
                break;
            }
            k -= s4;
        }
    }
    return (w << 6) + select_in_word(x, k);
}

// select_from for a start at most a few dozen bits before the one sought (a
// select sample): the first two words are read together, and the scan goes
// on only if the one lies beyond them.
__device__ __forceinline__ uint64_t select_near(const uint64_t* a, uint64_t words, uint64_t p, uint32_t k) {
    const uint64_t w = p >> 6;
    if (w + 1 >= words) return select_from(a, words, p, k);
    const uint64_t x0 = a[w] & (~0ull << (p & 63)), x1 = a[w + 1];
    const uint32_t c0 = (uint32_t)__popcll(x0);
    if (k < c0) return (w << 6) + select_in_word(x0, k);
    const uint32_t c1 = (uint32_t)__popcll(x1);
    if (k - c0 < c1) return ((w + 1) << 6) + select_in_word(x1, k - c0);
    return select_from(a, words, (w + 2) << 6, k - c0 - c1);
}

// Position of the first set bit at or after bit p (the end of a unary code,
// or the next one of an Elias-Fano upper-bits array); a position past the end
// if there is none (only in a corrupted structure).
__device__ __forceinline__ uint64_t next_one(const uint64_t* a, uint64_t words, uint64_t p) {
    uint64_t w = p >> 6;
    if (w >= words) return words << 6;
    uint64_t x = a[w] & (~0ull << (p & 63));
    while (!x) {
        if (++w >= words) return words << 6;
        x = a[w];
    }
    return (w << 6) + (uint64_t)__builtin_ctzll(x);
}

// Positions of the k-th and the (k+1)-th set bits at or after bit p.
__device__ __forceinline__ void select_pair(const uint64_t* a, uint64_t words, uint64_t p, uint32_t k,
                                            uint64_t& first, uint64_t& second) {
    first = select_from(a, words, p, k);
    second = first < (words << 6) ? next_one(a, words, first + 1) : words << 6;
}

// floor(x / d) for 1 <= d and x < 2^21: the single-precision estimate
// x * rcp(d) is within 0.4 of x / d (relative error below 2^-22), so its
// truncation is off by at most one, which the remainder corrects.
__device__ __forceinline__ uint32_t div_small(uint32_t x, uint32_t d) {
    uint32_t q = (uint32_t)((float)x * __builtin_amdgcn_rcpf((float)d));
    const int32_t r = (int32_t)(x - q * d);
    if (r < 0)
        q--;
    else if ((uint32_t)r >= d)
        q++;
    return q;
}

// nbits < 64 bits at bit position pos.  Both words are always read, without
// a branch (lanes of a wavefront read at different offsets): every array read
// this way (the Elias-Fano lower bits, the Golomb-Rice streams) ends with a
// guard word.
__device__ __forceinline__ uint64_t get_bits(const uint64_t* a, uint64_t pos, uint32_t nbits) {
    const uint64_t w = pos >> 6;
    const uint32_t o = (uint32_t)(pos & 63);
    const uint64_t v = (a[w] >> o) | ((a[w + 1] << 1) << (63 - o));
    return v & ~(~0ull << nbits);
}

// Where to start looking for the i-th one of list 0 (s) or 1 (z): the
// recorded one nearest below it in the two-level inventory, and how many ones
// are left to skip from there (Sec. 7.4).
__device__ __forceinline__ void inventory_start(const uint64_t* blob, const LookupArgs& a, uint64_t i, uint32_t list,
                                                uint64_t& start, uint32_t& k) {
    start = blob[a.inv_hi_off + 2 * (i >> kInvHi) + list];
    const uint64_t e = 2 * (i >> kInvLo) + list;
    const uint32_t d = (uint32_t)(blob[a.inv_lo_off + e / 4] >> (16 * (e % 4))) & 0xffffu;
    const bool near = d != kInvOverflow;
    start += near ? d : 0;
    k = (uint32_t)i & (near ? (1u << kInvLo) - 1 : (1u << kInvHi) - 1);
}

// The words of a query's Golomb-Rice bucket stream, read once: kTreeWin words
// from the bucket's first one, loaded together into the lane's LDS slots (one
// memory round trip), so that the descent's dependent reads of fixed parts,
// unary codes and skipped codes mostly hit LDS.  Words outside the window
// are read from the structure.
constexpr uint32_t kLookupBlock = 256;
constexpr uint32_t kTreeWin = 8;
struct TreeWin {
    const uint64_t* g;  // the Golomb-Rice streams
    uint64_t words;     // their length in words (with the guard word)
    uint64_t* l;        // this lane's slots: l[k * kLookupBlock] holds word w0 + k
    uint64_t w0;
    __device__ __forceinline__ void load(uint64_t first) {
        w0 = first;
        uint64_t x[kTreeWin];
#pragma unroll
        for (uint32_t k = 0; k < kTreeWin; k++) x[k] = w0 + k < words ? g[w0 + k] : 0;
#pragma unroll
        for (uint32_t k = 0; k < kTreeWin; k++) l[k * kLookupBlock] = x[k];
    }
    __device__ __forceinline__ uint64_t word(uint64_t w) const {
        const uint64_t k = w - w0;
        return k < kTreeWin ? l[k * kLookupBlock] : g[w];
    }
    // as get_bits (the guard word keeps w + 1 inside the array)
    __device__ __forceinline__ uint64_t bits(uint64_t pos, uint32_t nbits) const {
        const uint64_t w = pos >> 6;
        const uint32_t o = (uint32_t)(pos & 63);
        const uint64_t v = (word(w) >> o) | ((word(w + 1) << 1) << (63 - o));
        return v & ~(~0ull << nbits);
    }
    // as next_one
    __device__ __forceinline__ uint64_t next_one(uint64_t p) const {
        uint64_t w = p >> 6;
        if (w >= words) return words << 6;
        uint64_t x = word(w) & (~0ull << (p & 63));
        while (!x) {
            if (++w >= words) return words << 6;
            x = word(w);
        }
        return (w << 6) + (uint64_t)__builtin_ctzll(x);
    }
    // as select_near: the first two words from the window, the rest by select_from
    __device__ __forceinline__ uint64_t select(uint64_t p, uint32_t k) const {
        const uint64_t w = p >> 6;
        if (w + 1 >= words) return select_from(g, words, p, k);
        const uint64_t x0 = word(w) & (~0ull << (p & 63)), x1 = word(w + 1);
        const uint32_t c0 = (uint32_t)__popcll(x0);
        if (k < c0) return (w << 6) + select_in_word(x0, k);
        const uint32_t c1 = (uint32_t)__popcll(x1);
        if (k - c0 < c1) return ((w + 1) << 6) + select_in_word(x1, k - c0);
        return select_from(g, words, (w + 2) << 6, k - c0 - c1);
    }
};

// Per-size table reads of the descent: one packed word per size (footnote of
// Sec. 7.2) when every size of the structure fits it, else three arrays.
template <bool PACKED>
struct SizeTables {
    const LookupArgs& a;
    __device__ uint32_t r(uint32_t m) const { return PACKED ? packed_r(a.P[m]) : a.R[m]; }
    __device__ uint32_t F(uint32_t m) const { return PACKED ? packed_F(a.P[m]) : a.F[m]; }
    // fixed bits and coded nodes of a subtree of size m, in one read when packed
    __device__ void FN(uint32_t m, uint32_t& f, uint32_t& n) const {
        if (PACKED) {
            const uint32_t w = a.P[m];
            f = packed_F(w);
            n = packed_N(w);
        } else {
            f = a.F[m];
            n = a.N[m];
        }
    }
};

// Rank (minimal structure) or output value (WIDE: the non-minimal variant,
// whose leaves map into leaf_range(m, slack) values and whose first
// Elias-Fano list holds prefix sums of bucket ranges) of one key.  TAB16:
// every node is below 2^16 keys (every structure this library builds), so
// split shapes come from the per-size table and child indices from one
// multiply with the part size's reciprocal (exact while ph * unit < 2^32).
template <bool PACKED, bool WIDE, bool TAB16>
__device__ uint64_t rank_of(const LookupArgs& a, uint64_t hi, uint64_t lo, uint64_t* win) {
    const SizeTables<PACKED> T{a};
    const uint64_t* blob = a.blob;
    const uint64_t i = bucket_of(hi, a.nb);
    // Elias-Fano: the i-th one of the upper bits is at (y_i >> W) + i.
    const uint64_t* us = blob + a.us_off;
    const uint64_t* uz = blob + a.uz_off;
    const uint64_t* lower = blob + a.lower_off;
    const uint32_t wsz = a.Ws + a.Wz;
    uint64_t start_s, start_z;
    uint32_t k_s, k_z;
    if (a.samples) {  // (the same for every lane)
        const uint64_t g = i / kSelectSample;
        start_s = a.samples[g];
        start_z = a.samples[select_sample_groups(a.nb + 1) + g];
        k_s = k_z = (uint32_t)(i % kSelectSample);
    } else {
        inventory_start(blob, a, i, 0, start_s, k_s);
        inventory_start(blob, a, i, 1, start_z, k_z);
    }
    uint64_t ps, ps1;
    if (a.samples) {
        ps = select_near(us, a.us_words, start_s, k_s);
        ps1 = ps < (a.us_words << 6) ? next_one(us, a.us_words, ps + 1) : a.us_words << 6;
    } else {
        select_pair(us, a.us_words, start_s, k_s, ps, ps1);
    }
    uint64_t ys = ((ps - i) << a.Ws) | get_bits(lower, i * wsz, a.Ws);
    uint64_t ys1 = ((ps1 - i - 1) << a.Ws) | get_bits(lower, (i + 1) * wsz, a.Ws);
    uint64_t s_i = ys + i * a.delta_s;
    uint64_t s_i1 = ys1 + (i + 1) * a.delta_s;
    uint64_t pz = a.samples ? select_near(uz, a.uz_words, start_z, k_z) : select_from(uz, a.uz_words, start_z, k_z);
    uint64_t yz = ((pz - i) << a.Wz) | get_bits(lower, i * wsz + a.Ws, a.Wz);
    int64_t z = (int64_t)yz + (int64_t)i * a.delta_z;
    uint64_t o_i = (uint64_t)(z + (int64_t)((a.beta * s_i) >> 16));

    uint32_t m = (uint32_t)min(s_i1 - s_i, (uint64_t)a.maxm);
    if (WIDE) {  // the bucket's size: the one whose range is s_{i+1} - s_i (ranges grow with the size)
        const uint64_t range = s_i1 - s_i;
        uint32_t lo_m = 0, hi_m = a.maxm;
        while (lo_m < hi_m) {
            const uint32_t mid = (lo_m + hi_m + 1) >> 1;
            if (a.Q[mid] <= range) lo_m = mid;
            else hi_m = mid - 1;
        }
        m = lo_m;
    }
    TreeWin tw{blob + a.tree_off, a.tree_words, win, 0};
    tw.load(o_i >> 6);
    // without the tables: node sizes below 2^20 take div_small (every
    // dividend is then under 2^21), larger ones integer division
    const bool small = a.maxm < (1u << 20);
    uint64_t c = 0;
    uint32_t d = 0;
    uint64_t fp = o_i, up = o_i + T.F(m);
    while (m > a.leaf) {
        uint32_t r = T.r(m);
        uint64_t fixed = tw.bits(fp, r);
        fp += r;
        uint64_t one = tw.next_one(up);
        uint64_t v = ((one - up) << r) | fixed;
        up = one + 1;
        SplitShape sh;
        if (TAB16) {
            const uint32_t sw = a.S[m];
            sh.unit = sw & 0xffffu;
            sh.fanout = sw >> 16;
            sh.last = m - (sh.fanout - 1) * sh.unit;
        } else if (small) {
            if (m > a.upper) {
                sh.unit = div_small(m / 2 + a.upper - 1, a.upper) * a.upper;
                sh.fanout = 2;
                sh.last = m - sh.unit;
            } else {
                sh.unit = m > a.lower ? a.lower : a.leaf;
                sh.fanout = div_small(m + sh.unit - 1, sh.unit);
                sh.last = m - (sh.fanout - 1) * sh.unit;
            }
        } else {
            sh = split_shape(m, a.leaf, a.lower, a.upper);
        }
        const uint32_t ph = phi(lo, d, v, m);
        uint32_t q;
        if (TAB16) {
            const uint32_t rc = a.C[m];
            q = rc ? __umulhi(ph, rc) : ph;  // the reciprocal is 0 for parts of one key
        } else {
            q = small ? div_small(ph, sh.unit) : ph / sh.unit;
        }
        const uint32_t j = min(q, sh.fanout - 1);
        if (j) {
            uint32_t fu, nu;
            T.FN(sh.unit, fu, nu);
            fp += (uint64_t)j * fu;
            const uint32_t skip = j * nu;
            if (skip) up = tw.select(up, skip - 1) + 1;
        }
        c += (uint64_t)j * (WIDE ? a.Q[sh.unit] : sh.unit);
        m = j + 1 == sh.fanout ? sh.last : sh.unit;
        d++;
    }
    if (m >= 2) {
        uint32_t r = T.r(m);
        uint64_t fixed = tw.bits(fp, r);
        uint64_t one = tw.next_one(up);
        uint64_t v = ((one - up) << r) | fixed;
        c += phi(lo, d, v, WIDE ? leaf_range(m, a.slack) : m);
    }
    return s_i + c;
}

// One query per lane; q0 is the launch's first query (lookups of more
// queries than one grid holds are launched in chunks).
template <bool PACKED, bool WIDE, bool TAB16>
__global__ void k_lookup_u64(LookupArgs a, const uint64_t* __restrict__ keys, uint64_t q, uint64_t q0,
                             uint64_t* __restrict__ ranks) {
    uint64_t t = q0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q) return;
    __shared__ uint64_t win[kTreeWin * kLookupBlock];
    uint64_t hi, lo;
    signature_u64(keys[t], hi, lo);
    ranks[t] = rank_of<PACKED, WIDE, TAB16>(a, hi, lo, win + threadIdx.x);
}

template <bool PACKED, bool WIDE, bool TAB16>
__global__ void k_lookup_bytes(LookupArgs a, const uint8_t* __restrict__ data, const uint64_t* __restrict__ offsets,
                               uint64_t q, uint64_t q0, bool aligned, uint64_t* __restrict__ ranks) {
    uint64_t t = q0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q) return;
    uint64_t total = offsets[q];
    uint64_t s = offsets[t], e = offsets[t + 1];
    if (e < s || e > total) e = s = min(s, total);
    uint64_t hi, lo;
    signature_bytes(data, total, aligned, s, e, hi, lo);
    __shared__ uint64_t win[kTreeWin * kLookupBlock];
    ranks[t] = rank_of<PACKED, WIDE, TAB16>(a, hi, lo, win + threadIdx.x);
}

// Select samples of a structure that came as bytes: one thread per group of
// kSelectSample entries finds their first one from the two-level inventory.
__global__ void k_select_samples(LookupArgs a, uint32_t* __restrict__ out, uint64_t groups) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    const uint64_t i = g * kSelectSample;
    uint64_t start;
    uint32_t k;
    inventory_start(a.blob, a, i, 0, start, k);
    out[g] = (uint32_t)select_from(a.blob + a.us_off, a.us_words, start, k);
    inventory_start(a.blob, a, i, 1, start, k);
    out[groups + g] = (uint32_t)select_from(a.blob + a.uz_off, a.uz_words, start, k);
}

LookupArgs lookup_args(const rs_blob* blob, const Layout& L) {
    const Strategy st = make_strategy((uint32_t)L.leaf);
    const uint32_t* tab = blob->tables;
    const size_t w = blob->tab_stride;
    return LookupArgs{blob->words, tab, tab + w, tab + 2 * w, tab + 4 * w, tab + 5 * w, tab + 6 * w, tab + 7 * w,
                      blob->samples, L.nb, L.beta, L.delta_s, L.delta_z, L.Ws, L.Wz, L.lower_off, L.us_off,
                      L.uz_off, L.inv_hi_off, L.inv_lo_off, L.tree_off, L.us_words, L.uz_words, L.tree_words,
                      (uint32_t)L.leaf, st.lower, st.upper, (uint32_t)L.maxm, L.slack};
}

}  // namespace

}  // namespace rs

using namespace rs;

extern "C" int rs_lookup(const rs_blob* blob, const rs_keys* queries, uint64_t* ranks_dev, void* stream) {
    clear_error();
    if (!blob || !queries || (!ranks_dev && queries->n)) return fail(RS_EINVAL, "NULL argument");
    if (queries->n == 0) return RS_OK;
    if (!queries->data) return fail(RS_EINVAL, "NULL query data");
    Layout L = layout_of(blob->header);
    if (queries->kind != L.kind) return fail(RS_EINVAL, "query kind %u differs from the blob's (%u)",
                                             queries->kind, (uint32_t)L.kind);
    if (queries->kind == RS_KEYS_BYTES && !queries->offsets) return fail(RS_EINVAL, "NULL offsets");
    const LookupArgs a = lookup_args(blob, L);
    hipStream_t s = (hipStream_t)stream;
    if (blob->ready) RS_HIP(hipStreamWaitEvent(s, blob->ready, 0));  // built on another stream
    const uint32_t block = kLookupBlock;
    const uint64_t q = queries->n;
    // one query per lane, in launches of at most max_grid_blocks() blocks
    if (int rc = for_each_chunk(q, block, block, [&](uint64_t q0, uint64_t, uint64_t grid) -> int {
            if (!grid_fits(grid, block))
                return fail(RS_EINVAL, "lookup grid of %llu blocks does not fit", (unsigned long long)grid);
            const bool al = ((uintptr_t)queries->data & 7) == 0;
            const uint8_t* bytes = (const uint8_t*)queries->data;
            const uint64_t* u64 = (const uint64_t*)bytes;
            const uint64_t* offs = queries->offsets;
            // table reads: packed words (the packed table only exists up to
            // 2600 keys, so with the shape tables), three arrays, or three
            // arrays and the ranges; shape tables below 2^16 keys
            const bool t16 = L.maxm < (1u << 16);
            const dim3 g((uint32_t)grid), b(block);
            if (queries->kind == RS_KEYS_U64) {
                if (blob->packed && !L.slack) k_lookup_u64<true, false, true><<<g, b, 0, s>>>(a, u64, q, q0, ranks_dev);
                else if (L.slack && t16) k_lookup_u64<false, true, true><<<g, b, 0, s>>>(a, u64, q, q0, ranks_dev);
                else if (L.slack) k_lookup_u64<false, true, false><<<g, b, 0, s>>>(a, u64, q, q0, ranks_dev);
                else if (t16) k_lookup_u64<false, false, true><<<g, b, 0, s>>>(a, u64, q, q0, ranks_dev);
                else k_lookup_u64<false, false, false><<<g, b, 0, s>>>(a, u64, q, q0, ranks_dev);
            } else {
                if (blob->packed && !L.slack)
                    k_lookup_bytes<true, false, true><<<g, b, 0, s>>>(a, bytes, offs, q, q0, al, ranks_dev);
                else if (L.slack && t16)
                    k_lookup_bytes<false, true, true><<<g, b, 0, s>>>(a, bytes, offs, q, q0, al, ranks_dev);
                else if (L.slack)
                    k_lookup_bytes<false, true, false><<<g, b, 0, s>>>(a, bytes, offs, q, q0, al, ranks_dev);
                else if (t16)
                    k_lookup_bytes<false, false, true><<<g, b, 0, s>>>(a, bytes, offs, q, q0, al, ranks_dev);
                else
                    k_lookup_bytes<false, false, false><<<g, b, 0, s>>>(a, bytes, offs, q, q0, al, ranks_dev);
            }
            return RS_OK;
        }))
        return rc;
    RS_HIP(hipGetLastError());
    return RS_OK;
}

extern "C" uint64_t rs_blob_bytes(const rs_blob* blob) { return blob ? blob->bytes : 0; }

extern "C" const void* rs_blob_device_ptr(const rs_blob* blob) { return blob ? blob->words : nullptr; }

extern "C" int rs_blob_info(const rs_blob* blob, uint64_t* n, uint32_t* leaf, uint32_t* bucket) {
    if (!blob) return fail(RS_EINVAL, "NULL blob");
    if (n) *n = blob->header[2];
    if (leaf) *leaf = (uint32_t)blob->header[3];
    if (bucket) *bucket = (uint32_t)blob->header[4];
    return RS_OK;
}

extern "C" int rs_blob_to_host(const rs_blob* blob, void* dst, uint64_t cap) {
    clear_error();
    if (!blob || !dst) return fail(RS_EINVAL, "NULL argument");
    if (cap < blob->bytes) return fail(RS_EINVAL, "buffer of %llu bytes is smaller than the blob (%llu)",
                                       (unsigned long long)cap, (unsigned long long)blob->bytes);
    if (blob->ready) RS_HIP(hipEventSynchronize(blob->ready));
    RS_HIP(hipMemcpy(dst, blob->words, blob->bytes, hipMemcpyDeviceToHost));
    return RS_OK;
}

extern "C" int rs_blob_from_host(const void* src, uint64_t bytes, void* stream, rs_blob** out) {
    clear_error();
    if (!src || !out) return fail(RS_EINVAL, "NULL argument");
    if (bytes < kHeaderWords * 8 || bytes % 8) return fail(RS_EFORMAT, "blob too short");
    const uint64_t* h = (const uint64_t*)src;
    if (h[0] != kMagic || (h[1] & 0xffffffffull) != kVersion) return fail(RS_EFORMAT, "bad magic or version");
    Layout L = layout_of(h);
    if (L.leaf < 1 || L.leaf > kMaxLeaf || L.nb == 0 || L.n == 0 || L.maxm > L.n ||
        (L.kind != RS_KEYS_U64 && L.kind != RS_KEYS_BYTES) || L.total_words * 8 != bytes ||
        leaf_range((uint32_t)L.leaf, L.slack) > kMaxLeafRange || (h[7] >> 48) != 0)
        return fail(RS_EFORMAT, "inconsistent header");
    if (L.slack) {
        const TableView tv = host_tables((uint32_t)L.leaf, (uint32_t)L.maxm, L.gr_max, L.slack);
        if (!tv.data) return fail(RS_ENOMEM, "table allocation failed");
        if (!ranges_increasing(tv.Q(), (uint32_t)L.maxm)) return fail(RS_EFORMAT, "inconsistent header");
    }
    hipStream_t s = (hipStream_t)stream;
    rs_blob* b = new (std::nothrow) rs_blob;
    if (!b) return fail(RS_ENOMEM, "host allocation failed");
    memcpy(b->header, h, sizeof b->header);
    b->al = current_alloc();
    // the structure, then (from a 256-byte boundary) its select samples
    const bool with_samples = select_samples_fit(L.nb + 1);
    const uint64_t smp_off = (bytes / 8 + 31) & ~uint64_t(31), smp_groups = select_sample_groups(L.nb + 1);
    const uint64_t words = with_samples ? smp_off + select_samples_words(L.nb + 1) : bytes / 8;
    int rc = b->al.get((void**)&b->words, words * 8, s);
    if (!rc) rc = b->al.get((void**)&b->tables, (size_t)kTableCount * (L.maxm + 1) * 4, s);
    if (!rc) rc = upload_tables((uint32_t)L.leaf, (uint32_t)L.maxm, L.gr_max, L.slack, b->tables, s);
    if (!rc && hipMemcpyAsync(b->words, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fail(RS_EDEVICE, "copy to device failed");
    b->tab_stride = (uint32_t)(L.maxm + 1);
    if (!rc && with_samples) {
        uint32_t* smp = reinterpret_cast<uint32_t*>(b->words + smp_off);
        const uint64_t grid = (smp_groups + 255) / 256;
        if (!grid_fits(grid, 256)) {
            rc = fail(RS_EINVAL, "select-sample grid of %llu blocks does not fit", (unsigned long long)grid);
        } else {
            k_select_samples<<<dim3((uint32_t)grid), dim3(256), 0, s>>>(lookup_args(b, L), smp, smp_groups);
            if (hipGetLastError() != hipSuccess) rc = fail(RS_EDEVICE, "select-sample launch failed");
            else b->samples = smp;
        }
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(RS_EDEVICE, "stream synchronisation failed");
    if (rc) {
        b->al.put(b->words, s);
        b->al.put(b->tables, s);
        delete b;
        return rc;
    }
    b->bytes = bytes;
    {
        const TableView tv = host_tables((uint32_t)L.leaf, (uint32_t)L.maxm, L.gr_max, L.slack);
        b->packed = !L.slack && tv.data && packed_valid(tv.P(), (uint32_t)L.maxm);
    }
    b->ready = nullptr;  // complete: the copy above was waited for
    (void)hipGetDevice(&b->device);
    *out = b;
    return RS_OK;
}

extern "C" void rs_blob_free(rs_blob* blob) {
    if (!blob) return;
    if (blob->arena) {
        release_arena(blob->arena);
    } else {
        blob->al.put_idle(blob->words);
        blob->al.put_idle(blob->tables);
    }
    delete blob;
}

extern "C" int rs_set_allocator(rs_alloc_fn alloc, rs_free_fn release, void* ctx) {
    clear_error();
    if ((alloc == nullptr) != (release == nullptr))
        return fail(RS_EINVAL, "set both the allocation and the release function, or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.release = release;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return RS_OK;
}

extern "C" const char* rs_last_error(void) { return g_error.c_str(); }

extern "C" const char* rs_version(void) { return "librecsplit 0.1 (gfx950)"; }
