/*
 * RecSplit CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded, obviously-correct implementation of the
 * RecSplit construction and lookup (Esposito, Mueller Graf, Vigna,
 * "RecSplit: Minimal Perfect Hashing via Recursive Splitting", 2019).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * constant generator with the GPU library: every formula below is written
 * from the paper (section / equation cited at each function) and from the
 * bit-level format readings listed with the design notes.
 *
 * Pins (checked by the CPU test-suite, not by re-typing these formulas):
 *   mixer            published SplitMix64 outputs (Steele, Lea, Flood 2014)
 *   string keys      length folded in; one flipped bit changes about half
 *                    of both signature words (avalanche)
 *   buckets          chi-square against Binomial(n, 1/nb)         (Sec. 5);
 *                    ids monotone in the upper word, each bucket starting at
 *                    ceil(j 2^64 / nb)                           (Sec. 6.1)
 *   search           minimality by brute force; mean trials per
 *                    leaf/split size against m^m/m! and 1/p of eq. (2)
 *   strategy + r     Theorem 1 (invariance) and 50-digit evaluation of eq. (4)
 *   whole structure  lookup of every key is a permutation of [0,n)
 *   space            bits/key against the values printed in Table tab:1M
 *   inventory        every one found through it equals a plain scan, also
 *                    with 16-bit offsets that overflow       (Sec. 7.4)
 *   Elias-Fano       rescaling constants are the decoded lists' minimum
 *                    gaps; lower widths floor(lg(U/N)), also on the power-of-
 *                    two boundary; nb + 1 upper ones, all below bit 3 (nb + 1)
 *                                                      (Sec. 6.3, Sec. 7.4)
 * A separate test plants plausible mistakes in a copy of this file and checks
 * that each makes one of these pins fail.
 * Exact seeds and blob bytes beyond that are "parity unpinned" by the paper
 * (its worked examples, Figs. 1-2, are not available); they are defined by
 * this file and the format readings.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EDUPLICATE = 2, ORC_ENOMEM = 3, ORC_ESEARCH = 5, ORC_EFORMAT = 6 };
enum { ORC_KEYS_U64 = 1, ORC_KEYS_BYTES = 2 };

#define ORC_MAGIC 0x4648504D4C505352ULL /* "RSPLMPHF" little-endian */
#define ORC_VERSION 2ULL
#define ORC_HEADER_WORDS 16
#define ORC_MAX_FANOUT 16
#define ORC_INV_HI 14 /* a 64-bit anchor for every 2^14-th one (Sec. 7.4) */
#define ORC_INV_LO 8  /* a 16-bit offset from it for every 2^8-th one */
#define ORC_INV_OVERFLOW 0xffffu
#define ORC_DEFAULT_SEED_CAP (1ULL << 56)

/* ------------------------------------------------------------------------ */
/* Mixer: the SplitMix64 output function (Steele, Lea, Flood, "Fast          */
/* splittable pseudorandom number generators", OOPSLA 2014): two xor-shift / */
/* multiply rounds and a final xor-shift.  Bijective on 64-bit words.       */
/* ------------------------------------------------------------------------ */
static const uint64_t GAMMA = 0x9e3779b97f4a7c15ULL; /* SplitMix64 increment */

static uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* The SplitMix64 generator itself (state += GAMMA; output mix(state)), used
 * only to pin the mixer to published output values. */
void orc_splitmix64_stream(uint64_t seed, uint64_t count, uint64_t* out) {
    uint64_t state = seed;
    for (uint64_t i = 0; i < count; i++) {
        state += GAMMA;
        out[i] = mix(state);
    }
}

/* ------------------------------------------------------------------------ */
/* Signatures (Sec. 6.1: every key becomes a 128-bit signature; the upper 64  */
/* bits pick the bucket, the lower 64 bits drive the searches, Sec. 7.3).    */
/* ------------------------------------------------------------------------ */
static const uint64_t FP_HI = 0x243f6a8885a308d3ULL;
static const uint64_t FP_LO = 0x13198a2e03707344ULL;

/* u64 keys: two bijective images of the key, so distinct keys always give
 * distinct (and within a bucket distinct lower) signature words. */
void orc_fingerprint_u64(const uint64_t* keys, uint64_t n, uint64_t* hi, uint64_t* lo) {
    for (uint64_t i = 0; i < n; i++) {
        hi[i] = mix(keys[i] ^ FP_HI);
        lo[i] = mix(keys[i] ^ FP_LO);
    }
}

/* Byte-string keys: the string is read as little-endian 64-bit words (the
 * last one zero-padded); two chains absorb the words, one by xor and one by
 * addition, each chain state is mixed after every word; the length seeds both
 * chains and a final mix finishes each half. */
static void fingerprint_bytes_one(const uint8_t* p, uint64_t len, uint64_t* hi, uint64_t* lo) {
    uint64_t a = FP_HI ^ len, b = FP_LO ^ len;
    uint64_t nwords = (len + 7) / 8;
    for (uint64_t w = 0; w < nwords; w++) {
        uint64_t word = 0;
        for (uint64_t k = 0; k < 8; k++) {
            uint64_t pos = w * 8 + k;
            if (pos < len) word |= (uint64_t)p[pos] << (8 * k);
        }
        a = mix(a ^ word);
        b = mix(b + word);
    }
    *hi = mix(a);
    *lo = mix(b);
}

void orc_fingerprint_bytes(const uint8_t* data, const uint64_t* offsets, uint64_t n, uint64_t* hi, uint64_t* lo) {
    for (uint64_t i = 0; i < n; i++)
        fingerprint_bytes_one(data + offsets[i], offsets[i + 1] - offsets[i], &hi[i], &lo[i]);
}

/* Bucket of a signature (Sec. 6.1): floor(u * nb / 2^64), a fixed-point
 * multiplication of the upper signature word by the bucket count. */
static uint64_t bucket_of(uint64_t hi, uint64_t nb) {
    return (uint64_t)(((unsigned __int128)hi * nb) >> 64);
}

/* ------------------------------------------------------------------------ */
/* Hash family phi^m_{d,v} (Sec. 4 and 6.1): the v-th function used at tree   */
/* depth d maps a lower signature word x to [0, m) by fixed-point            */
/* multiplication of the upper 32 bits of mix(x + I * GAMMA) by m, where      */
/* I = d * 2^56 + v is the function's position in the SplitMix64 stream      */
/* seeded with x.  Different depths never share a position, so no function   */
/* is reused along a root-to-leaf path (Sec. 7.3).                           */
/* ------------------------------------------------------------------------ */
uint32_t orc_phi(uint64_t x, uint32_t depth, uint64_t v, uint32_t m) {
    uint64_t index = ((uint64_t)depth << 56) | v;
    uint64_t h = mix(x + index * GAMMA);
    return (uint32_t)(((h >> 32) * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Splitting strategy (Sec. 4 and "A splitting strategy" in Sec. 5).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t leaf, lower, upper;
    uint32_t slack; /* non-minimal variant: leaves of m >= 2 keys map into m + ceil(m slack / 256) values */
} strategy;

static strategy make_strategy(uint32_t leaf) {
    strategy st;
    st.slack = 0;
    /* s = max(2, ceil(0.35 l + 0.5)) and t = ceil(0.21 l + 0.9) (2 for l < 7),
     * written over the integers as ceil((35 l + 50)/100), ceil((21 l + 90)/100). */
    uint32_t s = (35 * leaf + 50 + 99) / 100;
    if (s < 2) s = 2;
    uint32_t t = leaf < 7 ? 2 : (21 * leaf + 90 + 99) / 100;
    st.leaf = leaf;
    st.lower = s * leaf;
    st.upper = s * t * leaf;
    return st;
}

/* Parts of a node of size m > leaf: all equal to the unit u except possibly
 * the last.  Above the second aggregation level the split is 2-way with left
 * part ceil(floor(m/2) / upper) * upper.  Returns the fanout. */
static uint32_t split_parts(const strategy* st, uint32_t m, uint32_t* parts, uint32_t* unit) {
    uint32_t u;
    if (m > st->upper) {
        u = ((m / 2 + st->upper - 1) / st->upper) * st->upper;
        parts[0] = u;
        parts[1] = m - u;
        *unit = u;
        return 2;
    }
    u = m > st->lower ? st->lower : st->leaf;
    uint32_t f = (m + u - 1) / u;
    for (uint32_t j = 0; j + 1 < f; j++) parts[j] = u;
    parts[f - 1] = m - (f - 1) * u;
    *unit = u;
    return f;
}

/* Non-minimal variant (the extension Sec. 9 names: a larger codomain).  A
 * leaf of m >= 2 keys searches the first index whose hash is injective into
 * leaf_range(m) = m + ceil(m slack / 256) values, and a subtree of m keys
 * covers range(m) output values: 1 for a single key, leaf_range(m) for a
 * leaf, the sum over the parts for a split.  slack = 0 is the minimal
 * structure (range(m) = m). */
static uint32_t leaf_range(const strategy* st, uint32_t m) {
    return m <= 1 ? m : m + (m * st->slack + 255) / 256;
}

static uint32_t split_parts(const strategy* st, uint32_t m, uint32_t* parts, uint32_t* unit);

static uint64_t subtree_range(const strategy* st, uint32_t m) {
    if (m <= st->leaf) return leaf_range(st, m);
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    uint64_t r = 0;
    for (uint32_t j = 0; j < f; j++) r += subtree_range(st, parts[j]);
    return r;
}

/* Child of a hash value: the part whose range [j u, (j+1) u) holds it; the
 * last part takes everything from (f-1) u on. */
static uint32_t child_of(uint32_t phi, uint32_t unit, uint32_t fanout) {
    uint32_t j = phi / unit;
    return j < fanout - 1 ? j : fanout - 1;
}

/* ------------------------------------------------------------------------ */
/* Golomb-Rice parameters (eq. (4)) and per-size subtree tables.             */
/* ------------------------------------------------------------------------ */
static double ln_factorial(uint32_t m) {
    double s = 0.0;
    for (uint32_t j = 2; j <= m; j++) s += log((double)j);
    return s;
}

/* ln of the success probability of a node: m!/m^m for a leaf (Sec. 5,
 * bijections); (m!/m^m) prod_j k_j^{k_j}/k_j! for a split (eq. (2)). */
static double ln_success(const strategy* st, uint32_t m) {
    if (m <= st->leaf && st->slack) {
        /* injective into M = leaf_range(m) values: prod_{i<m} (M - i) / M */
        double M = (double)leaf_range(st, m), lq = 0.0;
        for (uint32_t i = 0; i < m; i++) lq += log((M - (double)i) / M);
        return lq;
    }
    double lp = ln_factorial(m) - (double)m * log((double)m);
    if (m <= st->leaf) return lp;
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    for (uint32_t j = 0; j < f; j++) lp += (double)parts[j] * log((double)parts[j]) - ln_factorial(parts[j]);
    return lp;
}

/* r(p) = max{0, ceil(lg(-lg(golden) / lg(1-p)))}  (eq. (4)). */
static uint32_t golomb_rice_param(double p) {
    double golden = (1.0 + sqrt(5.0)) / 2.0;
    double ratio = log(golden) / -log1p(-p);
    double x = ceil(log2(ratio));
    return x > 0.0 ? (uint32_t)x : 0;
}

/* lambda(x): the index of the highest set bit of x >= 1, i.e. floor(lg x)
 * (Sec. 2). */
static uint32_t lambda_of(uint64_t x) {
    uint32_t l = 0;
    while (x > 1) {
        x >>= 1;
        l++;
    }
    return l;
}

/* The paper's integer approximation of the Golomb-Rice parameter of a split
 * of m keys into parts k_0..k_{s-1}, for large buckets (Sec. 7.2):
 *   ( ((s-1) * 5 >> 1) + sum_i lambda(k_i + (k_i >> 1)) - lambda(m) ) >> 1,
 * where lambda(x + (x >> 1)) is the integer rounding of lg x of Sec. 7.1.  A
 * negative value (none occurs for the strategy's splits) reads as 0. */
static uint32_t gr_param_approx(const strategy* st, uint32_t m) {
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    int64_t acc = (int64_t)(((f - 1) * 5) >> 1) - (int64_t)lambda_of(m);
    for (uint32_t j = 0; j < f; j++) acc += lambda_of((uint64_t)parts[j] + (parts[j] >> 1));
    return acc > 0 ? (uint32_t)(acc >> 1) : 0;
}

uint32_t orc_lambda(uint64_t x) { return x ? lambda_of(x) : 0; }

uint32_t orc_gr_param_approx(uint32_t leaf, uint32_t m) {
    strategy st = make_strategy(leaf);
    return m > leaf ? gr_param_approx(&st, m) : 0;
}

double orc_ln_success(uint32_t leaf, uint32_t m) {
    strategy st = make_strategy(leaf);
    return ln_success(&st, m);
}

/* Per-size tables for sizes 0..maxm: r (GR parameter of the node itself, 0
 * for uncoded nodes), F (fixed bits of the whole subtree) and N (coded nodes
 * in the subtree).  Leaves of size 0 or 1 carry no index (Fig. 1 caption).
 * r follows eq. (4) for every leaf and for splits of at most gr_max keys;
 * splits of more than gr_max keys take the integer approximation of Sec. 7.2
 * (gr_max = 0: eq. (4) everywhere). */
static int tables_impl(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack, uint32_t* r, uint32_t* F,
                       uint32_t* N) {
    if (leaf < 1 || leaf > 24) return ORC_EINVAL;
    strategy st = make_strategy(leaf);
    st.slack = slack;
    for (uint32_t m = 0; m <= maxm; m++) {
        if (m <= 1) {
            r[m] = 0; F[m] = 0; N[m] = 0;
            continue;
        }
        if (gr_max && m > leaf && m > gr_max) r[m] = gr_param_approx(&st, m);
        else r[m] = golomb_rice_param(exp(ln_success(&st, m)));
        F[m] = r[m];
        N[m] = 1;
        if (m > leaf) {
            uint32_t parts[ORC_MAX_FANOUT], unit;
            uint32_t f = split_parts(&st, m, parts, &unit);
            for (uint32_t j = 0; j < f; j++) {
                F[m] += F[parts[j]];
                N[m] += N[parts[j]];
            }
        }
    }
    return ORC_OK;
}

int orc_tables_ex(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t* r, uint32_t* F, uint32_t* N) {
    return tables_impl(leaf, maxm, gr_max, 0, r, F, N);
}

int orc_tables(uint32_t leaf, uint32_t maxm, uint32_t* r, uint32_t* F, uint32_t* N) {
    return orc_tables_ex(leaf, maxm, 0, r, F, N);
}

/* Tables of the non-minimal variant: r, F, N as orc_tables_ex (leaf r from the
 * probability of an injection), and the output range Q[m] of a subtree. */
int orc_tables_slack(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack, uint32_t* r, uint32_t* F,
                     uint32_t* N, uint64_t* Q) {
    int rc = tables_impl(leaf, maxm, gr_max, slack, r, F, N);
    if (rc) return rc;
    strategy st = make_strategy(leaf);
    st.slack = slack;
    for (uint32_t m = 0; m <= maxm; m++) Q[m] = subtree_range(&st, m);
    return ORC_OK;
}

/* The per-size tables in one 32-bit word per size (footnote of Sec. 7.2):
 * bits 0-4 hold r, bits 5-15 the coded nodes N of the subtree and bits 16-31
 * its fixed bits F.  ORC_EINVAL if some size up to maxm does not fit (the
 * paper states that one such table suffices for l >= 4 and b <= 2000). */
int orc_packed_table(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t* out) {
    uint32_t* r = malloc((maxm + 1) * 4);
    uint32_t* F = malloc((maxm + 1) * 4);
    uint32_t* N = malloc((maxm + 1) * 4);
    int rc = ORC_ENOMEM;
    if (r && F && N) rc = orc_tables_ex(leaf, maxm, gr_max, r, F, N);
    for (uint32_t m = 0; rc == ORC_OK && m <= maxm; m++) {
        if (r[m] >= 32 || N[m] >= 2048 || F[m] >= 65536) rc = ORC_EINVAL;
        else out[m] = r[m] | (N[m] << 5) | (F[m] << 16);
    }
    free(r); free(F); free(N);
    return rc;
}

void orc_strategy(uint32_t leaf, uint32_t* lower, uint32_t* upper) {
    strategy st = make_strategy(leaf);
    *lower = st.lower;
    *upper = st.upper;
}

uint32_t orc_split_parts(uint32_t leaf, uint32_t m, uint32_t* parts) {
    strategy st = make_strategy(leaf);
    uint32_t unit;
    if (m <= leaf) return 0;
    return split_parts(&st, m, parts, &unit);
}

/* ------------------------------------------------------------------------ */
/* Searches (Sec. 4): the FIRST index v = 0, 1, 2, ... that works.            */
/* ------------------------------------------------------------------------ */
/* The first v whose hash into cod values (cod = m for a bijection, more for
 * the non-minimal variant; cod <= 64) is injective on the leaf's keys. */
static int search_leaf(const uint64_t* keys, uint32_t m, uint32_t cod, uint32_t depth, uint64_t cap, uint64_t* out) {
    for (uint64_t v = 0; v < cap; v++) {
        uint64_t seen = 0;
        int ok = 1;
        for (uint32_t i = 0; i < m; i++) {
            uint32_t phi = orc_phi(keys[i], depth, v, cod);
            if (seen & (1ULL << phi)) {
                ok = 0;
                break;
            }
            seen |= 1ULL << phi;
        }
        if (ok) {
            *out = v;
            return ORC_OK;
        }
    }
    return ORC_ESEARCH;
}

static int search_split(const uint64_t* keys, uint32_t m, uint32_t depth, const uint32_t* parts, uint32_t f,
                        uint32_t unit, uint64_t cap, uint64_t* out) {
    for (uint64_t v = 0; v < cap; v++) {
        uint32_t count[ORC_MAX_FANOUT] = {0};
        for (uint32_t i = 0; i < m; i++) count[child_of(orc_phi(keys[i], depth, v, m), unit, f)]++;
        int ok = 1;
        for (uint32_t j = 0; j < f; j++) ok &= count[j] == parts[j];
        if (ok) {
            *out = v;
            return ORC_OK;
        }
    }
    return ORC_ESEARCH;
}

/* Recursive construction of one splitting tree: indices are emitted in
 * preorder together with the node size and depth. keys[] is permuted. */
typedef struct {
    uint64_t* v;
    uint32_t* m;
    uint32_t* d;
    uint64_t count;
    uint64_t cap;
    uint64_t* tmp;
} emitter;

static int build_tree(const strategy* st, uint64_t* keys, uint32_t m, uint32_t depth, emitter* e) {
    if (m <= 1) return ORC_OK;
    uint64_t v;
    int rc;
    if (m <= st->leaf) {
        rc = search_leaf(keys, m, leaf_range(st, m), depth, e->cap, &v);
        if (rc) return rc;
        e->v[e->count] = v; e->m[e->count] = m; e->d[e->count] = depth; e->count++;
        return ORC_OK;
    }
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    rc = search_split(keys, m, depth, parts, f, unit, e->cap, &v);
    if (rc) return rc;
    e->v[e->count] = v; e->m[e->count] = m; e->d[e->count] = depth; e->count++;
    /* stable partition of the keys by child */
    uint32_t start[ORC_MAX_FANOUT];
    uint32_t acc = 0;
    for (uint32_t j = 0; j < f; j++) { start[j] = acc; acc += parts[j]; }
    uint64_t* tmp = e->tmp;
    for (uint32_t i = 0; i < m; i++) {
        uint32_t j = child_of(orc_phi(keys[i], depth, v, m), unit, f);
        tmp[start[j]++] = keys[i];
    }
    memcpy(keys, tmp, (size_t)m * sizeof(uint64_t));
    acc = 0;
    for (uint32_t j = 0; j < f; j++) {
        rc = build_tree(st, keys + acc, parts[j], depth + 1, e);
        if (rc) return rc;
        acc += parts[j];
    }
    return ORC_OK;
}

/* One bucket's tree from its lower signature words: preorder lists of index,
 * node size and depth.  out_* must hold at least m entries. */
int orc_tree_slack(const uint64_t* lo, uint32_t m, uint32_t leaf, uint32_t slack, uint64_t seed_cap,
                   uint64_t* out_v, uint32_t* out_m, uint32_t* out_d, uint64_t* out_count) {
    if (leaf < 1 || leaf > 24) return ORC_EINVAL;
    strategy st = make_strategy(leaf);
    st.slack = slack;
    uint64_t* keys = malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    uint64_t* tmp = malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    if (!keys || !tmp) { free(keys); free(tmp); return ORC_ENOMEM; }
    memcpy(keys, lo, (size_t)m * sizeof(uint64_t));
    emitter e = {out_v, out_m, out_d, 0, seed_cap ? seed_cap : ORC_DEFAULT_SEED_CAP, tmp};
    int rc = build_tree(&st, keys, m, 0, &e);
    *out_count = e.count;
    free(keys);
    free(tmp);
    return rc;
}

int orc_tree(const uint64_t* lo, uint32_t m, uint32_t leaf, uint64_t seed_cap, uint64_t* out_v, uint32_t* out_m,
             uint32_t* out_d, uint64_t* out_count) {
    return orc_tree_slack(lo, m, leaf, 0, seed_cap, out_v, out_m, out_d, out_count);
}

/* Trees of buckets first..last-1 of a bucket-contiguous array of lower words
 * (bucket i holds sorted[s[i] .. s[i+1])).  Bucket i's coded nodes go to
 * node_v / node_m / node_d from slot s[i] on (a tree on m keys has at most m-1
 * coded nodes) and their count to node_count[i].  This is the tree loop of
 * orc_build; a test harness may run disjoint bucket ranges in separate
 * processes and pass the results to orc_build_with_trees. */
static int trees_impl(const uint64_t* sorted, const uint64_t* s, uint64_t first, uint64_t last, uint32_t leaf,
                      uint32_t slack, uint64_t seed_cap, uint64_t* node_v, uint32_t* node_m, uint32_t* node_d,
                      uint64_t* node_count) {
    if (leaf < 1 || leaf > 24) return ORC_EINVAL;
    strategy st = make_strategy(leaf);
    st.slack = slack;
    if (!seed_cap) seed_cap = ORC_DEFAULT_SEED_CAP;
    for (uint64_t i = first; i < last; i++) {
        uint64_t m = s[i + 1] - s[i];
        uint64_t* keys = malloc((m ? m : 1) * 8);
        uint64_t* scratch = malloc((m ? m : 1) * 8);
        if (!keys || !scratch) { free(keys); free(scratch); return ORC_ENOMEM; }
        memcpy(keys, sorted + s[i], m * 8);
        emitter e = {node_v + s[i], node_m + s[i], node_d + s[i], 0, seed_cap, scratch};
        int rc = build_tree(&st, keys, (uint32_t)m, 0, &e);
        free(keys);
        free(scratch);
        if (rc) return rc;
        node_count[i] = e.count;
    }
    return ORC_OK;
}

int orc_trees(const uint64_t* sorted, const uint64_t* s, uint64_t first, uint64_t last, uint32_t leaf,
              uint64_t seed_cap, uint64_t* node_v, uint32_t* node_m, uint32_t* node_d, uint64_t* node_count) {
    return trees_impl(sorted, s, first, last, leaf, 0, seed_cap, node_v, node_m, node_d, node_count);
}

/* ------------------------------------------------------------------------ */
/* Bit arrays: bit p lives in word p/64 at bit p%64 (LSB-first).             */
/* ------------------------------------------------------------------------ */
static void put_bits(uint64_t* a, uint64_t pos, uint64_t value, uint32_t nbits) {
    for (uint32_t b = 0; b < nbits; b++)
        if ((value >> b) & 1) a[(pos + b) / 64] |= 1ULL << ((pos + b) % 64);
}

static uint64_t get_bits(const uint64_t* a, uint64_t pos, uint32_t nbits) {
    uint64_t v = 0;
    for (uint32_t b = 0; b < nbits; b++) v |= ((a[(pos + b) / 64] >> ((pos + b) % 64)) & 1) << b;
    return v;
}

static int get_bit(const uint64_t* a, uint64_t pos) { return (int)((a[pos / 64] >> (pos % 64)) & 1); }

static int cmp_u64(const void* x, const void* y) {
    uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
    return a < b ? -1 : a > b;
}

/* Elias-Fano lower width: the largest W >= 0 with N * 2^W <= U, i.e.
 * max{0, floor(lg(U/N))} (Sec. 7.4). */
/* Two-level inventory of a bit array with `ones` set bits (Sec. 7.4): the
 * position of every one whose index is a multiple of 2^14 as a 64-bit integer,
 * and, for every one whose index is a multiple of 2^8, its distance from the
 * anchor of its 2^14 block as a 16-bit integer; a distance that does not fit
 * is stored as 0xffff, and a search then starts from the anchor.  The two
 * Elias-Fano lists of a structure interleave their entries, so the arrays are
 * written with a stride (hi[j*stride], lo[j*stride]). */
void orc_inventory_build(const uint64_t* bits, uint64_t ones, uint64_t* hi, uint16_t* lo, uint32_t stride) {
    uint64_t k = 0, pos = 0, anchor = 0;
    for (; k < ones; pos++) {
        if (!((bits[pos / 64] >> (pos % 64)) & 1)) continue;
        if (k % (1ULL << ORC_INV_HI) == 0) {
            anchor = pos;
            hi[(k >> ORC_INV_HI) * stride] = pos;
        }
        if (k % (1ULL << ORC_INV_LO) == 0) {
            uint64_t d = pos - anchor;
            lo[(k >> ORC_INV_LO) * stride] = (uint16_t)(d < ORC_INV_OVERFLOW ? d : ORC_INV_OVERFLOW);
        }
        k++;
    }
}

/* Position of the k-th one through the inventory: start at the nearest
 * recorded one and scan forward bit by bit. */
uint64_t orc_inventory_select(const uint64_t* bits, const uint64_t* hi, const uint16_t* lo, uint32_t stride,
                              uint64_t k) {
    uint64_t pos = hi[(k >> ORC_INV_HI) * stride];
    uint64_t left = k & ((1ULL << ORC_INV_HI) - 1);
    uint16_t d = lo[(k >> ORC_INV_LO) * stride];
    if (d != ORC_INV_OVERFLOW) {
        pos += d;
        left = k & ((1ULL << ORC_INV_LO) - 1);
    }
    for (;; pos++) {
        if ((bits[pos / 64] >> (pos % 64)) & 1) {
            if (left == 0) return pos;
            left--;
        }
    }
}

static uint32_t ef_width(uint64_t N, uint64_t U) {
    uint32_t W = 0;
    while (W < 62 && (N << (W + 1)) <= U && ((N << (W + 1)) >> (W + 1)) == N) W++;
    return W;
}

/* ------------------------------------------------------------------------ */
/* Construction (Sec. 4 and 6): buckets, trees, Golomb-Rice streams with all  */
/* fixed parts before all unary parts, concatenation, double Elias-Fano.     */
/* The blob is written to out (capacity cap bytes); *size receives its size;  */
/* if cap is too small only the size is reported.                            */
/* ------------------------------------------------------------------------ */
static int build_impl(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint32_t leaf,
                      uint32_t bucket, uint64_t seed_cap, uint32_t gr_max, uint32_t slack, const uint64_t* given_v,
                      const uint32_t* given_m, const uint64_t* given_count, void* out, uint64_t cap,
                      uint64_t* size) {
    if (n == 0 || leaf < 1 || leaf > 24 || bucket == 0 || !data || !size) return ORC_EINVAL;
    if (gr_max >= (1u << 24) || slack > 255) return ORC_EINVAL;
    strategy sts = make_strategy(leaf);
    sts.slack = slack;
    if (leaf_range(&sts, leaf) > 32) return ORC_EINVAL; /* a leaf's values fit one 32-bit mask */
    if (kind != ORC_KEYS_U64 && kind != ORC_KEYS_BYTES) return ORC_EINVAL;
    if (kind == ORC_KEYS_BYTES) {
        if (!offsets) return ORC_EINVAL;
        for (uint64_t i = 0; i < n; i++)
            if (offsets[i + 1] < offsets[i]) return ORC_EINVAL;
    }
    if (!seed_cap) seed_cap = ORC_DEFAULT_SEED_CAP;
    uint64_t nb = (n + bucket - 1) / bucket;
    int rc = ORC_ENOMEM;

    uint64_t *hi = malloc(n * 8), *lo = malloc(n * 8), *sorted = malloc(n * 8);
    uint64_t *sz = calloc(nb, 8), *s = calloc(nb + 1, 8), *o = calloc(nb + 1, 8), *cursor = calloc(nb, 8);
    uint64_t* node_v = malloc(n * 8);
    uint32_t *node_m = malloc(n * 4), *node_d = malloc(n * 4);
    uint64_t* node_count = calloc(nb, 8);
    uint64_t* qs = calloc(nb + 1, 8); /* the first Elias-Fano list: prefix sums of the buckets' output ranges */
    uint32_t *r = NULL, *F = NULL, *N = NULL;
    uint64_t *tree = NULL, *lower = NULL, *up_s = NULL, *up_z = NULL, *ys = NULL, *yz = NULL;
    int64_t* z = NULL;
    if (!hi || !lo || !sorted || !sz || !s || !o || !cursor || !node_v || !node_m || !node_d || !node_count || !qs)
        goto done;

    if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data, n, hi, lo);
    else orc_fingerprint_bytes((const uint8_t*)data, offsets, n, hi, lo);

    /* bucket sizes, prefix sums s_i, and bucket-contiguous lower words */
    for (uint64_t i = 0; i < n; i++) sz[bucket_of(hi[i], nb)]++;
    for (uint64_t i = 0; i < nb; i++) s[i + 1] = s[i] + sz[i];
    for (uint64_t i = 0; i < n; i++) {
        uint64_t bk = bucket_of(hi[i], nb);
        sorted[s[bk] + cursor[bk]++] = lo[i];
    }
    uint64_t maxm = 0;
    for (uint64_t i = 0; i < nb; i++) if (sz[i] > maxm) maxm = sz[i];

    /* equal lower words inside a bucket make every search fail: reject them
     * (this covers duplicate keys) */
    for (uint64_t i = 0; i < nb; i++) {
        qsort(sorted + s[i], sz[i], 8, cmp_u64);
        for (uint64_t k = 1; k < sz[i]; k++)
            if (sorted[s[i] + k] == sorted[s[i] + k - 1]) { rc = ORC_EDUPLICATE; goto done; }
    }

    r = malloc((maxm + 1) * 4); F = malloc((maxm + 1) * 4); N = malloc((maxm + 1) * 4);
    if (!r || !F || !N) goto done;
    tables_impl(leaf, (uint32_t)maxm, gr_max, slack, r, F, N);
    /* output ranges: s_i itself for the minimal structure; the range of a
     * subtree grows strictly with its size (checked), so lookups recover a
     * bucket's size from its range */
    for (uint64_t i = 0; i < nb; i++) qs[i + 1] = qs[i] + (slack ? subtree_range(&sts, (uint32_t)sz[i]) : sz[i]);
    for (uint32_t m = 1; slack && m <= maxm; m++)
        if (subtree_range(&sts, m) <= subtree_range(&sts, m - 1)) { rc = ORC_EINVAL; goto done; }

    /* trees; bucket i's coded nodes are stored from slot s_i on (a tree on m
     * keys has at most m-1 coded nodes), or taken as given */
    if (given_v) {
        memcpy(node_v, given_v, n * 8);
        memcpy(node_m, given_m, n * 4);
        memcpy(node_count, given_count, nb * 8);
    } else {
        rc = trees_impl(sorted, s, 0, nb, leaf, slack, seed_cap, node_v, node_m, node_d, node_count);
        if (rc) goto done;
        rc = ORC_ENOMEM;
    }

    /* Golomb-Rice stream lengths and offsets o_i */
    for (uint64_t i = 0; i < nb; i++) {
        uint64_t len = 0;
        for (uint64_t k = 0; k < node_count[i]; k++) {
            uint32_t rr = r[node_m[s[i] + k]];
            len += rr + (node_v[s[i] + k] >> rr) + 1;
        }
        o[i + 1] = o[i] + len;
    }
    uint64_t total_bits = o[nb];
    uint64_t tree_words = (total_bits + 63) / 64 + 1;
    tree = calloc(tree_words, 8);
    if (!tree) goto done;
    for (uint64_t i = 0; i < nb; i++) {
        uint64_t pos = o[i];
        for (uint64_t k = 0; k < node_count[i]; k++) { /* fixed parts, preorder */
            uint32_t rr = r[node_m[s[i] + k]];
            put_bits(tree, pos, node_v[s[i] + k] & ((1ULL << rr) - 1), rr);
            pos += rr;
        }
        for (uint64_t k = 0; k < node_count[i]; k++) { /* unary parts, preorder */
            uint32_t rr = r[node_m[s[i] + k]];
            pos += node_v[s[i] + k] >> rr; /* zeros */
            put_bits(tree, pos, 1, 1);      /* terminating one */
            pos += 1;
        }
    }

    /* double Elias-Fano of s_i and z_i = o_i - floor(beta s_i), beta in 16.16
     * fixed point; each list is rescaled by its minimum gap (Sec. 6.3). */
    uint64_t Nn = nb + 1;
    uint64_t beta = (total_bits << 16) / qs[nb];
    z = malloc(Nn * 8); ys = malloc(Nn * 8); yz = malloc(Nn * 8);
    if (!z || !ys || !yz) goto done;
    for (uint64_t i = 0; i < Nn; i++) z[i] = (int64_t)o[i] - (int64_t)((beta * qs[i]) >> 16);
    uint64_t delta_s = UINT64_MAX;
    int64_t delta_z = INT64_MAX;
    for (uint64_t i = 0; i + 1 < Nn; i++) {
        if (qs[i + 1] - qs[i] < delta_s) delta_s = qs[i + 1] - qs[i];
        if (z[i + 1] - z[i] < delta_z) delta_z = z[i + 1] - z[i];
    }
    for (uint64_t i = 0; i < Nn; i++) {
        ys[i] = qs[i] - i * delta_s;
        yz[i] = (uint64_t)(z[i] - (int64_t)i * delta_z);
    }
    uint32_t Ws = ef_width(Nn, ys[Nn - 1]), Wz = ef_width(Nn, yz[Nn - 1]);
    uint64_t us_bits = (ys[Nn - 1] >> Ws) + Nn, uz_bits = (yz[Nn - 1] >> Wz) + Nn;
    uint64_t us_words = (us_bits + 63) / 64, uz_words = (uz_bits + 63) / 64;
    uint64_t lower_words = (Nn * (Ws + Wz) + 63) / 64 + 1;
    uint64_t n_hi = (Nn + (1ULL << ORC_INV_HI) - 1) >> ORC_INV_HI;
    uint64_t n_lo = (Nn + (1ULL << ORC_INV_LO) - 1) >> ORC_INV_LO;
    uint64_t lo_words = (2 * n_lo + 3) / 4; /* 16-bit entries, four per word */
    uint64_t total_words = ORC_HEADER_WORDS + lower_words + us_words + uz_words + 2 * n_hi + lo_words + tree_words;
    *size = total_words * 8;
    if (!out || cap < *size) { rc = ORC_OK; goto done; }

    uint64_t* w = calloc(total_words, 8);
    if (!w) goto done;
    w[0] = ORC_MAGIC;
    w[1] = ORC_VERSION | ((uint64_t)kind << 32);
    w[2] = n; w[3] = leaf; w[4] = bucket; w[5] = nb; w[6] = maxm;
    w[7] = (uint64_t)Ws | ((uint64_t)Wz << 8) | ((uint64_t)gr_max << 16) | ((uint64_t)slack << 40);
    w[8] = delta_s; w[9] = (uint64_t)delta_z; w[10] = beta;
    w[11] = us_words; w[12] = uz_words; w[13] = lower_words; w[14] = tree_words; w[15] = total_bits;
    lower = w + ORC_HEADER_WORDS;
    up_s = lower + lower_words;
    up_z = up_s + us_words;
    uint64_t* inv_hi = up_z + uz_words;            /* s, z anchors interleaved */
    uint16_t* inv_lo = (uint16_t*)(inv_hi + 2 * n_hi); /* s, z offsets interleaved */
    uint64_t* tr = inv_hi + 2 * n_hi + lo_words;
    for (uint64_t i = 0; i < Nn; i++) {
        put_bits(lower, i * (Ws + Wz), ys[i] & ((1ULL << Ws) - 1), Ws);
        put_bits(lower, i * (Ws + Wz) + Ws, yz[i] & ((1ULL << Wz) - 1), Wz);
        put_bits(up_s, (ys[i] >> Ws) + i, 1, 1);
        put_bits(up_z, (yz[i] >> Wz) + i, 1, 1);
    }
    orc_inventory_build(up_s, Nn, inv_hi, inv_lo, 2);
    orc_inventory_build(up_z, Nn, inv_hi + 1, inv_lo + 1, 2);
    memcpy(tr, tree, tree_words * 8);
    memcpy(out, w, total_words * 8);
    free(w);
    rc = ORC_OK;

done:
    free(hi); free(lo); free(sorted); free(sz); free(s); free(o); free(cursor);
    free(node_v); free(node_m); free(node_d); free(node_count); free(qs);
    free(r); free(F); free(N); free(tree); free(z); free(ys); free(yz);
    return rc;
}

int orc_build(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint32_t leaf, uint32_t bucket,
              uint64_t seed_cap, void* out, uint64_t cap, uint64_t* size) {
    return build_impl(kind, data, offsets, n, leaf, bucket, seed_cap, 0, 0, NULL, NULL, NULL, out, cap, size);
}

/* orc_build with the Golomb-Rice parameters of splits of more than gr_max keys
 * from the integer approximation of Sec. 7.2 (recorded in the header, bits
 * 16-39 of word 7), and, for slack > 0, the non-minimal variant: leaves map
 * injectively into m + ceil(m slack / 256) values and the first Elias-Fano
 * list holds the prefix sums of the buckets' output ranges instead of their
 * sizes (slack in bits 40-47 of word 7).  Keys then map one-to-one into
 * [0, N), N the last value of that list. */
int orc_build_ex(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint32_t leaf,
                 uint32_t bucket, uint64_t seed_cap, uint32_t gr_max, uint32_t slack, void* out, uint64_t cap,
                 uint64_t* size) {
    return build_impl(kind, data, offsets, n, leaf, bucket, seed_cap, gr_max, slack, NULL, NULL, NULL, out, cap,
                      size);
}

/* orc_build with every bucket's tree supplied (as orc_trees writes them, for
 * all nb buckets of the same key set): the same bytes, with the trees computed
 * elsewhere (test harnesses run orc_trees over bucket ranges in parallel
 * processes).  The trees are not checked beyond their node counts. */
int orc_build_with_trees(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint32_t leaf,
                         uint32_t bucket, const uint64_t* node_v, const uint32_t* node_m, const uint64_t* node_count,
                         void* out, uint64_t cap, uint64_t* size) {
    if (!node_v || !node_m || !node_count) return ORC_EINVAL;
    return build_impl(kind, data, offsets, n, leaf, bucket, 0, 0, 0, node_v, node_m, node_count, out, cap, size);
}

/* Bucket-contiguous lower signature words of a key set (each bucket sorted
 * ascending) and the prefix sums s[0..nb] of the bucket sizes, as orc_build
 * arranges them; ORC_EDUPLICATE if a bucket holds two equal lower words. */
int orc_bucket_layout(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint64_t nb,
                      uint64_t* sorted, uint64_t* s) {
    uint64_t *hi = malloc((n ? n : 1) * 8), *lo = malloc((n ? n : 1) * 8), *cursor = calloc(nb ? nb : 1, 8);
    int rc = ORC_ENOMEM;
    if (!hi || !lo || !cursor) goto out;
    if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data, n, hi, lo);
    else orc_fingerprint_bytes((const uint8_t*)data, offsets, n, hi, lo);
    memset(s, 0, (nb + 1) * 8);
    for (uint64_t i = 0; i < n; i++) s[bucket_of(hi[i], nb) + 1]++;
    for (uint64_t i = 0; i < nb; i++) s[i + 1] += s[i];
    for (uint64_t i = 0; i < n; i++) {
        uint64_t bk = bucket_of(hi[i], nb);
        sorted[s[bk] + cursor[bk]++] = lo[i];
    }
    rc = ORC_OK;
    for (uint64_t i = 0; i < nb; i++) {
        qsort(sorted + s[i], s[i + 1] - s[i], 8, cmp_u64);
        for (uint64_t k = s[i] + 1; k < s[i + 1]; k++)
            if (sorted[k] == sorted[k - 1]) rc = ORC_EDUPLICATE;
    }
out:
    free(hi); free(lo); free(cursor);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Lookup (Sec. 4 and 6.2).  The oracle decodes the Elias-Fano lists by a     */
/* plain scan of the upper bits and each bucket's indices by reading all      */
/* fixed parts and then all unary parts in preorder; it then walks down the   */
/* tree, counting the keys left of the chosen child.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t n, leaf, nb, maxm, kind;
    strategy st;
    uint64_t* Q; /* output range of a subtree of each size 0..maxm */
    uint64_t* s; /* nb+1 prefix sums of the buckets' output ranges (of their sizes if minimal) */
    uint64_t* o; /* nb+1 bit offsets */
    const uint64_t* tree;
    uint32_t* r;
    const uint64_t* up[2];    /* upper bits of s and z */
    const uint64_t* inv_hi;   /* interleaved anchors */
    const uint16_t* inv_lo;   /* interleaved offsets */
} decoded;

static uint32_t coded_nodes(const strategy* st, uint32_t m) {
    if (m <= 1) return 0;
    if (m <= st->leaf) return 1;
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    uint32_t c = 1;
    for (uint32_t j = 0; j < f; j++) c += coded_nodes(st, parts[j]);
    return c;
}

/* sizes of the coded nodes of a tree on m keys, in preorder */
static void preorder_sizes(const strategy* st, uint32_t m, uint32_t* out, uint32_t* count) {
    if (m <= 1) return;
    out[(*count)++] = m;
    if (m <= st->leaf) return;
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(st, m, parts, &unit);
    for (uint32_t j = 0; j < f; j++) preorder_sizes(st, parts[j], out, count);
}

static uint64_t descend(const decoded* dc, uint64_t x, uint32_t m, uint32_t depth, const uint64_t* vs,
                        uint32_t* idx) {
    if (m <= 1) return 0;
    uint64_t v = vs[(*idx)++];
    if (m <= dc->st.leaf) return orc_phi(x, depth, v, leaf_range(&dc->st, m));
    uint32_t phi = orc_phi(x, depth, v, m);
    uint32_t parts[ORC_MAX_FANOUT], unit;
    uint32_t f = split_parts(&dc->st, m, parts, &unit);
    uint32_t j = child_of(phi, unit, f);
    uint64_t left = 0; /* the output values of the parts before the chosen one */
    for (uint32_t t = 0; t < j; t++) {
        *idx += coded_nodes(&dc->st, parts[t]);
        left += dc->Q[parts[t]];
    }
    return left + descend(dc, x, parts[j], depth + 1, vs, idx);
}

/* Parse a blob's header and decode both Elias-Fano lists (s_i and o_i for
 * i = 0..nb) by a plain scan of their upper bits (Sec. 6.3). */
static int blob_open(const void* blob, uint64_t bytes, decoded* dc) {
    const uint64_t* w = (const uint64_t*)blob;
    memset(dc, 0, sizeof(*dc));
    if (!blob || bytes < ORC_HEADER_WORDS * 8 || w[0] != ORC_MAGIC || (w[1] & 0xffffffffULL) != ORC_VERSION)
        return ORC_EFORMAT;
    dc->n = w[2]; dc->leaf = w[3]; dc->nb = w[5]; dc->maxm = w[6]; dc->kind = w[1] >> 32;
    if (dc->leaf < 1 || dc->leaf > 24) return ORC_EFORMAT;
    dc->st = make_strategy((uint32_t)dc->leaf);
    uint32_t Ws = (uint32_t)(w[7] & 0xff), Wz = (uint32_t)((w[7] >> 8) & 0xff);
    uint32_t gr_max = (uint32_t)((w[7] >> 16) & 0xffffff), slack = (uint32_t)((w[7] >> 40) & 0xff);
    dc->st.slack = slack;
    uint64_t delta_s = w[8];
    int64_t delta_z = (int64_t)w[9];
    uint64_t beta = w[10], us_words = w[11], uz_words = w[12], lower_words = w[13], tree_words = w[14];
    uint64_t Nn = dc->nb + 1;
    uint64_t n_hi = (Nn + (1ULL << ORC_INV_HI) - 1) >> ORC_INV_HI;
    uint64_t lo_words = (2 * ((Nn + (1ULL << ORC_INV_LO) - 1) >> ORC_INV_LO) + 3) / 4;
    if (bytes != (ORC_HEADER_WORDS + lower_words + us_words + uz_words + 2 * n_hi + lo_words + tree_words) * 8)
        return ORC_EFORMAT;
    const uint64_t* lower = w + ORC_HEADER_WORDS;
    const uint64_t* up_s = lower + lower_words;
    const uint64_t* up_z = up_s + us_words;
    dc->tree = up_z + uz_words + 2 * n_hi + lo_words;
    dc->up[0] = up_s;
    dc->up[1] = up_z;
    dc->inv_hi = up_z + uz_words;
    dc->inv_lo = (const uint16_t*)(dc->inv_hi + 2 * n_hi);

    dc->s = malloc(Nn * 8);
    dc->o = malloc(Nn * 8);
    dc->r = malloc((dc->maxm + 1) * 4);
    dc->Q = malloc((dc->maxm + 1) * 8);
    uint32_t* Ft = malloc((dc->maxm + 1) * 4);
    uint32_t* Nt = malloc((dc->maxm + 1) * 4);
    if (!dc->s || !dc->o || !dc->r || !dc->Q || !Ft || !Nt) {
        free(Ft); free(Nt);
        return ORC_ENOMEM;
    }
    orc_tables_slack((uint32_t)dc->leaf, (uint32_t)dc->maxm, gr_max, slack, dc->r, Ft, Nt, dc->Q);
    free(Ft);
    free(Nt);

    /* the i-th one of the upper bits sits at (y_i >> W) + i */
    uint64_t ps = 0, pz = 0;
    for (uint64_t i = 0; i < Nn; i++) {
        while (!get_bit(up_s, ps)) ps++;
        while (!get_bit(up_z, pz)) pz++;
        uint64_t ys = ((ps - i) << Ws) | get_bits(lower, i * (Ws + Wz), Ws);
        uint64_t yz = ((pz - i) << Wz) | get_bits(lower, i * (Ws + Wz) + Ws, Wz);
        dc->s[i] = ys + i * delta_s;
        int64_t zi = (int64_t)yz + (int64_t)i * delta_z;
        dc->o[i] = (uint64_t)(zi + (int64_t)((beta * dc->s[i]) >> 16));
        ps++;
        pz++;
    }
    return ORC_OK;
}

static void blob_close(decoded* dc) {
    free(dc->s); free(dc->o); free(dc->r); free(dc->Q);
    dc->s = dc->o = dc->Q = NULL;
    dc->r = NULL;
}

/* Size of bucket bk: the size whose subtree range is the bucket's range (the
 * range grows strictly with the size; for the minimal structure they are
 * equal). */
static uint32_t bucket_size(const decoded* dc, uint64_t bk) {
    uint64_t range = dc->s[bk + 1] - dc->s[bk];
    for (uint32_t m = 0; m <= dc->maxm; m++)
        if (dc->Q[m] == range) return m;
    return 0; /* not a range of this structure: a corrupted blob */
}

/* Indices of the coded nodes of bucket bk, in preorder (Sec. 6.2): all fixed
 * parts first, then all unary parts.  sizes/vs hold maxm+1 entries. */
static uint32_t bucket_codes(const decoded* dc, uint64_t bk, uint32_t* sizes, uint64_t* vs) {
    uint32_t m = bucket_size(dc, bk);
    uint32_t cnt = 0;
    preorder_sizes(&dc->st, m, sizes, &cnt);
    uint64_t pos = dc->o[bk];
    for (uint32_t k = 0; k < cnt; k++) { /* fixed parts */
        vs[k] = get_bits(dc->tree, pos, dc->r[sizes[k]]);
        pos += dc->r[sizes[k]];
    }
    for (uint32_t k = 0; k < cnt; k++) { /* unary parts */
        uint64_t zeros = 0;
        while (!get_bit(dc->tree, pos)) { zeros++; pos++; }
        pos++;
        vs[k] |= zeros << dc->r[sizes[k]];
    }
    return cnt;
}

int orc_lookup(const void* blob, uint64_t bytes, uint32_t kind, const void* data, const uint64_t* offsets, uint64_t q,
               uint64_t* ranks) {
    decoded dc;
    int rc = blob_open(blob, bytes, &dc);
    if (rc) { blob_close(&dc); return rc; }
    if (dc.kind != kind) { blob_close(&dc); return ORC_EINVAL; }
    uint32_t* sizes = malloc((dc.maxm + 1) * 4);
    uint64_t* vs = malloc((dc.maxm + 1) * 8);
    rc = ORC_ENOMEM;
    if (!sizes || !vs) goto out;
    for (uint64_t qi = 0; qi < q; qi++) {
        uint64_t hi, lo;
        if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data + qi, 1, &hi, &lo);
        else fingerprint_bytes_one((const uint8_t*)data + offsets[qi], offsets[qi + 1] - offsets[qi], &hi, &lo);
        uint64_t bk = bucket_of(hi, dc.nb);
        uint32_t m = bucket_size(&dc, bk);
        bucket_codes(&dc, bk, sizes, vs);
        uint32_t idx = 0;
        ranks[qi] = dc.s[bk] + descend(&dc, lo, m, 0, vs, &idx);
    }
    rc = ORC_OK;
out:
    free(sizes); free(vs);
    blob_close(&dc);
    return rc;
}

/* Decode one bucket of a blob: its first rank s_i, its first tree bit o_i,
 * and the index and size of each coded node in preorder.  out_v / out_m hold
 * cap entries; *out_count receives the node count (a count above cap means
 * the lists were cut).  Used to compare single buckets of large structures. */
int orc_blob_bucket(const void* blob, uint64_t bytes, uint64_t bucket, uint64_t* out_s, uint64_t* out_o,
                    uint64_t* out_v, uint32_t* out_m, uint64_t cap, uint64_t* out_count) {
    decoded dc;
    int rc = blob_open(blob, bytes, &dc);
    if (rc) { blob_close(&dc); return rc; }
    if (bucket >= dc.nb) { blob_close(&dc); return ORC_EINVAL; }
    uint32_t* sizes = malloc((dc.maxm + 1) * 4);
    uint64_t* vs = malloc((dc.maxm + 1) * 8);
    rc = ORC_ENOMEM;
    if (!sizes || !vs) goto out;
    uint32_t cnt = bucket_codes(&dc, bucket, sizes, vs);
    for (uint32_t k = 0; k < cnt && k < cap; k++) { out_v[k] = vs[k]; out_m[k] = sizes[k]; }
    *out_s = dc.s[bucket];
    *out_o = dc.o[bucket];
    *out_count = cnt;
    rc = ORC_OK;
out:
    free(sizes); free(vs);
    blob_close(&dc);
    return rc;
}

/* Both Elias-Fano lists of a blob decoded in full: s_i and o_i for
 * i = 0..nb (each output holds nb+1 entries). */
int orc_blob_prefix(const void* blob, uint64_t bytes, uint64_t* out_s, uint64_t* out_o) {
    decoded dc;
    int rc = blob_open(blob, bytes, &dc);
    if (rc == ORC_OK) {
        memcpy(out_s, dc.s, (dc.nb + 1) * 8);
        memcpy(out_o, dc.o, (dc.nb + 1) * 8);
    }
    blob_close(&dc);
    return rc;
}

/* Every k-th one of both upper-bit arrays found through the blob's inventory
 * against the plain scan the decoder does; returns the number of mismatches
 * in *bad (a round trip of the inventory, Sec. 7.4). */
int orc_blob_check_inventory(const void* blob, uint64_t bytes, uint64_t* bad) {
    decoded dc;
    int rc = blob_open(blob, bytes, &dc);
    if (rc) { blob_close(&dc); return rc; }
    uint64_t miss = 0;
    for (int list = 0; list < 2; list++) {
        uint64_t pos = 0;
        for (uint64_t k = 0; k <= dc.nb; k++, pos++) {
            while (!get_bit(dc.up[list], pos)) pos++;
            if (orc_inventory_select(dc.up[list], dc.inv_hi + list, dc.inv_lo + list, 2, k) != pos) miss++;
        }
    }
    *bad = miss;
    blob_close(&dc);
    return ORC_OK;
}

/* Rank of each key of one bucket inside the bucket (0..m-1), from the tree
 * the oracle builds for the bucket's lower signature words: the keys left of
 * the chosen child at every split plus the leaf's bijection (Sec. 4). */
/* In-bucket ranks of a bucket's m lower words given its tree's indices v (in
 * preorder, as orc_tree emits them): the descent of the lookup (Sec. 4). */
int orc_ranks_from_tree(const uint64_t* lo, uint32_t m, uint32_t leaf, const uint64_t* v, uint64_t* ranks) {
    if (leaf < 1 || leaf > 24) return ORC_EINVAL;
    decoded dc;
    memset(&dc, 0, sizeof(dc));
    dc.leaf = leaf;
    dc.st = make_strategy(leaf);
    dc.Q = malloc(((size_t)m + 1) * 8); /* minimal structure: a subtree's range is its size */
    if (!dc.Q) return ORC_ENOMEM;
    for (uint32_t k = 0; k <= m; k++) dc.Q[k] = k;
    for (uint32_t i = 0; i < m; i++) {
        uint32_t idx = 0;
        ranks[i] = descend(&dc, lo[i], m, 0, v, &idx);
    }
    free(dc.Q);
    return ORC_OK;
}

int orc_bucket_ranks(const uint64_t* lo, uint32_t m, uint32_t leaf, uint64_t seed_cap, uint64_t* ranks) {
    if (leaf < 1 || leaf > 24) return ORC_EINVAL;
    uint64_t* v = malloc((size_t)(m ? m : 1) * 8);
    uint32_t* mm = malloc((size_t)(m ? m : 1) * 4);
    uint32_t* d = malloc((size_t)(m ? m : 1) * 4);
    int rc = ORC_ENOMEM;
    if (!v || !mm || !d) goto out;
    uint64_t cnt = 0;
    rc = orc_tree(lo, m, leaf, seed_cap, v, mm, d, &cnt);
    if (rc) goto out;
    rc = orc_ranks_from_tree(lo, m, leaf, v, ranks);
out:
    free(v); free(mm); free(d);
    return rc;
}

/* Bucket of every signature (Sec. 6.1: floor(hi * nb / 2^64)). */
void orc_bucket_ids(const uint64_t* hi, uint64_t n, uint64_t nb, uint64_t* ids) {
    for (uint64_t i = 0; i < n; i++) ids[i] = bucket_of(hi[i], nb);
}

/* Bucket sizes only (for the bucket-distribution pin). */
int orc_bucket_sizes(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint64_t nb,
                     uint64_t* sizes) {
    uint64_t *hi = malloc(n * 8), *lo = malloc(n * 8);
    if (!hi || !lo) { free(hi); free(lo); return ORC_ENOMEM; }
    if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data, n, hi, lo);
    else orc_fingerprint_bytes((const uint8_t*)data, offsets, n, hi, lo);
    memset(sizes, 0, nb * 8);
    for (uint64_t i = 0; i < n; i++) sizes[bucket_of(hi[i], nb)]++;
    free(hi); free(lo);
    return ORC_OK;
}

/* Lower signature words of one bucket, sorted ascending (for per-bucket
 * parity checks on samples of large builds). Returns the bucket size. */
uint64_t orc_bucket_keys(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint64_t nb,
                         uint64_t bucket, uint64_t* out, uint64_t cap) {
    uint64_t cnt = 0, hi, lo;
    for (uint64_t i = 0; i < n; i++) {
        if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data + i, 1, &hi, &lo);
        else fingerprint_bytes_one((const uint8_t*)data + offsets[i], offsets[i + 1] - offsets[i], &hi, &lo);
        if (bucket_of(hi, nb) == bucket) {
            if (cnt < cap) out[cnt] = lo;
            cnt++;
        }
    }
    if (cnt <= cap) qsort(out, cnt, 8, cmp_u64);
    return cnt;
}

/* Indices (positions in the input) of the keys of one bucket, ascending.
 * Returns the bucket size; at most cap indices are written. */
uint64_t orc_bucket_members(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint64_t nb,
                            uint64_t bucket, uint64_t* out, uint64_t cap) {
    uint64_t cnt = 0, hi, lo;
    for (uint64_t i = 0; i < n; i++) {
        if (kind == ORC_KEYS_U64) orc_fingerprint_u64((const uint64_t*)data + i, 1, &hi, &lo);
        else fingerprint_bytes_one((const uint8_t*)data + offsets[i], offsets[i + 1] - offsets[i], &hi, &lo);
        if (bucket_of(hi, nb) == bucket) {
            if (cnt < cap) out[cnt] = i;
            cnt++;
        }
    }
    return cnt;
}
