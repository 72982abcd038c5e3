/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * CPU oracle (test infrastructure only).  It runs every exported entry point
 * of the oracle on small seeded inputs, its error paths included, and checks
 * the structural facts a correct run gives (lookups form a bijection onto
 * [0, n), or an injection into [0, R) for the non-minimal variant).  Any
 * memory error or undefined behaviour aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { KEYS_U64 = 1, KEYS_BYTES = 2 }; /* the oracle's key kinds */

void orc_splitmix64_stream(uint64_t seed, uint64_t count, uint64_t* out);
void orc_fingerprint_u64(const uint64_t* keys, uint64_t n, uint64_t* hi, uint64_t* lo);
int orc_tables_ex(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t* r, uint32_t* F, uint32_t* N);
int orc_tables_slack(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack, uint32_t* r, uint32_t* F,
                     uint32_t* N, uint64_t* Q);
int orc_packed_table(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t* out);
int orc_build_ex(uint32_t kind, const void* data, const uint64_t* offsets, uint64_t n, uint32_t leaf,
                 uint32_t bucket, uint64_t seed_cap, uint32_t gr_max, uint32_t slack, void* out, uint64_t cap,
                 uint64_t* size);
int orc_lookup(const void* blob, uint64_t bytes, uint32_t kind, const void* data, const uint64_t* offsets, uint64_t q,
               uint64_t* ranks);
int orc_blob_prefix(const void* blob, uint64_t bytes, uint64_t* out_s, uint64_t* out_o);
int orc_blob_check_inventory(const void* blob, uint64_t bytes, uint64_t* bad);
int orc_blob_bucket(const void* blob, uint64_t bytes, uint64_t bucket, uint64_t* out_s, uint64_t* out_o,
                    uint64_t* out_v, uint32_t* out_m, uint64_t cap, uint64_t* out_count);

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(2);                                                    \
        }                                                               \
    } while (0)

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

/* build, look every key up, and check the values are distinct and below the
 * last value of the first Elias-Fano list */
static void one(uint32_t kind, const void* data, const uint64_t* offs, uint64_t n, uint32_t leaf, uint32_t bucket,
                uint32_t gr_max, uint32_t slack) {
    uint64_t size = 0;
    CHECK(orc_build_ex(kind, data, offs, n, leaf, bucket, 0, gr_max, slack, NULL, 0, &size) == 0);
    uint8_t* blob = malloc(size);
    uint64_t size2 = 0;
    CHECK(blob && orc_build_ex(kind, data, offs, n, leaf, bucket, 0, gr_max, slack, blob, size, &size2) == 0);
    CHECK(size2 == size);
    uint64_t nb = (n + bucket - 1) / bucket;
    uint64_t *s = malloc((nb + 1) * 8), *o = malloc((nb + 1) * 8), *v = malloc(n * 8);
    CHECK(s && o && v && orc_blob_prefix(blob, size, s, o) == 0);
    uint64_t bad = 1;
    CHECK(orc_blob_check_inventory(blob, size, &bad) == 0 && bad == 0);
    CHECK(orc_lookup(blob, size, kind, data, offs, n, v) == 0);
    qsort(v, n, 8, cmp_u64);
    for (uint64_t i = 0; i < n; i++) {
        CHECK(v[i] < s[nb]);
        if (i) CHECK(v[i] > v[i - 1]);
    }
    if (!slack) CHECK(s[nb] == n && v[n - 1] == n - 1);
    uint64_t vv[64], s0 = 0, o0 = 0, cnt = 0;
    uint32_t mm[64];
    CHECK(orc_blob_bucket(blob, size, nb - 1, &s0, &o0, vv, mm, 64, &cnt) == 0 && s0 == s[nb - 1]);
    CHECK(orc_blob_bucket(blob, size, nb, &s0, &o0, vv, mm, 64, &cnt) != 0); /* out of range */
    /* a truncated or corrupted blob is refused, not read past its end */
    CHECK(orc_lookup(blob, size - 8, kind, data, offs, 1, v) != 0);
    blob[0] ^= 1;
    CHECK(orc_lookup(blob, size, kind, data, offs, 1, v) != 0);
    free(blob); free(s); free(o); free(v);
}

int main(void) {
    enum { N = 20000 };
    uint64_t* keys = malloc(N * 8);
    orc_splitmix64_stream(7, N, keys);
    /* n, l, b, gr_table_max, leaf_slack: leaves of at most 12 keys, or larger
     * leaves only with slack (a minimal leaf of 16-24 keys takes 10^6-10^9
     * trials, too slow under the sanitizers) */
    static const uint32_t shapes[][5] = {{N, 8, 100, 0, 0},     {N, 5, 5, 0, 0},       {N, 12, 9, 0, 0},
                                         {N, 1, 1, 0, 0},       {N, 2, 3, 0, 0},       {N, 12, 2000, 0, 0},
                                         {N, 8, 1000, 300, 0},  {N, 8, 100, 0, 64},    {N, 5, 5, 0, 255},
                                         {3000, 16, 200, 0, 128}, {500, 24, 48, 0, 85}, {N, 7, 1, 0, 0}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; i++)
        one(KEYS_U64, keys, NULL, shapes[i][0], shapes[i][1], shapes[i][2], shapes[i][3], shapes[i][4]);
    one(KEYS_U64, keys, NULL, 1, 8, 100, 0, 0);
    /* byte strings of lengths 0..40, unaligned */
    enum { NS = 3000 };
    uint64_t* offs = malloc((NS + 1) * 8);
    uint8_t* text = malloc(NS * 41 + 1);
    uint64_t pos = 1;
    offs[0] = 0;
    for (uint64_t i = 0; i < NS; i++) {
        uint32_t len = (uint32_t)(keys[i] % 41);
        for (uint32_t j = 0; j < len; j++) text[pos + j] = (uint8_t)('a' + (keys[i] >> (j % 56)) % 26);
        /* make every string distinct: its index in the first bytes */
        if (len >= 2) { text[pos] = (uint8_t)(i & 0xff); text[pos + 1] = (uint8_t)(i >> 8); }
        pos += len;
        offs[i + 1] = pos - 1;
    }
    /* strings of length < 2 may repeat: keep the set from index 100 on, whose
     * lengths are drawn again until each has at least 2 bytes */
    {
        uint64_t m = 0, p2 = 1;
        uint64_t* o2 = malloc((NS + 1) * 8);
        uint8_t* t2 = malloc(NS * 43 + 1);
        o2[0] = 0;
        for (uint64_t i = 0; i < NS; i++) {
            uint64_t len = offs[i + 1] - offs[i];
            if (len < 2) continue;
            memcpy(t2 + p2, text + 1 + offs[i], len);
            p2 += len;
            o2[++m] = p2 - 1;
        }
        one(KEYS_BYTES, t2 + 1, o2, m, 8, 100, 0, 0);
        one(KEYS_BYTES, t2 + 1, o2, m, 6, 50, 0, 32);
        free(o2); free(t2);
    }
    /* tables */
    uint32_t r[4097], F[4097], Nn[4097], P[4097];
    uint64_t Q[4097];
    for (uint32_t leaf = 1; leaf <= 24; leaf++) {
        CHECK(orc_tables_ex(leaf, 4096, 0, r, F, Nn) == 0);
        CHECK(orc_tables_ex(leaf, 4096, leaf * 10, r, F, Nn) == 0);
        (void)orc_packed_table(leaf, 2600, 0, P);
        CHECK(orc_tables_slack(leaf, 4096, 0, leaf <= 16 ? 200 : 80, r, F, Nn, Q) == 0);
    }
    /* error paths */
    uint64_t size = 0;
    CHECK(orc_build_ex(KEYS_U64, keys, NULL, 0, 8, 100, 0, 0, 0, NULL, 0, &size) != 0);
    CHECK(orc_build_ex(KEYS_U64, keys, NULL, 10, 25, 100, 0, 0, 0, NULL, 0, &size) != 0);
    CHECK(orc_build_ex(KEYS_U64, keys, NULL, 10, 24, 100, 0, 0, 86, NULL, 0, &size) != 0);
    CHECK(orc_build_ex(KEYS_U64, keys, NULL, 10, 8, 100, 0, 1u << 24, 0, NULL, 0, &size) != 0);
    uint64_t dup[4] = {5, 6, 5, 7};
    CHECK(orc_build_ex(KEYS_U64, dup, NULL, 4, 8, 100, 0, 0, 0, NULL, 0, &size) == 2);
    CHECK(orc_build_ex(KEYS_U64, keys, NULL, 200, 8, 100, 3, 0, 0, NULL, 0, &size) == 5); /* seed cap */
    free(keys); free(offs); free(text);
    printf("oracle sanitizer run: ok\n");
    return 0;
}
