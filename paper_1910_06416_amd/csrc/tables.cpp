// Host-side per-size tables of the splitting strategy (Sec. 5) and of the
// Golomb-Rice code (eq. (4), Sec. 6.2 and 7.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rs_internal.h"

namespace rs {

Strategy make_strategy(uint32_t leaf) {
    // s = max{2, ceil(0.35 l + 0.5)}; t = ceil(0.21 l + 0.9) for l >= 7, else 2.
    uint32_t s = std::max<uint32_t>(2u, (35u * leaf + 149u) / 100u);
    uint32_t t = leaf < 7 ? 2u : (21u * leaf + 189u) / 100u;
    return Strategy{leaf, s * leaf, s * t * leaf};
}

namespace {

// ln of the probability that one trial succeeds at a node of m keys:
// m!/m^m for a bijection, times prod k_j^k_j / k_j! for a split (eq. (2)).
// With slack, a leaf succeeds when its hash is injective into M =
// leaf_range(m) values: prod_{i<m} (M - i) / M.
double log_success(const Strategy& st, uint32_t m, uint32_t slack) {
    if (m <= st.leaf && slack) {
        const double M = (double)leaf_range(m, slack);
        return std::lgamma(M + 1.0) - std::lgamma(M - (double)m + 1.0) - (double)m * std::log(M);
    }
    double lp = std::lgamma((double)m + 1.0) - (double)m * std::log((double)m);
    if (m <= st.leaf) return lp;
    SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
    for (uint32_t j = 0; j < sh.fanout; j++) {
        double k = (double)(j + 1 == sh.fanout ? sh.last : sh.unit);
        lp += k * std::log(k) - std::lgamma(k + 1.0);
    }
    return lp;
}

// floor(lg x) for x >= 1 (lambda of Sec. 2).
uint32_t floor_lg(uint64_t x) { return 63u - (uint32_t)__builtin_clzll(x); }

// Integer approximation of the Golomb-Rice parameter of a large split
// (Sec. 7.2): with parts k_0..k_{f-1} of m keys, half of
// ((f-1) * 5 / 2, rounded down) + sum_i lambda(k_i + floor(k_i / 2)) - lambda(m),
// rounded down; a non-positive sum gives 0.
uint32_t rice_parameter_large(const Strategy& st, uint32_t m) {
    const SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
    int64_t sum = (int64_t)((sh.fanout - 1) * 5 / 2) - (int64_t)floor_lg(m);
    for (uint32_t j = 0; j < sh.fanout; j++) {
        const uint64_t k = j + 1 == sh.fanout ? sh.last : sh.unit;
        sum += floor_lg(k + k / 2);
    }
    return sum > 0 ? (uint32_t)(sum / 2) : 0u;
}

// Optimal Golomb-Rice parameter for a geometric source of parameter p (eq. (4)).
uint32_t rice_parameter(double p) {
    const double log_golden = std::log((1.0 + std::sqrt(5.0)) * 0.5);
    double e = std::log2(log_golden / -std::log1p(-p));
    return e > 0.0 ? (uint32_t)std::ceil(e) : 0u;
}

struct LeafTables {
    uint32_t cap = 0;
    uint32_t* data = nullptr;  // pinned host memory, never freed (copies may be in flight)
};

std::mutex g_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, LeafTables> g_cache;  // by (leaf, gr_max, slack)

// Lanes per candidate for the split search of a node of m keys: the 2^g
// minimising expected VALU work = steps * (keys per lane * cost per key +
// reduction), with steps = (expected trials + mean overshoot) / candidates
// per step; cost per key follows the counting mode the kernel uses.
uint32_t lanes_per_candidate(const Strategy& st, uint32_t m, double trials) {
    SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
    const uint32_t nt = sh.fanout - 1;
    uint32_t w = 0;
    while ((1u << w) <= m) w++;
    const bool onehot = sh.fanout == 4 && m < 256;
    const bool packed = !onehot && nt >= 4 && sh.fanout * w <= 64;
    const double per_key = 18.0 + (packed ? 6.0 : onehot ? 4.0 : 2.0 * nt);
    const double per_reduce = packed ? 4.0 : onehot ? 2.0 : 2.0 * nt;
    double best = 0;
    uint32_t best_g = 0;
    for (uint32_t g = 0; g <= 6; g++) {
        const double per_step = (double)(64u >> g);
        const double steps = std::max(1.0, (trials + (per_step - 1.0) / 2.0) / per_step);
        const double keys_per_lane = std::ceil((double)m / (double)(1u << g));
        const double cost = steps * (keys_per_lane * per_key + g * per_reduce + 12.0);
        if (g == 0 || cost < best) {
            best = cost;
            best_g = g;
        }
    }
    return best_g;
}

void fill(const Strategy& st, uint32_t cap, uint32_t* dst, uint32_t gr_max, uint32_t slack) {
    const size_t w = (size_t)cap + 1;
    uint32_t *r = dst, *F = dst + w, *N = dst + 2 * w, *G = dst + 3 * w, *P = dst + 4 * w, *Q = dst + 5 * w;
    uint32_t *S = dst + 6 * w, *C = dst + 7 * w;
    for (uint32_t m = 0; m <= cap; m++) {
        G[m] = 0;
        S[m] = C[m] = 0;
        if (m < 2) {
            r[m] = F[m] = N[m] = 0;
            P[m] = 0;
            Q[m] = m;
            continue;
        }
        const double lp = log_success(st, m, slack);
        r[m] = gr_max && m > st.leaf && m > gr_max ? rice_parameter_large(st, m) : rice_parameter(std::exp(lp));
        if (m > st.leaf) {
            const double trials = std::exp(-lp);
            G[m] = lanes_per_candidate(st, m, trials);
            if (trials * (double)m >= kCoopEvals) G[m] |= kCoopFlag;
        }
        F[m] = r[m];
        N[m] = 1;
        Q[m] = leaf_range(m, slack);
        if (m > st.leaf) {
            SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
            F[m] += (sh.fanout - 1) * F[sh.unit] + F[sh.last];
            N[m] += (sh.fanout - 1) * N[sh.unit] + N[sh.last];
            Q[m] = (sh.fanout - 1) * Q[sh.unit] + Q[sh.last];
            if (sh.unit < 65536u) S[m] = sh.unit | sh.fanout << 16;
            if (sh.unit > 1) C[m] = (uint32_t)(((1ull << 32) + sh.unit - 1) / sh.unit);
        }
        P[m] = r[m] < 32 && N[m] < 2048 && F[m] < 65536 ? r[m] | N[m] << 5 | F[m] << 16 : kNoPacked;
    }
}

}  // namespace

double expected_search_evals(uint32_t leaf, uint32_t bucket, uint64_t n) {
    if (n == 0 || bucket == 0 || leaf < 1 || leaf > kMaxLeaf) return 0.0;
    const Strategy st = make_strategy(leaf);
    const uint64_t nb = (n + bucket - 1) / bucket;
    const double lam = (double)n / (double)nb;
    const uint32_t kmax = (uint32_t)(lam + 12.0 * std::sqrt(lam) + 16.0);
    // E[m]: expected evaluations of the tree on m keys
    std::vector<double> E(kmax + 1, 0.0);
    for (uint32_t m = 2; m <= kmax; m++) {
        E[m] = std::exp(-log_success(st, m, 0)) * (double)m;
        if (m > st.leaf) {
            const SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
            E[m] += (double)(sh.fanout - 1) * E[sh.unit] + E[sh.last];
        }
    }
    // average over Poisson(lam) bucket sizes (summed from the mode both ways)
    double per_bucket = 0.0;
    const uint32_t mode = (uint32_t)lam;
    const double lp0 = (double)mode * std::log(lam) - lam - std::lgamma((double)mode + 1.0);
    double lp = lp0;
    for (uint32_t k = mode; k <= kmax; k++) {
        per_bucket += std::exp(lp) * E[k];
        lp += std::log(lam) - std::log((double)k + 1.0);
    }
    lp = lp0;
    for (uint32_t k = mode; k-- > 0;) {
        lp += std::log((double)k + 1.0) - std::log(lam);
        per_bucket += std::exp(lp) * E[k];
    }
    return per_bucket * (double)nb;
}

void fill_tables(uint32_t leaf, uint32_t maxm, uint32_t* dst, uint32_t gr_max, uint32_t slack) {
    fill(make_strategy(leaf), maxm, dst, gr_max, slack);
}

bool ranges_increasing(const uint32_t* Q, uint32_t maxm) {
    for (uint32_t m = 1; m <= maxm; m++)
        if (Q[m] <= Q[m - 1]) return false;
    return true;
}

bool packed_valid(const uint32_t* P, uint32_t maxm) {
    for (uint32_t m = 0; m <= maxm; m++)
        if (P[m] == kNoPacked) return false;
    return true;
}

TableView host_tables(uint32_t leaf, uint32_t maxm, uint32_t gr_max, uint32_t slack) {
    std::lock_guard<std::mutex> lock(g_mu);
    LeafTables& t = g_cache[{leaf, gr_max, slack}];
    if (t.data == nullptr || t.cap < maxm) {
        uint32_t cap = std::max<uint32_t>(maxm, std::max<uint32_t>(1024u, t.cap * 2));
        uint32_t* buf = nullptr;
        const size_t bytes = (size_t)kTableCount * (cap + 1) * sizeof(uint32_t);
        // pinned when a device is present (asynchronous uploads), plain otherwise
        if (hipHostMalloc((void**)&buf, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            buf = static_cast<uint32_t*>(std::malloc(bytes));
            if (!buf) return TableView{nullptr, 0};
        }
        fill(make_strategy(leaf), cap, buf, gr_max, slack);
        t.cap = cap;
        t.data = buf;  // the previous buffer is intentionally kept alive
    }
    return TableView{t.data, t.cap};
}

}  // namespace rs

extern "C" int rs_tables(uint32_t leaf, uint32_t maxm, uint32_t* r, uint32_t* F, uint32_t* N) {
    return rs_tables_ex(leaf, maxm, 0, r, F, N);
}

extern "C" int rs_tables_packed(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t* packed) {
    if (leaf < 1 || leaf > rs::kMaxLeaf || !packed) return RS_EINVAL;
    rs::TableView t = rs::host_tables(leaf, maxm, gr_table_max);
    if (!t.data) return RS_ENOMEM;
    if (!rs::packed_valid(t.P(), maxm)) return RS_EINVAL;
    for (uint32_t m = 0; m <= maxm; m++) packed[m] = t.P()[m];
    return RS_OK;
}

extern "C" int rs_tables_ex(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t* r, uint32_t* F,
                            uint32_t* N) {
    if (leaf < 1 || leaf > rs::kMaxLeaf || !r || !F || !N) return RS_EINVAL;
    rs::TableView t = rs::host_tables(leaf, maxm, gr_table_max);
    if (!t.data) return RS_ENOMEM;
    for (uint32_t m = 0; m <= maxm; m++) {
        r[m] = t.r()[m];
        F[m] = t.F()[m];
        N[m] = t.N()[m];
    }
    return RS_OK;
}

extern "C" int rs_tables_range(uint32_t leaf, uint32_t maxm, uint32_t gr_table_max, uint32_t leaf_slack, uint32_t* r,
                               uint32_t* F, uint32_t* N, uint32_t* Q) {
    if (leaf < 1 || leaf > rs::kMaxLeaf || leaf_slack > rs::kMaxSlack || !r || !F || !N || !Q) return RS_EINVAL;
    if (rs::leaf_range(leaf, leaf_slack) > rs::kMaxLeafRange) return RS_EINVAL;
    rs::TableView t = rs::host_tables(leaf, maxm, gr_table_max, leaf_slack);
    if (!t.data) return RS_ENOMEM;
    for (uint32_t m = 0; m <= maxm; m++) {
        r[m] = t.r()[m];
        F[m] = t.F()[m];
        N[m] = t.N()[m];
        Q[m] = t.Q()[m];
    }
    return RS_OK;
}
