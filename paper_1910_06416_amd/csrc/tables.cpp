// Host-side per-size tables of the splitting strategy (Sec. 5) and of the
// Golomb-Rice code (eq. (4), Sec. 6.2 and 7.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
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
double log_success(const Strategy& st, uint32_t m) {
    double lp = std::lgamma((double)m + 1.0) - (double)m * std::log((double)m);
    if (m <= st.leaf) return lp;
    SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
    for (uint32_t j = 0; j < sh.fanout; j++) {
        double k = (double)(j + 1 == sh.fanout ? sh.last : sh.unit);
        lp += k * std::log(k) - std::lgamma(k + 1.0);
    }
    return lp;
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
std::map<uint32_t, LeafTables> g_cache;

void fill(const Strategy& st, uint32_t cap, uint32_t* r, uint32_t* F, uint32_t* N) {
    for (uint32_t m = 0; m <= cap; m++) {
        if (m < 2) {
            r[m] = F[m] = N[m] = 0;
            continue;
        }
        r[m] = rice_parameter(std::exp(log_success(st, m)));
        F[m] = r[m];
        N[m] = 1;
        if (m > st.leaf) {
            SplitShape sh = split_shape(m, st.leaf, st.lower, st.upper);
            F[m] += (sh.fanout - 1) * F[sh.unit] + F[sh.last];
            N[m] += (sh.fanout - 1) * N[sh.unit] + N[sh.last];
        }
    }
}

}  // namespace

TableView host_tables(uint32_t leaf, uint32_t maxm) {
    std::lock_guard<std::mutex> lock(g_mu);
    LeafTables& t = g_cache[leaf];
    if (t.data == nullptr || t.cap < maxm) {
        uint32_t cap = std::max<uint32_t>(maxm, std::max<uint32_t>(1024u, t.cap * 2));
        uint32_t* buf = nullptr;
        const size_t bytes = 3ull * (cap + 1) * sizeof(uint32_t);
        // pinned when a device is present (asynchronous uploads), plain otherwise
        if (hipHostMalloc((void**)&buf, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            buf = static_cast<uint32_t*>(std::malloc(bytes));
            if (!buf) return TableView{nullptr, 0};
        }
        fill(make_strategy(leaf), cap, buf, buf + cap + 1, buf + 2 * (cap + 1));
        t.cap = cap;
        t.data = buf;  // the previous buffer is intentionally kept alive
    }
    return TableView{t.data, t.cap};
}

}  // namespace rs

extern "C" int rs_tables(uint32_t leaf, uint32_t maxm, uint32_t* r, uint32_t* F, uint32_t* N) {
    if (leaf < 1 || leaf > rs::kMaxLeaf || !r || !F || !N) return RS_EINVAL;
    rs::TableView t = rs::host_tables(leaf, maxm);
    if (!t.data) return RS_ENOMEM;
    for (uint32_t m = 0; m <= maxm; m++) {
        r[m] = t.r()[m];
        F[m] = t.F()[m];
        N[m] = t.N()[m];
    }
    return RS_OK;
}
