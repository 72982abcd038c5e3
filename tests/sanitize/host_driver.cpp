// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host-only code (test infrastructure): the per-size tables and
// their cache (tables.cpp), the schedule table (schedule.cpp) and the launch
// chunking (launch.h), called as the C ABI exposes them, errors included.
// The device-side translation units need a GPU and are not part of this
// build; the two error helpers they define are given here.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "recsplit.h"
#include "rs_host.h"

namespace rs {
namespace {
thread_local std::string g_err;
}
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
void clear_error() { g_err.clear(); }
}  // namespace rs

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(2);                                                     \
        }                                                                     \
    } while (0)

int main() {
    // tables of every leaf size, growing caps (the cache reallocates), with and
    // without the Sec. 7.2 approximation and the non-minimal slack
    std::vector<uint32_t> r(70000), F(70000), N(70000), Q(70000), P(70000);
    for (uint32_t leaf = 1; leaf <= 24; leaf++) {
        for (uint32_t maxm : {1u, 7u, 100u, 1025u, 2600u, 5000u, 65535u}) {
            CHECK(rs_tables(leaf, maxm, r.data(), F.data(), N.data()) == RS_OK);
            CHECK(rs_tables_ex(leaf, maxm, maxm / 3 + 1, r.data(), F.data(), N.data()) == RS_OK);
            const int pk = rs_tables_packed(leaf, maxm, 0, P.data());
            CHECK(pk == RS_OK || pk == RS_EINVAL);
            const uint32_t slack = leaf <= 16 ? 255 : 85;
            CHECK(rs_tables_range(leaf, maxm, 0, slack, r.data(), F.data(), N.data(), Q.data()) == RS_OK);
            for (uint32_t m = 1; m <= maxm; m++) CHECK(Q[m] > Q[m - 1]);
        }
    }
    CHECK(rs_tables(0, 10, r.data(), F.data(), N.data()) == RS_EINVAL);
    CHECK(rs_tables(25, 10, r.data(), F.data(), N.data()) == RS_EINVAL);
    CHECK(rs_tables_range(24, 10, 0, 86, r.data(), F.data(), N.data(), Q.data()) == RS_EINVAL);
    CHECK(rs_tables_range(8, 10, 0, 256, r.data(), F.data(), N.data(), Q.data()) == RS_EINVAL);
    CHECK(rs_tables_packed(8, 10, 0, nullptr) == RS_EINVAL);
    // the table cache from several threads at once
    {
        std::vector<std::thread> th;
        for (int t = 0; t < 8; t++)
            th.emplace_back([t] {
                std::vector<uint32_t> a(9000), b(9000), c(9000);
                for (uint32_t k = 0; k < 40; k++)
                    CHECK(rs_tables_ex(1 + (t + k) % 24, 1000 + 200 * k, k % 3 ? 0 : 500, a.data(), b.data(),
                                       c.data()) == RS_OK);
            });
        for (auto& x : th) x.join();
    }
    // schedule table
    rs_schedule s{9, 7, 4, 0, 0, 0, 0}, got{};
    CHECK(rs_schedule_set(8, 100, &s) == RS_OK);
    CHECK(rs_schedule_get(8, 100, &got) == RS_OK && got.waves == 4);
    CHECK(rs_schedule_get(8, 101, &got) == RS_EINVAL);
    s.waves = 3;
    CHECK(rs_schedule_set(8, 100, &s) == RS_EINVAL);
    CHECK(rs_schedule_set(8, 100, nullptr) == RS_EINVAL);
    rs_schedule_clear();
    CHECK(rs_schedule_get(8, 100, &got) == RS_EINVAL);
    // launch chunks: cover every unit exactly once and fit every grid
    for (uint64_t units : {0ull, 1ull, 255ull, 16777215ull, 16777216ull, 67108864ull, 111111111ull, 4294967297ull})
        for (uint64_t threads : {64ull, 128ull, 256ull, 512ull})
            for (uint64_t per : {1ull, 16ull, 256ull}) {
                uint64_t next = 0;
                CHECK(rs::for_each_chunk(units, threads, per, [&](uint64_t first, uint64_t count, uint64_t blocks) {
                          CHECK(first == next && count >= 1 && rs::grid_fits(blocks, threads));
                          CHECK(blocks * per >= count);
                          next = first + count;
                          return 0;
                      }) == 0);
                CHECK(next == units);
            }
    std::printf("host sanitizer run: ok\n");
    return 0;
}
