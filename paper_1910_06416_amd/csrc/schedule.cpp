// Process-wide table of seed-search schedules, one entry per (leaf, bucket)
// pair.  rs_autotune fills it by timing; callers may save entries and restore
// them in a later process with rs_schedule_set.
#include <map>
#include <mutex>
#include <utility>

#include "rs_host.h"

namespace rs {

namespace {
std::mutex g_mu;
std::map<std::pair<uint32_t, uint32_t>, rs_schedule> g_table;
}  // namespace

rs_schedule builtin_schedule(uint32_t leaf, uint64_t buckets, uint32_t bucket) {
    rs_schedule s{};
    s.stage_from = 9;
    s.group_max = 7;
    // Buckets of at most l keys (on average) are single leaves, and up to 2 l
    // keys a split and two leaves: a bucket's tree has no work for a second
    // wavefront (10^7 keys at l = 12, b = 9: 26.8 ms with 1 wavefront against
    // 47 ms with 4; l = 10, b = 16: 10.7 against 19.4 ms; 10^6 keys at l = 16,
    // b = 20: 213 against 542 ms with 8).
    if (bucket && bucket <= 2 * leaf) {
        s.waves = bucket <= leaf || buckets >= 4096 ? 1 : 2;
        return s;
    }
    // A launch with few buckets ends when its slowest bucket does, so more
    // wavefronts share each bucket's tree; with many buckets one wavefront per
    // bucket of small leaves keeps the most candidates in flight.  Measured on
    // MI355X at l = 8, b = 100: 4 wavefronts best up to ~1,000 buckets, 2 at
    // 10,000-30,000, 1 at 100,000; at l = 12, b = 1000, 8 at 100 buckets and
    // 4 from 10,000 on.  From l = 16 on, splits are heavy enough that their
    // shared search keeps 8 wavefronts busy (10^7 keys at l = 16, b = 2000:
    // 5.93 s against 6.11 s with 4).
    if (leaf <= 8)
        s.waves = buckets <= 4096 ? 4 : buckets <= 40000 ? 2 : 1;
    else if (leaf >= 16)
        s.waves = 8;
    else
        s.waves = leaf <= 12 && buckets <= 256 ? 8 : 4;
    return s;
}

bool schedule_valid(const rs_schedule& s) {
    const bool waves_ok = s.waves == 1 || s.waves == 2 || s.waves == 4 || s.waves == 8;
    return waves_ok && s.stage_from >= 2 && s.stage_from <= 25 && s.group_max >= 1 && s.group_max <= 7;
}

bool schedule_lookup(uint32_t leaf, uint32_t bucket, rs_schedule* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({leaf, bucket});
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

void schedule_store(uint32_t leaf, uint32_t bucket, const rs_schedule& s) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[{leaf, bucket}] = s;
}

}  // namespace rs

extern "C" int rs_schedule_get(uint32_t leaf, uint32_t bucket, rs_schedule* out) {
    rs::clear_error();
    if (!out) return rs::fail(RS_EINVAL, "NULL argument");
    rs_schedule s;
    if (!rs::schedule_lookup(leaf, bucket, &s))
        return rs::fail(RS_EINVAL, "no schedule for l=%u, b=%u", leaf, bucket);
    *out = s;
    return RS_OK;
}

extern "C" int rs_schedule_set(uint32_t leaf, uint32_t bucket, const rs_schedule* schedule) {
    rs::clear_error();
    if (!schedule) return rs::fail(RS_EINVAL, "NULL argument");
    if (leaf < 1 || leaf > rs::kMaxLeaf || bucket == 0) return rs::fail(RS_EINVAL, "l outside [1, 24] or b = 0");
    if (!rs::schedule_valid(*schedule))
        return rs::fail(RS_EINVAL, "schedule out of range (stage_from 2..25, group_max 1..7, waves 1/2/4/8)");
    rs::schedule_store(leaf, bucket, *schedule);
    return RS_OK;
}

extern "C" void rs_schedule_clear(void) {
    std::lock_guard<std::mutex> lk(rs::g_mu);
    rs::g_table.clear();
}
