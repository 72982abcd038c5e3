// Serving loop: construction and lookup requests of uneven sizes arrive over
// time and are run with continuous batching.
//
// Build requests wait in a first-in first-out queue.  A request is admitted
// when its estimated device footprint fits in the free part of the budget (a
// request is always admitted when nothing else is in flight, so an oversized
// one cannot wait forever).  Each build worker owns a stream; when it is free
// it takes the first request that may start and every admissible queued
// request of the same leaf size, and runs them as one batched construction
// (rs_build_batch).  Requests that arrive while a batch is on the device form
// the next worker's batch, so their work overlaps on the device.  A request
// whose modelled search time reaches kHeavySeconds is heavy: at most one
// batch with a heavy request is on the device at a time (two such searches
// sharing the compute units would each take about twice as long, which only
// delays both), while light requests start beside it.  A heavy search's
// workgroups take every CU they can get for seconds, so work launched beside
// it waits for CUs; with lookup_cus set, heavy batches run on a stream whose
// CU mask leaves that many CUs out, and light batches and lookups, on streams
// over every CU, always find those free.  A lookup worker runs lookup
// requests on its own stream.  All streams have the default priority.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rs_host.h"

namespace {

using Clock = std::chrono::steady_clock;

// Device bytes one build holds while in flight: the construction workspace
// (signatures, bucket ids, scattered keys, partition scratch, indices: 48 B per
// key), bucket arrays (~24 B per bucket) and the blob (< 1 B per key).
uint64_t build_footprint(uint64_t n, uint32_t bucket) {
    return 56 * n + 24 * (n / std::max<uint32_t>(bucket, 1) + 1) + (1u << 20);
}

// Modelled search time: expected hash evaluations (every key of every trial)
// at the rate that matches the measured searches on MI355X (10^7 keys: 6 s at
// l = 16, b = 2000 and 0.1 s at l = 12, b = 1000; the bijection search stops
// early in most trials, so it runs faster than one evaluation per slot).
constexpr double kEvalsPerSecond = 2.4e12;
constexpr double kHeavySeconds = 0.25;

struct Request {
    uint64_t ticket;
    bool is_build;
    rs_keys keys;
    uint32_t leaf = 0, bucket = 0;
    const rs_blob* blob = nullptr;
    uint64_t* ranks = nullptr;
    uint64_t footprint = 0;
    bool heavy = false;
    Clock::time_point arrival;
};

struct Result {
    bool done = false;
    int status = RS_OK;
    rs_blob* blob = nullptr;
    double latency_ms = 0;
    uint32_t batch_size = 0;
};

}  // namespace

struct rs_server {
    std::mutex mu;
    std::condition_variable cv_work;   // workers: new requests or freed budget
    std::condition_variable cv_done;   // waiters: a request completed
    std::deque<Request> builds, lookups;
    std::unordered_map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    uint64_t budget = 0, in_flight = 0, peak_in_flight = 0;
    uint64_t batches = 0, batched_requests = 0, max_batch = 0, concurrent = 0, max_concurrent = 0;
    uint32_t heavy_in_flight = 0;  // batches with a heavy request on the device
    uint32_t max_queue = 0;
    bool stopping = false;
    int device = 0;
    rs_options opts{};
    uint32_t lookup_cus = 0;
    std::vector<uint32_t> build_mask;  // CU mask of the build streams (empty: all CUs)
    std::vector<std::thread> workers;
};

namespace {

void finish(rs_server* s, const Request& r, int status, rs_blob* blob, uint32_t batch_size) {
    Result& res = s->results[r.ticket];
    res.done = true;
    res.status = status;
    res.blob = blob;
    res.batch_size = batch_size;
    res.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.arrival).count();
}

void build_worker(rs_server* s) {
    (void)hipSetDevice(s->device);
    // light batches on a stream over every CU; heavy ones, when CUs are kept
    // free of them, on a second stream whose CU mask leaves those out
    hipStream_t stream = nullptr, heavy_stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    if (!s->build_mask.empty() &&
        hipExtStreamCreateWithCUMask(&heavy_stream, (uint32_t)s->build_mask.size(), s->build_mask.data()) !=
            hipSuccess)
        heavy_stream = nullptr;
    for (;;) {
        std::vector<Request> batch;
        uint64_t bytes = 0;
        bool batch_heavy = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                // the first request that may start: a heavy one only while no other
                // heavy batch is on the device
                auto head = s->builds.begin();
                while (head != s->builds.end() && head->heavy && s->heavy_in_flight) ++head;
                if (head != s->builds.end()) {
                    // admit it (always, if nothing is in flight), then the later
                    // requests of its leaf size while the budget allows.  The
                    // requests of one batch finish together, so a batch holds one
                    // leaf size: a small l = 8 request never waits for an l = 16
                    // search of seconds; other leaf sizes go to the next free worker.
                    const uint32_t cls = head->leaf;
                    bool heavy_batch = false;
                    for (auto it = head; it != s->builds.end();) {
                        const Request& r = *it;
                        if (r.leaf != cls || (r.heavy && s->heavy_in_flight)) {
                            ++it;
                            continue;
                        }
                        const bool fits = s->in_flight + bytes + r.footprint <= s->budget;
                        if (!fits && !(s->in_flight == 0 && batch.empty())) {
                            if (batch.empty()) break;  // the head waits for budget
                            ++it;
                            continue;
                        }
                        bytes += r.footprint;
                        heavy_batch |= r.heavy;
                        batch.push_back(r);
                        it = s->builds.erase(it);
                    }
                    if (!batch.empty()) {
                        batch_heavy = heavy_batch;
                        break;
                    }
                }
                if (s->stopping && s->builds.empty()) break;
                s->cv_work.wait(lk);
            }
            if (batch.empty()) break;
            s->in_flight += bytes;
            s->heavy_in_flight += batch_heavy ? 1 : 0;
            s->peak_in_flight = std::max(s->peak_in_flight, s->in_flight);
            s->batches++;
            s->batched_requests += batch.size();
            s->max_batch = std::max<uint64_t>(s->max_batch, batch.size());
            s->concurrent++;
            s->max_concurrent = std::max(s->max_concurrent, s->concurrent);
        }
        const uint32_t count = (uint32_t)batch.size();
        std::vector<rs_keys> sets(count);
        std::vector<uint32_t> leafs(count), buckets(count);
        std::vector<rs_blob*> outs(count, nullptr);
        std::vector<int> status(count, RS_OK);
        for (uint32_t i = 0; i < count; i++) {
            sets[i] = batch[i].keys;
            leafs[i] = batch[i].leaf;
            buckets[i] = batch[i].bucket;
        }
        hipStream_t st = batch_heavy && heavy_stream ? heavy_stream : stream;
        int rc = rs_build_batch(sets.data(), count, leafs.data(), buckets.data(), &s->opts, st, outs.data(),
                                status.data());
        if (hipStreamSynchronize(st) != hipSuccess) rc = RS_EDEVICE;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (uint32_t i = 0; i < count; i++) {
                int code = status[i];
                if (code == RS_OK && !outs[i]) code = rc != RS_OK ? rc : RS_EDEVICE;
                finish(s, batch[i], code, outs[i], count);
            }
            s->in_flight -= bytes;
            s->heavy_in_flight -= batch_heavy ? 1 : 0;
            s->concurrent--;
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
    if (heavy_stream) (void)hipStreamDestroy(heavy_stream);
}

void lookup_worker(rs_server* s) {
    (void)hipSetDevice(s->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    for (;;) {
        Request r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return !s->lookups.empty() || s->stopping; });
            if (s->lookups.empty()) break;
            r = s->lookups.front();
            s->lookups.pop_front();
        }
        int rc = rs_lookup(r.blob, &r.keys, r.ranks, stream);
        if (rc == RS_OK && hipStreamSynchronize(stream) != hipSuccess) rc = RS_EDEVICE;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            finish(s, r, rc, nullptr, 1);
        }
        s->cv_done.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" int rs_server_create_ex(const rs_server_config* cfg, const rs_options* opts, rs_server** out) {
    rs::clear_error();
    if (!cfg || !out || cfg->hbm_budget_bytes == 0) return rs::fail(RS_EINVAL, "NULL argument or zero budget");
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    if (cfg->lookup_cus) {
        int nx = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            return rs::fail(RS_EDEVICE, "cannot read the compute-unit count");
        if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1) nx = 1;
        if (cfg->lookup_cus > (uint32_t)(ncu / nx))
            return rs::fail(RS_EINVAL, "lookup_cus exceeds the CUs of one XCD (%d)", ncu / nx);
    }
    rs_server* s = new (std::nothrow) rs_server;
    if (!s) return rs::fail(RS_ENOMEM, "host allocation failed");
    s->budget = cfg->hbm_budget_bytes;
    if (opts) s->opts = *opts;
    s->opts.flags &= ~(uint32_t)RS_OPT_TIMING;
    s->device = dev;
    if (cfg->lookup_cus) {
        // Every CU but lookup_cus of them, taken evenly from every XCD.  Whether
        // CU numbers run XCD by XCD or alternate between XCDs, CU
        // per*x + ((x + nxcd*j) mod per) lies on XCD x either way, so no XCD
        // loses more than its share (an XCD with fewer CUs would finish its
        // round-robin share of every launch last).
        int nx = 1;
        if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1) nx = 1;
        const uint32_t nxcd = (uint32_t)nx, per = (uint32_t)ncu / nxcd;
        std::vector<bool> left(ncu, false);
        for (uint32_t k = 0; k < cfg->lookup_cus; k++) {
            const uint32_t x = k % nxcd, j = k / nxcd;
            left[per * x + (x + nxcd * j) % per] = true;
        }
        s->lookup_cus = cfg->lookup_cus;
        s->build_mask.assign(((uint32_t)ncu + 31) / 32, 0u);
        for (uint32_t c = 0; c < (uint32_t)ncu; c++)
            if (!left[c]) s->build_mask[c / 32] |= 1u << (c % 32);
    }
    const uint32_t bw = cfg->build_workers;
    const uint32_t nw = std::max<uint32_t>(1, std::min<uint32_t>(bw ? bw : 2, 8));
    for (uint32_t i = 0; i < nw; i++) s->workers.emplace_back(build_worker, s);
    s->workers.emplace_back(lookup_worker, s);
    *out = s;
    return RS_OK;
}

extern "C" int rs_server_create(uint64_t hbm_budget_bytes, uint32_t build_workers, const rs_options* opts,
                                rs_server** out) {
    rs_server_config cfg{};
    cfg.hbm_budget_bytes = hbm_budget_bytes;
    cfg.build_workers = build_workers;
    return rs_server_create_ex(&cfg, opts, out);
}

static int submit(rs_server* s, Request r, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return rs::fail(RS_EBUSY, "server is stopping");
    r.ticket = s->next_ticket++;
    r.arrival = Clock::now();
    s->results[r.ticket] = Result{};
    if (r.is_build) s->builds.push_back(r);
    else s->lookups.push_back(r);
    s->max_queue = std::max<uint32_t>(s->max_queue, (uint32_t)(s->builds.size() + s->lookups.size()));
    *ticket = r.ticket;
    s->cv_work.notify_all();
    return RS_OK;
}

extern "C" int rs_server_submit_build(rs_server* s, const rs_keys* keys, uint32_t leaf, uint32_t bucket,
                                      uint64_t* ticket) {
    rs::clear_error();
    if (!s || !keys || !ticket) return rs::fail(RS_EINVAL, "NULL argument");
    Request r;
    r.is_build = true;
    r.keys = *keys;
    r.leaf = leaf;
    r.bucket = bucket;
    r.footprint = build_footprint(keys->n, bucket);
    r.heavy = rs::expected_search_evals(leaf, bucket, keys->n) / kEvalsPerSecond >= kHeavySeconds;
    return submit(s, r, ticket);
}

extern "C" int rs_server_submit_lookup(rs_server* s, const rs_blob* blob, const rs_keys* queries, uint64_t* ranks_dev,
                                       uint64_t* ticket) {
    rs::clear_error();
    if (!s || !blob || !queries || !ticket) return rs::fail(RS_EINVAL, "NULL argument");
    Request r;
    r.is_build = false;
    r.keys = *queries;
    r.blob = blob;
    r.ranks = ranks_dev;
    return submit(s, r, ticket);
}

static int take(rs_server* s, uint64_t ticket, bool wait, int* done, int* status, rs_blob** blob, double* latency,
                uint32_t* batch_size) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return rs::fail(RS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (wait) s->cv_done.wait(lk, [&] { return s->results[ticket].done; });
    it = s->results.find(ticket);
    if (done) *done = it->second.done;
    if (!it->second.done) return RS_OK;
    if (status) *status = it->second.status;
    if (blob) *blob = it->second.blob;
    if (latency) *latency = it->second.latency_ms;
    if (batch_size) *batch_size = it->second.batch_size;
    s->results.erase(it);  // a completed ticket is handed out once
    return RS_OK;
}

extern "C" int rs_server_poll(rs_server* s, uint64_t ticket, int* done, int* status, rs_blob** blob,
                              double* latency_ms, uint32_t* batch_size) {
    rs::clear_error();
    if (!s || !done) return rs::fail(RS_EINVAL, "NULL argument");
    return take(s, ticket, false, done, status, blob, latency_ms, batch_size);
}

extern "C" int rs_server_wait(rs_server* s, uint64_t ticket, int* status, rs_blob** blob, double* latency_ms,
                              uint32_t* batch_size) {
    rs::clear_error();
    if (!s) return rs::fail(RS_EINVAL, "NULL argument");
    int done = 0;
    return take(s, ticket, true, &done, status, blob, latency_ms, batch_size);
}

extern "C" int rs_server_get_stats(rs_server* s, rs_server_stats* out) {
    if (!s || !out) return rs::fail(RS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->batches = s->batches;
    out->batched_requests = s->batched_requests;
    out->max_batch = s->max_batch;
    out->max_concurrent_batches = s->max_concurrent;
    out->peak_in_flight_bytes = s->peak_in_flight;
    out->budget_bytes = s->budget;
    out->max_queue = s->max_queue;
    out->lookup_cus = s->lookup_cus;
    return RS_OK;
}

extern "C" void rs_server_destroy(rs_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->results)
        if (kv.second.blob) rs_blob_free(kv.second.blob);  // completed but never collected
    delete s;
}
