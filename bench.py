#!/usr/bin/env python3
"""RecSplit construction throughput on one MI355X.

Workload (one step): build the minimal perfect hash function of 10,000,000
random printable-ASCII strings of 8-32 bytes with leaf size l=8 and bucket
size b=100, then look all 10,000,000 keys up in shuffled order.  Inputs are
seeded and synthetic and already resident in HBM when the timed region
starts.  Also reported: one build of 10,000,000 random 64-bit keys at l=16,
b=2000 (the high-compression point), bits/key, p50/p99 build latency, the
seed-search kernel's share of the VALU integer peak, and the CPU oracle timed
on a bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Expected hash evaluations per key of the construction (model of the paper's
# analysis: leaf trials m^m/m! with early exit at the first collision, split
# trials 1/p of eq. (2) with m evaluations each, node census from the strategy
# averaged over Poisson(b) bucket sizes).
EVALS_PER_KEY = {(8, 100): 494.0, (12, 1000): 1.39e4, (16, 2000): 8.90e5}
# VALU instructions of one hash evaluation in the cheapest form the search
# kernel executes (the unrolled bijection loop: signature + stream offset,
# two xor-shift/multiply rounds keeping the upper word, range reduction and
# the bitmask update).  Every one of these issues at full rate on gfx950
# (measured), so this is also the number of full-rate VALU slots.
VALU_SLOTS_PER_EVAL = 18.0
# HBM bytes of one k_search launch on the 10M-string workload, from rocprofv3
# FETCH_SIZE (x2.0) / WRITE_SIZE (x1.0), the factors a 1 GiB device copy gives
# (51,438 and 29,034 KiB for the current kernel); to be set to None whenever the
# search kernel changes until re-measured.
SEARCH_TRAFFIC_BYTES = 135.0e6
# VALU lane-instructions that k_lookup_bytes executes per string query (rocprofv3
# SQ_INSTS_VALU x 64 / queries on the 10M-string workload): lookups are bound by
# the VALU and by dependent loads, not by HBM.
LOOKUP_VALU_PER_QUERY = 1437.0
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz full-rate 32-bit VALU lane-ops.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def cpu_baseline(keys_host, n_sample, leaf, bucket, gpu_blob=None):
    """The CPU oracle on the string workload: single-threaded on the first
    n_sample keys, and bucket-parallel (the oracle's own per-bucket tree loop
    in one process per host core, at most 16) on all keys, whose bytes are
    compared with the GPU's structure."""
    import oracle
    from oracle import parallel

    data, offsets = keys_host
    n = len(offsets) - 1
    sub_off = offsets[: n_sample + 1].copy()
    sub = (data[: int(sub_off[-1])], sub_off)
    t0 = time.perf_counter()
    blob = oracle.build(sub, leaf, bucket)
    dt = time.perf_counter() - t0
    workers = parallel.default_workers()
    pblob, timing = parallel.build(keys_host, leaf, bucket, workers=workers)
    return {"value": n_sample / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample:,} of the {n:,} strings, l={leaf}, b={bucket}, "
                      f"fingerprint to serialized blob in memory ({dt:.1f} s, one thread)",
            "bits_per_key": 8.0 * len(blob) / n_sample,
            "all_cores": {"value": n / timing["wall_s"], "unit": "keys/s", "cores": timing["workers"],
                          "sample": f"all {n:,} strings; trees of bucket ranges in {timing['workers']} processes, "
                                    f"layout and encoding in one ({timing['wall_s']:.1f} s wall, "
                                    f"{timing['tree_core_s']:.1f} core-s of trees)",
                          "timing": timing,
                          "same_bytes_as_gpu": None if gpu_blob is None else pblob == gpu_blob}}


def cpu_baseline_l16(keys_host, n_sub, leaf, bucket, n_full, single_buckets):
    """The oracle at l=16, b=2000 on the first n_sub keys of the workload
    (n_sub / b buckets): every bucket's tree in one process per host core (at
    most 16), and a few buckets one after another in one process; the rates
    are extrapolated to n_full keys (construction time is linear in n, Sec. 5),
    with standard errors from the per-bucket times."""
    import numpy as np

    from oracle import parallel

    import oracle

    sub = keys_host[:n_sub]
    nb = -(-n_sub // bucket)
    layout = oracle.bucket_layout(sub, nb)
    s_ = layout[1]
    sizes = (s_[1:] - s_[:-1]).astype(np.float64)
    workers = parallel.default_workers()
    t0 = time.perf_counter()
    res = parallel.bucket_trees(sub, leaf, bucket, range(nb), workers=workers, layout=layout)
    wall = time.perf_counter() - t0
    per_key = np.array([res[i][2] / sizes[i] for i in range(nb)])  # core-s per key of each bucket
    # single thread: the first buckets one after another in one process
    t1 = time.perf_counter()
    one = parallel.bucket_trees(sub, leaf, bucket, range(single_buckets), workers=1, layout=layout)
    wall1 = time.perf_counter() - t1
    per_key1 = np.array([one[i][2] / sizes[i] for i in range(single_buckets)])
    rate1 = float(sizes[:single_buckets].sum() / sum(one[i][2] for i in range(single_buckets)))
    rate_all = n_sub / wall

    def proj(per_key_arr, scale):
        se = float(per_key_arr.std(ddof=1) / np.sqrt(len(per_key_arr))) if len(per_key_arr) > 1 else None
        return (float(per_key_arr.mean()) * n_full / scale, None if se is None else se * n_full / scale)

    p1, se1 = proj(per_key1, 1.0)
    pa, sea = proj(per_key, workers)
    return {
        "single_thread": {"value": rate1, "unit": "keys/s", "cores": 1,
                          "sample": f"{single_buckets} buckets ({int(sizes[:single_buckets].sum()):,} keys) of the "
                                    f"first {n_sub:,} keys, one after another ({wall1:.1f} s)",
                          "projected_s_for_n": p1, "projected_se_s": se1},
        "all_cores": {"value": rate_all, "unit": "keys/s", "cores": workers,
                      "sample": f"all {nb} buckets of the first {n_sub:,} keys, one per task in {workers} processes "
                                f"({wall:.1f} s wall)",
                      "projected_s_for_n": n_full / rate_all, "projected_se_s": sea,
                      "per_bucket_core_s_mean": float(np.mean([res[i][2] for i in range(nb)]))},
        "n": n_full, "leaf": leaf, "bucket": bucket,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000, help="keys of the l=8, b=100 string workload")
    ap.add_argument("--l16-n", type=int, default=10_000_000, help="keys of the l=16, b=2000 build (0: skip)")
    ap.add_argument("--latency-builds", type=int, default=30, help="repeated 100,000-key builds for p50/p99")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000, help="oracle sample size (0: skip)")
    ap.add_argument("--cpu-l16-single", type=int, default=3,
                    help="buckets of the l=16 oracle leg timed one after another in one process")
    ap.add_argument("--l16-builds", type=int, default=3, help="timed l=16, b=2000 builds (p50/p99)")
    ap.add_argument("--workload", choices=["single", "batch", "serve", "table"], default="single",
                    help="single: 10M strings l=8 b=100 (+ l=16 point); batch: 4096 uneven builds, l=12 b=1000; "
                         "serve: Poisson stream of uneven build requests and 1M-key lookups; "
                         "table: the paper's Table tab:1M rows (10^6 random keys at four (l, b) points)")
    ap.add_argument("--table-n", type=int, default=1_000_000, help="table: keys per row")
    ap.add_argument("--batch-builds", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=1, help="timed batched calls of the 4096-build workload")
    ap.add_argument("--no-batch", action="store_true", help="single workload: skip the batched-build summary")
    ap.add_argument("--no-serve", action="store_true", help="single workload: skip the serving summary")
    ap.add_argument("--serve-requests", type=int, default=40, help="single workload: requests of the serving run")
    ap.add_argument("--serve-load", type=float, default=1.2,
                    help="single workload: offered load of the serving run (above 1 saturates the plain path)")
    ap.add_argument("--requests", type=int, default=60, help="serve: build requests")
    ap.add_argument("--load", type=float, default=0.6, help="serve: offered load (fraction of modelled capacity)")
    ap.add_argument("--lookup-cus", type=int, default=0,
                    help="serve: compute units the build streams leave to lookups (0: none)")
    ap.add_argument("--tune-ms", type=float, default=3000.0,
                    help="autotuner budget (search milliseconds) per (l, b) pair; l=16 pairs get ten times this")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in search schedule")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scales HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the construction of one "
              "structure runs on one device; see the design notes for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_06416_amd import inputs, recsplit

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    recsplit.lib()
    if args.workload == "batch":
        print(json.dumps(bench_batch(args, args.steps)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, args.requests, args.load)), flush=True)
        return
    if args.workload == "table":
        print(json.dumps(bench_table(args)), flush=True)
        return
    n, leaf, bucket = args.n, 8, 100

    log(f"[bench] generating {n:,} ASCII strings (seed 2) and the lookup order (seed 3)")
    keys_host = inputs.ascii_keys(n, 2)
    order = inputs.permutation(n, 3)
    queries_host = inputs.gather_strings(keys_host, order)
    dk = recsplit.device_keys(keys_host)
    dq = recsplit.device_keys(queries_host)
    ranks = torch.empty(n, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    schedules = {}
    if not args.no_tune:
        schedules["l8_b100"] = tune(recsplit, leaf, bucket, args, n)
    tuned = not args.no_tune

    for w in range(args.warmup):
        blob = recsplit.build(dk, leaf, bucket, timing=True, tuned=tuned)
        recsplit.lookup(blob, dq, out=ranks)
        torch.cuda.synchronize()
        blob.free()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")

    build_s, lookup_ms, search_ms, stats = [], [], [], None
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        tb = time.perf_counter()
        blob = recsplit.build(dk, leaf, bucket, timing=True, tuned=tuned)  # waits for its stream (timing mode)
        build_s.append(time.perf_counter() - tb)
        stats = recsplit.last_build_stats()
        search_ms.append(stats["ms_search"])
        ev0.record()
        recsplit.lookup(blob, dq, out=ranks)
        ev1.record()
        ev1.synchronize()
        lookup_ms.append(ev0.elapsed_time(ev1))
        if k + 1 < args.steps:
            blob.free()
        log(f"[bench] step {k + 1}/{args.steps}: build {build_s[-1] * 1e3:.2f} ms "
            f"(search {search_ms[-1]:.2f} ms), lookup {lookup_ms[-1]:.2f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    # the timed output is an MPHF: lookups of all keys are a permutation of [0, n)
    srt, _ = torch.sort(ranks)
    assert torch.equal(srt, torch.arange(n, dtype=torch.int64, device="cuda")), "lookups are not a bijection"
    bits_per_key = blob.bits_per_key()
    gpu_blob = blob.to_bytes() if args.cpu_sample else None
    blob.free()

    mean_build = float(np.mean(build_s))
    value = n / mean_build
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    mean_search = float(np.mean(search_ms))
    alg_evals = EVALS_PER_KEY[(leaf, bucket)] * n
    evals_per_s = alg_evals / (mean_search * 1e-3)
    lookup_rate = n / (float(np.mean(lookup_ms)) * 1e-3)
    lookup_bytes = int(queries_host[0].nbytes + queries_host[1].nbytes + 8 * n)

    result = {
        "metric": "keys/s built at l=8,b=100 and l=16,b=2000; bits/key; p99 build latency",
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "10M random ASCII strings (8-32 B), l=8, b=100, build + 10M shuffled lookups",
                   "n": n, "leaf": leaf, "bucket": bucket},
        "build_ms": mean_build * 1e3,
        "build_p50_ms": percentile(build_s, 50) * 1e3,
        "build_p99_ms": percentile(build_s, 99) * 1e3,
        "bits_per_key": bits_per_key,
        "search_ms": mean_search,
        "phase_ms": {k: stats[k] for k in ("ms_signature", "ms_scatter", "ms_search", "ms_offsets", "ms_fill")},
        "lookup_ms": float(np.mean(lookup_ms)),
        "lookup_keys_per_s": lookup_rate,
        "lookup_hbm": {"achieved": lookup_bytes / (float(np.mean(lookup_ms)) * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "bytes_per_query": lookup_bytes / n},
        # executed (not algorithmic) VALU work of the lookup kernel against the VALU peak
        "lookup_valu": {"achieved": lookup_rate * LOOKUP_VALU_PER_QUERY / 1e12, "peak": VALU_PEAK_TOPS,
                        "unit": "T lane-ops/s", "frac": lookup_rate * LOOKUP_VALU_PER_QUERY / 1e12 / VALU_PEAK_TOPS,
                        "valu_per_query": LOOKUP_VALU_PER_QUERY},
    }
    slots = VALU_SLOTS_PER_EVAL
    result["roofline"] = {
        "kernel": "k_search",
        "bound": "alu",
        "achieved": evals_per_s * slots / 1e12 if slots else None,
        "peak": VALU_PEAK_TOPS,
        "unit": "T lane-ops/s",
        "frac": evals_per_s * slots / 1e12 / VALU_PEAK_TOPS if slots else None,
        "traffic": SEARCH_TRAFFIC_BYTES,
        "algorithmic_evals_per_launch": alg_evals,
        "evals_per_s": evals_per_s,
        "valu_slots_per_eval": slots,
    }

    # latency over repeated 100,000-key builds (64-bit keys, l=8, b=100).  They
    # take the built-in schedule, whose wavefronts per bucket follow the call's
    # bucket count; the table's (8, 100) entry was tuned for the 10^7-key build.
    if args.latency_builds:
        small = recsplit.device_keys(inputs.u64_keys(100_000, 1))
        lat = []
        for i in range(args.latency_builds + 3):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            b = recsplit.build(small, 8, 100)
            torch.cuda.synchronize()  # until the blob is complete (the call returns before its last kernels end)
            dt = time.perf_counter() - tb
            b.free()
            if i >= 3:
                lat.append(dt)
        result["latency_100k_l8_b100_ms"] = {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3,
                                             "builds": len(lat), "schedule": "built-in"}
        log(f"[bench] 100k-key build latency p50 {result['latency_100k_l8_b100_ms']['p50']:.3f} ms")
        # the same builds through a captured plan (one graph launch and one wait per build)
        plan = recsplit.Plan([small], 8, 100)
        for b in plan.first:
            b.free()
        plat = []
        for i in range(args.latency_builds + 3):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            blobs, _ = plan.run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - tb
            blobs[0].free()
            if i >= 3:
                plat.append(dt)
        result["latency_100k_l8_b100_plan_ms"] = {"p50": percentile(plat, 50) * 1e3,
                                                  "p99": percentile(plat, 99) * 1e3, "builds": len(plat),
                                                  "plan": plan.info()}
        plan.close()
        log(f"[bench] 100k-key plan-run latency p50 {result['latency_100k_l8_b100_plan_ms']['p50']:.3f} ms")

    # high-compression point: 10M random 64-bit keys, l=16, b=2000 (one build)
    if args.l16_n:
        k16 = inputs.u64_keys(args.l16_n, 4)
        d16 = recsplit.device_keys(k16)
        if tuned:
            schedules["l16_b2000"] = tune(recsplit, 16, 2000, args, args.l16_n)
        warm = recsplit.build(recsplit.device_keys(inputs.u64_keys(4000, 5)), 16, 2000, timing=True, tuned=tuned)
        warm.free()
        t16, s16 = [], []
        for k in range(max(1, args.l16_builds)):
            log(f"[bench] l=16 b=2000 build {k + 1}/{args.l16_builds} of {args.l16_n:,} keys ...")
            torch.cuda.synchronize()
            tb = time.perf_counter()
            b16 = recsplit.build(d16, 16, 2000, timing=True, tuned=tuned)
            t16.append(time.perf_counter() - tb)
            st16 = recsplit.last_build_stats()
            s16.append(st16["ms_search"])
            bpk16 = b16.bits_per_key()
            r16 = recsplit.lookup(b16, d16)
            srt16, _ = torch.sort(r16)
            assert torch.equal(srt16, torch.arange(args.l16_n, dtype=torch.int64, device="cuda"))
            b16.free()
            del r16, srt16
        dt16 = float(np.mean(t16))
        ev16 = EVALS_PER_KEY[(16, 2000)] * args.l16_n / (float(np.mean(s16)) * 1e-3)
        result["l16_b2000"] = {
            "n": args.l16_n, "keys_per_s": args.l16_n / dt16, "build_s": dt16, "builds": len(t16),
            "build_p50_s": percentile(t16, 50), "build_p99_s": percentile(t16, 99), "build_s_all": t16,
            "search_ms": float(np.mean(s16)), "bits_per_key": bpk16, "evals_per_s": ev16,
            "valu_frac": ev16 * slots / 1e12 / VALU_PEAK_TOPS if slots else None,
        }
        log(f"[bench] l=16: {args.l16_n / dt16:,.0f} keys/s, {bpk16:.4f} bits/key")

    if not args.no_batch:
        log("[bench] batched builds: 4096 builds, l=12, b=1000 (batched call, plan, one call per build)")
        bb = bench_batch(args, args.batch_steps)
        result["batch_4096_l12_b1000"] = {k: bb[k] for k in (
            "value", "unit", "batched_s", "plain_s", "speedup_vs_plain", "plan_run_s", "plain_keys_per_s",
            "bits_per_key", "search_ms", "plain_build_latency_ms", "roofline", "config")}
    if not args.no_serve:
        log(f"[bench] serving: {args.serve_requests} requests at offered load {args.serve_load}")
        sv = bench_serve(args, args.serve_requests, args.serve_load, tuned=False)
        result["serve"] = {k: sv[k] for k in ("value", "unit", "served", "plain", "config", "requests")}
        result["serve"]["p99_vs_plain"] = sv["plain"]["p99_ms"] / sv["served"]["p99_ms"]
        result["serve"]["makespan_vs_plain"] = sv["plain"]["makespan_s"] / sv["served"]["makespan_s"]
    result["schedules"] = schedules if tuned else "built-in"
    if args.cpu_sample:
        log(f"[bench] CPU oracle on {args.cpu_sample:,} keys (one thread) and on all keys (all cores) ...")
        result["cpu_baseline"] = cpu_baseline(keys_host, args.cpu_sample, leaf, bucket, gpu_blob)
        result["cpu_baseline"]["host_cpu"] = _cpu_model()
        if args.l16_n:
            log("[bench] CPU oracle at l=16, b=2000 on the first 100,000 keys ...")
            result["cpu_baseline"]["l16_b2000"] = cpu_baseline_l16(k16, min(100_000, args.l16_n), 16, 2000,
                                                                   args.l16_n, args.cpu_l16_single)

    print(json.dumps(result), flush=True)


def bench_batch(args, steps):
    """4096 independent builds of uniform random 64-bit keys, sizes log-uniform
    in [1e3, 1e6], l=12, b=1000: one batched call against one call per build."""
    import numpy as np
    import torch

    from paper_1910_06416_amd import inputs, recsplit

    leaf, bucket = 12, 1000
    sizes = inputs.log_uniform_sizes(args.batch_builds, 5, 1e3, 1e6)
    log(f"[bench] batch: {len(sizes)} builds, {int(sizes.sum()):,} keys; generating keys")
    rng_keys = inputs.u64_keys(int(sizes.sum()), 5)  # disjoint slices: every build's keys are distinct
    offs = np.concatenate([[0], np.cumsum(sizes)])
    dall = recsplit.device_keys(rng_keys)
    sets = [dall[int(offs[i]):int(offs[i + 1])] for i in range(len(sizes))]
    total = int(sizes.sum())
    torch.cuda.synchronize()

    tuned = not args.no_tune
    schedule = tune(recsplit, leaf, bucket, args, total) if tuned else "built-in"
    # batched: warm-up on a small slice, then the timed call(s)
    recsplit.build_batch(sets[:8], leaf, bucket, tuned=tuned)
    times, stats = [], None
    for k in range(max(1, steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blobs, status = recsplit.build_batch(sets, leaf, bucket, timing=True, tuned=tuned)
        dt = time.perf_counter() - t0
        stats = recsplit.last_build_stats()
        assert all(x == 0 for x in status), "batched build failed"
        times.append(dt)
        log(f"[bench] batched call {k + 1}: {dt:.3f} s (search {stats['ms_search']:.1f} ms)")
        bits = sum(b.nbytes for b in blobs) * 8 / total
        # spot check: some builds' lookups are bijections
        for i in list(range(0, len(sizes), max(1, len(sizes) // 16))):
            r = recsplit.lookup(blobs[i], sets[i])
            srt, _ = torch.sort(r)
            assert torch.equal(srt, torch.arange(int(sizes[i]), dtype=torch.int64, device="cuda"))
        for b in blobs:
            b.free()
        del blobs

    # the same batch through a captured plan: one graph launch per rebuild
    log("[bench] batched call through a captured plan")
    plan = recsplit.Plan(sets, leaf, bucket, tuned=tuned)
    for b in plan.first:
        if b is not None:
            b.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pblobs, pstatus = plan.run()
    plan_s = time.perf_counter() - t0
    assert all(x == 0 for x in pstatus), "plan run failed"
    plan_info = plan.info()
    for b in pblobs:
        b.free()
    plan.close()
    log(f"[bench] plan run: {plan_s:.3f} s ({plan_info})")

    # plain path: one rs_build call per build, in order, each with the built-in
    # schedule (its wavefronts per bucket follow that build's bucket count, which
    # suits a lone build better than the schedule tuned for the whole batch)
    log("[bench] plain path: one call per build")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    for i, s_ in enumerate(sets):
        tb = time.perf_counter()
        b = recsplit.build(s_, leaf, bucket)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - tb)
        b.free()
    plain = time.perf_counter() - t0
    batched = float(np.mean(times))
    alg = EVALS_PER_KEY[(leaf, bucket)] * total
    ev = alg / (stats["ms_search"] * 1e-3)
    return {
        "metric": "keys/s built, 4096 uneven builds (batched vs one call per build)",
        "value": total / batched, "unit": "keys/s", "n_gpus": 1, "steps": len(times), "warmup": 1,
        "ms_per_step": batched * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{len(sizes)} builds of uniform random 64-bit keys, sizes log-uniform in "
                               f"[1e3, 1e6], l={leaf}, b={bucket}", "keys": total},
        "batched_s": batched, "plain_s": plain, "speedup_vs_plain": plain / batched,
        "plan_run_s": plan_s, "plan": plan_info,
        "plain_keys_per_s": total / plain, "bits_per_key": bits, "search_ms": stats["ms_search"],
        "phase_ms": {k: stats[k] for k in ("ms_signature", "ms_scatter", "ms_search", "ms_offsets", "ms_fill")},
        "plain_build_latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3},
        "schedule": schedule,
        "roofline": {"kernel": "k_search", "bound": "alu", "achieved": ev * VALU_SLOTS_PER_EVAL / 1e12,
                     "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                     "frac": ev * VALU_SLOTS_PER_EVAL / 1e12 / VALU_PEAK_TOPS, "traffic": None,
                     "algorithmic_evals_per_launch": alg, "evals_per_s": ev},
    }


# Expected hash evaluations per key by leaf size (leaf searches dominate; the
# bucket size moves these by a few tens of percent), used to set arrival rates.
EVALS_BY_LEAF = {8: 494.0, 12: 1.39e4, 16: 8.90e5}


def bench_serve(args, requests, load, tuned=None):
    """Poisson arrivals of build requests (sizes log-uniform in [1e4, 1e7], l in
    {8, 12, 16}, b in {100, 1000, 2000}) interleaved with 1M-key lookup batches,
    served with continuous batching; the same arrival schedule replayed through
    one rs_build call per request in arrival order."""
    import numpy as np
    import torch

    from paper_1910_06416_amd import inputs, recsplit

    rng = np.random.Generator(np.random.PCG64(6))
    R = requests
    sizes = inputs.log_uniform_sizes(R, 6, 1e4, 1e7)
    leafs = rng.choice([8, 12, 16], size=R)
    buckets = rng.choice([100, 1000, 2000], size=R)
    work_s = np.array([EVALS_BY_LEAF[int(l)] * int(n) for n, l in zip(sizes, leafs)]) / 1.3e12
    rate = load / work_s.mean()
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=R))
    lookup_times = np.cumsum(rng.exponential(1.0 / rate, size=R))
    total = int(sizes.sum())
    log(f"[bench] serve: {R} requests, {total:,} keys, modelled work {work_s.sum():.1f} s, "
        f"rate {rate:.2f}/s over {arrivals[-1]:.1f} s")
    allkeys = recsplit.device_keys(inputs.u64_keys(total, 6))
    offs = np.concatenate([[0], np.cumsum(sizes)])
    sets = [allkeys[int(offs[i]):int(offs[i + 1])] for i in range(R)]
    tuned = (not args.no_tune) if tuned is None else tuned
    schedules = {}
    if tuned:
        for l_ in (8, 12, 16):
            for b_ in (100, 1000, 2000):
                schedules[f"l{l_}_b{b_}"] = tune(recsplit, l_, b_, args, 2e6)
    warm = recsplit.build(sets[0][:1000], 16, 100, tuned=tuned)
    warm.free()
    torch.cuda.synchronize()

    # served run
    srv = recsplit.Server(budget_bytes=96 << 30, build_workers=3, tuned=tuned, lookup_cus=args.lookup_cus)
    t0 = time.perf_counter()
    tickets, lookups, done_blobs = [None] * R, [], {}
    li = 0
    for i in range(R):
        while li < R and lookup_times[li] < arrivals[i]:
            if done_blobs:  # a 1M-key lookup batch against a completed build
                j = sorted(done_blobs)[li % len(done_blobs)]
                q = sets[j][torch.randint(0, int(sizes[j]), (1_000_000,), device="cuda")]
                out = torch.empty(1_000_000, dtype=torch.int64, device="cuda")
                lookups.append(srv.submit_lookup(done_blobs[j], q, out))
            li += 1
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        tickets[i] = srv.submit_build(sets[i], int(leafs[i]), int(buckets[i]))
        for j in range(i):  # collect finished builds (lookups use them)
            if tickets[j] is not None and j not in done_blobs:
                r = srv.poll(tickets[j])
                if r is not None:
                    assert r["status"] == 0
                    done_blobs[j] = r["blob"]
                    tickets[j] = r
    lat = []
    for j in range(R):
        r = tickets[j] if isinstance(tickets[j], dict) else srv.wait(tickets[j])
        assert r["status"] == 0
        tickets[j] = r
        if j not in done_blobs:
            done_blobs[j] = r["blob"]
        lat.append(r["latency_ms"])
    lk_lat = [srv.wait(t)["latency_ms"] for t in lookups]
    served_s = time.perf_counter() - t0
    stats = srv.stats()
    bits = sum(b.nbytes for b in done_blobs.values()) * 8 / total
    srv.close()
    for b in done_blobs.values():
        b.free()
    log(f"[bench] served: makespan {served_s:.1f} s, p50 {np.percentile(lat, 50):.0f} ms, "
        f"p99 {np.percentile(lat, 99):.0f} ms, {stats}")

    # plain path: same arrivals, one rs_build per request in arrival order
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plat = []
    for i in range(R):
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        b = recsplit.build(sets[i], int(leafs[i]), int(buckets[i]), tuned=tuned)
        torch.cuda.synchronize()
        plat.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
        b.free()
    plain_s = time.perf_counter() - t0
    log(f"[bench] plain: makespan {plain_s:.1f} s, p50 {np.percentile(plat, 50):.0f} ms, "
        f"p99 {np.percentile(plat, 99):.0f} ms")
    return {
        "metric": "served build latency p50/p99 and keys/s (continuous batching vs one call per request)",
        "value": total / served_s, "unit": "keys/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": served_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{R} Poisson build requests, sizes log-uniform [1e4, 1e7], l in {{8,12,16}}, "
                               f"b in {{100,1000,2000}}, offered load {load}, plus 1M-key lookup batches",
                   "keys": total},
        "served": {"makespan_s": served_s, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                   "lookup_p50_ms": percentile(lk_lat, 50) if lk_lat else None,
                   "lookup_p99_ms": percentile(lk_lat, 99) if lk_lat else None, "lookups": len(lk_lat),
                   "stats": stats},
        "plain": {"makespan_s": plain_s, "p50_ms": percentile(plat, 50), "p99_ms": percentile(plat, 99),
                  "keys_per_s": total / plain_s},
        "requests": [{"n": int(sizes[i]), "leaf": int(leafs[i]), "bucket": int(buckets[i]),
                      "arrival_s": float(arrivals[i]), "served_ms": float(lat[i]),
                      "served_batch": int(tickets[i]["batch_size"]) if isinstance(tickets[i], dict) else None,
                      "plain_ms": float(plat[i])} for i in range(R)],
        "bits_per_key": bits,
        "schedules": schedules if tuned else "built-in",
    }


# Rows of the paper's Table tab:1M (10^6 random keys, one core of its test machine):
# (l, b) -> bits/key, construction ns/key, lookup ns/key.
PAPER_TAB_1M = {(8, 100): (1.79, 1027, 67), (12, 9): (2.23, 7245, 39), (5, 5): (2.95, 139, 47),
                (16, 2000): (1.56, 1733801, 87)}


def bench_table(args):
    """The paper's Table tab:1M points on the GPU: for each (l, b), build the
    structure of the same random 64-bit keys (steps times, after a warm-up)
    and look every key up; report bits/key and ns/key next to the paper's."""
    import numpy as np
    import torch

    from paper_1910_06416_amd import inputs, recsplit

    n = args.table_n
    if n > 100_000_000:  # distinct draws checked on the device (a host-side pass would sort 8 GB)
        keys = recsplit.device_keys(inputs.u64_keys_raw(n, 7))
        srt, _ = torch.sort(keys)
        assert not bool((srt[1:] == srt[:-1]).any()), "duplicate keys drawn; use another seed"
        del srt
    else:
        keys = recsplit.device_keys(inputs.u64_keys(n, 7))
    ranks = torch.empty(n, dtype=torch.int64, device="cuda")
    rows = []
    for (leaf, bucket), (p_bits, p_build, p_lookup) in PAPER_TAB_1M.items():
        if leaf >= 16 and n > 10_000_000:
            log(f"[bench] table l={leaf} b={bucket}: skipped at {n:,} keys (about {n / 1.45e6:.0f} s)")
            continue
        steps = max(1, args.steps if leaf < 16 else 1)
        schedule = tune(recsplit, leaf, bucket, args, n) if not args.no_tune else "built-in"
        recsplit.build(keys, leaf, bucket, tuned=not args.no_tune).free()
        bt = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            blob = recsplit.build(keys, leaf, bucket, tuned=not args.no_tune)
            torch.cuda.synchronize()
            bt.append(time.perf_counter() - t0)
            if len(bt) < steps:
                blob.free()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        recsplit.lookup(blob, keys, out=ranks)
        ev0.record()
        for _ in range(5):
            recsplit.lookup(blob, keys, out=ranks)
        ev1.record()
        ev1.synchronize()
        lk = ev0.elapsed_time(ev1) / 5 * 1e-3
        srt, _ = torch.sort(ranks)
        assert torch.equal(srt, torch.arange(n, dtype=torch.int64, device="cuda")), "lookups are not a bijection"
        bits = blob.bits_per_key()
        blob.free()
        build_s = float(np.median(bt))
        row = {"leaf": leaf, "bucket": bucket, "bits_per_key": bits, "build_ns_per_key": build_s / n * 1e9,
               "lookup_ns_per_key": lk / n * 1e9, "keys_per_s": n / build_s,
               "paper": {"bits_per_key": p_bits, "build_ns_per_key": p_build, "lookup_ns_per_key": p_lookup},
               "schedule": schedule}
        rows.append(row)
        log(f"[bench] table l={leaf} b={bucket}: {bits:.4f} bits/key (paper {p_bits}), "
            f"build {row['build_ns_per_key']:.3f} ns/key (paper {p_build}), "
            f"lookup {row['lookup_ns_per_key']:.4f} ns/key (paper {p_lookup})")
    first = rows[0]
    return {
        "metric": "keys/s built at the paper's Table tab:1M points (bits/key, construction and lookup ns/key)",
        "value": first["keys_per_s"], "unit": "keys/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": first["build_ns_per_key"] * n * 1e-6, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{n:,} uniform random 64-bit keys at (l, b) = (8, 100), (12, 9), (5, 5), (16, 2000)"
                               + (" (l=16 skipped above 10^7 keys)" if n > 10_000_000 else ""), "keys": n},
        "rows": rows,
    }


def tune(recsplit, leaf, bucket, args, keys):
    """Autotune the search schedule of (leaf, bucket) for builds of `keys` keys
    before the timed region."""
    budget = args.tune_ms * (10.0 if leaf >= 16 else 1.0)
    sc = recsplit.autotune(leaf, bucket, keys_hint=int(keys), budget_ms=budget)
    log(f"[bench] schedule l={leaf} b={bucket}: waves {sc['waves']}, stage_from {sc['stage_from']}, "
        f"group_max {sc['group_max']} ({sc['search_ms']:.2f} ms vs {sc['default_ms']:.2f} ms built-in on the "
        f"calibration sample; {sc['variants']} schedules in {sc['tune_ms'] / 1e3:.1f} s)")
    return sc


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs visible)"
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
