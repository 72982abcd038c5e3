"""Bucket-parallel harness around the CPU oracle (test infrastructure only).

Buckets are independent (Sec. 4 of the paper: every bucket's tree depends
only on the bucket's own keys), so the trees of disjoint bucket ranges can be
computed in separate worker processes, each calling the oracle's own
single-threaded tree loop (orc_trees).  The oracle is not changed or
threaded: build() lays the keys out with orc_bucket_layout, farms bucket
ranges out to the workers and assembles the structure with
orc_build_with_trees, which gives the same bytes as oracle.build().

Workers are started with the "spawn" method (a fresh interpreter that never
touches the GPU), at most 16 of them.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from . import bucket_layout, build_with_trees, ranks_from_tree, trees

MAX_WORKERS = 16


def default_workers() -> int:
    return max(1, min(MAX_WORKERS, os.cpu_count() or 1))


def _task(args):
    lo, s_local, leaf, seed_cap = args
    t0 = time.perf_counter()
    v, m, cnt = trees(lo, s_local, 0, len(s_local) - 1, leaf, seed_cap)
    return v, m, cnt, time.perf_counter() - t0


def _task_ranks(args):
    lo, s_local, leaf, seed_cap = args
    v, m, cnt, dt = _task(args)
    c = int(cnt[0])
    return v[:c], m[:c], cnt, dt, ranks_from_tree(lo, leaf, v[:c])


def _pool(workers: int):
    return mp.get_context("spawn").Pool(workers)


def _ranges(s_: np.ndarray, first: int, last: int, parts: int):
    """Split buckets [first, last) into at most `parts` contiguous ranges of
    about equal key counts."""
    total = int(s_[last] - s_[first])
    if total == 0 or parts <= 1:
        return [(first, last)]
    cuts = [first]
    for k in range(1, parts):
        target = int(s_[first]) + total * k // parts
        b = int(np.searchsorted(s_, target, side="left"))
        b = min(max(b, cuts[-1]), last)
        if b > cuts[-1]:
            cuts.append(b)
    if cuts[-1] != last:
        cuts.append(last)
    return list(zip(cuts[:-1], cuts[1:]))


def _local(sorted_lo, s_, a, b):
    base = int(s_[a])
    return sorted_lo[base:int(s_[b])], (s_[a:b + 1] - np.uint64(base)).astype(np.uint64)


def bucket_trees(keys, leaf: int, bucket: int, picks, workers: int | None = None, seed_cap: int = 0, layout=None,
                 with_ranks: bool = False):
    """Trees of the picked buckets, one task per bucket, computed in parallel.
    Returns {bucket: (v, m, seconds)}: the coded nodes' indices and sizes in
    preorder and the single-core time the oracle took for that bucket; with
    with_ranks, also the in-bucket ranks of the bucket's lower words in
    ascending order of the words (v, m, seconds, ranks)."""
    workers = workers or default_workers()
    n = len(keys[1]) - 1 if isinstance(keys, tuple) else len(keys)
    nb = -(-n // bucket)
    sorted_lo, s_ = layout if layout is not None else bucket_layout(keys, nb)
    picks = [int(i) for i in picks]
    tasks = []
    for i in picks:
        lo, s_local = _local(sorted_lo, s_, i, i + 1)
        tasks.append((lo, s_local, leaf, seed_cap))
    with _pool(min(workers, max(1, len(tasks)))) as pool:
        res = pool.map(_task_ranks if with_ranks else _task, tasks, chunksize=1)
    out = {}
    for i, r in zip(picks, res):
        c = int(r[2][0])
        out[i] = (r[0][:c].copy(), r[1][:c].copy(), r[3]) + ((r[4],) if with_ranks else ())
    return out


def build(keys, leaf: int, bucket: int, workers: int | None = None, seed_cap: int = 0, tasks_per_worker: int = 4):
    """The oracle's structure, with the per-bucket trees computed by `workers`
    processes.  Returns (blob bytes, timing dict)."""
    workers = workers or default_workers()
    t0 = time.perf_counter()
    n = len(keys[1]) - 1 if isinstance(keys, tuple) else len(keys)
    nb = -(-n // bucket)
    sorted_lo, s_ = bucket_layout(keys, nb)
    t1 = time.perf_counter()
    node_v = np.zeros(max(n, 1), dtype=np.uint64)
    node_m = np.zeros(max(n, 1), dtype=np.uint32)
    node_count = np.zeros(nb, dtype=np.uint64)
    ranges = _ranges(s_, 0, nb, workers * tasks_per_worker)
    tasks = []
    for a, b in ranges:
        lo, s_local = _local(sorted_lo, s_, a, b)
        tasks.append((lo, s_local, leaf, seed_cap))
    with _pool(min(workers, len(tasks))) as pool:
        res = pool.map(_task, tasks, chunksize=1)
    core_s = 0.0
    for (a, b), (v, m, cnt, dt) in zip(ranges, res):
        base, end = int(s_[a]), int(s_[b])
        node_v[base:end] = v[:end - base]
        node_m[base:end] = m[:end - base]
        node_count[a:b] = cnt[:b - a]
        core_s += dt
    t2 = time.perf_counter()
    blob = build_with_trees(keys, leaf, bucket, node_v[:n], node_m[:n], node_count)
    t3 = time.perf_counter()
    return blob, {"layout_s": t1 - t0, "trees_s": t2 - t1, "encode_s": t3 - t2, "wall_s": t3 - t0,
                  "tree_core_s": core_s, "workers": min(workers, len(tasks)), "tasks": len(tasks)}
