"""GPU parity: the HIP path reproduces the oracle's blob byte for byte and its
ranks element by element, on the same seeded inputs.  Integer work, so the
bar is bit-exactness."""
import os

import numpy as np
import pytest

from paper_1910_06416_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch

    assert torch.cuda.is_available()
    from paper_1910_06416_amd import recsplit

    recsplit.lib()
    return recsplit


def _first_difference(a: bytes, b: bytes, orc):
    if len(a) != len(b):
        return f"sizes differ: gpu {len(a)} oracle {len(b)}"
    x = np.frombuffer(a, dtype=np.uint64)
    y = np.frombuffer(b, dtype=np.uint64)
    bad = np.flatnonzero(x != y)
    h = orc.header(b)
    return f"{len(bad)} words differ, first at word {bad[0]} (header {h})"


def _check_build(rs, orc, keys, leaf, bucket, lookups=True):
    print(f"case n={len(keys[1]) - 1 if isinstance(keys, tuple) else len(keys)} leaf={leaf} bucket={bucket}",
          flush=True)
    blob = rs.build(rs.device_keys(keys), leaf, bucket)
    got = blob.to_bytes()
    want = orc.build(keys, leaf, bucket)
    assert got == want, _first_difference(got, want, orc)
    if lookups:
        ranks = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
        assert np.array_equal(ranks, orc.lookup(want, keys))
        n = len(ranks)
        assert np.array_equal(np.sort(ranks), np.arange(n, dtype=np.uint64))
    return blob, want


@pytest.mark.parametrize(
    "n,leaf,bucket",
    [(1, 8, 100), (2, 8, 100), (3, 1, 1), (17, 2, 3), (100, 8, 100), (1000, 5, 5), (3000, 12, 9), (5000, 8, 100),
     (2000, 4, 2000), (20000, 8, 1000), (4000, 3, 64), (777, 1, 10), (5000, 16, 40), (60, 24, 12), (1234, 7, 1)],
)
def test_blob_parity_u64_shapes(rs, orc, n, leaf, bucket):
    _check_build(rs, orc, inputs.u64_keys(n, 1000 + n + leaf), leaf, bucket)


@pytest.mark.parametrize("n,leaf,bucket,T", [(20000, 8, 1000, 300), (6000, 5, 2000, 31), (9000, 12, 3000, 250),
                                             (30000, 8, 100, 96)])
def test_blob_parity_large_split_approximation(rs, orc, n, leaf, bucket, T):
    """Golomb-Rice parameters of splits above T from the integer approximation
    of Sec. 7.2: blob bytes, ranks, and a round trip through host bytes."""
    keys = inputs.u64_keys(n, 4000 + T)
    print(f"case gr approximation n={n} leaf={leaf} bucket={bucket} T={T}", flush=True)
    blob = rs.build(rs.device_keys(keys), leaf, bucket, gr_table_max=T)
    want = orc.build(keys, leaf, bucket, gr_table_max=T)
    got = blob.to_bytes()
    assert got == want, _first_difference(got, want, orc)
    assert orc.header(got)["gr_table_max"] == T
    ranks = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
    assert np.array_equal(ranks, orc.lookup(want, keys))
    again = rs.from_bytes(want)
    assert np.array_equal(rs.lookup(again, rs.device_keys(keys)).cpu().numpy().view(np.uint64), ranks)


def test_blob_parity_cfg_100k_l8_b100(rs, orc):
    """100,000 uniform random 64-bit keys, l=8, b=100."""
    blob, want = _check_build(rs, orc, inputs.u64_keys(100_000, 1), 8, 100)
    assert 1.78 <= 8 * len(want) / 100_000 <= 1.82


def test_guessed_arena_and_its_refill(rs, orc, monkeypatch):
    """A single build of a shape this thread built before fills an arena
    guessed from that build before the call's one wait; a guess that is too
    small (RS_ARENA_GUESS scales it) is filled again into an exact arena.
    Every path gives the oracle's bytes."""
    keys = inputs.u64_keys(100_000, 31)
    want = orc.build(keys, 8, 100)
    dk = rs.device_keys(keys)
    paths = []
    for scale in ("0", None, None, "0.25", "0"):  # exact (and remembered), guessed twice, refilled, exact
        if scale is None:
            monkeypatch.delenv("RS_ARENA_GUESS", raising=False)
        else:
            monkeypatch.setenv("RS_ARENA_GUESS", scale)
        print(f"case guessed arena, scale {scale}", flush=True)
        blob = rs.build(dk, 8, 100, timing=True)
        st = rs.last_build_stats()
        got = blob.to_bytes()
        blob.free()
        assert got == want, _first_difference(got, want, orc)
        assert st["blob_bytes"] >= len(want)  # (the arena rounds each blob up to 256 bytes)
        paths.append((st["arena_bytes"] > st["blob_bytes"], int(st["refills"])))
    assert paths == [(False, 0), (True, 0), (True, 0), (False, 1), (False, 0)]
    # a key count more than twice away from the remembered one takes no guess
    # (a small set spends many more words per key on its header and index)
    monkeypatch.delenv("RS_ARENA_GUESS", raising=False)
    for n, guessed in ((500, False), (100_000, False), (100_000, True)):
        sub = keys[:n]
        print(f"case guessed arena, n {n}", flush=True)
        blob = rs.build(rs.device_keys(sub), 8, 100, timing=True)
        st = rs.last_build_stats()
        got = blob.to_bytes()
        blob.free()
        assert got == orc.build(sub, 8, 100)
        assert (st["arena_bytes"] > st["blob_bytes"], int(st["refills"])) == (guessed, 0)


@pytest.mark.parametrize("n,leaf,bucket", [(1, 8, 100), (777, 8, 100), (100_000, 8, 100), (5000, 6, 50)])
def test_blob_parity_strings(rs, orc, n, leaf, bucket):
    _check_build(rs, orc, inputs.ascii_keys(n, 2000 + n), leaf, bucket)


def test_blob_parity_strings_long_and_mixed(rs, orc):
    """Strings of 8-32 bytes mixed with 2% of 33-1,500 bytes at random places
    (groups of a wavefront's strings that overflow the LDS staging take the
    direct reads), and a buffer whose length is not a multiple of 8 (its last
    word is partial)."""
    rng = np.random.default_rng(4242)
    sd, so = inputs.ascii_keys(20_000, 4243, 8, 32)
    ld, lo = inputs.ascii_keys(400, 4244, 33, 1500)
    strings = [sd[so[i]:so[i + 1]].tobytes() for i in range(len(so) - 1)]
    strings += [ld[lo[i]:lo[i + 1]].tobytes() for i in range(len(lo) - 1)]
    strings = [strings[i] for i in rng.permutation(len(strings))]
    total = sum(len(x) for x in strings)
    strings.append(b"tail!" if (total + 5) % 8 else b"tail!!")
    offs = np.zeros(len(strings) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(x) for x in strings])
    assert int(offs[-1]) % 8
    data = np.frombuffer(b"".join(strings), dtype=np.uint8)
    _check_build(rs, orc, (data, offs), 8, 100)


def test_blob_parity_strings_unaligned_and_short(rs, orc):
    import torch

    strings = [b"", b"a", b"ab", b"abcdefgh", b"abcdefghi", b"\x00", b"\x00\x00", b"x" * 40, b"y" * 17]
    offs = np.zeros(len(strings) + 2, dtype=np.uint64)
    offs[2:] = 1 + np.cumsum([len(s) for s in strings])
    offs[1] = 1
    data = np.frombuffer(b"Z" + b"".join(strings), dtype=np.uint8)
    # key 0 is "Z"; data starts on an odd address inside the tensor for the rest
    keys = (data, offs)
    _check_build(rs, orc, keys, 2, 3)
    d, o = rs.device_keys(keys)
    sub = (d[1:], (o[1:] - 1).contiguous())  # misaligned data pointer
    blob = rs.build(sub, 2, 3)
    host = (data[1:].copy(), (offs[1:] - 1).astype(np.uint64))
    assert blob.to_bytes() == orc.build(host, 2, 3)


def test_blob_parity_l16_b2000(rs, orc):
    """l=16, b=2000 on 3 buckets (the high-compression regime)."""
    _check_build(rs, orc, inputs.u64_keys(6000, 4), 16, 2000)


def test_lookup_non_members_match_oracle(rs, orc):
    keys = inputs.u64_keys(50_000, 7)
    blob, want = _check_build(rs, orc, keys, 8, 100, lookups=False)
    other = inputs.u64_keys(200_000, 8)
    got = rs.lookup(blob, rs.device_keys(other)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, orc.lookup(want, other))
    assert got.max() <= 50_000


@pytest.mark.parametrize("n,bucket", [(30_000, 100), (300_000, 10)])
def test_roundtrip_from_bytes(rs, orc, n, bucket):
    """A structure loaded from its bytes (its select samples computed from
    the inventory; 30,000 buckets span two 2^14-one blocks) gives the
    oracle's ranks, as does the same structure built on the device."""
    keys = inputs.u64_keys(n, 9)
    print(f"case from bytes n={n} bucket={bucket}", flush=True)
    want = orc.build(keys, 8, bucket)
    blob = rs.from_bytes(want)
    assert blob.to_bytes() == want
    dk = rs.device_keys(keys)
    ranks = rs.lookup(blob, dk).cpu().numpy().view(np.uint64)
    assert np.array_equal(ranks, orc.lookup(want, keys))
    built = rs.build(dk, 8, bucket)
    assert built.to_bytes() == want
    assert np.array_equal(rs.lookup(built, dk).cpu().numpy().view(np.uint64), ranks)


@pytest.mark.parametrize("kind,n,leaf,bucket,slack",
                         [("u64", 300_000, 8, 10, 0), ("bytes", 60_000, 5, 5, 0), ("u64", 40_000, 8, 100, 32)])
def test_lookup_without_select_samples(rs, orc, kind, n, leaf, bucket, slack):
    """RS_OPT_NO_SAMPLES: the same structure, whose lookups start their
    selects at the two-level inventory, as those of structures too large for
    32-bit samples do (30,000 and 12,000 buckets span two and one 2^14-one
    blocks); ranks equal the sampled blob's and the oracle's."""
    keys = inputs.u64_keys(n, 5100 + n) if kind == "u64" else inputs.ascii_keys(n, 5100 + n)
    print(f"case no samples kind={kind} n={n} leaf={leaf} bucket={bucket} slack={slack}", flush=True)
    dk = rs.device_keys(keys)
    plain = rs.build(dk, leaf, bucket, leaf_slack=slack, samples=False)
    sampled = rs.build(dk, leaf, bucket, leaf_slack=slack, timing=True)
    st = rs.last_build_stats()
    assert (st["arena_bytes"], int(st["refills"])) == (st["blob_bytes"], 0)  # no guess across the two formats
    assert plain.to_bytes() == sampled.to_bytes()
    ranks = rs.lookup(plain, dk).cpu().numpy().view(np.uint64)
    assert np.array_equal(ranks, rs.lookup(sampled, dk).cpu().numpy().view(np.uint64))
    assert len(np.unique(ranks)) == n
    if not slack:
        want = orc.build(keys, leaf, bucket)
        assert plain.to_bytes() == want
        assert np.array_equal(ranks, orc.lookup(want, keys))


def test_errors(rs, orc):
    import torch

    keys = inputs.u64_keys(1000, 3)
    dup = np.concatenate([keys, keys[5:6]])
    print("case duplicate key l=8", flush=True)
    with pytest.raises(rs.RecSplitError) as e:
        rs.build(rs.device_keys(dup), 8, 100)
    assert e.value.code == rs.RS_EDUPLICATE
    dup1 = np.concatenate([keys[:40], keys[:1]])
    print("case duplicate key l=1", flush=True)
    with pytest.raises(rs.RecSplitError) as e:
        rs.build(rs.device_keys(dup1), 1, 100)
    assert e.value.code == rs.RS_EDUPLICATE
    print("case seed cap", flush=True)
    with pytest.raises(rs.RecSplitError) as e:
        rs.build(rs.device_keys(keys[:12]), 12, 100, seed_cap=3)
    assert e.value.code == rs.RS_ESEARCH
    with pytest.raises(rs.RecSplitError) as e:
        rs.build(rs.device_keys(keys), 0, 100)
    assert e.value.code == rs.RS_EINVAL
    d = torch.zeros(10, dtype=torch.uint8, device="cuda")
    o = torch.tensor([0, 5, 3, 10], dtype=torch.int64, device="cuda")
    with pytest.raises(rs.RecSplitError) as e:
        rs.build((d, o), 8, 100)
    assert e.value.code == rs.RS_EINVAL
    blob = rs.build(rs.device_keys(keys), 8, 100)
    with pytest.raises(rs.RecSplitError):
        rs.lookup(blob, (d, o))
    # the library still works after the errors
    assert blob.to_bytes() == orc.build(keys, 8, 100)


@pytest.mark.parametrize("n,leaf", [(12, 12), (7, 7), (16, 16), (30, 8), (200, 5), (90, 16)])
def test_seed_cap_boundary(rs, orc, n, leaf):
    """Exactly at the largest stored index the build must fail; one above it,
    succeed with the oracle's bytes (exercises the end-of-range flush of the
    staged bijection search and the cap test of the split search)."""
    keys = inputs.u64_keys(n, 50 + n + leaf)
    _, lo = orc.fingerprint(keys)
    v, _, _ = orc.tree(np.sort(lo), leaf)
    vmax = int(v.max())
    print(f"case cap boundary n={n} leaf={leaf} vmax={vmax}", flush=True)
    want = orc.build(keys, leaf, 1000, seed_cap=vmax + 1)
    assert rs.build(rs.device_keys(keys), leaf, 1000, seed_cap=vmax + 1).to_bytes() == want
    if vmax > 0:
        with pytest.raises(rs.RecSplitError) as e:
            rs.build(rs.device_keys(keys), leaf, 1000, seed_cap=vmax)
        assert e.value.code == rs.RS_ESEARCH


def test_batch_blobs_equal_oracle(rs, orc):
    """One batched call over uneven builds (sizes, leaf sizes, bucket sizes and
    key kinds differ) returns each build's oracle bytes."""
    specs = [(1000, 8, 100, "u64"), (1, 8, 100, "u64"), (7777, 12, 1000, "u64"), (2500, 8, 100, "ascii"),
             (300, 5, 5, "u64"), (20000, 8, 100, "u64"), (4000, 16, 2000, "u64"), (50, 1, 7, "ascii"),
             (12345, 12, 9, "u64")]
    host = [inputs.u64_keys(n, 300 + i) if kind == "u64" else inputs.ascii_keys(n, 300 + i)
            for i, (n, _, _, kind) in enumerate(specs)]
    print("case batch of", len(specs), flush=True)
    blobs, status = rs.build_batch([rs.device_keys(k) for k in host], [s[1] for s in specs], [s[2] for s in specs])
    assert status == [0] * len(specs)
    for (n, leaf, bucket, _), k, b in zip(specs, host, blobs):
        want = orc.build(k, leaf, bucket)
        assert b.to_bytes() == want, (n, leaf, bucket)
        ranks = rs.lookup(b, rs.device_keys(k)).cpu().numpy().view(np.uint64)
        assert np.array_equal(ranks, orc.lookup(want, k))
    for b in blobs:
        b.free()


def test_batch_isolates_failed_builds(rs, orc):
    good = inputs.u64_keys(3000, 41)
    dup = np.concatenate([inputs.u64_keys(500, 42), inputs.u64_keys(500, 42)[:1]])
    import torch

    empty = torch.zeros(0, dtype=torch.int64, device="cuda")
    print("case batch with failures", flush=True)
    blobs, status = rs.build_batch([rs.device_keys(good), rs.device_keys(dup), empty, rs.device_keys(good)],
                                   [8, 8, 8, 25], [100, 100, 100, 100])
    assert status == [rs.RS_OK, rs.RS_EDUPLICATE, rs.RS_EINVAL, rs.RS_EINVAL]
    assert blobs[1] is None and blobs[2] is None and blobs[3] is None
    assert blobs[0].to_bytes() == orc.build(good, 8, 100)
    # the surviving blob outlives the others of its call
    del blobs[1:]
    assert blobs[0].to_bytes() == orc.build(good, 8, 100)


def _server_mix():
    specs = [(30_000, 8, 100), (5000, 12, 1000), (200_000, 8, 100), (1000, 16, 2000), (77_777, 12, 1000),
             (12_345, 8, 2000), (3, 8, 100), (50_000, 16, 100), (123_456, 12, 1000), (9999, 8, 100)]
    return specs, [inputs.u64_keys(n, 700 + i) for i, (n, _, _) in enumerate(specs)]


@pytest.mark.parametrize("lookup_cus", [0, 16])
def test_server_results_equal_alone(rs, orc, lookup_cus):
    """Requests submitted together are batched and overlapped; each result is
    byte-identical to the same build done alone (also with build streams kept
    off some compute units)."""
    specs, host = _server_mix()
    dev = [rs.device_keys(k) for k in host]
    print(f"case server mix lookup_cus={lookup_cus}", flush=True)
    srv = rs.Server(budget_bytes=8 << 30, build_workers=2, lookup_cus=lookup_cus)
    tickets = [srv.submit_build(d, leaf, bucket) for d, (_, leaf, bucket) in zip(dev, specs)]
    res = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    assert all(r["status"] == 0 for r in res)
    for (n, leaf, bucket), d, r in zip(specs, dev, res):
        alone = rs.build(d, leaf, bucket)
        assert r["blob"].to_bytes() == alone.to_bytes(), (n, leaf, bucket)
    # lookups through the server equal direct lookups
    import torch

    outs = [torch.empty(d.numel(), dtype=torch.int64, device="cuda") for d in dev]
    lt = [srv.submit_lookup(r["blob"], d, o) for r, d, o in zip(res, dev, outs)]
    for t in lt:
        assert srv.wait(t)["status"] == 0
    for r, d, o in zip(res, dev, outs):
        assert torch.equal(o, rs.lookup(r["blob"], d))
    srv.close()
    assert stats["batched_requests"] == len(specs)
    assert stats["lookup_cus"] == lookup_cus
    print("server stats", stats, flush=True)


def test_server_tiny_budget_still_completes(rs, orc):
    specs, host = _server_mix()
    specs, host = specs[:5], host[:5]
    dev = [rs.device_keys(k) for k in host]
    print("case server tiny budget", flush=True)
    srv = rs.Server(budget_bytes=1, build_workers=3)
    tickets = [srv.submit_build(d, leaf, bucket) for d, (_, leaf, bucket) in zip(dev, specs)]
    res = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    assert stats["max_batch"] == 1 and stats["max_concurrent_batches"] == 1  # admitted one at a time
    for (n, leaf, bucket), k, r in zip(specs, host, res):
        assert r["blob"].to_bytes() == orc.build(k, leaf, bucket)


@pytest.mark.parametrize("n,leaf,bucket", [(20000, 8, 100), (6000, 12, 300), (3000, 16, 200), (60, 24, 12),
                                           (5000, 5, 5)])
def test_schedules_never_change_the_result(rs, orc, n, leaf, bucket):
    """Every wavefront count, staged-search threshold and split lane-group cap
    gives the oracle's blob."""
    print(f"case schedules n={n} leaf={leaf} bucket={bucket}", flush=True)
    keys = inputs.u64_keys(n, 3000 + n + leaf)
    want = orc.build(keys, leaf, bucket)
    dk = rs.device_keys(keys)
    for waves in (1, 2, 4, 8):
        for stage_from, group_max in [(2, 1), (7, 7), (25, 4), (9, 2)]:
            got = rs.build(dk, leaf, bucket, waves=waves, stage_from=stage_from, group_max=group_max).to_bytes()
            assert got == want, (waves, stage_from, group_max)


def test_autotuned_schedules_in_builds_and_batches(rs, orc):
    """The autotuner stores a valid schedule; builds and mixed batches that use
    the table (different wavefront counts per build in one launch) still give
    the oracle's blobs."""
    print("case autotune", flush=True)
    rs.clear_schedules()
    sc = rs.autotune(8, 100, keys_hint=200_000, budget_ms=200)
    assert sc["waves"] in (1, 2, 4, 8) and 2 <= sc["stage_from"] <= 25 and 1 <= sc["group_max"] <= 7
    assert sc["variants"] >= 2 and sc["search_ms"] <= sc["default_ms"]
    assert rs.get_schedule(8, 100)["waves"] == sc["waves"]
    keys = inputs.u64_keys(30000, 77)
    assert rs.build(rs.device_keys(keys), 8, 100, tuned=True).to_bytes() == orc.build(keys, 8, 100)
    rs.set_schedule(8, 100, stage_from=7, group_max=3, waves=1)
    rs.set_schedule(12, 300, stage_from=11, group_max=2, waves=8)
    specs = [(5000, 8, 100), (7000, 12, 300), (3000, 8, 100), (100, 12, 300)]
    host = [inputs.u64_keys(n, 500 + i) for i, (n, _, _) in enumerate(specs)]
    blobs, status = rs.build_batch([rs.device_keys(k) for k in host], [s[1] for s in specs], [s[2] for s in specs],
                                   tuned=True)
    assert status == [0] * len(specs)
    for b, k, (n, leaf, bucket) in zip(blobs, host, specs):
        assert b.to_bytes() == orc.build(k, leaf, bucket)
    with pytest.raises(rs.RecSplitError):
        rs.build(rs.device_keys(keys), 8, 100, waves=3)
    rs.clear_schedules()


def test_plan_runs_equal_oracle_and_fall_back_past_caps(rs, orc):
    """A captured plan rebuilds from the buffers' current contents: every run
    equals the oracle for the keys then in the buffers; contents whose largest
    bucket exceeds the plan's cap take the ordinary path, with the same result."""
    import torch

    print("case plan", flush=True)
    specs = [(20000, 8, 100), (5000, 12, 300), (777, 5, 7), (3, 8, 100)]
    host = [inputs.u64_keys(n, 900 + i) for i, (n, _, _) in enumerate(specs)]
    dev = [rs.device_keys(k) for k in host]
    leafs, buckets = [s[1] for s in specs], [s[2] for s in specs]
    plan = rs.Plan(dev, leafs, buckets)
    for b, k, (n, leaf, bucket) in zip(plan.first, host, specs):
        assert b.to_bytes() == orc.build(k, leaf, bucket)
    for run in range(3):
        # new contents in the same buffers
        host = [inputs.u64_keys(n, 1000 * (run + 1) + i) for i, (n, _, _) in enumerate(specs)]
        for d, k in zip(dev, host):
            d.copy_(torch.from_numpy(k.view(np.int64)))
        blobs, status = plan.run()
        assert status == [0] * len(specs)
        for b, k, (n, leaf, bucket) in zip(blobs, host, specs):
            assert b.to_bytes() == orc.build(k, leaf, bucket), (run, n, leaf, bucket)
            r = rs.lookup(b, rs.device_keys(k)).cpu().numpy().view(np.uint64)
            assert np.array_equal(np.sort(r), np.arange(n, dtype=np.uint64))
    info = plan.info()
    assert info["runs"] == 3 and info["fallbacks"] == 0
    # skewed contents: one bucket far above the cap (keys chosen by the oracle's bucket function)
    n, leaf, bucket = specs[0]
    nb = -(-n // bucket)
    big = info["bucket_cap"] + 50
    pool = inputs.u64_keys(4 * big * nb, 4242)
    hi, _ = orc.fingerprint(pool)
    in_zero = pool[(hi >> np.uint64(32)).astype(np.float64) * nb < 2.0 ** 32 * 0.9][:big]
    assert len(in_zero) == big
    rest = pool[~np.isin(pool, in_zero)][: n - len(in_zero)]
    skew = np.concatenate([in_zero, rest])
    assert len(skew) == n and len(np.unique(skew)) == n
    dev[0].copy_(torch.from_numpy(skew.view(np.int64)))
    blobs, status = plan.run()
    assert status[0] == 0 and blobs[0].to_bytes() == orc.build(skew, leaf, bucket)
    assert plan.info()["fallbacks"] == 1
    plan.close()


def test_library_loaded_before_torch_still_builds(rs, orc):
    """Loading the library before torch must not leave two HIP runtimes in the
    process (torch ships its own): a fresh process that loads the library
    first builds a structure equal to the oracle's."""
    import subprocess
    import sys

    print("case load order", flush=True)
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1910_06416_amd import recsplit, inputs\n"
        "recsplit.lib()\n"
        "import oracle\n"
        "keys = inputs.u64_keys(3000, 5)\n"
        "b = recsplit.build(recsplit.device_keys(keys), 8, 100, timing=True)\n"
        "assert b.to_bytes() == oracle.build(keys, 8, 100)\n"
        "print('ok')\n"
    ) % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))),)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0 and "ok" in res.stdout, res.stderr[-2000:]


def test_largest_buckets_that_fit_and_the_error_beyond(rs, orc):
    """Buckets of ~12,000 keys (the keys and node queue of one bucket in LDS)
    build and equal the oracle; a bucket too large for the local data share
    is refused with an error, not run."""
    print("case large buckets", flush=True)
    keys = inputs.u64_keys(24_000, 12)
    _check_build(rs, orc, keys, 8, 12_000)
    big = rs.device_keys(inputs.u64_keys(60_000, 13))
    with pytest.raises(rs.RecSplitError, match="local data share"):
        rs.build(big, 8, 60_000)
