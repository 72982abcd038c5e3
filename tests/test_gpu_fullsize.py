"""GPU parity at the full workload sizes, in the same calls the benchmark times.

* 10^7 ASCII strings, l=8, b=100: the whole blob byte for byte and every rank
  of a shuffled lookup batch against the oracle (the oracle builds it in well
  under a minute).
* 10^7 random 64-bit keys, l=16, b=2000: the oracle needs hours for the whole
  structure, so the test compares the header, both Elias-Fano lists of all
  5,000 buckets, and for 128 buckets (the largest and the smallest among
  them) every index, node size, Golomb-Rice length and key rank; the
  oracle's trees of those buckets are computed in parallel on the host
  cores (oracle/parallel.py).  It also checks that the lookup of all 10^7
  keys is a permutation of [0, n).
* 4096 uneven builds in one batched call, l=12, b=1000: the 16 smallest builds
  whole, and sampled buckets of the largest and of every 256th build. The
  lookup of every key of every build must be a bijection.
"""
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


def _is_permutation(ranks) -> bool:
    import torch

    srt, _ = torch.sort(ranks)
    return bool(torch.equal(srt, torch.arange(ranks.numel(), dtype=torch.int64, device=ranks.device)))


def _check_sampled_buckets(rs, orc, keys_host, blob_bytes, ranks_dev, leaf, picks):
    """Indices and in-bucket ranks of the picked buckets against the oracle's
    tree for each bucket's keys."""
    import torch

    h = orc.header(blob_bytes)
    nb = h["nb"]
    for i in picks:
        s_i, _, v, m = orc.blob_bucket(blob_bytes, i)
        idx = orc.bucket_members(keys_host, nb, i)
        _, lo = orc.fingerprint(keys_host[idx])
        tv, tm, _ = orc.tree(np.sort(lo), leaf)
        assert np.array_equal(m, tm), f"bucket {i}: node sizes differ"
        assert np.array_equal(v, tv), f"bucket {i}: indices differ"
        want = orc.bucket_ranks(lo, leaf) + np.uint64(s_i)
        sel = torch.from_numpy(idx.astype(np.int64)).to(ranks_dev.device)
        got = ranks_dev[sel].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want), f"bucket {i}: ranks differ"


# Workload sizes (the benchmark's).
STRINGS_N = 10_000_000
L16_N = 10_000_000
BATCH_BUILDS = 4096


def test_full_strings_10M_l8_b100(rs, orc):
    n = STRINGS_N
    print(f"case full strings n={n} leaf=8 bucket=100", flush=True)
    keys = inputs.ascii_keys(n, 2)
    blob = rs.build(rs.device_keys(keys), 8, 100)
    got = blob.to_bytes()
    want = orc.build(keys, 8, 100)
    assert got == want
    order = inputs.permutation(n, 3)
    queries = inputs.gather_strings(keys, order)
    ranks = rs.lookup(blob, rs.device_keys(queries))
    assert _is_permutation(ranks)
    assert np.array_equal(ranks.cpu().numpy().view(np.uint64), orc.lookup(want, queries))


L16_BUCKETS = 128


def test_full_u64_10M_l16_b2000(rs, orc):
    """128 of the 5,000 buckets (the largest, the smallest and 126 drawn at
    random) against the oracle's trees, computed bucket-parallel on the host
    cores by the oracle's own tree loop: every index and node size, the
    bucket's Golomb-Rice length o_{i+1} - o_i and the rank of every key."""
    import torch

    from oracle import parallel

    n, leaf, bucket = L16_N, 16, 2000
    print(f"case full u64 n={n} leaf={leaf} bucket={bucket}", flush=True)
    keys = inputs.u64_keys(n, 4)
    dkeys = rs.device_keys(keys)
    blob = rs.build(dkeys, leaf, bucket)
    got = blob.to_bytes()
    h = orc.header(got)
    nb = -(-n // bucket)
    hi, lo = orc.fingerprint(keys)
    ids = orc.bucket_ids(hi, nb).astype(np.int64)
    sizes = np.bincount(ids, minlength=nb)
    assert np.array_equal(sizes, orc.bucket_sizes(keys, nb))
    assert (h["n"], h["leaf"], h["bucket"], h["nb"], h["maxm"]) == (n, leaf, bucket, nb, int(sizes.max()))
    s_all, o_all = orc.blob_prefix(got)
    assert np.array_equal(s_all, np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64))
    assert o_all[-1] == h["tree_bits"]
    if n >= 1_000_000:
        assert 1.55 <= 8 * len(got) / n <= 1.57
    ranks = rs.lookup(blob, dkeys)
    assert _is_permutation(ranks)
    rng = np.random.default_rng(11)
    picks = {int(np.argmax(sizes)), int(np.argmin(sizes))}
    while len(picks) < min(L16_BUCKETS, nb):
        picks.add(int(rng.integers(0, nb)))
    picks = sorted(picks)
    print(f"oracle trees of {len(picks)} buckets on {parallel.default_workers()} host processes", flush=True)
    trees = parallel.bucket_trees(keys, leaf, bucket, picks, with_ranks=True)
    r, _, _ = orc.tables(leaf, h["maxm"])
    order = np.argsort(ids, kind="stable")
    starts = np.concatenate([[0], np.cumsum(sizes)])
    for i in picks:
        s_i, o_i, v, m = orc.blob_bucket(got, i)
        tv, tm, _, tranks = trees[i]
        assert np.array_equal(m, tm), f"bucket {i}: node sizes differ"
        assert np.array_equal(v, tv), f"bucket {i}: indices differ"
        bits = sum(int(r[mm]) + (int(vv) >> int(r[mm])) + 1 for vv, mm in zip(tv, tm))
        assert int(o_all[i + 1] - o_all[i]) == bits, f"bucket {i}: Golomb-Rice length differs"
        idx = order[starts[i]:starts[i + 1]]
        by_lo = idx[np.argsort(lo[idx], kind="stable")]  # members in ascending lower word, as the oracle ranks them
        got_r = ranks[torch.from_numpy(by_lo).to(ranks.device)].cpu().numpy().view(np.uint64)
        assert np.array_equal(got_r, tranks + np.uint64(s_i)), f"bucket {i}: ranks differ"


def test_full_batch_4096_l12_b1000(rs, orc):
    import torch

    leaf, bucket = 12, 1000
    sizes = inputs.log_uniform_sizes(BATCH_BUILDS, 5, 1e3, 1e6)
    total = int(sizes.sum())
    print(f"case full batch builds={len(sizes)} keys={total} leaf={leaf} bucket={bucket}", flush=True)
    keys = inputs.u64_keys(total, 5)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    dall = rs.device_keys(keys)
    sets = [dall[int(offs[i]):int(offs[i + 1])] for i in range(len(sizes))]
    blobs, status = rs.build_batch(sets, leaf, bucket)
    assert all(s == 0 for s in status)
    for i in range(len(sizes)):
        assert _is_permutation(rs.lookup(blobs[i], sets[i])), f"build {i}"
    order = np.argsort(sizes, kind="stable")
    whole = order[:16].tolist()
    for i in whole:
        part = keys[offs[i]:offs[i + 1]]
        assert blobs[i].to_bytes() == orc.build(part, leaf, bucket), f"build {i} (n={sizes[i]})"
    sampled = sorted(set(order[-4:].tolist() + list(range(0, len(sizes), 256))) - set(whole))
    rng = np.random.default_rng(12)
    for i in sampled:
        part = keys[offs[i]:offs[i + 1]]
        got = blobs[i].to_bytes()
        h = orc.header(got)
        nb = -(-int(sizes[i]) // bucket)
        bs = orc.bucket_sizes(part, nb)
        assert (h["n"], h["nb"], h["maxm"]) == (int(sizes[i]), nb, int(bs.max()))
        s_all, _ = orc.blob_prefix(got)
        assert np.array_equal(s_all, np.concatenate([[0], np.cumsum(bs)]).astype(np.uint64))
        ranks = rs.lookup(blobs[i], sets[i])
        _check_sampled_buckets(rs, orc, part, got, ranks, leaf, [int(rng.integers(0, nb))])
    for b in blobs:
        b.free()
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [30_000_000, 40_000_000])
def test_many_buckets_sorted_in_pieces(rs, orc, n):
    """b=1, so one bucket per key.  At 30M buckets the bucket sort has 3663
    bins of 8192 buckets (one piece each); at 40M each bin spans more buckets
    than it counts at once and is sorted in two pieces.  The Elias-Fano lists
    of every bucket, sampled buckets and the bijection are checked against the
    oracle."""
    leaf, bucket = 5, 1
    print(f"case many buckets n={n} leaf={leaf} bucket={bucket}", flush=True)
    keys = inputs.u64_keys(n, 8)
    dkeys = rs.device_keys(keys)
    blob = rs.build(dkeys, leaf, bucket)
    got = blob.to_bytes()
    h = orc.header(got)
    sizes = orc.bucket_sizes(keys, n)
    assert (h["n"], h["nb"], h["maxm"]) == (n, n, int(sizes.max()))
    s_all, o_all = orc.blob_prefix(got)
    assert np.array_equal(s_all, np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64))
    assert o_all[-1] == h["tree_bits"]
    ranks = rs.lookup(blob, dkeys)
    assert _is_permutation(ranks)
    picks = [int(np.argmax(sizes)), 16384 + 3, n - 1]
    _check_sampled_buckets(rs, orc, keys, got, ranks, leaf, picks)
