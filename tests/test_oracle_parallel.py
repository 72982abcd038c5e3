"""The bucket-parallel oracle harness (oracle/parallel.py) computes the same
bytes as the single-threaded oracle: it only runs the oracle's own per-bucket
tree loop for disjoint bucket ranges in worker processes."""
import numpy as np
import pytest

from paper_1910_06416_amd import inputs


@pytest.mark.parametrize("n,leaf,bucket,kind", [(100_000, 8, 100, "u64"), (20_000, 8, 100, "ascii"),
                                                (30_000, 12, 9, "u64"), (3000, 5, 5, "u64"), (1, 8, 100, "u64"),
                                                (777, 1, 10, "u64")])
def test_parallel_build_equals_oracle(orc, n, leaf, bucket, kind):
    from oracle import parallel

    keys = inputs.u64_keys(n, 5000 + n) if kind == "u64" else inputs.ascii_keys(n, 5000 + n)
    blob, timing = parallel.build(keys, leaf, bucket, workers=4)
    assert blob == orc.build(keys, leaf, bucket)
    assert timing["workers"] >= 1 and timing["wall_s"] > 0


def test_bucket_trees_equal_single_bucket_trees(orc):
    from oracle import parallel

    n, leaf, bucket = 40_000, 12, 1000
    keys = inputs.u64_keys(n, 77)
    nb = n // bucket
    picks = [0, 7, nb - 1]
    got = parallel.bucket_trees(keys, leaf, bucket, picks, workers=3)
    for i in picks:
        v, m, _ = orc.tree(orc.bucket_keys(keys, nb, i), leaf)
        assert np.array_equal(got[i][0], v) and np.array_equal(got[i][1], m)
        assert got[i][2] > 0


def test_layout_rejects_equal_lower_words(orc):
    keys = inputs.u64_keys(1000, 78)
    dup = np.concatenate([keys, keys[:1]])
    with pytest.raises(orc.OracleError) as e:
        orc.bucket_layout(dup, 10)
    assert e.value.code == orc.EDUPLICATE


def test_bucket_trees_with_ranks_equal_bucket_ranks(orc):
    from oracle import parallel

    n, leaf, bucket = 20_000, 8, 100
    keys = inputs.u64_keys(n, 79)
    nb = n // bucket
    got = parallel.bucket_trees(keys, leaf, bucket, [3, 150], workers=2, with_ranks=True)
    hi, lo = orc.fingerprint(keys)
    ids = orc.bucket_ids(hi, nb)
    for i in (3, 150):
        los = np.sort(lo[ids == i])
        assert np.array_equal(got[i][3], orc.bucket_ranks(los, leaf))
        assert np.array_equal(np.sort(got[i][3]), np.arange(len(los), dtype=np.uint64))
    assert np.array_equal(np.bincount(ids.astype(np.int64), minlength=nb), orc.bucket_sizes(keys, nb))
