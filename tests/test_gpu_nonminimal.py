"""GPU parity of the non-minimal variant (the larger codomain of Sec. 9):
leaves of m >= 2 keys take the first index whose hash is injective into
m + ceil(m slack / 256) values, and the first Elias-Fano list holds prefix
sums of bucket ranges.  The HIP path must give the oracle's bytes and the
oracle's output values, element by element (integer work: bit-exact)."""
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


def _range_total(orc, keys, leaf, bucket, slack):
    """Sum over buckets of the subtree range of the bucket's size (oracle tables)."""
    n = len(keys[1]) - 1 if isinstance(keys, tuple) else len(keys)
    nb = -(-n // bucket)
    sizes = orc.bucket_sizes(keys, nb).astype(np.int64)
    _, _, _, Q = orc.range_tables(leaf, int(sizes.max()), slack)
    return int(Q.astype(np.int64)[sizes].sum())


def _check(rs, orc, keys, leaf, bucket, slack):
    n = len(keys[1]) - 1 if isinstance(keys, tuple) else len(keys)
    print(f"case non-minimal n={n} leaf={leaf} bucket={bucket} slack={slack}", flush=True)
    blob = rs.build(rs.device_keys(keys), leaf, bucket, leaf_slack=slack)
    got = blob.to_bytes()
    want = orc.build(keys, leaf, bucket, leaf_slack=slack)
    assert len(got) == len(want)
    x, y = np.frombuffer(got, dtype=np.uint64), np.frombuffer(want, dtype=np.uint64)
    assert got == want, f"{int((x != y).sum())} words differ, first {int(np.flatnonzero(x != y)[0])}"
    assert orc.header(got)["leaf_slack"] == slack
    vals = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
    assert np.array_equal(vals, orc.lookup(want, keys))
    R = _range_total(orc, keys, leaf, bucket, slack)
    assert len(np.unique(vals)) == n and int(vals.max()) < R
    return blob, want


@pytest.mark.parametrize("n,leaf,bucket,slack", [
    (5000, 8, 100, 32), (20000, 8, 100, 255), (3000, 5, 5, 64), (9000, 12, 9, 16), (5000, 16, 200, 128),
    (500, 24, 48, 85), (777, 1, 10, 255), (400, 2, 7, 100), (1, 8, 100, 64), (2, 3, 100, 200), (30000, 7, 1000, 8),
])
def test_nonminimal_blob_and_values_equal_oracle(rs, orc, n, leaf, bucket, slack):
    _check(rs, orc, inputs.u64_keys(n, 5100 + n + slack), leaf, bucket, slack)


def test_nonminimal_strings(rs, orc):
    _check(rs, orc, inputs.ascii_keys(3000, 5200), 8, 100, 48)


def test_nonminimal_with_large_split_approximation(rs, orc):
    """Both header fields together (bits 16-39 and 40-47 of word 7)."""
    keys = inputs.u64_keys(20000, 5300)
    print("case non-minimal + gr approximation", flush=True)
    blob = rs.build(rs.device_keys(keys), 8, 1000, gr_table_max=300, leaf_slack=40)
    want = orc.build(keys, 8, 1000, gr_table_max=300, leaf_slack=40)
    assert blob.to_bytes() == want
    h = orc.header(want)
    assert h["gr_table_max"] == 300 and h["leaf_slack"] == 40
    vals = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
    assert np.array_equal(vals, orc.lookup(want, keys))


def test_nonminimal_roundtrip_and_non_members(rs, orc):
    keys = inputs.u64_keys(40000, 5400)
    want = orc.build(keys, 8, 100, leaf_slack=64)
    blob = rs.from_bytes(want)
    assert blob.to_bytes() == want
    vals = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
    assert np.array_equal(vals, orc.lookup(want, keys))
    other = inputs.u64_keys(100000, 5401)
    got = rs.lookup(blob, rs.device_keys(other)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, orc.lookup(want, other))


def test_nonminimal_batch(rs, orc):
    """One batched call of uneven builds, all with the same slack; each blob
    equals its oracle bytes."""
    specs = [(1000, 8, 100), (7777, 12, 1000), (300, 5, 5), (4000, 16, 2000), (2500, 8, 9)]
    host = [inputs.u64_keys(n, 5500 + i) for i, (n, _, _) in enumerate(specs)]
    print("case non-minimal batch", flush=True)
    blobs, status = rs.build_batch([rs.device_keys(k) for k in host], [s[1] for s in specs], [s[2] for s in specs],
                                   leaf_slack=24)
    assert status == [0] * len(specs)
    for (n, leaf, bucket), k, b in zip(specs, host, blobs):
        want = orc.build(k, leaf, bucket, leaf_slack=24)
        assert b.to_bytes() == want, (n, leaf, bucket)
        vals = rs.lookup(b, rs.device_keys(k)).cpu().numpy().view(np.uint64)
        assert np.array_equal(vals, orc.lookup(want, k))
    for b in blobs:
        b.free()


def test_nonminimal_schedules_never_change_the_result(rs, orc):
    keys = inputs.u64_keys(6000, 5600)
    want = orc.build(keys, 12, 300, leaf_slack=32)
    for waves in (1, 2, 4, 8):
        print(f"case non-minimal waves={waves}", flush=True)
        got = rs.build(rs.device_keys(keys), 12, 300, waves=waves, leaf_slack=32).to_bytes()
        assert got == want, waves


def test_nonminimal_refused_options(rs):
    keys = rs.device_keys(inputs.u64_keys(100, 5700))
    with pytest.raises(rs.RecSplitError):
        rs.build(keys, 24, 100, leaf_slack=86)
    with pytest.raises(rs.RecSplitError):
        rs.build(keys, 8, 100, leaf_slack=256)
