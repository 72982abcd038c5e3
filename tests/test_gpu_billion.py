"""10^9 random 64-bit keys (the scale of the paper's Table tab:1G) at
(l, b) = (8, 100) and (12, 9).  The second point has 1.1e8 buckets: it needs
seven search launches of four wavefronts and a bucket sort in four pieces per
bin.  Checked against the oracle: the header, the Elias-Fano lists of every
bucket (s_i against the oracle's bucket sizes, o_nb against the tree bits),
the indices and key ranks of sampled buckets, and that the lookup of all
10^9 keys is a permutation of [0, n).

It needs about 60 GB of host memory and several minutes, so it runs only
with RS_BIG_TESTS=1 in the environment."""
import os

import numpy as np
import pytest

from paper_1910_06416_amd import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("RS_BIG_TESTS") != "1",
                                 reason="10^9-key test: set RS_BIG_TESTS=1 (about 60 GB of host memory, minutes)")]

N = 1_000_000_000


@pytest.fixture(scope="module")
def rs():
    import torch

    assert torch.cuda.is_available()
    from paper_1910_06416_amd import recsplit

    recsplit.lib()
    return recsplit


@pytest.fixture(scope="module")
def billion(rs, orc):
    import torch

    print(f"drawing {N:,} keys", flush=True)
    keys = inputs.u64_keys_raw(N, 1001)
    d = rs.device_keys(keys)
    srt, _ = torch.sort(d)
    assert not bool((srt[1:] == srt[:-1]).any()), "duplicate draws (choose another seed)"
    del srt
    print("fingerprints on the host", flush=True)
    hi, lo = orc.fingerprint(keys)
    return keys, d, hi, lo


@pytest.mark.parametrize("leaf,bucket", [(8, 100), (12, 9)])
def test_billion_keys(rs, orc, billion, leaf, bucket):
    import torch

    keys, d, hi, lo = billion
    nb = -(-N // bucket)
    print(f"case billion l={leaf} b={bucket} nb={nb}", flush=True)
    blob = rs.build(d, leaf, bucket, timing=True)
    st = rs.last_build_stats()
    print(f"built in {st['ms_device']:.0f} ms device time, {8 * blob.nbytes / N:.4f} bits/key", flush=True)
    got = blob.to_bytes()
    h = orc.header(got)
    ids = orc.bucket_ids(hi, nb).astype(np.int64)
    sizes = np.bincount(ids, minlength=nb)
    assert (h["n"], h["leaf"], h["bucket"], h["nb"], h["maxm"]) == (N, leaf, bucket, nb, int(sizes.max()))
    s_all, o_all = orc.blob_prefix(got)
    assert np.array_equal(s_all, np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64))
    assert o_all[-1] == h["tree_bits"]
    print("lookups of every key", flush=True)
    ranks = rs.lookup(blob, d)
    srt, _ = torch.sort(ranks)
    assert bool(torch.equal(srt, torch.arange(N, dtype=torch.int64, device=srt.device)))
    del srt
    rng = np.random.default_rng(leaf)
    per = (2**32 - 1) // 256
    picks = sorted({int(np.argmax(sizes)), nb - 1, min(per, nb - 1)} | set(rng.integers(0, nb, 6).tolist()))
    r, _, _ = orc.tables(leaf, h["maxm"])
    for i in picks:
        s_i, _, v, m = orc.blob_bucket(got, i)
        idx = np.flatnonzero(ids == i)
        los = lo[idx]
        tv, tm, _ = orc.tree(np.sort(los), leaf)
        assert np.array_equal(m, tm) and np.array_equal(v, tv), f"bucket {i}"
        bits = sum(int(r[mm]) + (int(vv) >> int(r[mm])) + 1 for vv, mm in zip(tv, tm))
        assert int(o_all[i + 1] - o_all[i]) == bits, f"bucket {i}"
        want = orc.bucket_ranks(los, leaf) + np.uint64(s_i)
        got_r = ranks[torch.from_numpy(idx).to(ranks.device)].cpu().numpy().view(np.uint64)
        assert np.array_equal(got_r, want), f"bucket {i}"
    blob.free()
    del ranks
    torch.cuda.empty_cache()
