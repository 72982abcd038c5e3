"""The lookup divides node sizes and hash values below 2^21 by the split unit
with a single-precision reciprocal: q = trunc(float(x) * rcp(float(d))), then
one correction by the sign and size of x - q*d.  This checks on the CPU that the
correction always lands on floor(x / d) when the reciprocal is anywhere within
one unit in the last place of 1/d (the accuracy the hardware reciprocal
guarantees), for random and boundary operands up to 2^21.  The GPU lookups
themselves are compared with the oracle in the GPU tests."""
import numpy as np


def _corrected(x, d, rcp):
    est = (x.astype(np.float32) * rcp).astype(np.float32)
    q = np.trunc(est).astype(np.int64)
    r = x.astype(np.int64) - q * d.astype(np.int64)
    q = np.where(r < 0, q - 1, q)
    q = np.where(r >= d.astype(np.int64), q + 1, q)
    return q


def _check(x, d):
    x = np.asarray(x, dtype=np.uint32)
    d = np.asarray(d, dtype=np.uint32)
    exact = (x // d).astype(np.int64)
    r0 = (np.float32(1.0) / d.astype(np.float32)).astype(np.float32)
    for rcp in (r0, np.nextafter(r0, np.float32(0)), np.nextafter(r0, np.float32(2))):
        got = _corrected(x, d, rcp.astype(np.float32))
        bad = np.nonzero(got != exact)[0]
        assert bad.size == 0, (int(x[bad[0]]), int(d[bad[0]]), int(got[bad[0]]), int(exact[bad[0]]))


def test_random_operands():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 1 << 21, 2_000_000, dtype=np.uint64)
    d = np.maximum(1, (rng.random(x.size) * (x + 1)).astype(np.uint64))
    _check(x, d)
    d2 = rng.integers(1, 64, x.size, dtype=np.uint64)  # the units of small leaves
    _check(x, d2)


def test_quotient_boundaries():
    rng = np.random.default_rng(8)
    d = rng.integers(1, 1 << 20, 500_000, dtype=np.int64)
    k = rng.integers(0, np.maximum(1, ((1 << 21) - 2) // d))
    base = k * d
    for off in (-1, 0, 1):
        x = base + off
        keep = (x >= 0) & (x < (1 << 21))
        _check(x[keep], d[keep])
    # largest operands
    x = np.arange((1 << 21) - 4096, 1 << 21, dtype=np.int64)
    for dd in (1, 2, 3, 7, 8, 96, 112, 560, 1 << 20):
        _check(x, np.full(x.size, dd))


def test_reciprocal_multiply_is_exact_below_2_to_16():
    """Lookups of structures whose nodes are all below 2^16 keys take the child
    index as umulhi(ph, C) with C = ceil(2^32 / u): exact whenever ph * u <
    2^32 (then the error term ph * (C - 2^32/u) / 2^32 stays below 1/u).
    Checked for every part size u < 2^16 at the remainders that come closest
    to the next quotient (ph = q u + u - 1) and at exact multiples, for ph up
    to 2^16."""
    u = np.arange(2, 1 << 16, dtype=np.uint64)
    C = ((np.uint64(1) << np.uint64(32)) + u - np.uint64(1)) // u
    for q in range(0, 40):
        for off in (0, -1):
            ph = np.uint64(q) * u + (u - np.uint64(1) if off else np.uint64(0))
            keep = ph < (1 << 16)
            if not keep.any():
                continue
            p, uu, cc = ph[keep], u[keep], C[keep]
            got = (p * cc) >> np.uint64(32)
            assert np.array_equal(got, p // uu)
    # the largest quotients: small parts, ph near 2^16
    for uu in range(2, 300):
        p = np.arange((1 << 16) - 2 * uu, 1 << 16, dtype=np.uint64)
        cc = np.uint64(((1 << 32) + uu - 1) // uu)
        assert np.array_equal((p * cc) >> np.uint64(32), p // np.uint64(uu))


def test_equal_parts_child_index_identity():
    """Split searches whose parts all hold u keys (m = f u) take a key's part
    as floor(h f / 2^32) instead of floor(floor(h m / 2^32) / u): the nested
    floors of an integer division agree.  Checked for every fanout and part
    size the strategy makes up to l = 24 (f <= 9, u <= 24 * 9 * 7), on random
    and boundary 32-bit hash words."""
    rng = np.random.default_rng(9)
    h = np.concatenate([rng.integers(0, 1 << 32, 20000, dtype=np.uint64),
                        np.array([0, 1, (1 << 32) - 1, 1 << 31], dtype=np.uint64)])
    for f in range(2, 10):
        for u in list(range(1, 65)) + [96, 112, 160, 216, 240, 560, 1512]:
            m = np.uint64(f * u)
            want = ((h * m) >> np.uint64(32)) // np.uint64(u)
            got = (h * np.uint64(f)) >> np.uint64(32)
            assert np.array_equal(got, want), (f, u)
            # boundaries: the smallest h of every part
            edges = (np.arange(1, f, dtype=np.uint64) << np.uint64(32)) // np.uint64(f)
            for e in (edges, edges + np.uint64(1), np.maximum(edges, np.uint64(1)) - np.uint64(1)):
                assert np.array_equal((e * np.uint64(f)) >> np.uint64(32), ((e * m) >> np.uint64(32)) // np.uint64(u))
