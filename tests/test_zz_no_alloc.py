"""rs_build_noalloc (the construction for callers that cannot allocate) against
rs_build, called through the C ABI: byte-identical structures on two calls
in a row (the second smaller, so stale scratch contents would show), the
size query of a too-small buffer, and the refusal of key sets beyond the
scratch array."""
import ctypes

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


def _noalloc(rs, dkeys, leaf, bucket, cap):
    import torch

    k = rs._as_keys(dkeys)
    out = torch.zeros(max(cap, 1), dtype=torch.uint8, device="cuda")
    size = ctypes.c_uint64()
    rc = rs.lib().rs_build_noalloc(ctypes.byref(k), leaf, bucket, ctypes.c_void_p(out.data_ptr()), cap,
                                   ctypes.byref(size), rs._stream(None))
    return rc, size.value, out


@pytest.mark.parametrize("shapes", [[(200_000, 8, 100, 1), (30_000, 8, 100, 2)],
                                    [(50_000, 12, 1000, 3), (777, 5, 5, 4)],
                                    [(100_000, 16, 2000, 5), (3, 8, 100, 6)]])
def test_noalloc_equals_rs_build_on_two_calls(rs, orc, shapes):
    for n, leaf, bucket, seed in shapes:
        print(f"case noalloc n={n} leaf={leaf} bucket={bucket}", flush=True)
        keys = inputs.u64_keys(n, 7000 + seed)
        dk = rs.device_keys(keys)
        want = rs.build(dk, leaf, bucket).to_bytes()
        rc, size, out = _noalloc(rs, dk, leaf, bucket, len(want) + 4096)
        assert rc == rs.RS_OK, rs.lib().rs_last_error()
        assert size == len(want)
        got = out[:size].cpu().numpy().tobytes()
        assert got == want, (n, leaf, bucket)
        # the bytes past the structure are untouched
        assert not out[size:].any()
        if n <= 50_000:
            assert got == orc.build(keys, leaf, bucket)


def test_noalloc_size_query_and_limits(rs, orc):
    keys = inputs.u64_keys(20_000, 7100)
    dk = rs.device_keys(keys)
    want = rs.build(dk, 8, 100).to_bytes()
    print("case noalloc small buffer", flush=True)
    rc, size, _ = _noalloc(rs, dk, 8, 100, 16)
    assert rc == rs.RS_EINVAL and size == len(want)
    rc, size, out = _noalloc(rs, dk, 8, 100, size)
    assert rc == rs.RS_OK and out.cpu().numpy().tobytes() == want
    print("case noalloc beyond the scratch array", flush=True)
    big = rs.device_keys(inputs.u64_keys(3_000_000, 7101))
    rc, _, _ = _noalloc(rs, big, 8, 1, 1 << 20)
    assert rc == rs.RS_EINVAL and b"allocation-free" in rs.lib().rs_last_error()
    # still works after the refusals
    rc, size, out = _noalloc(rs, dk, 8, 100, len(want))
    assert rc == rs.RS_OK and out.cpu().numpy().tobytes() == want
